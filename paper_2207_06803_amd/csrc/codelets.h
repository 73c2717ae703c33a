// Forward DFT_R codelets in registers: v <- DFT_R v with DFT_R[m,n] = w_R^{mn},
// w_R = exp(-2 pi i / R) (the Section II definition at size R).  The inverse
// transform is obtained by the caller as conj(DFT(conj(x))).
//
// R = 2, 4, 8, 16 follow Eq. 2 applied inside the register block (radix-2 and
// radix-4 splits with the small twiddles written as constants); R = 3, 5, 7
// use the symmetric-pair form of the definition: with a_j = x_j + x_{R-j} and
// b_j = x_j - x_{R-j},
//   y_k     = x_0 + sum_j cos(2 pi jk/R) a_j - i sum_j sin(2 pi jk/R) b_j
//   y_{R-k} = x_0 + sum_j cos(2 pi jk/R) a_j + i sum_j sin(2 pi jk/R) b_j.
#pragma once
#include "cplx.h"

namespace fftc {

// cos / sin of 2 pi m / R, correctly rounded doubles.
struct Trig3 {
    static constexpr double c[3] = {1.0, -0.5, -0.5};
    static constexpr double s[3] = {0.0, 0.8660254037844386, -0.8660254037844386};
};
struct Trig5 {
    static constexpr double c[5] = {1.0, 0.30901699437494745, -0.8090169943749475,
                                    -0.8090169943749475, 0.30901699437494745};
    static constexpr double s[5] = {0.0, 0.9510565162951535, 0.5877852522924731,
                                    -0.5877852522924731, -0.9510565162951535};
};
struct Trig7 {
    static constexpr double c[7] = {1.0, 0.6234898018587335, -0.2225209339563144, -0.9009688679024191,
                                    -0.9009688679024191, -0.2225209339563144, 0.6234898018587335};
    static constexpr double s[7] = {0.0, 0.7818314824680298, 0.9749279121818236, 0.4338837391175581,
                                    -0.4338837391175581, -0.9749279121818236, -0.7818314824680298};
};

template <int R> struct TrigOf;
template <> struct TrigOf<3> : Trig3 {};
template <> struct TrigOf<5> : Trig5 {};
template <> struct TrigOf<7> : Trig7 {};

template <int R, typename C> struct Codelet;

template <typename C> struct Codelet<2, C> {
    __device__ __forceinline__ static void run(C* v) {
        C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <typename C> __device__ __forceinline__ void dft4(C& x0, C& x1, C& x2, C& x3) {
    C t0 = cadd(x0, x2), t1 = csub(x0, x2);
    C t2 = cadd(x1, x3), t3 = cmul_mi(csub(x1, x3));
    x0 = cadd(t0, t2);
    x2 = csub(t0, t2);
    x1 = cadd(t1, t3);
    x3 = csub(t1, t3);
}

template <typename C> struct Codelet<4, C> {
    __device__ __forceinline__ static void run(C* v) { dft4(v[0], v[1], v[2], v[3]); }
};

template <typename C> struct Codelet<8, C> {
    // even/odd split: a = DFT_4(x_even), b = DFT_4(x_odd), b_k *= w_8^k,
    // y_k = a_k + b_k, y_{k+4} = a_k - b_k.
    __device__ __forceinline__ static void run(C* v) {
        using Real = decltype(v[0].x);
        const Real h = (Real)0.7071067811865476;
        C a0 = v[0], a1 = v[2], a2 = v[4], a3 = v[6];
        C b0 = v[1], b1 = v[3], b2 = v[5], b3 = v[7];
        dft4(a0, a1, a2, a3);
        dft4(b0, b1, b2, b3);
        // w_8 = (1 - i) h, w_8^2 = -i, w_8^3 = (-1 - i) h
        b1 = mk((b1.x + b1.y) * h, (b1.y - b1.x) * h);
        b2 = cmul_mi(b2);
        b3 = mk((b3.y - b3.x) * h, -(b3.x + b3.y) * h);
        v[0] = cadd(a0, b0); v[4] = csub(a0, b0);
        v[1] = cadd(a1, b1); v[5] = csub(a1, b1);
        v[2] = cadd(a2, b2); v[6] = csub(a2, b2);
        v[3] = cadd(a3, b3); v[7] = csub(a3, b3);
    }
};

template <typename C> struct Codelet<16, C> {
    // Eq. 2 with K = M = 4: y[m + 4p] = sum_i w_4^{ip} w_16^{im} A_i[m],
    // A_i = DFT_4(x_i, x_{i+4}, x_{i+8}, x_{i+12}).
    __device__ __forceinline__ static void run(C* v) {
        using Real = decltype(v[0].x);
        const Real c = (Real)0.9238795325112867;  // cos(pi/8)
        const Real s = (Real)0.3826834323650898;  // sin(pi/8)
        const Real h = (Real)0.7071067811865476;
        for (int i = 0; i < 4; ++i) dft4(v[i], v[i + 4], v[i + 8], v[i + 12]);
        // A_i[m] sits in v[i + 4m]; multiply by w_16^{i m}
        const C w1 = mk(c, -s), w2 = mk(h, -h), w3 = mk(s, -c), w6 = mk(-h, -h), w9 = mk(-c, s);
        v[1 + 4] = cmul(v[1 + 4], w1);
        v[1 + 8] = cmul(v[1 + 8], w2);
        v[1 + 12] = cmul(v[1 + 12], w3);
        v[2 + 4] = cmul(v[2 + 4], w2);
        v[2 + 8] = cmul_mi(v[2 + 8]);
        v[2 + 12] = cmul(v[2 + 12], w6);
        v[3 + 4] = cmul(v[3 + 4], w3);
        v[3 + 8] = cmul(v[3 + 8], w6);
        v[3 + 12] = cmul(v[3 + 12], w9);
        // DFT_4 over i for each m; outputs y[m + 4p] for p = 0..3
        C o[16];
        for (int m = 0; m < 4; ++m) {
            C a0 = v[0 + 4 * m], a1 = v[1 + 4 * m], a2 = v[2 + 4 * m], a3 = v[3 + 4 * m];
            dft4(a0, a1, a2, a3);
            o[m] = a0; o[m + 4] = a1; o[m + 8] = a2; o[m + 12] = a3;
        }
        for (int q = 0; q < 16; ++q) v[q] = o[q];
    }
};

template <int R, typename C> struct OddCodelet {
    __device__ __forceinline__ static void run(C* v) {
        using Real = decltype(v[0].x);
        constexpr int H = (R - 1) / 2;
        C a[H + 1], b[H + 1];
        C y0 = v[0];
        for (int j = 1; j <= H; ++j) {
            a[j] = cadd(v[j], v[R - j]);
            b[j] = csub(v[j], v[R - j]);
            y0 = cadd(y0, a[j]);
        }
        C out[R];
        out[0] = y0;
        for (int k = 1; k <= H; ++k) {
            C re = v[0], im = mk((Real)0, (Real)0);
            for (int j = 1; j <= H; ++j) {
                const Real cc = (Real)TrigOf<R>::c[(j * k) % R];
                const Real ss = (Real)TrigOf<R>::s[(j * k) % R];
                re = mk(re.x + cc * a[j].x, re.y + cc * a[j].y);
                im = mk(im.x + ss * b[j].x, im.y + ss * b[j].y);
            }
            // y_k = re - i im, y_{R-k} = re + i im
            out[k] = mk(re.x + im.y, re.y - im.x);
            out[R - k] = mk(re.x - im.y, re.y + im.x);
        }
        for (int q = 0; q < R; ++q) v[q] = out[q];
    }
};

template <typename C> struct Codelet<3, C> : OddCodelet<3, C> {};
template <typename C> struct Codelet<5, C> : OddCodelet<5, C> {};
template <typename C> struct Codelet<7, C> : OddCodelet<7, C> {};

}  // namespace fftc
