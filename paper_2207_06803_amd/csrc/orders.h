// Alternative factorisation orders, for the autotuner to time against the
// Stockham kernels.  The paper writes Cooley-Tukey as Eq. 2 applied
// recursively and runs the recursive (decimation-in-time) form with its
// stride permutations made explicit; it names the Stockham and Pease orders
// as alternatives whose merit depends on the hardware.  For N = R^t, one
// workgroup per T transforms, everything in LDS:
//
//  ORDER_CT (Eq. 2 unrolled, decimation in time): the product of the
//    Pi^N_K factors of the recursion is the base-R digit reversal of the
//    input index, applied explicitly (the input is written to LDS at the
//    reversed position); then t in-place stages, stage s with m = R^s,
//    L = m R: for every butterfly (g, k), k < m, on the elements
//    g L + k + r m (r < R): v_r *= w_L^{r k}, v = DFT_R v, written back in
//    place.
//  ORDER_PEASE (constant geometry): every stage q (ns = R^q) reads
//    v_r = x[j + r N/R] w_{ns R}^{r rev_q(j mod ns)}, applies DFT_R and writes
//    y[j R + r] -- the same addresses in every stage (the perfect shuffle) --
//    with rev_q the reversal of the q low base-R digits; the result is in
//    digit-reversed order, and the explicit reversal is the store's read
//    address.  (Derived from the Stockham stages by conjugating each with the
//    digit permutation that makes its addressing constant.)
//  ORDER_WAVE (Stockham, N = 256 = 16 x 16, the exchange between the two
//    radix-16 stages inside the wave): each of 16 lanes loads one butterfly
//    of the first stage straight from HBM and keeps its 16 outputs (row j of
//    the 16 x 16 intermediate); the stride permutation L^256_16 is then the
//    transpose of that 16 x 16 array across the 16 lanes, done as an xor
//    butterfly over lane bits 1, 2, 4, 8 (at step m a lane swaps half of its
//    registers with lane ^ m: DPP quad permutes for m = 1, 2, ds_swizzle for
//    m = 4, 8) with no LDS and no barrier; the second stage's twiddles and
//    butterflies follow, stored straight to HBM in natural order.
//  ORDER_FOURSTEP (Eq. 2 applied once, the block form): N = K M with
//    M = R^ceil(t/2), K = R^floor(t/2).  The load applies Pi^N_K (element
//    x[j K + i] goes to row i, column j of a K x M array); the K rows are
//    transformed by DFT_M (Stockham stages of radix R on each contiguous
//    row); the first stage of the column transforms multiplies element
//    (i, p) by w_N^{i p} (D^N_M); the M columns (stride M) are transformed by
//    DFT_K, which leaves y[q M + p] in natural order.
//
// Twiddles come from one table of w_N^e, e < N (w_L^a = w_N^{a N / L}).
#pragma once
#include "codelets.h"
#include "kconfig.h"
#include "stockham.h"

namespace fftc {

enum { ORDER_STOCKHAM = 0, ORDER_CT = 1, ORDER_PEASE = 2, ORDER_FOURSTEP = 3, ORDER_WAVE = 4 };

constexpr int ilog(int n, int r) { return n <= 1 ? 0 : 1 + ilog(n / r, r); }
constexpr int ipow(int r, int e) { return e == 0 ? 1 : r * ipow(r, e - 1); }

// reversal of the D low base-R digits of e
template <int R, int D> __device__ __forceinline__ int drev(int e) {
    int o = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        o = o * R + e % R;
        e /= R;
    }
    return o;
}

template <typename Real, int N, int R, int TPT, int T, bool INV, int ORDER>
__global__ void __launch_bounds__(TPT * T)
order_kernel(const cplx<Real>* in, cplx<Real>* out, const cplx<Real>* __restrict__ twn, int64_t batch) {
    using C = cplx<Real>;
    constexpr int TS = ilog(N, R);  // stages
    constexpr int NR = N / R, BPT = NR / TPT, NTH = TPT * T;
    constexpr int LDSN = lds_len(N);
    constexpr int NBUF = ORDER == ORDER_CT ? 1 : 2;
    // four-step split: rows of M = R^TM, columns of K = R^TK
    constexpr int TK = TS / 2, TM = TS - TK, M = ipow(R, TM), K = ipow(R, TK);
    static_assert(NR % TPT == 0, "butterflies must split evenly");
    __shared__ C lds[NBUF * T * LDSN];
    const int tid = (int)threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * T;
    const int count = (int)min((int64_t)T, batch - b0);
    const int tr = tid / TPT, t = tid - tr * TPT;
    // load: consecutive lanes on consecutive elements; CT writes the
    // digit-reversed position
    constexpr int TOT = T * N, IT = (TOT + NTH - 1) / NTH;
    C buf[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int l = tid + i * NTH;
        const int q = min(l / N, count - 1);  // clamped to a real transform
        buf[i] = ld_in<INV>(in + (b0 + q) * N + (l % N));
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int l = tid + i * NTH;
        if (l < TOT) {
            const int e = l % N;
            const int dst = ORDER == ORDER_CT         ? drev<R, TS>(e)
                            : ORDER == ORDER_FOURSTEP ? (e % K) * M + e / K  // Pi^N_K
                                                      : e;
            lds[(l / N) * LDSN + lds_pad(dst)] = buf[i];
        }
    }
    __syncthreads();
    C* a = lds + tr * LDSN;
    C* b = lds + (T + tr) * LDSN;  // Pease: second buffer
#pragma unroll
    for (int s = 0; s < TS; ++s) {
        int m = 1;
#pragma unroll
        for (int u = 0; u < s; ++u) m *= R;
        if constexpr (ORDER == ORDER_CT) {
#pragma unroll
            for (int i = 0; i < BPT; ++i) {
                const int bf = t + i * TPT;
                const int g = bf / m, k = bf - g * m;
                const int base = g * m * R + k;
                C v[R];
#pragma unroll
                for (int r = 0; r < R; ++r) v[r] = a[lds_pad(base + r * m)];
                if (s > 0) {
#pragma unroll
                    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], twn[r * k * (N / (m * R))]);
                }
                Codelet<R, C>::run(v);
#pragma unroll
                for (int r = 0; r < R; ++r) a[lds_pad(base + r * m)] = v[r];
            }
            __syncthreads();
        } else if constexpr (ORDER == ORDER_FOURSTEP) {
            if (s < TM) {
                // DFT_M on each contiguous row, Stockham stage s (ns = m)
                constexpr int MR = M / R;
#pragma unroll
                for (int i = 0; i < BPT; ++i) {
                    const int bf = t + i * TPT;
                    const int row = bf / MR, j = bf - row * MR;
                    const int k = j % m;
                    C v[R];
#pragma unroll
                    for (int r = 0; r < R; ++r) v[r] = a[lds_pad(row * M + j + r * MR)];
                    if (s > 0) {
#pragma unroll
                        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], twn[r * k * (N / (m * R))]);
                    }
                    Codelet<R, C>::run(v);
#pragma unroll
                    for (int r = 0; r < R; ++r) b[lds_pad(row * M + (j / m) * m * R + r * m + k)] = v[r];
                }
            } else {
                // DFT_K on each column (stride M), Stockham stage s - TM; its
                // first stage also applies D^N_M
                constexpr int KR = K / R;
                int ns = 1;
#pragma unroll
                for (int u = TM; u < s; ++u) ns *= R;
#pragma unroll
                for (int i = 0; i < BPT; ++i) {
                    const int bf = t + i * TPT;
                    const int j = bf / M, p = bf - j * M;
                    const int k = j % ns;
                    C v[R];
#pragma unroll
                    for (int r = 0; r < R; ++r) v[r] = a[lds_pad((j + r * KR) * M + p)];
                    if (s == TM) {
#pragma unroll
                        for (int r = 0; r < R; ++r) v[r] = cmul(v[r], twn[(j + r * KR) * p]);  // < K M = N
                    } else {
#pragma unroll
                        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], twn[r * k * (N / (ns * R))]);
                    }
                    Codelet<R, C>::run(v);
#pragma unroll
                    for (int r = 0; r < R; ++r) b[lds_pad(((j / ns) * ns * R + r * ns + k) * M + p)] = v[r];
                }
            }
            __syncthreads();
            C* tmp = a;
            a = b;
            b = tmp;
        } else {
#pragma unroll
            for (int i = 0; i < BPT; ++i) {
                const int j = t + i * TPT;
                C v[R];
#pragma unroll
                for (int r = 0; r < R; ++r) v[r] = a[lds_pad(j + r * NR)];
                if (s > 0) {
                    // reversal of the s low digits of j: reverse all TS digits of
                    // (j mod m) < R^s, then drop the TS - s trailing zeros
                    const int kk = drev<R, TS>(j % m) / (N / m);
#pragma unroll
                    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], twn[r * kk * (N / (m * R))]);
                }
                Codelet<R, C>::run(v);
#pragma unroll
                for (int r = 0; r < R; ++r) b[lds_pad(j * R + r)] = v[r];
            }
            __syncthreads();
            C* tmp = a;
            a = b;
            b = tmp;
        }
    }
    // store natural order; Pease reads the digit-reversed position
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int l = tid + i * NTH;
        const int q = l / N, e = l % N;
        if (l < TOT && q < count) {
            C* src = (ORDER != ORDER_CT && (TS % 2 == 1)) ? lds + (T + q) * LDSN : lds + q * LDSN;
            st_out<INV>(out + (b0 + q) * N + e, src[lds_pad(ORDER == ORDER_PEASE ? drev<R, TS>(e) : e)]);
        }
    }
}

// Exchange of one 32-bit word with lane ^ M (M < 16, within a row of 16):
// DPP quad permutes for M = 1, 2, ds_swizzle's bit mode (xor mask) for 4, 8.
template <int M> __device__ __forceinline__ int xor_lane(int v) {
    if constexpr (M == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);       // quad_perm 1,0,3,2
    else if constexpr (M == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);  // quad_perm 2,3,0,1
    else return __builtin_amdgcn_ds_swizzle(v, (M << 10) | 0x1F);
}
template <int M> __device__ __forceinline__ float xor_lane_val(float v) { return __int_as_float(xor_lane<M>(__float_as_int(v))); }
template <int M> __device__ __forceinline__ double xor_lane_val(double v) {
    const int lo = xor_lane<M>(__double2loint(v)), hi = xor_lane<M>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

// One step of the 16 x 16 transpose across 16 lanes: for each register pair
// (j, j + M), j without bit M, the lane with bit M of its lane index set
// sends register j and receives into it; the other sends j + M and receives
// into j + M.  After steps M = 1, 2, 4, 8, register j of lane t holds what
// register t of lane j held.
template <int M, typename C> __device__ __forceinline__ void transpose_step(C* v, int t) {
    const bool hi = (t & M) != 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (j & M) continue;
        const C a = v[j], b = v[j | M];
        const C send = mk(hi ? a.x : b.x, hi ? a.y : b.y);
        const C recv = mk(xor_lane_val<M>(send.x), xor_lane_val<M>(send.y));
        v[j] = mk(hi ? recv.x : a.x, hi ? recv.y : a.y);
        v[j | M] = mk(hi ? b.x : recv.x, hi ? b.y : recv.y);
    }
}

template <typename Real, bool INV>
__global__ void __launch_bounds__(256)
wave_order_kernel(const cplx<Real>* in, cplx<Real>* out, const cplx<Real>* __restrict__ twn, int64_t batch) {
    using C = cplx<Real>;
    constexpr int N = 256, T = 16;
    const int tid = (int)threadIdx.x, t = tid & 15;
    const int64_t b0 = (int64_t)blockIdx.x * T;
    const int q = tid >> 4;
    const bool valid = b0 + q < batch;
    const int64_t off = (valid ? b0 + q : batch - 1) * N;  // past the end: a real transform, not stored
    C v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = ld_in<INV>(in + off + t + 16 * r);
    Codelet<16, C>::run(v);  // lane t: element 16 t + r of the intermediate
    transpose_step<1>(v, t);
    transpose_step<2>(v, t);
    transpose_step<4>(v, t);
    transpose_step<8>(v, t);  // lane t: element t + 16 r, r = 0..15
#pragma unroll
    for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], twn[r * t]);  // w_256^{r t}
    Codelet<16, C>::run(v);
    if (valid) {
#pragma unroll
        for (int r = 0; r < 16; ++r) st_out<INV>(out + off + t + 16 * r, v[r]);
    }
}

template <typename Real, int N, int R, int ORDER>
struct OrderInst {
    static constexpr int BPT0 = kMaxElemsPerThread / R >= 1 ? kMaxElemsPerThread / R : 1;
    static constexpr int TPT0 = (N / R) / BPT0 >= 1 ? (N / R) / BPT0 : 1;
    static constexpr int TPT = TPT0 > 1024 ? 1024 : TPT0;
    static constexpr int NBUF = ORDER == ORDER_CT ? 1 : 2;
    static constexpr int CS = (int)sizeof(cplx<Real>);
    static constexpr int T0 = TPT >= 256 ? 1 : 256 / TPT;
    static constexpr int T = (T0 * NBUF * lds_len(N) * CS > kLdsMaxPerGroup) ? 1 : T0;
    static_assert(NBUF * T * lds_len(N) * CS <= kLdsMaxPerGroup, "order kernel LDS");
    static OrderEntry entry(int dtype) {
        OrderEntry e{dtype, N, ORDER, R, TPT, T,
                     reinterpret_cast<const void*>(&order_kernel<Real, N, R, TPT, T, false, ORDER>),
                     reinterpret_cast<const void*>(&order_kernel<Real, N, R, TPT, T, true, ORDER>)};
        return e;
    }
};

// The in-wave exchange: N = 256, radix 16, 16 lanes per transform, 16
// transforms per 256-thread workgroup.
template <typename Real>
struct WaveOrderInst {
    static OrderEntry entry(int dtype) {
        OrderEntry e{dtype, 256, ORDER_WAVE, 16, 16, 16,
                     reinterpret_cast<const void*>(&wave_order_kernel<Real, false>),
                     reinterpret_cast<const void*>(&wave_order_kernel<Real, true>)};
        return e;
    }
};

}  // namespace fftc
