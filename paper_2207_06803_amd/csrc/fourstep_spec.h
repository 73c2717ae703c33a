// Two-pass (Eq. 2) plans with compiled Stockham bodies for the column
// transforms.  Same data movement as four_step_pass in exec.hip -- a
// workgroup owns TC adjacent columns, loads them with consecutive lanes on
// consecutive columns (TC * sizeof(complex) contiguous bytes per row), runs
// the column transforms LDS to LDS, and stores -- but the stages are a
// compiled radix list, so every index is a compile-time shift or multiply.
//   pass 1: column i < K of x (stride K), DFT_M, times w_N^{i p}, to row i
//   pass 2: column p < M of z (stride M), DFT_K, to y (stride M)
#pragma once
#include "spec_table.h"

namespace fftc {

constexpr int ilog2_ceil(int x) { return x <= 1 ? 0 : 1 + ilog2_ceil((x + 1) / 2); }
static_assert(ilog2_ceil(16) == 4 && ilog2_ceil(17) == 5 && ilog2_ceil(2) == 1 && ilog2_ceil(1) == 0, "");

template <class K, int PASS, bool INV, int... Rs>
__global__ void __launch_bounds__(K::TPT * K::T)
fourstep_spec(const typename K::C* src, typename K::C* dst, const typename K::C* __restrict__ tw,
              const typename K::C* __restrict__ twn, int64_t n, int ncols) {
    using C = typename K::C;
    constexpr int LEN = K::N, TPT = K::TPT, TC = K::T, NTH = TPT * TC;
    constexpr int LDSN = tile_pitch(LEN);
    constexpr int TOT = TC * LEN, IT = (TOT + NTH - 1) / NTH;
    __shared__ C lds[TC * LDSN];
    const int tid = (int)threadIdx.x;
    const int col0 = (int)blockIdx.x * TC;
    const int cols = min(TC, ncols - col0);
    const int64_t base = (int64_t)blockIdx.y * n;
    // column-fastest load; a missing column reads column 0 of the tile
    C buf[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int l = tid + i * NTH;
        const int c = l % TC, j = min(l / TC, LEN - 1);
        const int cc = c < cols ? c : 0;
        C v = src[base + (int64_t)j * ncols + col0 + cc];
        if (PASS == 1 && INV) v = cconj(v);
        buf[i] = v;
    }
    // pass 1: the twiddles of the elements this thread stores, fetched with
    // the data so their latency is spent before the stages, not after.  A
    // thread stores PP distinct rows p, and for each the columns
    // c = c0 + s S, s < CN, of its tile, so
    //   w_N^{(col0 + c) p} = w_N^{(col0 + c0) p} (w_N^{S p})^s:
    // the first factor from the fine and coarse tables once per p, and the
    // powers w_N^{2^b S p} (b < log2 CN) from the table twc[c M + p] = w_N^{c p}
    // (c < TC) that follows them, read with consecutive lanes on consecutive
    // p.  The other powers are products of these (at most log2 CN - 1 extra
    // roundings), formed after the stages.
    constexpr bool REPEAT = NTH % LEN == 0 || LEN % NTH == 0;
    constexpr int PP = !REPEAT ? 1 : NTH % LEN == 0 ? 1 : LEN / NTH;  // distinct p per thread
    constexpr int S = !REPEAT ? 1 : NTH % LEN == 0 ? NTH / LEN : 1;   // column step between a p's stores
    constexpr int CN = (IT + PP - 1) / PP;                             // stores per p
    constexpr int NB = (PASS == 1 && REPEAT) ? ilog2_ceil(CN) : 0;     // loaded powers per p
    C a[PP], pw[PP][NB > 0 ? NB : 1];
    if constexpr (PASS == 1 && REPEAT) {
        const C* twc = twn + kTwSplit + (int)((n + kTwSplit - 1) / kTwSplit);
        const int c0 = NTH % LEN == 0 ? tid / LEN : 0;
#pragma unroll
        for (int pp = 0; pp < PP; ++pp) {
            const int p = (tid % LEN) + pp * NTH;
            const int e = (col0 + c0) * p;  // < N <= 2^20
            a[pp] = cmul(twn[e % kTwSplit], twn[kTwSplit + e / kTwSplit]);
#pragma unroll
            for (int b = 0; b < NB; ++b) pw[pp][b] = twc[((S << b) % TC) * LEN + p];
        }
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int l = tid + i * NTH;
        if (l < TOT) lds[(l % TC) * LDSN + lds_pad(l / TC)] = buf[i];
    }
    __syncthreads();
    const int tr = tid / TPT, t = tid - tr * TPT;
    spec_stages<K, 1, 0, true, false, false, Rs...>((const C*)nullptr, (C*)nullptr, lds + tr * LDSN, tw, t, true,
                                                     true);
    if constexpr (PASS == 1) {
        // row-major store of column i = col0 + c: z[i M + p] w_N^{i p} (i p < N)
        // (lengths whose rows do not repeat per thread read both tables per
        // element).  v[i] = w_N^{(col0 + c) p} of store i, built from an
        // earlier store's factor of the same p times one loaded power.
        C v[REPEAT ? IT : 1];
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int l = tid + i * NTH;
            const int c = l / LEN, p = l % LEN;
            if constexpr (REPEAT) {
                const int pp = i % PP, s = i / PP;
                if (s == 0) {
                    v[i] = a[pp];
                } else {
                    const int hb = 31 - __builtin_clz(s);  // compile-time after unrolling
                    v[i] = cmul(v[i - (PP << hb)], pw[pp][hb]);
                }
            }
            if (l < TOT && c < cols) {
                C w;
                if constexpr (REPEAT) {
                    w = v[i];
                } else {
                    const int e = (col0 + c) * p;
                    w = cmul(twn[e % kTwSplit], twn[kTwSplit + e / kTwSplit]);
                }
                dst[base + (int64_t)(col0 + c) * LEN + p] = cmul(lds[c * LDSN + lds_pad(p)], w);
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int l = tid + i * NTH;
            const int c = l % TC, q = l / TC;
            if (l < TOT && c < cols) {
                C v = lds[c * LDSN + lds_pad(q)];
                dst[base + (int64_t)q * ncols + col0 + c] = INV ? cconj(v) : v;
            }
        }
    }
}

template <typename Real, int TC_, int N, int... Rs>
struct FourStepInst {
    static constexpr int TC = TC_;
    static constexpr int rs[sizeof...(Rs)] = {Rs...};
    static constexpr int TPT = round_tpt(required_tpt(N, rs, (int)sizeof...(Rs)));
    static_assert(TPT * TC <= 1024, "four-step tile too large");
    static_assert(TC * tile_pitch(N) * (int)sizeof(cplx<Real>) <= kLdsMaxPerGroup, "four-step LDS too large");
    using K = SpecCfg<Real, N, TPT, TC, false>;
    static FourStepEntry entry(int dtype) {
        FourStepEntry e{dtype, N, (int)sizeof...(Rs), {Rs...}, TPT, TC, {}};
        e.fn[0][0] = reinterpret_cast<const void*>(&fourstep_spec<K, 1, false, Rs...>);
        e.fn[0][1] = reinterpret_cast<const void*>(&fourstep_spec<K, 1, true, Rs...>);
        e.fn[1][0] = reinterpret_cast<const void*>(&fourstep_spec<K, 2, false, Rs...>);
        e.fn[1][1] = reinterpret_cast<const void*>(&fourstep_spec<K, 2, true, Rs...>);
        return e;
    }
};

}  // namespace fftc
