// Layout plans whose transforms are interleaved element by element (a
// layout with dist < stride: the columns of a row-major array).  Loading
// one transform per lane group would touch one element per row; instead a
// workgroup owns TC consecutive transforms and moves the tile between HBM
// and LDS in the order the layout makes contiguous -- consecutive lanes on
// consecutive transforms for a column-like side, on consecutive elements
// otherwise -- then runs the compiled Stockham stages LDS to LDS (the
// column kernels of the two-pass plans, with the layout accessors).
#pragma once
#include "spec_table.h"

namespace fftc {

template <class K, bool INV, class ACC, int... Rs>
__global__ void __launch_bounds__(K::TPT * K::T)
stockham_tile_layout(ACC in, ACC out, const typename K::C* __restrict__ tw, int64_t batch, int in_cols,
                     int out_cols) {
    using C = typename K::C;
    constexpr int LEN = K::N, TPT = K::TPT, TC = K::T, NTH = TPT * TC;
    constexpr int LDSN = tile_pitch(LEN);
    constexpr int TOT = TC * LEN, IT = (TOT + NTH - 1) / NTH;
    __shared__ C lds[TC * LDSN];
    const int tid = (int)threadIdx.x;
    const int64_t col0 = (int64_t)blockIdx.x * TC;
    const int cols = (int)min((int64_t)TC, batch - col0);
    C buf[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int l = tid + i * NTH;
        const int c = in_cols ? l % TC : l / LEN, j = in_cols ? l / TC : l % LEN;
        // clamped: every load reads a real element of a real transform
        const int cc = (c < cols) ? c : 0, jj = min(j, LEN - 1);
        buf[i] = gld<INV>(gshift(in, col0 + cc), jj);
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int l = tid + i * NTH;
        const int c = in_cols ? l % TC : l / LEN, j = in_cols ? l / TC : l % LEN;
        if (l < TOT) lds[c * LDSN + lds_pad(j)] = buf[i];
    }
    __syncthreads();
    const int tr = tid / TPT, t = tid - tr * TPT;
    spec_stages<K, 1, 0, true, false, false, Rs...>((const C*)nullptr, (C*)nullptr, lds + tr * LDSN, tw, t, true,
                                                     true);
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int l = tid + i * NTH;
        const int c = out_cols ? l % TC : l / LEN, j = out_cols ? l / TC : l % LEN;
        if (l < TOT && c < cols) gst<INV>(gshift(out, col0 + c), j, lds[c * LDSN + lds_pad(j)]);
    }
}

// Column-like layouts of lengths whose tile would hold too few transforms
// (N > 1024): Eq. 2 with N = M K in two passes over TC transforms at a time,
// through a scratch array kept column-like (element e of transform c at
// e B + c, B = batch) so both passes move rows of TC contiguous elements.
//   pass 1 (blockIdx.y = i < K): v_j = x_c[j K + i], j < M; DFT_M; times
//          w_N^{i p}; scratch[(i M + p) B + c]
//   pass 2 (blockIdx.y = p < M): v_i = scratch[(i M + p) B + c], i < K;
//          DFT_K; y_c[p + q M], q < K
// The inverse conjugates on pass 1's loads and pass 2's stores.
template <class K, int PASS, bool INV, class ACC, int... Rs>
__global__ void __launch_bounds__(K::TPT * K::T)
col_two_pass(ACC in, ACC out, typename K::C* scratch,
             const typename K::C* __restrict__ tw, const typename K::C* __restrict__ twn, int64_t batch,
             int other) {
    using C = typename K::C;
    constexpr int LEN = K::N, TPT = K::TPT, TC = K::T, NTH = TPT * TC;
    constexpr int LDSN = tile_pitch(LEN);
    constexpr int TOT = TC * LEN, IT = (TOT + NTH - 1) / NTH;
    __shared__ C lds[TC * LDSN];
    const int tid = (int)threadIdx.x;
    const int64_t col0 = (int64_t)blockIdx.x * TC;
    const int cols = (int)min((int64_t)TC, batch - col0);
    const int sub = (int)blockIdx.y;  // pass 1: i < K (other = K); pass 2: p < M (other = M)
    C buf[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int l = tid + i * NTH;
        const int c = l % TC, j = min(l / TC, LEN - 1);
        const int cc = c < cols ? c : 0;  // a missing transform reads the tile's first
        if constexpr (PASS == 1)
            buf[i] = gld<INV>(gshift(in, col0 + cc), j * other + sub);
        else
            buf[i] = scratch[((int64_t)j * other + sub) * batch + col0 + cc];
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
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int l = tid + i * NTH;
        const int c = l % TC, q = l / TC;
        if (l < TOT && c < cols) {
            C v = lds[c * LDSN + lds_pad(q)];
            if constexpr (PASS == 1) {
                const int e = sub * q;  // i p < N <= 2^20
                v = cmul(v, cmul(twn[e % kTwSplit], twn[kTwSplit + e / kTwSplit]));
                scratch[((int64_t)sub * LEN + q) * batch + col0 + c] = v;
            } else {
                gst<INV>(gshift(out, col0 + c), sub + q * other, v);
            }
        }
    }
}

template <typename Real, int TC, int N, int... Rs>
struct ColPassInst {
    static constexpr int rs[sizeof...(Rs)] = {Rs...};
    static constexpr int TPT = round_tpt(required_tpt(N, rs, (int)sizeof...(Rs)));
    static_assert(TPT * TC <= 1024, "column tile too large");
    static_assert(TC * tile_pitch(N) * (int)sizeof(cplx<Real>) <= kLdsMaxPerGroup, "column tile LDS");
    using K = SpecCfg<Real, N, TPT, TC, false>;
    static FourStepEntry entry(int dtype) {
        FourStepEntry e{dtype, N, (int)sizeof...(Rs), {Rs...}, TPT, TC, {}};
        using GA = GAcc<Real>;
        using GI = GAccI<Real>;
        e.fn[0][0] = reinterpret_cast<const void*>(&col_two_pass<K, 1, false, GA, Rs...>);
        e.fn[0][1] = reinterpret_cast<const void*>(&col_two_pass<K, 1, true, GA, Rs...>);
        e.fn[1][0] = reinterpret_cast<const void*>(&col_two_pass<K, 2, false, GA, Rs...>);
        e.fn[1][1] = reinterpret_cast<const void*>(&col_two_pass<K, 2, true, GA, Rs...>);
        e.fn_il[0][0] = reinterpret_cast<const void*>(&col_two_pass<K, 1, false, GI, Rs...>);
        e.fn_il[0][1] = reinterpret_cast<const void*>(&col_two_pass<K, 1, true, GI, Rs...>);
        e.fn_il[1][0] = reinterpret_cast<const void*>(&col_two_pass<K, 2, false, GI, Rs...>);
        e.fn_il[1][1] = reinterpret_cast<const void*>(&col_two_pass<K, 2, true, GI, Rs...>);
        return e;
    }
};

// Transforms per tile: 128 contiguous bytes per row where LDS allows.
constexpr int tile_cols(int n, int csize) {
    int tc = 128 / csize;
    while (tc > 1 && tc * tile_pitch(n) * csize > kLdsMaxPerGroup) tc /= 2;
    return tc;
}

template <typename Real, int N, int... Rs>
struct TileInst {
    static constexpr int rs[sizeof...(Rs)] = {Rs...};
    static constexpr int TC0 = tile_cols(N, (int)sizeof(cplx<Real>));
    static constexpr int TPT = round_tpt(required_tpt(N, rs, (int)sizeof...(Rs)));
    static constexpr int TC = (TPT * TC0 > 1024) ? 1024 / TPT : TC0;
    static_assert(TC >= 1 && TPT * TC <= 1024, "tile too large");
    using K = SpecCfg<Real, N, TPT, TC, false>;
    static void fill(SpecEntry* e) {
        e->tile_fwd = reinterpret_cast<const void*>(&stockham_tile_layout<K, false, GAcc<Real>, Rs...>);
        e->tile_inv = reinterpret_cast<const void*>(&stockham_tile_layout<K, true, GAcc<Real>, Rs...>);
        e->tile_il_fwd = reinterpret_cast<const void*>(&stockham_tile_layout<K, false, GAccI<Real>, Rs...>);
        e->tile_il_inv = reinterpret_cast<const void*>(&stockham_tile_layout<K, true, GAccI<Real>, Rs...>);
        e->tile_tpt = TPT;
        e->tile_tc = TC;
    }
};

template <typename Real, int N, int... Rs>
SpecEntry layout_entry_with_tile(int dtype) {
    SpecEntry e = SpecInst<Real, N, Rs...>::layout_entry(dtype);
    TileInst<Real, N, Rs...>::fill(&e);
    return e;
}

}  // namespace fftc
