// Stockham stages with a runtime length and radix list (same stage algebra
// as stockham.h).  Used for lengths without a compiled specialisation and as
// the body of the persistent mixed-length kernel.
#pragma once
#include <stdint.h>

#include "stockham.h"

namespace fftc {

struct StageRt {
    int r;            // radix
    int ns;           // product of the earlier radices
    int twoff;        // offset of this stage's twiddles in the table
    uint32_t ns_mul;  // ceil(2^32 / ns) for ns > 1 (index < 2^16 divides exactly)
};

struct GenDesc {
    int n;        // transform length
    int nst;      // number of stages
    int tpt;      // threads per transform
    int t;        // transforms per workgroup
    StageRt st[kMaxStages];
};

__device__ __forceinline__ int div_ns(int j, const StageRt& s) {
    return s.ns == 1 ? j : (int)__umulhi((uint32_t)j, s.ns_mul);
}

template <int R, bool INV, typename C>
__device__ __forceinline__ void gen_stage(const C* gin, C* gout, C* lds, const C* __restrict__ tw,
                                          const StageRt& s, int n, int tpt, int t, bool valid,
                                          bool src_global, bool dst_global) {
    constexpr int NB = nb_cap(R);
    const int nr = n / R;
    const int ns = s.ns;
    C v[NB][R];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int j = t + i * tpt;
        if (j < nr) {
            if (src_global) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[i][r] = ld_in<INV>(gin + j + r * nr);
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) v[i][r] = lds[lds_pad(j + r * nr)];
            }
            if (ns > 1) apply_twiddles_ns<R>(v[i], tw + s.twoff + (j - div_ns(j, s) * ns), ns);
            Codelet<R, C>::run(v[i]);
        }
    }
    if (!src_global) __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int j = t + i * tpt;
        if (j < nr) {
            const int q = div_ns(j, s);
            const int k = j - q * ns;
            const int base = q * ns * R + k;
            if (dst_global) {
                if (valid) {
#pragma unroll
                    for (int r = 0; r < R; ++r) st_out<INV>(gout + base + r * ns, v[i][r]);
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) lds[lds_pad(base + r * ns)] = v[i][r];
            }
        }
    }
    if (!dst_global) __syncthreads();
}

// The same stage as a called (not inlined) function: a kernel whose stage
// loop switches over seven inlined radix bodies lets their register ranges
// pile up; calls keep each body's registers separate at a small call cost.
template <int R, bool INV, typename C>
__device__ __noinline__ void gen_stage_call(const C* gin, C* gout, C* lds, const C* __restrict__ tw,
                                            StageRt s, int n, int tpt, int t, bool valid, bool src_global,
                                            bool dst_global) {
    gen_stage<R, INV>(gin, gout, lds, tw, s, n, tpt, t, valid, src_global, dst_global);
}

template <int R, bool INV, bool CALL, typename C>
__device__ __forceinline__ void gen_stage_sel(const C* gin, C* gout, C* lds, const C* __restrict__ tw,
                                              const StageRt& s, int n, int tpt, int t, bool valid,
                                              bool src_global, bool dst_global) {
    if constexpr (CALL)
        gen_stage_call<R, INV>(gin, gout, lds, tw, s, n, tpt, t, valid, src_global, dst_global);
    else
        gen_stage<R, INV>(gin, gout, lds, tw, s, n, tpt, t, valid, src_global, dst_global);
}

// All stages of one transform.  Every thread of the workgroup must call this
// (the stages synchronise the workgroup); `t` is the thread's index inside its
// transform, `valid` whether it has a real transform to store (gin must point
// at a real transform either way: loads are unconditional).  With
// in_global the first stage reads gin (HBM), else the transform is already in
// lds; with out_global the last stage writes gout, else it leaves the result
// in lds in natural order.
template <bool INV, bool CALL = false, typename C>
__device__ __forceinline__ void gen_transform(const C* gin, C* gout, C* lds, const C* __restrict__ tw,
                                              const GenDesc& d, int t, bool valid, bool in_global = true,
                                              bool out_global = true) {
    for (int q = 0; q < d.nst; ++q) {
        const StageRt s = d.st[q];
        const bool first = (q == 0) && in_global, last = (q == d.nst - 1) && out_global;
        switch (s.r) {
            case 2: gen_stage_sel<2, INV, CALL>(gin, gout, lds, tw, s, d.n, d.tpt, t, valid, first, last); break;
            case 3: gen_stage_sel<3, INV, CALL>(gin, gout, lds, tw, s, d.n, d.tpt, t, valid, first, last); break;
            case 4: gen_stage_sel<4, INV, CALL>(gin, gout, lds, tw, s, d.n, d.tpt, t, valid, first, last); break;
            case 5: gen_stage_sel<5, INV, CALL>(gin, gout, lds, tw, s, d.n, d.tpt, t, valid, first, last); break;
            case 7: gen_stage_sel<7, INV, CALL>(gin, gout, lds, tw, s, d.n, d.tpt, t, valid, first, last); break;
            case 8: gen_stage_sel<8, INV, CALL>(gin, gout, lds, tw, s, d.n, d.tpt, t, valid, first, last); break;
            default: gen_stage_sel<16, INV, CALL>(gin, gout, lds, tw, s, d.n, d.tpt, t, valid, first, last); break;
        }
    }
}

}  // namespace fftc
