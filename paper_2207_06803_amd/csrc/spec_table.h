// Registry entries for compile-time specialised Stockham kernels.
#pragma once
#include <type_traits>

#include "internal.h"
#include "stockham.h"
#include "stockham_half.h"

namespace fftc {

template <typename Real, int N, int... Rs>
struct SpecInst {
    static constexpr int rs[sizeof...(Rs)] = {Rs...};
    static constexpr int NR = sizeof...(Rs);
    static constexpr int TPT = round_tpt(required_tpt(N, rs, NR));
    static constexpr int T = pick_t(TPT, N, (int)sizeof(cplx<Real>), NR > 1);
    static_assert(TPT * T <= 1024, "workgroup too large");
    static_assert(T * lds_len(N) * (int)sizeof(cplx<Real>) <= kLdsMaxPerGroup, "LDS too large");
    using KF = SpecCfg<Real, N, TPT, T, false>;
    using KI = SpecCfg<Real, N, TPT, T, true>;
    template <bool INV> using K = typename std::conditional<INV, KI, KF>::type;
    // bodies of the persistent mixed kernel: 256-thread workgroups, results
    // left in LDS for the kernel to store
    static constexpr int TM = pick_t_for(kWorkgroupTarget, TPT, N, (int)sizeof(cplx<Real>), NR > 1);
    template <bool INV> using KM = SpecCfg<Real, N, TPT, TM, INV, true>;
    // lists whose full LDS exchange fits one workgroup per CU run with the
    // half-width exchange (two per CU)
    static constexpr bool HALF = use_half_exchange<KF, Rs...>();
    template <class KK> static const void* kernel() {
        if constexpr (HALF)
            return reinterpret_cast<const void*>(&stockham_spec_half<KK, Rs...>);
        else
            return reinterpret_cast<const void*>(&stockham_spec<KK, Rs...>);
    }
    static SpecEntry entry(int dtype, int id) {
        SpecEntry e{dtype, N, NR, {Rs...}, TPT, T, kernel<KF>(), kernel<KI>(), id};
        e.tm = TM;
        e.half = HALF;
        return e;
    }
    template <class KK> static const void* reqs_kernel() {
        if constexpr (HALF)
            return reinterpret_cast<const void*>(&stockham_spec_half_reqs<KK, Rs...>);
        else
            return reinterpret_cast<const void*>(&stockham_spec_reqs<KK, Rs...>);
    }
    static SpecEntry reqs_entry(int dtype) {
        SpecEntry e{dtype, N, NR, {Rs...}, TPT, T, reqs_kernel<KF>(), reqs_kernel<KI>(), -1};
        e.half = HALF;
        return e;
    }
    // general accessors on both sides (planar or interleaved), and the
    // interleaved accessor (one vector access per element) on the
    // interleaved side(s): [in interleaved][out interleaved]
    static SpecEntry layout_entry(int dtype) {
        using GA = GAcc<Real>;
        using GI = GAccI<Real>;
        SpecEntry e{dtype, N, NR, {Rs...}, TPT, T,
                    reinterpret_cast<const void*>(&stockham_spec_layout<KF, GA, GA, Rs...>),
                    reinterpret_cast<const void*>(&stockham_spec_layout<KI, GA, GA, Rs...>), -1};
        e.il_fwd = reinterpret_cast<const void*>(&stockham_spec_layout<KF, GI, GI, Rs...>);
        e.il_inv = reinterpret_cast<const void*>(&stockham_spec_layout<KI, GI, GI, Rs...>);
        e.pi_fwd = reinterpret_cast<const void*>(&stockham_spec_layout<KF, GA, GI, Rs...>);
        e.pi_inv = reinterpret_cast<const void*>(&stockham_spec_layout<KI, GA, GI, Rs...>);
        e.ip_fwd = reinterpret_cast<const void*>(&stockham_spec_layout<KF, GI, GA, Rs...>);
        e.ip_inv = reinterpret_cast<const void*>(&stockham_spec_layout<KI, GI, GA, Rs...>);
        return e;
    }
};

// Lengths whose full LDS exchange exceeds a workgroup's LDS (complex64
// N = 32768 and complex128 N = 16384 take 278 KB): one 1024-thread workgroup
// per transform, N / 1024 elements per thread, with the half-width exchange
// (139 KB, one workgroup per CU).  Against the two passes of Eq. 2 these
// lengths would otherwise take, every element crosses HBM once each way
// instead of twice.  No mixed-kernel body (id -1).
template <typename Real, int N, int... Rs>
struct WideSpecInst {
    static constexpr int TPT = 1024;
    using KF = SpecCfg<Real, N, TPT, 1, false>;
    using KI = SpecCfg<Real, N, TPT, 1, true>;
    static_assert(use_half_exchange<KF, Rs...>(), "wide lists run with the half-width exchange");
    static_assert(N / TPT <= 32, "at most 32 elements per thread");
    static_assert(lds_len(N) * (int)sizeof(Real) <= kLdsMaxPerGroup, "half-width exchange LDS");
    static SpecEntry entry(int dtype) {
        SpecEntry e{dtype, N, (int)sizeof...(Rs), {Rs...}, TPT, 1,
                    reinterpret_cast<const void*>(&stockham_spec_half<KF, Rs...>),
                    reinterpret_cast<const void*>(&stockham_spec_half<KI, Rs...>), -1};
        e.half = true;
        return e;
    }
    static SpecEntry reqs_entry(int dtype) {
        SpecEntry e{dtype, N, (int)sizeof...(Rs), {Rs...}, TPT, 1,
                    reinterpret_cast<const void*>(&stockham_spec_half_reqs<KF, Rs...>),
                    reinterpret_cast<const void*>(&stockham_spec_half_reqs<KI, Rs...>), -1};
        e.half = true;
        return e;
    }
};

// One work item of a compiled list inside the persistent mixed-length kernel:
// `count` transforms at offsets offs[0..count), results left in LDS (not
// inlined, so each body keeps its own registers; a function waits for its
// stores before it returns, so the kernel stores instead).  Internal linkage:
// every call site is in the one kernel, so the compiler sees that `lds` and
// `offs` point into LDS and emits LDS instructions for them rather than
// generic (flat) accesses; the global data goes through pointers typed as
// global memory for the same reason.
struct ListOff {
    const int64_t* offs;
    __device__ __forceinline__ int64_t operator()(int q) const { return offs[q]; }
};

template <class K, int NTH, int... Rs>
static __device__ __noinline__ void spec_body(const typename K::C* in, const int64_t* offs, int count,
                                              typename K::C* lds, const typename K::C* __restrict__ tw, int tid) {
    using C = typename K::C;
    static_assert(K::OUT_LDS, "mixed bodies leave their results in LDS");
    spec_group<K, NTH, ListOff, Rs...>(GIn<C>{(const FFTC_GLOBAL C*)in}, GOut<C>{nullptr}, ListOff{offs}, count,
                                       lds, tw, tid);
}

}  // namespace fftc
