// Registry entries for compile-time specialised Stockham kernels.
#pragma once
#include <type_traits>

#include "internal.h"
#include "stockham.h"

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
    // bodies of the persistent mixed kernel: 256-thread workgroups
    static constexpr int TM = pick_t_for(kWorkgroupTarget, TPT, N, (int)sizeof(cplx<Real>), NR > 1);
    template <bool INV> using KM = SpecCfg<Real, N, TPT, TM, INV>;
    static SpecEntry entry(int dtype, int id) {
        SpecEntry e{dtype, N, NR, {Rs...}, TPT, T,
                    reinterpret_cast<const void*>(&stockham_spec<KF, Rs...>),
                    reinterpret_cast<const void*>(&stockham_spec<KI, Rs...>), id};
        e.tm = TM;
        return e;
    }
    static SpecEntry reqs_entry(int dtype) {
        SpecEntry e{dtype, N, NR, {Rs...}, TPT, T,
                    reinterpret_cast<const void*>(&stockham_spec_reqs<KF, Rs...>),
                    reinterpret_cast<const void*>(&stockham_spec_reqs<KI, Rs...>), -1};
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

// One work item of a compiled list inside the persistent mixed-length kernel:
// `count` transforms at offsets offs[0..count) (not inlined, so each body
// keeps its own registers).
struct ListOff {
    const int64_t* offs;
    __device__ __forceinline__ int64_t operator()(int q) const { return offs[q]; }
};

template <class K, int NTH, int... Rs>
__device__ __noinline__ void spec_body(const typename K::C* in, typename K::C* out, const int64_t* offs,
                                       int count, typename K::C* lds, const typename K::C* __restrict__ tw,
                                       int tid) {
    spec_group<K, NTH, ListOff, Rs...>(in, out, ListOff{offs}, count, lds, tw, tid);
}

}  // namespace fftc
