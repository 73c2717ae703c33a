// Registry entries for compile-time specialised Stockham kernels.
#pragma once
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
    static_assert((NR > 1 ? T * lds_len(N) * (int)sizeof(cplx<Real>) : 0) <= kLdsMaxPerGroup,
                  "LDS too large");
    using KF = SpecCfg<Real, N, TPT, T, false>;
    using KI = SpecCfg<Real, N, TPT, T, true>;
    static SpecEntry entry(int dtype) {
        SpecEntry e{dtype, N, NR, {Rs...}, TPT, T,
                    reinterpret_cast<const void*>(&stockham_spec<KF, Rs...>),
                    reinterpret_cast<const void*>(&stockham_spec<KI, Rs...>)};
        return e;
    }
};

}  // namespace fftc
