// Transforms whose full LDS exchange leaves room for one workgroup per CU
// (complex128 N = 8192: 139 KB of LDS) or does not fit at all (complex64
// N = 32768, complex128 N = 16384: 278 KB).  The exchange between two stages
// moves the real parts through an LDS array of N reals, then the imaginary
// parts through the same array, so a workgroup needs half the LDS: two fit on
// a CU where one did (while one exchanges, the other loads, computes or
// stores), and the longest lengths run in one kernel instead of the two
// passes of Eq. 2.  An exchange takes four barriers instead of two.
// (Measured at 2^24 elements: complex128 N = 8192 123 -> 101 us; complex64
// N = 32768 107 -> 76 us and complex128 N = 16384 237 -> 125 us against two
// passes.  complex64 N = 16384 has the same LDS footprint as complex128
// 8192, but two 1024-thread workgroups per CU leave 64 VGPRs per lane and the
// kernel then spills: 96 us against 66 us with the full exchange, and 73 us
// with 512 threads of 32 elements.)
//
// Stage q (radix R after NS) is the Stockham step of the other kernels: the
// thread's butterflies j = t + i TPT read x[j + r N/R], apply w_{NS R}^{r k}
// (k = j mod NS), run DFT_R and write y[(j div NS) NS R + r NS + k].  Every
// stage must give each thread the same N / TPT elements (TPT divides N / R).
#pragma once
#include "stockham.h"

namespace fftc {

template <int A, int... Rest> struct FirstOf {
    static constexpr int value = A;
};

template <class K, int... Rs> constexpr bool half_even() { return (((K::N / Rs) % K::TPT == 0) && ...); }

// Workgroups per CU with the half-width exchange: as many as the LDS holds,
// up to 32 waves per CU.
template <class K> constexpr int half_groups() {
    constexpr int by_lds = kLdsMaxPerGroup / (lds_len(K::N) * (int)sizeof(typename K::RealT));
    constexpr int by_waves = 32 / (K::TPT / 64);
    return by_lds < by_waves ? by_lds : by_waves;
}

// Whether a compiled list runs with the half-width exchange: one transform
// per workgroup whose full exchange takes more than a quarter of the LDS.
template <class K, int... Rs> constexpr bool use_half_exchange() {
    return K::T == 1 && !K::STAGED && sizeof...(Rs) > 1 && K::TPT % 64 == 0 && half_even<K, Rs...>() &&
           lds_len(K::N) * (int)sizeof(typename K::C) > kLdsMaxPerGroup / 4;
}

template <class K, int NS, int TWOFF, bool FIRST, int R, int... Rest>
__device__ __forceinline__ void half_stages(GIn<typename K::C> gin, GOut<typename K::C> gout,
                                            typename K::RealT* lds, const typename K::C* __restrict__ tw, int t,
                                            typename K::C (&v)[K::N / K::TPT]) {
    using C = typename K::C;
    constexpr int N = K::N, TPT = K::TPT, NR = N / R, NB = NR / TPT;
    constexpr bool LAST = sizeof...(Rest) == 0;
    static_assert(NB * R == N / TPT, "every stage holds N / TPT elements per thread");
    if constexpr (FIRST) {
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int r = 0; r < R; ++r) v[i * R + r] = gld<K::INV>(gin, t + i * TPT + r * NR);
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        if constexpr (NS > 1)
            apply_twiddles<R, NS>(&v[i * R], (const FFTC_GLOBAL C*)tw + TWOFF + (t + i * TPT) % NS);
        Codelet<R, C>::run(&v[i * R]);
    }
    if constexpr (LAST) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int j = t + i * TPT;
            const int base = (j / NS) * NS * R + j % NS;
#pragma unroll
            for (int r = 0; r < R; ++r) gst<K::INV>(gout, base + r * NS, v[i * R + r]);
        }
    } else {
        constexpr int R2 = FirstOf<Rest...>::value;  // the next stage's radix
        constexpr int NR2 = N / R2, NB2 = NR2 / TPT;
        // Padded LDS indices as one per-thread base plus compile-time offsets
        // (immediate offsets of the LDS instructions, so the addresses take
        // two registers instead of 2 N / TPT):
        //   write  lds_pad(base + r NS) = lds_pad(base) + r NS + floor(r NS / 16),
        //          exact when NS and R are powers of two (base mod 16 + (r NS
        //          mod 16) never carries);
        //   read   lds_pad(t + i TPT + r NR2) = lds_pad(t) + (i TPT + r NR2) 17 / 16,
        //          exact when TPT and NR2 are multiples of 16.
        static_assert((NS & (NS - 1)) == 0 && (R & (R - 1)) == 0, "power-of-two radices and strides");
        static_assert(TPT % 16 == 0 && NR2 % 16 == 0, "reads at multiples of 16");
        int wb[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int j = t + i * TPT;
            wb[i] = lds_pad((j / NS) * NS * R + j % NS);
        }
        const int rb = lds_pad(t);
        C w[N / TPT];
        if constexpr (!FIRST) __syncthreads();  // the previous exchange's reads are done
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int r = 0; r < R; ++r) lds[wb[i] + r * NS + (r * NS) / 16] = v[i * R + r].x;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NB2; ++i)
#pragma unroll
            for (int r = 0; r < R2; ++r) w[i * R2 + r].x = lds[rb + (i * TPT + r * NR2) / 16 * 17];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int r = 0; r < R; ++r) lds[wb[i] + r * NS + (r * NS) / 16] = v[i * R + r].y;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NB2; ++i)
#pragma unroll
            for (int r = 0; r < R2; ++r) w[i * R2 + r].y = lds[rb + (i * TPT + r * NR2) / 16 * 17];
        half_stages<K, NS * R, TWOFF + (R - 1) * NS, false, Rest...>(gin, gout, lds, tw, t, w);
    }
}

// One transform per workgroup, half_groups() workgroups per CU (the second
// bound is in waves per SIMD: that many workgroups of TPT / 64 waves over the
// CU's 4 SIMDs).
template <class K, int... Rs>
__global__ void __launch_bounds__(K::TPT, (half_groups<K>() * K::TPT / 64 + 3) / 4)
stockham_spec_half(const typename K::C* in, typename K::C* out, const typename K::C* __restrict__ tw,
                   int64_t batch) {
    using C = typename K::C;
    static_assert(use_half_exchange<K, Rs...>(), "list not suited to the half-width exchange");
    __shared__ typename K::RealT lds[lds_len(K::N)];
    const int64_t b = blockIdx.x;  // one block per transform: b < batch
    (void)batch;
    C v[K::N / K::TPT];
    half_stages<K, 1, 0, true, Rs...>(GIn<C>{(const FFTC_GLOBAL C*)(in + b * K::N)},
                                      GOut<C>{(FFTC_GLOBAL C*)(out + b * K::N)}, lds, tw, (int)threadIdx.x, v);
}

// The serving runtime's several-requests launch (as stockham_spec_reqs) with
// the same stages, so a request gives the same bits fused or alone.
template <class K, int... Rs>
__global__ void __launch_bounds__(K::TPT, (half_groups<K>() * K::TPT / 64 + 3) / 4)
stockham_spec_half_reqs(ReqList L, const typename K::C* __restrict__ tw) {
    using C = typename K::C;
    static_assert(use_half_exchange<K, Rs...>(), "list not suited to the half-width exchange");
    __shared__ typename K::RealT lds[lds_len(K::N)];
    const int64_t blk = blockIdx.x;
    int r = 0;
    while (r + 1 < L.count && L.gstart[r + 1] <= blk) ++r;
    const int64_t b = blk - L.gstart[r];  // one block per transform: b < L.batch[r]
    C v[K::N / K::TPT];
    half_stages<K, 1, 0, true, Rs...>(GIn<C>{(const FFTC_GLOBAL C*)(static_cast<const C*>(L.in[r]) + b * K::N)},
                                      GOut<C>{(FFTC_GLOBAL C*)(static_cast<C*>(L.out[r]) + b * K::N)}, lds, tw,
                                      (int)threadIdx.x, v);
}

}  // namespace fftc
