// Single-kernel Stockham FFT: one workgroup owns T whole transforms.
//
// The factorisation is DFT_N = S_t ... S_1 with, for stage q of radix R after
// Ns = R_1 ... R_{q-1} (Eq. 2 applied recursively, in Stockham order):
//   for j < N/R, k = j mod Ns:
//     v_r = x[j + r N/R] * w_{Ns R}^{r k}            (twiddle diagonal)
//     v   = DFT_R v                                  (DFT_R (x) I_{N/R})
//     y[(j div Ns) Ns R + r Ns + k] = v_r            (stride permutation)
// Stage 1 reads HBM directly (unit stride in j), the last stage (Ns R = N)
// writes y[j + r N/R] to HBM in natural order, and the stages in between
// exchange through LDS.  The LDS index is padded by one element every 16 so
// that the stride-R writes of the early stages spread over the banks.
#pragma once
#include <stdint.h>

#include "codelets.h"
#include "kconfig.h"

namespace fftc {

__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 4); }

// Transform data is streamed exactly once in and once out: nontemporal
// vector accesses (one dwordx2 / dwordx4 per element) keep it from displacing
// the twiddle tables in the caches.
template <bool INV, typename C> __device__ __forceinline__ C ld_in(const C* p) {
    using V = typename vec_of<C>::type;
    const V t = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
    C v = mk(t.x, t.y);
    return INV ? cconj(v) : v;
}
template <bool INV, typename C> __device__ __forceinline__ void st_out(C* p, C v) {
    using V = typename vec_of<C>::type;
    if (INV) v = cconj(v);
    V t;
    t.x = v.x;
    t.y = v.y;
    __builtin_nontemporal_store(t, reinterpret_cast<V*>(p));
}

// Contiguous data through pointers typed as global memory: for code outside a
// kernel (the mixed kernel's bodies are functions), where a plain pointer
// argument would be accessed with generic (flat) instructions.
#define FFTC_GLOBAL __attribute__((address_space(1)))
template <typename C> struct GIn {
    const FFTC_GLOBAL C* p;
};
template <typename C> struct GOut {
    FFTC_GLOBAL C* p;
};
template <typename C> __device__ __forceinline__ GIn<C> gshift(GIn<C> a, int64_t off) {
    a.p += off;
    return a;
}
template <typename C> __device__ __forceinline__ GOut<C> gshift(GOut<C> a, int64_t off) {
    a.p += off;
    return a;
}
template <bool INV, typename C> __device__ __forceinline__ C gld(const GIn<C>& a, int e) {
    using V = typename vec_of<C>::type;
    const V t = __builtin_nontemporal_load(reinterpret_cast<const FFTC_GLOBAL V*>(a.p + e));
    C v = mk(t.x, t.y);
    return INV ? cconj(v) : v;
}
template <bool INV, typename C> __device__ __forceinline__ void gst(const GOut<C>& a, int e, C v) {
    using V = typename vec_of<C>::type;
    if (INV) v = cconj(v);
    V t;
    t.x = v.x;
    t.y = v.y;
    __builtin_nontemporal_store(t, reinterpret_cast<FFTC_GLOBAL V*>(a.p + e));
}

// Any other layout (planar re / im arrays, element strides, gaps between
// transforms): element e of transform q at re[q ts + e es] and
// im[q ts + e es] (interleaved complex: im = re + 1 and es, ts counted in
// reals).  The kernels address a transform through gshift (transform
// offset) and gld / gst (element e), with a plain complex pointer for the
// default contiguous layout.
template <typename Real> struct GAcc {
    Real* re;
    Real* im;
    int64_t es, ts;
};

template <typename C> __device__ __forceinline__ C* gshift(C* p, int64_t off) { return p + off; }
template <typename C> __device__ __forceinline__ const C* gshift(const C* p, int64_t off) { return p + off; }
template <typename Real> __device__ __forceinline__ GAcc<Real> gshift(GAcc<Real> a, int64_t q) {
    a.re += q * a.ts;
    a.im += q * a.ts;
    return a;
}
template <bool INV, typename C> __device__ __forceinline__ C gld(const C* p, int e) { return ld_in<INV>(p + e); }
template <bool INV, typename Real> __device__ __forceinline__ cplx<Real> gld(const GAcc<Real>& a, int e) {
    const int64_t o = (int64_t)e * a.es;
    cplx<Real> v = mk(__builtin_nontemporal_load(a.re + o), __builtin_nontemporal_load(a.im + o));
    return INV ? cconj(v) : v;
}
template <bool INV, typename C> __device__ __forceinline__ void gst(C* p, int e, C v) { st_out<INV>(p + e, v); }
template <bool INV, typename Real> __device__ __forceinline__ void gst(const GAcc<Real>& a, int e, cplx<Real> v) {
    const int64_t o = (int64_t)e * a.es;
    if (INV) v = cconj(v);
    __builtin_nontemporal_store(v.x, a.re + o);
    __builtin_nontemporal_store(v.y, a.im + o);
}

// The planar accessor with ordinary (cached) accesses, for kernels whose
// lanes on one transform cover fewer than 128 bytes of one array per access
// (fewer than 32 threads per complex64 transform): each cache line is then
// reached by two accesses, and the second must find it in the cache.
template <typename Real> struct GAccT : GAcc<Real> {};
template <typename Real> __device__ __forceinline__ GAccT<Real> gshift(GAccT<Real> a, int64_t q) {
    a.re += q * a.ts;
    a.im += q * a.ts;
    return a;
}
template <bool INV, typename Real> __device__ __forceinline__ cplx<Real> gld(const GAccT<Real>& a, int e) {
    const int64_t o = (int64_t)e * a.es;
    cplx<Real> v = mk(a.re[o], a.im[o]);
    return INV ? cconj(v) : v;
}
template <bool INV, typename Real> __device__ __forceinline__ void gst(const GAccT<Real>& a, int e, cplx<Real> v) {
    const int64_t o = (int64_t)e * a.es;
    if (INV) v = cconj(v);
    a.re[o] = v.x;
    a.im[o] = v.y;
}
// Planar sides of short-row kernels use the cached accessor.
template <class K, class A> struct LayoutAcc { using type = A; };
template <class K> struct LayoutAcc<K, GAcc<typename K::RealT>> {
    using type = typename std::conditional<(K::TPT * (int)sizeof(typename K::RealT) < 128 && !K::STAGED),
                                           GAccT<typename K::RealT>, GAcc<typename K::RealT>>::type;
};
template <class K, class A> __device__ __forceinline__ typename LayoutAcc<K, A>::type layout_acc(const A& a) {
    typename LayoutAcc<K, A>::type r;
    static_cast<A&>(r) = a;
    return r;
}

// Interleaved complex data at any element and transform strides (es, ts in
// complex elements): one 8-byte (complex64) or 16-byte (complex128) access
// per element, where GAcc would make two of half the width.
template <typename Real> struct GAccI {
    cplx<Real>* p;
    int64_t es, ts;
};
template <typename Real> __device__ __forceinline__ GAccI<Real> gshift(GAccI<Real> a, int64_t q) {
    a.p += q * a.ts;
    return a;
}
template <bool INV, typename Real> __device__ __forceinline__ cplx<Real> gld(const GAccI<Real>& a, int e) {
    return ld_in<INV>(a.p + (int64_t)e * a.es);
}
template <bool INV, typename Real> __device__ __forceinline__ void gst(const GAccI<Real>& a, int e, cplx<Real> v) {
    st_out<INV>(a.p + (int64_t)e * a.es, v);
}

// Multiply v[r] (r >= 1) by w_{Ns R}^{r k}, with tq = table + k (entry
// [(r-1) Ns + k] at tq[(r-1) ns]).  For R = 8 and 16 only the factors
// r = 1, 2, 3 and r = 4, 8, 12 are read and the rest formed as one product
// w^{r k} = w^{(r mod 4) k} w^{4 (r div 4) k}: 6 loads instead of 15 for
// radix 16 (one extra rounding in the formed factors).
// Entry k of a twiddle table, through a plain or a global-typed pointer.
template <typename C> __device__ __forceinline__ C ldtw(const C* p, int k) { return p[k]; }
template <typename C> __device__ __forceinline__ C ldtw(const FFTC_GLOBAL C* p, int k) {
    using V = typename vec_of<C>::type;
    const V t = *reinterpret_cast<const FFTC_GLOBAL V*>(p + k);
    return mk(t.x, t.y);
}

template <int R, typename C, typename P>
__device__ __forceinline__ void apply_twiddles_ns(C* v, P tq, int ns) {
    if constexpr (R == 16 || R == 8) {
        C a[4], b[4];
        a[1] = ldtw(tq, 0 * ns);
        a[2] = ldtw(tq, 1 * ns);
        a[3] = ldtw(tq, 2 * ns);
        b[1] = ldtw(tq, 3 * ns);
        if constexpr (R == 16) {
            b[2] = ldtw(tq, 7 * ns);
            b[3] = ldtw(tq, 11 * ns);
        }
#pragma unroll
        for (int r = 1; r < R; ++r) {
            const int ra = r & 3, rb = r >> 2;
            const C w = (rb == 0) ? a[ra] : (ra == 0 ? b[rb] : cmul(a[ra], b[rb]));
            v[r] = cmul(v[r], w);
        }
    } else {
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], ldtw(tq, (r - 1) * ns));
    }
}

template <int R, int NS, typename C, typename P>
__device__ __forceinline__ void apply_twiddles(C* v, P tq) {
    apply_twiddles_ns<R>(v, tq, NS);
}

// ---------------------------------------------------------------------------
// Compile-time specialised kernel: N, radix sequence, threads per transform
// (TPT) and transforms per workgroup (T) are template parameters, so every
// index division folds to shifts / multiplies.
//
// With TPT >= 16 the first stage reads HBM and the last writes it directly
// (each wave access covers >= 128 contiguous bytes per transform).  Below
// that (short transforms, many per group) the group's transforms are staged:
// loaded cooperatively with consecutive lanes on consecutive elements into
// LDS, transformed LDS to LDS, and stored back the same way.
// ---------------------------------------------------------------------------
// OUT_LDS: the group's results stay in LDS (transform q at q LDSN, element e
// at lds_pad(e), natural order, conjugated for the inverse) for the caller to
// store.
template <typename Real, int N_, int TPT_, int T_, bool INV_, bool OUT_LDS_ = false>
struct SpecCfg {
    using RealT = Real;
    using C = cplx<Real>;
    static constexpr int N = N_, TPT = TPT_, T = T_;
    static constexpr bool INV = INV_;
    static constexpr bool STAGED = TPT_ < 16;
    static constexpr bool OUT_LDS = OUT_LDS_;
};

template <class K, int R, int NS, int TWOFF, bool SRC_G, bool DST_G, class GI, class GO>
__device__ __forceinline__ void spec_stage(GI gin, GO gout, typename K::C* lds,
                                           const typename K::C* __restrict__ tw, int t, bool valid,
                                           bool active) {
    using C = typename K::C;
    constexpr int N = K::N, TPT = K::TPT;
    constexpr int NR = N / R;
    constexpr int NB = (NR + TPT - 1) / TPT;
    constexpr bool EVEN = (NR % TPT) == 0;
    C v[NB][R];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int j = t + i * TPT;
        if (active && (EVEN || j < NR)) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if constexpr (SRC_G) {
                    // unconditional: the caller points gin at a real transform
                    // for out-of-range slots, whose results are never stored
                    v[i][r] = gld<K::INV>(gin, j + r * NR);
                } else {
                    v[i][r] = lds[lds_pad(j + r * NR)];
                }
            }
            // the tables are global memory (typed so, also inside functions)
            if constexpr (NS > 1)
                apply_twiddles<R, NS>(v[i], (const FFTC_GLOBAL C*)tw + TWOFF + j % NS);
            Codelet<R, C>::run(v[i]);
        }
    }
    if constexpr (!SRC_G) __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int j = t + i * TPT;
        if (active && (EVEN || j < NR)) {
            const int k = j % NS;
            const int base = (j / NS) * NS * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if constexpr (DST_G) {
                    if (valid) gst<K::INV>(gout, base + r * NS, v[i][r]);
                } else {
                    lds[lds_pad(base + r * NS)] = v[i][r];
                }
            }
        }
    }
    if constexpr (!DST_G) __syncthreads();
}

template <class K, int NS, int TWOFF, bool FIRST, bool SG, bool DG, int R, int... Rest, class GI, class GO>
__device__ __forceinline__ void spec_stages(GI gin, GO gout, typename K::C* lds,
                                            const typename K::C* __restrict__ tw, int t, bool valid,
                                            bool active) {
    constexpr bool LAST = sizeof...(Rest) == 0;
    spec_stage<K, R, NS, TWOFF, FIRST && SG, LAST && DG>(gin, gout, lds, tw, t, valid, active);
    if constexpr (!LAST)
        spec_stages<K, NS * R, TWOFF + (R - 1) * NS, false, SG, DG, Rest...>(gin, gout, lds, tw, t, valid,
                                                                          active);
}

template <class K, int NR> struct SpecLds {
    static constexpr int LDSN = (NR > 1 || K::STAGED || K::OUT_LDS) ? lds_len(K::N) : 1;
};

// The transforms of one group: transform q < count starts at element toff(q)
// of in and out.  All NTH threads of the workgroup call this (NTH >= TPT T).
template <class K, int NTH, class OffF, int... Rs, class GI, class GO>
__device__ __forceinline__ void spec_group(GI in, GO out, OffF toff, int count, typename K::C* lds,
                                           const typename K::C* __restrict__ tw, int tid) {
    using C = typename K::C;
    constexpr int N = K::N, TPT = K::TPT, T = K::T;
    constexpr int LDSN = SpecLds<K, sizeof...(Rs)>::LDSN;
    const int tr = (T == 1) ? (tid < TPT ? 0 : 1) : tid / TPT;
    const int t = (T == 1) ? tid : tid - tr * TPT;
    const bool member = tr < T;
    const bool valid = member && tr < count;
    C* mylds = lds + (member ? tr : 0) * LDSN;
    if constexpr (K::STAGED) {
        constexpr int TOT = T * N;
        constexpr int ITER = (TOT + NTH - 1) / NTH;
        C buf[ITER];
#pragma unroll
        for (int i = 0; i < ITER; ++i) {
            const int l = tid + i * NTH;
            const int q = min(l / N, count - 1);  // clamp: always a real transform
            buf[i] = gld<K::INV>(gshift(in, toff(q)), l % N);
        }
#pragma unroll
        for (int i = 0; i < ITER; ++i) {
            const int l = tid + i * NTH;
            if (l < TOT) lds[(l / N) * LDSN + lds_pad(l % N)] = buf[i];
        }
        __syncthreads();
        spec_stages<K, 1, 0, true, false, false, Rs...>((const C*)nullptr, (C*)nullptr, mylds, tw, t, valid,
                                                         member);
        if constexpr (!K::OUT_LDS) {
#pragma unroll
            for (int i = 0; i < ITER; ++i) {
                const int l = tid + i * NTH;
                const int q = l / N;
                if (l < TOT && q < count) gst<K::INV>(gshift(out, toff(q)), l % N, lds[q * LDSN + lds_pad(l % N)]);
            }
        }
    } else {
        const int64_t off = toff(valid ? tr : 0);
        spec_stages<K, 1, 0, true, true, !K::OUT_LDS, Rs...>(gshift(in, off), gshift(out, off), mylds, tw, t,
                                                              valid, member);
    }
}

struct ContigOff {
    int64_t base, n;
    __device__ __forceinline__ int64_t operator()(int q) const { return base + (int64_t)q * n; }
};

// Staged group with 16-byte accesses: the group's T transforms are one
// contiguous range; each lane moves two complex64 per access (measured on
// 2^24 complex64 elements: N = 16 48.9 -> 44.3 us, N = 64 53.3 -> 46.4 us).
template <class K, int NTH, int... Rs>
__device__ __forceinline__ void staged_pairs(const float2* gin, float2* gout, int count, float2* lds,
                                             const float2* __restrict__ tw, int tid) {
    using C = float2;
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    constexpr int N = K::N, TPT = K::TPT, T = K::T;
    constexpr int LDSN = SpecLds<K, sizeof...(Rs)>::LDSN;
    constexpr int TOT2 = T * N / 2, IT2 = (TOT2 + NTH - 1) / NTH;
    const int valid2 = count * N / 2;
    const int tr = (T == 1) ? (tid < TPT ? 0 : 1) : tid / TPT;
    const int t = (T == 1) ? tid : tid - tr * TPT;
    const bool member = tr < T;
    const bool valid = member && tr < count;
    f32x4 buf[IT2];
#pragma unroll
    for (int i = 0; i < IT2; ++i) {
        const int l2 = min(tid + i * NTH, valid2 - 1);
        buf[i] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(gin) + l2);
    }
#pragma unroll
    for (int i = 0; i < IT2; ++i) {
        const int l = 2 * (tid + i * NTH);
        if (l < 2 * TOT2) {
            C a = mk(buf[i].x, buf[i].y), b = mk(buf[i].z, buf[i].w);
            if (K::INV) { a = cconj(a); b = cconj(b); }
            lds[(l / N) * LDSN + lds_pad(l % N)] = a;
            lds[((l + 1) / N) * LDSN + lds_pad((l + 1) % N)] = b;
        }
    }
    __syncthreads();
    spec_stages<K, 1, 0, true, false, false, Rs...>((const C*)nullptr, (C*)nullptr, lds + (member ? tr : 0) * LDSN,
                                                     tw, t, valid, member);
#pragma unroll
    for (int i = 0; i < IT2; ++i) {
        const int l2 = tid + i * NTH;
        const int l = 2 * l2;
        if (l2 < valid2) {
            C a = lds[(l / N) * LDSN + lds_pad(l % N)], b = lds[((l + 1) / N) * LDSN + lds_pad((l + 1) % N)];
            if (K::INV) { a = cconj(a); b = cconj(b); }
            f32x4 v;
            v.x = a.x; v.y = a.y; v.z = b.x; v.w = b.y;
            __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(gout) + l2);
        }
    }
}

// Transforms b0 .. b0 + count - 1 of contiguous batch-major data.
template <class K, int... Rs>
__device__ __forceinline__ void spec_contig(const typename K::C* in, typename K::C* out, int64_t b0, int count,
                                            typename K::C* lds, const typename K::C* __restrict__ tw) {
    using C = typename K::C;
    constexpr int N = K::N, NTH = K::TPT * K::T;
    if constexpr (K::STAGED && sizeof(C) == 8 && N % 2 == 0) {
        // 16-byte aligned buffers (the group's range starts at an even element)
        if ((((uintptr_t)in | (uintptr_t)out) & 15) == 0) {
            staged_pairs<K, NTH, Rs...>(reinterpret_cast<const float2*>(in) + b0 * N,
                                        reinterpret_cast<float2*>(out) + b0 * N, count,
                                        reinterpret_cast<float2*>(lds), reinterpret_cast<const float2*>(tw),
                                        (int)threadIdx.x);
            return;
        }
    }
    spec_group<K, NTH, ContigOff, Rs...>(in, out, ContigOff{b0 * N, N}, count, lds, tw, (int)threadIdx.x);
}

template <class K, int... Rs>
__global__ void __launch_bounds__(K::TPT * K::T)
stockham_spec(const typename K::C* in, typename K::C* out,
              const typename K::C* __restrict__ tw, int64_t batch) {
    using C = typename K::C;
    constexpr int T = K::T;
    __shared__ C lds[T * SpecLds<K, sizeof...(Rs)>::LDSN];
    const int64_t b0 = (int64_t)blockIdx.x * T;
    const int count = (int)min((int64_t)T, batch - b0);
    spec_contig<K, Rs...>(in, out, b0, count, lds, tw);
}

// Several requests of one length in one launch (the serving runtime's fused
// steps): request r has its own in / out and batch; its workgroups are
// gstart[r] .. gstart[r + 1] - 1.
constexpr int kMaxFused = 16;
struct ReqList {
    const void* in[kMaxFused];
    void* out[kMaxFused];
    int64_t batch[kMaxFused];
    int64_t gstart[kMaxFused + 1];
    int count;
};

template <class K, int... Rs>
__global__ void __launch_bounds__(K::TPT * K::T)
stockham_spec_reqs(ReqList L, const typename K::C* __restrict__ tw) {
    using C = typename K::C;
    constexpr int T = K::T;
    __shared__ C lds[T * SpecLds<K, sizeof...(Rs)>::LDSN];
    const int64_t blk = blockIdx.x;
    int r = 0;
    while (r + 1 < L.count && L.gstart[r + 1] <= blk) ++r;
    const int64_t b0 = (blk - L.gstart[r]) * T;
    const int count = (int)min((int64_t)T, L.batch[r] - b0);
    spec_contig<K, Rs...>(static_cast<const C*>(L.in[r]), static_cast<C*>(L.out[r]), b0, count, lds, tw);
}

// The same transform for any other layout (GAcc): transform q of the
// launch is transform b0 + q of the layout.
struct IndexOff {
    int64_t base;
    __device__ __forceinline__ int64_t operator()(int q) const { return base + q; }
};

template <class K, class AI, class AO, int... Rs>
__global__ void __launch_bounds__(K::TPT * K::T)
stockham_spec_layout(AI in, AO out, const typename K::C* __restrict__ tw, int64_t batch) {
    using C = typename K::C;
    constexpr int T = K::T, NTH = K::TPT * K::T;
    __shared__ C lds[T * SpecLds<K, sizeof...(Rs)>::LDSN];
    const int64_t b0 = (int64_t)blockIdx.x * T;
    const int count = (int)min((int64_t)T, batch - b0);
    spec_group<K, NTH, IndexOff, Rs...>(layout_acc<K>(in), layout_acc<K>(out), IndexOff{b0}, count, lds, tw,
                                        (int)threadIdx.x);
}

}  // namespace fftc
