// The persistent mixed-length kernel (instantiated per element type in
// mixed_c64.hip / mixed_c128.hip, which supply the list of compiled bodies).
//
// Workgroup g runs the items wg_start[g] .. wg_start[g + 1] - 1, which the
// plan assigned ahead of time (longest first, each to the least loaded
// workgroup), so every workgroup knows its next item from the start: while
// an item runs, the next one's record and its transform offsets are already
// being fetched (into registers, then LDS).  An item with a compiled Stockham
// list runs that list's body, which loads the item's transforms and leaves
// the results in LDS; the kernel stores them.  Other lengths run the
// runtime-radix stages, which read and write global memory themselves.
// Threads beyond an item's transforms only take part in the barriers.
#pragma once
#include "mixed.h"
#include "spec_table.h"

namespace fftc {

extern "C" __shared__ __align__(16) unsigned char fftc_dyn_lds[];

// Only lists a mixed plan can run are compiled in as bodies: length at most
// kMixedMaxLen, and a 256-thread workgroup's worth of transforms.
template <typename Real, int N, int... Rs>
constexpr bool mixed_body_ok() {
    using S = SpecInst<Real, N, Rs...>;
    return N <= kMixedMaxLen && S::TPT * S::TM <= kMixedThreads;
}

// The item's results from LDS (element e of transform q at q ldsn +
// lds_pad(e)) to global memory; the stores are left in flight.
template <typename Real, bool INV>
__device__ __forceinline__ void mixed_store(cplx<Real>* out, const cplx<Real>* lds, const MixedItem& item,
                                            const int64_t* offs) {
    using C = cplx<Real>;
    using V = typename vec_of<C>::type;
    const int tot = item.count * item.n;
    for (int l = (int)threadIdx.x; l < tot; l += kMixedThreads) {
        const int q = (int)__umulhi((unsigned)l, item.magic);
        const int e = l - q * item.n;
        C v = lds[q * item.ldsn + lds_pad(e)];
        if (INV) v = cconj(v);
        V w;
        w.x = v.x;
        w.y = v.y;
        __builtin_nontemporal_store(w, reinterpret_cast<V*>(out + offs[q] + e));
    }
}

#define FFTC_BODY_CASE(ID, N, ...)                                                                   \
    case ID:                                                                                         \
        if constexpr (mixed_body_ok<Real, N, __VA_ARGS__>())                                         \
            spec_body<typename SpecInst<Real, N, __VA_ARGS__>::template KM<INV>, kMixedThreads, __VA_ARGS__>( \
                in, offs, item.count, lds, tw + item.twbase, (int)threadIdx.x);                      \
        break;

#define FFTC_DEFINE_MIXED_KERNEL(NAME, LIST)                                                         \
    template <typename Real, bool INV>                                                               \
    __global__ void __launch_bounds__(kMixedThreads, mixed_groups_per_cu<Real>())                    \
    NAME(const cplx<Real>* in, cplx<Real>* out, const cplx<Real>* __restrict__ tw,                  \
         const MixedClass* __restrict__ classes, const MixedItem* __restrict__ items,                \
         const int* __restrict__ wg_start, const int64_t* __restrict__ offsets) {                    \
        using C = cplx<Real>;                                                                        \
        C* lds = reinterpret_cast<C*>(fftc_dyn_lds);                                                 \
        __shared__ int64_t s_offs[2][kMixedThreads];                                                 \
        const int i0 = wg_start[blockIdx.x], i1 = wg_start[blockIdx.x + 1];                          \
        if (i0 >= i1) return;                                                                        \
        MixedItem item = items[i0];                                                                  \
        if ((int)threadIdx.x < item.count) s_offs[0][threadIdx.x] = offsets[item.first + threadIdx.x]; \
        __syncthreads();                                                                             \
        for (int i = i0, buf = 0; i < i1; ++i, buf ^= 1) {                                           \
            /* the next item's record and offsets, in flight during this one */                    \
            const bool more = i + 1 < i1;                                                            \
            MixedItem next = item;                                                                   \
            int64_t noff = 0;                                                                        \
            if (more) {                                                                              \
                next = items[i + 1];                                                                 \
                if ((int)threadIdx.x < next.count) noff = offsets[next.first + threadIdx.x];         \
            }                                                                                        \
            const int64_t* offs = s_offs[buf];                                                       \
            if (item.body >= 0) {                                                                    \
                switch (item.body) {                                                                 \
                    LIST(FFTC_BODY_CASE)                                                             \
                    default: break;                                                                  \
                }                                                                                    \
                /* the body ended with a barrier: its results are in LDS */                         \
                mixed_store<Real, INV>(out, lds, item, offs);                                        \
            } else {                                                                                 \
                const GenDesc& d = classes[item.cls].desc;                                           \
                const int tr = (int)threadIdx.x / d.tpt;                                             \
                const bool member = tr < d.t;                                                        \
                const int t = member ? (int)threadIdx.x - tr * d.tpt : (1 << 28);                    \
                const bool valid = member && tr < item.count;                                        \
                const int64_t toff = offs[valid ? tr : 0];                                           \
                if (d.nst == 0) {                                                                    \
                    if (valid && t == 0) out[toff] = in[toff];                                       \
                } else {                                                                             \
                    C* ldsp = lds + (member ? tr : 0) * classes[item.cls].ldsn;                      \
                    gen_transform<INV, true>(in + toff, out + toff, ldsp, tw, d, t, valid);          \
                }                                                                                    \
            }                                                                                        \
            if (more && (int)threadIdx.x < next.count) s_offs[buf ^ 1][threadIdx.x] = noff;          \
            __syncthreads();                                                                         \
            item = next;                                                                             \
        }                                                                                            \
    }

}  // namespace fftc
