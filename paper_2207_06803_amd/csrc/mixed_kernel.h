// The persistent mixed-length kernel (instantiated per element type in
// mixed_c64.hip / mixed_c128.hip, which supply the list of compiled bodies).
//
// Each resident workgroup loops over items: its first is its own index, each
// later one comes from the atomic counter (counter[0], offset by the grid
// size); it leaves when the item is past the end, otherwise runs the item's
// transforms with its class's body -- a compiled Stockham list when one
// exists, else the runtime-radix stages.  Threads beyond the class's
// transforms only take part in the barriers.  Every workgroup counts its exit
// in counter[1]; the last one resets both counters, so consecutive launches
// need no separate reset.
#pragma once
#include "mixed.h"
#include "spec_table.h"

namespace fftc {

extern "C" __shared__ __align__(16) unsigned char fftc_dyn_lds[];

#define FFTC_BODY_CASE(ID, N, ...)                                                                   \
    case ID:                                                                                         \
        spec_body<typename SpecInst<Real, N, __VA_ARGS__>::template KM<INV>, kMixedThreads, __VA_ARGS__>( \
            in, out, offsets + item.first, item.count, lds, twc, (int)threadIdx.x);                  \
        break;

#define FFTC_DEFINE_MIXED_KERNEL(NAME, LIST)                                                         \
    template <typename Real, bool INV>                                                               \
    __global__ void __launch_bounds__(kMixedThreads)                                                 \
    NAME(const cplx<Real>* in, cplx<Real>* out, const cplx<Real>* __restrict__ tw,                  \
         const MixedClass* __restrict__ classes, const MixedItem* __restrict__ items,                \
         const int64_t* __restrict__ offsets, int nitems, unsigned int* counter) {                   \
        using C = cplx<Real>;                                                                        \
        C* lds = reinterpret_cast<C*>(fftc_dyn_lds);                                                 \
        __shared__ int s_item;                                                                       \
        /* the first item is the workgroup's own index (the grid never exceeds \
           the item count); later ones come from the counter, requested at the \
           start of an item and read after it, so the atomic's latency hides */ \
        int it = (int)blockIdx.x;                                                                    \
        for (;;) {                                                                                   \
            if (it >= nitems) {                                                                      \
                /* the last workgroup out clears both counters for the next launch */               \
                if (threadIdx.x == 0 && atomicAdd(counter + 1, 1u) == gridDim.x - 1) {               \
                    atomicExch(counter, 0u);                                                         \
                    atomicExch(counter + 1, 0u);                                                     \
                }                                                                                    \
                break;                                                                               \
            }                                                                                        \
            unsigned int nx = 0;                                                                     \
            if (threadIdx.x == 0) nx = gridDim.x + atomicAdd(counter, 1u);                           \
            const MixedItem item = items[it];                                                        \
            const MixedClass& c = classes[item.cls];                                                 \
            const GenDesc& d = c.desc;                                                               \
            const int tr = (int)threadIdx.x / d.tpt;                                                 \
            const bool member = tr < d.t;                                                            \
            const int t = member ? (int)threadIdx.x - tr * d.tpt : (1 << 28);                        \
            const bool valid = member && tr < item.count;                                            \
            const int64_t toff = offsets[item.first + (valid ? tr : 0)];                             \
            C* ldsp = lds + (member ? tr : 0) * c.ldsn;                                              \
            if (d.nst == 0) {                                                                        \
                if (valid && t == 0) out[toff] = in[toff];                                           \
            } else if (c.body >= 0) {                                                                \
                const C* twc = tw + c.twbase;                                                        \
                switch (c.body) {                                                                    \
                    LIST(FFTC_BODY_CASE)                                                             \
                    default: break;                                                                  \
                }                                                                                    \
            } else {                                                                                 \
                gen_transform<INV, true>(in + toff, out + toff, ldsp, tw, d, t, valid);              \
            }                                                                                        \
            if (threadIdx.x == 0) s_item = (int)nx;                                                  \
            __syncthreads();                                                                         \
            it = s_item;                                                                             \
            __syncthreads();                                                                         \
        }                                                                                            \
    }

}  // namespace fftc
