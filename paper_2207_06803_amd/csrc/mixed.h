// Mixed-length persistent plans: device-side descriptors and host state.
#pragma once
#include "generic.h"
#include "internal.h"

namespace fftc {

constexpr int kMixedThreads = 256;             // threads per persistent workgroup
// Resident workgroups per CU the kernel is compiled for (its register budget:
// 512 / (groups x waves per group) VGPRs per lane): three for complex64,
// two for complex128, whose bodies hold twice the registers.
template <typename Real> constexpr int mixed_groups_per_cu() { return sizeof(Real) == 4 ? 3 : 2; }
constexpr int kMixedMaxLen = 4096;             // longest transform in a mixed plan
constexpr int kMixedLdsElems = lds_len(4096);  // LDS elements per workgroup

struct MixedClass {
    GenDesc desc;  // length, radix list, threads per transform, transforms per item
    int body;      // id of the compiled list in spec_list.inc, -1: runtime radices
    int twbase;    // first twiddle of this class in the shared table
    int ldsn;      // LDS elements per transform (0 for single-stage lists)
    int pad;
};

struct MixedItem {
    int cls;     // class index
    int first;   // first entry in the grouped transform-offset list
    int count;   // transforms in this item (<= desc.t <= kMixedThreads)
    int body;    // the class's compiled list (spec_list.inc id), -1: runtime radices
    int twbase;  // the class's first twiddle in the shared table
    int n;       // transform length
    int ldsn;    // LDS elements per transform (compiled bodies leave results there)
    uint32_t magic;  // ceil(2^32 / n): floor(l / n) = umulhi(l, magic) for l < 2^32 / n
};

// Persistent kernels (mixed_c64.hip / mixed_c128.hip).
const void* mixed_kernel_c64(bool inv);
const void* mixed_kernel_c128(bool inv);

struct MixedArgs {
    const void* in;
    void* out;
};

struct MixedState {
    int64_t count = 0, total = 0;
    int nitems = 0, groups = 0;
    size_t lds_bytes = 0;
    void* dev = nullptr;  // one allocation: classes, items, workgroup ranges, offsets, twiddles
    size_t dev_bytes = 0;
    MixedClass* d_classes = nullptr;
    MixedItem* d_items = nullptr;
    int* d_wg_start = nullptr;  // workgroup g runs items [wg_start[g], wg_start[g + 1])
    int64_t* d_offsets = nullptr;
    void* d_tw = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t kernel_node = nullptr;
    const void* fn = nullptr;
    bool direct = false;       // launch the kernel on the stream instead of replaying the graph
    bool graph_stale = false;  // a direct launch changed args after the graph's parameters were set
    MixedArgs args{};
    void* kargs[7] = {};
    std::vector<int64_t> class_len;
    std::vector<std::vector<int>> class_radices;

    hipKernelNodeParams kernel_params(const void* fn);
};

}  // namespace fftc
