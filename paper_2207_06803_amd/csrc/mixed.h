// Mixed-length persistent plans: device-side descriptors and host state.
#pragma once
#include "generic.h"
#include "internal.h"

namespace fftc {

constexpr int kMixedThreads = 256;             // threads per persistent workgroup
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
    int cls;    // class index
    int first;  // first entry in the grouped transform-offset list
    int count;  // transforms in this item (<= desc.t)
    int pad;
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
    void* dev = nullptr;  // one allocation: counter, classes, items, offsets, twiddles
    size_t dev_bytes = 0;
    unsigned int* counter = nullptr;  // [0] next item, [1] workgroups finished
    MixedClass* d_classes = nullptr;
    MixedItem* d_items = nullptr;
    int64_t* d_offsets = nullptr;
    void* d_tw = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t kernel_node = nullptr;
    const void* fn = nullptr;
    MixedArgs args{};
    void* kargs[8] = {};
    std::vector<int64_t> class_len;
    std::vector<std::vector<int>> class_radices;

    hipKernelNodeParams kernel_params(const void* fn);
};

}  // namespace fftc
