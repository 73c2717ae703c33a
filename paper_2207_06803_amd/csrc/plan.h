// The plan object behind fftc_plan_t.
#pragma once
#include <vector>

#include "formula.h"
#include "generic.h"
#include "internal.h"
#include "mixed.h"

struct fftc_plan_s {
    int64_t n = 0, batch = 0;
    int direction = FFTC_FORWARD, dtype = FFTC_C64;
    int variant = FFTC_VARIANT_SINGLE_GENERIC;
    int device = 0;
    std::vector<int> radices;       // single kernel: the Stockham list
    // single-kernel launch
    const fftc::SpecEntry* spec = nullptr;
    fftc::GenDesc gdesc{};
    int tpt = 0, t = 0;
    size_t lds_bytes = 0;
    void* tw = nullptr;             // device twiddle table
    size_t tw_bytes = 0;
    // two-pass (Eq. 2 four-step): n = m k
    int64_t m = 0, k = 0;
    fftc::GenDesc pass1{}, pass2{};  // length m (k columns), length k (m columns)
    std::vector<int> r1, r2;
    const fftc::FourStepEntry* fs1 = nullptr;  // compiled column kernels, if any
    const fftc::FourStepEntry* fs2 = nullptr;
    int64_t tw1_off = 0, tw2_off = 0, twn_off = 0;  // table offsets (elements)
    void* scratch = nullptr;  // two-pass in-place intermediate (absent: in place refused)
    size_t scratch_bytes = 0;
    // mixed-length persistent plan
    fftc::MixedState* mixed = nullptr;
    // formula plan: lowered passes, or the ordinary plan it folded to
    fftc::FormulaExec* formula = nullptr;
    fftc_plan_s* inner = nullptr;
    int64_t fold_n = 0, fold_p = 0;
    int formula_passes = 0, formula_kernels = 0;
    bool formula_lds = false;
    // layout plan: the compiled kernel with layout accessors, and the layouts
    bool has_layout = false;
    fftc_layout lin{}, lout{};
    // column-like layouts beyond the tile kernel: two passes through `scratch`
    // (m, k, r1, r2, tw1_off, tw2_off, twn_off as for two-pass plans)
    const fftc::FourStepEntry* col1 = nullptr;
    const fftc::FourStepEntry* col2 = nullptr;
    // order plan
    const fftc::OrderEntry* order = nullptr;
};

namespace fftc {

// `batch` <= p->batch: run the first `batch` transforms.
fftc_status launch_single(const fftc_plan_s* p, const void* in, void* out, int64_t batch, hipStream_t s);
fftc_status launch_order(const fftc_plan_s* p, const void* in, void* out, int64_t batch, hipStream_t s);
fftc_status launch_copy16(const void* in, void* out, int64_t nvec, hipStream_t s);
// Requests of one length in one launch (serving): `groups` workgroups in all.
fftc_status launch_reqs(const SpecEntry* e, bool inv, const ReqList& list, int64_t groups, const void* tw,
                        hipStream_t s);
fftc_status launch_layout(const fftc_plan_s* p, const void* in_re, const void* in_im, void* out_re, void* out_im,
                          int64_t batch, hipStream_t s);
fftc_status launch_two_pass(const fftc_plan_s* p, const void* in, void* out, int64_t batch, hipStream_t s);
fftc_status build_mixed(fftc_plan_s* p, const int64_t* n, int64_t count);
fftc_status launch_mixed(fftc_plan_s* p, const void* in, void* out, hipStream_t s);
void destroy_mixed(MixedState* m);
// Radix lists, variant, launch shape and twiddle segments of a Stockham,
// two-pass or split plan (fields of *p other than n, batch, direction and
// dtype); touches no device memory.
fftc_status shape_plan(fftc_plan_s* p, const int* radices, int count, std::vector<TwSegment>* segs,
                       int64_t* entries);
// fftc_plan's argument checks for a plan without an explicit radix list.
fftc_status check_static_args(int64_t n, int64_t batch, int direction, int dtype);
// Let the dynamic-LDS kernels use up to the per-workgroup maximum (once).
fftc_status enable_large_lds();
// Fill a runtime descriptor for a radix list (twoff relative to twbase).
void fill_gen_desc(int64_t n, const std::vector<int>& rs, int tpt, int t, int64_t twbase, GenDesc* d);

}  // namespace fftc
