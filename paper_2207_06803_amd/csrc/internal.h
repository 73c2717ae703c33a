// Host-side internals shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/fftc.h"
#include "kconfig.h"

namespace fftc {

// ---- errors ---------------------------------------------------------------
fftc_status fail(fftc_status s, const std::string& msg);
fftc_status fail_hip(hipError_t e, const char* what);
void clear_error();

// A launch's workgroup count must fit the grid's x dimension.
inline bool grid_fits(int64_t groups) { return groups >= 0 && groups <= 0x7fffffff; }

// Every device allocation of the library goes through dev_malloc, and every
// allocation of the serving arena asks fault_hit first: with FFTC_FAULT=k in
// the environment (or fftc_fault_set(k)) the k-th such allocation counted
// from then fails as out of memory before any HIP call, so failure paths can
// be tested on purpose (on a CPU with the mock executor).
bool fault_hit();
fftc_status dev_malloc(void** p, size_t bytes, const char* what);
// FFTC_LOG=1 in the environment: one line per plan, server start and stop
// and injected fault on stderr.
bool log_on();
void log_line(const char* fmt, ...);
// FFTC_ROCTX=1 in the environment: roctx ranges (rocprofv3 --marker-trace)
// around plan creation, execution and the server's launch rounds, through
// the ROCm profiler's roctx library loaded at run time (no link dependency).
void range_push(const char* name);
void range_pop();
struct Range {
    explicit Range(const char* name) { range_push(name); }
    ~Range() { range_pop(); }
};

#define FFTC_HIP_TRY(call)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return ::fftc::fail_hip(e_, #call); \
    } while (0)

// ---- factorisation (planner.cpp, host only) -------------------------------
bool is_7smooth(int64_t n);
// Every supported length up to max_single_n runs as one kernel (generic or
// compiled); above it, the lengths with compiled wide lists do too (complex64
// 32768, complex128 16384), the rest run as two passes of Eq. 2.
int64_t max_single_n(int dtype);
bool single_kernel(int64_t n, int dtype);
// The compiled wide lists of n, fastest measured first (empty for other n).
std::vector<std::vector<int>> wide_lists(int64_t n, int dtype);
int64_t max_total_n(int dtype);
// Radix lists that multiply to n, in preference order (first = heuristic pick).
std::vector<std::vector<int>> radix_candidates(int64_t n, int max_lists = 12);
// Threads per transform and transforms per workgroup for a radix list.
void launch_shape(int64_t n, const std::vector<int>& rs, int csize, int* tpt, int* t);
// Two-pass split n = m k (pass 1: k columns of length m; pass 2: m of length k).
bool two_pass_split(int64_t n, int dtype, int64_t* m, int64_t* k);
// Radix list a plan uses: the tuning database's entry, else candidates[0]
// (for a wide length: a recorded list only if it is compiled, else the first
// wide list).
std::vector<int> choose_radices(int64_t n, int dtype);
// Tuning database: best radix list for (n, dtype), if recorded.
bool tune_lookup(int64_t n, int dtype, std::vector<int>* rs);
void tune_record(int64_t n, int dtype, const std::vector<int>& rs, double ms);
// Alternative order recorded for (n, dtype) (FFTC_ORDER_CT / _PEASE), if any.
bool tune_lookup_order(int64_t n, int dtype, int* order, int* radix);
void tune_record_order(int64_t n, int dtype, int order, int radix, double ms);
int tune_load_file(const char* path);
// "<arch> <toolchain>": the part of a database line that must match.
const char* tune_key();
int tune_save_file(const char* path);
void tune_clear_all();

// ---- kernels ----------------------------------------------------------------
struct SpecEntry {
    int dtype, n, nr;
    int radices[kMaxStages];
    int tpt, t;
    const void* fwd;
    const void* inv;
    int id;  // index in the dtype's compiled list (body id in mixed kernels)
    // layout entries: the tile kernel for column-like layouts
    const void* tile_fwd = nullptr;
    const void* tile_inv = nullptr;
    int tile_tpt = 0, tile_tc = 0;
    int tm = 0;  // transforms per 256-thread workgroup in the mixed kernel's body
    bool half = false;  // exchanges through LDS in half width (real, then imaginary parts)
    // layout entries, both sides interleaved (one vector access per element)
    const void* il_fwd = nullptr;
    const void* il_inv = nullptr;
    const void* tile_il_fwd = nullptr;
    const void* tile_il_inv = nullptr;
    // planar in / interleaved out, and interleaved in / planar out
    const void* pi_fwd = nullptr;
    const void* pi_inv = nullptr;
    const void* ip_fwd = nullptr;
    const void* ip_inv = nullptr;
};
// Compiled specialisations, in kSpecParts translation units per dtype.
constexpr int kSpecParts = 4;
const SpecEntry* spec_part(int dtype, int part, int* count);
const SpecEntry* find_spec(int dtype, int64_t n, const std::vector<int>& rs);
// The same transforms compiled with the layout accessors (planar / strided
// data): the preferred list of every compiled length.
const SpecEntry* find_layout(int dtype, int64_t n, const std::vector<int>& rs);
// Several-requests kernels (one launch for requests of one length).
const SpecEntry* find_serve(int dtype, int64_t n, const std::vector<int>& rs);
// Wide single-kernel lists (spec_wide.hip): plain and several-requests kernels.
const SpecEntry* wide_table(int dtype, int* count);
const SpecEntry* wide_serve_table(int dtype, int* count);

// Two-pass column kernels with compiled bodies (fourstep_c64/c128.hip):
// the four kernels (pass x direction) of one column length.
struct FourStepEntry {
    int dtype, len, nr;
    int radices[kMaxStages];
    int tpt, tc;
    const void* fn[2][2];  // [pass - 1][inverse]
    const void* fn_il[2][2] = {};  // column-layout passes, both sides interleaved
};
const FourStepEntry* find_fourstep(int dtype, int64_t len, const std::vector<int>& rs);
// Two-pass kernels for column-like layouts (layout_tile.h), same lengths.
const FourStepEntry* find_colpass(int dtype, int64_t len, const std::vector<int>& rs);

// Alternative orders (orders.h): N = radix^t in one LDS-resident kernel.
struct OrderEntry {
    int dtype, n, order, radix;
    int tpt, t;
    const void* fwd;
    const void* inv;
};
const OrderEntry* order_table(int dtype, int* count);
const OrderEntry* find_order(int dtype, int64_t n, int order, int radix);

struct TwSegment {
    int64_t off;      // first entry in the table
    int64_t count;    // entries
    int64_t ns;       // entry idx -> a = idx / ns + a0, b = idx % ns
    int64_t len;      // value = w_len^{(mul a b) mod len}
    int64_t mul = 1;
    int64_t a0 = 1;
};
// Fill table[seg.off + idx] = exp(-2 pi i ((mul a b) mod len) / len) in fp64,
// stored as float2 (rounded to nearest) or double2.
// Two-pass plans: the factor w_N^e, e < N, is read as the product of
// w_N^{e mod 1024} and w_N^{1024 (e div 1024)} from two small tables.
constexpr int kTwSplit = 1024;
fftc_status make_twiddles(void* table, int dtype, const std::vector<TwSegment>& segs,
                          hipStream_t stream);

// Stage-twiddle segments for a Stockham radix list, appended at `base`.
int64_t stage_segments(const std::vector<int>& rs, int64_t base, std::vector<TwSegment>* segs);

}  // namespace fftc
