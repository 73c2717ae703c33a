// C ABI: plans, execution, errors.  No exception crosses this boundary.
#include <dlfcn.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <new>
#include <string>

#include "plan.h"
#include "split16.h"

namespace fftc {

static thread_local std::string t_last_error;
// Set by the server while it builds plans it only runs out of place.
thread_local bool t_plan_no_scratch = false;

fftc_status fail(fftc_status s, const std::string& msg) {
    t_last_error = msg;
    return s;
}

fftc_status fail_hip(hipError_t e, const char* what) {
    t_last_error = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
    return e == hipErrorOutOfMemory ? FFTC_ERR_OUT_OF_MEMORY : FFTC_ERR_HIP;
}

void clear_error() { t_last_error.clear(); }

// ---- fault injection and logging -------------------------------------------
static std::once_flag g_env_once;
static std::atomic<int64_t> g_fault_at{0}, g_alloc_count{0};
static std::atomic<bool> g_log{false};

using RangePushFn = int (*)(const char*);
using RangePopFn = int (*)();
static RangePushFn g_range_push = nullptr;
static RangePopFn g_range_pop = nullptr;

static void read_env() {
    std::call_once(g_env_once, [] {
        if (const char* f = getenv("FFTC_FAULT")) g_fault_at = atoll(f);
        if (const char* l = getenv("FFTC_LOG")) g_log = *l && strcmp(l, "0") != 0;
        const char* r = getenv("FFTC_ROCTX");
        if (r && *r && strcmp(r, "0") != 0) {
            void* h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_GLOBAL);
            if (!h) h = dlopen("librocprofiler-sdk-roctx.so", RTLD_NOW | RTLD_GLOBAL);
            if (h) {
                auto push = reinterpret_cast<RangePushFn>(dlsym(h, "roctxRangePushA"));
                auto pop = reinterpret_cast<RangePopFn>(dlsym(h, "roctxRangePop"));
                if (push && pop) {
                    g_range_push = push;
                    g_range_pop = pop;
                }
            }
        }
    });
}

void range_push(const char* name) {
    read_env();
    if (g_range_push) g_range_push(name);
}

void range_pop() {
    if (g_range_pop) g_range_pop();
}

bool log_on() {
    read_env();
    return g_log.load(std::memory_order_relaxed);
}

void log_line(const char* fmt, ...) {
    if (!log_on()) return;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    fprintf(stderr, "fftc: %s\n", buf);
}

bool fault_hit() {
    read_env();
    const int64_t at = g_fault_at.load();
    if (at <= 0) return false;
    const bool hit = g_alloc_count.fetch_add(1) + 1 == at;
    if (hit) log_line("injected allocation failure (allocation %lld)", (long long)at);
    return hit;
}

fftc_status dev_malloc(void** p, size_t bytes, const char* what) {
    *p = nullptr;
    if (fault_hit()) return fail(FFTC_ERR_OUT_OF_MEMORY, std::string(what) + ": injected allocation failure");
    const hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail_hip(e, what);
    }
    return FFTC_OK;
}

fftc_status enable_large_lds();
int two_pass_cols(int dtype);

const SpecEntry* find_spec(int dtype, int64_t n, const std::vector<int>& rs) {
    for (int part = 0; part < kSpecParts; ++part) {
        int cnt = 0;
        const SpecEntry* tab = spec_part(dtype, part, &cnt);
        for (int i = 0; i < cnt; ++i) {
            const SpecEntry& e = tab[i];
            if (e.n != n || e.nr != (int)rs.size()) continue;
            bool same = true;
            for (int q = 0; q < e.nr; ++q) same = same && e.radices[q] == rs[q];
            if (same) return &e;
        }
    }
    int cnt = 0;
    const SpecEntry* tab = wide_table(dtype, &cnt);
    for (int i = 0; i < cnt; ++i) {
        const SpecEntry& e = tab[i];
        if (e.n != n || e.nr != (int)rs.size()) continue;
        bool same = true;
        for (int q = 0; q < e.nr; ++q) same = same && e.radices[q] == rs[q];
        if (same) return &e;
    }
    return nullptr;
}

static size_t csize_of(int dtype) { return dtype == FFTC_C128 ? 16 : 8; }  // split modes: complex64

static fftc_status check_radices(int64_t n, const std::vector<int>& rs) {
    int64_t prod = 1;
    for (int r : rs) {
        if (r != 2 && r != 3 && r != 4 && r != 5 && r != 7 && r != 8 && r != 16)
            return fail(FFTC_ERR_INVALID_ARG, "radix " + std::to_string(r) + " not in {2,3,4,5,7,8,16}");
        prod *= r;
    }
    if ((int)rs.size() > kMaxStages) return fail(FFTC_ERR_INVALID_ARG, "too many stages");
    if (prod != n) return fail(FFTC_ERR_INVALID_ARG, "radices do not multiply to n");
    return FFTC_OK;
}


// Shape a single-kernel transform of length n with list rs.
static fftc_status shape_single(fftc_plan_s* p, const std::vector<int>& rs) {
    const size_t cs = csize_of(p->dtype);
    p->radices = rs;
    p->spec = find_spec(p->dtype, p->n, rs);
    if (p->spec) {
        p->tpt = p->spec->tpt;
        p->t = p->spec->t;
        p->variant = FFTC_VARIANT_SINGLE_SPECIALISED;
    } else {
        launch_shape(p->n, rs, (int)cs, &p->tpt, &p->t);
        p->variant = FFTC_VARIANT_SINGLE_GENERIC;
    }
    if (p->n > max_single_n(p->dtype) && !p->spec)
        return fail(FFTC_ERR_UNSUPPORTED_SIZE, "n = " + std::to_string(p->n) +
                                                   " runs only its compiled radix lists (fftc_compiled_entry)");
    if (p->tpt * p->t > 1024) return fail(FFTC_ERR_UNSUPPORTED_SIZE, "radix list needs more than 1024 threads");
    // the half-width exchange moves one real per element at a time
    p->lds_bytes = rs.size() > 1 ? (size_t)p->t * lds_len((int)p->n) * cs / (p->spec && p->spec->half ? 2 : 1) : 0;
    if (p->lds_bytes > (size_t)kLdsMaxPerGroup) return fail(FFTC_ERR_UNSUPPORTED_SIZE, "transform too large for LDS");
    fill_gen_desc(p->n, rs, p->tpt, p->t, 0, &p->gdesc);
    return FFTC_OK;
}

static fftc_status alloc_tables(fftc_plan_s* p, const std::vector<TwSegment>& segs, int64_t entries) {
    const size_t cs = csize_of(p->dtype);
    p->tw_bytes = (size_t)std::max<int64_t>(entries, 1) * cs;
    fftc_status st = dev_malloc(&p->tw, p->tw_bytes, "hipMalloc(twiddles)");
    if (st != FFTC_OK) return st;
    return make_twiddles(p->tw, p->dtype, segs, nullptr);
}

// An order plan (orders.h) for a compiled (n, order, radix); the caller has
// validated direction, dtype and batch.
static fftc_status plan_order_impl(int64_t n, int64_t batch, int direction, int dtype, const OrderEntry* o,
                                   fftc_plan_t* out) {
    fftc_plan_s* p = new (std::nothrow) fftc_plan_s();
    if (!p) return fail(FFTC_ERR_OUT_OF_MEMORY, "host allocation failed");
    p->n = n;
    p->batch = batch;
    p->direction = direction;
    p->dtype = dtype;
    const hipError_t de = hipGetDevice(&p->device);
    if (de != hipSuccess) {
        delete p;
        return fail_hip(de, "hipGetDevice");
    }
    p->variant = FFTC_VARIANT_ORDER;
    p->order = o;
    p->tpt = o->tpt;
    p->t = o->t;
    for (int64_t m = n; m > 1; m /= o->radix) p->radices.push_back(o->radix);
    // one table of w_N^e, e < N
    TwSegment seg;
    seg.off = 0;
    seg.count = n;
    seg.ns = n;
    seg.len = n;
    fftc_status st = alloc_tables(p, {seg}, n);
    if (st != FFTC_OK) {
        std::string keep = t_last_error;
        fftc_destroy_plan(p);
        t_last_error = keep;
        return st;
    }
    *out = p;
    return FFTC_OK;
}

// Argument checks shared by fftc_plan, fftc_plan_radices and
// fftc_execute_static; nothing touches the device.
static fftc_status check_plan_args(int64_t n, int64_t batch, int direction, int dtype, const int* radices,
                                   int count) {
    if (direction != FFTC_FORWARD && direction != FFTC_INVERSE)
        return fail(FFTC_ERR_INVALID_ARG, "direction must be FFTC_FORWARD (-1) or FFTC_INVERSE (+1)");
    if (dtype != FFTC_C64 && dtype != FFTC_C128 && !is_split_dtype(dtype))
        return fail(FFTC_ERR_INVALID_ARG, "dtype must be FFTC_C64, FFTC_C128 or a split-precision mode");
    if (batch < 1) return fail(FFTC_ERR_INVALID_ARG, "batch must be >= 1");
    if (is_split_dtype(dtype)) {
        if (!split_supported(n))
            return fail(FFTC_ERR_UNSUPPORTED_SIZE, "split-precision plans take n in {256, 512, ..., 16384}");
        if (radices) return fail(FFTC_ERR_INVALID_ARG, "split-precision plans use their own radix list");
        if (batch > 0x7fffffff) return fail(FFTC_ERR_INVALID_ARG, "batch too large");
    }
    if (n < 1 || n > max_total_n(dtype) || !is_7smooth(n))
        return fail(FFTC_ERR_UNSUPPORTED_SIZE,
                    "n = " + std::to_string(n) + " unsupported (need 1 <= n <= 2^20 with prime factors <= 7)");
    if (batch > (int64_t(1) << 40) / n) return fail(FFTC_ERR_INVALID_ARG, "batch * n too large");
    if (radices && !single_kernel(n, dtype))
        return fail(FFTC_ERR_INVALID_ARG, "explicit radix lists are for single-kernel lengths only");
    if (radices) {
        if (count < 0 || count > kMaxStages || (count == 0 && n != 1))
            return fail(FFTC_ERR_INVALID_ARG, "bad radix count");
        const std::vector<int> rs(radices, radices + count);
        fftc_status cr = check_radices(n, rs);
        if (cr != FFTC_OK) return cr;
        if (n > max_single_n(dtype) && !find_spec(dtype, n, rs))
            return fail(FFTC_ERR_UNSUPPORTED_SIZE, "n = " + std::to_string(n) +
                                                       " runs only its compiled radix lists (fftc_compiled_entry)");
    }
    return FFTC_OK;
}

// Everything a Stockham, two-pass or split plan holds except device memory:
// radix lists, variant, launch shape, table offsets, and the twiddle
// segments its table needs (*entries elements in all).
fftc_status shape_plan(fftc_plan_s* p, const int* radices, int count, std::vector<TwSegment>* segs,
                       int64_t* entries) {
    const int64_t n = p->n;
    const int dtype = p->dtype;
    const size_t cs = csize_of(dtype);
    segs->clear();
    *entries = 0;
    if (is_split_dtype(dtype)) {
        p->variant = FFTC_VARIANT_SPLIT_MFMA;
        p->radices = split_radices(n);
        p->tpt = split_threads(n);
        p->t = 1;
        *entries = stage_segments(p->radices, 0, segs);
        return FFTC_OK;
    }
    if (single_kernel(n, dtype)) {
        std::vector<int> rs;
        if (radices) {
            rs.assign(radices, radices + count);
        } else {
            rs = choose_radices(n, dtype);
        }
        // DFT_1 is the identity: an empty radix list (the kernel copies)
        if (n == 1) rs.clear();
        if (n > 1 && rs.empty()) return fail(FFTC_ERR_UNSUPPORTED_SIZE, "no factorisation");
        fftc_status st = shape_single(p, rs);
        if (st != FFTC_OK) return st;
        *entries = stage_segments(rs, 0, segs);
        return FFTC_OK;
    }
    int64_t m = 0, k = 0;
    if (!two_pass_split(n, dtype, &m, &k)) return fail(FFTC_ERR_UNSUPPORTED_SIZE, "no two-pass split");
    p->variant = FFTC_VARIANT_TWO_PASS;
    p->m = m;
    p->k = k;
    // prefer a column list with compiled kernels: the tuned or preferred
    // list, else the planner's first candidate
    auto pick = [&](int64_t len, const FourStepEntry** fs) {
        std::vector<int> rs = choose_radices(len, dtype);
        *fs = find_fourstep(dtype, len, rs);
        if (!*fs) {
            auto c = radix_candidates(len, 1);
            if (!c.empty() && (*fs = find_fourstep(dtype, len, c[0])) != nullptr) rs = c[0];
        }
        return rs;
    };
    p->r1 = pick(m, &p->fs1);
    p->r2 = pick(k, &p->fs2);
    const int tc = two_pass_cols(dtype);
    // columns per pass-1 tile (the compiled kernel's own width)
    const int tc1 = p->fs1 ? p->fs1->tc : tc;
    int tpt1, tpt2, tdummy;
    launch_shape(m, p->r1, (int)cs, &tpt1, &tdummy);
    launch_shape(k, p->r2, (int)cs, &tpt2, &tdummy);
    if (tpt1 * tc > 1024 || tpt2 * tc > 1024 ||
        (size_t)tc * tile_pitch((int)std::max(m, k)) * cs > (size_t)kLdsMaxPerGroup)
        return fail(FFTC_ERR_UNSUPPORTED_SIZE, "two-pass tile does not fit a workgroup");
    p->tw1_off = 0;
    const int64_t e1 = stage_segments(p->r1, 0, segs);
    p->tw2_off = e1;
    const int64_t e2 = stage_segments(p->r2, e1, segs);
    p->twn_off = e1 + e2;
    // w_N^e for e < N as fine (e mod 1024) x coarse (e div 1024) tables
    const int64_t nhi = (n + kTwSplit - 1) / kTwSplit;
    segs->push_back({p->twn_off, kTwSplit, kTwSplit, n, 1});
    segs->push_back({p->twn_off + kTwSplit, nhi, nhi, n, kTwSplit});
    // then w_N^{c p} at [c M + p] for the c < tc1 columns of a tile
    segs->push_back({p->twn_off + kTwSplit + nhi, tc1 * m, m, n, 1, 0});
    fill_gen_desc(m, p->r1, tpt1, tc, p->tw1_off, &p->pass1);
    fill_gen_desc(k, p->r2, tpt2, tc, p->tw2_off, &p->pass2);
    p->radices = p->r1;
    p->radices.insert(p->radices.end(), p->r2.begin(), p->r2.end());
    p->tpt = tpt1;
    p->t = tc;
    *entries = p->twn_off + kTwSplit + nhi + tc1 * m;
    return FFTC_OK;
}

static fftc_status plan_impl(int64_t n, int64_t batch, int direction, int dtype, const int* radices,
                             int count, fftc_plan_t* out) {
    clear_error();
    if (!out) return fail(FFTC_ERR_INVALID_ARG, "plan_out is NULL");
    *out = nullptr;
    fftc_status st = check_plan_args(n, batch, direction, dtype, radices, count);
    if (st != FFTC_OK) return st;
    if (!radices && !is_split_dtype(dtype)) {  // an alternative order the order autotuner recorded
        int order = 0, radix = 0;
        const OrderEntry* o = nullptr;
        if (tune_lookup_order(n, dtype, &order, &radix) && (o = find_order(dtype, n, order, radix)) != nullptr &&
            batch <= (int64_t(1) << 31))
            return plan_order_impl(n, batch, direction, dtype, o, out);
    }
    st = enable_large_lds();
    if (st != FFTC_OK) return st;

    fftc_plan_s* p = new (std::nothrow) fftc_plan_s();
    if (!p) return fail(FFTC_ERR_OUT_OF_MEMORY, "host allocation failed");
    p->n = n;
    p->batch = batch;
    p->direction = direction;
    p->dtype = dtype;
    const hipError_t de = hipGetDevice(&p->device);
    if (de != hipSuccess) {
        delete p;
        return fail_hip(de, "hipGetDevice");
    }
    std::vector<TwSegment> segs;
    int64_t entries = 0;
    st = shape_plan(p, radices, count, &segs, &entries);
    if (st == FFTC_OK) st = alloc_tables(p, segs, entries);
    if (st == FFTC_OK && p->variant == FFTC_VARIANT_TWO_PASS && !t_plan_no_scratch) {
        p->scratch_bytes = (size_t)batch * (size_t)n * csize_of(dtype);
        st = dev_malloc(&p->scratch, p->scratch_bytes, "hipMalloc(two-pass scratch)");
    }
    if (st != FFTC_OK) {
        std::string keep = t_last_error;
        fftc_destroy_plan(p);
        t_last_error = keep;
        return st;
    }
    if (log_on()) {
        std::string rs;
        for (int r : p->radices) rs += (rs.empty() ? "" : ",") + std::to_string(r);
        log_line("plan n=%lld batch=%lld %s dtype=%d variant=%d radices=%s tables=%zu B scratch=%zu B",
                 (long long)n, (long long)batch, direction == FFTC_INVERSE ? "inverse" : "forward", dtype,
                 p->variant, rs.c_str(), p->tw_bytes, p->scratch_bytes);
    }
    *out = p;
    return FFTC_OK;
}

fftc_status check_static_args(int64_t n, int64_t batch, int direction, int dtype) {
    return check_plan_args(n, batch, direction, dtype, nullptr, 0);
}

}  // namespace fftc

using namespace fftc;

extern "C" {

const char* fftc_status_string(fftc_status s) {
    switch (s) {
        case FFTC_OK: return "FFTC_OK";
        case FFTC_ERR_INVALID_ARG: return "FFTC_ERR_INVALID_ARG";
        case FFTC_ERR_UNSUPPORTED_SIZE: return "FFTC_ERR_UNSUPPORTED_SIZE";
        case FFTC_ERR_OUT_OF_MEMORY: return "FFTC_ERR_OUT_OF_MEMORY";
        case FFTC_ERR_TOO_LARGE: return "FFTC_ERR_TOO_LARGE";
        case FFTC_ERR_HIP: return "FFTC_ERR_HIP";
        case FFTC_ERR_SHUTDOWN: return "FFTC_ERR_SHUTDOWN";
        case FFTC_ERR_INTERNAL: return "FFTC_ERR_INTERNAL";
    }
    return "FFTC_ERR_UNKNOWN";
}

const char* fftc_last_error(void) { return t_last_error.c_str(); }

fftc_status fftc_fault_set(int64_t k) {
    read_env();
    g_fault_at = k > 0 ? k : 0;
    g_alloc_count = 0;
    return FFTC_OK;
}

int64_t fftc_fault_count(void) { return g_alloc_count.load(); }

fftc_status fftc_plan(int64_t n, int64_t batch, int direction, int dtype, fftc_plan_t* plan_out) {
    Range r("fftc_plan");
    try {
        return plan_impl(n, batch, direction, dtype, nullptr, 0, plan_out);
    } catch (...) {
        return fail(FFTC_ERR_INTERNAL, "exception in fftc_plan");
    }
}

fftc_status fftc_plan_radices(int64_t n, int64_t batch, int direction, int dtype, const int* radices,
                              int count, fftc_plan_t* plan_out) {
    if (!radices) return fail(FFTC_ERR_INVALID_ARG, "radices is NULL");
    try {
        return plan_impl(n, batch, direction, dtype, radices, count, plan_out);
    } catch (...) {
        return fail(FFTC_ERR_INTERNAL, "exception in fftc_plan_radices");
    }
}

fftc_status fftc_plan_mixed(const int64_t* n, int64_t count, int direction, int dtype, fftc_plan_t* plan_out) {
    clear_error();
    if (!plan_out) return fail(FFTC_ERR_INVALID_ARG, "plan_out is NULL");
    *plan_out = nullptr;
    if (!n || count < 1) return fail(FFTC_ERR_INVALID_ARG, "need count >= 1 lengths");
    if (direction != FFTC_FORWARD && direction != FFTC_INVERSE)
        return fail(FFTC_ERR_INVALID_ARG, "direction must be FFTC_FORWARD (-1) or FFTC_INVERSE (+1)");
    if (dtype != FFTC_C64 && dtype != FFTC_C128) return fail(FFTC_ERR_INVALID_ARG, "bad dtype");
    if (count > (int64_t(1) << 30)) return fail(FFTC_ERR_INVALID_ARG, "too many transforms");
    for (int64_t i = 0; i < count; ++i)
        if (n[i] < 1 || n[i] > kMixedMaxLen || !is_7smooth(n[i]))
            return fail(FFTC_ERR_UNSUPPORTED_SIZE, "mixed length n[" + std::to_string(i) + "] = " +
                                                       std::to_string(n[i]) + " unsupported (1..4096, 7-smooth)");
    try {
        fftc_status st = enable_large_lds();
        if (st != FFTC_OK) return st;
        fftc_plan_s* p = new (std::nothrow) fftc_plan_s();
        if (!p) return fail(FFTC_ERR_OUT_OF_MEMORY, "host allocation failed");
        p->n = 0;
        p->batch = count;
        p->direction = direction;
        p->dtype = dtype;
        p->variant = FFTC_VARIANT_MIXED_PERSISTENT;
        hipGetDevice(&p->device);
        st = build_mixed(p, n, count);
        if (st != FFTC_OK) {
            std::string keep = t_last_error;
            fftc_destroy_plan(p);
            t_last_error = keep;
            return st;
        }
        *plan_out = p;
        return FFTC_OK;
    } catch (...) {
        return fail(FFTC_ERR_INTERNAL, "exception in fftc_plan_mixed");
    }
}

fftc_status fftc_plan_mixed_set_launch(fftc_plan_t p, int mode) {
    clear_error();
    if (!p) return fail(FFTC_ERR_INVALID_ARG, "plan is NULL");
    if (p->variant != FFTC_VARIANT_MIXED_PERSISTENT || !p->mixed)
        return fail(FFTC_ERR_INVALID_ARG, "not a mixed plan");
    if (mode != FFTC_MIXED_LAUNCH_GRAPH && mode != FFTC_MIXED_LAUNCH_DIRECT)
        return fail(FFTC_ERR_INVALID_ARG, "mode must be FFTC_MIXED_LAUNCH_GRAPH or FFTC_MIXED_LAUNCH_DIRECT");
    p->mixed->direct = mode == FFTC_MIXED_LAUNCH_DIRECT;
    return FFTC_OK;
}

static fftc_status execute_impl(fftc_plan_t p, const void* in, void* out, int64_t batch, void* stream) {
    clear_error();
    if (!p) return fail(FFTC_ERR_INVALID_ARG, "plan is NULL");
    if (!in || !out) return fail(FFTC_ERR_INVALID_ARG, "in/out is NULL");
    const uintptr_t align = p->dtype == FFTC_C128 ? 16 : 8;
    if (((uintptr_t)in % align) || ((uintptr_t)out % align))
        return fail(FFTC_ERR_INVALID_ARG, "in/out not aligned to the complex element size");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (p->variant == FFTC_VARIANT_MIXED_PERSISTENT) {
        if (batch != p->batch) return fail(FFTC_ERR_INVALID_ARG, "mixed plans run their whole list");
        return launch_mixed(p, in, out, s);
    }
    if (batch < 1 || batch > p->batch) return fail(FFTC_ERR_INVALID_ARG, "batch must be in [1, plan batch]");
    if (p->variant == FFTC_VARIANT_ORDER) return launch_order(p, in, out, batch, s);
    if (p->has_layout) {
        if (p->lin.planar || p->lout.planar)
            return fail(FFTC_ERR_INVALID_ARG, "planar layout plans run through fftc_execute_layout");
        return launch_layout(p, in, nullptr, out, nullptr, batch, s);
    }
    if (p->variant == FFTC_VARIANT_FORMULA) {
        if (p->inner) return execute_impl(p->inner, in, out, batch * p->fold_p, stream);
        return formula_launch(p->formula, in, out, batch, p->direction == FFTC_INVERSE, s);
    }
    if (p->variant == FFTC_VARIANT_SPLIT_MFMA) return launch_split(p, in, out, batch, s);
    if (p->variant == FFTC_VARIANT_TWO_PASS) return launch_two_pass(p, in, out, batch, s);
    return launch_single(p, in, out, batch, s);
}

fftc_status fftc_execute(fftc_plan_t p, const void* in, void* out, void* stream) {
    Range r("fftc_execute");
    return execute_impl(p, in, out, p ? p->batch : 0, stream);
}

fftc_status fftc_execute_batch(fftc_plan_t p, const void* in, void* out, int64_t batch, void* stream) {
    Range r("fftc_execute_batch");
    return execute_impl(p, in, out, batch, stream);
}

fftc_status fftc_destroy_plan(fftc_plan_t p) {
    if (!p) return FFTC_OK;
    fftc_status st = FFTC_OK;
    if (p->tw) {
        hipError_t e = hipFree(p->tw);
        if (e != hipSuccess) st = fail_hip(e, "hipFree(twiddles)");
    }
    if (p->scratch) {
        hipError_t e = hipFree(p->scratch);
        if (e != hipSuccess) st = fail_hip(e, "hipFree(scratch)");
    }
    if (p->mixed) destroy_mixed(p->mixed);
    if (p->formula) formula_destroy(p->formula);
    if (p->inner) {
        fftc_status si = fftc_destroy_plan(p->inner);
        if (st == FFTC_OK) st = si;
    }
    delete p;
    return st;
}

fftc_status fftc_plan_describe(fftc_plan_t p, fftc_plan_desc* d) {
    if (!p || !d) return fail(FFTC_ERR_INVALID_ARG, "NULL argument");
    memset(d, 0, sizeof(*d));
    d->n = p->n;
    d->batch = p->batch;
    d->direction = p->direction;
    d->dtype = p->dtype;
    d->variant = p->variant;
    d->nradices = (int)std::min<size_t>(p->radices.size(), 16);
    for (int i = 0; i < d->nradices; ++i) d->radices[i] = p->radices[i];
    d->threads_per_transform = p->tpt;
    d->transforms_per_group = p->t;
    d->split_m = p->m;
    d->split_k = p->k;
    d->twiddle_bytes = p->tw_bytes;
    d->scratch_bytes = p->scratch_bytes;
    if (p->mixed) {
        d->mixed_transforms = p->mixed->count;
        d->mixed_elements = p->mixed->total;
        d->mixed_classes = (int)p->mixed->class_len.size();
        d->mixed_items = p->mixed->nitems;
        d->persistent_groups = p->mixed->groups;
        d->twiddle_bytes = p->mixed->dev_bytes;
    }
    if (p->order) {
        d->order = p->order->order;
        d->order_radix = p->order->radix;
    }
    if (p->has_layout) {
        d->has_layout = 1;
        d->layout_in = p->lin;
        d->layout_out = p->lout;
    }
    if (p->variant == FFTC_VARIANT_FORMULA) {
        d->formula_passes = p->formula_passes;
        d->formula_folded = p->inner ? 1 : 0;
        d->formula_lds = p->formula_lds ? 1 : 0;
        d->formula_kernels = p->inner ? 0 : p->formula_kernels;
        d->formula_fold_n = p->fold_n;
        d->formula_fold_p = p->fold_p;
        if (p->inner) {
            d->nradices = (int)std::min<size_t>(p->inner->radices.size(), 16);
            for (int i = 0; i < d->nradices; ++i) d->radices[i] = p->inner->radices[i];
            d->split_m = p->inner->m;
            d->split_k = p->inner->k;
            d->twiddle_bytes = p->inner->tw_bytes;
            d->scratch_bytes = p->inner->scratch_bytes;
        }
    }
    return FFTC_OK;
}

fftc_status fftc_plan_order(int64_t n, int64_t batch, int direction, int dtype, int order, int radix,
                            fftc_plan_t* plan_out) {
    try {
        clear_error();
        if (!plan_out) return fail(FFTC_ERR_INVALID_ARG, "plan_out is NULL");
        *plan_out = nullptr;
        if (direction != FFTC_FORWARD && direction != FFTC_INVERSE)
            return fail(FFTC_ERR_INVALID_ARG, "direction must be FFTC_FORWARD (-1) or FFTC_INVERSE (+1)");
        if (dtype != FFTC_C64 && dtype != FFTC_C128)
            return fail(FFTC_ERR_INVALID_ARG, "order plans take FFTC_C64 or FFTC_C128");
        if (batch < 1 || batch > (int64_t(1) << 31)) return fail(FFTC_ERR_INVALID_ARG, "batch must be in [1, 2^31]");
        if (order != FFTC_ORDER_CT && order != FFTC_ORDER_PEASE && order != FFTC_ORDER_FOURSTEP &&
            order != FFTC_ORDER_WAVE)
            return fail(FFTC_ERR_INVALID_ARG,
                        "order must be FFTC_ORDER_CT, FFTC_ORDER_PEASE, FFTC_ORDER_FOURSTEP or FFTC_ORDER_WAVE");
        const OrderEntry* o = find_order(dtype, n, order, radix);
        if (!o)
            return fail(FFTC_ERR_UNSUPPORTED_SIZE, "no compiled kernel for n = " + std::to_string(n) + ", radix " +
                                                       std::to_string(radix) + " in this order");
        return plan_order_impl(n, batch, direction, dtype, o, plan_out);
    } catch (...) {
        return fail(FFTC_ERR_INTERNAL, "exception in fftc_plan_order");
    }
}

int fftc_order_count(int dtype) {
    int cnt = 0;
    if (dtype != FFTC_C64 && dtype != FFTC_C128) return 0;
    order_table(dtype, &cnt);
    return cnt;
}

fftc_status fftc_order_entry(int dtype, int i, int64_t* n, int* order, int* radix) {
    clear_error();
    if (!n || !order || !radix) return fail(FFTC_ERR_INVALID_ARG, "NULL argument");
    if (dtype != FFTC_C64 && dtype != FFTC_C128) return fail(FFTC_ERR_INVALID_ARG, "bad dtype");
    int cnt = 0;
    const OrderEntry* tab = order_table(dtype, &cnt);
    if (i < 0 || i >= cnt) return fail(FFTC_ERR_INVALID_ARG, "index out of range");
    *n = tab[i].n;
    *order = tab[i].order;
    *radix = tab[i].radix;
    return FFTC_OK;
}

static fftc_status check_layout(const fftc_layout& l, int64_t n, int64_t batch, const char* side) {
    const std::string w = std::string(side) + " layout: ";
    if (l.planar != 0 && l.planar != 1) return fail(FFTC_ERR_INVALID_ARG, w + "planar must be 0 or 1");
    const int64_t lim = int64_t(1) << 40;
    if (l.stride < 1 || l.dist < 1 || l.stride > lim || l.dist > lim)
        return fail(FFTC_ERR_INVALID_ARG, w + "stride and dist must be in [1, 2^40]");
    const bool blocks = l.dist >= (n - 1) * l.stride + 1;
    const bool interleaved = l.stride / l.dist >= batch;
    if (!blocks && !interleaved)
        return fail(FFTC_ERR_INVALID_ARG, w + "transforms share elements (need dist >= (n-1) stride + 1 or "
                                              "stride >= batch dist)");
    return FFTC_OK;
}

fftc_status fftc_plan_layout(int64_t n, int64_t batch, int direction, int dtype, const fftc_layout* in,
                             const fftc_layout* out, fftc_plan_t* plan_out) {
    try {
        clear_error();
        if (!plan_out) return fail(FFTC_ERR_INVALID_ARG, "plan_out is NULL");
        *plan_out = nullptr;
        if (direction != FFTC_FORWARD && direction != FFTC_INVERSE)
            return fail(FFTC_ERR_INVALID_ARG, "direction must be FFTC_FORWARD (-1) or FFTC_INVERSE (+1)");
        if (dtype != FFTC_C64 && dtype != FFTC_C128)
            return fail(FFTC_ERR_INVALID_ARG, "layout plans take FFTC_C64 or FFTC_C128");
        if (batch < 1 || batch > (int64_t(1) << 40)) return fail(FFTC_ERR_INVALID_ARG, "batch must be in [1, 2^40]");
        if (n < 2 || n > max_total_n(dtype) || !is_7smooth(n))
            return fail(FFTC_ERR_UNSUPPORTED_SIZE, "layout plans take 2 <= n <= 2^20 with prime factors <= 7");
        const fftc_layout dflt{1, n, 0};
        const fftc_layout li = in ? *in : dflt, lo = out ? *out : dflt;
        fftc_status st = check_layout(li, n, batch, "in");
        if (st == FFTC_OK) st = check_layout(lo, n, batch, "out");
        if (st != FFTC_OK) return st;
        // the single-kernel form (compiled with the layout accessors)
        std::vector<int> rs;
        const SpecEntry* e = nullptr;
        if (n <= max_single_n(dtype)) {
            rs = choose_radices(n, dtype);
            if (!(e = find_layout(dtype, n, rs))) {
                auto c = radix_candidates(n, 1);
                if (!c.empty() && (e = find_layout(dtype, n, c[0])) != nullptr) rs = c[0];
            }
        }
        // a column-like side whose tile would hold fewer than 8 transforms (or
        // a length without a single kernel): Eq. 2 in two passes of TC
        // transforms each, with compiled column kernels for both factors
        const bool cols = li.dist < li.stride || lo.dist < lo.stride;
        const FourStepEntry *c1 = nullptr, *c2 = nullptr;
        int64_t m = 0, k = 0;
        std::vector<int> r1, r2;
        if (cols && (!e || e->tile_tc < 8)) {
            for (int64_t a = 2; a <= 1024; ++a) {  // most balanced split with both factors <= 1024
                if (n % a || n / a > 1024 || n / a < 2) continue;
                if (!m || std::llabs(a - n / a) < std::llabs(m - k)) {
                    m = a;
                    k = n / a;
                }
            }
            auto pick = [&](int64_t len, const FourStepEntry** fs) {
                std::vector<int> r = choose_radices(len, dtype);
                if (!(*fs = find_colpass(dtype, len, r))) {
                    auto c = radix_candidates(len, 1);
                    if (!c.empty() && (*fs = find_colpass(dtype, len, c[0])) != nullptr) r = c[0];
                }
                return r;
            };
            if (m) {
                r1 = pick(m, &c1);
                r2 = pick(k, &c2);
            }
            if (!c1 || !c2) c1 = c2 = nullptr;
        }
        if (!e && !c1)
            return fail(FFTC_ERR_UNSUPPORTED_SIZE, "no compiled layout kernel for n = " + std::to_string(n) +
                                                       (cols ? "" : " (lengths above the single-kernel limit "
                                                                    "take column-like layouts only)"));
        fftc_plan_s* p = new (std::nothrow) fftc_plan_s();
        if (!p) return fail(FFTC_ERR_OUT_OF_MEMORY, "host allocation failed");
        p->n = n;
        p->batch = batch;
        p->direction = direction;
        p->dtype = dtype;
        hipGetDevice(&p->device);
        p->has_layout = true;
        p->lin = li;
        p->lout = lo;
        std::vector<TwSegment> segs;
        int64_t entries = 0;
        if (c1) {
            p->variant = FFTC_VARIANT_TWO_PASS;
            p->col1 = c1;
            p->col2 = c2;
            p->m = m;
            p->k = k;
            p->r1 = r1;
            p->r2 = r2;
            p->radices = r1;
            p->radices.insert(p->radices.end(), r2.begin(), r2.end());
            p->tpt = c1->tpt;
            p->t = c1->tc;
            p->tw1_off = 0;
            entries += stage_segments(r1, entries, &segs);
            p->tw2_off = entries;
            entries += stage_segments(r2, entries, &segs);
            p->twn_off = entries;
            const int64_t nhi = (n + kTwSplit - 1) / kTwSplit;
            segs.push_back({p->twn_off, kTwSplit, kTwSplit, n, 1});
            segs.push_back({p->twn_off + kTwSplit, nhi, nhi, n, kTwSplit});
            entries += kTwSplit + nhi;
        } else {
            p->variant = FFTC_VARIANT_SINGLE_SPECIALISED;
            p->radices = rs;
            p->spec = e;
            p->tpt = e->tpt;
            p->t = e->t;
            entries = stage_segments(rs, 0, &segs);
        }
        st = alloc_tables(p, segs, entries);
        if (st == FFTC_OK && p->col1) {
            p->scratch_bytes = (size_t)batch * (size_t)n * csize_of(dtype);
            st = dev_malloc(&p->scratch, p->scratch_bytes, "hipMalloc(column scratch)");
        }
        if (st != FFTC_OK) {
            std::string keep = t_last_error;
            fftc_destroy_plan(p);
            t_last_error = keep;
            return st;
        }
        *plan_out = p;
        return FFTC_OK;
    } catch (...) {
        return fail(FFTC_ERR_INTERNAL, "exception in fftc_plan_layout");
    }
}

fftc_status fftc_execute_layout(fftc_plan_t p, const void* in_re, const void* in_im, void* out_re, void* out_im,
                                void* stream) {
    clear_error();
    if (!p) return fail(FFTC_ERR_INVALID_ARG, "plan is NULL");
    if (!p->has_layout) return fail(FFTC_ERR_INVALID_ARG, "not a layout plan (fftc_plan_layout)");
    if (!in_re || !out_re) return fail(FFTC_ERR_INVALID_ARG, "in_re/out_re is NULL");
    if (p->lin.planar ? !in_im : in_im != nullptr)
        return fail(FFTC_ERR_INVALID_ARG, p->lin.planar ? "planar input needs in_im" : "interleaved input: in_im must be NULL");
    if (p->lout.planar ? !out_im : out_im != nullptr)
        return fail(FFTC_ERR_INVALID_ARG, p->lout.planar ? "planar output needs out_im" : "interleaved output: out_im must be NULL");
    const uintptr_t real = p->dtype == FFTC_C128 ? 8 : 4;
    auto aligned = [&](const void* q, bool planar) { return q == nullptr || (uintptr_t)q % (planar ? real : 2 * real) == 0; };
    if (!aligned(in_re, p->lin.planar) || !aligned(in_im, true) || !aligned(out_re, p->lout.planar) ||
        !aligned(out_im, true))
        return fail(FFTC_ERR_INVALID_ARG, "pointer not aligned to its element type");
    const bool touch = in_re == out_re || (in_im && (in_im == out_re || in_im == out_im)) || (out_im && in_re == out_im);
    if (touch) {
        const bool same = in_re == out_re && in_im == out_im && p->lin.planar == p->lout.planar &&
                          p->lin.stride == p->lout.stride && p->lin.dist == p->lout.dist;
        if (!same) return fail(FFTC_ERR_INVALID_ARG, "in place needs equal layouts and equal pointers");
    }
    return launch_layout(p, in_re, in_im, out_re, out_im, p->batch, static_cast<hipStream_t>(stream));
}

fftc_status fftc_plan_formula(const char* formula, int64_t batch, int direction, int dtype, int flags,
                              fftc_plan_t* plan_out) {
    try {
        clear_error();
        if (!plan_out) return fail(FFTC_ERR_INVALID_ARG, "plan_out is NULL");
        *plan_out = nullptr;
        if (!formula) return fail(FFTC_ERR_INVALID_ARG, "formula is NULL");
        if (direction != FFTC_FORWARD && direction != FFTC_INVERSE)
            return fail(FFTC_ERR_INVALID_ARG, "direction must be FFTC_FORWARD (-1) or FFTC_INVERSE (+1)");
        if (dtype != FFTC_C64 && dtype != FFTC_C128)
            return fail(FFTC_ERR_INVALID_ARG, "formula plans take FFTC_C64 or FFTC_C128");
        if (batch < 1) return fail(FFTC_ERR_INVALID_ARG, "batch must be >= 1");
        FormulaProgram prog;
        fftc_status st = compile_formula(formula, flags, dtype, &prog);
        if (st != FFTC_OK) return st;
        if (batch >= (int64_t(1) << 31) / prog.dim)
            return fail(FFTC_ERR_INVALID_ARG, "formula plans take batch * dim < 2^31 elements");
        fftc_plan_s* p = new (std::nothrow) fftc_plan_s();
        if (!p) return fail(FFTC_ERR_OUT_OF_MEMORY, "host allocation failed");
        p->n = prog.dim;
        p->batch = batch;
        p->direction = direction;
        p->dtype = dtype;
        p->variant = FFTC_VARIANT_FORMULA;
        hipGetDevice(&p->device);
        if (prog.folded) {
            p->fold_n = prog.fold_n;
            p->fold_p = prog.fold_p;
            st = plan_impl(prog.fold_n, batch * prog.fold_p, direction, dtype, nullptr, 0, &p->inner);
        } else {
            p->fold_p = 1;
            p->formula_passes = (int)prog.passes.size();
            st = formula_prepare(prog, dtype, batch, flags, &p->formula, &p->tw_bytes, &p->scratch_bytes,
                                 &p->formula_kernels);
            if (st == FFTC_OK) p->formula_lds = p->scratch_bytes == 0;  // one LDS-resident kernel
        }
        if (st != FFTC_OK) {
            std::string keep = t_last_error;
            fftc_destroy_plan(p);
            t_last_error = keep;
            return st;
        }
        *plan_out = p;
        return FFTC_OK;
    } catch (...) {
        return fail(FFTC_ERR_INTERNAL, "exception in fftc_plan_formula");
    }
}

fftc_status fftc_formula_lower(const char* formula, int flags, int dtype, int64_t* dim, char* text,
                               size_t text_len) {
    try {
        clear_error();
        if (!formula || !dim) return fail(FFTC_ERR_INVALID_ARG, "NULL argument");
        if (dtype != FFTC_C64 && dtype != FFTC_C128)
            return fail(FFTC_ERR_INVALID_ARG, "formula plans take FFTC_C64 or FFTC_C128");
        FormulaProgram prog;
        fftc_status st = compile_formula(formula, flags, dtype, &prog);
        if (st != FFTC_OK) return st;
        *dim = prog.dim;
        if (text && text_len) {
            const std::string d = describe_formula(prog);
            const size_t n = std::min(d.size(), text_len - 1);
            memcpy(text, d.data(), n);
            text[n] = 0;
        }
        return FFTC_OK;
    } catch (...) {
        return fail(FFTC_ERR_INTERNAL, "exception in fftc_formula_lower");
    }
}

int64_t fftc_formula_max_lds_dim(int dtype) { return formula_lds_max_dim(dtype); }

fftc_status fftc_factorize(int64_t n, int dtype, int* radices, int max_count, int* count, int64_t* split_m) {
    clear_error();
    if (!count || (max_count > 0 && !radices)) return fail(FFTC_ERR_INVALID_ARG, "NULL argument");
    if (dtype != FFTC_C64 && dtype != FFTC_C128) return fail(FFTC_ERR_INVALID_ARG, "bad dtype");
    if (n < 1 || n > max_total_n(dtype) || !is_7smooth(n)) return fail(FFTC_ERR_UNSUPPORTED_SIZE, "unsupported n");
    std::vector<int> rs;
    int64_t m = 0, k = 0;
    if (single_kernel(n, dtype)) {
        if (n > 1) rs = choose_radices(n, dtype);
    } else {
        if (!two_pass_split(n, dtype, &m, &k)) return fail(FFTC_ERR_UNSUPPORTED_SIZE, "no split");
        rs = choose_radices(m, dtype);
        auto r2 = choose_radices(k, dtype);
        rs.insert(rs.end(), r2.begin(), r2.end());
    }
    if (split_m) *split_m = m;
    *count = (int)rs.size();
    if ((int)rs.size() > max_count) return fail(FFTC_ERR_INVALID_ARG, "max_count too small");
    for (size_t i = 0; i < rs.size(); ++i) radices[i] = rs[i];
    return FFTC_OK;
}

int64_t fftc_max_single_n(int dtype) { return max_single_n(dtype); }

fftc_status fftc_copy(const void* in, void* out, size_t bytes, void* stream) {
    try {
        if (bytes == 0) return FFTC_OK;
        if (!in || !out) return fail(FFTC_ERR_INVALID_ARG, "NULL pointer");
        if ((((uintptr_t)in | (uintptr_t)out | (uintptr_t)bytes) & 15) != 0)
            return fail(FFTC_ERR_INVALID_ARG, "fftc_copy needs 16-byte aligned pointers and a multiple of 16 bytes");
        const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
        if (a < b + bytes && b < a + bytes) return fail(FFTC_ERR_INVALID_ARG, "fftc_copy ranges overlap");
        return launch_copy16(in, out, (int64_t)(bytes / 16), static_cast<hipStream_t>(stream));
    } catch (...) {
        return fail(FFTC_ERR_INTERNAL, "exception in fftc_copy");
    }
}

int fftc_compiled_count(int dtype) {
    if (dtype != FFTC_C64 && dtype != FFTC_C128) return 0;
    int total = 0;
    for (int part = 0; part < kSpecParts; ++part) {
        int cnt = 0;
        spec_part(dtype, part, &cnt);
        total += cnt;
    }
    int wide = 0;
    wide_table(dtype, &wide);
    return total + wide;
}

fftc_status fftc_compiled_entry(int dtype, int i, int64_t* n, int* radices, int max_count, int* count) {
    clear_error();
    if (!n || !radices || !count) return fail(FFTC_ERR_INVALID_ARG, "NULL argument");
    if (dtype != FFTC_C64 && dtype != FFTC_C128) return fail(FFTC_ERR_INVALID_ARG, "bad dtype");
    int base = 0;
    for (int part = 0; part < kSpecParts; ++part) {
        int cnt = 0;
        const SpecEntry* tab = spec_part(dtype, part, &cnt);
        if (i >= base && i < base + cnt) {
            const SpecEntry& e = tab[i - base];
            if (e.nr > max_count) return fail(FFTC_ERR_INVALID_ARG, "max_count too small");
            *n = e.n;
            *count = e.nr;
            for (int q = 0; q < e.nr; ++q) radices[q] = e.radices[q];
            return FFTC_OK;
        }
        base += cnt;
    }
    int wide = 0;
    const SpecEntry* tab = wide_table(dtype, &wide);
    if (i >= base && i < base + wide) {
        const SpecEntry& e = tab[i - base];
        if (e.nr > max_count) return fail(FFTC_ERR_INVALID_ARG, "max_count too small");
        *n = e.n;
        *count = e.nr;
        for (int q = 0; q < e.nr; ++q) radices[q] = e.radices[q];
        return FFTC_OK;
    }
    return fail(FFTC_ERR_INVALID_ARG, "index out of range");
}

fftc_status fftc_candidates(int64_t n, int* radices, int* lens, int max_lists, int* nlists) {
    clear_error();
    if (!nlists || (max_lists > 0 && (!radices || !lens))) return fail(FFTC_ERR_INVALID_ARG, "NULL argument");
    if (n < 2 || !is_7smooth(n) || n > (int64_t(1) << 20)) return fail(FFTC_ERR_UNSUPPORTED_SIZE, "unsupported n");
    auto c = radix_candidates(n, 12);
    *nlists = (int)c.size();
    for (int i = 0; i < (int)c.size() && i < max_lists; ++i) {
        lens[i] = (int)c[i].size();
        for (size_t q = 0; q < c[i].size(); ++q) radices[i * 16 + q] = c[i][q];
    }
    return FFTC_OK;
}

}  // extern "C"
