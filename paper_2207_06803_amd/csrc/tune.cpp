// Autotuner: time candidate Stockham radix lists on the device and record the
// fastest in the tuning database (the planner the paper lacks, Section VI).
#include <math.h>

#include <algorithm>

#include <string>

#include "plan.h"

namespace fftc {

namespace {

// Candidates are timed at the HBM-bound shape: at least 2^24 elements per
// launch, launches rotating over four input/output pairs (1 GiB in all for
// complex64, past the 256 MB last-level cache), each launch timed by its own
// event pair.
constexpr int kTunePairs = 4;
constexpr int64_t kTuneMinElems = int64_t(1) << 24;

struct DeviceBuffers {
    void* in[kTunePairs] = {};
    void* out[kTunePairs] = {};
    hipStream_t s = nullptr;
    std::vector<hipEvent_t> ev;
    ~DeviceBuffers() {
        for (hipEvent_t e : ev)
            if (e) hipEventDestroy(e);
        if (s) hipStreamDestroy(s);
        for (int i = 0; i < kTunePairs; ++i) {
            if (in[i]) hipFree(in[i]);
            if (out[i]) hipFree(out[i]);
        }
    }
};

int64_t tune_batch(int64_t n, int64_t batch) { return std::max(batch, (kTuneMinElems + n - 1) / n); }

fftc_status alloc_buffers(DeviceBuffers& b, size_t bytes, int reps) {
    FFTC_HIP_TRY(hipStreamCreate(&b.s));
    for (int i = 0; i < kTunePairs; ++i) {
        fftc_status st = dev_malloc(&b.in[i], bytes, "hipMalloc(autotune input)");
        if (st == FFTC_OK) st = dev_malloc(&b.out[i], bytes, "hipMalloc(autotune output)");
        if (st != FFTC_OK) return st;
        FFTC_HIP_TRY(hipMemsetAsync(b.in[i], 0x3c, bytes, b.s));  // small finite values
    }
    b.ev.assign(reps + 1, nullptr);
    for (auto& e : b.ev) FFTC_HIP_TRY(hipEventCreate(&e));
    return FFTC_OK;
}

struct Timing {
    double med = 0, spread = 0;  // median microseconds per launch; interquartile range / median
};

fftc_status time_plan(fftc_plan_t p, DeviceBuffers& b, int reps, Timing* t) {
    fftc_status st;
    for (int i = 0; i < 2 * kTunePairs; ++i)
        if ((st = fftc_execute(p, b.in[i % kTunePairs], b.out[i % kTunePairs], b.s)) != FFTC_OK) return st;
    FFTC_HIP_TRY(hipEventRecord(b.ev[0], b.s));
    for (int i = 0; i < reps; ++i) {
        if ((st = fftc_execute(p, b.in[i % kTunePairs], b.out[i % kTunePairs], b.s)) != FFTC_OK) return st;
        FFTC_HIP_TRY(hipEventRecord(b.ev[i + 1], b.s));
    }
    FFTC_HIP_TRY(hipEventSynchronize(b.ev[reps]));
    std::vector<double> us(reps);
    for (int i = 0; i < reps; ++i) {
        float ms = 0.f;
        FFTC_HIP_TRY(hipEventElapsedTime(&ms, b.ev[i], b.ev[i + 1]));
        us[i] = 1000.0 * ms;
    }
    std::sort(us.begin(), us.end());
    auto q = [&](double f) { return us[(size_t)std::min<double>(reps - 1, std::floor(f * (reps - 1) + 0.5))]; };
    t->med = q(0.5);
    t->spread = t->med > 0 ? (q(0.75) - q(0.25)) / t->med : 0;
    return FFTC_OK;
}

// Two medians differ when they are further apart than the launches' own
// spread: twice the larger relative interquartile range, and at least 3%
// (run-to-run differences of the medians on one device reach about that).
double tie_window(const Timing& a, const Timing& b) { return std::max(0.03, 2.0 * std::max(a.spread, b.spread)); }

// The pick among timed candidates: every candidate within the tie window of
// the fastest counts as equally fast, and among those the first by `prefer`
// wins.  Choosing from the whole tied set, rather than comparing each
// candidate with the best so far, keeps the pick the same from run to run
// whenever the candidates' true times differ by less than the window.
template <class Prefer>
size_t pick(const std::vector<Timing>& t, Prefer prefer) {
    size_t f = 0;
    for (size_t i = 1; i < t.size(); ++i)
        if (t[i].med < t[f].med) f = i;
    size_t bi = f;
    for (size_t i = 0; i < t.size(); ++i)
        if (t[i].med <= (1 + tie_window(t[i], t[f])) * t[f].med && prefer(i, bi)) bi = i;
    return bi;
}

}  // namespace
}  // namespace fftc

using namespace fftc;

extern "C" {

fftc_status fftc_autotune(int64_t n, int64_t batch, int dtype, int reps, int* radices, int max_count,
                          int* count, double* best_us) {
    clear_error();
    if (!count || (max_count > 0 && !radices)) return fail(FFTC_ERR_INVALID_ARG, "NULL argument");
    if (dtype != FFTC_C64 && dtype != FFTC_C128) return fail(FFTC_ERR_INVALID_ARG, "bad dtype");
    if (batch < 1 || reps < 1) return fail(FFTC_ERR_INVALID_ARG, "batch and reps must be >= 1");
    if (reps > 100000) return fail(FFTC_ERR_INVALID_ARG, "reps must be <= 100000");
    if (n < 2 || !single_kernel(n, dtype) || !is_7smooth(n))
        return fail(FFTC_ERR_UNSUPPORTED_SIZE, "autotune takes single-kernel lengths (2.." +
                                                   std::to_string(max_single_n(dtype)) + " and the wide lengths)");
    try {
        const size_t cs = dtype == FFTC_C128 ? 16 : 8;
        const int64_t tb = tune_batch(n, batch);
        DeviceBuffers b;
        fftc_status sa = alloc_buffers(b, (size_t)tb * (size_t)n * cs, reps);
        if (sa != FFTC_OK) return sa;
        std::vector<std::vector<int>> lists;
        std::vector<Timing> times;
        // a wide length: its compiled lists (the only ones it runs)
        for (const auto& rs : n > max_single_n(dtype) ? wide_lists(n, dtype) : radix_candidates(n, 12)) {
            fftc_plan_t p = nullptr;
            fftc_status st = fftc_plan_radices(n, tb, FFTC_FORWARD, dtype, rs.data(), (int)rs.size(), &p);
            if (st != FFTC_OK) continue;  // list does not fit this device's limits
            Timing t;
            st = time_plan(p, b, reps, &t);
            fftc_destroy_plan(p);
            if (st != FFTC_OK) return st;
            lists.push_back(rs);
            times.push_back(t);
        }
        if (lists.empty()) return fail(FFTC_ERR_UNSUPPORTED_SIZE, "no candidate radix list could be planned");
        // among equally fast lists: fewer stages, then the planner's order
        const size_t bi = pick(times, [&](size_t i, size_t j) {
            return lists[i].size() != lists[j].size() ? lists[i].size() < lists[j].size() : i < j;
        });
        const std::vector<int>& best = lists[bi];
        const Timing& best_t = times[bi];
        tune_record(n, dtype, best, best_t.med * 1e-3);
        *count = (int)best.size();
        if (best_us) *best_us = best_t.med;
        if ((int)best.size() > max_count) return fail(FFTC_ERR_INVALID_ARG, "max_count too small");
        for (size_t i = 0; i < best.size(); ++i) radices[i] = best[i];
        return FFTC_OK;
    } catch (...) {
        return fail(FFTC_ERR_INTERNAL, "exception in fftc_autotune");
    }
}

fftc_status fftc_autotune_orders(int64_t n, int64_t batch, int dtype, int reps, int* orders, int* radices,
                                 double* us, int max, int* count, int* best) {
    clear_error();
    if (!count || !best || (max > 0 && (!orders || !radices || !us))) return fail(FFTC_ERR_INVALID_ARG, "NULL argument");
    if (dtype != FFTC_C64 && dtype != FFTC_C128) return fail(FFTC_ERR_INVALID_ARG, "bad dtype");
    if (batch < 1 || reps < 1) return fail(FFTC_ERR_INVALID_ARG, "batch and reps must be >= 1");
    if (reps > 100000) return fail(FFTC_ERR_INVALID_ARG, "reps must be <= 100000");
    if (n < 2 || !single_kernel(n, dtype) || !is_7smooth(n))
        return fail(FFTC_ERR_UNSUPPORTED_SIZE, "autotune takes single-kernel lengths (2.." +
                                                   std::to_string(max_single_n(dtype)) + " and the wide lengths)");
    try {
        const size_t cs = dtype == FFTC_C128 ? 16 : 8;
        const int64_t tb = std::min<int64_t>(tune_batch(n, batch), int64_t(1) << 31);
        DeviceBuffers b;
        fftc_status sa = alloc_buffers(b, (size_t)tb * (size_t)n * cs, reps);
        if (sa != FFTC_OK) return sa;
        // candidates: the Stockham plan, then every compiled order for n
        std::vector<std::pair<int, int>> cands{{FFTC_ORDER_STOCKHAM, 0}};
        int cnt = 0;
        const OrderEntry* tab = order_table(dtype, &cnt);
        for (int i = 0; i < cnt; ++i)
            if (tab[i].n == n) cands.push_back({tab[i].order, tab[i].radix});
        const std::vector<int> stock = choose_radices(n, dtype);
        std::vector<Timing> times;
        for (const auto& c : cands) {
            fftc_plan_t p = nullptr;
            fftc_status st = c.first == FFTC_ORDER_STOCKHAM
                                 ? fftc_plan_radices(n, tb, FFTC_FORWARD, dtype, stock.data(), (int)stock.size(), &p)
                                 : fftc_plan_order(n, tb, FFTC_FORWARD, dtype, c.first, c.second, &p);
            if (st != FFTC_OK) return st;
            Timing t;
            st = time_plan(p, b, reps, &t);
            fftc_destroy_plan(p);
            if (st != FFTC_OK) return st;
            times.push_back(t);
        }
        // Stockham unless another order is faster beyond the tie window
        const size_t bi = pick(times, [](size_t i, size_t j) { return i < j; });
        if (bi == 0)
            tune_record(n, dtype, stock, times[0].med * 1e-3);
        else
            tune_record_order(n, dtype, cands[bi].first, cands[bi].second, times[bi].med * 1e-3);
        *count = (int)cands.size();
        *best = (int)bi;
        for (int i = 0; i < (int)cands.size() && i < max; ++i) {
            orders[i] = cands[i].first;
            radices[i] = cands[i].second;
            us[i] = times[i].med;
        }
        return FFTC_OK;
    } catch (...) {
        return fail(FFTC_ERR_INTERNAL, "exception in fftc_autotune_orders");
    }
}

fftc_status fftc_tune_load(const char* path, int* entries) {
    clear_error();
    if (!path) return fail(FFTC_ERR_INVALID_ARG, "path is NULL");
    const int k = tune_load_file(path);
    if (k < 0) return fail(FFTC_ERR_INVALID_ARG, std::string("cannot read ") + path);
    if (entries) *entries = k;
    return FFTC_OK;
}

fftc_status fftc_tune_save(const char* path, int* entries) {
    clear_error();
    if (!path) return fail(FFTC_ERR_INVALID_ARG, "path is NULL");
    const int k = tune_save_file(path);
    if (k < 0) return fail(FFTC_ERR_INVALID_ARG, std::string("cannot write ") + path);
    if (entries) *entries = k;
    return FFTC_OK;
}

const char* fftc_tune_key(void) { return tune_key(); }

fftc_status fftc_tune_clear(void) {
    tune_clear_all();
    return FFTC_OK;
}

}  // extern "C"
