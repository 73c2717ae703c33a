// Autotuner: time candidate Stockham radix lists on the device and record the
// fastest in the tuning database (the planner the paper lacks, Section VI).
#include <math.h>

#include <string>

#include "plan.h"

namespace fftc {

namespace {

struct DeviceBuffers {
    void* in = nullptr;
    void* out = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~DeviceBuffers() {
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
        if (s) hipStreamDestroy(s);
        if (in) hipFree(in);
        if (out) hipFree(out);
    }
};

// Mean microseconds per launch: best of three trials of `reps` launches.
fftc_status time_plan(fftc_plan_t p, DeviceBuffers& b, int reps, double* us) {
    fftc_status st;
    for (int i = 0; i < 2; ++i)
        if ((st = fftc_execute(p, b.in, b.out, b.s)) != FFTC_OK) return st;
    double best = 1e30;
    for (int trial = 0; trial < 3; ++trial) {
        FFTC_HIP_TRY(hipEventRecord(b.e0, b.s));
        for (int i = 0; i < reps; ++i)
            if ((st = fftc_execute(p, b.in, b.out, b.s)) != FFTC_OK) return st;
        FFTC_HIP_TRY(hipEventRecord(b.e1, b.s));
        FFTC_HIP_TRY(hipEventSynchronize(b.e1));
        float ms = 0.f;
        FFTC_HIP_TRY(hipEventElapsedTime(&ms, b.e0, b.e1));
        best = std::min(best, 1000.0 * ms / reps);
    }
    *us = best;
    return FFTC_OK;
}

// a better than b: faster by more than 1%, else fewer stages, else larger
// leading radix
bool better(double ta, const std::vector<int>& a, double tb, const std::vector<int>& b) {
    if (ta < 0.99 * tb) return true;
    if (tb < 0.99 * ta) return false;
    if (a.size() != b.size()) return a.size() < b.size();
    if (!a.empty() && !b.empty() && a[0] != b[0]) return a[0] > b[0];
    return ta < tb;
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
    if (n < 2 || n > max_single_n(dtype) || !is_7smooth(n))
        return fail(FFTC_ERR_UNSUPPORTED_SIZE, "autotune takes single-kernel lengths 2.." +
                                                   std::to_string(max_single_n(dtype)));
    try {
        const size_t cs = dtype == FFTC_C128 ? 16 : 8;
        const size_t bytes = (size_t)batch * (size_t)n * cs;
        DeviceBuffers b;
        FFTC_HIP_TRY(hipMalloc(&b.in, bytes));
        FFTC_HIP_TRY(hipMalloc(&b.out, bytes));
        FFTC_HIP_TRY(hipStreamCreate(&b.s));
        FFTC_HIP_TRY(hipEventCreate(&b.e0));
        FFTC_HIP_TRY(hipEventCreate(&b.e1));
        FFTC_HIP_TRY(hipMemsetAsync(b.in, 0x3c, bytes, b.s));  // small finite values
        std::vector<int> best;
        double best_t = 0;
        for (const auto& rs : radix_candidates(n, 12)) {
            fftc_plan_t p = nullptr;
            fftc_status st = fftc_plan_radices(n, batch, FFTC_FORWARD, dtype, rs.data(), (int)rs.size(), &p);
            if (st != FFTC_OK) continue;  // list does not fit this device's limits
            double us = 0;
            st = time_plan(p, b, reps, &us);
            fftc_destroy_plan(p);
            if (st != FFTC_OK) return st;
            if (best.empty() || better(us, rs, best_t, best)) {
                best = rs;
                best_t = us;
            }
        }
        if (best.empty()) return fail(FFTC_ERR_UNSUPPORTED_SIZE, "no candidate radix list could be planned");
        tune_record(n, dtype, best, best_t * 1e-3);
        *count = (int)best.size();
        if (best_us) *best_us = best_t;
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
    if (n < 2 || n > max_single_n(dtype) || !is_7smooth(n))
        return fail(FFTC_ERR_UNSUPPORTED_SIZE, "autotune takes single-kernel lengths 2.." +
                                                   std::to_string(max_single_n(dtype)));
    try {
        const size_t cs = dtype == FFTC_C128 ? 16 : 8;
        const size_t bytes = (size_t)batch * (size_t)n * cs;
        DeviceBuffers b;
        FFTC_HIP_TRY(hipMalloc(&b.in, bytes));
        FFTC_HIP_TRY(hipMalloc(&b.out, bytes));
        FFTC_HIP_TRY(hipStreamCreate(&b.s));
        FFTC_HIP_TRY(hipEventCreate(&b.e0));
        FFTC_HIP_TRY(hipEventCreate(&b.e1));
        FFTC_HIP_TRY(hipMemsetAsync(b.in, 0x3c, bytes, b.s));  // small finite values
        // candidates: the Stockham plan, then every compiled order for n
        std::vector<std::pair<int, int>> cands{{FFTC_ORDER_STOCKHAM, 0}};
        int cnt = 0;
        const OrderEntry* tab = order_table(dtype, &cnt);
        for (int i = 0; i < cnt; ++i)
            if (tab[i].n == n) cands.push_back({tab[i].order, tab[i].radix});
        const std::vector<int> stock = choose_radices(n, dtype);
        std::vector<double> times;
        for (const auto& c : cands) {
            fftc_plan_t p = nullptr;
            fftc_status st = c.first == FFTC_ORDER_STOCKHAM
                                 ? fftc_plan_radices(n, batch, FFTC_FORWARD, dtype, stock.data(), (int)stock.size(), &p)
                                 : fftc_plan_order(n, batch, FFTC_FORWARD, dtype, c.first, c.second, &p);
            if (st != FFTC_OK) return st;
            double t = 0;
            st = time_plan(p, b, reps, &t);
            fftc_destroy_plan(p);
            if (st != FFTC_OK) return st;
            times.push_back(t);
        }
        size_t bi = 0;  // Stockham unless another order is faster by more than 1%
        for (size_t i = 1; i < cands.size(); ++i)
            if (times[i] < 0.99 * times[bi] && (bi != 0 || times[i] < 0.99 * times[0])) bi = i;
        if (bi == 0)
            tune_record(n, dtype, stock, times[0] * 1e-3);
        else
            tune_record_order(n, dtype, cands[bi].first, cands[bi].second, times[bi] * 1e-3);
        *count = (int)cands.size();
        *best = (int)bi;
        for (int i = 0; i < (int)cands.size() && i < max; ++i) {
            orders[i] = cands[i].first;
            radices[i] = cands[i].second;
            us[i] = times[i];
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

fftc_status fftc_tune_clear(void) {
    tune_clear_all();
    return FFTC_OK;
}

}  // extern "C"
