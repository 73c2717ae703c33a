// Serving runtime: FFT requests of different lengths and batch sizes are
// taken as they arrive and run with continuous batching on one GPU.
//
//  - Plans (and their twiddle tables) stay resident, one per (n, direction,
//    dtype), built once for the largest batch the budget can hold; requests
//    run the first `batch` transforms of the plan.
//  - Outputs come from one device arena of `budget_bytes` (first fit with
//    coalescing, 256-byte granules).  A request is admitted in arrival order
//    when its output fits in the free arena and an in-flight slot is free;
//    otherwise it -- and everything behind it -- waits (FIFO, so no request
//    starves).  A request larger than the whole budget is refused at submit.
//  - Each admitted request is launched at once on the next stream of a pool,
//    so work admitted while earlier requests are still on the GPU overlaps
//    with them; an event per request marks its completion, which the
//    dispatcher observes and publishes with arrival / admit / start / done
//    timestamps.  The output stays owned by the client until fftc_release.
//  - With `fuse`, the requests admitted in one round that share
//    (n, direction, dtype) form one step: a single launch of the
//    several-requests kernel (each request keeps its own input, output and
//    batch), with every request's event recorded after it.
//  - With `hold_at` = k > 0, a round admitted while k or more requests are
//    on the device waits (with its slots and outputs) and launches with the
//    later rounds as soon as fewer than k are: under load, rounds grow and
//    more requests share a launch; below it, nothing waits.
//  - A host-only mock executor (no HIP calls, no computation) replaces the
//    device for testing admission and scheduling on a CPU.
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "plan.h"
#include "split16.h"

namespace fftc {

extern thread_local bool t_plan_no_scratch;

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

namespace {

constexpr size_t kGranule = 256;

// First-fit allocator over [0, cap) with coalescing of free neighbours.
class Arena {
   public:
    void reset(size_t cap) {
        cap_ = cap;
        free_.clear();
        if (cap) free_[0] = cap;
        used_ = peak_ = 0;
    }
    bool alloc(size_t sz, size_t* off) {
        sz = round(sz);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= sz) {
                *off = it->first;
                const size_t rest = it->second - sz;
                const size_t at = it->first + sz;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += sz;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t sz) {
        sz = round(sz);
        used_ -= sz;
        auto it = free_.emplace(off, sz).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t cap() const { return cap_; }
    static size_t round(size_t s) { return (s + kGranule - 1) / kGranule * kGranule; }

   private:
    size_t cap_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

struct Pending {
    fftc_request r;
    size_t bytes;
};

struct InFlight {
    Pending q;
    size_t off;
    void* out;
    int64_t admit_ns, start_ns, mock_done_ns;
    hipEvent_t ev;
    fftc_status status;
    int stream;  // index of the stream it was launched on (-1: none)
};

size_t elem_bytes(int dtype) { return dtype == FFTC_C128 ? 16 : 8; }

class Server {
   public:
    fftc_status start(const fftc_server_config& cfg) {
        cfg_ = cfg;
        mock_ = cfg.executor == FFTC_EXECUTOR_MOCK;
        if (cfg_.n_streams < 1) cfg_.n_streams = 1;
        if (cfg_.max_inflight < 1) cfg_.max_inflight = 1;
        arena_.reset(cfg.budget_bytes / kGranule * kGranule);
        stats_ = fftc_server_stats{};
        stats_.budget_bytes = arena_.cap();
        fused_launches_ = 0;
        fused_requests_ = 0;
        if (cfg_.tune_db && *cfg_.tune_db && tune_load_file(cfg_.tune_db) < 0)
            return fail(FFTC_ERR_INVALID_ARG, std::string("cannot read tune_db ") + cfg_.tune_db);
        if (!mock_) {
            FFTC_HIP_TRY(hipGetDevice(&device_));
            fftc_status sa = dev_malloc(&base_, std::max<size_t>(arena_.cap(), kGranule), "hipMalloc(server arena)");
            if (sa != FFTC_OK) return sa;
            // touch the whole arena once now (about 13 ms for 64 GiB), so no
            // request pays the first use of its pages
            FFTC_HIP_TRY(hipMemset(base_, 0, std::max<size_t>(arena_.cap(), kGranule)));
            streams_.resize(cfg_.n_streams);
            for (auto& s : streams_) FFTC_HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            for (int i = 0; i < cfg_.max_inflight; ++i) {
                hipEvent_t e;
                FFTC_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
                events_.push_back(e);
            }
        } else {
            base_ = reinterpret_cast<void*>(uintptr_t(1) << 40);  // fake, never dereferenced
        }
        stop_ = false;
        drain_ = true;
        th_ = std::thread([this] { loop(); });
        log_line("server start: budget %zu B, %d streams, %d in flight, %s executor, fuse %d", arena_.cap(),
                 cfg_.n_streams, cfg_.max_inflight, mock_ ? "mock" : "GPU", cfg_.fuse);
        return FFTC_OK;
    }

    // Build the plan, and on the GPU run it once (and the several-requests
    // kernel of its length) on a scratch pair of its own, so the first request
    // does not pay for loading the kernels' code.
    fftc_status prepare(int64_t n, int direction, int dtype, int64_t max_batch) {
        std::lock_guard<std::mutex> g(plan_mu_);
        fftc_plan_t p = nullptr;
        fftc_status st = get_plan(n, direction, dtype, max_batch, &p);
        if (st != FFTC_OK || mock_) return st;
        const size_t bytes = (size_t)n * elem_bytes(dtype);
        void* buf = nullptr;
        hipStream_t s = nullptr;
        st = dev_malloc(&buf, 2 * bytes, "hipMalloc(prepare buffer)");
        if (st != FFTC_OK) return st;
        hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipMemsetAsync(buf, 0, 2 * bytes, s);
        if (e == hipSuccess) {
            void* out = static_cast<char*>(buf) + bytes;
            st = fftc_execute_batch(p, buf, out, 1, s);
            const SpecEntry* se = (p->variant == FFTC_VARIANT_SINGLE_SPECIALISED && p->spec && !p->has_layout &&
                                   !p->order)
                                      ? find_serve(p->dtype, p->n, p->radices)
                                      : nullptr;
            if (st == FFTC_OK && cfg_.fuse && se) {
                ReqList l{};
                l.count = 1;
                l.in[0] = buf;
                l.out[0] = out;
                l.batch[0] = 1;
                l.gstart[1] = 1;
                st = launch_reqs(se, direction == FFTC_INVERSE, l, 1, p->tw, s);
            }
            e = hipStreamSynchronize(s);
        }
        if (s) (void)hipStreamDestroy(s);
        (void)hipFree(buf);
        if (e != hipSuccess) return fail_hip(e, "server prepare");
        return st;
    }

    fftc_status submit(const fftc_request& r) {
        if (r.n < 1 || r.batch < 1 || !r.in) return fail(FFTC_ERR_INVALID_ARG, "bad request (n, batch, in)");
        if (r.direction != FFTC_FORWARD && r.direction != FFTC_INVERSE) return fail(FFTC_ERR_INVALID_ARG, "bad direction");
        if (r.dtype != FFTC_C64 && r.dtype != FFTC_C128 && !is_split_dtype(r.dtype))
            return fail(FFTC_ERR_INVALID_ARG, "bad dtype");
        if (!is_7smooth(r.n) || r.n > max_total_n(r.dtype)) return fail(FFTC_ERR_UNSUPPORTED_SIZE, "unsupported n");
        const size_t bytes = Arena::round((size_t)r.n * (size_t)r.batch * elem_bytes(r.dtype));
        std::lock_guard<std::mutex> g(mu_);
        if (stop_) return fail(FFTC_ERR_SHUTDOWN, "server is stopping");
        if (bytes > arena_.cap()) {
            ++stats_.rejected;
            return fail(FFTC_ERR_TOO_LARGE, "request output exceeds the memory budget");
        }
        incoming_.push_back(Pending{r, bytes});
        ++stats_.submitted;
        wakes_.fetch_add(1, std::memory_order_release);
        cv_.notify_one();
        return FFTC_OK;
    }

    int poll(fftc_completion* out, int max) {
        std::lock_guard<std::mutex> g(mu_);
        int k = 0;
        while (k < max && !done_.empty()) {
            out[k++] = done_.front();
            done_.pop_front();
        }
        return k;
    }

    fftc_status release(void* out) {
        std::lock_guard<std::mutex> g(mu_);
        auto it = live_.find(out);
        if (it == live_.end()) return fail(FFTC_ERR_INVALID_ARG, "pointer is not a live server output");
        arena_.release(it->second.first, it->second.second);
        live_.erase(it);
        stats_.bytes_in_use = arena_.used();
        wakes_.fetch_add(1, std::memory_order_release);
        cv_.notify_one();
        return FFTC_OK;
    }

    // Stop taking requests; with drain, queued requests still run (their
    // outputs must be released by the client meanwhile if memory is short),
    // else they complete with FFTC_ERR_SHUTDOWN.  Waits for the GPU work.
    fftc_status stop(bool drain) {
        log_line("server stop (%s)", drain ? "drain" : "cancel queued");
        {
            std::lock_guard<std::mutex> g(mu_);
            stop_ = true;
            drain_ = drain;
            wakes_.fetch_add(1, std::memory_order_release);
            cv_.notify_one();
        }
        if (th_.joinable()) th_.join();
        fftc_status st = FFTC_OK;
        {
            std::lock_guard<std::mutex> g(plan_mu_);
            for (auto& kv : plans_) fftc_destroy_plan(kv.second);
            plans_.clear();
        }
        if (!mock_) {
            for (auto e : events_) (void)hipEventDestroy(e);
            for (auto s : streams_) (void)hipStreamDestroy(s);
            if (base_ && hipFree(base_) != hipSuccess) st = fail(FFTC_ERR_HIP, "hipFree(arena)");
        }
        events_.clear();
        streams_.clear();
        base_ = nullptr;
        live_.clear();
        return st;
    }

    void stats(fftc_server_stats* s) {
        std::lock_guard<std::mutex> g(mu_);
        stats_.bytes_in_use = arena_.used();
        stats_.peak_bytes = arena_.peak();
        stats_.pending = (int)(incoming_.size() + pending_.size());
        stats_.inflight = running_count_;
        stats_.fused_launches = fused_launches_.load();
        stats_.fused_requests = fused_requests_.load();
        stats_.plan_bytes = plan_bytes_.load();
        *s = stats_;
    }

   private:
    // plan cache; plan_mu_ held.  One plan per (n, direction, dtype), built
    // for the largest batch the budget can hold (a longer request is refused
    // at submit), so no request ever needs a bigger one: a plan's device
    // memory (its twiddle tables; the server never runs in place, so no
    // scratch) does not depend on its batch.
    fftc_status get_plan(int64_t n, int direction, int dtype, int64_t batch, fftc_plan_t* out) {
        const auto key = std::make_tuple(n, direction, dtype);
        auto it = plans_.find(key);
        if (it != plans_.end()) {
            if (it->second->batch < batch) return fail(FFTC_ERR_TOO_LARGE, "request batch beyond the budget");
            *out = it->second;
            return FFTC_OK;
        }
        int64_t cap = (int64_t)(arena_.cap() / ((size_t)n * elem_bytes(dtype)));
        cap = std::min<int64_t>(std::max<int64_t>({cap, batch, 1}), std::min<int64_t>((int64_t(1) << 40) / n, 0x7fffffff));
        fftc_plan_t p = nullptr;
        t_plan_no_scratch = true;  // the server never runs in place
        fftc_status st = fftc_plan(n, cap, direction, dtype, &p);
        t_plan_no_scratch = false;
        if (st != FFTC_OK) return st;
        plans_[key] = p;
        plan_bytes_ += p->tw_bytes + p->scratch_bytes;
        *out = p;
        return FFTC_OK;
    }

    // mu_ held by caller for state; launches outside the lock are fine since
    // only this thread touches streams, events and plans
    fftc_status launch(InFlight& f, int slot) {
        f.start_ns = now_ns();
        if (mock_) {
            const double mb = (double)f.q.bytes / (1 << 20);
            f.mock_done_ns = f.start_ns + (int64_t)(cfg_.mock_ns_per_mb * mb);
            return FFTC_OK;
        }
        fftc_plan_t p = nullptr;
        {
            std::lock_guard<std::mutex> g(plan_mu_);
            fftc_status st = get_plan(f.q.r.n, f.q.r.direction, f.q.r.dtype, f.q.r.batch, &p);
            if (st != FFTC_OK) return st;
        }
        const int si = next_stream_;
        hipStream_t s = streams_[si];
        next_stream_ = (next_stream_ + 1) % (int)streams_.size();
        fftc_status st = fftc_execute_batch(p, f.q.r.in, f.out, f.q.r.batch, s);
        if (st != FFTC_OK) return st;
        f.stream = si;
        f.ev = events_[slot];
        hipError_t e = hipEventRecord(f.ev, s);
        if (e != hipSuccess) return fail_hip(e, "hipEventRecord");
        return FFTC_OK;
    }

    // One step for requests of one (n, direction, dtype): fused launches of
    // up to kMaxFused requests when the plan's list has a several-requests
    // kernel; returns false (nothing launched) when it has none.
    bool launch_fused(std::vector<std::pair<InFlight, int>*>& grp) {
        const fftc_request& r0 = grp[0]->first.q.r;
        int64_t maxb = 0;
        for (auto* g : grp) maxb = std::max(maxb, g->first.q.r.batch);
        fftc_plan_t p = nullptr;
        {
            std::lock_guard<std::mutex> g(plan_mu_);
            if (get_plan(r0.n, r0.direction, r0.dtype, maxb, &p) != FFTC_OK) return false;
        }
        if (p->variant != FFTC_VARIANT_SINGLE_SPECIALISED || !p->spec || p->has_layout || p->order) return false;
        const SpecEntry* e = find_serve(p->dtype, p->n, p->radices);
        if (!e || e->tpt != p->spec->tpt || e->t != p->spec->t) return false;
        for (size_t c0 = 0; c0 < grp.size(); c0 += kMaxFused) {
            const size_t c1 = std::min(grp.size(), c0 + kMaxFused);
            ReqList l{};
            l.count = (int)(c1 - c0);
            int64_t groups = 0;
            for (size_t i = c0; i < c1; ++i) {
                InFlight& f = grp[i]->first;
                l.in[i - c0] = f.q.r.in;
                l.out[i - c0] = f.out;
                l.batch[i - c0] = f.q.r.batch;
                l.gstart[i - c0] = groups;
                groups += (f.q.r.batch + e->t - 1) / e->t;
            }
            l.gstart[l.count] = groups;
            const int si = next_stream_;
            hipStream_t s = streams_[si];
            next_stream_ = (next_stream_ + 1) % (int)streams_.size();
            const int64_t t0 = now_ns();
            fftc_status st = launch_reqs(e, r0.direction == FFTC_INVERSE, l, groups, p->tw, s);
            ++fused_launches_;
            for (size_t i = c0; i < c1; ++i) {
                InFlight& f = grp[i]->first;
                f.start_ns = t0;
                f.status = st;
                if (st != FFTC_OK) continue;
                f.ev = events_[grp[i]->second];
                f.stream = si;
                hipError_t err = hipEventRecord(f.ev, s);
                if (err != hipSuccess) f.status = fail_hip(err, "hipEventRecord");
            }
        }
        return true;
    }

    void launch_round(std::vector<std::pair<InFlight, int>>& to_launch) {
        if (to_launch.empty()) return;
        Range range("fftc_server_round");
        if (!cfg_.fuse || mock_ || to_launch.size() < 2) {
            for (auto& fl : to_launch) fl.first.status = launch(fl.first, fl.second);
            return;
        }
        std::map<std::tuple<int64_t, int, int>, std::vector<std::pair<InFlight, int>*>> groups;
        for (auto& fl : to_launch)
            groups[std::make_tuple(fl.first.q.r.n, fl.first.q.r.direction, fl.first.q.r.dtype)].push_back(&fl);
        for (auto& kv : groups) {
            if (kv.second.size() >= 2 && launch_fused(kv.second)) {
                fused_requests_ += (int64_t)kv.second.size();
                continue;
            }
            for (auto* fl : kv.second) fl->first.status = launch(fl->first, fl->second);
        }
    }

    bool finished(InFlight& f) {
        if (f.status != FFTC_OK) return true;
        if (mock_) return now_ns() >= f.mock_done_ns;
        hipError_t e = hipEventQuery(f.ev);
        if (e == hipErrorNotReady) return false;
        if (e != hipSuccess) f.status = FFTC_ERR_HIP;
        return true;
    }

    void loop() {
        if (!mock_) (void)hipSetDevice(device_);
        std::vector<int> free_slots;
        for (int i = cfg_.max_inflight - 1; i >= 0; --i) free_slots.push_back(i);
        // running work: per stream in launch order (a stream completes its
        // work in order, so only the oldest entry of each needs an event
        // query); the mock executor's work and failed launches in `other`
        std::vector<std::deque<std::pair<InFlight, int>>> by_stream(std::max<size_t>(streams_.size(), 1));
        std::vector<std::pair<InFlight, int>> other;
        std::vector<std::pair<InFlight, int>> held;  // admitted, waiting for the device to drain (hold_at)
        auto n_running = [&]() {
            size_t k = other.size();
            for (auto& q : by_stream) k += q.size();
            return k;
        };
        for (;;) {
            bool progressed = false;
            std::vector<std::pair<InFlight, int>> to_launch;
            bool stopping, drain;
            {
                std::unique_lock<std::mutex> lk(mu_);
                while (!incoming_.empty()) {
                    pending_.push_back(incoming_.front());
                    incoming_.pop_front();
                }
                stopping = stop_;
                drain = drain_;
                if (stopping && !drain) {
                    for (auto& q : pending_) {
                        fftc_completion c{};
                        c.tag = q.r.tag;
                        c.status = FFTC_ERR_SHUTDOWN;
                        c.arrival_ns = q.r.arrival_ns;
                        c.done_ns = now_ns();
                        done_.push_back(c);
                        ++stats_.cancelled;
                    }
                    pending_.clear();
                }
                // admission in arrival order: the head waits for room
                while (!pending_.empty() && !free_slots.empty()) {
                    size_t off = 0;
                    if (fault_hit()) {  // an injected allocation failure fails this request only
                        fftc_completion c{};
                        c.tag = pending_.front().r.tag;
                        c.status = FFTC_ERR_OUT_OF_MEMORY;
                        c.arrival_ns = pending_.front().r.arrival_ns;
                        c.admit_ns = c.start_ns = c.done_ns = now_ns();
                        c.n = pending_.front().r.n;
                        c.batch = pending_.front().r.batch;
                        pending_.pop_front();
                        done_.push_back(c);
                        ++stats_.completed;
                        ++stats_.failed;
                        continue;
                    }
                    if (!arena_.alloc(pending_.front().bytes, &off)) break;
                    InFlight f{};
                    f.stream = -1;
                    f.q = pending_.front();
                    pending_.pop_front();
                    f.off = off;
                    f.out = static_cast<char*>(base_) + off;
                    f.admit_ns = now_ns();
                    f.status = FFTC_OK;
                    live_[f.out] = {off, f.q.bytes};
                    to_launch.emplace_back(f, free_slots.back());
                    free_slots.pop_back();
                    ++stats_.admitted;
                }
                running_count_ = (int)(n_running() + held.size() + to_launch.size());
                stats_.max_inflight_seen = std::max<int>(stats_.max_inflight_seen, running_count_);
            }
            // continuous batching under load: while hold_at or more requests
            // are on the device, admitted requests wait (holding their slots
            // and outputs) and launch as one round when it drains below that,
            // so more of them share a length and run fused
            if (cfg_.hold_at > 0 && !stopping && (int)n_running() >= cfg_.hold_at) {
                if (!to_launch.empty()) progressed = true;
                held.insert(held.end(), to_launch.begin(), to_launch.end());
                to_launch.clear();
            } else if (!held.empty()) {
                to_launch.insert(to_launch.begin(), held.begin(), held.end());  // arrival order
                held.clear();
            }
            launch_round(to_launch);
            for (auto& fl : to_launch) {
                if (!mock_ && fl.first.status == FFTC_OK && fl.first.stream >= 0)
                    by_stream[fl.first.stream].push_back(fl);
                else
                    other.push_back(fl);
                progressed = true;
            }
            // completions
            std::vector<fftc_completion> fin;
            std::vector<void*> failed_out;
            auto complete = [&](std::pair<InFlight, int>& r) {
                InFlight& f = r.first;
                fftc_completion c{};
                c.tag = f.q.r.tag;
                c.status = f.status;
                c.out = f.status == FFTC_OK ? f.out : nullptr;
                c.arrival_ns = f.q.r.arrival_ns;
                c.admit_ns = f.admit_ns;
                c.start_ns = f.start_ns;
                c.done_ns = now_ns();
                c.n = f.q.r.n;
                c.batch = f.q.r.batch;
                if (f.status != FFTC_OK) failed_out.push_back(f.out);
                fin.push_back(c);
                free_slots.push_back(r.second);
                progressed = true;
            };
            for (auto& q : by_stream) {
                while (!q.empty() && finished(q.front().first)) {
                    complete(q.front());
                    q.pop_front();
                }
            }
            for (size_t i = 0; i < other.size();) {
                if (finished(other[i].first)) {
                    complete(other[i]);
                    other[i] = other.back();
                    other.pop_back();
                } else {
                    ++i;
                }
            }
            {
                std::unique_lock<std::mutex> lk(mu_);
                for (void* o : failed_out) {  // a failed launch gives its output back
                    auto it = live_.find(o);
                    if (it != live_.end()) {
                        arena_.release(it->second.first, it->second.second);
                        live_.erase(it);
                    }
                }
                for (auto& c : fin) {
                    done_.push_back(c);
                    ++stats_.completed;
                    if (c.status != FFTC_OK) ++stats_.failed;
                }
                const size_t nrun = n_running();
                running_count_ = (int)nrun;
                if (stop_ && nrun == 0 && held.empty() && incoming_.empty() && pending_.empty()) break;
                // idle, or the queue head waits for memory or a slot: sleep
                // until a submit, release or stop (or a short timeout)
                if (!progressed && nrun == 0) {
                    // idle: poll briefly for a submit, release or stop before
                    // sleeping, so a request arriving soon after does not pay
                    // for waking this thread
                    const uint64_t seen = wakes_.load(std::memory_order_acquire);
                    lk.unlock();
                    const int64_t t0 = now_ns();
                    while (wakes_.load(std::memory_order_acquire) == seen && now_ns() - t0 < kIdleSpinNs)
                        std::this_thread::yield();
                    lk.lock();
                    if (wakes_.load(std::memory_order_acquire) == seen)
                        cv_.wait_for(lk, std::chrono::milliseconds(2));
                }
            }
            // work on the GPU: poll its events without a timed sleep
            if (!progressed && n_running() > 0) std::this_thread::yield();
        }
    }

    fftc_server_config cfg_{};
    bool mock_ = false;
    int device_ = 0;
    void* base_ = nullptr;
    Arena arena_;
    std::vector<hipStream_t> streams_;
    std::vector<hipEvent_t> events_;
    int next_stream_ = 0;
    std::thread th_;
    std::mutex mu_, plan_mu_;
    std::condition_variable cv_;
    bool stop_ = false, drain_ = true;
    std::deque<Pending> incoming_, pending_;
    int running_count_ = 0;
    std::deque<fftc_completion> done_;
    std::unordered_map<void*, std::pair<size_t, size_t>> live_;
    std::map<std::tuple<int64_t, int, int>, fftc_plan_t> plans_;
    std::atomic<size_t> plan_bytes_{0};  // device memory of the resident plans
    fftc_server_stats stats_{};
    std::atomic<int64_t> fused_launches_{0}, fused_requests_{0};  // written by the dispatcher only
    std::atomic<uint64_t> wakes_{0};  // submits, releases and stops, for the dispatcher's idle poll
    static constexpr int64_t kIdleSpinNs = 100000;  // idle poll before sleeping: 100 us
};

std::mutex g_server_mu;
Server* g_server = nullptr;
bool g_server_stopping = false;

}  // namespace
}  // namespace fftc

using namespace fftc;

extern "C" {

int64_t fftc_now_ns(void) { return now_ns(); }

fftc_status fftc_server_start(const fftc_server_config* cfg) {
    clear_error();
    if (!cfg) return fail(FFTC_ERR_INVALID_ARG, "cfg is NULL");
    if (cfg->executor != FFTC_EXECUTOR_GPU && cfg->executor != FFTC_EXECUTOR_MOCK)
        return fail(FFTC_ERR_INVALID_ARG, "bad executor");
    if (cfg->budget_bytes < 256) return fail(FFTC_ERR_INVALID_ARG, "budget too small");
    std::lock_guard<std::mutex> g(g_server_mu);
    if (g_server) return fail(FFTC_ERR_INVALID_ARG, "server already running");
    try {
        Server* s = new Server();
        fftc_status st = s->start(*cfg);
        if (st != FFTC_OK) {
            std::string keep = fftc_last_error();
            s->stop(false);
            delete s;
            return fail(st, keep);
        }
        g_server = s;
        return FFTC_OK;
    } catch (...) {
        return fail(FFTC_ERR_INTERNAL, "exception in fftc_server_start");
    }
}

fftc_status fftc_server_prepare(int64_t n, int direction, int dtype, int64_t max_batch) {
    clear_error();
    std::lock_guard<std::mutex> g(g_server_mu);
    if (!g_server) return fail(FFTC_ERR_SHUTDOWN, "server not running");
    return g_server->prepare(n, direction, dtype, max_batch);
}

fftc_status fftc_submit(const fftc_request* req) {
    clear_error();
    if (!req) return fail(FFTC_ERR_INVALID_ARG, "req is NULL");
    std::lock_guard<std::mutex> g(g_server_mu);
    if (!g_server) return fail(FFTC_ERR_SHUTDOWN, "server not running");
    return g_server->submit(*req);
}

fftc_status fftc_poll(fftc_completion* out, int max, int* n_out) {
    clear_error();
    if (!n_out || (max > 0 && !out)) return fail(FFTC_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(g_server_mu);
    if (!g_server) return fail(FFTC_ERR_SHUTDOWN, "server not running");
    *n_out = g_server->poll(out, max);
    return FFTC_OK;
}

fftc_status fftc_release(void* out) {
    clear_error();
    std::lock_guard<std::mutex> g(g_server_mu);
    if (!g_server) return fail(FFTC_ERR_SHUTDOWN, "server not running");
    return g_server->release(out);
}

fftc_status fftc_server_stats_get(fftc_server_stats* s) {
    clear_error();
    if (!s) return fail(FFTC_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(g_server_mu);
    if (!g_server) return fail(FFTC_ERR_SHUTDOWN, "server not running");
    g_server->stats(s);
    return FFTC_OK;
}

fftc_status fftc_server_stop(int drain) {
    clear_error();
    Server* s;
    {
        std::lock_guard<std::mutex> g(g_server_mu);
        s = g_server;
        if (!s || g_server_stopping) return fail(FFTC_ERR_SHUTDOWN, "server not running");
        g_server_stopping = true;
    }
    // the server stays reachable (poll, release) while it drains
    fftc_status st = s->stop(drain != 0);
    {
        std::lock_guard<std::mutex> g(g_server_mu);
        g_server = nullptr;
        g_server_stopping = false;
    }
    delete s;
    return st;
}

}  // extern "C"
