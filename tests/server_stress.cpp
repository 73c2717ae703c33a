// Multi-threaded stress of the serving runtime with the mock executor (no
// device use): client threads submit, one thread polls and releases, one
// reads the statistics.  Checks that every request completes exactly once
// with FFTC_OK and that the arena never holds more than the budget.  Built
// and run by test_server_race.py, also under ThreadSanitizer.
#include <stdio.h>

#include <atomic>
#include <random>
#include <thread>
#include <vector>

#include "fftc.h"

int main(int argc, char** argv) {
    const int clients = argc > 1 ? atoi(argv[1]) : 4;
    const int per = argc > 2 ? atoi(argv[2]) : 1500;
    const size_t budget = 8u << 20;
    fftc_server_config cfg{};
    cfg.budget_bytes = budget;
    cfg.n_streams = 2;
    cfg.max_inflight = 6;
    cfg.executor = FFTC_EXECUTOR_MOCK;
    cfg.mock_ns_per_mb = 20000;
    if (fftc_server_start(&cfg) != FFTC_OK) {
        fprintf(stderr, "start: %s\n", fftc_last_error());
        return 2;
    }
    const int total = clients * per;
    std::vector<std::atomic<int>> seen(total);
    for (auto& s : seen) s = 0;
    std::atomic<int> completed{0}, bad{0};
    std::atomic<bool> stop_stats{false};
    std::vector<std::thread> th;
    for (int c = 0; c < clients; ++c)
        th.emplace_back([&, c] {
            std::mt19937 g(c + 1);
            for (int i = 0; i < per; ++i) {
                fftc_request r{};
                r.n = int64_t(1) << (6 + g() % 8);
                r.batch = 1 + g() % 32;
                r.direction = (g() & 1) ? FFTC_FORWARD : FFTC_INVERSE;
                r.dtype = FFTC_C64;
                r.in = reinterpret_cast<const void*>(uintptr_t(0x10000));  // never read by the mock
                r.tag = uint64_t(c) * per + i;
                r.arrival_ns = fftc_now_ns();
                if (fftc_submit(&r) != FFTC_OK) bad++;
            }
        });
    std::thread poller([&] {
        fftc_completion buf[64];
        while (completed.load() < total) {
            int k = 0;
            if (fftc_poll(buf, 64, &k) != FFTC_OK) bad++;
            for (int i = 0; i < k; ++i) {
                if (buf[i].status != FFTC_OK || buf[i].tag >= (uint64_t)total || seen[buf[i].tag]++ != 0) bad++;
                if (!(buf[i].arrival_ns <= buf[i].admit_ns && buf[i].admit_ns <= buf[i].start_ns &&
                      buf[i].start_ns <= buf[i].done_ns))
                    bad++;
                if (buf[i].out && fftc_release(buf[i].out) != FFTC_OK) bad++;
                completed++;
            }
            if (!k) std::this_thread::yield();
        }
    });
    std::thread stats([&] {
        while (!stop_stats.load()) {
            fftc_server_stats s{};
            if (fftc_server_stats_get(&s) != FFTC_OK || s.bytes_in_use > budget || s.peak_bytes > budget) bad++;
            std::this_thread::yield();
        }
    });
    for (auto& t : th) t.join();
    poller.join();
    stop_stats = true;
    stats.join();
    fftc_server_stats s{};
    fftc_server_stats_get(&s);
    const fftc_status st = fftc_server_stop(1);
    printf("requests %d completed %d bad %d peak %zu/%zu stop %d\n", total, completed.load(), bad.load(),
           s.peak_bytes, budget, (int)st);
    return (bad.load() == 0 && completed.load() == total && st == FFTC_OK && s.completed == total) ? 0 : 1;
}
