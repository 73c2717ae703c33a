// Planner: factorisation of N into Stockham radix lists, launch shapes,
// two-pass splits and the tuning database.  Host code only, no GPU calls.
//
// The choice of factorisation is the paper's central degree of freedom
// (Section I: different factorisations suit different hardware; Section VI
// names the missing planner as one cause of its performance gap).  Every
// list here multiplies to N and is a valid Stockham factorisation (Eq. 2
// applied recursively); the tuning database records which one measured
// fastest on the device.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <tuple>

#include "internal.h"

namespace fftc {

bool is_7smooth(int64_t n) {
    if (n < 1) return false;
    for (int p : {2, 3, 5, 7})
        while (n % p == 0) n /= p;
    return n == 1;
}

int64_t max_single_n(int dtype) { return dtype == FFTC_C128 ? 8192 : 16384; }

std::vector<std::vector<int>> wide_lists(int64_t n, int dtype) {
    std::vector<std::vector<int>> out;
    int cnt = 0;
    const SpecEntry* tab = wide_table(dtype, &cnt);
    for (int i = 0; i < cnt; ++i)
        if (tab[i].n == n) out.emplace_back(tab[i].radices, tab[i].radices + tab[i].nr);
    return out;
}

bool single_kernel(int64_t n, int dtype) {
    return n <= max_single_n(dtype) || (n <= max_total_n(dtype) && !wide_lists(n, dtype).empty());
}
int64_t max_total_n(int /*dtype*/) { return int64_t(1) << 20; }

static void pow2_multisets(int a, std::vector<int>& cur, int maxpart,
                           std::vector<std::vector<int>>* out) {
    if (a == 0) {
        out->push_back(cur);
        return;
    }
    for (int p = std::min(maxpart, a); p >= 1; --p) {
        cur.push_back(1 << p);
        pow2_multisets(a - p, cur, p, out);
        cur.pop_back();
    }
}

std::vector<std::vector<int>> radix_candidates(int64_t n, int max_lists) {
    std::vector<std::vector<int>> res;
    if (!is_7smooth(n)) return res;
    if (n == 1) {
        res.push_back({});
        return res;
    }
    int a = 0;
    int64_t m = n;
    while (m % 2 == 0) { m /= 2; ++a; }
    std::vector<int> odd;
    for (int p : {7, 5, 3})
        while (m % p == 0) { m /= p; odd.push_back(p); }

    std::vector<std::vector<int>> sets;  // pow2 parts, each descending
    std::vector<int> cur;
    pow2_multisets(a, cur, 4, &sets);
    size_t minparts = 1000;
    for (auto& s : sets) minparts = std::min(minparts, s.size());
    // fewest stages first; among equal counts the most balanced (largest
    // smallest radix) first
    std::stable_sort(sets.begin(), sets.end(), [](const std::vector<int>& x, const std::vector<int>& y) {
        if (x.size() != y.size()) return x.size() < y.size();
        const int mx = x.empty() ? 99 : x.back(), my = y.empty() ? 99 : y.back();
        return mx > my;
    });

    std::set<std::vector<int>> seen;
    auto push = [&](const std::vector<int>& rs) {
        if (rs.empty() || (int)res.size() >= max_lists) return;
        if ((int)rs.size() > kMaxStages) return;
        int r[kMaxStages];
        for (size_t i = 0; i < rs.size(); ++i) r[i] = rs[i];
        if (required_tpt((int)std::min<int64_t>(n, 1 << 30), r, (int)rs.size()) > 1024) return;
        if (seen.insert(rs).second) res.push_back(rs);
    };
    for (auto& s : sets) {
        if (s.size() > minparts + 1) continue;
        std::vector<int> asc(s.rbegin(), s.rend()), desc(s.begin(), s.end());
        std::vector<int> v;
        // odd radices first, powers of two ascending
        v = odd; v.insert(v.end(), asc.begin(), asc.end()); push(v);
        // powers of two descending, odd radices last
        v = desc; v.insert(v.end(), odd.begin(), odd.end()); push(v);
        // odd first, descending
        v = odd; v.insert(v.end(), desc.begin(), desc.end()); push(v);
        // ascending, odd last
        v = asc; v.insert(v.end(), odd.begin(), odd.end()); push(v);
    }
    return res;
}

void launch_shape(int64_t n, const std::vector<int>& rs, int csize, int* tpt, int* t) {
    int r[kMaxStages];
    for (size_t i = 0; i < rs.size() && i < (size_t)kMaxStages; ++i) r[i] = rs[i];
    const int need = required_tpt((int)n, r, (int)rs.size());
    *tpt = round_tpt(need);
    *t = pick_t(*tpt, (int)n, csize, rs.size() > 1);
}

bool two_pass_split(int64_t n, int dtype, int64_t* m_out, int64_t* k_out) {
    (void)dtype;
    if (single_kernel(n, dtype) || n > max_total_n(dtype) || !is_7smooth(n)) return false;
    // most balanced m k = n with both factors <= 1024 (the column tile of a
    // pass holds T columns of one length in LDS)
    int64_t best_m = 0;
    for (int64_t m = 1; m <= 1024; ++m) {
        if (n % m) continue;
        const int64_t k = n / m;
        if (k > 1024) continue;
        if (!best_m || std::llabs(m - k) < std::llabs(best_m - n / best_m) ||
            (std::llabs(m - k) == std::llabs(best_m - n / best_m) && m > best_m))
            best_m = m;
    }
    if (!best_m) return false;
    *m_out = best_m;
    *k_out = n / best_m;
    return true;
}

std::vector<int> choose_radices(int64_t n, int dtype) {
    std::vector<int> rs;
    if (n > max_single_n(dtype)) {  // a wide length runs its compiled lists only
        const auto w = wide_lists(n, dtype);
        if (tune_lookup(n, dtype, &rs) && std::find(w.begin(), w.end(), rs) != w.end()) return rs;
        return w.empty() ? std::vector<int>() : w[0];
    }
    if (tune_lookup(n, dtype, &rs)) return rs;
    auto c = radix_candidates(n, 1);
    return c.empty() ? rs : c[0];
}

// ---- tuning database ----------------------------------------------------------
// Text file, one line per entry:
//   <arch> <toolchain> <c64|c128> <n> [<order>:]<r1,r2,...> <ms>
// with <toolchain> the HIP version the library's kernels were compiled with
// ("hip7.2.53211"): timings hold for one device and one compiler's code.
// <order> is "ct", "pease", "fourstep" or "wave" for an alternative order (its
// list is the radix repeated), none for Stockham.  Lines for another architecture or
// toolchain, lines in another format, and lists that do not multiply to n are
// ignored.
namespace {
struct TuneEntry {
    std::vector<int> rs;
    double ms;
    int order;  // 0: Stockham
};
std::mutex g_tune_mu;
std::map<std::pair<int64_t, int>, TuneEntry> g_tune;
bool g_tune_env_done = false;
const char* kTuneArch = "gfx950";
#define FFTC_STR2(x) #x
#define FFTC_STR(x) FFTC_STR2(x)
const char* kTuneToolchain = "hip" FFTC_STR(HIP_VERSION_MAJOR) "." FFTC_STR(HIP_VERSION_MINOR) "." FFTC_STR(
    HIP_VERSION_PATCH);

int load_locked(const char* path) {
    FILE* f = fopen(path, "r");
    if (!f) return -1;
    char line[512], arch[64], tc[64], dt[16], rl[256], extra[8];
    long long n;
    double ms;
    int added = 0;
    while (fgets(line, sizeof line, f)) {
        if (sscanf(line, "%63s %63s %15s %lld %255s %lf %7s", arch, tc, dt, &n, rl, &ms, extra) != 6) continue;
        if (strcmp(arch, kTuneArch) != 0 || strcmp(tc, kTuneToolchain) != 0) continue;
        if (strcmp(dt, "c64") != 0 && strcmp(dt, "c128") != 0) continue;
        const int dtype = strcmp(dt, "c128") == 0 ? FFTC_C128 : FFTC_C64;
        int order = 0;
        char* list = rl;
        if (char* colon = strchr(rl, ':')) {
            *colon = 0;
            order = strcmp(rl, "ct") == 0         ? 1
                    : strcmp(rl, "pease") == 0    ? 2
                    : strcmp(rl, "fourstep") == 0 ? 3
                    : strcmp(rl, "wave") == 0     ? 4
                                                  : -1;
            list = colon + 1;
        }
        if (order < 0) continue;
        std::vector<int> rs;
        int64_t prod = 1;
        bool ok = n > 1;
        for (char* tok = strtok(list, ","); tok && ok; tok = strtok(nullptr, ",")) {
            const int r = atoi(tok);
            ok = ok && (r == 2 || r == 3 || r == 4 || r == 5 || r == 7 || r == 8 || r == 16);
            rs.push_back(r);
            prod *= r;
            ok = ok && prod <= n;
        }
        if (order > 0) {  // one radix repeated
            for (int r : rs) ok = ok && r == rs[0];
            ok = ok && !rs.empty() && find_order(dtype, n, order, rs[0]) != nullptr;
        }
        if (ok && prod == n && (order > 0 || (int)rs.size() <= kMaxStages)) {
            g_tune[{(int64_t)n, dtype}] = {rs, ms, order};
            ++added;
        }
    }
    fclose(f);
    return added;
}

void env_locked() {
    if (g_tune_env_done) return;
    g_tune_env_done = true;
    const char* p = getenv("FFTC_TUNE_DB");
    if (p && *p) load_locked(p);
}
}  // namespace

bool tune_lookup_order(int64_t n, int dtype, int* order, int* radix) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    env_locked();
    auto it = g_tune.find({n, dtype});
    if (it == g_tune.end() || it->second.order == 0) return false;
    *order = it->second.order;
    *radix = it->second.rs[0];
    return true;
}

void tune_record_order(int64_t n, int dtype, int order, int radix, double ms) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    env_locked();
    std::vector<int> rs;
    for (int64_t m = n; m > 1; m /= radix) rs.push_back(radix);
    g_tune[{n, dtype}] = {rs, ms, order};
}

bool tune_lookup(int64_t n, int dtype, std::vector<int>* rs) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    env_locked();
    auto it = g_tune.find({n, dtype});
    if (it == g_tune.end() || it->second.order != 0) return false;  // Stockham entries only
    *rs = it->second.rs;
    return true;
}

void tune_record(int64_t n, int dtype, const std::vector<int>& rs, double ms) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    env_locked();
    g_tune[{n, dtype}] = {rs, ms, 0};
}

int tune_load_file(const char* path) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    env_locked();
    return load_locked(path);
}

int tune_save_file(const char* path) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    FILE* f = fopen(path, "w");
    if (!f) return -1;
    for (auto& kv : g_tune) {
        fprintf(f, "%s %s %s %lld ", kTuneArch, kTuneToolchain, kv.first.second == FFTC_C128 ? "c128" : "c64",
                (long long)kv.first.first);
        if (kv.second.order)
            fprintf(f, "%s:", kv.second.order == 1   ? "ct"
                              : kv.second.order == 2 ? "pease"
                              : kv.second.order == 3 ? "fourstep"
                                                     : "wave");
        const auto& rs = kv.second.rs;
        for (size_t i = 0; i < rs.size(); ++i) fprintf(f, i ? ",%d" : "%d", rs[i]);
        fprintf(f, " %.6f\n", kv.second.ms);
    }
    fclose(f);
    return (int)g_tune.size();
}

const char* tune_key() {
    static const std::string key = std::string(kTuneArch) + " " + kTuneToolchain;
    return key.c_str();
}

void tune_clear_all() {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune.clear();
    g_tune_env_done = true;
}

int64_t stage_segments(const std::vector<int>& rs, int64_t base, std::vector<TwSegment>* segs) {
    int64_t ns = 1, off = base;
    for (int r : rs) {
        if (ns > 1) segs->push_back({off, (r - 1) * ns, ns, ns * r, 1});
        off += (r - 1) * ns;
        ns *= r;
    }
    return off - base;
}

}  // namespace fftc
