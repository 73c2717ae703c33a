// Launch-shape rules shared by the host planner and the kernels.
#pragma once

namespace fftc {

constexpr int kMaxStages = 8;
constexpr int kMaxElemsPerThread = 16;   // register block per thread and stage
constexpr int kWorkgroupTarget = 256;    // threads per workgroup when T > 1 (128 <= N <= 256)
constexpr int kLdsBudgetPerGroup = 65536;
constexpr int kLdsMaxPerGroup = 163840;  // gfx950: 160 KB per workgroup

// LDS elements for one transform: one pad element every 16.
__host__ __device__ constexpr int lds_len(int n) { return n + (n >> 4); }

// LDS elements per transform in a column tile (kernels whose HBM side moves
// rows of adjacent transforms): the padded length made odd, so the tile's
// transforms at one element index fall in different banks.
__host__ __device__ constexpr int tile_pitch(int n) { return lds_len(n) | 1; }

// Butterflies of radix r one thread holds at most in a stage.
__host__ __device__ constexpr int nb_cap(int r) { return r >= kMaxElemsPerThread ? 1 : kMaxElemsPerThread / r; }

// Threads needed per transform so every stage fits the register block.
constexpr int required_tpt(int n, const int* rs, int nr) {
    int m = 1;
    for (int q = 0; q < nr; ++q) {
        const int cap = nb_cap(rs[q]);
        const int need = (n / rs[q] + cap - 1) / cap;
        if (need > m) m = need;
    }
    return m;
}

// Round up to a power of two below one wave, to whole waves above.
constexpr int round_tpt(int x) {
    if (x >= 64) return (x + 63) / 64 * 64;
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Transforms per workgroup: fill the target thread count within the LDS budget.
// One-wave workgroups for N <= 64 and N >= 512: more independent workgroups
// per CU overlap one another's loads, stages and stores (measured on 2^24
// complex64 elements: N = 1024 51.5 -> 46.9 us, N = 64 46.5 -> 44.4 us, no
// change at 4096 and up); N = 128, 256 keep 256-thread groups.
constexpr int wg_target(int n) { return (n >= 512 || n <= 64) ? 64 : kWorkgroupTarget; }
// Transforms per workgroup for a given thread target.
constexpr int pick_t_for(int target, int tpt, int n, int csize, bool multi_stage) {
    if (tpt >= target || (target % tpt) != 0) return 1;
    int t = target / tpt;
    const int per = multi_stage ? lds_len(n) * csize : 0;
    while (t > 1 && t * per > kLdsBudgetPerGroup) t >>= 1;
    return t;
}
constexpr int pick_t(int tpt, int n, int csize, bool multi_stage) {
    return pick_t_for(wg_target(n), tpt, n, csize, multi_stage);
}

}  // namespace fftc
