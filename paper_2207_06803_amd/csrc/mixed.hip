// Mixed-length batches in one persistent launch: plan construction.
//
// Transforms of different lengths N_i are packed back to back (offset =
// prefix sum of the lengths).  Transforms of equal length form a class with
// its own Stockham radix list (from the tuning database or the planner) and
// twiddle segment in one shared table.  Work items hold up to T_c transforms
// of one class -- as many as one 256-thread workgroup can hold in registers
// and LDS.  A grid sized to fill the GPU once runs them: the plan assigns the
// items, longest first, each to the workgroup with the least work so far
// (longest-processing-time scheduling, work = bytes moved plus a fixed cost
// per item), and lays each workgroup's items out contiguously.  The launch
// is recorded in a hipGraph at plan time and replayed per execution.
#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <queue>

#include "plan.h"

namespace fftc {

static const void* mixed_fn(int dtype, int direction) {
    const bool inv = direction == FFTC_INVERSE;
    return dtype == FFTC_C128 ? mixed_kernel_c128(inv) : mixed_kernel_c64(inv);
}

static void free_mixed(MixedState* m) {
    if (!m) return;
    if (m->exec) hipGraphExecDestroy(m->exec);
    if (m->graph) hipGraphDestroy(m->graph);
    if (m->dev) hipFree(m->dev);
    delete m;
}

void destroy_mixed(MixedState* m) { free_mixed(m); }

fftc_status build_mixed(fftc_plan_s* p, const int64_t* n, int64_t count) {
    const int dtype = p->dtype;
    const size_t cs = dtype == FFTC_C128 ? 16 : 8;
    MixedState* m = new (std::nothrow) MixedState();
    if (!m) return fail(FFTC_ERR_OUT_OF_MEMORY, "host allocation failed");
    p->mixed = m;

    // classes, offsets
    std::map<int64_t, int> cls_of;
    std::vector<int64_t> offsets(count);
    int64_t total = 0;
    for (int64_t i = 0; i < count; ++i) {
        offsets[i] = total;
        total += n[i];
        if (!cls_of.count(n[i])) cls_of[n[i]] = 0;
    }
    std::vector<int64_t> lens;
    for (auto& kv : cls_of) {
        kv.second = (int)lens.size();
        lens.push_back(kv.first);
    }
    const int ncls = (int)lens.size();
    std::vector<MixedClass> classes(ncls);
    std::vector<TwSegment> segs;
    int64_t twoff = 0;
    size_t lds_need = 0;
    for (int c = 0; c < ncls; ++c) {
        const int64_t len = lens[c];
        std::vector<int> rs;
        if (len > 1) rs = choose_radices(len, dtype);
        if (len > 1 && rs.empty()) return fail(FFTC_ERR_UNSUPPORTED_SIZE, "no factorisation");
        int tpt, t;
        const int64_t per = rs.size() > 1 ? lds_len((int)len) : 0;
        const SpecEntry* spec = len > 1 ? find_spec(dtype, len, rs) : nullptr;
        int64_t ldsn = per;
        if (spec && spec->id >= 0 && spec->tpt * spec->tm <= kMixedThreads) {
            // compiled body: its shape for 256-thread workgroups; short lists stage through LDS
            tpt = spec->tpt;
            t = spec->tm;
            classes[c].body = spec->id;
            ldsn = lds_len((int)len);
        } else {
            launch_shape(len, rs, (int)cs, &tpt, &t);
            if (tpt > kMixedThreads) return fail(FFTC_ERR_UNSUPPORTED_SIZE, "radix list needs too many threads");
            // transforms per item: fill the workgroup and the per-item LDS budget
            t = std::max(1, kMixedThreads / tpt);
            if (per > 0) t = (int)std::min<int64_t>(t, std::max<int64_t>(1, kMixedLdsElems / per));
            classes[c].body = -1;
        }
        classes[c].twbase = (int)twoff;
        classes[c].ldsn = (int)ldsn;
        const int64_t used = stage_segments(rs, twoff, &segs);
        fill_gen_desc(len, rs, tpt, t, twoff, &classes[c].desc);
        twoff += used;
        lds_need = std::max(lds_need, (size_t)(ldsn * t) * cs);
        m->class_len.push_back(len);
        m->class_radices.push_back(rs);
    }
    // items: per class, chunks of up to t transforms, in input order
    std::vector<std::vector<int64_t>> members(ncls);
    for (int64_t i = 0; i < count; ++i) members[cls_of[n[i]]].push_back(i);
    std::vector<int64_t> order;  // transform ids grouped by class
    std::vector<MixedItem> items;
    std::vector<double> cost;
    // a fixed cost per item (descriptor and first-load latency) in bytes
    const double kItemBytes = 16384.0;
    for (int c = 0; c < ncls; ++c) {
        const int t = classes[c].desc.t;
        if (t > kMixedThreads) return fail(FFTC_ERR_INTERNAL, "mixed item larger than a workgroup");
        for (size_t s = 0; s < members[c].size(); s += t) {
            MixedItem it{};
            it.cls = c;
            it.first = (int)order.size();
            it.count = (int)std::min<size_t>(t, members[c].size() - s);
            it.body = classes[c].body;
            it.twbase = classes[c].twbase;
            it.n = (int)lens[c];
            it.ldsn = classes[c].ldsn;
            it.magic = lens[c] > 1 ? (uint32_t)(((uint64_t(1) << 32) + lens[c] - 1) / lens[c]) : 0;
            if ((int64_t)t * lens[c] >= (int64_t(1) << 32) / std::max<int64_t>(lens[c], 1))
                return fail(FFTC_ERR_INTERNAL, "mixed item too long for its index division");
            for (int q = 0; q < it.count; ++q) order.push_back(members[c][s + q]);
            items.push_back(it);
            cost.push_back(2.0 * (double)cs * (double)lens[c] * it.count + kItemBytes);
        }
    }
    if (order.size() > (size_t)0x7fffffff) return fail(FFTC_ERR_INVALID_ARG, "too many transforms");
    std::vector<int64_t> toffs(order.size());
    for (size_t i = 0; i < order.size(); ++i) toffs[i] = offsets[order[i]];

    m->count = count;
    m->total = total;
    m->nitems = (int)items.size();
    m->lds_bytes = std::max<size_t>(lds_need, 16);

    // persistent grid: every resident workgroup slot once
    const void* fn = mixed_fn(dtype, p->direction);
    FFTC_HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)m->lds_bytes));
    int per_cu = 0, dev = 0, cus = 0;
    FFTC_HIP_TRY(hipGetDevice(&dev));
    FFTC_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    FFTC_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kMixedThreads, m->lds_bytes));
    const int groups = std::max(1, std::min(per_cu * cus, m->nitems));
    m->groups = groups;

    // longest first, each to the least loaded workgroup; a workgroup's items
    // are contiguous, in the order it received them
    std::vector<size_t> idx(items.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
    using Load = std::pair<double, int>;
    std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
    for (int g = 0; g < groups; ++g) heap.push({0.0, g});
    std::vector<std::vector<int>> per_wg(groups);
    for (size_t i : idx) {
        Load l = heap.top();
        heap.pop();
        per_wg[l.second].push_back((int)i);
        heap.push({l.first + cost[i], l.second});
    }
    std::vector<MixedItem> sorted;
    sorted.reserve(items.size());
    std::vector<int> wg_start(groups + 1, 0);
    for (int g = 0; g < groups; ++g) {
        wg_start[g] = (int)sorted.size();
        for (int i : per_wg[g]) sorted.push_back(items[i]);
    }
    wg_start[groups] = (int)sorted.size();

    // device block: classes | items | workgroup ranges | offsets | twiddles
    auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t o_cls = 0;
    const size_t o_items = align(o_cls + sizeof(MixedClass) * ncls);
    const size_t o_wg = align(o_items + sizeof(MixedItem) * sorted.size());
    const size_t o_offs = align(o_wg + sizeof(int) * wg_start.size());
    const size_t o_tw = align(o_offs + sizeof(int64_t) * toffs.size());
    const size_t bytes = o_tw + (size_t)std::max<int64_t>(twoff, 1) * cs;
    {
        fftc_status sa = dev_malloc(&m->dev, bytes, "hipMalloc(mixed plan tables)");
        if (sa != FFTC_OK) return sa;
    }
    m->dev_bytes = bytes;
    char* base = static_cast<char*>(m->dev);
    m->d_classes = reinterpret_cast<MixedClass*>(base + o_cls);
    m->d_items = reinterpret_cast<MixedItem*>(base + o_items);
    m->d_wg_start = reinterpret_cast<int*>(base + o_wg);
    m->d_offsets = reinterpret_cast<int64_t*>(base + o_offs);
    m->d_tw = base + o_tw;
    FFTC_HIP_TRY(hipMemcpy(m->d_classes, classes.data(), sizeof(MixedClass) * ncls, hipMemcpyHostToDevice));
    FFTC_HIP_TRY(hipMemcpy(m->d_items, sorted.data(), sizeof(MixedItem) * sorted.size(), hipMemcpyHostToDevice));
    FFTC_HIP_TRY(hipMemcpy(m->d_wg_start, wg_start.data(), sizeof(int) * wg_start.size(), hipMemcpyHostToDevice));
    FFTC_HIP_TRY(hipMemcpy(m->d_offsets, toffs.data(), sizeof(int64_t) * toffs.size(), hipMemcpyHostToDevice));
    fftc_status st = make_twiddles(m->d_tw, dtype, segs, nullptr);
    if (st != FFTC_OK) return st;

    // graph: the persistent kernel
    FFTC_HIP_TRY(hipGraphCreate(&m->graph, 0));
    {
        m->args.in = nullptr;
        m->args.out = nullptr;
        hipKernelNodeParams kp = m->kernel_params(fn);
        FFTC_HIP_TRY(hipGraphAddKernelNode(&m->kernel_node, m->graph, nullptr, 0, &kp));
    }
    FFTC_HIP_TRY(hipGraphInstantiate(&m->exec, m->graph, nullptr, nullptr, 0));
    m->fn = fn;
    return FFTC_OK;
}

hipKernelNodeParams MixedState::kernel_params(const void* fn_) {
    kargs[0] = &args.in;
    kargs[1] = &args.out;
    kargs[2] = &d_tw;
    kargs[3] = &d_classes;
    kargs[4] = &d_items;
    kargs[5] = &d_wg_start;
    kargs[6] = &d_offsets;
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(fn_);
    kp.gridDim = dim3((unsigned)groups);
    kp.blockDim = dim3(kMixedThreads);
    kp.sharedMemBytes = (unsigned)lds_bytes;
    kp.kernelParams = kargs;
    kp.extra = nullptr;
    return kp;
}

fftc_status launch_mixed(fftc_plan_s* p, const void* in, void* out, hipStream_t s) {
    MixedState* m = p->mixed;
    if (m->direct) {  // the same kernel and arguments, launched on the stream
        m->args.in = in;
        m->args.out = out;
        hipKernelNodeParams kp = m->kernel_params(m->fn);
        FFTC_HIP_TRY(hipLaunchKernel(kp.func, kp.gridDim, kp.blockDim, kp.kernelParams, kp.sharedMemBytes, s));
        // the graph's pointer arguments no longer match args: refresh them on the next replay
        m->graph_stale = true;
        return FFTC_OK;
    }
    if (in != m->args.in || out != m->args.out || m->graph_stale) {
        m->graph_stale = false;
        m->args.in = in;
        m->args.out = out;
        hipKernelNodeParams kp = m->kernel_params(m->fn);
        FFTC_HIP_TRY(hipGraphExecKernelNodeSetParams(m->exec, m->kernel_node, &kp));
    }
    FFTC_HIP_TRY(hipGraphLaunch(m->exec, s));
    return FFTC_OK;
}

}  // namespace fftc
