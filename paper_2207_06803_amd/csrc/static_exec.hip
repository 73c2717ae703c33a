// fftc_execute_static: one call that plans and runs a batched transform
// without allocating device memory.  The twiddle tables and the two-pass
// intermediate of an in-place call live in `scratch`, a file-scope device
// array of kStaticBytes that each GPU the library runs on holds until the
// process ends; the kernels are the ordinary plans' kernels.
#include <mutex>

#include "plan.h"
#include "twiddle_dev.h"

namespace fftc {

constexpr size_t kStaticBytes = size_t(64) << 20;      // the whole array
constexpr size_t kStaticTableBytes = size_t(2) << 20;  // twiddle tables at its start
constexpr int kStaticSegs = 2 * kMaxStages + 3;        // table segments of one plan
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

// Device address of `scratch` on each GPU, taken once per device with that
// device current (the array's host-side name is no device address).
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static fftc_status scratch_on(int dev, unsigned char** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(FFTC_ERR_INVALID_ARG, "device index beyond the static table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(FFTC_ERR_INTERNAL, "hipGetSymbolAddress(scratch) gave NULL");
        g_scratch_ptr[dev] = ptr;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
    return FFTC_OK;
}

struct SegPack {
    int64_t off[kStaticSegs], count[kStaticSegs], ns[kStaticSegs], len[kStaticSegs], mul[kStaticSegs],
        a0[kStaticSegs];
};

// The segments travel by value in the kernel arguments: no descriptor buffer.
template <typename C>
__global__ void __launch_bounds__(256) twiddle_static(C* table, SegPack pk) {
    const int g = blockIdx.y;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < pk.count[g];
         idx += (int64_t)gridDim.x * blockDim.x)
        table[pk.off[g] + idx] = twiddle_entry<C>(idx, pk.ns[g], pk.len[g], pk.mul[g], pk.a0[g]);
}

static fftc_status tables_async(void* table, int dtype, const std::vector<TwSegment>& segs, hipStream_t s) {
    if (segs.empty()) return FFTC_OK;
    if (segs.size() > (size_t)kStaticSegs) return fail(FFTC_ERR_INTERNAL, "too many twiddle segments");
    SegPack pk{};
    int64_t maxc = 1;
    for (size_t i = 0; i < segs.size(); ++i) {
        pk.off[i] = segs[i].off;
        pk.count[i] = segs[i].count;
        pk.ns[i] = segs[i].ns;
        pk.len[i] = segs[i].len;
        pk.mul[i] = segs[i].mul;
        pk.a0[i] = segs[i].a0;
        maxc = std::max<int64_t>(maxc, segs[i].count);
    }
    const int block = 256;
    dim3 grid((unsigned)std::min<int64_t>((maxc + block - 1) / block, 4096), (unsigned)segs.size());
    if (dtype == FFTC_C128)
        hipLaunchKernelGGL(twiddle_static<double2>, grid, dim3(block), 0, s, (double2*)table, pk);
    else
        hipLaunchKernelGGL(twiddle_static<float2>, grid, dim3(block), 0, s, (float2*)table, pk);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? FFTC_OK : fail_hip(e, "launch(twiddle_static)");
}

static fftc_status execute_static(int64_t n, int64_t batch, int direction, int dtype, const void* in, void* out,
                                  void* stream) {
    clear_error();
    if (dtype != FFTC_C64 && dtype != FFTC_C128)
        return fail(FFTC_ERR_INVALID_ARG, "fftc_execute_static takes FFTC_C64 or FFTC_C128");
    fftc_status st = check_static_args(n, batch, direction, dtype);
    if (st != FFTC_OK) return st;
    if (!in || !out) return fail(FFTC_ERR_INVALID_ARG, "in/out is NULL");
    const size_t cs = dtype == FFTC_C128 ? 16 : 8;
    if (((uintptr_t)in % cs) || ((uintptr_t)out % cs))
        return fail(FFTC_ERR_INVALID_ARG, "in/out not aligned to the complex element size");
    int dev = 0;
    FFTC_HIP_TRY(hipGetDevice(&dev));
    unsigned char* base = nullptr;
    st = scratch_on(dev, &base);
    if (st != FFTC_OK) return st;
    st = enable_large_lds();
    if (st != FFTC_OK) return st;

    fftc_plan_s p;
    p.n = n;
    p.batch = batch;
    p.direction = direction;
    p.dtype = dtype;
    p.device = dev;
    std::vector<TwSegment> segs;
    int64_t entries = 0;
    st = shape_plan(&p, nullptr, 0, &segs, &entries);
    if (st != FFTC_OK) return st;
    if ((size_t)std::max<int64_t>(entries, 1) * cs > kStaticTableBytes)
        return fail(FFTC_ERR_TOO_LARGE, "twiddle tables of n = " + std::to_string(n) + " exceed the " +
                                            std::to_string(kStaticTableBytes) + "-byte static table region");
    hipStream_t s = static_cast<hipStream_t>(stream);
    p.tw = base;
    p.tw_bytes = (size_t)std::max<int64_t>(entries, 1) * cs;
    st = tables_async(p.tw, dtype, segs, s);
    if (st != FFTC_OK) return st;
    if (p.variant != FFTC_VARIANT_TWO_PASS) return launch_single(&p, in, out, batch, s);
    if (in != out) return launch_two_pass(&p, in, out, batch, s);  // the intermediate goes through out
    // in place: the intermediate goes through the rest of the array, as
    // many transforms at a time as it holds
    const size_t per = (size_t)n * cs;
    const int64_t cap = (int64_t)((kStaticBytes - kStaticTableBytes) / per);
    if (cap < 1) return fail(FFTC_ERR_TOO_LARGE, "one transform exceeds the static scratch");
    p.scratch = base + kStaticTableBytes;
    p.scratch_bytes = (size_t)cap * per;
    for (int64_t b0 = 0; b0 < batch; b0 += cap) {
        const int64_t nb = std::min<int64_t>(cap, batch - b0);
        const unsigned char* ci = static_cast<const unsigned char*>(in) + (size_t)b0 * per;
        unsigned char* co = static_cast<unsigned char*>(out) + (size_t)b0 * per;
        st = launch_two_pass(&p, ci, co, nb, s);
        if (st != FFTC_OK) return st;
    }
    return FFTC_OK;
}

}  // namespace fftc

extern "C" fftc_status fftc_execute_static(int64_t n, int64_t batch, int direction, int dtype, const void* in,
                                           void* out, void* stream) {
    try {
        return fftc::execute_static(n, batch, direction, dtype, in, out, stream);
    } catch (...) {
        return fftc::fail(FFTC_ERR_INTERNAL, "exception in fftc_execute_static");
    }
}

extern "C" size_t fftc_static_scratch_bytes(void) { return fftc::kStaticBytes; }
