// Twiddle tables, generated on the GPU in fp64.
//
// Each segment describes entries value(idx) = w_L^{(m a b) mod L} with
// a = idx / ns + a0 (a0 = 1 unless stated), b = idx mod ns and
// w_L = exp(-2 pi i / L) (twiddle_dev.h computes one entry).  For a
// Stockham stage of radix R after Ns (the twiddle diagonal of Eq. 2 at
// length Ns R) this is the [r - 1][k] table of w_{Ns R}^{r k}; with ns = L
// it is the plain table w_L^b, and with a multiplier m the coarse table
// w_L^{m b} of the two-pass plans; with a0 = 0 it is the diagonal D^L_ns
// of Eq. 2 (entry i ns + j = w_L^{i j}).  The exponent is
// reduced exactly in integers and the angle is taken in (-pi, pi] before
// sincospi, so the quarter turns come out exact.  complex64 plans round
// the fp64 value to nearest fp32.
#include "internal.h"
#include "twiddle_dev.h"

namespace fftc {

struct TwSegDev {
    int64_t off, count, ns, len, mul, a0;
};

template <typename C>
__global__ void twiddle_kernel(C* table, const TwSegDev* __restrict__ segs) {
    const TwSegDev s = segs[blockIdx.y];
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < s.count;
         idx += (int64_t)gridDim.x * blockDim.x)
        table[s.off + idx] = twiddle_entry<C>(idx, s.ns, s.len, s.mul, s.a0);
}

fftc_status make_twiddles(void* table, int dtype, const std::vector<TwSegment>& segs,
                          hipStream_t stream) {
    if (segs.empty()) return FFTC_OK;
    std::vector<TwSegDev> h(segs.size());
    int64_t maxc = 1;
    for (size_t i = 0; i < segs.size(); ++i) {
        h[i] = {segs[i].off, segs[i].count, segs[i].ns, segs[i].len, segs[i].mul, segs[i].a0};
        maxc = std::max<int64_t>(maxc, segs[i].count);
    }
    if (segs.size() > 65535) return fail(FFTC_ERR_INTERNAL, "too many twiddle segments");
    TwSegDev* d = nullptr;
    {
        fftc_status st = dev_malloc((void**)&d, sizeof(TwSegDev) * h.size(), "hipMalloc(twiddle segments)");
        if (st != FFTC_OK) return st;
    }
    hipError_t e = hipMemcpyAsync(d, h.data(), sizeof(TwSegDev) * h.size(), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) {
        const int block = 256;
        const int64_t gx = std::min<int64_t>((maxc + block - 1) / block, 4096);
        dim3 grid((unsigned)gx, (unsigned)h.size());
        if (dtype == FFTC_C128)
            hipLaunchKernelGGL(twiddle_kernel<double2>, grid, dim3(block), 0, stream, (double2*)table, d);
        else
            hipLaunchKernelGGL(twiddle_kernel<float2>, grid, dim3(block), 0, stream, (float2*)table, d);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    hipError_t e2 = hipFree(d);
    if (e != hipSuccess) return fail_hip(e, "twiddle generation");
    if (e2 != hipSuccess) return fail_hip(e2, "hipFree(twiddle segments)");
    return FFTC_OK;
}

}  // namespace fftc
