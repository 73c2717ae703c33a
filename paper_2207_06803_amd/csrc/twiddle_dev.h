// One twiddle-table entry, computed in fp64 on the device: entry idx of a
// segment is w_len^{(mul a b) mod len} with a = idx / ns + a0, b = idx mod ns
// and w_len = exp(-2 pi i / len).  The exponent is reduced exactly in
// integers and the angle taken in (-pi, pi] before sincospi, so quarter turns
// come out exact; complex64 tables round the fp64 value to nearest fp32.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fftc {

template <typename C>
__device__ inline C twiddle_entry(int64_t idx, int64_t ns, int64_t len, int64_t mul, int64_t a0) {
    const int64_t a = idx / ns + a0, b = idx % ns;
    int64_t m = ((mul * a) % len) * b % len;
    if (2 * m > len) m -= len;  // angle in (-pi, pi]
    double sn, cs;
    // w = exp(-2 pi i m / L) = cos(2 pi m/L) - i sin(2 pi m/L)
    sincospi(2.0 * (double)m / (double)len, &sn, &cs);
    C v;
    v.x = cs;
    v.y = -sn;
    return v;
}

}  // namespace fftc
