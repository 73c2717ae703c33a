// Complex arithmetic on HIP's float2 / double2 (x = real, y = imaginary).
#pragma once
#include <hip/hip_runtime.h>

namespace fftc {

template <typename Real> struct cplx_of;
template <> struct cplx_of<float> { using type = float2; };
template <> struct cplx_of<double> { using type = double2; };
template <typename Real> using cplx = typename cplx_of<Real>::type;

// Native two-element vectors of the same layout, for whole-element loads.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename C> struct vec_of;
template <> struct vec_of<float2> { using type = f32x2; };
template <> struct vec_of<double2> { using type = f64x2; };

__device__ __forceinline__ float2 mk(float a, float b) { return make_float2(a, b); }
__device__ __forceinline__ double2 mk(double a, double b) { return make_double2(a, b); }

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return mk(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return mk(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cconj(C a) { return mk(a.x, -a.y); }
// multiply by -i: (x + iy)(-i) = y - ix
template <typename C> __device__ __forceinline__ C cmul_mi(C a) { return mk(a.y, -a.x); }
// multiply by +i
template <typename C> __device__ __forceinline__ C cmul_pi(C a) { return mk(-a.y, a.x); }
// full complex product, FMA-contracted by the compiler
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C, typename Real> __device__ __forceinline__ C cscale(C a, Real s) {
    return mk(a.x * s, a.y * s);
}

}  // namespace fftc
