// Single-kernel lists of the lengths whose full LDS exchange does not fit a
// workgroup (complex64 N = 32768, complex128 N = 16384), with the half-width
// exchange: the plain kernels and the serving runtime's several-requests
// kernels, fastest measured list first.
#include "spec_list.inc"
#include "spec_table.h"

namespace fftc {

#define E64(N, ...) WideSpecInst<float, N, __VA_ARGS__>::entry(FFTC_C64),
#define E128(N, ...) WideSpecInst<double, N, __VA_ARGS__>::entry(FFTC_C128),
#define R64(N, ...) WideSpecInst<float, N, __VA_ARGS__>::reqs_entry(FFTC_C64),
#define R128(N, ...) WideSpecInst<double, N, __VA_ARGS__>::reqs_entry(FFTC_C128),
static const SpecEntry k_c64[] = {FFTC_WIDE_LIST_C64(E64)};
static const SpecEntry k_c128[] = {FFTC_WIDE_LIST_C128(E128)};
static const SpecEntry k_reqs_c64[] = {FFTC_WIDE_LIST_C64(R64)};
static const SpecEntry k_reqs_c128[] = {FFTC_WIDE_LIST_C128(R128)};
#undef E64
#undef E128
#undef R64
#undef R128

const SpecEntry* wide_table(int dtype, int* count) {
    *count = dtype == FFTC_C128 ? (int)(sizeof(k_c128) / sizeof(k_c128[0])) : (int)(sizeof(k_c64) / sizeof(k_c64[0]));
    return dtype == FFTC_C128 ? k_c128 : k_c64;
}

const SpecEntry* wide_serve_table(int dtype, int* count) {
    *count = dtype == FFTC_C128 ? (int)(sizeof(k_reqs_c128) / sizeof(k_reqs_c128[0]))
                                : (int)(sizeof(k_reqs_c64) / sizeof(k_reqs_c64[0]));
    return dtype == FFTC_C128 ? k_reqs_c128 : k_reqs_c64;
}

}  // namespace fftc
