// Two-pass column kernels with compiled Stockham bodies, c128 (8 columns
// per workgroup: 8 x sizeof(complex) = 128 contiguous bytes per row).
#include "fourstep_spec.h"
#include "spec_list.inc"

namespace fftc {

#define E(N, ...) FourStepInst<double, 8, N, __VA_ARGS__>::entry(FFTC_C128),
static const FourStepEntry k_table[] = {FFTC_FOURSTEP_LIST_C128(E)};
#undef E

const FourStepEntry* fourstep_table_c128(int* count) {
    *count = (int)(sizeof(k_table) / sizeof(k_table[0]));
    return k_table;
}

}  // namespace fftc
