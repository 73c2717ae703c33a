// Two-pass column kernels with compiled Stockham bodies, c64 (16 columns
// per workgroup: 16 x sizeof(complex) = 128 contiguous bytes per row).
#include "fourstep_spec.h"
#include "spec_list.inc"

namespace fftc {

#define E(N, ...) FourStepInst<float, 16, N, __VA_ARGS__>::entry(FFTC_C64),
static const FourStepEntry k_table[] = {FFTC_FOURSTEP_LIST_C64(E)};
#undef E

const FourStepEntry* fourstep_table_c64(int* count) {
    *count = (int)(sizeof(k_table) / sizeof(k_table[0]));
    return k_table;
}

}  // namespace fftc
