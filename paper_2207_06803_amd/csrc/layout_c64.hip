// c64 Stockham kernels with the layout accessors (planar and strided data):
// the preferred radix list of every compiled length, each with its tile
// kernel for column-like layouts.
#include "spec_list.inc"
#include "layout_tile.h"

namespace fftc {

#define E(N, ...) layout_entry_with_tile<float, N, __VA_ARGS__>(FFTC_C64),
static const SpecEntry k_table[] = {FFTC_LAYOUT_LIST_C64(E)};
#undef E

const SpecEntry* layout_table_c64(int* count) {
    *count = (int)(sizeof(k_table) / sizeof(k_table[0]));
    return k_table;
}

// two-pass column kernels: the column lengths of the two-pass plans
#define C(N, ...) ColPassInst<float, 16, N, __VA_ARGS__>::entry(FFTC_C64),
static const FourStepEntry k_cols[] = {FFTC_FOURSTEP_LIST_C64(C)};
#undef C

const FourStepEntry* colpass_table_c64(int* count) {
    *count = (int)(sizeof(k_cols) / sizeof(k_cols[0]));
    return k_cols;
}

}  // namespace fftc
