// c64 Stockham kernels with the layout accessors (planar and strided data):
// the preferred radix list of every compiled length.
#include "spec_list.inc"
#include "spec_table.h"

namespace fftc {

#define E(N, ...) SpecInst<float, N, __VA_ARGS__>::layout_entry(FFTC_C64),
static const SpecEntry k_table[] = {FFTC_LAYOUT_LIST_C64(E)};
#undef E

const SpecEntry* layout_table_c64(int* count) {
    *count = (int)(sizeof(k_table) / sizeof(k_table[0]));
    return k_table;
}

}  // namespace fftc
