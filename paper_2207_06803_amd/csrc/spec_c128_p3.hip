// Compiled c128 Stockham specialisations, part 3 of the list in spec_list.inc.
#include "spec_list.inc"
#include "spec_table.h"

namespace fftc {

#define E(ID, N, ...) SpecInst<double, N, __VA_ARGS__>::entry(FFTC_C128, ID),
static const SpecEntry k_table[] = {FFTC_SPEC_LIST_C128_PART3(E)};
#undef E

const SpecEntry* spec_part_c128_3(int* count) {
    *count = (int)(sizeof(k_table) / sizeof(k_table[0]));
    return k_table;
}

}  // namespace fftc
