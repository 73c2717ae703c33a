// c128 several-requests Stockham kernels (the serving runtime's fused
// steps): the preferred list of every power of two.
#include "spec_list.inc"
#include "spec_table.h"

namespace fftc {

#define E(N, ...) SpecInst<double, N, __VA_ARGS__>::reqs_entry(FFTC_C128),
static const SpecEntry k_table[] = {FFTC_SERVE_LIST_C128(E)};
#undef E

const SpecEntry* serve_table_c128(int* count) {
    *count = (int)(sizeof(k_table) / sizeof(k_table[0]));
    return k_table;
}

}  // namespace fftc
