// c64 several-requests Stockham kernels (the serving runtime's fused
// steps): the preferred list of every power of two.
#include "spec_list.inc"
#include "spec_table.h"

namespace fftc {

#define E(N, ...) SpecInst<float, N, __VA_ARGS__>::reqs_entry(FFTC_C64),
static const SpecEntry k_table[] = {FFTC_SERVE_LIST_C64(E)};
#undef E

const SpecEntry* serve_table_c64(int* count) {
    *count = (int)(sizeof(k_table) / sizeof(k_table[0]));
    return k_table;
}

}  // namespace fftc
