// Compiled complex128 Stockham specialisations: power-of-two lengths 8..8192.
#include "spec_table.h"

namespace fftc {

#define E(N, ...) SpecInst<double, N, __VA_ARGS__>::entry(FFTC_C128)

static const SpecEntry k_table[] = {
    E(8, 8), E(16, 16),
    E(32, 2, 16), E(32, 8, 4),
    E(64, 4, 16), E(64, 8, 8),
    E(128, 8, 16), E(128, 16, 8),
    E(256, 16, 16), E(256, 4, 4, 16),
    E(512, 8, 8, 8), E(512, 2, 16, 16),
    E(1024, 4, 16, 16), E(1024, 16, 16, 4), E(1024, 8, 8, 16),
    E(2048, 8, 16, 16), E(2048, 16, 16, 8),
    E(4096, 16, 16, 16), E(4096, 8, 8, 8, 8),
    E(8192, 2, 16, 16, 16), E(8192, 16, 16, 16, 2),
};

#undef E

const SpecEntry* spec_table_c128(int* count) {
    *count = (int)(sizeof(k_table) / sizeof(k_table[0]));
    return k_table;
}

}  // namespace fftc
