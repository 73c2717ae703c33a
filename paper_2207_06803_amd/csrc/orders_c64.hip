// c64 kernels of the alternative orders (orders.h): recursive Cooley-Tukey
// with the explicit digit reversal, Pease's constant geometry, the
// four-step (block) form of Eq. 2, and the in-wave exchange for N = 256.
#include "internal.h"
#include "orders.h"

namespace fftc {

#define ORDER_LIST(X) X(64, 2) X(64, 4) X(64, 8) X(256, 2) X(256, 4) X(256, 16) X(1024, 2) X(1024, 4) \
    X(4096, 2) X(4096, 4) X(4096, 8) X(4096, 16)
#define E(N, R)                                                              \
    OrderInst<float, N, R, ORDER_CT>::entry(FFTC_C64), OrderInst<float, N, R, ORDER_PEASE>::entry(FFTC_C64), \
        OrderInst<float, N, R, ORDER_FOURSTEP>::entry(FFTC_C64),
static const OrderEntry k_table[] = {ORDER_LIST(E) WaveOrderInst<float>::entry(FFTC_C64)};
#undef E

const OrderEntry* order_table_c64(int* count) {
    *count = (int)(sizeof(k_table) / sizeof(k_table[0]));
    return k_table;
}

}  // namespace fftc
