// Persistent mixed-length kernel for c128, dispatching to every compiled
// Stockham list of spec_list.inc.
#include "mixed_kernel.h"
#include "spec_list.inc"

namespace fftc {

FFTC_DEFINE_MIXED_KERNEL(mixed_persistent_c128, FFTC_SPEC_LIST_C128)

const void* mixed_kernel_c128(bool inv) {
    return inv ? reinterpret_cast<const void*>(&mixed_persistent_c128<double, true>)
               : reinterpret_cast<const void*>(&mixed_persistent_c128<double, false>);
}

}  // namespace fftc
