// Persistent mixed-length kernel for c64, dispatching to every compiled
// Stockham list of spec_list.inc.
#include "mixed_kernel.h"
#include "spec_list.inc"

namespace fftc {

FFTC_DEFINE_MIXED_KERNEL(mixed_persistent_c64, FFTC_SPEC_LIST_C64)

const void* mixed_kernel_c64(bool inv) {
    return inv ? reinterpret_cast<const void*>(&mixed_persistent_c64<float, true>)
               : reinterpret_cast<const void*>(&mixed_persistent_c64<float, false>);
}

}  // namespace fftc
