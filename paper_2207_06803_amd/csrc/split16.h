// Split-precision MFMA plans (split16.hip).
#pragma once
#include <vector>

#include "internal.h"

struct fftc_plan_s;

namespace fftc {

inline bool is_split_dtype(int dtype) {
    return dtype == FFTC_C64_SPLIT_F16 || dtype == FFTC_C64_SPLIT_BF16 || dtype == FFTC_C64_SPLIT3_BF16 ||
           dtype == FFTC_C64_F16;
}
bool split_supported(int64_t n);
std::vector<int> split_radices(int64_t n);
int split_threads(int64_t n);
fftc_status launch_split(const fftc_plan_s* p, const void* in, void* out, int64_t batch, hipStream_t s);

}  // namespace fftc
