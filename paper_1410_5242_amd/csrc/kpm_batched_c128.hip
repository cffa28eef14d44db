// Instantiations of the batched persistent solver for complex128 storage,
// and its dtype dispatch.
#include "kpm_batched.h"

namespace kpm {

hipError_t launch_batched_c64(int R, const BatchArgs& a, hipStream_t s);
int batched_max_waves_c64(int R);

hipError_t launch_batched(int dtype, int R, const BatchArgs& a, hipStream_t s) {
    if (dtype == KPM_C128) return batch::launch_dtype<double>(R, a, s);
    return launch_batched_c64(R, a, s);
}

int batched_max_waves(int dtype, int R) {
    return dtype == KPM_C128 ? batch::max_waves<double>(R) : batched_max_waves_c64(R);
}

}  // namespace kpm
