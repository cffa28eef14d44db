// Instantiations of the batched persistent solver for complex64 storage.
#include "kpm_batched.h"

namespace kpm {

hipError_t launch_batched_c64(int R, const BatchArgs& a, hipStream_t s) {
    return batch::launch_dtype<float>(R, a, s);
}
int batched_max_waves_c64(int R) { return batch::max_waves<float>(R); }

}  // namespace kpm
