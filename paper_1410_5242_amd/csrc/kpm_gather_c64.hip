// Instantiations of the staged-gather sweep for complex64 storage.
#include "kpm_gather.h"

namespace kpm {

hipError_t launch_gather_c64(int R, int variant, const SweepArgs& a, hipStream_t s) {
    return gather::launch_dtype<float>(R, variant, a, s);
}
int gather_waves_c64(int R) { return gather::waves_for<float>(R); }
int gather_lds_c64(int R) { return gather::lds_for<float>(R); }
int gather_window_lds_c64(int R) { return gather::window_lds_for<float>(R); }
int gather_window_side_c64(int R) { return gather::window_side_for<float>(R); }

}  // namespace kpm
