// Instantiations of the staged-gather sweep for complex128 storage, and its
// dtype dispatch.
#include "kpm_gather.h"

namespace kpm {

hipError_t launch_gather_c64(int R, int variant, const SweepArgs& a, hipStream_t s);
int gather_waves_c64(int R);
int gather_lds_c64(int R);
int gather_window_lds_c64(int R);
int gather_window_side_c64(int R);

hipError_t launch_gather(int dtype, int R, int variant, const SweepArgs& a, hipStream_t s) {
    if (dtype == KPM_C128) return gather::launch_dtype<double>(R, variant, a, s);
    return launch_gather_c64(R, variant, a, s);
}

int gather_waves(int dtype, int R) {
    return dtype == KPM_C128 ? gather::waves_for<double>(R) : gather_waves_c64(R);
}

int gather_lds(int dtype, int R) {
    return dtype == KPM_C128 ? gather::lds_for<double>(R) : gather_lds_c64(R);
}

int gather_window_lds(int dtype, int R) {
    return dtype == KPM_C128 ? gather::window_lds_for<double>(R) : gather_window_lds_c64(R);
}

int gather_window_side(int dtype, int R) {
    return dtype == KPM_C128 ? gather::window_side_for<double>(R) : gather_window_side_c64(R);
}

}  // namespace kpm
