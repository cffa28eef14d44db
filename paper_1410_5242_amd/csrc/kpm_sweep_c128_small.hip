// Instantiations of the fused sweep for complex128 storage, block widths 1, 2, 4, 8, 16.
#include "kpm_sweep.h"

namespace kpm {

hipError_t launch_sweep_c128_small(int R, int variant, const SweepArgs& a, hipStream_t s) {
    switch (R) {
    case 1: return sweep::launch_variant<double, 1>(variant, a, s);
    case 2: return sweep::launch_variant<double, 2>(variant, a, s);
    case 4: return sweep::launch_variant<double, 4>(variant, a, s);
    case 8: return sweep::launch_variant<double, 8>(variant, a, s);
    case 16: return sweep::launch_variant<double, 16>(variant, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace kpm
