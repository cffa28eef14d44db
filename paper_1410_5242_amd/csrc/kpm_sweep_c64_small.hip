// Instantiations of the fused sweep for complex64 storage, block widths 1, 2, 4, 8, 16.
#include "kpm_sweep.h"

namespace kpm {

hipError_t launch_sweep_c64_small(int R, int variant, const SweepArgs& a, hipStream_t s) {
    switch (R) {
    case 1: return sweep::launch_variant<float, 1>(variant, a, s);
    case 2: return sweep::launch_variant<float, 2>(variant, a, s);
    case 4: return sweep::launch_variant<float, 4>(variant, a, s);
    case 8: return sweep::launch_variant<float, 8>(variant, a, s);
    case 16: return sweep::launch_variant<float, 16>(variant, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace kpm
