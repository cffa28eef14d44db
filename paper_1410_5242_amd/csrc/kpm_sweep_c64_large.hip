// Instantiations of the fused sweep for complex64 storage, block widths 32, 64.
#include "kpm_sweep.h"

namespace kpm {

hipError_t launch_sweep_c64_large(int R, int variant, const SweepArgs& a, hipStream_t s) {
    switch (R) {
    case 32: return sweep::launch_variant<float, 32>(variant, a, s);
    case 64: return sweep::launch_variant<float, 64>(variant, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace kpm
