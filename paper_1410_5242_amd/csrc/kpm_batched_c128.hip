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

namespace {
template <typename T>
int rows_per_pass(int R) {
    switch (R) {
    case 1: return batch::Shape<T, 1>::RPW;
    case 2: return batch::Shape<T, 2>::RPW;
    case 4: return batch::Shape<T, 4>::RPW;
    case 8: return batch::Shape<T, 8>::RPW;
    case 16: return batch::Shape<T, 16>::RPW;
    case 32: return batch::Shape<T, 32>::RPW;
    case 64: return batch::Shape<T, 64>::RPW;
    }
    return 1;
}
}  // namespace

int batched_rows_per_pass(int dtype, int R) {
    return dtype == KPM_C128 ? rows_per_pass<double>(R) : rows_per_pass<float>(R);
}

}  // namespace kpm
