// Random-phase start blocks for the stochastic trace (section "Problem
// Description": the trace is estimated from R random vectors), drawn on the
// device from a counter-based generator so that a block of any size is
// produced at memory speed and reproducibly from (seed, element index).
//
// Generator: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014).  The state of
// element c = i R + r is key + (c + 1) gamma, gamma = 0x9E3779B97F4A7C15,
// key = mix(seed + gamma); u = (top 53 bits of mix(state)) / 2^53 and
// v_ir = exp(2 pi i u) / sqrt(N), computed in FP64 and rounded to the
// storage precision.
#include "kpm_internal.h"

namespace kpm {
namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename T>
__global__ void __launch_bounds__(256)
phase_block_kernel(T* __restrict__ V, int64_t n, uint64_t key, double scale) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const uint64_t z = mix64(key + static_cast<uint64_t>(c + 1) * kGamma);
    const double u = static_cast<double>(z >> 11) * (1.0 / 9007199254740992.0);
    double s, co;
    sincos(6.283185307179586476925286766559 * u, &s, &co);
    V[2 * c] = static_cast<T>(co * scale);
    V[2 * c + 1] = static_cast<T>(s * scale);
}

}  // namespace

hipError_t launch_phase_block(void* V, int64_t N, int R, int dtype, uint64_t seed, hipStream_t s) {
    const int64_t n = N * R;
    const uint64_t key = mix64(seed + kGamma);
    const double scale = 1.0 / std::sqrt(static_cast<double>(N));
    const int blocks = static_cast<int>((n + 255) / 256);
    if (dtype == KPM_C128)
        phase_block_kernel<double><<<blocks, 256, 0, s>>>(static_cast<double*>(V), n, key, scale);
    else
        phase_block_kernel<float><<<blocks, 256, 0, s>>>(static_cast<float*>(V), n, key, scale);
    return hipGetLastError();
}

}  // namespace kpm
