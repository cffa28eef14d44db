// Random-phase start blocks for the stochastic trace (section "Problem
// Description": the trace is estimated from R random vectors), drawn on the
// device from a counter-based generator so that a block of any size is
// produced at memory speed and reproducibly from (seed, element index).
//
// Generator: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014).  The state of
// element c = i R + r is key + (c + 1) gamma, gamma = 0x9E3779B97F4A7C15,
// key = mix(seed + gamma); u = (top 53 bits of mix(state)) / 2^53 and
// v_ir = exp(2 pi i u) / sqrt(N), computed in FP64 and rounded to the
// storage precision.  The disorder potential of a Hamiltonian built without
// a caller array draws from the same generator under the key
// mix(seed + 2 gamma) (the second SplitMix64 output of the seed).
#include "kpm_internal.h"

#include <cmath>

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

// Disorder potential V_n = gamma (u_n - 1/2) ~ U[-gamma/2, gamma/2) of the
// Hamiltonian (eq. "Ham", onsite term), site n drawing counter n under `key`
__global__ void __launch_bounds__(256)
potential_kernel(double* __restrict__ pot, int64_t n, uint64_t key, double gamma) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const uint64_t z = mix64(key + static_cast<uint64_t>(c + 1) * kGamma);
    const double u = static_cast<double>(z >> 11) * (1.0 / 9007199254740992.0);
    pot[c] = gamma * (u - 0.5);
}

// Deterministic start vectors of the local and momentum-resolved spectral
// quantities (the local DOS and A(k, E) of Fig. "topi_demo"): column r is
// the unit vector of row rows[r], or the plane wave of momentum k[r] on
// orbital orb[r], sum_n exp(i k . (x, y, z)_n) |n, orb> / sqrt(sites).
struct SiteRows {
    int64_t row[kMaxStartColumns];
};
struct PlaneWaves {
    double k[kMaxStartColumns][3];
    int32_t orb[kMaxStartColumns];
};

template <typename T>
__global__ void __launch_bounds__(256)
site_block_kernel(T* __restrict__ V, int64_t N, int R, SiteRows rows) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= N * R) return;
    const int64_t i = c / R;
    const int r = static_cast<int>(c - i * R);
    V[2 * c] = i == rows.row[r] ? T(1) : T(0);
    V[2 * c + 1] = T(0);
}

template <typename T>
__global__ void __launch_bounds__(256)
plane_wave_kernel(T* __restrict__ V, int Lx, int Ly, int Lz, int R, PlaneWaves pw, double scale) {
    const int64_t N = 4 * static_cast<int64_t>(Lx) * Ly * Lz;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= N * R) return;
    const int64_t i = c / R;
    const int r = static_cast<int>(c - i * R);
    const int o = static_cast<int>(i & 3);
    const int64_t n = i >> 2;
    const int64_t x = n % Lx, y = (n / Lx) % Ly, z = n / (static_cast<int64_t>(Lx) * Ly);
    double re = 0.0, im = 0.0;
    if (o == pw.orb[r]) {
        const double ph = pw.k[r][0] * static_cast<double>(x) + pw.k[r][1] * static_cast<double>(y) +
                          pw.k[r][2] * static_cast<double>(z);
        sincos(ph, &im, &re);
        re *= scale;
        im *= scale;
    }
    V[2 * c] = static_cast<T>(re);
    V[2 * c + 1] = static_cast<T>(im);
}

}  // namespace

hipError_t launch_site_block(void* V, int64_t N, int R, const int64_t* rows, int dtype, hipStream_t s) {
    SiteRows sr{};
    for (int r = 0; r < R; ++r) sr.row[r] = rows[r];
    const int blocks = static_cast<int>((N * R + 255) / 256);
    if (dtype == KPM_C128)
        site_block_kernel<double><<<blocks, 256, 0, s>>>(static_cast<double*>(V), N, R, sr);
    else
        site_block_kernel<float><<<blocks, 256, 0, s>>>(static_cast<float*>(V), N, R, sr);
    return hipGetLastError();
}

hipError_t launch_plane_wave_block(void* V, const int L[3], int R, const double* k, const int32_t* orb, int dtype,
                                   hipStream_t s) {
    PlaneWaves pw{};
    for (int r = 0; r < R; ++r) {
        for (int j = 0; j < 3; ++j) pw.k[r][j] = k[3 * r + j];
        pw.orb[r] = orb[r];
    }
    const int64_t sites = static_cast<int64_t>(L[0]) * L[1] * L[2];
    const double scale = 1.0 / std::sqrt(static_cast<double>(sites));
    const int blocks = static_cast<int>((4 * sites * R + 255) / 256);
    if (dtype == KPM_C128)
        plane_wave_kernel<double><<<blocks, 256, 0, s>>>(static_cast<double*>(V), L[0], L[1], L[2], R, pw, scale);
    else
        plane_wave_kernel<float><<<blocks, 256, 0, s>>>(static_cast<float*>(V), L[0], L[1], L[2], R, pw, scale);
    return hipGetLastError();
}

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

hipError_t launch_potential(double* pot, int64_t nsite, double gamma, uint64_t seed, hipStream_t s) {
    if (nsite <= 0) return hipSuccess;
    // second output of SplitMix64 started at `seed` (the start block uses the first)
    const uint64_t key = mix64(seed + 2 * kGamma);
    potential_kernel<<<static_cast<int>((nsite + 255) / 256), 256, 0, s>>>(pot, nsite, key, gamma);
    return hipGetLastError();
}

}  // namespace kpm
