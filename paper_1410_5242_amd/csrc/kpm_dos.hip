// Density-of-states reconstruction from Chebyshev moments: the "second,
// computationally inexpensive step" that the paper leaves to the KPM
// literature (section "Problem Description").
//
//   mubar_n = (1/R) sum_r mu[r][n]            (stochastic trace over R vectors)
//   c_n     = g_n mubar_n                      (damping kernel)
//   rho(E)  = [c_0 + 2 sum_{n>=1} c_n T_n(x)] / (pi a sqrt(1 - x^2)),  x = (E-b)/a
//
// One thread per energy point runs the three-term Chebyshev recurrence
// T_{n+1} = 2x T_n - T_{n-1} in FP64; the c_n are staged through LDS in
// chunks shared by the workgroup.
#include "kpm_internal.h"

namespace kpm {
namespace {

constexpr int kDosThreads = 256;
constexpr int kChunk = 2048;

__device__ inline double damping(int kernel, double kparam, int n, int M) {
    if (kernel == KPM_JACKSON) {
        const double q = M_PI / (M + 1);
        return ((M - n + 1) * cos(q * n) + sin(q * n) * (cos(q) / sin(q))) / (M + 1);
    }
    if (kernel == KPM_LORENTZ) return sinh(kparam * (1.0 - static_cast<double>(n) / M)) / sinh(kparam);
    return 1.0;
}

__global__ void __launch_bounds__(kDosThreads)
dos_kernel(const double* __restrict__ mu, int R, int M, int kernel, double kparam, double a,
           double b, const double* __restrict__ E, int K, double* __restrict__ rho) {
    __shared__ double c[kChunk];
    const int k = blockIdx.x * kDosThreads + threadIdx.x;
    const double x = (k < K) ? (E[k] - b) / a : 0.0;
    double tm1 = 0.0, t0 = 1.0;   // T_{n-1}, T_n
    double s = 0.0;
    for (int n0 = 0; n0 < M; n0 += kChunk) {
        const int len = min(kChunk, M - n0);
        __syncthreads();
        for (int i = threadIdx.x; i < len; i += kDosThreads) {
            const int n = n0 + i;
            double m = 0.0;
            for (int r = 0; r < R; ++r) m += mu[static_cast<int64_t>(r) * M + n];
            c[i] = damping(kernel, kparam, n, M) * (m / R) * (n == 0 ? 1.0 : 2.0);
        }
        __syncthreads();
        for (int i = 0; i < len; ++i) {
            const int n = n0 + i;
            if (n == 0) {
                s += c[i];           // T_0 = 1
            } else {
                const double tn = (n == 1) ? x : 2.0 * x * t0 - tm1;
                tm1 = t0;
                t0 = tn;
                s += c[i] * tn;
            }
        }
    }
    if (k < K) rho[k] = (fabs(x) < 1.0) ? s / (M_PI * a * sqrt(1.0 - x * x)) : 0.0;
}

}  // namespace

hipError_t launch_dos(const double* mu, int R, int M, int kernel, double kparam, double a,
                      double b, const double* E, int K, double* rho, hipStream_t s) {
    dos_kernel<<<(K + kDosThreads - 1) / kDosThreads, kDosThreads, 0, s>>>(
        mu, R, M, kernel, kparam, a, b, E, K, rho);
    return hipGetLastError();
}

}  // namespace kpm
