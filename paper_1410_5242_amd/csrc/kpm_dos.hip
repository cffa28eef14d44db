// Density-of-states reconstruction from Chebyshev moments: the cheap
// follow-up to the moment computation, whose formulas the paper takes from
// the KPM literature (section "Problem Description").
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

// Instance blockIdx.y of a batch: moments mu + inst * R * ld (the first M
// of each row of length ld), scaling a[inst], b[inst] (device arrays) or the
// scalars when those are NULL, output rho + inst * K.
__global__ void __launch_bounds__(kDosThreads)
dos_kernel(const double* __restrict__ mu, int R, int ld, int M, int kernel, double kparam, double a0,
           double b0, const double* __restrict__ a_arr, const double* __restrict__ b_arr,
           const double* __restrict__ E, int K, double* __restrict__ rho) {
    __shared__ double c[kChunk];
    const int inst = blockIdx.y;
    mu += static_cast<int64_t>(inst) * R * ld;
    rho += static_cast<int64_t>(inst) * K;
    const double a = a_arr ? a_arr[inst] : a0;
    const double b = b_arr ? b_arr[inst] : b0;
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
            for (int r = 0; r < R; ++r) m += mu[static_cast<int64_t>(r) * ld + n];
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

// rho[inst][k] <- rho[inst][k] / sum_j rho[inst][j] (sum in index order):
// DOS masses per bin of a uniform energy grid.
__global__ void __launch_bounds__(kDosThreads)
normalize_rows_kernel(double* __restrict__ rho, int K) {
    __shared__ double part[kDosThreads];
    double* r = rho + static_cast<int64_t>(blockIdx.x) * K;
    const int per = (K + kDosThreads - 1) / kDosThreads;
    const int lo = threadIdx.x * per, hi = min(K, lo + per);
    double s = 0.0;
    for (int k = lo; k < hi; ++k) s += r[k];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < kDosThreads; ++i) t += part[i];
        part[0] = t;
    }
    __syncthreads();
    const double tot = part[0];
    for (int k = threadIdx.x; k < K; k += kDosThreads) r[k] = tot != 0.0 ? r[k] / tot : 0.0;
}

// x[inst][f] = (1/R) sum_r mu[inst][r][f] for f < n_mom (float), then
// x[inst][n_mom] = extra[inst] when extra is set.
__global__ void __launch_bounds__(kDosThreads)
features_kernel(const double* __restrict__ mu, int n_inst, int R, int ld, int n_mom,
                const float* __restrict__ extra, float* __restrict__ x) {
    const int width = n_mom + (extra ? 1 : 0);
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= static_cast<int64_t>(n_inst) * width) return;
    const int inst = static_cast<int>(i / width), f = static_cast<int>(i % width);
    if (f == n_mom) {
        x[i] = extra[inst];
        return;
    }
    const double* m = mu + static_cast<int64_t>(inst) * R * ld + f;
    double s = 0.0;
    for (int r = 0; r < R; ++r) s += m[static_cast<int64_t>(r) * ld];
    x[i] = static_cast<float>(s / R);
}

}  // namespace

hipError_t launch_dos(const double* mu, int R, int M, int kernel, double kparam, double a,
                      double b, const double* E, int K, double* rho, hipStream_t s) {
    dos_kernel<<<dim3((K + kDosThreads - 1) / kDosThreads, 1), kDosThreads, 0, s>>>(
        mu, R, M, M, kernel, kparam, a, b, nullptr, nullptr, E, K, rho);
    return hipGetLastError();
}

hipError_t launch_dos_batched(const double* mu, int n_inst, int R, int ld, int M, int kernel, double kparam,
                              const double* a, const double* b, const double* E, int K, int masses,
                              double* rho, hipStream_t s) {
    dos_kernel<<<dim3((K + kDosThreads - 1) / kDosThreads, n_inst), kDosThreads, 0, s>>>(
        mu, R, ld, M, kernel, kparam, 1.0, 0.0, a, b, E, K, rho);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !masses) return e;
    normalize_rows_kernel<<<n_inst, kDosThreads, 0, s>>>(rho, K);
    return hipGetLastError();
}

hipError_t launch_features(const double* mu, int n_inst, int R, int ld, int n_mom, const float* extra,
                           float* x, hipStream_t s) {
    const int64_t n = static_cast<int64_t>(n_inst) * (n_mom + (extra ? 1 : 0));
    features_kernel<<<static_cast<int>((n + kDosThreads - 1) / kDosThreads), kDosThreads, 0, s>>>(
        mu, n_inst, R, ld, n_mom, extra, x);
    return hipGetLastError();
}

}  // namespace kpm
