// Spectral bounds from a few Lanczos steps (section "Problem Description":
// the scaling a, b may come from Gershgorin's theorem or from a few Lanczos
// sweeps).  The three-term recurrence
//   w = H q_j - alpha_j q_j - beta_{j-1} q_{j-1},  alpha_j = <q_j|H q_j>,
//   beta_j = |w|,  q_{j+1} = w / beta_j
// runs entirely on the device: alpha and beta stay in device memory and the
// vector kernels read them from there, so the host does not wait inside the
// loop.  The extreme eigenvalues of the tridiagonal matrix T_k (the extreme
// Ritz values) are found by bisection on Sturm sequence counts in one
// workgroup.  Without reorthogonalisation the Ritz values may repeat, which
// does not move the extremes.
#include "kpm_internal.h"

#include <cfloat>

namespace kpm {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 2048;

int blocks_for(int64_t n) {
    const int64_t b = (n + kThreads - 1) / kThreads;
    return static_cast<int>(b < 1 ? 1 : (b > kMaxBlocks ? kMaxBlocks : b));
}

// w <- w - alpha q - beta qp over n complex elements; alpha = ab[0] (the real
// part of <q|Hq>), beta = ab[1] (0 for the first step)
template <typename T>
__global__ void __launch_bounds__(kThreads)
lanczos_update_kernel(int64_t n, const double* __restrict__ ab, const T* __restrict__ q, const T* __restrict__ qp,
                      T* __restrict__ w) {
    const T alpha = static_cast<T>(ab[0]), beta = static_cast<T>(ab[1]);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < 2 * n; i += stride)
        w[i] = w[i] - alpha * q[i] - beta * qp[i];
}

// q <- w / sqrt(nrm[0]); records beta = sqrt(nrm[0]) at *beta_out (thread 0
// of block 0); a zero norm (invariant subspace found) leaves q = 0
template <typename T>
__global__ void __launch_bounds__(kThreads)
lanczos_normalise_kernel(int64_t n, const double* __restrict__ nrm, const T* __restrict__ w, T* __restrict__ q,
                         double* __restrict__ beta_out) {
    const double b = sqrt(nrm[0]);
    const T inv = b > 0.0 ? static_cast<T>(1.0 / b) : T(0);
    if (blockIdx.x == 0 && threadIdx.x == 0) *beta_out = b;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < 2 * n; i += stride)
        q[i] = w[i] * inv;
}

// ab_j[0] <- Re dot_j[0] (alpha_j), ab_j[1] <- beta_{j-1}
__global__ void lanczos_pack_kernel(const double* __restrict__ dot, const double* __restrict__ beta_prev,
                                    double* __restrict__ ab) {
    ab[0] = dot[0];
    ab[1] = beta_prev ? *beta_prev : 0.0;
}

// Number of eigenvalues of the k x k tridiagonal matrix (diagonal d, off
// diagonal e[0 .. k-2]) below x: the negative pivots of the LDL^T
// factorisation of T - x (Sturm count).
__device__ int sturm_count(const double* d, const double* e, int k, double x) {
    int c = 0;
    double q = d[0] - x;
    if (q < 0.0) ++c;
    for (int i = 1; i < k; ++i) {
        const double qq = (q == 0.0) ? DBL_EPSILON * (fabs(e[i - 1]) + DBL_MIN) : q;
        q = d[i] - x - e[i - 1] * e[i - 1] / qq;
        if (q < 0.0) ++c;
    }
    return c;
}

// out[0] = smallest, out[1] = largest eigenvalue of T_k (alpha_j = ab[2 j],
// beta_j = beta[j]); thread 0 bisects the Gershgorin interval of T_k to
// full double precision
__global__ void tridiag_extremes_kernel(const double* __restrict__ ab, const double* __restrict__ beta, int k,
                                        double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    constexpr int kMax = 1024;
    double d[kMax], e[kMax];
    for (int i = 0; i < k; ++i) {
        d[i] = ab[2 * i];
        e[i] = beta[i];
    }
    double lo = DBL_MAX, hi = -DBL_MAX;
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < k ? fabs(e[i]) : 0.0);
        lo = fmin(lo, d[i] - r);
        hi = fmax(hi, d[i] + r);
    }
    for (int which = 0; which < 2; ++which) {
        // which 0: smallest (count >= 1), 1: largest (count >= k)
        const int target = which == 0 ? 1 : k;
        double a = lo, b = hi;
        for (int it = 0; it < 200 && b - a > 4.0 * DBL_EPSILON * fmax(fabs(a), fabs(b)); ++it) {
            const double m = 0.5 * (a + b);
            if (sturm_count(d, e, k, m) >= target)
                b = m;
            else
                a = m;
        }
        out[which] = 0.5 * (a + b);
    }
}

template <typename T>
hipError_t update_t(int64_t n, const double* ab, const void* q, const void* qp, void* w, hipStream_t s) {
    lanczos_update_kernel<T><<<blocks_for(2 * n), kThreads, 0, s>>>(n, ab, static_cast<const T*>(q),
                                                                   static_cast<const T*>(qp), static_cast<T*>(w));
    return hipGetLastError();
}

template <typename T>
hipError_t normalise_t(int64_t n, const double* nrm, const void* w, void* q, double* beta_out, hipStream_t s) {
    lanczos_normalise_kernel<T><<<blocks_for(2 * n), kThreads, 0, s>>>(n, nrm, static_cast<const T*>(w),
                                                                      static_cast<T*>(q), beta_out);
    return hipGetLastError();
}

}  // namespace

int lanczos_max_steps() { return 1024; }

hipError_t launch_lanczos_update(int dtype, int64_t n, const double* ab, const void* q, const void* qp, void* w,
                                 hipStream_t s) {
    return dtype == KPM_C128 ? update_t<double>(n, ab, q, qp, w, s) : update_t<float>(n, ab, q, qp, w, s);
}

hipError_t launch_lanczos_normalise(int dtype, int64_t n, const double* nrm, const void* w, void* q, double* beta_out,
                                    hipStream_t s) {
    return dtype == KPM_C128 ? normalise_t<double>(n, nrm, w, q, beta_out, s)
                             : normalise_t<float>(n, nrm, w, q, beta_out, s);
}

hipError_t launch_lanczos_pack(const double* dot, const double* beta_prev, double* ab, hipStream_t s) {
    lanczos_pack_kernel<<<1, 1, 0, s>>>(dot, beta_prev, ab);
    return hipGetLastError();
}

hipError_t launch_tridiag_extremes(const double* ab, const double* beta, int k, double* out, hipStream_t s) {
    tridiag_extremes_kernel<<<1, 64, 0, s>>>(ab, beta, k, out);
    return hipGetLastError();
}

}  // namespace kpm
