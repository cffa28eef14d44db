// Spectral bounds from a short Lanczos run (section "Problem Description":
// the scaling a, b comes either from Gershgorin's theorem or from Lanczos
// iterations).  The three-term recurrence
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

// w <- w - alpha q - beta qp over n complex elements; alpha = Re dot[0]
// (<q|Hq>), beta = *beta_prev (0 for the first step, beta_prev NULL); thread
// 0 of block 0 records (alpha, beta) at ab
template <typename T>
__global__ void __launch_bounds__(kThreads)
lanczos_update_kernel(int64_t n, const double* __restrict__ dot, const double* __restrict__ beta_prev,
                      double* __restrict__ ab, const T* __restrict__ q, const T* __restrict__ qp, T* __restrict__ w) {
    const double a = dot[0], b = beta_prev ? *beta_prev : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ab[0] = a;
        ab[1] = b;
    }
    const T alpha = static_cast<T>(a), beta = static_cast<T>(b);
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

constexpr int kMaxSteps = 1024;
constexpr int kLanes = 64;

// out[0] = smallest, out[1] = largest eigenvalue of T_k (alpha_j = ab[2 j],
// beta_j = beta[j]).  One wave: the matrix is copied to LDS, then each round
// of multisection evaluates 64 Sturm counts at equally spaced points of the
// current interval (one per lane) and keeps the sub-interval where the
// count reaches its target, shrinking the interval 65-fold per round.
__global__ void __launch_bounds__(kLanes)
tridiag_extremes_kernel(const double* __restrict__ ab, const double* __restrict__ beta, int k,
                        double* __restrict__ out) {
    __shared__ double d[kMaxSteps], e[kMaxSteps];
    __shared__ double lo_s, hi_s;
    __shared__ int first;
    const int t = threadIdx.x;
    for (int i = t; i < k; i += kLanes) {
        d[i] = ab[2 * i];
        e[i] = beta[i];
    }
    __syncthreads();
    if (t == 0) {
        // Gershgorin interval of T_k
        double lo = DBL_MAX, hi = -DBL_MAX;
        for (int i = 0; i < k; ++i) {
            const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < k ? fabs(e[i]) : 0.0);
            lo = fmin(lo, d[i] - r);
            hi = fmax(hi, d[i] + r);
        }
        lo_s = lo;
        hi_s = hi;
    }
    __syncthreads();
    const double glo = lo_s, ghi = hi_s;
    for (int which = 0; which < 2; ++which) {
        // which 0: smallest (count >= 1), 1: largest (count >= k)
        const int target = which == 0 ? 1 : k;
        double a = glo, b = ghi;
        for (int round = 0; round < 16 && b - a > 4.0 * DBL_EPSILON * fmax(fabs(a), fabs(b)); ++round) {
            const double h = (b - a) / (kLanes + 1);
            const double x = a + h * (t + 1);
            const bool reached = sturm_count(d, e, k, x) >= target;
            // lowest lane whose point reaches the target (counts grow with x)
            if (t == 0) first = kLanes;
            __syncthreads();
            if (reached) atomicMin(&first, t);
            __syncthreads();
            const int f = first;
            __syncthreads();
            b = f < kLanes ? a + h * (f + 1) : b;
            a = a + h * f;
        }
        if (t == 0) out[which] = 0.5 * (a + b);
    }
}

template <typename T>
hipError_t update_t(int64_t n, const double* dot, const double* beta_prev, double* ab, const void* q, const void* qp,
                    void* w, hipStream_t s) {
    lanczos_update_kernel<T><<<blocks_for(2 * n), kThreads, 0, s>>>(n, dot, beta_prev, ab, static_cast<const T*>(q),
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

int lanczos_max_steps() { return kMaxSteps; }

hipError_t launch_lanczos_update(int dtype, int64_t n, const double* dot, const double* beta_prev, double* ab,
                                 const void* q, const void* qp, void* w, hipStream_t s) {
    return dtype == KPM_C128 ? update_t<double>(n, dot, beta_prev, ab, q, qp, w, s)
                             : update_t<float>(n, dot, beta_prev, ab, q, qp, w, s);
}

hipError_t launch_lanczos_normalise(int dtype, int64_t n, const double* nrm, const void* w, void* q, double* beta_out,
                                    hipStream_t s) {
    return dtype == KPM_C128 ? normalise_t<double>(n, nrm, w, q, beta_out, s)
                             : normalise_t<float>(n, nrm, w, q, beta_out, s);
}

hipError_t launch_tridiag_extremes(const double* ab, const double* beta, int k, double* out, hipStream_t s) {
    tridiag_extremes_kernel<<<1, kLanes, 0, s>>>(ab, beta, k, out);
    return hipGetLastError();
}

}  // namespace kpm
