// The BLAS level-1 kernels of the naive KPM-DOS algorithm (Alg.
// "kpm_naive": per step one SpMV u <- H v, then u <- u - b v (axpy),
// w <- -w (scal), w <- w + 2a u (axpy), eta_2m = <v|v> (nrm2) and
// eta_2m+1 = <w|v> (dot), one call each, with the traffic of Table
// "kpm_analysis").  They exist to measure what the fused sweep saves; each
// is a plain HBM stream: 16 bytes per lane and instruction, a grid-stride
// loop over whole 16-byte units and a scalar tail.
//
// The scalar products accumulate in FP64 (complex64 elements are promoted
// before the products) and are reduced in two stages, per-workgroup
// partials and one workgroup that sums them in index order, so a result
// does not depend on timing.
#include <mutex>
#include <vector>

#include "kpm_internal.h"

namespace kpm {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 2048;   // 8 workgroups per CU

typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

// 16-byte unit of a vector of reals of type T
template <typename T> struct Unit;
template <> struct Unit<double> { using type = d2; static constexpr int kReals = 2; };
template <> struct Unit<float> { using type = f4; static constexpr int kReals = 4; };

int blocks_for(int64_t units) {
    const int64_t b = (units + kThreads - 1) / kThreads;
    return static_cast<int>(b < 1 ? 1 : (b > kMaxBlocks ? kMaxBlocks : b));
}

// y <- y + alpha x over nr reals
template <typename T>
__global__ void __launch_bounds__(kThreads)
axpy_kernel(int64_t nr, T alpha, const T* __restrict__ x, T* __restrict__ y) {
    using U = typename Unit<T>::type;
    constexpr int K = Unit<T>::kReals;
    const int64_t nu = nr / K;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
    const U* xu = reinterpret_cast<const U*>(x);
    U* yu = reinterpret_cast<U*>(y);
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < nu; i += stride)
        yu[i] = yu[i] + alpha * xu[i];
    const int64_t t = nu * K + static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (t < nr) y[t] = y[t] + alpha * x[t];
}

// x <- alpha x over nr reals
template <typename T>
__global__ void __launch_bounds__(kThreads)
scal_kernel(int64_t nr, T alpha, T* __restrict__ x) {
    using U = typename Unit<T>::type;
    constexpr int K = Unit<T>::kReals;
    const int64_t nu = nr / K;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
    U* xu = reinterpret_cast<U*>(x);
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < nu; i += stride)
        xu[i] = alpha * xu[i];
    const int64_t t = nu * K + static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (t < nr) x[t] = alpha * x[t];
}

// Workgroup sum of (re, im) in a fixed order: wave shuffles, then the waves
// in index order.
__device__ inline void block_sum(double& re, double& im) {
    __shared__ double s[2][kThreads / 64];
    for (int o = 32; o > 0; o >>= 1) {
        re += __shfl_xor(re, o);
        im += __shfl_xor(im, o);
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s[0][wave] = re;
        s[1][wave] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        re = 0.0;
        im = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) {
            re += s[0][w];
            im += s[1][w];
        }
    }
}

// part[block] = sum over this block's elements of conj(x_i) y_i (n complex
// elements); NRM: x == y, the imaginary part is 0 by definition.
template <typename T, bool NRM>
__global__ void __launch_bounds__(kThreads)
dot_partial_kernel(int64_t n, const T* __restrict__ x, const T* __restrict__ y, double* __restrict__ part) {
    using U = typename Unit<T>::type;
    constexpr int K = Unit<T>::kReals;   // reals per unit: K / 2 complex
    const int64_t nu = 2 * n / K;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
    const U* xu = reinterpret_cast<const U*>(x);
    const U* yu = reinterpret_cast<const U*>(y);
    double re = 0.0, im = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < nu; i += stride) {
        const U a = xu[i];
        const U b = NRM ? a : yu[i];
#pragma unroll
        for (int c = 0; c < K; c += 2) {
            const double ar = a[c], ai = a[c + 1], br = b[c], bi = b[c + 1];
            re = fma(ar, br, fma(ai, bi, re));
            if (!NRM) im = fma(ar, bi, fma(-ai, br, im));
        }
    }
    // a complex element left over (complex64 with n odd)
    const int64_t t = nu * (K / 2) + static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (t < n) {
        const double ar = x[2 * t], ai = x[2 * t + 1];
        const double br = NRM ? ar : static_cast<double>(y[2 * t]);
        const double bi = NRM ? ai : static_cast<double>(y[2 * t + 1]);
        re = fma(ar, br, fma(ai, bi, re));
        if (!NRM) im = fma(ar, bi, fma(-ai, br, im));
    }
    block_sum(re, im);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = re;
        part[2 * blockIdx.x + 1] = im;
    }
}

// out[0..1] = sum of the nb partials, in index order per thread and then
// over the threads in a fixed order
__global__ void __launch_bounds__(kThreads)
dot_final_kernel(const double* __restrict__ part, int nb, double* __restrict__ out) {
    double re = 0.0, im = 0.0;
    const int per = (nb + kThreads - 1) / kThreads;
    const int b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
    for (int b = b0; b < b1; ++b) {
        re += part[2 * b];
        im += part[2 * b + 1];
    }
    block_sum(re, im);
    if (threadIdx.x == 0) {
        out[0] = re;
        out[1] = im;
    }
}

// v[i] = V[i R + r] for i < n (complex elements)
template <typename T>
__global__ void __launch_bounds__(kThreads)
column_kernel(int64_t n, int R, int r, const T* __restrict__ V, T* __restrict__ v) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride) {
        v[2 * i] = V[2 * (i * R + r)];
        v[2 * i + 1] = V[2 * (i * R + r) + 1];
    }
}

// dst [n][G] <- columns c0 .. c0 + G - 1 of src [n][R] (a column group of a
// block, 64-bit indexing: the block may exceed 4 GiB)
template <typename T>
__global__ void __launch_bounds__(kThreads)
columns_kernel(int64_t n, int R, int c0, int G, const T* __restrict__ V, T* __restrict__ v) {
    const int64_t total = n * G;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; k < total; k += stride) {
        const int64_t i = k / G;
        const int64_t src = i * R + c0 + (k - i * G);
        v[2 * k] = V[2 * src];
        v[2 * k + 1] = V[2 * src + 1];
    }
}

template <typename T>
hipError_t axpy_t(int64_t n, double alpha, const void* x, void* y, hipStream_t s) {
    const int64_t nr = 2 * n;
    axpy_kernel<T><<<blocks_for(nr / Unit<T>::kReals), kThreads, 0, s>>>(nr, static_cast<T>(alpha),
                                                                          static_cast<const T*>(x), static_cast<T*>(y));
    return hipGetLastError();
}

template <typename T>
hipError_t scal_t(int64_t n, double alpha, void* x, hipStream_t s) {
    const int64_t nr = 2 * n;
    scal_kernel<T><<<blocks_for(nr / Unit<T>::kReals), kThreads, 0, s>>>(nr, static_cast<T>(alpha), static_cast<T*>(x));
    return hipGetLastError();
}

template <typename T>
hipError_t dot_t(int64_t n, const void* x, const void* y, double* part, double* out, hipStream_t s) {
    const int nb = blocks_for(2 * n / Unit<T>::kReals);
    if (x == y)
        dot_partial_kernel<T, true><<<nb, kThreads, 0, s>>>(n, static_cast<const T*>(x), static_cast<const T*>(y), part);
    else
        dot_partial_kernel<T, false><<<nb, kThreads, 0, s>>>(n, static_cast<const T*>(x), static_cast<const T*>(y), part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dot_final_kernel<<<1, kThreads, 0, s>>>(part, nb, out);
    return hipGetLastError();
}

template <typename T>
hipError_t column_t(int64_t n, int R, int r, const void* V, void* v, hipStream_t s) {
    column_kernel<T><<<blocks_for(n), kThreads, 0, s>>>(n, R, r, static_cast<const T*>(V), static_cast<T*>(v));
    return hipGetLastError();
}

// Partial sums of kpm_dot_noalloc: one array per GPU, held for the life of
// the process.  Host code never passes this name to a kernel (on the host it
// is a stand-in, not a device address); it resolves the device address once
// per device with hipGetSymbolAddress and uses that.
static __device__ __align__(256) double scratch[2 * kMaxBlocks];

std::mutex g_scratch_lock;
std::vector<double*> g_scratch_ptr;   // per device; nullptr until resolved

}  // namespace

int naive_dot_partials() { return kMaxBlocks; }

hipError_t dot_scratch(double** out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> g(g_scratch_lock);
    if (static_cast<int>(g_scratch_ptr.size()) <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_axpy(int dtype, int64_t n, double alpha, const void* x, void* y, hipStream_t s) {
    return dtype == KPM_C128 ? axpy_t<double>(n, alpha, x, y, s) : axpy_t<float>(n, alpha, x, y, s);
}

hipError_t launch_scal(int dtype, int64_t n, double alpha, void* x, hipStream_t s) {
    return dtype == KPM_C128 ? scal_t<double>(n, alpha, x, s) : scal_t<float>(n, alpha, x, s);
}

hipError_t launch_dot(int dtype, int64_t n, const void* x, const void* y, double* part, double* out, hipStream_t s) {
    return dtype == KPM_C128 ? dot_t<double>(n, x, y, part, out, s) : dot_t<float>(n, x, y, part, out, s);
}

hipError_t launch_column(int dtype, int64_t n, int R, int r, const void* V, void* v, hipStream_t s) {
    return dtype == KPM_C128 ? column_t<double>(n, R, r, V, v, s) : column_t<float>(n, R, r, V, v, s);
}

hipError_t launch_columns(int dtype, int64_t n, int R, int c0, int G, const void* V, void* v, hipStream_t s) {
    if (dtype == KPM_C128)
        columns_kernel<double><<<blocks_for(n * G), kThreads, 0, s>>>(n, R, c0, G, static_cast<const double*>(V),
                                                                      static_cast<double*>(v));
    else
        columns_kernel<float><<<blocks_for(n * G), kThreads, 0, s>>>(n, R, c0, G, static_cast<const float*>(V),
                                                                     static_cast<float*>(v));
    return hipGetLastError();
}

}  // namespace kpm
