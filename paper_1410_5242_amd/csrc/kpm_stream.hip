// Attainable memory bandwidth: STREAM-style copy and triad kernels.
//
// The paper measures the attainable bandwidth b of each machine with a copy
// kernel and bounds every kernel by it (Table "tab:architectures", the
// roofline of eq. "eq:roofline_mem"); these kernels give the same reference
// on MI355X, written for its memory system: every lane moves 16 bytes per
// instruction (global_load/store_dwordx4), each thread keeps four such loads
// in flight before it stores, and stores may carry the non-temporal hint so
// that written lines do not displace anything in L2 / the last-level cache.
//
//   copy:   c[i] = a[i]                  (16 bytes read and 16 written per unit)
//   triad:  c[i] = a[i] + s * b[i]       (FP64 pairs; 32 read, 16 written per unit)
//   read:   c[g] = sum of the FP64 values workgroup g read (16 bytes read per
//           unit; eight loads in flight per thread, non-temporal loads when
//           asked, so that the last-level cache keeps nothing of the stream)
//
// On MI355X one 256-lane workgroup per compute unit streams fastest: more
// workgroups interleave more address streams and lose bandwidth.
#include "kpm_internal.h"

namespace kpm {
namespace {

constexpr int kThreads = 256;
constexpr int kUnroll = 4;

typedef double d2 __attribute__((ext_vector_type(2)));

template <bool NT>
__device__ inline void put(d2* p, d2 v) {
    if (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <bool NT>
__global__ void __launch_bounds__(kThreads)
copy_kernel(const d2* __restrict__ a, d2* __restrict__ c, int64_t n) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
    int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
        d2 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = a[i + u * stride];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) put<NT>(c + i + u * stride, v[u]);
    }
    for (; i < n; i += stride) put<NT>(c + i, a[i]);
}

template <bool NT>
__global__ void __launch_bounds__(kThreads)
triad_kernel(const d2* __restrict__ a, const d2* __restrict__ b, d2* __restrict__ c, double s, int64_t n) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
    int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
        d2 x[kUnroll], y[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            x[u] = a[i + u * stride];
            y[u] = b[i + u * stride];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) put<NT>(c + i + u * stride, x[u] + s * y[u]);
    }
    for (; i < n; i += stride) put<NT>(c + i, a[i] + s * b[i]);
}

template <bool NT>
__device__ inline d2 get(const d2* p) {
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}

template <bool NT>
__global__ void __launch_bounds__(kThreads)
read_kernel(const d2* __restrict__ a, double* __restrict__ part, int64_t n) {
    constexpr int U = 2 * kUnroll;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
    int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    d2 acc = {0.0, 0.0};
    for (; i + (U - 1) * stride < n; i += U * stride) {
        d2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = get<NT>(a + i + u * stride);
#pragma unroll
        for (int u = 0; u < U; ++u) acc += v[u];
    }
    for (; i < n; i += stride) acc += get<NT>(a + i);
    // workgroup sum in a fixed order: wave butterflies, then the waves in index order
    double s = acc.x + acc.y;
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    __shared__ double w[kThreads / 64];
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kThreads / 64; ++k) t += w[k];
        part[blockIdx.x] = t;
    }
}

}  // namespace

int stream_grid(int64_t units, int wg_per_cu) {
    int64_t grid = static_cast<int64_t>(device_cus()) * wg_per_cu;
    const int64_t need = (units + kThreads - 1) / kThreads;
    if (grid > need) grid = need;
    return static_cast<int>(grid < 1 ? 1 : grid);
}

hipError_t launch_stream(int kind, int nontemporal, void* c, const void* a, const void* b, double s, int64_t units,
                         int wg_per_cu, hipStream_t st) {
    if (units <= 0) return hipSuccess;
    const int g = stream_grid(units, wg_per_cu);
    const d2* A = static_cast<const d2*>(a);
    d2* C = static_cast<d2*>(c);
    if (kind == KPM_STREAM_READ) {
        double* P = static_cast<double*>(c);
        if (nontemporal) read_kernel<true><<<g, kThreads, 0, st>>>(A, P, units);
        else read_kernel<false><<<g, kThreads, 0, st>>>(A, P, units);
    } else if (kind == KPM_STREAM_COPY) {
        if (nontemporal) copy_kernel<true><<<g, kThreads, 0, st>>>(A, C, units);
        else copy_kernel<false><<<g, kThreads, 0, st>>>(A, C, units);
    } else {
        const d2* B = static_cast<const d2*>(b);
        if (nontemporal) triad_kernel<true><<<g, kThreads, 0, st>>>(A, B, C, s, units);
        else triad_kernel<false><<<g, kThreads, 0, st>>>(A, B, C, s, units);
    }
    return hipGetLastError();
}

}  // namespace kpm
