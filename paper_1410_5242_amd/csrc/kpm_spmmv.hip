// Small kernels around the fused sweep (deterministic reduction of the
// per-workgroup scalar-product partials, the eta -> mu doubling identity,
// the moment sanity check), the sweep's tuning state and its dispatch to the
// per-precision instantiations.
#include <atomic>

#include "kpm_internal.h"

namespace kpm {
namespace {


// eta[sweep] from the partial sums of nslots consecutive sweeps, one
// workgroup per sweep.  Each output sums the workgroup partials in kChunks
// contiguous runs (in parallel, each in index order), then the runs in
// order: the same fixed summation order on every call, with 1/kChunks of
// the dependent-load chain of a single running sum.
constexpr int kChunks = 8;
constexpr int kMaxN3 = 3 * 64;

__global__ void __launch_bounds__(256)
reduce_partials_kernel(const double* __restrict__ part, int grid, int R, int sweep0,
                       double* __restrict__ eta) {
    __shared__ double run[kChunks][kMaxN3];
    const int n3 = 3 * R;
    const double* p = part + static_cast<int64_t>(blockIdx.x) * grid * n3;
    const int sweep = sweep0 + blockIdx.x;
    for (int j = threadIdx.x; j < kChunks * n3; j += blockDim.x) {
        const int c = j / n3, i = j % n3;
        const int g0 = grid * c / kChunks, g1 = grid * (c + 1) / kChunks;
        double acc = 0.0;
        for (int g = g0; g < g1; ++g) acc += p[static_cast<int64_t>(g) * n3 + i];
        run[c][i] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n3; i += blockDim.x) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < kChunks; ++c) acc += run[c][i];
        const int q = i / R, r = i % R;
        if (q == 0) {
            eta[(static_cast<int64_t>(2 * sweep) * R + r) * 2] = acc;
            eta[(static_cast<int64_t>(2 * sweep) * R + r) * 2 + 1] = 0.0;
        } else {
            eta[(static_cast<int64_t>(2 * sweep + 1) * R + r) * 2 + (q - 1)] = acc;
        }
    }
}

__global__ void __launch_bounds__(256) zero_ints_kernel(int* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// dst[i] = src[i] over n 16-byte units, grid-stride
__global__ void __launch_bounds__(256)
copy16_kernel(const int4* __restrict__ src, int4* __restrict__ dst, int64_t n, int tail8) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
    // a block of complex64 with an odd element count ends in half a unit
    if (tail8 && blockIdx.x == 0 && threadIdx.x == 0)
        *reinterpret_cast<int2*>(dst + n) = *reinterpret_cast<const int2*>(src + n);
}

// mu_{2m} = 2 eta_{2m} - mu_0, mu_{2m+1} = 2 Re eta_{2m+1} - mu_1.
__global__ void __launch_bounds__(256)
eta_to_mu_kernel(const double* __restrict__ eta, int R, int M, double* __restrict__ mu) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= static_cast<int64_t>(R) * M) return;
    const int r = static_cast<int>(i / M), n = static_cast<int>(i % M);
    const double ref = eta[(static_cast<int64_t>(n & 1) * R + r) * 2];   // mu_0 or mu_1
    mu[i] = 2.0 * eta[(static_cast<int64_t>(n) * R + r) * 2] - ref;
}

// flag = 1 if any moment is non-finite or |mu_n| > mu_0 (1 + 1e-6).
__global__ void __launch_bounds__(256)
check_moments_kernel(const double* __restrict__ mu, int R, int M, int* __restrict__ flag) {
    int bad = 0;
    for (int64_t i = threadIdx.x; i < static_cast<int64_t>(R) * M; i += blockDim.x) {
        const int r = static_cast<int>(i / M);
        const double m0 = mu[static_cast<int64_t>(r) * M];
        const double x = mu[i];
        if (!isfinite(x) || fabs(x) > m0 * (1.0 + 1e-6) + 1e-300) bad = 1;
    }
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) *flag = bad;
}

}  // namespace

namespace {
// wg_per_cu, xcd_ways, chunk_tiles, pencil, dynamic, prefetch, stream,
// lattice, gather, tile_order, slab, gather_tile
constexpr kpm_sweep_tuning kDefaultTuning = {0, kXcds, 8, 16, 0, 2, 3, 1, 1, 3, 4, 0};
std::mutex g_tuning_lock;
kpm_sweep_tuning g_tuning = kDefaultTuning;
thread_local const kpm_sweep_tuning* t_call = nullptr;   // snapshot of the running call

kpm_sweep_tuning global_tuning() {
    std::lock_guard<std::mutex> g(g_tuning_lock);
    return g_tuning;
}
}  // namespace

kpm_sweep_tuning default_tuning() { return kDefaultTuning; }
kpm_sweep_tuning get_tuning() { return t_call ? *t_call : global_tuning(); }
void set_tuning(const kpm_sweep_tuning& t) {
    std::lock_guard<std::mutex> g(g_tuning_lock);
    g_tuning = t;
}

TuningScope::TuningScope(const kpm_sweep_tuning* override)
    : snap_(override ? *override : get_tuning()), prev_(t_call) {
    t_call = &snap_;
}
TuningScope::~TuningScope() { t_call = prev_; }

kpm_status check_tuning(const kpm_sweep_tuning& t) {
    if (t.wg_per_cu < 0 || t.xcd_ways < 0 || t.chunk_tiles < 0 || t.pencil < 0 || t.dynamic < 0 ||
        t.prefetch < 0 || t.prefetch > 2 || t.stream < 0 || t.stream > 3 || t.lattice < 0 || t.lattice > 2 ||
        t.gather < 0 || t.gather > 4 || t.tile_order < 0 || t.tile_order > 3 || t.slab < 0 || t.gather_tile < 0) {
        set_error("tuning field out of range (negative, or above its largest option)");
        return KPM_EINVAL;
    }
    if (t.wg_per_cu > 64 || t.xcd_ways > 64 || t.chunk_tiles > (1 << 20) || t.pencil > 4096 || t.slab > 65536 ||
        t.gather_tile > 4096) {
        set_error("tuning field out of range");
        return KPM_EINVAL;
    }
    return KPM_OK;
}

int device_cus() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    static std::atomic<int> cached[64];
    if (dev < 0 || dev >= 64) return 256;
    int c = cached[dev].load(std::memory_order_relaxed);
    if (!c) {
        hipDeviceProp_t p;
        c = hipGetDeviceProperties(&p, dev) == hipSuccess ? p.multiProcessorCount : 256;
        cached[dev].store(c, std::memory_order_relaxed);
    }
    return c;
}

bool use_gather(int dtype, int R, int64_t nrows) {
    const kpm_sweep_tuning g_tuning = get_tuning();
    if (g_tuning.gather == 2) return false;
    // 32-bit buffer offsets with room for the read-ahead past the last pass
    const uint64_t rs = dtype == KPM_C128 ? 8 : 4;
    const uint64_t lim = (1ull << 32) - (1ull << 24);
    const uint64_t n = static_cast<uint64_t>(nrows);
    if (n * R * 2 * rs >= lim || n * kWidth * 2 * rs >= lim) return false;
    return g_tuning.gather == 1 || g_tuning.gather >= 3 || R != 32;
}

int sweep_grid(int dtype, int R, int64_t nrows, bool window) {
    const kpm_sweep_tuning g_tuning = get_tuning();
    int per_cu;
    if (use_gather(dtype, R, nrows)) {
        // 16 waves per CU by default, no more workgroups than the LDS holds
        // (the window sweep's ring: one workgroup of 8 waves per CU)
        const int wl = window ? gather_window_lds(dtype, R) : 0;
        const int w = wl ? 16 : gather_waves(dtype, R);
        const int fit = (160 * 1024) / (wl ? wl : gather_lds(dtype, R));
        per_cu = g_tuning.wg_per_cu > 0 ? g_tuning.wg_per_cu : 16 / w;
        if (per_cu > fit) per_cu = fit > 0 ? fit : 1;
    } else {
        per_cu = g_tuning.wg_per_cu > 0 ? g_tuning.wg_per_cu : 8;   // 32 waves per CU
    }
    const int g = device_cus() * per_cu;
    return (g + kXcds - 1) / kXcds * kXcds;
}

hipError_t launch_sweep(int dtype, int R, int variant, const SweepArgs& a_in, hipStream_t s) {
    const kpm_sweep_tuning g_tuning = get_tuning();
    SweepArgs a = a_in;
    a.xcd_ways = g_tuning.xcd_ways > 0 ? g_tuning.xcd_ways : 1;
    a.slab = g_tuning.slab;
    a.tile = g_tuning.gather_tile;
    a.order = g_tuning.tile_order;
    a.stream = g_tuning.stream;
    if (use_gather(dtype, R, a.nrows)) return launch_gather(dtype, R, variant, a, s);
    a.chunk = g_tuning.chunk_tiles > 0 ? g_tuning.chunk_tiles : 1;
    if (!g_tuning.dynamic) a.queue = nullptr;
    a.prefetch = g_tuning.prefetch == 1 ? 1 : 0;   // the touch pass is option 1 only
    if (dtype == KPM_C128) return R >= 32 ? launch_sweep_c128_large(R, variant, a, s)
                                          : launch_sweep_c128_small(R, variant, a, s);
    return R >= 32 ? launch_sweep_c64_large(R, variant, a, s) : launch_sweep_c64_small(R, variant, a, s);
}

hipError_t launch_reduce_partials(const double* partials, int nslots, int grid, int R,
                                  int sweep0, double* eta, hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    reduce_partials_kernel<<<nslots, 256, 0, s>>>(partials, grid, R, sweep0, eta);
    return hipGetLastError();
}

hipError_t launch_zero_ints(int* p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    zero_ints_kernel<<<(n + 255) / 256, 256, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_copy16(void* dst, const void* src, size_t bytes, hipStream_t s) {
    const int64_t n = static_cast<int64_t>(bytes / 16);
    const int tail8 = (bytes % 16) >= 8 ? 1 : 0;
    if (n <= 0 && !tail8) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    const int64_t cap = static_cast<int64_t>(device_cus()) * 16;   // 16 workgroups of 256 per CU
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    copy16_kernel<<<static_cast<int>(blocks), 256, 0, s>>>(static_cast<const int4*>(src), static_cast<int4*>(dst), n,
                                                          tail8);
    return hipGetLastError();
}

hipError_t launch_eta_to_mu(const double* eta, int R, int M, double* mu, hipStream_t s) {
    const int64_t n = static_cast<int64_t>(R) * M;
    eta_to_mu_kernel<<<static_cast<int>((n + 255) / 256), 256, 0, s>>>(eta, R, M, mu);
    return hipGetLastError();
}

hipError_t launch_check_moments(const double* mu, int R, int M, int* flag, hipStream_t s) {
    check_moments_kernel<<<1, 256, 0, s>>>(mu, R, M, flag);
    return hipGetLastError();
}

}  // namespace kpm
