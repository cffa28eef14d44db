// Device construction of the topological-insulator Hamiltonian (eq. "Ham")
// in the library's row-major slot format, fused with the per-row Gershgorin
// discs used for the spectral scaling (section "Problem Description").
//
// Row 4*n + o (site n = x + Lx*(y + Ly*z), orbital o = 2*tau + s) stores 13
// slots, diagonal first, then for each axis j = x, y, z and each neighbour
// n - e_j, n + e_j two slots: the same orbital (Gamma^1 part of the hopping
// block) and the partner orbital (Gamma^{j+1} = tau_x (x) sigma_j part).
//
//   block at (rows of n+e_j, cols of n):   T_j = -t (Gamma^1 - i Gamma^{j+1}) / 2
//   block at (rows of n, cols of n+e_j):   T_j^dagger
//
// Row (n, o) therefore sees T_j[o][.] towards n - e_j and T_j^dagger[o][.]
// towards n + e_j.  With Gamma^1[o][o] = g1 = +-1 and G = Gamma^{j+1}[o][p]:
//   same orbital, either side:   -t g1 / 2
//   partner p, towards n - e_j:  +i t G / 2
//   partner p, towards n + e_j:  -i t G / 2
// A neighbour beyond an open side becomes two padding slots (value 0,
// column = the row itself), which leaves every product unchanged.
#include <cfloat>

#include "kpm_internal.h"

namespace kpm {
namespace {

constexpr int kBuildThreads = 256;

template <typename T>
__device__ inline void put(T* __restrict__ val, int32_t* __restrict__ col, int64_t row, int slot,
                           double re, double im, int64_t c) {
    const int64_t k = row * kWidth + slot;
    val[2 * k] = static_cast<T>(re);
    val[2 * k + 1] = static_cast<T>(im);
    col[k] = static_cast<int32_t>(c);
}

template <typename T>
__global__ void __launch_bounds__(kBuildThreads)
build_ti_kernel(int Lx, int Ly, int Lz, int px, int py, int pz, double t,
                const double* __restrict__ pot, T* __restrict__ val, int32_t* __restrict__ col,
                int64_t nrows, double* __restrict__ block_bounds) {
    __shared__ double s_lo[kBuildThreads];
    __shared__ double s_hi[kBuildThreads];
    const int64_t row = static_cast<int64_t>(blockIdx.x) * kBuildThreads + threadIdx.x;
    double lo = DBL_MAX, hi = -DBL_MAX;
    if (row < nrows) {
        const int64_t n = row >> 2;
        const int o = static_cast<int>(row & 3);
        const int tau = o >> 1, s = o & 1;
        const int L[3] = {Lx, Ly, Lz};
        const int per[3] = {px, py, pz};
        int xyz[3];
        xyz[0] = static_cast<int>(n % Lx);
        xyz[1] = static_cast<int>((n / Lx) % Ly);
        xyz[2] = static_cast<int>(n / (static_cast<int64_t>(Lx) * Ly));
        const double g1 = tau ? -1.0 : 1.0;
        const double diag = pot[n] + 2.0 * g1;
        put(val, col, row, 0, diag, 0.0, row);
        double radius = 0.0;
        int slot = 1;
        for (int j = 0; j < 3; ++j) {
            // partner orbital of tau_x (x) sigma_j and the matrix element G
            const int ps = (j == 2) ? s : 1 - s;
            const int p = 2 * (1 - tau) + ps;
            double gre, gim;
            if (j == 0) { gre = 1.0; gim = 0.0; }                  // sigma_x
            else if (j == 1) { gre = 0.0; gim = s ? 1.0 : -1.0; }  // sigma_y
            else { gre = s ? -1.0 : 1.0; gim = 0.0; }              // sigma_z
            for (int dir = -1; dir <= 1; dir += 2) {
                int c[3] = {xyz[0], xyz[1], xyz[2]};
                int q = c[j] + dir;
                bool ok = true;
                if (q < 0 || q >= L[j]) {
                    if (per[j]) q = (q + L[j]) % L[j];
                    else ok = false;
                }
                if (!ok) {
                    put(val, col, row, slot++, 0.0, 0.0, row);
                    put(val, col, row, slot++, 0.0, 0.0, row);
                    continue;
                }
                c[j] = q;
                const int64_t m = c[0] + static_cast<int64_t>(Lx) * (c[1] + static_cast<int64_t>(Ly) * c[2]);
                const double same = -0.5 * t * g1;
                // (+-i t/2) * (gre + i gim)
                const double sgn = (dir < 0) ? 1.0 : -1.0;
                const double pre = -sgn * 0.5 * t * gim;
                const double pim = sgn * 0.5 * t * gre;
                put(val, col, row, slot++, same, 0.0, 4 * m + o);
                put(val, col, row, slot++, pre, pim, 4 * m + p);
                radius += fabs(same) + sqrt(pre * pre + pim * pim);
            }
        }
        lo = diag - radius;
        hi = diag + radius;
    }
    s_lo[threadIdx.x] = lo;
    s_hi[threadIdx.x] = hi;
    __syncthreads();
    for (int w = kBuildThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s_lo[threadIdx.x] = fmin(s_lo[threadIdx.x], s_lo[threadIdx.x + w]);
            s_hi[threadIdx.x] = fmax(s_hi[threadIdx.x], s_hi[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        block_bounds[2 * blockIdx.x] = s_lo[0];
        block_bounds[2 * blockIdx.x + 1] = s_hi[0];
    }
}

__global__ void __launch_bounds__(kBuildThreads)
bounds_reduce_kernel(const double* __restrict__ block_bounds, int nblocks, double* __restrict__ out) {
    __shared__ double s_lo[kBuildThreads];
    __shared__ double s_hi[kBuildThreads];
    double lo = DBL_MAX, hi = -DBL_MAX;
    for (int i = threadIdx.x; i < nblocks; i += kBuildThreads) {
        lo = fmin(lo, block_bounds[2 * i]);
        hi = fmax(hi, block_bounds[2 * i + 1]);
    }
    s_lo[threadIdx.x] = lo;
    s_hi[threadIdx.x] = hi;
    __syncthreads();
    for (int w = kBuildThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s_lo[threadIdx.x] = fmin(s_lo[threadIdx.x], s_lo[threadIdx.x + w]);
            s_hi[threadIdx.x] = fmax(s_hi[threadIdx.x], s_hi[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s_lo[0];
        out[1] = s_hi[0];
    }
}

// Gershgorin discs of SELL-C-sigma storage, one sorted position per
// thread: centre Re h_ii (every entry in the row's own column), radius the
// sum of |h_ij| over the other columns (padding, column N, is skipped).
// Values are read in the storage precision and summed in FP64.
template <typename T>
__global__ void __launch_bounds__(kBuildThreads)
sell_bounds_kernel(const T* __restrict__ val, const int32_t* __restrict__ col, const int64_t* __restrict__ start,
                   const int32_t* __restrict__ width, const int32_t* __restrict__ perm, int64_t nrows, int clog,
                   double* __restrict__ block_bounds) {
    __shared__ double s_lo[kBuildThreads];
    __shared__ double s_hi[kBuildThreads];
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kBuildThreads + threadIdx.x;
    double lo = DBL_MAX, hi = -DBL_MAX;
    if (p < nrows) {
        const int64_t ch = p >> clog;
        const int64_t C = int64_t{1} << clog;
        const int64_t row = perm ? perm[p] : p;
        const int w = width[ch];
        int64_t e = start[ch] + (p & (C - 1));
        double centre = 0.0, radius = 0.0;
        for (int j = 0; j < w; ++j, e += C) {
            const int64_t c = col[e];
            if (c == row) centre += static_cast<double>(val[2 * e]);
            else if (c < nrows) radius += hypot(static_cast<double>(val[2 * e]), static_cast<double>(val[2 * e + 1]));
        }
        lo = centre - radius;
        hi = centre + radius;
    }
    s_lo[threadIdx.x] = lo;
    s_hi[threadIdx.x] = hi;
    __syncthreads();
    for (int w = kBuildThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s_lo[threadIdx.x] = fmin(s_lo[threadIdx.x], s_lo[threadIdx.x + w]);
            s_hi[threadIdx.x] = fmax(s_hi[threadIdx.x], s_hi[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        block_bounds[2 * blockIdx.x] = s_lo[0];
        block_bounds[2 * blockIdx.x + 1] = s_hi[0];
    }
}

}  // namespace

hipError_t launch_sell_bounds(int dtype, const void* val, const int32_t* col, const int64_t* start,
                              const int32_t* width, const int32_t* perm, int64_t nrows, int clog,
                              double* block_bounds, double* bounds_out, hipStream_t s) {
    const int nblocks = build_blocks(nrows);
    if (dtype == KPM_C128)
        sell_bounds_kernel<double><<<nblocks, kBuildThreads, 0, s>>>(static_cast<const double*>(val), col, start,
                                                                     width, perm, nrows, clog, block_bounds);
    else
        sell_bounds_kernel<float><<<nblocks, kBuildThreads, 0, s>>>(static_cast<const float*>(val), col, start,
                                                                    width, perm, nrows, clog, block_bounds);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    bounds_reduce_kernel<<<1, kBuildThreads, 0, s>>>(block_bounds, nblocks, bounds_out);
    return hipGetLastError();
}

int build_blocks(int64_t nrows) {
    return static_cast<int>((nrows + kBuildThreads - 1) / kBuildThreads);
}

hipError_t launch_build_ti(int Lx, int Ly, int Lz, const int* periodic, double t,
                           const double* pot_dev, int dtype, void* val, int32_t* col,
                           double* block_bounds, int nblocks, double* bounds_out, hipStream_t s) {
    const int64_t nrows = 4LL * Lx * Ly * Lz;
    if (dtype == KPM_C128) {
        build_ti_kernel<double><<<nblocks, kBuildThreads, 0, s>>>(
            Lx, Ly, Lz, periodic[0], periodic[1], periodic[2], t, pot_dev,
            static_cast<double*>(val), col, nrows, block_bounds);
    } else {
        build_ti_kernel<float><<<nblocks, kBuildThreads, 0, s>>>(
            Lx, Ly, Lz, periodic[0], periodic[1], periodic[2], t, pot_dev,
            static_cast<float*>(val), col, nrows, block_bounds);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    bounds_reduce_kernel<<<1, kBuildThreads, 0, s>>>(block_bounds, nblocks, bounds_out);
    return hipGetLastError();
}

}  // namespace kpm
