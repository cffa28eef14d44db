// The fused augmented block sweep ("aug_spmmv", Alg. "kpm_improved_blocked")
// and the small kernels around it: deterministic reduction of the per-
// workgroup scalar-product partials, the eta -> mu doubling identity and the
// moment sanity check.
//
// Data layout (row-major, "interleaved" block vectors as the paper requires
// for SpMMV):  a block of R complex vectors is N rows of E = 2R reals
// (re, im of column 0, re, im of column 1, ...).  The matrix is stored as
// N x 13 slots, row-major, (re, im) values plus an int32 column index, with
// the diagonal in slot 0.
//
// Thread mapping (wave64): one lane owns ONE real number of a block row, i.e.
// either the real or the imaginary part of one column.  For R >= 32 a whole
// wave owns a block row, so the row index, and with it every matrix entry,
// is wave-uniform: the compiler fetches (value, column) with scalar loads and
// feeds them to the FMAs as scalar operands, and each gathered V row is one
// contiguous, fully coalesced 64-lane load.  For R < 32 a wave owns 32/R
// rows.  A lane holding the real part accumulates A = sum hr*vr and
// B = sum hi*vr, its partner (lane ^ 1) A' = sum hr*vi and B' = sum hi*vi;
// one DPP swap per row then gives (H v)_re = A - B' and (H v)_im = A' + B.
// The scalar-product accumulators live in registers for the whole sweep
// (the lane -> column map never changes), so cross-lane work happens once
// per workgroup, not once per row.
#include "kpm_internal.h"

namespace kpm {
namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;

// Exchange a value with the neighbouring lane (lane ^ 1) through DPP
// quad_perm [1, 0, 3, 2].
__device__ inline float swap_pair(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
}
__device__ inline double swap_pair(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0xB1, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Same-size unsigned integer type: matrix values are fetched through it so
// that the compiler can prove the in-loop stores to W (floating point) never
// clobber them and selects scalar loads for the wave-uniform entries.
template <typename T> struct Bits;
template <> struct Bits<double> { using type = unsigned long long; };
template <> struct Bits<float> { using type = unsigned int; };

// V rows are gathered with buffer loads: the row offset (column index times
// the row pitch) is a scalar operand and the lane's offset a fixed VGPR, so
// a gather costs no vector ALU work.  Requires the block to span < 4 GiB.
template <typename T>
__device__ inline T buffer_load(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff);
template <>
__device__ inline double buffer_load<double>(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
}
template <>
__device__ inline float buffer_load<float>(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0));
}

// Word 3 of a raw (untyped, stride 0) buffer descriptor on gfx9-family parts.
constexpr int kBufferWord3 = 0x00020000;

template <int R>
struct Geo {
    static constexpr int E = 2 * R;                      // reals per block row
    static constexpr int RPW = (E >= 64) ? 1 : 64 / E;   // block rows per wave
    static constexpr int EPL = (E >= 64) ? E / 64 : 1;   // reals per lane
    static constexpr int TR = kWaves * RPW;              // rows per workgroup tile
};

// W <- alpha H V + beta V + gamma W; FULL also accumulates <V|V>, <W|V>.
template <typename T, int R, int VARIANT, bool BUF>
__global__ void __launch_bounds__(kThreads)
aug_spmmv_kernel(const T* __restrict__ val, const int32_t* __restrict__ col, int64_t nrows,
                 const T* __restrict__ V, T* __restrict__ W, T alpha, T beta, T gamma,
                 double* __restrict__ partials) {
    using G = Geo<R>;
    using U = typename Bits<T>::type;
    const U* __restrict__ vbits = reinterpret_cast<const U*>(val);
    const __amdgpu_buffer_rsrc_t vrs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<T*>(V), 0, BUF ? static_cast<int>(0xFFFFFFFFu) : 0, kBufferWord3);
    constexpr int EPL = G::EPL;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sub = (G::RPW == 1) ? 0 : lane / G::E;
    const int e0 = (G::RPW == 1) ? lane : lane % G::E;
    const bool im_part = (e0 & 1) != 0;
    const T sgn = im_part ? T(1) : T(-1);

    double acc_e[EPL], acc_or[EPL], acc_oi[EPL];
#pragma unroll
    for (int k = 0; k < EPL; ++k) acc_e[k] = acc_or[k] = acc_oi[k] = 0.0;

    // Workgroups are dealt to the XCDs round-robin; give each XCD one
    // contiguous range of row tiles so that neighbouring rows share an L2.
    const int ngrid = gridDim.x;
    const int X = (ngrid % kXcds == 0) ? kXcds : 1;
    const int xcd = blockIdx.x % X;
    const int slot = blockIdx.x / X;
    const int per = ngrid / X;
    const int64_t ntiles = (nrows + G::TR - 1) / G::TR;
    const int64_t t_lo = ntiles * xcd / X;
    int64_t t_hi = ntiles * (xcd + 1) / X;
    if constexpr (G::RPW == 1) {
        // last tile in which this wave still owns a row (a loop bound rather
        // than a break keeps the row index provably wave-uniform)
        const int64_t t_wave = (nrows - wave + G::TR - 1) / G::TR;
        t_hi = t_hi < t_wave ? t_hi : t_wave;
    }

    for (int64_t tile = t_lo + slot; tile < t_hi; tile += per) {
        const int64_t row = tile * G::TR + wave * G::RPW + sub;
        const bool active = (G::RPW == 1) || row < nrows;
        const int64_t rr = active ? row : nrows - 1;
        const int64_t base = rr * kWidth;
        T A[EPL], B[EPL], vs[EPL];
#pragma unroll
        for (int k = 0; k < EPL; ++k) A[k] = B[k] = T(0);
#pragma unroll
        for (int j = 0; j < kWidth; ++j) {
            const int64_t c = col[base + j];
            const T hr = __builtin_bit_cast(T, vbits[2 * (base + j)]);
            const T hi = __builtin_bit_cast(T, vbits[2 * (base + j) + 1]);
            const T* vr = V + c * G::E + e0;
#pragma unroll
            for (int k = 0; k < EPL; ++k) {
                T v;
                if constexpr (BUF)
                    v = buffer_load<T>(vrs, static_cast<unsigned>((e0 + 64 * k) * sizeof(T)),
                                       static_cast<unsigned>(c) * static_cast<unsigned>(G::E * sizeof(T)));
                else
                    v = vr[64 * k];
                if (j == 0) vs[k] = v;
                A[k] = fma(hr, v, A[k]);
                B[k] = fma(hi, v, B[k]);
            }
        }
        T* wr = W + rr * G::E + e0;
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
            const T hv = fma(sgn, swap_pair(B[k]), A[k]);
            if constexpr (VARIANT == KPM_PLAIN) {
                if (active) wr[64 * k] = hv;
            } else {
                T w = fma(alpha, hv, beta * vs[k]);
                if (gamma != T(0)) w = fma(gamma, wr[64 * k], w);
                if (active) wr[64 * k] = w;
                if constexpr (VARIANT == KPM_FULL) {
                    const double v = static_cast<double>(vs[k]);
                    const double vsw = static_cast<double>(swap_pair(vs[k]));
                    const double wd = active ? static_cast<double>(w) : 0.0;
                    acc_e[k] = fma(active ? v : 0.0, v, acc_e[k]);
                    acc_or[k] = fma(wd, v, acc_or[k]);
                    acc_oi[k] = fma(wd, vsw, acc_oi[k]);
                }
            }
        }
    }

    if constexpr (VARIANT == KPM_FULL) {
        // Re-part lane of each (re, im) pair: <v|v> and Re<w|v> are sums over
        // both lanes, Im<w|v> = sum (w_re v_im - w_im v_re) is a difference.
        __shared__ double red[kWaves][3][R];
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
            double e = acc_e[k] + swap_pair(acc_e[k]);
            double o_r = acc_or[k] + swap_pair(acc_or[k]);
            double o_i = acc_oi[k] - swap_pair(acc_oi[k]);
            // lanes e0, e0 + E, e0 + 2E, ... of a wave hold the same column
            for (int off = G::E; off < 64; off <<= 1) {
                e += __shfl_xor(e, off);
                o_r += __shfl_xor(o_r, off);
                o_i += __shfl_xor(o_i, off);
            }
            if (sub == 0 && !im_part) {
                const int r = (e0 >> 1) + 32 * k;
                red[wave][0][r] = e;
                red[wave][1][r] = o_r;
                red[wave][2][r] = o_i;
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < 3 * R; i += kThreads) {
            const int q = i / R, r = i % R;
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) s += red[w][q][r];
            partials[static_cast<int64_t>(blockIdx.x) * 3 * R + i] = s;
        }
    }
}

template <typename T, int R, int VARIANT>
hipError_t launch_one(const SweepArgs& a, hipStream_t s) {
    const uint64_t vbytes = static_cast<uint64_t>(a.nrows) * 2 * R * sizeof(T);
    if (vbytes < (1ull << 32)) {
        aug_spmmv_kernel<T, R, VARIANT, true><<<a.grid, kThreads, 0, s>>>(
            static_cast<const T*>(a.val), a.col, a.nrows, static_cast<const T*>(a.V),
            static_cast<T*>(a.W), static_cast<T>(a.alpha), static_cast<T>(a.beta),
            static_cast<T>(a.gamma), a.partials);
    } else {
        aug_spmmv_kernel<T, R, VARIANT, false><<<a.grid, kThreads, 0, s>>>(
            static_cast<const T*>(a.val), a.col, a.nrows, static_cast<const T*>(a.V),
            static_cast<T*>(a.W), static_cast<T>(a.alpha), static_cast<T>(a.beta),
            static_cast<T>(a.gamma), a.partials);
    }
    return hipGetLastError();
}

template <typename T, int R>
hipError_t launch_variant(int variant, const SweepArgs& a, hipStream_t s) {
    switch (variant) {
    case KPM_FULL: return launch_one<T, R, KPM_FULL>(a, s);
    case KPM_NODOT: return launch_one<T, R, KPM_NODOT>(a, s);
    case KPM_PLAIN: return launch_one<T, R, KPM_PLAIN>(a, s);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_dtype(int R, int variant, const SweepArgs& a, hipStream_t s) {
    switch (R) {
    case 1: return launch_variant<T, 1>(variant, a, s);
    case 2: return launch_variant<T, 2>(variant, a, s);
    case 4: return launch_variant<T, 4>(variant, a, s);
    case 8: return launch_variant<T, 8>(variant, a, s);
    case 16: return launch_variant<T, 16>(variant, a, s);
    case 32: return launch_variant<T, 32>(variant, a, s);
    case 64: return launch_variant<T, 64>(variant, a, s);
    }
    return hipErrorInvalidValue;
}

// eta[sweep] from the partial sums of nslots consecutive sweeps, one
// workgroup per sweep, each output summed over the workgroups in index order.
__global__ void __launch_bounds__(256)
reduce_partials_kernel(const double* __restrict__ part, int grid, int R, int sweep0,
                       double* __restrict__ eta) {
    const int n3 = 3 * R;
    const double* p = part + static_cast<int64_t>(blockIdx.x) * grid * n3;
    const int sweep = sweep0 + blockIdx.x;
    for (int i = threadIdx.x; i < n3; i += blockDim.x) {
        double acc = 0.0;
        for (int g = 0; g < grid; ++g) acc += p[static_cast<int64_t>(g) * n3 + i];
        const int q = i / R, r = i % R;
        if (q == 0) {
            eta[(static_cast<int64_t>(2 * sweep) * R + r) * 2] = acc;
            eta[(static_cast<int64_t>(2 * sweep) * R + r) * 2 + 1] = 0.0;
        } else {
            eta[(static_cast<int64_t>(2 * sweep + 1) * R + r) * 2 + (q - 1)] = acc;
        }
    }
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

int sweep_grid(int dtype, int R) {
    static int cached[2][8] = {};
    const int di = (dtype == KPM_C64) ? 1 : 0;
    int ri = 0;
    while ((1 << ri) < R && ri < 7) ++ri;
    if (cached[di][ri]) return cached[di][ri];
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
    }
    int per_cu = 8;   // 32 waves per CU with 4-wave workgroups
    const char* env = getenv("KPM_SWEEP_WG_PER_CU");
    if (env && atoi(env) > 0) per_cu = atoi(env);
    int g = cus * per_cu;
    g = (g + kXcds - 1) / kXcds * kXcds;
    cached[di][ri] = g;
    return g;
}

hipError_t launch_sweep(int dtype, int R, int variant, const SweepArgs& a, hipStream_t s) {
    if (dtype == KPM_C128) return launch_dtype<double>(R, variant, a, s);
    return launch_dtype<float>(R, variant, a, s);
}

hipError_t launch_reduce_partials(const double* partials, int nslots, int grid, int R,
                                  int sweep0, double* eta, hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    reduce_partials_kernel<<<nslots, 256, 0, s>>>(partials, grid, R, sweep0, eta);
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
