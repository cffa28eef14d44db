// Cache-blocked fused sweep for lattice Hamiltonians at R = 32.
//
// The generic sweep gathers all 13 neighbour rows of every output row from
// global memory; at R = 32 that is 13 x 512 B per row through each CU's
// texture path, whose address/data units then limit the sweep long before
// HBM does.  This kernel exploits what the library knows about its own
// matrix: slot j of row (n, o) couples to a fixed lattice neighbour of site
// n (slot order as written by the builder: diagonal, then for x, y, z the
// neighbours n - e_j and n + e_j, each with the same orbital and with the
// partner orbital o ^ 3 for x and y, o ^ 2 for z).
//
// One workgroup of 16 waves owns a 4 x 4 column of sites and walks it plane
// by plane along z ("pencil").  A ring of four z-planes of V for the 16
// sites lives in LDS, so the diagonal, both z neighbours and every in-tile x
// and y neighbour are read from LDS; only neighbours across the tile edge
// are gathered from memory (and mostly hit L2, since the adjacent tiles of
// a die fetch the same plane at the same time).  While plane s is
// computed, plane s + 2 of V and the old W rows and matrix rows of plane
// s + 1 are already in flight, so a step waits only on its own
// edge-neighbour loads.  Matrix values are read once per sweep; the column
// indices are implied by the slot order and are not read.
//
// Work distribution: tiles are numbered row-major over the tile grid and
// split into 8 contiguous ranges; workgroup g takes range g % 8 (the die the
// dispatcher deals it to) and strides over it, so that the tiles a die
// holds in its L2 are spatial neighbours.
#include "kpm_sweep.h"

namespace kpm {
namespace lattice {
namespace {

using sweep::from_words;
using sweep::scalar_rsrc;
using sweep::sload;
using sweep::swap_pair;

constexpr int kP = 4;            // tile side in sites
constexpr int kNW = kP * kP;     // waves per workgroup: one per tile site
constexpr int kR = 32;           // block width handled here
constexpr int kE = 2 * kR;       // reals per block row = lanes per wave
constexpr int kThreadsL = 64 * kNW;

template <typename T>
__device__ inline T gload(__amdgpu_buffer_rsrc_t rs, int lane, int64_t row) {
    return sweep::buffer_load<T>(rs, static_cast<unsigned>(lane * sizeof(T)),
                                 static_cast<unsigned>(row * kE * static_cast<int64_t>(sizeof(T))));
}

// The matrix rows of one site (4 rows x 13 complex entries) are one
// contiguous record; lane l < 52 of a wave loads entry l % 13 of row l / 13
// (16 bytes in complex128, 8 in complex64) with a single vector load, and
// v_readlane hands each entry to the FMAs as a wave-uniform scalar operand.
// Unlike scalar loads (which complete out of order, so every wait drains all
// of them) these loads can be issued a whole step ahead.
template <typename T> struct SiteRec;
template <> struct SiteRec<double> {
    using V = int4;
    static __device__ V load(const double* site_vals, int lane) {
        return lane < 4 * kWidth ? reinterpret_cast<const int4*>(site_vals)[lane] : int4{0, 0, 0, 0};
    }
    static __device__ double re(const V& v, int l) {
        return __hiloint2double(__builtin_amdgcn_readlane(v.y, l), __builtin_amdgcn_readlane(v.x, l));
    }
    static __device__ double im(const V& v, int l) {
        return __hiloint2double(__builtin_amdgcn_readlane(v.w, l), __builtin_amdgcn_readlane(v.z, l));
    }
};
template <> struct SiteRec<float> {
    using V = int2;
    static __device__ V load(const float* site_vals, int lane) {
        return lane < 4 * kWidth ? reinterpret_cast<const int2*>(site_vals)[lane] : int2{0, 0};
    }
    static __device__ float re(const V& v, int l) { return __int_as_float(__builtin_amdgcn_readlane(v.x, l)); }
    static __device__ float im(const V& v, int l) { return __int_as_float(__builtin_amdgcn_readlane(v.y, l)); }
};

// Neighbour in the x-y plane: absent (open side), in this tile (LDS, local
// wave index) or outside it (global, site index within a plane).
struct Nb {
    int kind;   // 0 absent, 1 LDS, 2 global
    int idx;
};

__device__ inline Nb xy_neighbour(int nx, int ny, int Lx, int Ly, int px, int py, int x0, int y0,
                                  int Lxv, int Lyv) {
    Nb r{0, 0};
    if (nx < 0 || nx >= Lx) {
        if (!px) return r;
        nx = (nx + Lx) % Lx;
    }
    if (ny < 0 || ny >= Ly) {
        if (!py) return r;
        ny = (ny + Ly) % Ly;
    }
    if (nx >= x0 && nx < x0 + Lxv && ny >= y0 && ny < y0 + Lyv) {
        r.kind = 1;
        r.idx = (nx - x0) + kP * (ny - y0);
    } else {
        r.kind = 2;
        r.idx = nx + Lx * ny;
    }
    return r;
}

template <typename T>
__device__ inline T wload(const T* p, bool nt) {
    return nt ? __builtin_nontemporal_load(p) : *p;
}

// VALS: how the matrix rows reach the FMAs as wave-uniform operands.
//   0  scalar buffer loads when the row is processed
//   1  one vector load per site a step ahead, v_readlane per entry
//   2  scalar loads, with the site's rows pulled into L2 by a vector load a
//      step ahead (the scalar loads then wait on L2, not on HBM)

template <typename T, int VARIANT, int VALS, int STREAM>
__global__ void __launch_bounds__(kThreadsL)
lattice_kernel(const T* __restrict__ val, const T* __restrict__ V, T* __restrict__ W,
               T alpha, T beta, T gamma, double* __restrict__ partials,
               int Lx, int Ly, int Lz, int px, int py, int pz, int ntx, int ntiles, int order) {
    __shared__ T ring[4][kNW][4][kE];
    __shared__ double red[kNW][3][kR];

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ti = wave % kP, tj = wave / kP;
    const bool im_part = (lane & 1) != 0;
    const T sgn = im_part ? T(1) : T(-1);
    const bool need_w = VARIANT != KPM_PLAIN && gamma != T(0);
    constexpr int kValWords = 2 * kWidth * static_cast<int>(sizeof(T)) / 4;
    constexpr int wpv = static_cast<int>(sizeof(T)) / 4;
    const v4i32 val_rs = scalar_rsrc(val, 0xFFFFFFFFu);
    const __amdgpu_buffer_rsrc_t vrs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<T*>(V), 0, static_cast<int>(0xFFFFFFFFu), sweep::kBufferWord3);
    const int64_t plane_sites = static_cast<int64_t>(Lx) * Ly;

    double acc_e = 0.0, acc_or = 0.0, acc_oi = 0.0;

    const int ngrid = gridDim.x;
    const int X = (order != 2 && ngrid % kXcds == 0) ? kXcds : 1;
    const int xcd = blockIdx.x % X;
    const int slot = blockIdx.x / X;
    const int per = ngrid / X;
    const int k_lo = static_cast<int>(static_cast<int64_t>(ntiles) * xcd / X);
    const int k_hi = static_cast<int>(static_cast<int64_t>(ntiles) * (xcd + 1) / X);
    const int nty = ntiles / ntx;
    // order 0: each die takes a 2-D block of (ntx/2) x (nty/4) tiles, so that
    // most tiles whose edge rows it gathers are its own; order 1: each die
    // takes a contiguous run of tile rows; order 2: no die mapping
    const bool blocks = order == 0 && X == kXcds && ntx % 2 == 0 && nty % 4 == 0;

    constexpr bool VEC_VALS = VALS == 1;
    unsigned sink = 0;   // keeps the L2 warm-up loads of VALS == 2

    for (int k = k_lo + slot; k < k_hi; k += per) {
        int tx = k % ntx, ty = k / ntx;
        if (blocks) {
            const int bw = ntx / 2, bh = nty / 4, i = k - k_lo;
            tx = (xcd % 2) * bw + i % bw;
            ty = (xcd / 2) * bh + i / bw;
        }
        const int x0 = tx * kP, y0 = ty * kP;
        const int Lxv = min(kP, Lx - x0), Lyv = min(kP, Ly - y0);   // valid extent of the tile (>= 2)
        const int x = x0 + ti, y = y0 + tj;
        const bool active = ti < Lxv && tj < Lyv;                     // wave-uniform
        const int64_t sxy = static_cast<int64_t>(x) + static_cast<int64_t>(Lx) * y;
        Nb nb[4];
        nb[0] = xy_neighbour(x - 1, y, Lx, Ly, px, py, x0, y0, Lxv, Lyv);
        nb[1] = xy_neighbour(x + 1, y, Lx, Ly, px, py, x0, y0, Lxv, Lyv);
        nb[2] = xy_neighbour(x, y - 1, Lx, Ly, px, py, x0, y0, Lxv, Lyv);
        nb[3] = xy_neighbour(x, y + 1, Lx, Ly, px, py, x0, y0, Lxv, Lyv);
        // A tile is at least 2 sites wide in x and y, so a site has at most
        // one neighbour across the tile edge in x and one in y: halo slot 0
        // holds the x one (direction hx), slot 1 the y one (direction hy).
        const int hx = nb[0].kind == 2 ? 0 : (nb[1].kind == 2 ? 1 : -1);
        const int hy = nb[2].kind == 2 ? 2 : (nb[3].kind == 2 ? 3 : -1);

        // plane index of step s' (with periodic wrap); -1 when it does not exist
        auto plane_of = [&](int sp) -> int {
            if (sp >= 0 && sp < Lz) return sp;
            return pz ? (sp + Lz) % Lz : -1;
        };
        // the four rows of each halo neighbour of this site in plane zp
        auto load_halo = [&](int zp, T (&h)[2][4]) {
            if (hx >= 0) {
                const int64_t nbase = 4 * (static_cast<int64_t>(nb[hx].idx) + plane_sites * zp);
#pragma unroll
                for (int o = 0; o < 4; ++o) h[0][o] = gload<T>(vrs, lane, nbase + o);
            }
            if (hy >= 0) {
                const int64_t nbase = 4 * (static_cast<int64_t>(nb[hy].idx) + plane_sites * zp);
#pragma unroll
                for (int o = 0; o < 4; ++o) h[1][o] = gload<T>(vrs, lane, nbase + o);
            }
        };

        // prologue: planes -1, 0, 1 into ring slots 3, 0, 1; halo, old W and
        // matrix rows of step 0
        T h_c[2][4], w_c[4];
        typename SiteRec<T>::V hv_c{};
        if (active) {
            for (int sp = -1; sp <= 1; ++sp) {
                const int zp = plane_of(sp);
                if (zp < 0) continue;
                const int64_t base = 4 * (sxy + plane_sites * zp);
#pragma unroll
                for (int o = 0; o < 4; ++o) ring[sp & 3][wave][o][lane] = gload<T>(vrs, lane, base + o);
            }
            load_halo(0, h_c);
            const int64_t base = 4 * sxy;
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                if constexpr (STREAM & 1) w_c[o] = need_w ? __builtin_nontemporal_load(W + (base + o) * kE + lane) : T(0);
                else w_c[o] = need_w ? W[(base + o) * kE + lane] : T(0);
            }
            if constexpr (VEC_VALS) hv_c = SiteRec<T>::load(val + base * 2 * kWidth, lane);
        }
        __syncthreads();

        for (int s = 0; s < Lz; ++s) {
            // Loads for later steps only: the halo and old W rows of step
            // s + 1, plane s + 2 and (VALS 1, 2) the matrix rows of step s + 1.
            // Nothing this step computes waits on them.
            const int zn2 = plane_of(s + 2);
            const int zn1 = (s + 1 < Lz) ? s + 1 : -1;
            T h_n[2][4], p_n[4], w_n[4];
            typename SiteRec<T>::V hv_n{};
            if (active) {
                if (zn1 >= 0) load_halo(zn1, h_n);
                if (zn2 >= 0) {
                    const int64_t base = 4 * (sxy + plane_sites * zn2);
#pragma unroll
                    for (int o = 0; o < 4; ++o) p_n[o] = gload<T>(vrs, lane, base + o);
                }
                if (zn1 >= 0) {
                    const int64_t base = 4 * (sxy + plane_sites * zn1);
#pragma unroll
                    for (int o = 0; o < 4; ++o) {
                        if constexpr (STREAM & 1) w_n[o] = need_w ? __builtin_nontemporal_load(W + (base + o) * kE + lane) : T(0);
                        else w_n[o] = need_w ? W[(base + o) * kE + lane] : T(0);
                    }
                    if constexpr (VALS != 0) hv_n = SiteRec<T>::load(val + base * 2 * kWidth, lane);
                }
            }
            const bool zdn = plane_of(s - 1) >= 0, zup = plane_of(s + 1) >= 0;
            if (active) {
                const int64_t site = sxy + plane_sites * s;
#pragma unroll
                for (int o = 0; o < 4; ++o) {
                    const int64_t row = 4 * site + o;
                    int wv[VEC_VALS ? 1 : kValWords];
                    if constexpr (!VEC_VALS) sload<kValWords>(val_rs, static_cast<unsigned>(row * kValWords * 4), wv);
                    T v[kWidth];
                    v[0] = ring[s & 3][wave][o][lane];
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        const int sl = 1 + 2 * d;
                        if (nb[d].kind == 1) {
                            v[sl] = ring[s & 3][nb[d].idx][o][lane];
                            v[sl + 1] = ring[s & 3][nb[d].idx][o ^ 3][lane];
                        } else if (nb[d].kind == 2) {
                            const int hs = d < 2 ? 0 : 1;
                            v[sl] = h_c[hs][o];
                            v[sl + 1] = h_c[hs][o ^ 3];
                        } else {
                            v[sl] = v[sl + 1] = T(0);
                        }
                    }
                    v[9] = zdn ? ring[(s - 1) & 3][wave][o][lane] : T(0);
                    v[10] = zdn ? ring[(s - 1) & 3][wave][o ^ 2][lane] : T(0);
                    v[11] = zup ? ring[(s + 1) & 3][wave][o][lane] : T(0);
                    v[12] = zup ? ring[(s + 1) & 3][wave][o ^ 2][lane] : T(0);
                    // two partial sums per product: shorter FMA dependency chains
                    T A[2] = {T(0), T(0)}, B[2] = {T(0), T(0)};
                    if constexpr (VEC_VALS) {
#pragma unroll
                        for (int j = 0; j < kWidth; ++j) {
                            A[j & 1] = fma(SiteRec<T>::re(hv_c, kWidth * o + j), v[j], A[j & 1]);
                            B[j & 1] = fma(SiteRec<T>::im(hv_c, kWidth * o + j), v[j], B[j & 1]);
                        }
                    } else {
#pragma unroll
                        for (int j = 0; j < kWidth; ++j) {
                            A[j & 1] = fma(from_words<T>(wv + (2 * j) * wpv), v[j], A[j & 1]);
                            B[j & 1] = fma(from_words<T>(wv + (2 * j + 1) * wpv), v[j], B[j & 1]);
                        }
                    }
                    const T hv = fma(sgn, swap_pair(B[0] + B[1]), A[0] + A[1]);
                    T* wr = W + row * kE + lane;
                    if constexpr (VARIANT == KPM_PLAIN) {
                        if constexpr (STREAM & 2) __builtin_nontemporal_store(hv, wr);
                        else *wr = hv;
                    } else {
                        T w = fma(alpha, hv, beta * v[0]);
                        if (need_w) w = fma(gamma, w_c[o], w);
                        if constexpr (STREAM & 2) __builtin_nontemporal_store(w, wr);
                        else *wr = w;
                        if constexpr (VARIANT == KPM_FULL) {
                            const double vd = static_cast<double>(v[0]);
                            const double vsw = static_cast<double>(swap_pair(v[0]));
                            const double wd = static_cast<double>(w);
                            acc_e = fma(vd, vd, acc_e);
                            acc_or = fma(wd, vd, acc_or);
                            acc_oi = fma(wd, vsw, acc_oi);
                        }
                    }
                }
            }
            // plane s + 2 replaces plane s - 2 (last read in step s - 1)
            if (active && zn2 >= 0) {
#pragma unroll
                for (int o = 0; o < 4; ++o) ring[(s + 2) & 3][wave][o][lane] = p_n[o];
            }
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                w_c[o] = w_n[o];
                h_c[0][o] = h_n[0][o];
                h_c[1][o] = h_n[1][o];
            }
            if constexpr (VALS == 2) {
                sink ^= static_cast<unsigned>(__builtin_amdgcn_readfirstlane(hv_n.x));
            } else {
                hv_c = hv_n;
            }
            __syncthreads();
        }
    }
    asm volatile("" ::"s"(sink));

    if constexpr (VARIANT == KPM_FULL) {
        const double e = acc_e + swap_pair(acc_e);
        const double o_r = acc_or + swap_pair(acc_or);
        const double o_i = acc_oi - swap_pair(acc_oi);
        if (!im_part) {
            red[wave][0][lane >> 1] = e;
            red[wave][1][lane >> 1] = o_r;
            red[wave][2][lane >> 1] = o_i;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < 3 * kR; i += kThreadsL) {
            const int q = i / kR, r = i % kR;
            double sum = 0.0;
            for (int w = 0; w < kNW; ++w) sum += red[w][q][r];
            partials[static_cast<int64_t>(blockIdx.x) * 3 * kR + i] = sum;
        }
    }
}

template <typename T, int STREAM>
hipError_t launch_ts(int variant, const LatticeArgs& a, hipStream_t s) {
    const int ntx = (a.L[0] + kP - 1) / kP, nty = (a.L[1] + kP - 1) / kP;
    const int ntiles = ntx * nty;
#define KPM_LAUNCH(VAR, VALS)                                                                    \
    lattice_kernel<T, VAR, VALS, STREAM><<<a.grid, kThreadsL, 0, s>>>(                           \
        static_cast<const T*>(a.val), static_cast<const T*>(a.V), static_cast<T*>(a.W),          \
        static_cast<T>(a.alpha), static_cast<T>(a.beta), static_cast<T>(a.gamma), a.partials,  \
        a.L[0], a.L[1], a.L[2], a.periodic[0], a.periodic[1], a.periodic[2], ntx, ntiles, a.order)
#define KPM_LAUNCH_V(VAR)                          \
    switch (a.prefetch) {                          \
    case 1: KPM_LAUNCH(VAR, 1); break;             \
    case 2: KPM_LAUNCH(VAR, 2); break;             \
    default: KPM_LAUNCH(VAR, 0); break;            \
    }
    switch (variant) {
    case KPM_FULL: KPM_LAUNCH_V(KPM_FULL); break;
    case KPM_NODOT: KPM_LAUNCH_V(KPM_NODOT); break;
    case KPM_PLAIN: KPM_LAUNCH_V(KPM_PLAIN); break;
    default: return hipErrorInvalidValue;
    }
#undef KPM_LAUNCH_V
#undef KPM_LAUNCH
    return hipGetLastError();
}

template <typename T>
hipError_t launch_t(int variant, const LatticeArgs& a, hipStream_t s) {
    switch (a.stream) {
    case 1: return launch_ts<T, 1>(variant, a, s);
    case 2: return launch_ts<T, 2>(variant, a, s);
    case 3: return launch_ts<T, 3>(variant, a, s);
    default: return launch_ts<T, 0>(variant, a, s);
    }
}

}  // namespace
}  // namespace lattice

int lattice_tiles(const kpm_hamiltonian* H) {
    return ((H->L[0] + lattice::kP - 1) / lattice::kP) * ((H->L[1] + lattice::kP - 1) / lattice::kP);
}

bool lattice_supported(const kpm_hamiltonian* H, int R) {
    if (R != lattice::kR) return false;
    // every tile must be at least 2 sites wide in x and y (at most one
    // neighbour across each tile edge): no side with L mod 4 == 1
    if (H->L[0] % lattice::kP == 1 || H->L[1] % lattice::kP == 1) return false;
    const uint64_t vbytes = static_cast<uint64_t>(H->nrows) * 2 * R *
                            (H->dtype == KPM_C128 ? sizeof(double) : sizeof(float));
    return vbytes < (1ull << 32) && H->L[0] > 0;
}

int lattice_grid(const kpm_hamiltonian* H) {
    const int ntiles = lattice_tiles(H);
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
    }
    const int per_cu = (H->dtype == KPM_C128) ? 1 : 2;   // LDS: 140 KB or 76 KB per workgroup
    int g = cus * per_cu;
    if (g > ntiles) g = ntiles;
    if (g >= kXcds) g -= g % kXcds;
    return g > 0 ? g : 1;
}

hipError_t launch_lattice(int dtype, int variant, const LatticeArgs& a, hipStream_t s) {
    if (dtype == KPM_C128) return lattice::launch_t<double>(variant, a, s);
    return lattice::launch_t<float>(variant, a, s);
}

}  // namespace kpm
