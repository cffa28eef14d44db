#pragma once
// Staged-gather fused sweep: one aug_spmmv over a whole matrix by the whole
// grid (Alg. "kpm_improved_blocked", the fused body), for any block width.
//
// It shares the per-wave pass structure of the batched solver: a lane owns
// CPL consecutive complex elements of a block row (16 bytes where the block
// is wide enough), a wave covers 64 CPL / R block rows per pass, the matrix
// rows of its next pass (values and column indices, contiguous) are copied
// into the wave's LDS slot with coalesced loads while the current pass
// computes, and the 13 neighbour rows of V are gathered with 16-byte loads.
// Compared with the scalar-operand sweep (one block row per wave), this
// needs far fewer vector-memory instructions per block row when R < 32,
// which is what limits a gather-heavy sweep on gfx950.
//
// Order (ORDER): 0 natural row order; 1 slab order, the lattice in blocks
// of `slab` y-lines, each block plane by plane (batch::Slabs), so that the
// V rows gathered for the z neighbours of a pass were touched a few lines
// earlier; 2 pencil order (batch::TileWalk), one workgroup per run of
// z-planes of a tile of sites, its waves sharing each plane of the tile, so
// that the rows a pass gathers were fetched at most a plane of the tile
// earlier or by the workgroup of the adjacent tile on the same die.  Every
// order visits every row exactly once; only where a row's neighbours are in
// the cache depends on it, so any matrix in this format, whatever its
// columns, gives the same result in every order.
//
// Work distribution (orders 0 and 1): the passes are split into xcd_ways
// contiguous ranges, workgroup g takes range g % xcd_ways (the die the
// dispatcher deals it to) and its waves interleave over the range, so that
// the rows a die gathers are the rows its own L2 holds.  Scalar products:
// per-lane FP64 accumulators, summed over the wave and the workgroup in a
// fixed order into one [3][R] partial per workgroup.
#include "kpm_batched.h"

#include <type_traits>

namespace kpm {
namespace gather {

using batch::kStream;
using batch::Lanes;
using batch::Pair;
using batch::rsrc;
using batch::Shape;
using batch::wave_sync;
using batch::Words;

template <typename T, int R, int WAVES>
constexpr int lds_bytes() {
    using S = Shape<T, R>;
    return WAVES * (S::kAhead ? 2 : 1) * S::kStageWords * 4 + WAVES * 3 * R * 8;
}

template <typename T, int R, int WAVES>
constexpr bool instantiable() {
    return lds_bytes<T, R, WAVES>() <= batch::kLdsMax && WAVES <= batch::kMaxWaves<T>;
}

template <typename T, int R, int WAVES>
constexpr int min_waves() {
    const int wg_per_cu = batch::kLdsMax / lds_bytes<T, R, WAVES>();
    const int occ = wg_per_cu * WAVES / 4;
    return occ < 1 ? 1 : (occ < batch::kMinWaves<T> ? occ : batch::kMinWaves<T>);
}

// W <- alpha H V + beta V + gamma W (FULL, NODOT) or W <- H V (PLAIN);
// FULL also writes this workgroup's <V|V>, <W|V> partial.
template <typename T, int R, int WAVES, int VARIANT, int ORDER, int AUX>
__global__ void __launch_bounds__(64 * WAVES, (min_waves<T, R, WAVES>()))
gather_sweep_kernel(const T* __restrict__ val, const int32_t* __restrict__ col, int64_t N,
                    const T* __restrict__ V, T* __restrict__ W, T alpha, T beta, T gamma,
                    double* __restrict__ partials, int xcd_ways, SlabGeom geom, TileGeom tgeom) {
    using S = Shape<T, R>;
    constexpr int CPL = S::CPL;
    using LV = Lanes<T, CPL>;
    using Cv = typename LV::type;
    using P2 = typename Pair<T>::type;
    using WV = Words<S::kVecV>;
    using WC = Words<S::kVecC>;
    constexpr int LPR = S::LPR;
    constexpr int RPW = S::RPW;
    constexpr int kVW = S::kValWords;
    constexpr int kBufs = S::kAhead ? 2 : 1;
    constexpr int kWpv = static_cast<int>(sizeof(T)) / 4;
    constexpr unsigned kCB = 2 * sizeof(T);
    __shared__ __attribute__((aligned(16))) int stage[WAVES][kBufs][S::kStageWords];
    __shared__ double red[WAVES][3][R];

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sub = lane / LPR;
    const int cc = lane % LPR;

    constexpr bool SLAB = ORDER == 1;
    const int ngrid = gridDim.x;
    const int X = (xcd_ways > 1 && ngrid % xcd_ways == 0) ? xcd_ways : 1;
    const int xcd = blockIdx.x % X;
    const int per = ngrid / X;
    std::conditional_t<ORDER == 2, batch::TileWalk, batch::PassOrder<SLAB>> sl;
    int64_t hi = 0, stride = 0, q0 = 0;
    if constexpr (ORDER == 2) {
        sl.init(tgeom, blockIdx.x, ngrid, kXcds, wave, WAVES);
    } else {
        sl.init(N, geom, RPW, 0, 1);
        const int64_t npass = sl.npass();
        const int64_t lo = npass * xcd / X;
        hi = npass * (xcd + 1) / X;
        stride = static_cast<int64_t>(per) * WAVES;
        q0 = lo + static_cast<int64_t>(blockIdx.x / X) * WAVES + wave;
        sl.init(N, geom, RPW, q0, stride);   // this wave's passes q0, q0 + stride, ...
    }

    const uint64_t vbytes = static_cast<uint64_t>(N) * R * kCB;
    const __amdgpu_buffer_rsrc_t val_rs = rsrc(val, static_cast<uint64_t>(N) * kVW * 4);
    const __amdgpu_buffer_rsrc_t col_rs = rsrc(col, static_cast<uint64_t>(N) * kWidth * 4);
    const __amdgpu_buffer_rsrc_t vrs = rsrc(V, vbytes);
    const __amdgpu_buffer_rsrc_t wrs = rsrc(W, vbytes);
    // old W only where it enters the result; a resource of size zero reads zeros
    const bool need_w = VARIANT != KPM_PLAIN && gamma != T(0);
    const __amdgpu_buffer_rsrc_t wold_rs = rsrc(W, need_w ? vbytes : 0);

    // matrix rows of the pass starting at row r0 (values, then column
    // indices); lanes past the end of a part fetch words that are never read
    auto fetch = [&](int64_t r0, typename WV::type* wv, typename WC::type* wc) {
        const unsigned pv = static_cast<unsigned>(r0) * (kVW * 4);
        const unsigned pc = static_cast<unsigned>(r0) * (kWidth * 4);
#pragma unroll
        for (int i = 0; i < S::kLoadsV; ++i) wv[i] = WV::template load<AUX>(val_rs, pv + (lane + 64 * i) * (4 * S::kVecV));
#pragma unroll
        for (int i = 0; i < S::kLoadsC; ++i) wc[i] = WC::template load<AUX>(col_rs, pc + (lane + 64 * i) * (4 * S::kVecC));
    };
    auto put = [&](int* dst, const typename WV::type* wv, const typename WC::type* wc) {
#pragma unroll
        for (int i = 0; i < S::kLoadsV; ++i)
            *reinterpret_cast<typename WV::type*>(dst + (lane + 64 * i) * S::kVecV) = wv[i];
#pragma unroll
        for (int i = 0; i < S::kLoadsC; ++i)
            *reinterpret_cast<typename WC::type*>(dst + S::kColOff + (lane + 64 * i) * S::kVecC) = wc[i];
    };

    double ae[CPL], aor[CPL], aoi[CPL];
#pragma unroll
    for (int t = 0; t < CPL; ++t) ae[t] = aor[t] = aoi[t] = 0.0;
    typename WV::type wv[S::kLoadsV];
    typename WC::type wc[S::kLoadsC];
    int buf = 0;
    int64_t row0, nr;
    sl.cur(row0, nr);
    if constexpr (S::kAhead) {
        fetch(row0, wv, wc);
        put(stage[wave][0], wv, wc);
    }
    // orders 0 and 1 end at the die's last pass, the pencil walk reports its
    // end as a pass of no rows
    for (int64_t q = q0; ORDER == 2 ? nr > 0 : q < hi; q += stride) {
        if constexpr (!S::kAhead) {
            wave_sync();
            fetch(row0, wv, wc);
            put(stage[wave][0], wv, wc);
        }
        wave_sync();
        const int* st = stage[wave][buf];
        Cv v[kWidth];
#pragma unroll
        for (int j = 0; j < kWidth; ++j) {
            const unsigned c = static_cast<unsigned>(st[S::kColOff + sub * kWidth + j]);
            v[j] = LV::load(vrs, (c * R + cc * CPL) * kCB);
        }
        const int64_t row = row0 + sub;
        // slab and pencil order: rows past the end of a pass belong to other
        // passes and get an offset past the block (the old-W load reads
        // zero, the store is dropped; pencil passes are always whole);
        // natural order: only rows past N are inactive, and their offsets
        // are past the block
        bool act;
        unsigned off;
        if constexpr (ORDER != 0) {
            act = sub < nr;
            off = act ? static_cast<unsigned>(row * R + cc * CPL) * kCB : 0xFFFFFFF0u;
        } else {
            act = row < N;
            off = static_cast<unsigned>(row * R + cc * CPL) * kCB;
        }
        const Cv wo = LV::template load<AUX>(wold_rs, off);
        int64_t row0n, nrn;
        sl.advance();
        sl.cur(row0n, nrn);
        if constexpr (S::kAhead) fetch(row0n, wv, wc);
        const int* sv = st + sub * kVW;
        Cv acc;
#pragma unroll
        for (int e = 0; e < 2 * CPL; ++e) acc[e] = T(0);
#pragma unroll
        for (int j = 0; j < kWidth; ++j) {
            const P2 h = *reinterpret_cast<const P2*>(sv + 2 * j * kWpv);
#pragma unroll
            for (int t = 0; t < CPL; ++t) {
                acc[2 * t] = fma(h.x, v[j][2 * t], acc[2 * t]);
                acc[2 * t] = fma(-h.y, v[j][2 * t + 1], acc[2 * t]);
                acc[2 * t + 1] = fma(h.x, v[j][2 * t + 1], acc[2 * t + 1]);
                acc[2 * t + 1] = fma(h.y, v[j][2 * t], acc[2 * t + 1]);
            }
        }
        Cv wn;
        if constexpr (VARIANT == KPM_PLAIN) {
            wn = acc;
        } else {
#pragma unroll
            for (int e = 0; e < 2 * CPL; ++e) wn[e] = fma(gamma, wo[e], fma(alpha, acc[e], beta * v[0][e]));
        }
        // rows past N: the store is dropped (offset beyond the block), products masked
        LV::template store<AUX>(wn, wrs, off);
        if constexpr (VARIANT == KPM_FULL) {
#pragma unroll
            for (int t = 0; t < CPL; ++t) {
                const double vr = act ? static_cast<double>(v[0][2 * t]) : 0.0;
                const double vi = act ? static_cast<double>(v[0][2 * t + 1]) : 0.0;
                const double wr = wn[2 * t], wi = wn[2 * t + 1];
                ae[t] = fma(vr, vr, fma(vi, vi, ae[t]));
                aor[t] = fma(wr, vr, fma(wi, vi, aor[t]));
                aoi[t] = fma(wr, vi, fma(-wi, vr, aoi[t]));
            }
        }
        if constexpr (S::kAhead) {
            put(stage[wave][buf ^ 1], wv, wc);
            buf ^= 1;
        }
        row0 = row0n;
        nr = nrn;
    }
    if constexpr (VARIANT == KPM_FULL) {
#pragma unroll
        for (int t = 0; t < CPL; ++t) {
#pragma unroll
            for (int o = LPR; o < 64; o <<= 1) {
                ae[t] += __shfl_xor(ae[t], o);
                aor[t] += __shfl_xor(aor[t], o);
                aoi[t] += __shfl_xor(aoi[t], o);
            }
            if (sub == 0) {
                red[wave][0][cc * CPL + t] = ae[t];
                red[wave][1][cc * CPL + t] = aor[t];
                red[wave][2][cc * CPL + t] = aoi[t];
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < 3 * R; i += 64 * WAVES) {
            const int qq = i / R, r = i % R;
            double sum = 0.0;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) sum += red[w][qq][r];
            partials[static_cast<int64_t>(blockIdx.x) * 3 * R + i] = sum;
        }
    }
}

template <typename T, int R, int WAVES, int VARIANT, int ORDER, int AUX>
void launch_k(const SweepArgs& a, const TileGeom& tg, hipStream_t s) {
    const SlabGeom geom = ORDER == 1 ? SlabGeom::make(a.L[0], a.L[1], a.L[2], a.slab, Shape<T, R>::RPW) : SlabGeom{};
    gather_sweep_kernel<T, R, WAVES, VARIANT, ORDER, AUX><<<a.grid, 64 * WAVES, 0, s>>>(
        static_cast<const T*>(a.val), a.col, a.nrows, static_cast<const T*>(a.V), static_cast<T*>(a.W),
        static_cast<T>(a.alpha), static_cast<T>(a.beta), static_cast<T>(a.gamma), a.partials, a.xcd_ways, geom,
        tg);
}

// Pencil order for this launch: a lattice, tile side > 0, and passes of at
// most one site (rpw <= 4: R >= 16 in complex128, R >= 32 in complex64).
template <typename T, int R>
bool pencil_order(const SweepArgs& a, TileGeom& tg) {
    constexpr int rpw = Shape<T, R>::RPW;
    if (rpw > 4 || a.tile <= 0 || a.L[0] <= 0 || a.grid <= 0) return false;
    if (static_cast<int64_t>(a.L[0]) * a.L[1] * a.L[2] * 4 != a.nrows) return false;
    tg = TileGeom::make(a.L[0], a.L[1], a.L[2], a.tile, rpw, a.grid, kXcds);
    return true;
}

// ---- Window sweep: the staged-gather sweep in pencil order with a ring of
// z-planes of V in LDS ----
//
// In pencil order a tile's rows gather most of their neighbours from the
// tile's own planes z - 1, z, z + 1.  This variant keeps those planes of V
// in LDS (a ring of three: plane z + 2 is fetched with coalesced loads
// while plane z is computed, and stored where plane z - 1 was once every
// wave is done with it) and reads only the other neighbours from memory, so
// the per-CU gather path moves about 2 instead of 13 rows of V per row.
// It still reads the matrix's column indices and nothing else about its
// structure: when a wave stages the matrix rows of a pass in LDS, each
// column index is decoded once into its site (x, y, z) and replaced by
// either a ring row (the column's site lies in the tile and within one
// plane of the pass) or itself (any other column, gathered from memory).
// Any matrix over the lattice's rows (any couplings, any range) gives the
// result of the staged-gather sweep; only how many neighbours come from the
// ring depends on it.

// Tile side: the ring of three tile planes must fit in LDS beside the
// matrix staging.
template <typename T, int R>
constexpr int win_side() {
    return R * 2 * static_cast<int>(sizeof(T)) <= 512 ? 4 : 2;
}

// One workgroup of 16 waves per CU (its LDS): measured against 8 waves with
// a ring of four planes (one barrier per plane) and 12 waves, 16 hide the
// latency of a pass best.
template <typename T, int R>
struct Win {
    using S = Shape<T, R>;
    static constexpr int kWaves = 16;
    static constexpr int kRing = 3;                              // tile planes in the ring
    static constexpr int kThreads = 64 * kWaves;
    static constexpr unsigned kCB = 2 * sizeof(T);
    static constexpr unsigned kRB = R * kCB;                   // bytes per block row
    static constexpr int kSide = win_side<T, R>();
    static constexpr int kTileRows = 4 * kSide * kSide;
    static constexpr unsigned kPlaneBytes = kTileRows * kRB;
    static constexpr int kLoadsP = (kPlaneBytes / 16 + kThreads - 1) / kThreads;   // 16-byte loads per thread
    static constexpr unsigned kRingBytes = kRing * kPlaneBytes;   // then one zero row
    // two staging slots per wave (the pass being computed, the next one)
    static constexpr int kStageBytes = kWaves * 2 * S::kStageWords * 4;
    static constexpr int kLds = static_cast<int>(kRingBytes + kRB) + kStageBytes;
    static constexpr bool ok = S::RPW <= 4 && S::kAhead && kLds <= batch::kLdsMax &&
                               3 * R * 8 * kWaves <= static_cast<int>(kRingBytes);
};

// Geometry of a window sweep: the pencil order (tiles of Win::kSide) and
// the divisions that turn a site index into (x, y, z).
struct WinGeom {
    TileGeom t;
    FastDiv by_lx, by_sxy;   // Lx, Lx Ly
};

template <typename T, int R, int VARIANT, int AUX>
__global__ void __launch_bounds__((Win<T, R>::kThreads), 1)
window_sweep_kernel(const T* __restrict__ val, const int32_t* __restrict__ col, int64_t N,
                    const T* __restrict__ V, T* __restrict__ W, T alpha, T beta, T gamma,
                    double* __restrict__ partials, WinGeom wg) {
    using C = Win<T, R>;
    using S = Shape<T, R>;
    constexpr int WAVES = C::kWaves;
    constexpr int CPL = S::CPL;
    using LV = Lanes<T, CPL>;
    using Cv = typename LV::type;
    using P2 = typename Pair<T>::type;
    using WV = Words<S::kVecV>;
    using WC = Words<S::kVecC>;
    using I4 = Words<4>;
    constexpr int LPR = S::LPR;
    constexpr int RPW = S::RPW;
    constexpr int kVW = S::kValWords;
    constexpr int kWpv = static_cast<int>(sizeof(T)) / 4;
    constexpr unsigned kCB = C::kCB;
    constexpr unsigned RB = C::kRB;
    constexpr unsigned kOut = 0xFFFFFFF0u;   // offset past every buffer: loads read 0, stores are dropped
    constexpr uint32_t NR = C::kRing;
    __shared__ __attribute__((aligned(16))) char ring[C::kRingBytes + RB];
    __shared__ __attribute__((aligned(16))) int stage[WAVES][2][S::kStageWords];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int sub = lane / LPR;
    const int cc = lane % LPR;
    const unsigned lp = cc * CPL * kCB;   // this lane's bytes within a block row

    TileGeom tg = wg.t;
    const uint32_t ngrid = gridDim.x;
    const uint32_t X = tg.dies > 1 && ngrid % tg.dies == 0 ? tg.dies : 1;
    if (X != kXcds) tg.bw = tg.bh = 0;
    const uint32_t die = blockIdx.x % X, per = ngrid / X;
    const uint32_t nitems = tg.nitems();
    const uint32_t k_lo = static_cast<uint32_t>(static_cast<uint64_t>(nitems) * die / X);
    const uint32_t k_hi = static_cast<uint32_t>(static_cast<uint64_t>(nitems) * (die + 1) / X);
    const uint32_t Lx = tg.Lx, Lz = tg.Lz, sxy = tg.Lx * tg.Ly;
    const uint32_t line_rows = tg.line_rows, plane_rows = tg.plane_rows;

    const uint64_t vbytes = static_cast<uint64_t>(N) * RB;
    const __amdgpu_buffer_rsrc_t val_rs = rsrc(val, static_cast<uint64_t>(N) * kVW * 4);
    const __amdgpu_buffer_rsrc_t col_rs = rsrc(col, static_cast<uint64_t>(N) * kWidth * 4);
    const __amdgpu_buffer_rsrc_t vrs = rsrc(V, vbytes);
    const __amdgpu_buffer_rsrc_t wrs = rsrc(W, vbytes);
    const bool need_w = VARIANT != KPM_PLAIN && gamma != T(0);
    const __amdgpu_buffer_rsrc_t wold_rs = rsrc(W, need_w ? vbytes : 0);

    for (unsigned u = tid * 16; u < RB; u += C::kThreads * 16)
        *reinterpret_cast<int4*>(ring + C::kRingBytes + u) = int4{0, 0, 0, 0};

    auto fetch = [&](uint32_t r0, typename WV::type* wv, typename WC::type* wc) {
        const unsigned pv = r0 * (kVW * 4);
        const unsigned pc = r0 * (kWidth * 4);
#pragma unroll
        for (int i = 0; i < S::kLoadsV; ++i) wv[i] = WV::template load<AUX>(val_rs, pv + (lane + 64 * i) * (4 * S::kVecV));
#pragma unroll
        for (int i = 0; i < S::kLoadsC; ++i) wc[i] = WC::template load<AUX>(col_rs, pc + (lane + 64 * i) * (4 * S::kVecC));
    };

    double ae[CPL], aor[CPL], aoi[CPL];
#pragma unroll
    for (int t = 0; t < CPL; ++t) ae[t] = aor[t] = aoi[t] = 0.0;
    for (uint32_t k = k_lo + blockIdx.x / X; k < k_hi; k += per) {
        uint32_t x0, y0, ex, ey, z0, z1;
        batch::tile_item(tg, k, k_lo, die, x0, y0, ex, ey, z0, z1);
        const uint32_t ppl = 4 * ex / RPW;                 // passes per line of the tile
        const uint32_t base = y0 * line_rows + 4 * x0;     // first row of the tile in a plane
        // column -> ring row (flag bit 31) for a pass in plane zp, whose plane
        // zp - 1 sits in ring slot sm, or the column itself
        auto code = [&](uint32_t c, uint32_t zp, uint32_t sm) -> uint32_t {
            const uint32_t n = c >> 2;
            const uint32_t zc = wg.by_sxy.div(n);
            const uint32_t r = n - zc * sxy;
            const uint32_t yc = wg.by_lx.div(r);
            const uint32_t lx = r - yc * Lx - x0, ly = yc - y0, dz = zc - zp + 1;
            const bool in = lx < ex && ly < ey && dz < 3;
            uint32_t slot = sm + dz;
            slot -= slot >= NR ? NR : 0u;
            const uint32_t local = slot * C::kTileRows + (ly * ex + lx) * 4 + (c & 3u);
            return in ? (0x80000000u | local) : c;
        };
        // ring slot of plane p
        auto slot_of = [&](uint32_t p) { return p % NR; };
        auto put = [&](int* dst, const typename WV::type* wv, const typename WC::type* wc, uint32_t zp) {
            const uint32_t sm = slot_of(zp + NR - 1);
#pragma unroll
            for (int i = 0; i < S::kLoadsV; ++i)
                *reinterpret_cast<typename WV::type*>(dst + (lane + 64 * i) * S::kVecV) = wv[i];
#pragma unroll
            for (int i = 0; i < S::kLoadsC; ++i) {
                typename WC::type w = wc[i];
                if constexpr (S::kVecC == 1) {
                    w = static_cast<int>(code(static_cast<uint32_t>(w), zp, sm));
                } else {
#pragma unroll
                    for (int e = 0; e < S::kVecC; ++e) w[e] = static_cast<int>(code(static_cast<uint32_t>(w[e]), zp, sm));
                }
                *reinterpret_cast<typename WC::type*>(dst + S::kColOff + (lane + 64 * i) * S::kVecC) = w;
            }
        };
        // this thread's share of a tile plane: 16-byte units u = tid + kThreads i,
        // line by line (4 ex rows per line, contiguous in memory and in the ring)
        const uint32_t lunits = 4 * ex * RB / 16, units = ey * lunits;
        unsigned grel[C::kLoadsP];
#pragma unroll
        for (int i = 0; i < C::kLoadsP; ++i) {
            const uint32_t u = tid + C::kThreads * i;
            const uint32_t ln = u / lunits;
            grel[i] = u < units ? ln * line_rows * RB + (u - ln * lunits) * 16 : kOut;
        }
        auto pload = [&](uint32_t zp, typename I4::type (&r)[C::kLoadsP]) {
            const unsigned pb = (zp * plane_rows + base) * RB;
#pragma unroll
            for (int i = 0; i < C::kLoadsP; ++i) r[i] = I4::load(vrs, grel[i] == kOut ? kOut : pb + grel[i]);
        };
        auto pstore = [&](uint32_t zp, const typename I4::type (&r)[C::kLoadsP]) {
            char* dst = ring + slot_of(zp) * C::kPlaneBytes;
#pragma unroll
            for (int i = 0; i < C::kLoadsP; ++i) {
                const uint32_t u = tid + C::kThreads * i;
                if (u < units) *reinterpret_cast<typename I4::type*>(dst + u * 16) = r[i];
            }
        };

        // planes z0 - 1, z0, z0 + 1 into the ring (after every wave is done
        // with the previous item's ring)
        __syncthreads();
        for (uint32_t p = z0 > 0 ? z0 - 1 : z0; p <= z0 + 1 && p < Lz; ++p) {
            typename I4::type r[C::kLoadsP];
            pload(p, r);
            pstore(p, r);
        }
        __syncthreads();

        // this wave's passes in a plane: (line, o) = (l0, o0), then steps of
        // WAVES passes as digits (dl, dout); the matrix rows of the next pass
        // are requested before a pass is computed and staged after it
        const uint32_t l0 = wave / ppl, o0 = wave - l0 * ppl;
        const uint32_t dl = WAVES / ppl, dout = WAVES - dl * ppl;
        auto prow = [&](uint32_t zp, uint32_t ln, uint32_t o) { return zp * plane_rows + base + ln * line_rows + o * RPW; };
        typename WV::type wv[S::kLoadsV];
        typename WC::type wc[S::kLoadsC];
        int buf = 0;
        if (l0 < ey) {
            fetch(prow(z0, l0, o0), wv, wc);
            put(stage[wave][0], wv, wc, z0);
        }
        for (uint32_t z = z0; z < z1; ++z) {
            const bool pre = z + 2 < Lz && z + 2 <= z1;   // plane z + 2, needed by step z + 1
            typename I4::type nx[C::kLoadsP];
            if (pre) pload(z + 2, nx);
            for (uint32_t ln = l0, o = o0; ln < ey;) {
                wave_sync();
                const int* st = stage[wave][buf];
                // neighbours outside the ring from memory (the others read 0
                // there and are taken from the ring when the products are
                // formed); slot 0, the diagonal, is the row itself, always in
                // the ring; only slots some row of the pass takes from memory
                // cost a load
                Cv g[kWidth];
#pragma unroll
                for (int j = 1; j < kWidth; ++j) {
                    const uint32_t cd = static_cast<uint32_t>(st[S::kColOff + sub * kWidth + j]);
                    const bool out = (cd >> 31) == 0;
                    if (__builtin_amdgcn_ballot_w64(out) != 0) g[j] = LV::load(vrs, out ? cd * RB + lp : kOut);
                    else g[j] = Cv{};
                }
                const unsigned off = (prow(z, ln, o) + sub) * RB + lp;
                const Cv wo = LV::template load<AUX>(wold_rs, off);
                // next pass of this wave: same plane, else the next plane of the item
                uint32_t nln = ln + dl, no = o + dout, nzp = z;
                if (no >= ppl) {
                    no -= ppl;
                    ++nln;
                }
                const bool next_plane = nln >= ey;
                if (next_plane) {
                    nln = l0;
                    no = o0;
                    nzp = z + 1;
                }
                // past the item: reads of a row beyond the matrix return zeros
                fetch(nzp < z1 ? prow(nzp, nln, no) : static_cast<uint32_t>(N), wv, wc);
                const int* sv = st + sub * kVW;
                Cv acc, v0;
#pragma unroll
                for (int e = 0; e < 2 * CPL; ++e) acc[e] = T(0);
#pragma unroll
                for (int j = 0; j < kWidth; ++j) {
                    const uint32_t cd = static_cast<uint32_t>(st[S::kColOff + sub * kWidth + j]);
                    const bool in = (cd >> 31) != 0;
                    // exactly one of the two reads is the neighbour, the other reads zeros
                    const Cv l = *reinterpret_cast<const Cv*>(ring + (in ? (cd & 0x7FFFFFFFu) * RB : C::kRingBytes) + lp);
                    const Cv v = j == 0 ? l : l + g[j];
                    if (j == 0) v0 = v;
                    const P2 h = *reinterpret_cast<const P2*>(sv + 2 * j * kWpv);
#pragma unroll
                    for (int t = 0; t < CPL; ++t) {
                        acc[2 * t] = fma(h.x, v[2 * t], acc[2 * t]);
                        acc[2 * t] = fma(-h.y, v[2 * t + 1], acc[2 * t]);
                        acc[2 * t + 1] = fma(h.x, v[2 * t + 1], acc[2 * t + 1]);
                        acc[2 * t + 1] = fma(h.y, v[2 * t], acc[2 * t + 1]);
                    }
                }
                Cv wn;
                if constexpr (VARIANT == KPM_PLAIN) {
                    wn = acc;
                } else {
#pragma unroll
                    for (int e = 0; e < 2 * CPL; ++e) wn[e] = fma(gamma, wo[e], fma(alpha, acc[e], beta * v0[e]));
                }
                if constexpr (VARIANT == KPM_FULL) {
#pragma unroll
                    for (int t = 0; t < CPL; ++t) {
                        const double vr = v0[2 * t], vi = v0[2 * t + 1];
                        const double wr = wn[2 * t], wi = wn[2 * t + 1];
                        ae[t] = fma(vr, vr, fma(vi, vi, ae[t]));
                        aor[t] = fma(wr, vr, fma(wi, vi, aor[t]));
                        aoi[t] = fma(wr, vi, fma(-wi, vr, aoi[t]));
                    }
                }
                LV::template store<AUX>(wn, wrs, off);
                put(stage[wave][buf ^ 1], wv, wc, nzp);
                buf ^= 1;
                if (next_plane) break;
                ln = nln;
                o = no;
            }
            __syncthreads();   // plane z - 1's slot is free
            if (pre) pstore(z + 2, nx);
            __syncthreads();
        }
    }
    if constexpr (VARIANT == KPM_FULL) {
        __syncthreads();   // the ring is free: it holds the per-wave sums
        double (*red)[3][R] = reinterpret_cast<double (*)[3][R]>(ring);
#pragma unroll
        for (int t = 0; t < CPL; ++t) {
#pragma unroll
            for (int o = LPR; o < 64; o <<= 1) {
                ae[t] += __shfl_xor(ae[t], o);
                aor[t] += __shfl_xor(aor[t], o);
                aoi[t] += __shfl_xor(aoi[t], o);
            }
            if (sub == 0) {
                red[wave][0][cc * CPL + t] = ae[t];
                red[wave][1][cc * CPL + t] = aor[t];
                red[wave][2][cc * CPL + t] = aoi[t];
            }
        }
        __syncthreads();
        for (int i = tid; i < 3 * R; i += C::kThreads) {
            const int qq = i / R, r = i % R;
            double sum = 0.0;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) sum += red[w][qq][r];
            partials[static_cast<int64_t>(blockIdx.x) * 3 * R + i] = sum;
        }
    }
}

// The window sweep for this launch: requested, a shape it exists for, and
// a lattice.
template <typename T, int R>
bool window_geom(const SweepArgs& a, WinGeom& g) {
    if constexpr (!Win<T, R>::ok) {
        return false;
    } else {
        if (!a.window || a.L[0] <= 0 || a.grid <= 0) return false;
        if (static_cast<int64_t>(a.L[0]) * a.L[1] * a.L[2] * 4 != a.nrows) return false;
        // tiles dealt to the dies (in 2-D blocks where possible) unless the
        // tuning's tile order asks for no die mapping
        g.t = TileGeom::make(a.L[0], a.L[1], a.L[2], Win<T, R>::kSide, Shape<T, R>::RPW, a.grid,
                             a.order == 2 ? 1 : kXcds);
        g.by_lx.init(static_cast<uint32_t>(a.L[0]));
        g.by_sxy.init(static_cast<uint32_t>(a.L[0]) * static_cast<uint32_t>(a.L[1]));
        return true;
    }
}

template <typename T, int R, int VARIANT, int AUX>
void launch_window(const SweepArgs& a, const WinGeom& g, hipStream_t s) {
    if constexpr (Win<T, R>::ok) {
        window_sweep_kernel<T, R, VARIANT, AUX><<<a.grid, Win<T, R>::kThreads, 0, s>>>(
            static_cast<const T*>(a.val), a.col, a.nrows, static_cast<const T*>(a.V), static_cast<T*>(a.W),
            static_cast<T>(a.alpha), static_cast<T>(a.beta), static_cast<T>(a.gamma), a.partials, g);
    }
}

// Bytes a sweep streams; above the 256 MB Infinity Cache nothing it reads
// survives to the next sweep anyway.
constexpr uint64_t kCacheBytes = 256ull << 20;

template <typename T, int R, int WAVES, int VARIANT>
hipError_t launch_v(const SweepArgs& a, hipStream_t s) {
    if constexpr (instantiable<T, R, WAVES>()) {
        // the slab order only where it changes the order (a lattice, slab <
        // Ly) and pays: up to R = 16 (beyond, its index arithmetic costs
        // more occupancy than the shorter z reuse distance saves)
        const bool slab = R <= 16 && a.slab > 0 && a.L[0] > 0 && a.slab < a.L[1];
        // non-temporal matrix and W streams (batch::kStream) only when a
        // sweep's data exceeds the last-level cache: on smaller problems
        // they would throw away what the next sweep reads again
        const uint64_t bytes = static_cast<uint64_t>(a.nrows) *
                               (kWidth * (2 * sizeof(T) + 4) + 3ull * R * 2 * sizeof(T));
        const bool nt = bytes > kCacheBytes;
        WinGeom wgm;
        if (window_geom<T, R>(a, wgm)) {
            // streams through L2 with the default policy: the non-temporal
            // hint measured no faster here (0-3 % slower at R = 16 and 32)
            launch_window<T, R, VARIANT, 0>(a, wgm, s);
            return hipGetLastError();
        }
        TileGeom tg;
        if constexpr (Shape<T, R>::RPW <= 4) {
            if (pencil_order<T, R>(a, tg)) {
                // the matrix and W streams may bypass L2 (tuning `stream`),
                // which then keeps the V planes the adjacent tiles gather
                if (nt && a.stream != 0) launch_k<T, R, WAVES, VARIANT, 2, 2>(a, tg, s);
                else launch_k<T, R, WAVES, VARIANT, 2, 0>(a, tg, s);
                return hipGetLastError();
            }
        }
        if constexpr (kStream<R> != 0) {
            if (slab && nt) launch_k<T, R, WAVES, VARIANT, 1, kStream<R>>(a, tg, s);
            else if (slab) launch_k<T, R, WAVES, VARIANT, 1, 0>(a, tg, s);
            else if (nt) launch_k<T, R, WAVES, VARIANT, 0, kStream<R>>(a, tg, s);
            else launch_k<T, R, WAVES, VARIANT, 0, 0>(a, tg, s);
        } else if constexpr (R <= 16) {
            if (slab) launch_k<T, R, WAVES, VARIANT, 1, 0>(a, tg, s);
            else launch_k<T, R, WAVES, VARIANT, 0, 0>(a, tg, s);
        } else {
            launch_k<T, R, WAVES, VARIANT, 0, 0>(a, tg, s);
        }
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

template <typename T, int R, int WAVES>
hipError_t launch_variant(int variant, const SweepArgs& a, hipStream_t s) {
    switch (variant) {
    case KPM_FULL: return launch_v<T, R, WAVES, KPM_FULL>(a, s);
    case KPM_NODOT: return launch_v<T, R, WAVES, KPM_NODOT>(a, s);
    case KPM_PLAIN: return launch_v<T, R, WAVES, KPM_PLAIN>(a, s);
    }
    return hipErrorInvalidValue;
}

// Waves per workgroup of the staged-gather sweep: 8, or 4 where the LDS
// slot of a wave is large (small R).
template <typename T, int R>
constexpr int kWavesFor = instantiable<T, R, 8>() && lds_bytes<T, R, 8>() <= 80 * 1024 ? 8 : 4;

template <typename T>
hipError_t launch_dtype(int R, int variant, const SweepArgs& a, hipStream_t s) {
    switch (R) {
    case 1: return launch_variant<T, 1, kWavesFor<T, 1>>(variant, a, s);
    case 2: return launch_variant<T, 2, kWavesFor<T, 2>>(variant, a, s);
    case 4: return launch_variant<T, 4, kWavesFor<T, 4>>(variant, a, s);
    case 8: return launch_variant<T, 8, kWavesFor<T, 8>>(variant, a, s);
    case 16: return launch_variant<T, 16, kWavesFor<T, 16>>(variant, a, s);
    case 32: return launch_variant<T, 32, kWavesFor<T, 32>>(variant, a, s);
    case 64: return launch_variant<T, 64, kWavesFor<T, 64>>(variant, a, s);
    }
    return hipErrorInvalidValue;
}

template <typename T>
int waves_for(int R) {
    switch (R) {
    case 1: return kWavesFor<T, 1>;
    case 2: return kWavesFor<T, 2>;
    case 4: return kWavesFor<T, 4>;
    case 8: return kWavesFor<T, 8>;
    case 16: return kWavesFor<T, 16>;
    case 32: return kWavesFor<T, 32>;
    case 64: return kWavesFor<T, 64>;
    }
    return 4;
}

// LDS of the window sweep at block width R (0: no window sweep there).
template <typename T, int R>
constexpr int kWinLds = Win<T, R>::ok ? Win<T, R>::kLds : 0;

template <typename T, int R>
constexpr int kWinSide = Win<T, R>::ok ? Win<T, R>::kSide : 0;

template <typename T>
int window_side_for(int R) {
    switch (R) {
    case 16: return kWinSide<T, 16>;
    case 32: return kWinSide<T, 32>;
    case 64: return kWinSide<T, 64>;
    }
    return 0;
}

template <typename T>
int window_lds_for(int R) {
    switch (R) {
    case 16: return kWinLds<T, 16>;
    case 32: return kWinLds<T, 32>;
    case 64: return kWinLds<T, 64>;
    }
    return 0;
}

template <typename T>
int lds_for(int R) {
    switch (R) {
    case 1: return lds_bytes<T, 1, kWavesFor<T, 1>>();
    case 2: return lds_bytes<T, 2, kWavesFor<T, 2>>();
    case 4: return lds_bytes<T, 4, kWavesFor<T, 4>>();
    case 8: return lds_bytes<T, 8, kWavesFor<T, 8>>();
    case 16: return lds_bytes<T, 16, kWavesFor<T, 16>>();
    case 32: return lds_bytes<T, 32, kWavesFor<T, 32>>();
    case 64: return lds_bytes<T, 64, kWavesFor<T, 64>>();
    }
    return batch::kLdsMax;
}

}  // namespace gather
}  // namespace kpm
