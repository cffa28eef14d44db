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
// Order: the passes walk the lattice in blocks of `slab` y-lines, each block
// plane by plane (batch::Slabs), so that the V rows gathered for the z
// neighbours of a pass were touched a few lines earlier and are still in L2.
//
// Work distribution: the passes are split into xcd_ways contiguous ranges,
// workgroup g takes range g % xcd_ways (the die the dispatcher deals it to)
// and its waves interleave over the range, so that the rows a die gathers
// are the rows its own L2 holds.  Scalar products: per-lane FP64
// accumulators, summed over the wave and the workgroup in a fixed order into
// one [3][R] partial per workgroup.
#include "kpm_batched.h"

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
template <typename T, int R, int WAVES, int VARIANT, bool SLAB, int AUX>
__global__ void __launch_bounds__(64 * WAVES, (min_waves<T, R, WAVES>()))
gather_sweep_kernel(const T* __restrict__ val, const int32_t* __restrict__ col, int64_t N,
                    const T* __restrict__ V, T* __restrict__ W, T alpha, T beta, T gamma,
                    double* __restrict__ partials, int xcd_ways, SlabGeom geom) {
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

    const int ngrid = gridDim.x;
    const int X = (xcd_ways > 1 && ngrid % xcd_ways == 0) ? xcd_ways : 1;
    const int xcd = blockIdx.x % X;
    const int per = ngrid / X;
    batch::PassOrder<SLAB> sl;
    sl.init(N, geom, RPW, 0, 1);
    const int64_t npass = sl.npass();
    const int64_t lo = npass * xcd / X, hi = npass * (xcd + 1) / X;
    const int64_t stride = static_cast<int64_t>(per) * WAVES;
    const int64_t q0 = lo + static_cast<int64_t>(blockIdx.x / X) * WAVES + wave;
    sl.init(N, geom, RPW, q0, stride);   // this wave's passes q0, q0 + stride, ...

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
    for (int64_t q = q0; q < hi; q += stride) {
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
        // slab order: rows past the end of a pass belong to other passes and
        // get an offset past the block (the old-W load reads zero, the store
        // is dropped); natural order: only rows past N are inactive, and
        // their offsets are past the block
        bool act;
        unsigned off;
        if constexpr (SLAB) {
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

template <typename T, int R, int WAVES, int VARIANT, bool SLAB, int AUX>
void launch_k(const SweepArgs& a, hipStream_t s) {
    const SlabGeom geom = SLAB ? SlabGeom::make(a.L[0], a.L[1], a.L[2], a.slab, Shape<T, R>::RPW) : SlabGeom{};
    gather_sweep_kernel<T, R, WAVES, VARIANT, SLAB, AUX><<<a.grid, 64 * WAVES, 0, s>>>(
        static_cast<const T*>(a.val), a.col, a.nrows, static_cast<const T*>(a.V), static_cast<T*>(a.W),
        static_cast<T>(a.alpha), static_cast<T>(a.beta), static_cast<T>(a.gamma), a.partials, a.xcd_ways, geom);
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
        if constexpr (kStream<R> != 0) {
            if (slab && nt) launch_k<T, R, WAVES, VARIANT, true, kStream<R>>(a, s);
            else if (slab) launch_k<T, R, WAVES, VARIANT, true, 0>(a, s);
            else if (nt) launch_k<T, R, WAVES, VARIANT, false, kStream<R>>(a, s);
            else launch_k<T, R, WAVES, VARIANT, false, 0>(a, s);
        } else if constexpr (R <= 16) {
            if (slab) launch_k<T, R, WAVES, VARIANT, true, 0>(a, s);
            else launch_k<T, R, WAVES, VARIANT, false, 0>(a, s);
        } else {
            launch_k<T, R, WAVES, VARIANT, false, 0>(a, s);
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
