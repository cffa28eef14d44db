#pragma once
// The fused augmented block sweep ("aug_spmmv", Alg. "kpm_improved_blocked"):
// kernel template and its launch dispatch, included by one translation unit
// per storage precision and range of block widths.
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

// LLVM's scalar buffer-load intrinsics (s_buffer_load_dword{,x2,x4,x8,x16}).
typedef int v2i32 __attribute__((ext_vector_type(2)));
typedef int v4i32 __attribute__((ext_vector_type(4)));
typedef int v8i32 __attribute__((ext_vector_type(8)));
typedef int v16i32 __attribute__((ext_vector_type(16)));
__device__ int sbuf_load1(v4i32 rsrc, int off, int cp) __asm("llvm.amdgcn.s.buffer.load.i32");
__device__ v2i32 sbuf_load2(v4i32 rsrc, int off, int cp) __asm("llvm.amdgcn.s.buffer.load.v2i32");
__device__ v4i32 sbuf_load4(v4i32 rsrc, int off, int cp) __asm("llvm.amdgcn.s.buffer.load.v4i32");
__device__ v8i32 sbuf_load8(v4i32 rsrc, int off, int cp) __asm("llvm.amdgcn.s.buffer.load.v8i32");
__device__ v16i32 sbuf_load16(v4i32 rsrc, int off, int cp) __asm("llvm.amdgcn.s.buffer.load.v16i32");

namespace kpm {
namespace sweep {


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

// Hardware id (0..7) of the accelerator die (XCD) the calling wave runs on.
__device__ inline int xcc_id() {
    unsigned x;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(x));
    return static_cast<int>(x & (kXcds - 1));
}

// Explicit scalar (SMEM) buffer loads.  For R >= 32 the row a wave works
// on is wave-uniform, and its column indices and values are fetched with
// s_buffer_load into SGPRs, which feed the FMAs directly as scalar operands.

// Raw buffer descriptor (4 x 32 bits) over `bytes` bytes starting at p.
__device__ inline v4i32 scalar_rsrc(const void* p, unsigned bytes) {
    const unsigned long long a = reinterpret_cast<unsigned long long>(p);
    v4i32 r;
    r.x = __builtin_amdgcn_readfirstlane(static_cast<int>(a & 0xFFFFFFFFull));
    r.y = __builtin_amdgcn_readfirstlane(static_cast<int>((a >> 32) & 0xFFFFull));
    r.z = static_cast<int>(bytes);
    r.w = kBufferWord3;
    return r;
}

// N consecutive dwords at byte offset `off` into out[0..N).
template <int N>
__device__ inline void sload(v4i32 rs, unsigned off, int* out) {
    int i = 0;
#pragma unroll
    for (; i + 16 <= N; i += 16) {
        const v16i32 v = sbuf_load16(rs, static_cast<int>(off + 4 * i), 0);
#pragma unroll
        for (int k = 0; k < 16; ++k) out[i + k] = v[k];
    }
    if constexpr (N % 16 >= 8) {
        const v8i32 v = sbuf_load8(rs, static_cast<int>(off + 4 * i), 0);
#pragma unroll
        for (int k = 0; k < 8; ++k) out[i + k] = v[k];
        i += 8;
    }
    if constexpr (N % 8 >= 4) {
        const v4i32 v = sbuf_load4(rs, static_cast<int>(off + 4 * i), 0);
#pragma unroll
        for (int k = 0; k < 4; ++k) out[i + k] = v[k];
        i += 4;
    }
    if constexpr (N % 4 >= 2) {
        const v2i32 v = sbuf_load2(rs, static_cast<int>(off + 4 * i), 0);
        out[i] = v.x;
        out[i + 1] = v.y;
        i += 2;
    }
    if constexpr (N % 2 == 1) out[i] = sbuf_load1(rs, static_cast<int>(off + 4 * i), 0);
}

template <typename T> __device__ inline T from_words(const int* w);
template <> __device__ inline double from_words<double>(const int* w) {
    return __hiloint2double(w[1], w[0]);
}
template <> __device__ inline float from_words<float>(const int* w) { return __int_as_float(w[0]); }

// One wave's share of the fused sweep over the row tiles [first, last):
// for each tile the wave owns one block row (RPW == 1) or RPW block rows.
// The column indices and the old W row of the next tile are fetched while
// the current row's gathers are in flight, so that the gathers of a row
// can be issued as soon as the row starts.
template <typename T, int R, int VARIANT, bool BUF, int STREAM>
struct SweepWave {
    using G = Geo<R>;
    static constexpr int EPL = G::EPL;
    static constexpr int kValWords = 2 * kWidth * static_cast<int>(sizeof(T)) / 4;

    const T* __restrict__ val;
    const int32_t* __restrict__ col;
    const int32_t* __restrict__ sched;
    const T* __restrict__ V;
    T* __restrict__ W;
    __amdgpu_buffer_rsrc_t vrs;
    v4i32 val_rs, col_rs, sched_rs;
    int64_t nrows;
    T alpha, beta, gamma, sgn;
    int wave, sub, e0;
    double acc_e[EPL], acc_or[EPL], acc_oi[EPL];

    // position in the processing order -> matrix row (4 rows per site)
    __device__ int64_t row_of(int64_t tile, bool& active) const {
        const int64_t pos = tile * G::TR + wave * G::RPW + sub;
        active = (G::RPW == 1) || pos < nrows;
        const int64_t pp = active ? pos : nrows - 1;
        if (!sched) return pp;
        int site;
        if constexpr (G::RPW == 1)
            site = sbuf_load1(sched_rs, static_cast<int>(4 * (pp >> 2)), 0);
        else
            site = sched[pp >> 2];
        return 4 * static_cast<int64_t>(site) + (pp & 3);
    }

    // W is read once and written once per sweep; with `stream` set those
    // accesses carry the non-temporal hint so that they do not push the
    // reused V rows out of L2.
    __device__ T load_w(const T* p) const {
        if constexpr (STREAM & 1) return __builtin_nontemporal_load(p);
        else return *p;
    }
    __device__ void store_w(T* p, T x) const {
        if constexpr (STREAM & 2) __builtin_nontemporal_store(x, p);
        else *p = x;
    }

    __device__ void load_cols(int64_t r, int* c) const {
        if constexpr (G::RPW == 1) {
            sload<kWidth>(col_rs, static_cast<unsigned>(r * kWidth * 4), c);
        } else {
#pragma unroll
            for (int j = 0; j < kWidth; ++j) c[j] = col[r * kWidth + j];
        }
    }

    __device__ void load_vals(int64_t r, T* hr, T* hi) const {
        if constexpr (G::RPW == 1) {
            int w[kValWords];
            sload<kValWords>(val_rs, static_cast<unsigned>(r * kValWords * 4), w);
            constexpr int wpv = static_cast<int>(sizeof(T)) / 4;
#pragma unroll
            for (int j = 0; j < kWidth; ++j) {
                hr[j] = from_words<T>(w + (2 * j) * wpv);
                hi[j] = from_words<T>(w + (2 * j + 1) * wpv);
            }
        } else {
#pragma unroll
            for (int j = 0; j < kWidth; ++j) {
                hr[j] = val[2 * (r * kWidth + j)];
                hi[j] = val[2 * (r * kWidth + j) + 1];
            }
        }
    }

    // Touch every 64-byte line of the matrix rows and old W rows this wave
    // streams in tiles [first, last) with one word load per line, so that
    // the per-row loads hit L2 instead of waiting on HBM.  The words are
    // folded into the return value, which the caller keeps alive.
    __device__ unsigned prefetch(int64_t first, int64_t last, bool with_w) const {
        constexpr int kLine = 64;
        constexpr int kValBytes = 2 * kWidth * static_cast<int>(sizeof(T));
        constexpr int kValLines = (kValBytes + kLine - 1) / kLine + 1;
        constexpr int kColLines = (kWidth * 4 + kLine - 1) / kLine + 1;
        constexpr int kWBytes = G::E * static_cast<int>(sizeof(T));
        constexpr int kWLines = (kWBytes + kLine - 1) / kLine;
        constexpr int kPerRow = kValLines + kColLines + kWLines;
        const int lane = threadIdx.x & 63;
        const int nrow = static_cast<int>(last - first) * G::RPW;
        unsigned sink = 0;
        for (int f = lane; f < nrow * kPerRow; f += 64) {
            const int i = f / kPerRow, q = f % kPerRow;
            const int64_t pos = (first + i / G::RPW) * G::TR + wave * G::RPW + (i % G::RPW);
            const int64_t pp = pos < nrows ? pos : nrows - 1;
            const int64_t r = sched ? 4 * static_cast<int64_t>(sched[pp >> 2]) + (pp & 3) : pp;
            const unsigned* p;
            if (q < kValLines) {
                const int off = min(q * kLine, kValBytes - 4);
                p = reinterpret_cast<const unsigned*>(reinterpret_cast<const char*>(val + 2 * r * kWidth) + off);
            } else if (q < kValLines + kColLines) {
                const int off = min((q - kValLines) * kLine, kWidth * 4 - 4);
                p = reinterpret_cast<const unsigned*>(reinterpret_cast<const char*>(col + r * kWidth) + off);
            } else {
                if (!with_w) continue;
                const int off = (q - kValLines - kColLines) * kLine;
                p = reinterpret_cast<const unsigned*>(reinterpret_cast<const char*>(W + r * G::E) + off);
            }
            sink ^= __builtin_nontemporal_load(p);
        }
        return sink;
    }

    __device__ void run(int64_t first, int64_t last) {
        if (first >= last) return;
        const bool need_w = VARIANT != KPM_PLAIN && gamma != T(0);
        bool act_c;
        int64_t r_c = row_of(first, act_c);
        int c[kWidth];
        load_cols(r_c, c);
        T w_c[EPL];
#pragma unroll
        for (int k = 0; k < EPL; ++k) w_c[k] = need_w ? load_w(W + r_c * G::E + e0 + 64 * k) : T(0);

        for (int64_t tile = first; tile < last; ++tile) {
            // gathers of the current row
            T v[kWidth][EPL];
#pragma unroll
            for (int j = 0; j < kWidth; ++j) {
#pragma unroll
                for (int k = 0; k < EPL; ++k) {
                    if constexpr (BUF)
                        v[j][k] = buffer_load<T>(vrs, static_cast<unsigned>((e0 + 64 * k) * sizeof(T)),
                                                 static_cast<unsigned>(c[j]) * static_cast<unsigned>(G::E * sizeof(T)));
                    else
                        v[j][k] = V[static_cast<int64_t>(c[j]) * G::E + e0 + 64 * k];
                }
            }
            // matrix values of the current row
            T hr[kWidth], hi[kWidth];
            load_vals(r_c, hr, hi);
            // next row (the last row re-fetches itself): indices and old W
            const int64_t tn = (tile + 1 < last) ? tile + 1 : tile;
            bool act_n;
            const int64_t r_n = row_of(tn, act_n);
            load_cols(r_n, c);
            T w_n[EPL];
#pragma unroll
            for (int k = 0; k < EPL; ++k) w_n[k] = need_w ? load_w(W + r_n * G::E + e0 + 64 * k) : T(0);

            T A[EPL], B[EPL];
#pragma unroll
            for (int k = 0; k < EPL; ++k) A[k] = B[k] = T(0);
#pragma unroll
            for (int j = 0; j < kWidth; ++j) {
#pragma unroll
                for (int k = 0; k < EPL; ++k) {
                    A[k] = fma(hr[j], v[j][k], A[k]);
                    B[k] = fma(hi[j], v[j][k], B[k]);
                }
            }
            T* wr = W + r_c * G::E + e0;
#pragma unroll
            for (int k = 0; k < EPL; ++k) {
                const T hv = fma(sgn, swap_pair(B[k]), A[k]);
                if constexpr (VARIANT == KPM_PLAIN) {
                    if (act_c) store_w(wr + 64 * k, hv);
                } else {
                    const T vs = v[0][k];   // slot 0 is the diagonal: V of this row
                    T w = fma(alpha, hv, beta * vs);
                    if (need_w) w = fma(gamma, w_c[k], w);
                    if (act_c) store_w(wr + 64 * k, w);
                    if constexpr (VARIANT == KPM_FULL) {
                        const double vd = static_cast<double>(vs);
                        const double vsw = static_cast<double>(swap_pair(vs));
                        const double wd = act_c ? static_cast<double>(w) : 0.0;
                        acc_e[k] = fma(act_c ? vd : 0.0, vd, acc_e[k]);
                        acc_or[k] = fma(wd, vd, acc_or[k]);
                        acc_oi[k] = fma(wd, vsw, acc_oi[k]);
                    }
                }
            }
            r_c = r_n;
            act_c = act_n;
#pragma unroll
            for (int k = 0; k < EPL; ++k) w_c[k] = w_n[k];
        }
    }
};

// W <- alpha H V + beta V + gamma W; FULL also accumulates <V|V>, <W|V>.
//
// Work distribution.  The row tiles (TR rows each) are split into kXcds
// contiguous ranges, one per die, so that the rows a die gathers are the
// rows its own L2 holds.  With `queue` set, a workgroup reads the id of the
// die it runs on and takes `chunk` tiles at a time from that range's
// counter (queue[x], zero before the sweep); when its range is exhausted it
// helps the other ranges in turn, so every tile is processed exactly once
// whatever the placement of workgroups on dies.  Without `queue` the
// mapping is static: workgroup g takes range g % xcd_ways and strides over
// it in steps of `chunk` tiles.
template <typename T, int R, int VARIANT, bool BUF, int STREAM>
__global__ void __launch_bounds__(kThreads)
aug_spmmv_kernel(const T* __restrict__ val, const int32_t* __restrict__ col, int64_t nrows,
                 const T* __restrict__ V, T* __restrict__ W, T alpha, T beta, T gamma,
                 double* __restrict__ partials, int xcd_ways, int chunk,
                 const int32_t* __restrict__ sched, int* __restrict__ queue, int prefetch) {
    using G = Geo<R>;
    constexpr int EPL = G::EPL;
    const int lane = threadIdx.x & 63;
    SweepWave<T, R, VARIANT, BUF, STREAM> sw;
    sw.val = val;
    sw.col = col;
    sw.val_rs = scalar_rsrc(val, 0xFFFFFFFFu);
    sw.col_rs = scalar_rsrc(col, 0xFFFFFFFFu);
    sw.sched_rs = scalar_rsrc(sched, 0xFFFFFFFFu);
    sw.sched = sched;
    sw.V = V;
    sw.W = W;
    sw.vrs = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(V), 0,
                                               BUF ? static_cast<int>(0xFFFFFFFFu) : 0, kBufferWord3);
    sw.nrows = nrows;
    sw.alpha = alpha;
    sw.beta = beta;
    sw.gamma = gamma;
    sw.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    sw.sub = (G::RPW == 1) ? 0 : lane / G::E;
    sw.e0 = (G::RPW == 1) ? lane : lane % G::E;
    const bool im_part = (sw.e0 & 1) != 0;
    sw.sgn = im_part ? T(1) : T(-1);
#pragma unroll
    for (int k = 0; k < EPL; ++k) sw.acc_e[k] = sw.acc_or[k] = sw.acc_oi[k] = 0.0;
    const int sub = sw.sub, e0 = sw.e0, wave = sw.wave;

    unsigned sink = 0;
    const int64_t ntiles = (nrows + G::TR - 1) / G::TR;
    // last tile in which this wave still owns a row (RPW == 1): a loop
    // bound rather than a break keeps the row index provably wave-uniform
    const int64_t t_wave = (G::RPW == 1) ? (nrows - wave + G::TR - 1) / G::TR : ntiles;

    if (queue) {
        __shared__ int s_grab;
        const int home = xcc_id();
        for (int k = 0; k < kXcds; ++k) {
            const int x = (home + k) & (kXcds - 1);
            const int64_t lo = ntiles * x / kXcds;
            const int64_t hi = ntiles * (x + 1) / kXcds;
            const int64_t nchunks = (hi - lo + chunk - 1) / chunk;
            if (threadIdx.x == 0) s_grab = atomicAdd(&queue[x], 1);
            __syncthreads();
            int64_t c = __builtin_amdgcn_readfirstlane(s_grab);
            while (c < nchunks) {
                __syncthreads();                       // everyone has read s_grab
                if (threadIdx.x == 0) s_grab = atomicAdd(&queue[x], 1);
                const int64_t first = lo + c * chunk;
                int64_t last = first + chunk < hi ? first + chunk : hi;
                last = last < t_wave ? last : t_wave;
                if (prefetch) sink ^= sw.prefetch(first, last, VARIANT != KPM_PLAIN && gamma != T(0));
                sw.run(first, last);
                __syncthreads();                       // s_grab is written
                c = __builtin_amdgcn_readfirstlane(s_grab);
            }
        }
    } else {
        const int ngrid = gridDim.x;
        const int X = (xcd_ways > 1 && ngrid % xcd_ways == 0) ? xcd_ways : 1;
        const int xcd = blockIdx.x % X;
        const int slot = blockIdx.x / X;
        const int per = ngrid / X;
        const int64_t t_lo = ntiles * xcd / X;
        const int64_t t_hi = ntiles * (xcd + 1) / X;
        const int64_t n_super = (t_hi - t_lo + chunk - 1) / chunk;
        for (int64_t st = slot; st < n_super; st += per) {
            const int64_t first = t_lo + st * chunk;
            int64_t last = (first + chunk < t_hi) ? first + chunk : t_hi;
            last = last < t_wave ? last : t_wave;
            if (prefetch) sink ^= sw.prefetch(first, last, VARIANT != KPM_PLAIN && gamma != T(0));
            sw.run(first, last);
        }
    }
    asm volatile("" ::"v"(sink));   // the prefetch loads are kept
    double* acc_e = sw.acc_e;
    double* acc_or = sw.acc_or;
    double* acc_oi = sw.acc_oi;

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

template <typename T, int R, int VARIANT, bool BUF, int STREAM>
hipError_t launch_shape(const SweepArgs& a, hipStream_t s) {
    aug_spmmv_kernel<T, R, VARIANT, BUF, STREAM><<<a.grid, kThreads, 0, s>>>(
        static_cast<const T*>(a.val), a.col, a.nrows, static_cast<const T*>(a.V),
        static_cast<T*>(a.W), static_cast<T>(a.alpha), static_cast<T>(a.beta),
        static_cast<T>(a.gamma), a.partials, a.xcd_ways, a.chunk, a.sched, a.queue, a.prefetch);
    return hipGetLastError();
}

template <typename T, int R, int VARIANT, bool BUF>
hipError_t launch_stream(const SweepArgs& a, hipStream_t s) {
    switch (a.stream) {
    case 1: return launch_shape<T, R, VARIANT, BUF, 1>(a, s);
    case 2: return launch_shape<T, R, VARIANT, BUF, 2>(a, s);
    case 3: return launch_shape<T, R, VARIANT, BUF, 3>(a, s);
    default: return launch_shape<T, R, VARIANT, BUF, 0>(a, s);
    }
}

template <typename T, int R, int VARIANT>
hipError_t launch_one(const SweepArgs& a, hipStream_t s) {
    const uint64_t vbytes = static_cast<uint64_t>(a.nrows) * 2 * R * sizeof(T);
    if (vbytes < (1ull << 32)) return launch_stream<T, R, VARIANT, true>(a, s);
    return launch_stream<T, R, VARIANT, false>(a, s);
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

}  // namespace sweep
}  // namespace kpm
