// Fused sweep over a general sparse matrix stored in SELL-C-sigma (the
// unified format the paper builds on, section "Related Work"; chunk height
// C = 1 is the CRS of section "Testbed and Implementation"): the fused body
// of Alg. "kpm_improved_blocked", W <- alpha H V + beta V + gamma W with
// the scalar products <V|V>, <W|V>, for matrices whose rows have any
// number of entries.
//
// Storage (built on the host by kpm_import_csr): rows are sorted by
// decreasing length inside windows of sigma rows; sorted position p holds
// matrix row perm[p] and belongs to chunk p / C; chunk c is stored
// column-major from entry start[c], width[c] entries deep (its longest
// row), so entry j of position p sits at start[p / C] + j C + p mod C.
// Entries past a row's end are padding: value zero and column N, an offset
// just past the vector block, which a buffer load turns into zeros without
// touching memory.  The vector blocks keep the matrix's own row order (the
// permutation only reorders the work), so callers see no difference.
//
// Mapping: a lane owns CPL consecutive complex elements of a block row (16
// bytes where the block is that wide), a wave takes RPW = 64 CPL / R
// consecutive sorted positions per pass.  Where a pass has many rows (RPW >=
// 16) each lane reads the entry of its own row directly: with C >= RPW the
// entries of one slot of a pass are adjacent (one coalesced access).  Where
// it has few (wide blocks) the rows of a pass would all read the same few
// entries per slot, so instead the wave stages the entries of 64 / RPW slots
// of its rows with one coalesced load per lane (lane l: slot l / RPW of row
// l mod RPW), writes them to its LDS slot and every lane reads its row's
// entry back, all lanes of a row at one address (a broadcast).  Either way
// the V rows are gathered four slots at a time (four gathers in flight per
// wave), and the slot loop runs while any row of the pass has entries left.
//
// Work distribution: the passes are split into one contiguous range per die
// (workgroup g runs on die g mod 8), and each die's range into one
// contiguous run per workgroup, whose waves take consecutive passes.
// Contiguous runs keep a workgroup inside a few sorting windows, so that
// the long rows a window starts with are spread over all workgroups.
#include "kpm_batched.h"

namespace kpm {
namespace sell {

using batch::Lanes;
using batch::Pair;
using batch::rsrc;
using batch::Shape;
using batch::wave_sync;
using batch::Words;

constexpr int kWaves = 4;       // waves per workgroup
constexpr int kGroup = 4;       // slots per group, direct loads (gathers in flight per wave)
#ifndef KPM_SELL_STAGED
#define KPM_SELL_STAGED 8
#endif
constexpr int kStaged = KPM_SELL_STAGED;   // slots per group, staged passes (a lattice row: 13)
constexpr unsigned kOut = 0xFFFFFFF0u;   // a buffer offset past every block

// Stage the entries through LDS where a pass has at most this many rows.
template <typename T, int R>
constexpr bool staged() { return Shape<T, R>::RPW <= 8; }

template <typename T, int R, int VARIANT>
__global__ void __launch_bounds__(64 * kWaves, 4)
sell_sweep_kernel(const T* __restrict__ val, const int32_t* __restrict__ col, const int64_t* __restrict__ start,
                  const int32_t* __restrict__ width, const int32_t* __restrict__ perm, int64_t N,
                  int64_t stored, int clog, const T* __restrict__ V, T* __restrict__ W, T alpha, T beta,
                  T gamma, double* __restrict__ partials) {
    using S = Shape<T, R>;
    constexpr int CPL = S::CPL;
    constexpr int LPR = S::LPR;
    constexpr int RPW = S::RPW;
    constexpr bool STAGED = staged<T, R>();
    constexpr int SPG = 64 / RPW;                            // slots per staged group
    using LV = Lanes<T, CPL>;
    using Cv = typename LV::type;
    using P2 = typename Pair<T>::type;
    using WE = Words<2 * static_cast<int>(sizeof(T)) / 4>;   // one stored value
    constexpr unsigned kCB = 2 * sizeof(T);                  // bytes per complex number
    __shared__ double red[kWaves][3][R];
    __shared__ P2 sval[STAGED ? kWaves : 1][64];
    __shared__ unsigned scol[STAGED ? kWaves : 1][64];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int sub = lane / LPR;
    const int cc = lane % LPR;
    const int C = 1 << clog;

    const uint64_t vbytes = static_cast<uint64_t>(N) * R * kCB;
    const __amdgpu_buffer_rsrc_t val_rs = rsrc(val, static_cast<uint64_t>(stored) * kCB);
    const __amdgpu_buffer_rsrc_t col_rs = rsrc(col, static_cast<uint64_t>(stored) * 4);
    const __amdgpu_buffer_rsrc_t vrs = rsrc(V, vbytes);
    const __amdgpu_buffer_rsrc_t wrs = rsrc(W, vbytes);
    // old W only where it enters the result; a resource of size zero reads zeros
    const bool need_w = VARIANT != KPM_PLAIN && gamma != T(0);
    const __amdgpu_buffer_rsrc_t wold_rs = rsrc(W, need_w ? vbytes : 0);
    const unsigned vstep = static_cast<unsigned>(C) * kCB;   // next slot of a chunk
    const unsigned cstep = static_cast<unsigned>(C) * 4;
    const unsigned pad = static_cast<unsigned>(N);           // the padding column

    double ae[CPL], aor[CPL], aoi[CPL];
#pragma unroll
    for (int t = 0; t < CPL; ++t) ae[t] = aor[t] = aoi[t] = 0.0;

    // this workgroup's run of passes
    const int64_t npass = (N + RPW - 1) / RPW;
    const int ngrid = gridDim.x;
    const int X = (ngrid % kXcds == 0) ? kXcds : 1;
    const int per = ngrid / X;
    const int64_t dlo = npass * (blockIdx.x % X) / X, dhi = npass * (blockIdx.x % X + 1) / X;
    const int64_t k = blockIdx.x / X;
    const int64_t qlo = dlo + (dhi - dlo) * k / per, qhi = dlo + (dhi - dlo) * (k + 1) / per;

    // Per-pass metadata, loaded two passes ahead: the lane's own row
    // (compute role: chunk width, V / W offset) and the row whose entries
    // it loads (staging role in a staged pass: lane l loads slot
    // l / RPW of row l mod RPW; otherwise its own row).
    const int ls = STAGED ? lane % RPW : sub;
    const int js = STAGED ? lane / RPW : 0;
    struct Meta {
        int w, ws;               // chunk width of the own row, of the staged row
        unsigned own, ve, ce;    // own V / W offset; first value and column offsets to load
    };
    auto meta = [&](int64_t q) {
        Meta m;
        const int64_t p = q * RPW + sub;
        const bool act = q < qhi && p < N;
        const int64_t pc = act ? p : 0;
        m.w = act ? width[pc >> clog] : 0;
        const int64_t row = (perm && act) ? static_cast<int64_t>(perm[pc]) : pc;
        m.own = act ? static_cast<unsigned>((row * R + cc * CPL) * kCB) : kOut;
        const int64_t ps = q * RPW + ls;
        const bool acts = q < qhi && ps < N;
        const int64_t pcs = acts ? ps : 0;
        m.ws = acts ? width[pcs >> clog] : 0;
        const int64_t e = (acts ? start[pcs >> clog] + (pcs & (C - 1)) : 0) + static_cast<int64_t>(js) * C;
        m.ve = static_cast<unsigned>(e) * kCB;
        m.ce = static_cast<unsigned>(e) * 4;
        return m;
    };
    // one staged load: slot j0 + js of the staged row (padding past its width)
    auto stage = [&](const Meta& m, int j0, P2& hv, unsigned& cv) {
        const bool ok = j0 + js < m.ws;
        hv = __builtin_bit_cast(P2, WE::load(val_rs, ok ? m.ve + j0 * vstep : kOut));
        cv = ok ? static_cast<unsigned>(Words<1>::load(col_rs, m.ce + j0 * cstep)) : pad;
    };

    int64_t q = qlo + wave;
    Meta cur = meta(q), nxt = meta(q + kWaves);
    P2 hv{T(0), T(0)};
    unsigned cv = pad;
    if constexpr (STAGED) stage(cur, 0, hv, cv);
    for (; q < qhi; q += kWaves) {
        const Meta m = cur;
        const Cv vo = LV::load(vrs, m.own);
        const Cv wo = LV::load(wold_rs, m.own);
        const Meta after = meta(q + 2 * kWaves);
        Cv acc;
#pragma unroll
        for (int e = 0; e < 2 * CPL; ++e) acc[e] = T(0);
        // kG slots: their V rows, then the products
        auto slots = [&](const auto& h, const auto& c) {
            constexpr int kG = sizeof(c) / sizeof(c[0]);
            Cv v[kG];
#pragma unroll
            for (int u = 0; u < kG; ++u) v[u] = LV::load(vrs, (c[u] * R + cc * CPL) * kCB);
#pragma unroll
            for (int u = 0; u < kG; ++u) {
#pragma unroll
                for (int t = 0; t < CPL; ++t) {
                    acc[2 * t] = fma(h[u].x, v[u][2 * t], acc[2 * t]);
                    acc[2 * t] = fma(-h[u].y, v[u][2 * t + 1], acc[2 * t]);
                    acc[2 * t + 1] = fma(h[u].x, v[u][2 * t + 1], acc[2 * t + 1]);
                    acc[2 * t + 1] = fma(h[u].y, v[u][2 * t], acc[2 * t + 1]);
                }
            }
        };
        if constexpr (STAGED) {
            P2 hn;
            unsigned cn;
            for (int j0 = 0;;) {
                wave_sync();
                sval[wave][lane] = hv;
                scol[wave][lane] = cv;
                wave_sync();
                const bool more = __builtin_amdgcn_ballot_w64(j0 + SPG < m.ws) != 0;
                // the next group of this pass's rows, or the first group of
                // the next pass: issued right after this group's first
                // gathers, so that waiting for those does not wait for it
                auto next = [&] {
                    if (more) stage(m, j0 + SPG, hn, cn);
                    else stage(nxt, 0, hn, cn);
                };
                bool issued = false;
                for (int u0 = 0; u0 < SPG && __builtin_amdgcn_ballot_w64(j0 + u0 < m.w) != 0; u0 += kStaged) {
                    unsigned c[kStaged];
                    Cv v[kStaged];
#pragma unroll
                    for (int u = 0; u < kStaged; ++u) c[u] = scol[wave][(u0 + u) * RPW + sub];
#pragma unroll
                    for (int u = 0; u < kStaged; ++u) v[u] = LV::load(vrs, (c[u] * R + cc * CPL) * kCB);
                    if (!issued) {
                        next();
                        issued = true;
                    }
#pragma unroll
                    for (int u = 0; u < kStaged; ++u) {
                        const P2 h = sval[wave][(u0 + u) * RPW + sub];
#pragma unroll
                        for (int t = 0; t < CPL; ++t) {
                            acc[2 * t] = fma(h.x, v[u][2 * t], acc[2 * t]);
                            acc[2 * t] = fma(-h.y, v[u][2 * t + 1], acc[2 * t]);
                            acc[2 * t + 1] = fma(h.x, v[u][2 * t + 1], acc[2 * t + 1]);
                            acc[2 * t + 1] = fma(h.y, v[u][2 * t], acc[2 * t + 1]);
                        }
                    }
                }
                if (!issued) next();   // a group without entries
                hv = hn;
                cv = cn;
                if (!more) break;
                j0 += SPG;
            }
        } else {
            unsigned ve = m.ve, ce = m.ce;
            for (int j0 = 0; __builtin_amdgcn_ballot_w64(j0 < m.w) != 0; j0 += kGroup) {
                P2 h[kGroup];
                unsigned c[kGroup];
#pragma unroll
                for (int u = 0; u < kGroup; ++u) {
                    // slots past the row's chunk read zeros and gather nothing
                    const bool ok = j0 + u < m.w;
                    h[u] = __builtin_bit_cast(P2, WE::load(val_rs, ok ? ve + u * vstep : kOut));
                    c[u] = ok ? static_cast<unsigned>(Words<1>::load(col_rs, ce + u * cstep)) : pad;
                }
                slots(h, c);
                ve += kGroup * vstep;
                ce += kGroup * cstep;
            }
        }
        cur = nxt;
        nxt = after;
        const bool act = m.own != kOut;
        const unsigned own = m.own;
        Cv wn;
        if constexpr (VARIANT == KPM_PLAIN) {
            wn = acc;
        } else {
#pragma unroll
            for (int e = 0; e < 2 * CPL; ++e) wn[e] = fma(gamma, wo[e], fma(alpha, acc[e], beta * vo[e]));
        }
        LV::store(wn, wrs, own);   // positions past N: the offset is past the block, the store is dropped
        if constexpr (VARIANT == KPM_FULL) {
#pragma unroll
            for (int t = 0; t < CPL; ++t) {
                const double vr = act ? static_cast<double>(vo[2 * t]) : 0.0;
                const double vi = act ? static_cast<double>(vo[2 * t + 1]) : 0.0;
                const double wr = act ? static_cast<double>(wn[2 * t]) : 0.0;
                const double wi = act ? static_cast<double>(wn[2 * t + 1]) : 0.0;
                ae[t] = fma(vr, vr, fma(vi, vi, ae[t]));
                aor[t] = fma(wr, vr, fma(wi, vi, aor[t]));
                aoi[t] = fma(wr, vi, fma(-wi, vr, aoi[t]));
            }
        }
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
        for (int i = threadIdx.x; i < 3 * R; i += 64 * kWaves) {
            const int qq = i / R, r = i % R;
            double sum = 0.0;
#pragma unroll
            for (int kk = 0; kk < kWaves; ++kk) sum += red[kk][qq][r];
            partials[static_cast<int64_t>(blockIdx.x) * 3 * R + i] = sum;
        }
    }
}

template <typename T, int R, int VARIANT>
hipError_t launch_v(const SellArgs& a, hipStream_t s) {
    sell_sweep_kernel<T, R, VARIANT><<<a.grid, 64 * kWaves, 0, s>>>(
        static_cast<const T*>(a.val), a.col, a.start, a.width, a.perm, a.nrows, a.stored, a.clog,
        static_cast<const T*>(a.V), static_cast<T*>(a.W), static_cast<T>(a.alpha), static_cast<T>(a.beta),
        static_cast<T>(a.gamma), a.partials);
    return hipGetLastError();
}

template <typename T, int R>
hipError_t launch_r(int variant, const SellArgs& a, hipStream_t s) {
    if (variant == KPM_FULL) return launch_v<T, R, KPM_FULL>(a, s);
    if (variant == KPM_NODOT) return launch_v<T, R, KPM_NODOT>(a, s);
    return launch_v<T, R, KPM_PLAIN>(a, s);
}

template <typename T>
hipError_t launch_t(int R, int variant, const SellArgs& a, hipStream_t s) {
    switch (R) {
        case 1: return launch_r<T, 1>(variant, a, s);
        case 2: return launch_r<T, 2>(variant, a, s);
        case 4: return launch_r<T, 4>(variant, a, s);
        case 8: return launch_r<T, 8>(variant, a, s);
        case 16: return launch_r<T, 16>(variant, a, s);
        case 32: return launch_r<T, 32>(variant, a, s);
        case 64: return launch_r<T, 64>(variant, a, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
int rows_per_pass(int R) {
    switch (R) {
        case 1: return Shape<T, 1>::RPW;
        case 2: return Shape<T, 2>::RPW;
        case 4: return Shape<T, 4>::RPW;
        case 8: return Shape<T, 8>::RPW;
        case 16: return Shape<T, 16>::RPW;
        case 32: return Shape<T, 32>::RPW;
        default: return Shape<T, 64>::RPW;
    }
}

}  // namespace sell

hipError_t launch_sell(int dtype, int R, int variant, const SellArgs& a, hipStream_t s) {
    if (a.grid <= 0) return hipErrorInvalidValue;
    if (dtype == KPM_C128) return sell::launch_t<double>(R, variant, a, s);
    return sell::launch_t<float>(R, variant, a, s);
}

// Workgroups of four waves, at most eight per CU (32 waves, the most a CU
// holds), never more than there are passes for.
int sell_grid(int dtype, int R, int64_t nrows) {
    const int rpw = dtype == KPM_C128 ? sell::rows_per_pass<double>(R) : sell::rows_per_pass<float>(R);
    const int64_t npass = (nrows + rpw - 1) / rpw;
    const int64_t want = (npass + sell::kWaves - 1) / sell::kWaves;
    const int64_t cap = static_cast<int64_t>(device_cus()) * 8;
    const int64_t g = want < cap ? want : cap;
    return static_cast<int>(g > 0 ? g : 1);
}

int sell_rows_per_pass(int dtype, int R) {
    return dtype == KPM_C128 ? sell::rows_per_pass<double>(R) : sell::rows_per_pass<float>(R);
}

}  // namespace kpm
