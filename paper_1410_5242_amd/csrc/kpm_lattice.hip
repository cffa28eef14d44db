// Cache-blocked fused sweep for lattice Hamiltonians at R = 32 (and 64).
//
// The generic sweep gathers all 13 neighbour rows of every output row from
// global memory; at R = 32 that is 13 x 512 B per row through each CU's
// texture path, whose address/data units then limit the sweep long before
// HBM does.  Wider blocks are swept one 32-column slice at a time (a wave
// holds one real of each of 32 columns; the LDS ring has room for one
// slice of V at complex128), reading the matrix once per slice.  This kernel exploits what the library knows about its own
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
// a die fetch the same plane at the same time).  Matrix values are read
// once per sweep; the column indices are implied by the slot order and are
// not read.
//
// Pipelining.  During step s a wave has in flight: V of plane s + 2 (stored
// to the ring at the end of the step), the edge neighbours and matrix record
// of step s + 1, and (issued after the compute) the old W rows of step
// s + 1.  Three rules keep those loads in flight instead of being waited on
// early:
//   * every wave issues the same memory instructions every step: an access
//     that must not happen uses a buffer descriptor of size 0 (loads read 0,
//     stores are dropped) instead of a branch, so the compiler's counts of
//     outstanding memory operations stay exact;
//   * the register sets of consecutive steps alternate (the step loop is
//     unrolled by two), so no value is copied out of a register whose load
//     is still pending;
//   * per axis, the neighbour that may lie across the tile edge ("outer")
//     is always taken from registers and the other ("inner") from LDS; which
//     matrix slots they pair with is wave-uniform and is resolved by where
//     the scalar words are fetched from (or which lane is read), so the
//     product loop has no data-dependent selects.
//
// Work distribution: workgroup g works for die g % 8 (the die the
// dispatcher deals it to) and strides over that die's tiles: by default a
// 2-D block of the tile grid (most edge rows a tile gathers then belong to
// tiles of the same die and its L2), else a run of tile rows or no die
// mapping (tuning tile_order).
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

// V and W rows hold R = 32 nsl columns; a wave works on one 32-column slice
// of a row: voff = byte offset of this lane's value within the row (slice
// and lane), soff = byte offset of the row.  The whole array is below 4 GiB,
// so 32-bit offsets suffice.
template <typename T>
__device__ inline T gload(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff) {
    return sweep::buffer_load<T>(rs, voff, soff);
}

typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

// Row `row` of W through a buffer descriptor (one lane offset VGPR shared by
// every access); NT selects the non-temporal cache policy.
template <typename T, bool NT>
__device__ inline T wload(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff) {
    constexpr int aux = NT ? 2 : 0;
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, aux));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, aux));
}
template <typename T, bool NT>
__device__ inline void wstore(T x, __amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff) {
    constexpr int aux = NT ? 2 : 0;
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), rs, voff, soff, aux);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), rs, voff, soff, aux);
}

// The matrix rows of one site (4 rows x 13 complex entries) are one
// contiguous record, read once per sweep with the non-temporal hint (L2 keeps
// the V planes instead); lane l < 52 of a wave loads the entry of row l / 13
// that product l % 13 of that row needs (lane_off; lanes past 52 repeat the
// last entry)
// (16 bytes in complex128, 8 in complex64) with a single vector load, and
// v_readlane hands each entry to the FMAs as a wave-uniform scalar operand.
// Unlike scalar loads (which complete out of order, so every wait drains all
// of them) these loads can be issued a whole step ahead.
template <typename T> struct SiteRec;
template <> struct SiteRec<double> {
    using V = int4;
    static __device__ V load(__amdgpu_buffer_rsrc_t rs, unsigned lane_off, int64_t site) {
        const auto w = __builtin_amdgcn_raw_buffer_load_b128(rs, lane_off, static_cast<unsigned>(site * 4 * kWidth * 16), 2);
        return int4{static_cast<int>(w[0]), static_cast<int>(w[1]), static_cast<int>(w[2]), static_cast<int>(w[3])};
    }
    static __device__ double re(const V& v, int l) {
        return __hiloint2double(__builtin_amdgcn_readlane(v.y, l), __builtin_amdgcn_readlane(v.x, l));
    }
    static __device__ double im(const V& v, int l) {
        return __hiloint2double(__builtin_amdgcn_readlane(v.w, l), __builtin_amdgcn_readlane(v.z, l));
    }
    // an entry already in every lane (read back from LDS)
    static __device__ double re(const V& v) { return __hiloint2double(v.y, v.x); }
    static __device__ double im(const V& v) { return __hiloint2double(v.w, v.z); }
};
template <> struct SiteRec<float> {
    using V = int2;
    static __device__ V load(__amdgpu_buffer_rsrc_t rs, unsigned lane_off, int64_t site) {
        const auto w = __builtin_amdgcn_raw_buffer_load_b64(rs, lane_off, static_cast<unsigned>(site * 4 * kWidth * 8), 2);
        return int2{static_cast<int>(w[0]), static_cast<int>(w[1])};
    }
    static __device__ float re(const V& v, int l) { return __int_as_float(__builtin_amdgcn_readlane(v.x, l)); }
    static __device__ float im(const V& v, int l) { return __int_as_float(__builtin_amdgcn_readlane(v.y, l)); }
    static __device__ float re(const V& v) { return __int_as_float(v.x); }
    static __device__ float im(const V& v) { return __int_as_float(v.y); }
};

// Exchange with lane ^ 1 (DPP quad_perm [1, 0, 3, 2]); every lane of the wave
// is active in this kernel, so the "old" operand is never used.
__device__ inline double swap_lanes(double x) {
    const int lo = __double2loint(x), hi = __double2hiint(x);
    return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0xB1, 0xF, 0xF, false),
                            __builtin_amdgcn_update_dpp(lo, lo, 0xB1, 0xF, 0xF, false));
}
__device__ inline float swap_lanes(float x) {
    const int b = __float_as_int(x);
    return __int_as_float(__builtin_amdgcn_update_dpp(b, b, 0xB1, 0xF, 0xF, false));
}

// Values a step carries for the next one: V rows of the (at most two)
// neighbours across the tile edge, old W rows, and the matrix-row record.
template <typename T> struct StepRegs {
    T h[2][4];
    T w[4];
    typename SiteRec<T>::V hv;   // VALS 1 and 3
    unsigned warm;               // VALS 2
};

// VALS 2: one dword of every 128-byte line that the site's matrix record
// (4 rows x 13 complex entries) touches; lanes past the last line repeat the
// record's last dword.
template <typename T>
__device__ inline unsigned warm_load(__amdgpu_buffer_rsrc_t rs, int lane, int64_t site) {
    constexpr int kRec = 4 * kWidth * 2 * static_cast<int>(sizeof(T));
    const unsigned voff = static_cast<unsigned>(min(lane * 128, kRec - 4));
    return __builtin_amdgcn_raw_buffer_load_b32(rs, voff, static_cast<unsigned>(site * kRec), 2);
}

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

// VALS: how the matrix rows reach the FMAs as wave-uniform operands.
//   0  scalar buffer loads when the row is processed
//   1  one vector load per site a step ahead, v_readlane per entry
//   2  scalar loads, with the site's rows pulled into L2 by a vector load a
//      step ahead (the scalar loads then wait on L2, not on HBM)
//   3  the vector load of 1, written to the wave's slot in LDS at the start
//      of the step and read back per entry with every lane at the same
//      address (a broadcast): no v_readlane and none of the wait states a
//      VALU read of its scalar result needs, at the cost of LDS reads

// NSL: 32-column slices per block row (0: run-time value nsl, for R > 32).
// SPLIT: pencils are cut into npc z-pieces (run-time npc); otherwise a work
// item is a whole pencil.  BIG: V, W or the matrix reach 4 GiB; every
// access then goes through a descriptor over the one z-plane it reads or
// writes (32-bit offsets within a plane), built where it is used.
template <typename T, int VARIANT, int VALS, int STREAM, int NSL, bool SPLIT, bool BIG = false>
__global__ void __launch_bounds__(kThreadsL)
lattice_kernel(const T* __restrict__ val, const T* __restrict__ V, T* __restrict__ W,
               T alpha, T beta, T gamma, double* __restrict__ partials,
               int Lx, int Ly, int Lz, int px, int py, int pz, int ntx, int ntiles, int order, int nsl, int npc) {
    __shared__ T ring[4][kNW][4][kE];
    __shared__ T zrow[4][kE];          // rows of zeros: neighbours beyond an open side
    __shared__ double red[kNW][3][kR];
    // VALS 3: the step's matrix record of every wave, in the space of the
    // partial sums (those are written only after a slice's last step, which
    // ends with a workgroup barrier, and read before the next slice starts)
    using Rec = typename SiteRec<T>::V;
    static_assert(VALS != 3 || sizeof(Rec) * kNW * 64 <= sizeof(red), "record slots exceed the partial sums");
    Rec (*recs)[64] = reinterpret_cast<Rec (*)[64]>(&red[0][0][0]);

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ti = wave % kP, tj = wave / kP;
    const bool im_part = (lane & 1) != 0;
    const T sgn = im_part ? T(1) : T(-1);
    const bool need_w = VARIANT != KPM_PLAIN && gamma != T(0);
    constexpr int kValWords = 2 * kWidth * static_cast<int>(sizeof(T)) / 4;
    constexpr int wpv = static_cast<int>(sizeof(T)) / 4;
    const int64_t plane_sites = static_cast<int64_t>(Lx) * Ly;
    const int64_t nrows = 4 * plane_sites * Lz;
    // Every global access goes through a buffer descriptor clipped to its
    // array.  An access that must not happen (inactive wave, step past the
    // end of the pencil, no halo neighbour, no old W) uses a descriptor of
    // size 0: loads return 0 and stores are dropped, so every wave issues
    // the same sequence of memory instructions each step and the compiler's
    // memory-counter waits stay exact.
    const int nslice = NSL > 0 ? NSL : nsl;
    const unsigned rowb = static_cast<unsigned>(nslice * kE * static_cast<int>(sizeof(T)));
    const unsigned vbytes = static_cast<unsigned>(nrows * rowb);
    // byte offset of a row of V or W
    auto roff = [&](int64_t row) -> unsigned {
        if constexpr (NSL == 1) return static_cast<unsigned>(row * kE * static_cast<int64_t>(sizeof(T)));
        else return static_cast<unsigned>(row) * rowb;
    };
    const unsigned mbytes = static_cast<unsigned>(nrows * 2 * kWidth * static_cast<int64_t>(sizeof(T)));
    auto rsrc = [](const void* p, unsigned bytes) {
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, static_cast<int>(bytes),
                                                 sweep::kBufferWord3);
    };
    // descriptors are rebuilt where used (only the size word differs), which
    // keeps fewer scalar registers live than holding both variants
    auto vrs = [&](bool on) { return rsrc(V, on ? vbytes : 0u); };
    auto wrs = [&](bool on) { return rsrc(W, on ? vbytes : 0u); };
    auto mrs = [&](bool on) { return rsrc(val, on ? mbytes : 0u); };
    // BIG: descriptors over plane z of V, W and the matrix (size 0 when off)
    const uint64_t pvb = static_cast<uint64_t>(4 * plane_sites) * rowb;
    const uint64_t pmb = static_cast<uint64_t>(4 * plane_sites) * 2 * kWidth * sizeof(T);
    auto vrsp = [&](bool on, int64_t z) {
        return rsrc(reinterpret_cast<const char*>(V) + (on ? z : 0) * pvb, on ? static_cast<unsigned>(pvb) : 0u);
    };
    auto wrsp = [&](bool on, int64_t z) {
        return rsrc(reinterpret_cast<const char*>(W) + (on ? z : 0) * pvb, on ? static_cast<unsigned>(pvb) : 0u);
    };
    auto mrsp = [&](bool on, int64_t z) {
        return rsrc(reinterpret_cast<const char*>(val) + (on ? z : 0) * pmb, on ? static_cast<unsigned>(pmb) : 0u);
    };

    if (wave < 4) zrow[wave][lane] = T(0);

    const int ngrid = gridDim.x;
    const int X = (order != 2 && ngrid % kXcds == 0) ? kXcds : 1;
    const int xcd = blockIdx.x % X;
    const int slot = blockIdx.x / X;
    const int per = ngrid / X;
    // work items: npc consecutive z-pieces of every pencil (npc = 1: whole
    // pencils)
    const int npieces = SPLIT ? npc : 1;
    const int nitems = ntiles * npieces;
    const int k_lo = static_cast<int>(static_cast<int64_t>(nitems) * xcd / X);
    const int k_hi = static_cast<int>(static_cast<int64_t>(nitems) * (xcd + 1) / X);
    const int nty = ntiles / ntx;
    // order 0: each die takes a 2-D block of (ntx/2) x (nty/4) tiles, so that
    // most tiles whose edge rows it gathers are its own; order 1: each die
    // takes a contiguous run of tile rows; order 2: no die mapping
    const bool blocks = order == 0 && X == kXcds && ntx % 2 == 0 && nty % 4 == 0 && !SPLIT;

    constexpr bool VEC_VALS = VALS == 1 || VALS == 3;
    unsigned sink = 0;   // keeps the L2 warm-up loads of VALS == 2

    // Blocks wider than 32 columns: every workgroup sweeps its tiles once per
    // 32-column slice (the matrix is read once per slice).
    for (int sl = 0; sl < nslice; ++sl) {
    const unsigned voff = static_cast<unsigned>((sl * kE + lane) * static_cast<int>(sizeof(T)));
    double acc_e = 0.0, acc_or = 0.0, acc_oi = 0.0;

    for (int k = k_lo + slot; k < k_hi; k += per) {
        const int tile = SPLIT ? k / npieces : k;
        const int piece = SPLIT ? k - tile * npieces : 0;
        const int z0 = SPLIT ? piece * Lz / npieces : 0;               // planes [z0, z1) of this item
        const int z1 = SPLIT ? (piece + 1) * Lz / npieces : Lz;
        int tx = tile % ntx, ty = tile / ntx;
        if (blocks) {
            const int bw = ntx / 2, bh = nty / 4, i = k - k_lo;
            tx = (xcd % 2) * bw + i % bw;
            ty = (xcd / 2) * bh + i / bw;
        }
        const int x0 = tx * kP, y0 = ty * kP;
        const int Lxv = min(kP, Lx - x0), Lyv = min(kP, Ly - y0);   // valid extent of the tile (>= 2)
        const int x = x0 + ti, y = y0 + tj;
        const bool active = ti < Lxv && tj < Lyv;                     // wave-uniform
        // an inactive wave (tile cut by the lattice edge) runs the same code
        // on its own ring slot (zeros) with every global access disabled
        const int64_t sxy = active ? static_cast<int64_t>(x) + static_cast<int64_t>(Lx) * y : 0;
        Nb nb[4];
        nb[0] = xy_neighbour(x - 1, y, Lx, Ly, px, py, x0, y0, Lxv, Lyv);
        nb[1] = xy_neighbour(x + 1, y, Lx, Ly, px, py, x0, y0, Lxv, Lyv);
        nb[2] = xy_neighbour(x, y - 1, Lx, Ly, px, py, x0, y0, Lxv, Lyv);
        nb[3] = xy_neighbour(x, y + 1, Lx, Ly, px, py, x0, y0, Lxv, Lyv);
        // A tile is at least 2 sites wide in x and y, so a site has at most
        // one neighbour across the tile edge in x and one in y.  Per axis,
        // the "outer" neighbour lives in registers (r.h[axis]): the one
        // across the tile edge, gathered from memory a step ahead, else
        // (interior site, or a side beyond an open boundary) copied from LDS
        // at the start of the step.  The "inner" one is read from LDS (ring
        // slot of an in-tile site, or zero rows).  Only constant indices into
        // nb: a run-time index would place the array in scratch memory.
        auto outer_of = [&](const Nb& m, const Nb& p) -> int {
            if (m.kind == 2) return 0;
            if (p.kind == 2) return 1;
            if (p.kind == 0) return 1;
            if (m.kind == 0) return 0;
            return 1;
        };
        const int dox = outer_of(nb[0], nb[1]), doy = outer_of(nb[2], nb[3]);
        const Nb ox = dox ? nb[1] : nb[0], ix = dox ? nb[0] : nb[1];
        const Nb oy = doy ? nb[3] : nb[2], iy = doy ? nb[2] : nb[3];
        const bool hx_on = active && ox.kind == 2, hy_on = active && oy.kind == 2;
        // VALS 1: lane l holds the matrix entry of product l % 13 of row l / 13
        // (product order: slot 0, outer x pair, inner x pair, outer y pair,
        // inner y pair, slots 9..12), so every hand-over reads a fixed lane
        unsigned rec_off = 0;
        if constexpr (VEC_VALS) {
            const int e = min(lane, 4 * kWidth - 1), r = e / kWidth, j = e % kWidth;
            int sl = j;
            if (j >= 1 && j <= 4) sl = (j <= 2) ? j + 2 * dox : j - 2 * dox;
            if (j >= 5 && j <= 8) sl = (j <= 6) ? j + 2 * doy : j - 2 * doy;
            rec_off = static_cast<unsigned>((r * kWidth + sl) * 2 * static_cast<int>(sizeof(T)));
        }
        const int64_t hxs = hx_on ? ox.idx : 0;   // halo sites (within a plane)
        const int64_t hys = hy_on ? oy.idx : 0;
        const __amdgpu_buffer_rsrc_t wst = wrs(active);   // new-W stores
        const v4i32 val_rs = scalar_rsrc(val, active ? mbytes : 0u);

        // plane index of step s' (with periodic wrap); -1 when it does not exist
        auto plane_of = [&](int sp) -> int {
            if (sp >= 0 && sp < Lz) return sp;
            return pz ? (sp + Lz) % Lz : -1;
        };
        // halo neighbours, old W rows and (VALS 1) matrix rows of the step in
        // plane zp (on = the step exists)
        auto load_step = [&](bool on, int zp, StepRegs<T>& r) {
            const int64_t z = on ? zp : 0;
            if constexpr (BIG) {
                const __amdgpu_buffer_rsrc_t hx = vrsp(on && hx_on, z);
                const __amdgpu_buffer_rsrc_t hy = vrsp(on && hy_on, z);
#pragma unroll
                for (int o = 0; o < 4; ++o) r.h[0][o] = gload<T>(hx, voff, roff(4 * hxs + o));
#pragma unroll
                for (int o = 0; o < 4; ++o) r.h[1][o] = gload<T>(hy, voff, roff(4 * hys + o));
                r.hv = SiteRec<T>::load(mrsp(on && active, z), rec_off, sxy);
            } else {
                const __amdgpu_buffer_rsrc_t hx = vrs(on && hx_on);
                const __amdgpu_buffer_rsrc_t hy = vrs(on && hy_on);
#pragma unroll
                for (int o = 0; o < 4; ++o) r.h[0][o] = gload<T>(hx, voff, roff(4 * (hxs + plane_sites * z) + o));
#pragma unroll
                for (int o = 0; o < 4; ++o) r.h[1][o] = gload<T>(hy, voff, roff(4 * (hys + plane_sites * z) + o));
                const int64_t base = 4 * (sxy + plane_sites * z);
                if constexpr (VEC_VALS) r.hv = SiteRec<T>::load(mrs(on && active), rec_off, base / 4);
            }
        };
        // this site's rows of V in plane zp (zeros when off)
        auto load_wold = [&](bool on, int zp, StepRegs<T>& r) {
            if constexpr (BIG) {
                const __amdgpu_buffer_rsrc_t wl = wrsp(on && active && need_w, zp);
#pragma unroll
                for (int o = 0; o < 4; ++o) r.w[o] = wload<T, (STREAM & 1) != 0>(wl, voff, roff(4 * sxy + o));
            } else {
                const __amdgpu_buffer_rsrc_t wl = wrs(on && active && need_w);
                const int64_t base = 4 * (sxy + plane_sites * (on ? zp : 0));
#pragma unroll
                for (int o = 0; o < 4; ++o) r.w[o] = wload<T, (STREAM & 1) != 0>(wl, voff, roff(base + o));
            }
        };
        auto load_plane = [&](bool on, int zp, T (&p)[4]) {
            if constexpr (BIG) {
                const __amdgpu_buffer_rsrc_t rs = vrsp(on && active, zp);
#pragma unroll
                for (int o = 0; o < 4; ++o) p[o] = gload<T>(rs, voff, roff(4 * sxy + o));
            } else {
                const __amdgpu_buffer_rsrc_t rs = vrs(on && active);
                const int64_t base = 4 * (sxy + plane_sites * (on ? zp : 0));
#pragma unroll
                for (int o = 0; o < 4; ++o) p[o] = gload<T>(rs, voff, roff(base + o));
            }
        };

        // One z-step.  Register sets alternate between even and odd steps,
        // so nothing is copied out of a set whose loads are still in flight:
        //   cur    halo, old W and matrix rows of step s (loaded in step s - 1)
        //   nxt    receives those of step s + 1
        //   p      receives V of plane s + 2, stored to the ring at the end
        //          of the step
        // Loads are issued warm-up first, then the plane, then the rest, so
        // the waits at the end of the step leave the later loads in flight.
        auto step = [&](int s, StepRegs<T>& cur, StepRegs<T>& nxt) {
            const bool on1 = s + 1 < z1;                       // step s + 1 exists
            const int zn2 = on1 ? plane_of(s + 2) : -1;        // plane used by step s + 1
            T p[4];
            if constexpr (VALS == 2)
                nxt.warm = warm_load<T>(mrs(on1 && active), lane, sxy + plane_sites * (on1 ? s + 1 : 0));
            load_plane(zn2 >= 0, zn2, p);
            load_step(on1, s + 1, nxt);

            // outer neighbours not gathered from memory: copy from LDS
            if (ox.kind != 2) {
                const T* src = ox.kind == 1 ? &ring[s & 3][ox.idx][0][lane] : &zrow[0][lane];
#pragma unroll
                for (int o = 0; o < 4; ++o) cur.h[0][o] = src[o * kE];
            }
            if (oy.kind != 2) {
                const T* src = oy.kind == 1 ? &ring[s & 3][oy.idx][0][lane] : &zrow[0][lane];
#pragma unroll
                for (int o = 0; o < 4; ++o) cur.h[1][o] = src[o * kE];
            }
            const T* inx = ix.kind == 1 ? &ring[s & 3][ix.idx][0][lane] : &zrow[0][lane];
            const T* iny = iy.kind == 1 ? &ring[s & 3][iy.idx][0][lane] : &zrow[0][lane];
            const T* zdn = plane_of(s - 1) >= 0 ? &ring[(s - 1) & 3][wave][0][lane] : &zrow[0][lane];
            const T* zup = plane_of(s + 1) >= 0 ? &ring[(s + 1) & 3][wave][0][lane] : &zrow[0][lane];
            const int64_t site = sxy + plane_sites * s;
            // new-W stores of this step (BIG: a descriptor over plane s)
            __amdgpu_buffer_rsrc_t wss = wst;
            if constexpr (BIG) wss = wrsp(active, s);
            if constexpr (VALS == 3) {
                // this step's record into the wave's LDS slot (the previous
                // step's reads of the slot come first: LDS executes a wave's
                // accesses in order, the fences only stop the compiler)
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                recs[wave][lane] = cur.hv;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                const int64_t row = 4 * site + o;
                // matrix entries as scalar words, in product order: slot 0,
                // the outer and inner x pairs, the outer and inner y pairs,
                // slots 9..12.  Which pair is outer is wave-uniform (dox,
                // doy) and is chosen by where the words are loaded from, not
                // by moving vector data.
                int wv[VEC_VALS ? 1 : kValWords];
                if constexpr (!VEC_VALS) {
                    constexpr int SW = 2 * wpv;   // words per slot
                    const unsigned rb = static_cast<unsigned>(row * kValWords * 4);
                    sload<SW>(val_rs, rb, wv);
                    sload<2 * SW>(val_rs, rb + (1 + 2 * dox) * SW * 4, wv + SW);
                    sload<2 * SW>(val_rs, rb + (3 - 2 * dox) * SW * 4, wv + 3 * SW);
                    sload<2 * SW>(val_rs, rb + (5 + 2 * doy) * SW * 4, wv + 5 * SW);
                    sload<2 * SW>(val_rs, rb + (7 - 2 * doy) * SW * 4, wv + 7 * SW);
                    sload<4 * SW>(val_rs, rb + 9 * SW * 4, wv + 9 * SW);
                }
                T v[kWidth];
                v[0] = ring[s & 3][wave][o][lane];
                v[1] = cur.h[0][o];
                v[2] = cur.h[0][o ^ 3];
                v[3] = inx[o * kE];
                v[4] = inx[(o ^ 3) * kE];
                v[5] = cur.h[1][o];
                v[6] = cur.h[1][o ^ 3];
                v[7] = iny[o * kE];
                v[8] = iny[(o ^ 3) * kE];
                v[9] = zdn[o * kE];
                v[10] = zdn[(o ^ 2) * kE];
                v[11] = zup[o * kE];
                v[12] = zup[(o ^ 2) * kE];
                T A = T(0), B = T(0);
                if constexpr (VALS == 3) {
#pragma unroll
                    for (int j = 0; j < kWidth; ++j) {
                        const typename SiteRec<T>::V e = recs[wave][kWidth * o + j];
                        A = fma(SiteRec<T>::re(e), v[j], A);
                        B = fma(SiteRec<T>::im(e), v[j], B);
                    }
                } else if constexpr (VEC_VALS) {
#pragma unroll
                    for (int j = 0; j < kWidth; ++j) {
                        A = fma(SiteRec<T>::re(cur.hv, kWidth * o + j), v[j], A);
                        B = fma(SiteRec<T>::im(cur.hv, kWidth * o + j), v[j], B);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < kWidth; ++j) {
                        A = fma(from_words<T>(wv + (2 * j) * wpv), v[j], A);
                        B = fma(from_words<T>(wv + (2 * j + 1) * wpv), v[j], B);
                    }
                }
                const T hv = fma(sgn, swap_lanes(B), A);
                const int64_t srow = BIG ? 4 * sxy + o : row;   // row within the stores' descriptor
                if constexpr (VARIANT == KPM_PLAIN) {
                    wstore<T, (STREAM & 2) != 0>(hv, wss, voff, roff(srow));
                } else {
                    // cur.w holds zeros when no old W is read (need_w false)
                    const T w = fma(gamma, cur.w[o], fma(alpha, hv, beta * v[0]));
                    wstore<T, (STREAM & 2) != 0>(w, wss, voff, roff(srow));
                    if constexpr (VARIANT == KPM_FULL) {
                        const double vd = static_cast<double>(v[0]);
                        const double vsw = static_cast<double>(swap_lanes(v[0]));
                        const double wd = static_cast<double>(w);
                        acc_e = fma(vd, vd, acc_e);
                        acc_or = fma(wd, vd, acc_or);
                        acc_oi = fma(wd, vsw, acc_oi);
                    }
                }
            }
            // plane s + 2 (zeros when it does not exist) replaces plane s - 2,
            // last read in step s - 1
            load_wold(on1, s + 1, nxt);
#pragma unroll
            for (int o = 0; o < 4; ++o) ring[(s + 2) & 3][wave][o][lane] = p[o];
            // VALS 2: consume the warm-up load (older than the plane just stored)
            if constexpr (VALS == 2) sink ^= static_cast<unsigned>(__builtin_amdgcn_readfirstlane(nxt.warm));
            __syncthreads();
        };

        // prologue: planes z0 - 1, z0, z0 + 1 into their ring slots (zeros
        // where a plane does not exist); halo, old W and matrix rows of step z0
        {
            T q[3][4];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int zp = plane_of(z0 + i - 1);
                load_plane(zp >= 0, zp, q[i]);
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
#pragma unroll
                for (int o = 0; o < 4; ++o) ring[(z0 + i + 3) & 3][wave][o][lane] = q[i][o];
            }
        }
        StepRegs<T> ra, rb;
        load_step(true, z0, ra);
        load_wold(true, z0, ra);
        __syncthreads();

        int s = z0;
        for (; s + 1 < z1; s += 2) {
            step(s, ra, rb);
            step(s + 1, rb, ra);
        }
        if (s < z1) step(s, ra, rb);
    }

    // this slice's columns of the workgroup's [3][R] partial sums
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
        const int64_t R = static_cast<int64_t>(nslice) * kR;
        for (int i = threadIdx.x; i < 3 * kR; i += kThreadsL) {
            const int q = i / kR, r = i % kR;
            double sum = 0.0;
            for (int w = 0; w < kNW; ++w) sum += red[w][q][r];
            partials[static_cast<int64_t>(blockIdx.x) * 3 * R + q * R + sl * kR + r] = sum;
        }
        __syncthreads();   // red is rewritten by the next slice
    }
    }
    asm volatile("" ::"s"(sink));
}

// z-pieces per pencil: 2 when more pencils than workgroups leave the last
// round of pencils partly empty and halving the pencils shortens the longest
// workgroup's work (rounds x (planes + 2 steps of pipeline fill)), else 1
int pieces(int ntiles, int grid, int Lz) {
    if (grid <= 0 || ntiles <= grid || Lz < 8) return 1;
    auto cost = [&](int p) {
        const int64_t rounds = (static_cast<int64_t>(ntiles) * p + grid - 1) / grid;
        return rounds * (Lz / p + 2);
    };
    return cost(2) < cost(1) ? 2 : 1;
}

// V, W or the matrix reach 4 GiB: the per-plane descriptors of BIG
bool big_arrays(const int L[3], int R, size_t real) {
    const uint64_t n = 4ull * L[0] * L[1] * L[2];
    return n * R * 2 * real >= (1ull << 32) || n * kWidth * 2 * real >= (1ull << 32);
}

template <typename T, int STREAM>
hipError_t launch_ts(int variant, const LatticeArgs& a, hipStream_t s) {
    const int ntx = (a.L[0] + kP - 1) / kP, nty = (a.L[1] + kP - 1) / kP;
    const int ntiles = ntx * nty;
    const bool big = big_arrays(a.L, a.R, sizeof(T));
    // pencils are split only at R = 32 on the record path (prefetch 2), and
    // not with the per-plane descriptors
    const int npc = (!big && a.R == kR && a.prefetch == 2) ? pieces(ntiles, a.grid, a.L[2]) : 1;
#define KPM_LAUNCH(VAR, VALS, NSL) KPM_LAUNCH_S(VAR, VALS, NSL, false)
#define KPM_LAUNCH_S(VAR, VALS, NSL, SPLIT) KPM_LAUNCH_B(VAR, VALS, NSL, SPLIT, false)
#define KPM_LAUNCH_B(VAR, VALS, NSL, SPLIT, BIG)                                                 \
    lattice_kernel<T, VAR, VALS, STREAM, NSL, SPLIT, BIG><<<a.grid, kThreadsL, 0, s>>>(          \
        static_cast<const T*>(a.val), static_cast<const T*>(a.V), static_cast<T*>(a.W),          \
        static_cast<T>(a.alpha), static_cast<T>(a.beta), static_cast<T>(a.gamma), a.partials,  \
        a.L[0], a.L[1], a.L[2], a.periodic[0], a.periodic[1], a.periodic[2], ntx, ntiles, a.order, \
        a.R / kR, npc)
// tuning `prefetch`: 2 (default) the site's matrix record a step ahead in
// registers (VALS 1 in complex128; VALS 3 in complex64, where the
// v_readlane hand-over and its wait states made the sweep VALU-bound, and
// the record's 8-byte entries leave room for the LDS reads: 0.57 -> 0.73 of
// peak on 128 x 128 x 64; in complex128 the 16-byte entries read from LDS
// spill registers), 1 scalar loads after an L2 warm-up (VALS 2), 0 plain
// scalar loads.  Blocks wider than 32 columns always take the record path.
    constexpr int REC = sizeof(T) == 4 ? 3 : 1;
#define KPM_LAUNCH_V(VAR)                          \
    if (big) {                                     \
        if (a.R > kR) KPM_LAUNCH_B(VAR, REC, 0, false, true);  \
        else KPM_LAUNCH_B(VAR, REC, 1, false, true);           \
    } else if (a.R > kR) {                         \
        KPM_LAUNCH(VAR, REC, 0);                   \
    } else if (npc > 1) {                          \
        KPM_LAUNCH_S(VAR, REC, 1, true);           \
    } else {                                       \
        switch (a.prefetch) {                      \
        case 2: KPM_LAUNCH(VAR, REC, 1); break;    \
        case 1: KPM_LAUNCH(VAR, 2, 1); break;      \
        default: KPM_LAUNCH(VAR, 0, 1); break;     \
        }                                          \
    }
    if (a.R <= 0 || a.R % kR != 0) return hipErrorInvalidValue;
    switch (variant) {
    case KPM_FULL: KPM_LAUNCH_V(KPM_FULL); break;
    case KPM_NODOT: KPM_LAUNCH_V(KPM_NODOT); break;
    case KPM_PLAIN: KPM_LAUNCH_V(KPM_PLAIN); break;
    default: return hipErrorInvalidValue;
    }
#undef KPM_LAUNCH_V
#undef KPM_LAUNCH_B
#undef KPM_LAUNCH_S
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
    if (R <= 0 || R % lattice::kR != 0) return false;
    // every tile must be at least 2 sites wide in x and y (at most one
    // neighbour across each tile edge): no side with L mod 4 == 1
    if (H->L[0] % lattice::kP == 1 || H->L[1] % lattice::kP == 1) return false;
    // arrays of 4 GiB or more take per-plane descriptors: one plane of the
    // block and of the matrix must stay below 4 GiB
    const size_t real = H->dtype == KPM_C128 ? sizeof(double) : sizeof(float);
    const uint64_t plane_rows = 4ull * H->L[0] * H->L[1];
    return H->L[0] > 0 && plane_rows * R * 2 * real < (1ull << 32) && plane_rows * kWidth * 2 * real < (1ull << 32);
}

int lattice_grid(const kpm_hamiltonian* H) {
    const int ntiles = lattice_tiles(H);
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
    }
    // LDS per workgroup: 142 KB (complex128) or 77 KB (complex64), so at
    // most 1 or 2 workgroups fit on a CU; default 1
    const int max_per_cu = (H->dtype == KPM_C128) ? 1 : 2;
    const int want = get_tuning().wg_per_cu;
    const int per_cu = want > 0 ? (want < max_per_cu ? want : max_per_cu) : 1;
    int g = cus * per_cu;
    if (g > ntiles) g = ntiles;
    if (g >= kXcds) g -= g % kXcds;
    return g > 0 ? g : 1;
}

int lattice_pieces(const kpm_hamiltonian* H, int R, int grid, int prefetch) {
    // as launch_ts: pencils are split only at R = 32 on the record path,
    // with the whole-array descriptors
    const size_t real = H->dtype == KPM_C128 ? sizeof(double) : sizeof(float);
    if (lattice::big_arrays(H->L, R, real)) return 1;
    return (R == lattice::kR && prefetch == 2) ? lattice::pieces(lattice_tiles(H), grid, H->L[2]) : 1;
}

hipError_t launch_lattice(int dtype, int variant, const LatticeArgs& a, hipStream_t s) {
    if (dtype == KPM_C128) return lattice::launch_t<double>(variant, a, s);
    return lattice::launch_t<float>(variant, a, s);
}

}  // namespace kpm
