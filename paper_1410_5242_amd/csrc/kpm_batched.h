#pragma once
// Batched persistent KPM solver: many independent Hamiltonians (disorder
// realisations, lattices of different size) solved in one launch.
//
// Every instance is the whole iteration of Alg. "kpm_improved_blocked"
// (M/2 fused sweeps, eta reduction, eta -> mu) for its own H and start
// block.  Instances share nothing, so one workgroup owns one instance from
// its first sweep to its moments and synchronises only with itself: the
// only barrier between sweep k and sweep k + 1 is a workgroup barrier, and
// the scalar products of a sweep are summed inside the workgroup in a fixed
// order, so the result of an instance does not depend on which workgroup
// ran it or on what else ran beside it.
//
// Work distribution: the host lists the instances longest-first; the
// persistent grid takes them from that list through an atomic counter
// (greedy longest-processing-time scheduling), or, without the counter,
// workgroup g takes entries g, g + grid, ...
//
// Thread mapping (wave64): a lane owns CPL consecutive complex elements of
// a block row (16 bytes where the block is wide enough), so a wave covers
// 64 CPL / R block rows per pass.  The matrix values of a pass (contiguous
// in memory) are copied by the wave into its own LDS slot with coalesced
// loads one pass ahead, and every lane then reads the entries of its own row
// from LDS; the 13 neighbour rows of V are gathered straight from memory.
//
// Column indices are not read: every Hamiltonian of the library comes from
// its lattice builder, whose slot order fixes the column of each entry (slot
// 0 the row itself; then for axis x, y, z the site n - e_j and n + e_j, each
// with the same orbital o and the partner orbital, o ^ 3 for x and y, o ^ 2
// for z; a neighbour beyond an open side is a padding slot of value 0).  A
// lane derives its row's site (x, y, z) with two reciprocal multiplications
// and forms the 13 gather offsets, which saves the 13 x 4 bytes of indices
// per row that a sweep would otherwise stream.  The extra integer work per
// pass needs two waves per SIMD to hide (8-wave workgroups).
//
// The pass body has no divergent branches, so that the compiler's count of
// outstanding memory operations stays exact and a pass never waits for the
// stores of the previous one: every access goes through a buffer resource
// clipped to its array (reads past the end return zero, writes past it are
// dropped), which makes the ragged last pass and the read-ahead past the
// last pass safe without per-lane conditions, and a resource of size zero
// switches off the old-W read of the first sweep.
#include "kpm_internal.h"

namespace kpm {
namespace batch {

constexpr int kLdsMax = 160 * 1024;

// Waves per SIMD the register allocation must leave room for: complex128
// keeps 13 gathered (re, im) pairs of doubles per row in flight per lane and
// gets up to 256 registers (at most 8 waves per workgroup).
template <typename T> constexpr int kMinWaves = sizeof(T) == 8 ? 2 : 4;
template <typename T> constexpr int kMaxWaves = sizeof(T) == 8 ? 8 : 16;

// A lane owns CPL consecutive complex elements of a block row, 16 bytes
// where the block is wide enough: every vector memory instruction of the
// sweep then moves 16 bytes per lane (the texture-address path, not HBM,
// limits a gather-heavy sweep, and its cost is per lane and instruction).
template <typename T, int R>
constexpr int cpl() {
    return (16 / (2 * static_cast<int>(sizeof(T)))) < R ? 16 / (2 * static_cast<int>(sizeof(T))) : R;
}

template <typename T, int R>
struct Shape {
    static constexpr int CPL = cpl<T, R>();                                 // complex per lane
    static constexpr int LPR = R / CPL;                                      // lanes per row
    static constexpr int RPW = 64 / LPR;                                     // rows per pass
    static constexpr int kValWords = kWidth * 2 * static_cast<int>(sizeof(T)) / 4;   // per row
    static constexpr int kV = RPW * kValWords;                              // value words per pass
    static constexpr int kC = RPW * kWidth;                                 // column words per pass
    // widest load (in words) that divides a part, so that every load of a
    // pass is aligned (passes start at multiples of RPW rows)
    static constexpr int kVecV = kV % 4 == 0 ? 4 : kV % 2 == 0 ? 2 : 1;
    static constexpr int kVecC = kC % 4 == 0 ? 4 : kC % 2 == 0 ? 2 : 1;
    static constexpr int kLoadsV = (kV / kVecV + 63) / 64;                   // loads per lane
    static constexpr int kLoadsC = (kC / kVecC + 63) / 64;
    // every lane loads and stores whole vectors: the parts are padded to
    // multiples of 64 loads
    static constexpr int kColOff = kLoadsV * 64 * kVecV;
    static constexpr int kStageWords = kColOff + kLoadsC * 64 * kVecC;
    // staging one pass ahead keeps the staged words live across the pass
    static constexpr bool kAhead = kLoadsV * kVecV + kLoadsC * kVecC <= 16;
};

// The batched solver stages the values only (its columns follow from the
// lattice): the value part of Shape.
template <typename T, int R>
struct ValShape : Shape<T, R> {
    using B = Shape<T, R>;
    static constexpr int kStageWords = B::kColOff;
    static constexpr bool kAhead = B::kLoadsV * B::kVecV <= 16;
};

// Byte offsets, within a block of rows of R complex numbers of kCB bytes, of
// the 13 rows that row `row` gathers (site n = row / 4, orbital o = row % 4),
// in the lattice builder's slot order, plus the lane's part lp of a row.  A
// neighbour beyond an open side is taken as if the side were periodic: its
// two slots hold exact zeros, so any finite row serves, and the wrapped site
// is always a valid row.  That keeps the computation free of per-slot
// selects: per axis and direction one compare, one select and two adds.
template <int R, unsigned kCB>
__host__ __device__ inline void gather_offsets(uint32_t row, const BatchInst& d, uint32_t lp,
                                               uint32_t (&off)[kWidth]) {
    constexpr uint32_t RB = R * kCB;     // bytes per block row
    constexpr uint32_t SB = 4 * RB;      // bytes per site
    const uint32_t n = row >> 2, o = row & 3u;
    const uint32_t Lx = static_cast<uint32_t>(d.L[0]), Ly = static_cast<uint32_t>(d.L[1]);
    const uint32_t Lz = static_cast<uint32_t>(d.L[2]);
    const uint32_t sxy = Lx * Ly;
    const uint32_t q = d.by_lx.div(n);          // n / Lx
    const uint32_t z = d.by_lxy.div(n);         // n / (Lx Ly)
    const uint32_t x = n - q * Lx, y = q - z * Ly;
    const uint32_t so = o * RB + lp;            // same orbital
    const uint32_t sp = (o ^ 3u) * RB + lp;     // partner orbital, x and y
    const uint32_t sz = (o ^ 2u) * RB + lp;     // partner orbital, z
    const uint32_t m[6] = {x > 0 ? n - 1 : n + (Lx - 1),         x + 1 < Lx ? n + 1 : n - (Lx - 1),
                           y > 0 ? n - Lx : n + (Ly - 1) * Lx,   y + 1 < Ly ? n + Lx : n - (Ly - 1) * Lx,
                           z > 0 ? n - sxy : n + (Lz - 1) * sxy, z + 1 < Lz ? n + sxy : n - (Lz - 1) * sxy};
    off[0] = n * SB + so;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const uint32_t base = m[k] * SB;
        off[1 + 2 * k] = base + so;
        off[2 + 2 * k] = base + (k < 4 ? sp : sz);
    }
}

// Order in which the passes of a sweep visit a lattice's rows (site n =
// x + Lx (y + Ly z), rows 4n .. 4n + 3).  The lattice is cut into blocks of
// `lines` consecutive y-lines; blocks are walked one after the other, each
// plane by plane, so that the rows a pass gathers for its z neighbours were
// touched one block-plane earlier (a few lines of the lattice instead of a
// whole plane).  A block-plane is a contiguous row range; passes cover it in
// pieces of rpw rows, the last piece possibly shorter.  lines >= Ly (or 0)
// is the natural row order, one plane at a time.  This random-access form
// defines the order (and is what the host check compares against); the
// kernels walk it incrementally with SlabWalk below.
struct Slabs {
    int64_t plane_rows = 0, line_rows = 0;
    int64_t pf = 0, pl = 0;          // passes per block-plane: full block, last block
    int64_t nfull = 0, npass = 0;    // passes in the full blocks, in total
    int64_t rows_full = 0, rows_last = 0;
    int Lz = 1, lines = 1, nblk = 0, rpw = 1;

    __host__ __device__ void init(int Lx, int Ly, int Lz_, int lines_, int rpw_) {
        Lz = Lz_;
        rpw = rpw_;
        lines = (lines_ <= 0 || lines_ > Ly) ? Ly : lines_;
        line_rows = 4 * static_cast<int64_t>(Lx);
        plane_rows = line_rows * Ly;
        nblk = Ly / lines;
        rows_full = line_rows * lines;
        rows_last = line_rows * (Ly - nblk * lines);
        pf = (rows_full + rpw - 1) / rpw;
        pl = (rows_last + rpw - 1) / rpw;
        nfull = static_cast<int64_t>(nblk) * Lz * pf;
        npass = nfull + static_cast<int64_t>(Lz) * pl;
    }
    // first row of pass p and its number of rows (0 rows, first row past the
    // lattice, for p >= npass)
    __host__ __device__ void pass(int64_t p, int64_t& row0, int64_t& nrows) const {
        if (p >= npass) {
            row0 = plane_rows * Lz;
            nrows = 0;
            return;
        }
        int64_t b, r, per_plane, rows_blk;
        if (p < nfull) {
            per_plane = pf;
            rows_blk = rows_full;
            b = p / (static_cast<int64_t>(Lz) * pf);
            r = p - b * Lz * pf;
        } else {
            per_plane = pl;
            rows_blk = rows_last;
            b = nblk;
            r = p - nfull;
        }
        const int64_t z = r / per_plane, o = r - z * per_plane;
        row0 = z * plane_rows + b * rows_full + o * rpw;
        const int64_t left = rows_blk - o * rpw;
        nrows = left < rpw ? left : rpw;
    }
};

// Slab order walked incrementally by one wave: its passes are p0, p0 +
// stride, p0 + 2 stride, ...; the pass index is kept as mixed-radix digits
// (block, plane, piece) and the stride is added digit by digit with carries,
// so a pass costs a few scalar operations.
struct SlabWalk {
    SlabGeom g;   // kpm::SlabGeom
    uint32_t sb = 0, sz = 0, so = 0;   // stride as digits
    uint32_t b = 0, z = 0, o = 0;      // current pass as digits (b >= nblk: past the end)

    __host__ __device__ void digits(int64_t n, uint32_t& db, uint32_t& dz, uint32_t& d0) const {
        if (n >= g.npass) {
            db = g.nblk;
            dz = d0 = 0;
            return;
        }
        const uint32_t u = static_cast<uint32_t>(n);
        db = g.per_blk.div(u);
        const uint32_t r = u - db * (g.Lz * g.pf);
        dz = g.per_piece.div(r);
        d0 = r - dz * g.pf;
    }
    __host__ __device__ void init(const SlabGeom& geom, int64_t p0, int64_t stride) {
        g = geom;
        digits(p0, b, z, o);
        digits(stride, sb, sz, so);
    }
    // first row and row count of the current pass (0 rows past the end)
    __host__ __device__ void cur(int64_t& row0, int64_t& nr) const {
        if (b >= g.nblk) {
            row0 = g.nrows;
            nr = 0;
            return;
        }
        row0 = static_cast<int64_t>(z) * g.plane_rows + static_cast<int64_t>(b) * g.rows_full +
               static_cast<int64_t>(o) * g.rpw;
        const uint32_t left = g.rows_full - o * g.rpw;
        nr = left < g.rpw ? left : g.rpw;
    }
    __host__ __device__ void advance() {
        if (b >= g.nblk) return;
        o += so;
        uint32_t c = o >= g.pf ? 1u : 0u;
        o -= c * g.pf;
        z += sz + c;
        c = z >= g.Lz ? 1u : 0u;
        z -= c * g.Lz;
        b += sb + c;
    }
};

// Natural row order with the same interface: pass p covers rows p * rpw ..
// nr is always rpw: rows past the end lie outside every buffer descriptor
// (loads read 0, stores are dropped) and the kernels mask their scalar
// products with row < N, so the pass size stays a compile-time constant.
struct RowWalk {
    int64_t p = 0, stride = 1, npass = 0, nrows = 0;
    int rpw = 1;
    __host__ __device__ void init(int64_t n, int rpw_, int64_t p0, int64_t stride_) {
        nrows = n;
        rpw = rpw_;
        npass = (n + rpw - 1) / rpw;
        p = p0;
        stride = stride_;
    }
    __host__ __device__ void cur(int64_t& row0, int64_t& nr) const {
        row0 = p < npass ? p * rpw : nrows;
        nr = rpw;
    }
    __host__ __device__ void advance() { p += stride; }
};

// Pass order of a kernel: the slab order (SLAB) or the natural one.
template <bool SLAB> struct PassOrder;
template <> struct PassOrder<true> {
    SlabWalk w;
    __device__ void init(int64_t, const SlabGeom& g, int, int64_t p0, int64_t stride) { w.init(g, p0, stride); }
    __device__ int64_t npass() const { return w.g.npass; }
    __device__ void cur(int64_t& row0, int64_t& nr) const { w.cur(row0, nr); }
    __device__ void advance() { w.advance(); }
};
template <> struct PassOrder<false> {
    RowWalk w;
    __device__ void init(int64_t n, const SlabGeom&, int rpw, int64_t p0, int64_t stride) { w.init(n, rpw, p0, stride); }
    __device__ int64_t npass() const { return w.npass; }
    __device__ void cur(int64_t& row0, int64_t& nr) const { w.cur(row0, nr); }
    __device__ void advance() { w.advance(); }
};

// Work item k of the pencil order (TileGeom) for die `die`, whose items are
// k_lo .. : tile origin (x0, y0), extent ex x ey sites, planes [z0, z1).
__host__ __device__ inline void tile_item(const TileGeom& g, uint32_t k, uint32_t k_lo, uint32_t die, uint32_t& x0,
                                          uint32_t& y0, uint32_t& ex, uint32_t& ey, uint32_t& z0, uint32_t& z1) {
    uint32_t tx, ty, piece;
    if (g.bw) {
        const uint32_t tpd = g.bw * g.bh, i = k - k_lo, t = i % tpd;
        piece = i / tpd;
        tx = (die % 2) * g.bw + t % g.bw;
        ty = (die / 2) * g.bh + t / g.bw;
    } else {
        const uint32_t nt = g.ntiles(), t = k % nt;
        piece = k / nt;
        tx = t % g.ntx;
        ty = t / g.ntx;
    }
    z0 = piece * g.Lz / g.npieces;
    z1 = (piece + 1) * g.Lz / g.npieces;
    x0 = tx * g.side;
    y0 = ty * g.side;
    ex = g.Lx - x0 < g.side ? g.Lx - x0 : g.side;
    ey = g.Ly - y0 < g.side ? g.Ly - y0 : g.side;
}

// Pencil order walked by one wave of the staged-gather sweep (TileGeom):
// workgroup `block` of `grid` works for die block % dies and takes that
// die's items k, k + per, ... (per = grid / dies workgroups per die); inside
// an item the waves of the workgroup take its passes wave, wave + waves, ...
// The pass is kept as digits (plane, line, piece of line) and the stride is
// added digit by digit; an item a wave has no pass in is skipped.
struct TileWalk {
    TileGeom g;
    uint32_t die = 0, X = 1, k = 0, k_lo = 0, k_hi = 0, per = 1, first = 0, step = 1;
    uint32_t nz = 0, ey = 0, ppl = 1;       // planes, lines, passes per line of the item
    uint32_t sz = 0, sl = 0, so = 0;        // stride as digits
    uint32_t z = 0, line = 0, o = 0;        // current pass as digits
    int64_t base = 0;                       // first row of the item (plane z0, line y0, site x0)

    // set up item k; false past the die's last item
    __host__ __device__ bool load() {
        if (k >= k_hi) return false;
        uint32_t x0, y0, ex, z0, z1;
        tile_item(g, k, k_lo, die, x0, y0, ex, ey, z0, z1);
        nz = z1 - z0;
        ppl = 4 * ex / g.rpw;
        const uint32_t ppp = ey * ppl;
        sz = step / ppp;
        sl = (step % ppp) / ppl;
        so = (step % ppp) % ppl;
        z = first / ppp;
        line = (first % ppp) / ppl;
        o = (first % ppp) % ppl;
        base = static_cast<int64_t>(z0) * g.plane_rows + static_cast<int64_t>(y0) * g.line_rows + 4 * x0;
        return true;
    }
    // move to the first item (from k on) that has a pass for this wave
    __host__ __device__ void settle() {
        while (load() && z >= nz) k += per;
    }
    __host__ __device__ void init(const TileGeom& geom, uint32_t block, uint32_t grid, uint32_t dies,
                                  uint32_t wave, uint32_t waves) {
        g = geom;
        X = (dies > 1 && grid % dies == 0) ? dies : 1;
        if (X != 8) g.bw = g.bh = 0;
        die = block % X;
        per = grid / X;
        const uint32_t n = g.nitems();
        k_lo = static_cast<uint32_t>(static_cast<uint64_t>(n) * die / X);
        k_hi = static_cast<uint32_t>(static_cast<uint64_t>(n) * (die + 1) / X);
        k = k_lo + block / X;
        first = wave;
        step = waves;
        settle();
    }
    __host__ __device__ void cur(int64_t& row0, int64_t& nr) const {
        if (k >= k_hi) {
            row0 = g.nrows;
            nr = 0;
            return;
        }
        row0 = base + static_cast<int64_t>(z) * g.plane_rows + static_cast<int64_t>(line) * g.line_rows + o * g.rpw;
        nr = g.rpw;
    }
    __host__ __device__ void advance() {
        if (k >= k_hi) return;
        o += so;
        uint32_t c = o >= ppl ? 1u : 0u;
        o -= c * ppl;
        line += sl + c;
        c = line >= ey ? 1u : 0u;
        line -= c * ey;
        z += sz + c;
        if (z >= nz) {
            k += per;
            settle();
        }
    }
};

template <typename T, int R, int WAVES>
constexpr int lds_bytes() {
    using S = ValShape<T, R>;
    return WAVES * (S::kAhead ? 2 : 1) * S::kStageWords * 4 + 2 * WAVES * 3 * R * 8 + 16;
}

template <typename T, int R, int WAVES>
constexpr bool instantiable() {
    return lds_bytes<T, R, WAVES>() <= kLdsMax && WAVES <= kMaxWaves<T>;
}

template <int VW> struct Words;
template <> struct Words<1> {
    using type = int;
    template <int AUX = 0> static __device__ type load(__amdgpu_buffer_rsrc_t rs, unsigned off) {
        return static_cast<int>(__builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, AUX));
    }
    template <int AUX = 0> static __device__ void store(type x, __amdgpu_buffer_rsrc_t rs, unsigned off) {
        __builtin_amdgcn_raw_buffer_store_b32(static_cast<unsigned>(x), rs, off, 0, AUX);
    }
};
template <> struct Words<2> {
    using type = int __attribute__((ext_vector_type(2)));
    template <int AUX = 0> static __device__ type load(__amdgpu_buffer_rsrc_t rs, unsigned off) {
        return __builtin_bit_cast(type, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, AUX));
    }
    template <int AUX = 0> static __device__ void store(type x, __amdgpu_buffer_rsrc_t rs, unsigned off) {
        __builtin_amdgcn_raw_buffer_store_b64(x, rs, off, 0, AUX);
    }
};
template <> struct Words<4> {
    using type = int __attribute__((ext_vector_type(4)));
    template <int AUX = 0> static __device__ type load(__amdgpu_buffer_rsrc_t rs, unsigned off) {
        return __builtin_bit_cast(type, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, AUX));
    }
    template <int AUX = 0> static __device__ void store(type x, __amdgpu_buffer_rsrc_t rs, unsigned off) {
        __builtin_amdgcn_raw_buffer_store_b128(x, rs, off, 0, AUX);
    }
};

// Raw buffer resource over `bytes` bytes at p (at most 4 GiB - 1).
__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* p, uint64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, static_cast<int>(bytes), 0x00020000);
}

// CPL complex numbers of storage type T as (re, im, re, im, ...).
template <typename T, int CPL>
struct Lanes {
    static constexpr int kWords = 2 * CPL * static_cast<int>(sizeof(T)) / 4;
    using W = Words<kWords>;
    using type = T __attribute__((ext_vector_type(2 * CPL)));
    template <int AUX = 0> static __device__ type load(__amdgpu_buffer_rsrc_t rs, unsigned off) {
        return __builtin_bit_cast(type, W::template load<AUX>(rs, off));
    }
    template <int AUX = 0> static __device__ void store(const type& x, __amdgpu_buffer_rsrc_t rs, unsigned off) {
        W::template store<AUX>(__builtin_bit_cast(typename W::type, x), rs, off);
    }
};

// Orders LDS writes of a wave before later LDS reads of other lanes of the
// same wave (the LDS executes one wave's accesses in order; this only stops
// the compiler from moving them).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cache policy of the streams a sweep touches once (matrix rows, old and new
// W): non-temporal at block widths 4..16, so that L2 keeps the V rows that
// neighbouring rows gather again (measured on 64^3: 5-9 % faster there and
// on the batched family; 2-9 % slower at R = 1, 2 and 64, where it stays
// off).  The single-instance sweep uses it only on problems larger than the
// last-level cache; the batched solver always (its instances together
// exceed it).
template <int R>
constexpr int kStream = (R >= 4 && R <= 16) ? 2 : 0;

template <typename T> struct Pair;
template <> struct Pair<float> { using type = float __attribute__((ext_vector_type(2))); };
template <> struct Pair<double> { using type = double __attribute__((ext_vector_type(2))); };

// Waves per SIMD to allocate registers for: kMinWaves<T>, or fewer where
// the workgroup's LDS already limits the workgroups per CU.
template <typename T, int R, int WAVES>
constexpr int min_waves() {
    const int wg_per_cu = kLdsMax / lds_bytes<T, R, WAVES>();
    const int occ = wg_per_cu * WAVES / 4;
    return occ < 1 ? 1 : (occ < kMinWaves<T> ? occ : kMinWaves<T>);
}

template <typename T, int R, int WAVES, bool SLAB>
__global__ void __launch_bounds__(64 * WAVES, (min_waves<T, R, WAVES>()))
batched_kernel(const BatchInst* __restrict__ insts, const int32_t* __restrict__ order, int n_inst,
               int* __restrict__ counter, int* __restrict__ flag, int M, int slab) {
    using S = ValShape<T, R>;
    constexpr int CPL = S::CPL;
    using LV = Lanes<T, CPL>;
    using Cv = typename LV::type;
    using P2 = typename Pair<T>::type;
    using WV = Words<S::kVecV>;
    constexpr int LPR = S::LPR;
    constexpr int RPW = S::RPW;
    constexpr int kVW = S::kValWords;
    constexpr int kBufs = S::kAhead ? 2 : 1;
    constexpr int kWpv = static_cast<int>(sizeof(T)) / 4;   // words per real
    constexpr unsigned kCB = 2 * sizeof(T);                 // bytes per complex
    __shared__ __attribute__((aligned(16))) int stage[WAVES][kBufs][S::kStageWords];
    __shared__ double red[2][WAVES][3][R];
    __shared__ int s_next;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int sub = lane / LPR;          // block row within a pass
    const int cc = lane % LPR;           // the lane's columns: cc * CPL + t, t < CPL
    const int sweeps = M / 2;

    for (int it = 0;; ++it) {
        int idx;
        if (counter) {
            if (threadIdx.x == 0) s_next = atomicAdd(counter, 1);
            __syncthreads();
            idx = s_next;
        } else {
            idx = blockIdx.x + it * static_cast<int>(gridDim.x);
        }
        idx = __builtin_amdgcn_readfirstlane(idx);
        if (idx >= n_inst) break;
        const BatchInst d = insts[order[idx]];
        const int64_t N = d.nrows;
        PassOrder<SLAB> sl0;   // this wave's passes wave, wave + WAVES, ... (every sweep)
        sl0.init(N, d.geom, RPW, wave, WAVES);
        const int64_t npass = sl0.npass();
        const uint64_t vbytes = static_cast<uint64_t>(N) * R * kCB;
        const __amdgpu_buffer_rsrc_t val_rs = rsrc(d.val, static_cast<uint64_t>(N) * kVW * 4);

        // nu_0 -> a: the recurrence overwrites the block holding nu_{k-1}
        {
            const __amdgpu_buffer_rsrc_t src = rsrc(d.v0, vbytes);
            const __amdgpu_buffer_rsrc_t dst = rsrc(d.a, vbytes);
            const unsigned n16 = static_cast<unsigned>((vbytes + 15) / 16);
            for (unsigned i = threadIdx.x; i < n16; i += 64 * WAVES)
                Words<4>::store(Words<4>::load(src, 16 * i), dst, 16 * i);
        }
        // every wave gathers rows of nu_0 that other waves copied: the whole
        // block must be stored before the first sweep reads it
        __syncthreads();

        // matrix values of the pass starting at row r0; lanes past the end of
        // the pass fetch words that are never read
        auto fetch = [&](int64_t r0, typename WV::type* wv) {
            const unsigned pv = static_cast<unsigned>(r0) * (kVW * 4);
#pragma unroll
            for (int i = 0; i < S::kLoadsV; ++i)
                wv[i] = WV::template load<kStream<R>>(val_rs, pv + (lane + 64 * i) * (4 * S::kVecV));
        };
        auto put = [&](int* dst, const typename WV::type* wv) {
#pragma unroll
            for (int i = 0; i < S::kLoadsV; ++i)
                *reinterpret_cast<typename WV::type*>(dst + (lane + 64 * i) * S::kVecV) = wv[i];
        };

        for (int k = 0; k < sweeps; ++k) {
            // k = 0: nu_1 = Htilde nu_0 into b; k >= 1: the block holding
            // nu_{k-1} is overwritten by nu_{k+1} = 2 Htilde nu_k - nu_{k-1}
            const void* V = (k & 1) ? d.b : d.a;
            void* W = (k & 1) ? d.a : d.b;
            const T alpha = static_cast<T>(k == 0 ? d.inv_a : 2.0 * d.inv_a);
            const T beta = static_cast<T>(k == 0 ? -d.shift : -2.0 * d.shift);
            const __amdgpu_buffer_rsrc_t vrs = rsrc(V, vbytes);
            const __amdgpu_buffer_rsrc_t wrs = rsrc(W, vbytes);
            const __amdgpu_buffer_rsrc_t wold_rs = rsrc(W, k == 0 ? 0 : vbytes);   // zeros in sweep 0
            double ae[CPL], aor[CPL], aoi[CPL];
#pragma unroll
            for (int t = 0; t < CPL; ++t) ae[t] = aor[t] = aoi[t] = 0.0;
            typename WV::type wv[S::kLoadsV];
            int buf = 0;
            PassOrder<SLAB> sl = sl0;
            int64_t row0, nr;
            sl.cur(row0, nr);
            if constexpr (S::kAhead) {
                fetch(row0, wv);
                put(stage[wave][0], wv);
            }
            for (int64_t q = wave; q < npass; q += WAVES) {
                if constexpr (!S::kAhead) {
                    wave_sync();   // every lane has read the slot before it is refilled
                    fetch(row0, wv);
                    put(stage[wave][0], wv);
                }
                wave_sync();
                const int* st = stage[wave][buf];
                const int64_t row = row0 + sub;
                // gathers of the 13 neighbour rows (a lane past the end of the
                // pass or of the lattice takes those of the last row)
                uint32_t goff[kWidth];
                gather_offsets<R, kCB>(static_cast<uint32_t>(row < N ? row : N - 1), d, cc * CPL * kCB, goff);
                Cv v[kWidth];
#pragma unroll
                for (int j = 0; j < kWidth; ++j) v[j] = LV::load(vrs, goff[j]);
                // slab order: rows past the end of a pass belong to other
                // passes and get an offset past the block (the old-W load
                // reads zero, the store is dropped); natural order: only rows
                // past N are inactive, and their offsets are past the block
                bool act;
                unsigned off;
                if constexpr (SLAB) {
                    act = sub < nr;
                    off = act ? static_cast<unsigned>(row * R + cc * CPL) * kCB : 0xFFFFFFF0u;
                } else {
                    act = row < N;
                    off = static_cast<unsigned>(row * R + cc * CPL) * kCB;
                }
                const Cv wo = LV::template load<kStream<R>>(wold_rs, off);
                // matrix rows of this wave's next pass (zeros past the end)
                int64_t row0n, nrn;
                sl.advance();
                sl.cur(row0n, nrn);
                if constexpr (S::kAhead) fetch(row0n, wv);
                const int* sv = st + sub * kVW;
                Cv acc;
#pragma unroll
                for (int e = 0; e < 2 * CPL; ++e) acc[e] = T(0);
#pragma unroll
                for (int j = 0; j < kWidth; ++j) {
                    // (re, im) of entry j: one 8- or 16-byte LDS read
                    const P2 h = *reinterpret_cast<const P2*>(sv + 2 * j * kWpv);
#pragma unroll
                    for (int t = 0; t < CPL; ++t) {
                        acc[2 * t] = fma(h.x, v[j][2 * t], acc[2 * t]);
                        acc[2 * t] = fma(-h.y, v[j][2 * t + 1], acc[2 * t]);
                        acc[2 * t + 1] = fma(h.x, v[j][2 * t + 1], acc[2 * t + 1]);
                        acc[2 * t + 1] = fma(h.y, v[j][2 * t], acc[2 * t + 1]);
                    }
                }
                // slot 0 is the diagonal: v[0] is V of this row
                Cv wn;
#pragma unroll
                for (int e = 0; e < 2 * CPL; ++e) wn[e] = fma(alpha, acc[e], beta * v[0][e]) - wo[e];
                // rows past N: the store is dropped, the products masked
                LV::template store<kStream<R>>(wn, wrs, off);
#pragma unroll
                for (int t = 0; t < CPL; ++t) {
                    const double vr = act ? static_cast<double>(v[0][2 * t]) : 0.0;
                    const double vi = act ? static_cast<double>(v[0][2 * t + 1]) : 0.0;
                    const double wr = wn[2 * t], wi = wn[2 * t + 1];
                    ae[t] = fma(vr, vr, fma(vi, vi, ae[t]));
                    aor[t] = fma(wr, vr, fma(wi, vi, aor[t]));
                    aoi[t] = fma(wr, vi, fma(-wi, vr, aoi[t]));
                }
                if constexpr (S::kAhead) {
                    put(stage[wave][buf ^ 1], wv);
                    buf ^= 1;
                }
                row0 = row0n;
                nr = nrn;
            }
            // lanes cc, cc + LPR, ... of a wave hold the same columns
#pragma unroll
            for (int t = 0; t < CPL; ++t) {
#pragma unroll
                for (int o = LPR; o < 64; o <<= 1) {
                    ae[t] += __shfl_xor(ae[t], o);
                    aor[t] += __shfl_xor(aor[t], o);
                    aoi[t] += __shfl_xor(aoi[t], o);
                }
                if (sub == 0) {
                    red[k & 1][wave][0][cc * CPL + t] = ae[t];
                    red[k & 1][wave][1][cc * CPL + t] = aor[t];
                    red[k & 1][wave][2][cc * CPL + t] = aoi[t];
                }
            }
            // all of W is written (it is the next sweep's V) and red is full
            __syncthreads();
            if (threadIdx.x < 3 * R) {
                const int qq = threadIdx.x / R, r = threadIdx.x % R;
                double sum = 0.0;
#pragma unroll
                for (int wvi = 0; wvi < WAVES; ++wvi) sum += red[k & 1][wvi][qq][r];
                d.eta[(static_cast<int64_t>(k) * 3 + qq) * R + r] = sum;
            }
        }
        __syncthreads();   // eta of every sweep is visible to the workgroup
        // mu_0 = eta_0, mu_1 = Re eta_1, mu_{2m} = 2 eta_{2m} - mu_0,
        // mu_{2m+1} = 2 Re eta_{2m+1} - mu_1
        int bad = 0;
        for (int i = threadIdx.x; i < R * M; i += 64 * WAVES) {
            const int r = i / M, n = i % M;
            const double mu0 = d.eta[r];
            const double ref = d.eta[(n & 1) * R + r];
            const double x = 2.0 * d.eta[(static_cast<int64_t>(n >> 1) * 3 + (n & 1)) * R + r] - ref;
            d.mu[i] = x;
            if (!isfinite(x) || fabs(x) > mu0 * (1.0 + 1e-6) + 1e-300) bad = 1;
        }
        if (bad) flag[0] = 1;
        __syncthreads();   // the grab slot and LDS are free for the next instance
    }
}

template <typename T, int R, int WAVES>
hipError_t launch_waves(const BatchArgs& a, hipStream_t s) {
    if constexpr (instantiable<T, R, WAVES>()) {
        int* counter = a.dynamic ? a.counter : nullptr;
        if (a.slab > 0)
            batched_kernel<T, R, WAVES, true><<<a.grid, 64 * WAVES, 0, s>>>(a.inst, a.order, a.n_inst, counter,
                                                                          a.flag, a.M, a.slab);
        else
            batched_kernel<T, R, WAVES, false><<<a.grid, 64 * WAVES, 0, s>>>(a.inst, a.order, a.n_inst, counter,
                                                                           a.flag, a.M, 0);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

template <typename T, int R>
hipError_t launch_r(const BatchArgs& a, hipStream_t s) {
    switch (a.waves) {
    case 4: return launch_waves<T, R, 4>(a, s);
    case 8: return launch_waves<T, R, 8>(a, s);
    case 16: return launch_waves<T, R, 16>(a, s);
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_dtype(int R, const BatchArgs& a, hipStream_t s) {
    switch (R) {
    case 1: return launch_r<T, 1>(a, s);
    case 2: return launch_r<T, 2>(a, s);
    case 4: return launch_r<T, 4>(a, s);
    case 8: return launch_r<T, 8>(a, s);
    case 16: return launch_r<T, 16>(a, s);
    case 32: return launch_r<T, 32>(a, s);
    case 64: return launch_r<T, 64>(a, s);
    }
    return hipErrorInvalidValue;
}

// Largest workgroup (4, 8 or 16 waves) that can be launched for this R, or
// 0 if none.
template <typename T, int R>
int max_waves_r() {
    return instantiable<T, R, 16>() ? 16 : instantiable<T, R, 8>() ? 8 : instantiable<T, R, 4>() ? 4 : 0;
}

template <typename T>
int max_waves(int R) {
    switch (R) {
    case 1: return max_waves_r<T, 1>();
    case 2: return max_waves_r<T, 2>();
    case 4: return max_waves_r<T, 4>();
    case 8: return max_waves_r<T, 8>();
    case 16: return max_waves_r<T, 16>();
    case 32: return max_waves_r<T, 32>();
    case 64: return max_waves_r<T, 64>();
    }
    return 0;
}

}  // namespace batch
}  // namespace kpm
