// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/kpm.h"

namespace kpm {

// Stored entries per matrix row: the diagonal plus two entries per hopping
// block (same orbital through Gamma^1, partner orbital through Gamma^{j+1})
// for the six neighbours n -/+ e_j.
constexpr int kWidth = 13;

// Number of accelerator complex dies (XCDs) the dispatcher deals workgroups
// to round-robin on gfx950.
constexpr int kXcds = 8;

// Buffers of the calls on one stream.  Calls enqueued on one stream run in
// order, so they may reuse these; calls on different streams get different
// sets (see kpm_hamiltonian::ws).
struct Workspace {
    void* vbuf[2] = {nullptr, nullptr};   // two [N][R] blocks
    size_t vbytes = 0;
    double* partials = nullptr;            // [slots][grid][3][R]
    int* queue = nullptr;                  // [slots][kXcds] tile counters
    size_t qbytes = 0;
    size_t pbytes = 0;
    double* eta = nullptr;                 // [M][R][2]
    size_t etabytes = 0;
    double* mu = nullptr;                  // [R][M] device moments for callers with host mu
    size_t mubytes = 0;
    int* flag = nullptr;                   // spectrum check flag (device)
    int* flag_host = nullptr;              // pinned mirror
    void* naive[3] = {nullptr, nullptr, nullptr};   // v, w, u of the naive algorithm ([N] each)
    size_t naive_bytes = 0;
    double* dot_part = nullptr;            // [naive_dot_partials()][2] scalar-product partials
    double* lanczos = nullptr;             // alpha, beta and scalars of the Lanczos bounds
    size_t lanczos_bytes = 0;
    // HIP graph of the kpm_moments launch sequence (captured on a private
    // stream, replayed on this workspace's stream) and what it was made for
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<unsigned char> graph_key;
};


// SELL-C-sigma storage of an imported matrix (kpm_import_csr): sorted
// position p holds row perm[p] (no perm: p itself) and lies in chunk p / C,
// stored column-major from entry start[p / C], width[p / C] entries deep.
struct SellStore {
    int C = 0;                      // chunk height (a power of two, 1..64); 0: not SELL storage
    int clog = 0;                   // log2 C
    int sigma = 1;                  // sorting window in rows (1: unsorted)
    int64_t nchunks = 0;
    int64_t stored = 0;             // stored entries, padding included
    int64_t nnz = 0;                // entries of the imported matrix
    int64_t* start = nullptr;       // device [nchunks + 1]
    int32_t* width = nullptr;       // device [nchunks]
    int32_t* perm = nullptr;        // device [N], or nullptr when sigma == 1
    std::vector<int32_t> len;       // host row lengths by sorted position (for export)
    std::vector<int32_t> perm_host; // host copy of perm (empty when sigma == 1)
    std::vector<int64_t> start_host;
};
}  // namespace kpm

struct kpm_hamiltonian {
    int dtype = KPM_C128;           // storage precision of val and of vector blocks
    int64_t nrows = 0;              // N
    int width = kpm::kWidth;        // slots per row (row-major, diagonal first); SELL: longest row
    void* val = nullptr;            // [N][width] complex (re, im) in dtype; SELL: [stored]
    int32_t* col = nullptr;         // [N][width]; SELL: [stored]
    kpm::SellStore sell;            // SELL-C-sigma storage (sell.C > 0) instead of the lattice layout
    int L[3] = {0, 0, 0};           // lattice sides
    int periodic[3] = {0, 0, 0};
    double a = 1.0, b = 0.0;        // Htilde = (H - b)/a
    double emin = 0.0, emax = 0.0;  // Gershgorin interval
    int device = 0;
    // Guards the two maps below; buffers are only ever added to them (and
    // released by kpm_destroy_hamiltonian), so a pointer taken under the lock
    // stays valid while another thread adds entries.
    std::mutex lock;
    std::map<hipStream_t, kpm::Workspace*> ws;   // per caller stream
    std::map<int, int32_t*> sched;              // device [N/4] site schedule per pencil side
};

namespace kpm {

void set_error(const std::string& msg);

// ---- device launchers (implemented in the .hip files) ----

// Builds the row-major slot arrays and per-block Gershgorin bounds.
hipError_t launch_build_ti(int Lx, int Ly, int Lz, const int* periodic, double t,
                           const double* pot_dev, int dtype, void* val, int32_t* col,
                           double* block_bounds /* [nblocks][2] */, int nblocks,
                           double* bounds_out /* [2] */, hipStream_t s);
int build_blocks(int64_t nrows);

struct SweepArgs {
    const void* val;
    const int32_t* col;
    int64_t nrows;
    const void* V;
    void* W;
    const int32_t* sched;   // sites in processing order, or nullptr
    double alpha, beta, gamma;
    double* partials;   // this sweep's [grid][3][R] slot (FULL only)
    int grid;           // workgroups
    int* queue = nullptr;   // this sweep's [kXcds] tile counters (zero), or nullptr
    int xcd_ways = 1;   // filled by launch_sweep from the tuning
    int chunk = 1;
    int prefetch = 1;
    int stream = 0;
    int L[3] = {0, 0, 0};   // lattice sides of H (rows 4 (x + Lx (y + Ly z)) + o)
    int slab = 0;           // staged-gather sweep: y-lines per block of the pass order
    int tile = 0;           // staged-gather sweep: tile side of the pencil order (0: off)
    int window = 0;         // staged-gather sweep: run its LDS-window variant (on a lattice)
    int order = 0;          // window sweep: 2 = no die mapping of its tiles (tuning tile_order)
};

// Fused sweep over SELL-C-sigma storage (kpm_sell.hip).
struct SellArgs {
    const void* val;
    const int32_t* col;
    const int64_t* start;
    const int32_t* width;
    const int32_t* perm;    // or nullptr (no sorting)
    int64_t nrows;
    int64_t stored;
    int clog;
    const void* V;
    void* W;
    double alpha, beta, gamma;
    double* partials;       // this sweep's [grid][3][R] slot (FULL only)
    int grid;
};
hipError_t launch_sell(int dtype, int R, int variant, const SellArgs& a, hipStream_t s);
int sell_grid(int dtype, int R, int64_t nrows);
int sell_rows_per_pass(int dtype, int R);
// Per-block Gershgorin bounds of SELL storage, then their reduction into
// bounds_out[2] (block_bounds holds build_blocks(nrows) pairs).
hipError_t launch_sell_bounds(int dtype, const void* val, const int32_t* col, const int64_t* start,
                              const int32_t* width, const int32_t* perm, int64_t nrows, int clog,
                              double* block_bounds, double* bounds_out, hipStream_t s);

// Cache-blocked sweep for the library's lattice Hamiltonians at R = 32 k.
struct LatticeArgs {
    const void* val;
    const void* V;
    void* W;
    double alpha, beta, gamma;
    double* partials;   // this sweep's [grid][3][R] slot (FULL only)
    int L[3];
    int periodic[3];
    int grid;
    int prefetch;       // matrix rows through one vector load per site (a step ahead)
    int stream;         // non-temporal hint: bit 0 old-W loads, bit 1 new-W stores
    int order;          // tiles to dies: 0 2-D blocks, 1 runs of tile rows, 2 none
    int R;              // block width, a multiple of 32
};
bool lattice_supported(const kpm_hamiltonian* H, int R);
int lattice_tiles(const kpm_hamiltonian* H);
int lattice_grid(const kpm_hamiltonian* H);
// z-pieces per pencil the lattice sweep cuts its pencils into at this grid
int lattice_pieces(const kpm_hamiltonian* H, int R, int grid, int prefetch);
hipError_t launch_lattice(int dtype, int variant, const LatticeArgs& a, hipStream_t s);

// Unsigned 32-bit division by a divisor fixed on the host: multiply-high by
// a rounded-up reciprocal (the round-up method of Granlund and Montgomery),
// exact for every 32-bit dividend.  The reciprocal is computed on the host,
// so the kernels only multiply (scalar instructions); a division by a
// run-time value would be expanded on the vector unit.
struct FastDiv {
    uint32_t d = 1, m = 0, s = 0;
    void init(uint32_t d_) {   // host
        d = d_ ? d_ : 1;
        m = 0;
        s = 0;
        if (d == 1) return;
        uint32_t l = 0;
        while ((1ull << l) < d) ++l;                       // ceil(log2 d), d >= 2
        m = static_cast<uint32_t>(((1ull << 32) * ((1ull << l) - d)) / d + 1);
        s = l - 1;
    }
    __host__ __device__ uint32_t div(uint32_t n) const {
        if (d == 1) return n;
#if defined(__HIP_DEVICE_COMPILE__)
        const uint32_t t = __umulhi(n, m);
#else
        const uint32_t t = static_cast<uint32_t>((static_cast<uint64_t>(n) * m) >> 32);
#endif
        return (t + ((n - t) >> 1)) >> s;
    }
};

// Geometry of the slab order of one lattice, built on the host: blocks of
// `lines` y-lines (the largest divisor of Ly not above the request, so all
// blocks are whole), each walked plane by plane in pieces of rpw rows.
struct SlabGeom {
    uint32_t pf = 1, Lz = 1, nblk = 0, rpw = 1, rows_full = 0, plane_rows = 0;
    FastDiv per_blk, per_piece;   // Lz * pf, pf
    int64_t npass = 0, nrows = 0;

    static SlabGeom make(int Lx, int Ly, int Lz, int lines, int rpw) {   // host
        SlabGeom g;
        if (lines <= 0 || lines > Ly) lines = Ly;
        while (Ly % lines) --lines;
        g.Lz = static_cast<uint32_t>(Lz);
        g.rpw = static_cast<uint32_t>(rpw);
        const uint32_t line_rows = 4u * static_cast<uint32_t>(Lx);
        g.plane_rows = line_rows * static_cast<uint32_t>(Ly);
        g.rows_full = line_rows * static_cast<uint32_t>(lines);
        g.nblk = static_cast<uint32_t>(Ly / lines);
        g.pf = (g.rows_full + g.rpw - 1) / g.rpw;
        g.npass = static_cast<int64_t>(g.nblk) * g.Lz * g.pf;
        g.nrows = static_cast<int64_t>(g.plane_rows) * g.Lz;
        g.per_blk.init(g.Lz * g.pf);
        g.per_piece.init(g.pf);
        return g;
    }
};

// Geometry of the pencil order of one lattice (staged-gather sweep), built
// on the host.  The x-y plane is cut into tiles of side x side sites (tiles
// at the lattice edge may be narrower), and each tile's column of sites into
// npieces runs of consecutive z-planes; a work item is one run of one tile,
// walked plane by plane, line by line, in passes of rpw rows (rpw divides
// the 4 rows of a site, so no pass straddles two lines).  Items go to the
// dies as 2-D blocks of bw x bh tiles where the tile grid splits that way
// (most rows a tile gathers across its edge then belong to tiles whose
// planes the same L2 holds), else as runs of consecutive items.
struct TileGeom {
    uint32_t Lx = 1, Ly = 1, Lz = 1, side = 1, ntx = 1, nty = 1, npieces = 1, rpw = 1;
    uint32_t bw = 0, bh = 0;
    uint32_t dies = 1;                  // dies the items are split over (1: no die mapping)
    uint32_t line_rows = 0, plane_rows = 0;
    int64_t nrows = 0;

    __host__ __device__ uint32_t ntiles() const { return ntx * nty; }
    __host__ __device__ uint32_t nitems() const { return ntx * nty * npieces; }

    // npieces: enough items for `grid` workgroups, at least 4 planes per run
    static TileGeom make(int Lx, int Ly, int Lz, int side, int rpw, int grid, int dies) {   // host
        TileGeom g;
        g.Lx = static_cast<uint32_t>(Lx);
        g.Ly = static_cast<uint32_t>(Ly);
        g.Lz = static_cast<uint32_t>(Lz);
        const int s = side < 1 ? 1 : side;
        g.side = static_cast<uint32_t>(s);
        g.ntx = static_cast<uint32_t>((Lx + s - 1) / s);
        g.nty = static_cast<uint32_t>((Ly + s - 1) / s);
        g.rpw = static_cast<uint32_t>(rpw);
        const uint32_t nt = g.ntiles();
        uint32_t np = grid > 0 ? (static_cast<uint32_t>(grid) + nt - 1) / nt : 1;
        const uint32_t cap = Lz >= 8 ? static_cast<uint32_t>(Lz / 4) : 1;
        g.npieces = np < 1 ? 1 : (np > cap ? cap : np);
        g.dies = dies > 1 ? static_cast<uint32_t>(dies) : 1u;
        if (dies == 8 && g.ntx % 2 == 0 && g.nty % 4 == 0) {
            g.bw = g.ntx / 2;
            g.bh = g.nty / 4;
        }
        g.line_rows = 4u * g.Lx;
        g.plane_rows = g.line_rows * g.Ly;
        g.nrows = static_cast<int64_t>(g.plane_rows) * g.Lz;
        return g;
    }
};

// One instance of the batched solver (device-side descriptor).
struct BatchInst {
    const void* val;        // H: [N][kWidth] complex, diagonal in slot 0 (the builder's slot order:
                            // the columns follow from the row and the lattice, see batched_kernel)
    const void* v0;         // start block [N][R] (read-only)
    void* a;                // work blocks [N][R]
    void* b;
    double* eta;            // [M/2][3][R]: <v|v>, Re <w|v>, Im <w|v> per sweep
    double* mu;             // [R][M] output
    int64_t nrows;          // N
    double inv_a;           // 1/a
    double shift;           // b/a
    int32_t L[3];           // lattice sides (rows 4 (x + Lx (y + Ly z)) + o)
    int32_t pad;
    FastDiv by_lx, by_lxy;  // site index -> (x, y, z): division by Lx and by Lx Ly
    SlabGeom geom;          // slab pass order of this instance (used when the slab tuning is on)
};

// Rows per pass of the batched solver's waves (the slab geometry needs it).
int batched_rows_per_pass(int dtype, int R);

struct BatchArgs {
    const BatchInst* inst;  // [n_inst]
    const int32_t* order;   // [n_inst] processing order (longest first)
    int n_inst;
    int* counter;           // zero before the launch (dynamic mapping)
    int* flag;              // set to 1 when a moment leaves [-mu_0, mu_0]
    int M;
    int grid;
    int waves;              // waves per workgroup: 4, 8 or 16
    int dynamic;
    int slab;               // y-lines per block of the pass order (0: natural order)
};
hipError_t launch_batched(int dtype, int R, const BatchArgs& a, hipStream_t s);
// Largest workgroup (in waves, <= 16) that can run this dtype and R.
int batched_max_waves(int dtype, int R);
int device_cus();

// Sweep tuning.  get_tuning() returns the running call's snapshot (see
// TuningScope) or, outside a call, the process-wide setting; set_tuning
// replaces the process-wide setting (mutex-protected, so calls that run
// meanwhile on other threads keep the snapshot they started with).
kpm_sweep_tuning default_tuning();
kpm_sweep_tuning get_tuning();
void set_tuning(const kpm_sweep_tuning& t);
// For the lifetime of the object, get_tuning() on this thread returns
// *override, or the process-wide setting as it was at construction.
class TuningScope {
public:
    explicit TuningScope(const kpm_sweep_tuning* override);
    ~TuningScope();
    TuningScope(const TuningScope&) = delete;
    TuningScope& operator=(const TuningScope&) = delete;
private:
    kpm_sweep_tuning snap_;
    const kpm_sweep_tuning* prev_;
};
// Validation of a tuning record (KPM_OK or KPM_EINVAL with a message).
kpm_status check_tuning(const kpm_sweep_tuning& t);

// Which generic sweep kernel runs for this dtype / R / N (see kpm_sweep_tuning::gather):
// true = the staged-gather sweep, false = the scalar-operand sweep.
bool use_gather(int dtype, int R, int64_t nrows);
// Grid size (workgroups) of the generic sweep kernel for this dtype / R / N.
// (window: the LDS-window variant of the staged-gather sweep runs)
int sweep_grid(int dtype, int R, int64_t nrows, bool window = false);
hipError_t launch_gather(int dtype, int R, int variant, const SweepArgs& a, hipStream_t s);
int gather_waves(int dtype, int R);
int gather_lds(int dtype, int R);
int gather_window_lds(int dtype, int R);    // 0 where the window sweep does not exist
int gather_window_side(int dtype, int R);   // its tile side in sites (0: none)
hipError_t launch_sweep(int dtype, int R, int variant, const SweepArgs& a, hipStream_t s);
// per-precision instantiations of the sweep kernel (R <= 16 and R >= 32)
hipError_t launch_sweep_c128_small(int R, int variant, const SweepArgs& a, hipStream_t s);
hipError_t launch_sweep_c128_large(int R, int variant, const SweepArgs& a, hipStream_t s);
hipError_t launch_sweep_c64_small(int R, int variant, const SweepArgs& a, hipStream_t s);
hipError_t launch_sweep_c64_large(int R, int variant, const SweepArgs& a, hipStream_t s);

// eta[(sweep0 + s)*2 + q] for s < nslots from partials[s][grid][3][R].
hipError_t launch_reduce_partials(const double* partials, int nslots, int grid, int R,
                                  int sweep0, double* eta, hipStream_t s);
hipError_t launch_eta_to_mu(const double* eta, int R, int M, double* mu, hipStream_t s);
hipError_t launch_zero_ints(int* p, int n, hipStream_t s);
// dst[0 .. bytes) = src[0 .. bytes) (16-byte aligned, bytes a multiple of 8):
// a kernel rather than a copy node, so that it can sit in a captured graph
hipError_t launch_copy16(void* dst, const void* src, size_t bytes, hipStream_t s);
hipError_t launch_check_moments(const double* mu, int R, int M, int* flag, hipStream_t s);
hipError_t launch_dos(const double* mu, int R, int M, int kernel, double kparam, double a,
                      double b, const double* E, int K, double* rho, hipStream_t s);
hipError_t launch_dos_batched(const double* mu, int n_inst, int R, int ld, int M, int kernel, double kparam,
                              const double* a, const double* b, const double* E, int K, int masses,
                              double* rho, hipStream_t s);
// BLAS level-1 kernels of the naive algorithm (n complex elements of the
// given storage type; scalar products in FP64, out = sum conj(x_i) y_i
// through part[naive_dot_partials()][2]); column r of an [n][R] block.
int naive_dot_partials();
// Device address, on the current device, of the library's file-scope array of
// naive_dot_partials() x 2 doubles that kpm_dot_noalloc reduces through
// (resolved on the first call per device, no allocation).
hipError_t dot_scratch(double** out);
hipError_t launch_axpy(int dtype, int64_t n, double alpha, const void* x, void* y, hipStream_t s);
hipError_t launch_scal(int dtype, int64_t n, double alpha, void* x, hipStream_t s);
hipError_t launch_dot(int dtype, int64_t n, const void* x, const void* y, double* part, double* out, hipStream_t s);
hipError_t launch_column(int dtype, int64_t n, int R, int r, const void* V, void* v, hipStream_t s);
// columns c0 .. c0 + G - 1 of an [n][R] block into a contiguous [n][G] block
hipError_t launch_columns(int dtype, int64_t n, int R, int c0, int G, const void* V, void* v, hipStream_t s);
// Lanczos bounds: the recurrence's vector steps with alpha, beta read from
// device memory, and the extreme eigenvalues of the tridiagonal matrix.
int lanczos_max_steps();
hipError_t launch_lanczos_update(int dtype, int64_t n, const double* dot, const double* beta_prev, double* ab,
                                 const void* q, const void* qp, void* w, hipStream_t s);
hipError_t launch_lanczos_normalise(int dtype, int64_t n, const double* nrm, const void* w, void* q, double* beta_out,
                                    hipStream_t s);
hipError_t launch_tridiag_extremes(const double* ab, const double* beta, int k, double* out, hipStream_t s);

// Deterministic start blocks (at most kMaxStartColumns columns): unit
// vectors of given rows; plane waves of given momenta on given orbitals.
constexpr int kMaxStartColumns = 64;
hipError_t launch_site_block(void* V, int64_t N, int R, const int64_t* rows, int dtype, hipStream_t s);
hipError_t launch_plane_wave_block(void* V, const int L[3], int R, const double* k, const int32_t* orb, int dtype,
                                   hipStream_t s);
hipError_t launch_phase_block(void* V, int64_t N, int R, int dtype, uint64_t seed, hipStream_t s);
// Disorder potential V_n = gamma (u_n - 1/2), n < nsite, u_n from the counter
// generator of launch_phase_block under the second key of the seed.
hipError_t launch_potential(double* pot, int64_t nsite, double gamma, uint64_t seed, hipStream_t s);
// STREAM-style copy / triad over `units` 16-byte units (kpm_stream)
hipError_t launch_stream(int kind, int nontemporal, void* c, const void* a, const void* b, double s, int64_t units,
                         int wg_per_cu, hipStream_t st);
hipError_t launch_features(const double* mu, int n_inst, int R, int ld, int n_mom, const float* extra,
                           float* x, hipStream_t s);

}  // namespace kpm
