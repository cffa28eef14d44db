/*
 * kpm.h -- C ABI of the MI355X (gfx950) Kernel Polynomial Method library.
 *
 * The library computes the Chebyshev moments and the density of states (DOS)
 * of the topological-insulator Hamiltonian of Kreutzer et al., "Performance
 * Engineering of the Kernel Polynomial Method on Large-Scale CPU-GPU
 * Systems" (arXiv:1410.5242), with the fused, blocked, augmented sparse
 * matrix times multiple-vector product ("aug_spmmv") of the paper's
 * blocked algorithm (Alg. "kpm_improved_blocked") as its hot path.
 *
 * Conventions shared by every entry point
 *  - Every function returns a kpm_status; KPM_OK (0) means success.  On any
 *    other value kpm_last_error() returns a message for the calling thread.
 *  - "device" pointers are HIP device allocations on the current device;
 *    "host" pointers are ordinary host memory.  The caller owns every buffer
 *    it passes in; the library owns the Hamiltonian handle and its internal
 *    workspaces (released by kpm_destroy_hamiltonian).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on it.  Unless stated otherwise a call returns once the
 *    work is enqueued; device outputs are valid after the stream is
 *    synchronised.
 *  - Complex numbers are stored as interleaved (re, im) pairs of the storage
 *    precision.  A block of R vectors of length N is row-major ("interleaved"):
 *    element (i, r) is complex number i*R + r.
 *  - Scaling: Htilde = (H - b)/a, with b the centre and a the half-width of
 *    an interval containing the spectrum (the paper writes the same map as
 *    a(H - b) with a reciprocal a; this ABI uses the half-width form).
 */
#ifndef KPM_H
#define KPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KPM_OK = 0,
    KPM_EINVAL = -1,     /* invalid argument (null pointer, bad size, odd M, ...) */
    KPM_ENOMEM = -2,     /* device allocation failed or the size is absurd */
    KPM_EDEVICE = -3,    /* a HIP runtime call failed */
    KPM_ENOTSUP = -4,    /* valid request that this library does not implement */
    KPM_ESPECTRUM = -5,  /* moments left [-mu_0, mu_0]: the spectrum is not inside [-1, 1] */
    KPM_EINTERNAL = -6
} kpm_status;

/* Storage precision of H and of the vector blocks.  The moment scalar
 * products and their reductions are always accumulated in FP64. */
typedef enum { KPM_C128 = 0, KPM_C64 = 1 } kpm_dtype;

/* Damping kernel g_n of the DOS reconstruction. */
typedef enum { KPM_JACKSON = 0, KPM_DIRICHLET = 1, KPM_LORENTZ = 2 } kpm_kernel;

/* Sweep variants: the full fused sweep and the two diagnostic reductions of
 * it that the paper uses to split bottlenecks (section "GPU Performance
 * Model"): without the scalar products, and the plain SpMMV Y = H X. */
typedef enum { KPM_FULL = 0, KPM_NODOT = 1, KPM_PLAIN = 2 } kpm_variant;

typedef struct {
    int32_t L[3];            /* lattice sides Lx, Ly, Lz (>= 1) */
    int32_t periodic[3];     /* nonzero: periodic along that axis (side must be >= 3) */
    double t;                /* hopping amplitude */
    double gamma;            /* disorder strength when potential is NULL (>= 0) */
    uint64_t seed;           /* generator seed when potential is NULL */
    const double* potential; /* host [Lx*Ly*Lz] onsite V_n, site n = x + Lx*(y + Ly*z), or NULL:
                                V_n = gamma (u_n - 1/2), u_n = (top 53 bits of SplitMix64 output) / 2^53
                                at counter n, state key + (n + 1) * 0x9E3779B97F4A7C15,
                                key = mix(seed + 2 * 0x9E3779B97F4A7C15) (the second output of
                                SplitMix64 seeded with `seed`; kpm_random_phase_block uses the first) */
    int32_t dtype;           /* kpm_dtype */
    double margin;           /* half-width factor applied to the Gershgorin interval (e.g. 1.01) */
    int32_t fixed_scale;     /* nonzero: use a, b below instead of the Gershgorin bound */
    double a, b;             /* caller-fixed scaling when fixed_scale != 0 (a > 0) */
    int32_t sell_C;          /* 0: the lattice layout (13 slots per row, the lattice sweeps);
                                else store the built matrix in SELL-C-sigma with this chunk
                                height, as kpm_import_csr would (padding slots dropped) */
    int32_t sell_sigma;      /* sorting window for sell_C > 0 (0: 128 sell_C) */
} kpm_lattice_desc;

typedef struct kpm_hamiltonian kpm_hamiltonian; /* opaque, library-owned */

/* Build H of eq. "Ham" (section "Application Scenario") on the device:
 *   H = -t sum_{j,n} (Psi^dag_{n+e_j} (Gamma^1 - i Gamma^{j+1})/2 Psi_n + h.c.)
 *       + sum_n Psi^dag_n (V_n Gamma^0 + 2 Gamma^1) Psi_n
 * with Gamma^0 = 1, Gamma^1 = tau_z(x)s_0, Gamma^{2,3,4} = tau_x(x)s_{x,y,z},
 * orbital o = 2*tau + s, row 4*n + o.  N = 4*Lx*Ly*Lz rows, 13 stored
 * entries per row (open boundaries pad missing neighbours with explicit
 * zeros).  Then the Gershgorin interval [E_min, E_max] (section "Problem
 * Description": a and b from Gershgorin's circle theorem) gives
 * b = (E_max + E_min)/2 and a = margin (E_max - E_min)/2, unless
 * desc->fixed_scale.  Synchronises `stream` (the bounds are read back).
 * The storage is row-major with 13 slots per row: the lattice rows all have
 * the same length, so the SELL-C-sigma format of the paper's section
 * "Testbed and Implementation" reduces to chunk height 1 without sorting.
 * Errors: KPM_EINVAL (null desc/out, side <= 0, non-finite potential, t or
 * gamma, gamma < 0, margin < 1, a <= 0), KPM_ENOTSUP (a periodic side < 3),
 * KPM_ENOMEM, KPM_EDEVICE; with sell_C > 0 also the layout errors of
 * kpm_import_csr.  *out is NULL on error. */
kpm_status kpm_build_hamiltonian(const kpm_lattice_desc* desc, void* stream,
                                 kpm_hamiltonian** out);

/* Sizes and scaling of a built H.  Any output pointer may be NULL.
 * nnz_stored counts stored entries including padding (= width * N in the
 * lattice layout; the SELL-C-sigma storage's entries for an imported H, whose
 * width is its longest row). */
kpm_status kpm_hamiltonian_info(const kpm_hamiltonian* H, int64_t* N, int64_t* nnz_stored,
                                int32_t* width, int32_t* dtype, double* a, double* b,
                                double* emin, double* emax);

/* Copy H to host CRS for inspection: rowptr [N+1], col [nnz], val [2*nnz]
 * (re, im as double).  Lattice layout: explicit padding zeros are dropped and
 * each row keeps the library's slot order (diagonal first).  SELL-C-sigma
 * storage: the rows as imported (their order of entries, explicit zeros of
 * the input kept), padding dropped.  Pass col = val = NULL to get only
 * rowptr (and so the count).  Synchronous.  Errors: KPM_EINVAL. */
kpm_status kpm_export_csr(const kpm_hamiltonian* H, int64_t* rowptr, int32_t* col, double* val);

/* Release H and its workspaces (synchronises the device).  NULL is a no-op. */
void kpm_destroy_hamiltonian(kpm_hamiltonian* H);

/* A general sparse Hermitian matrix in host CRS, for kpm_import_csr. */
typedef struct {
    int64_t N;               /* rows = columns, >= 1 */
    const int64_t* rowptr;   /* host [N+1]: rowptr[0] = 0, non-decreasing; row i is entries
                                rowptr[i] .. rowptr[i+1]-1 */
    const int32_t* col;      /* host [nnz], 0 <= col < N, any order (repeated columns add up) */
    const double* val;       /* host [2*nnz] (re, im) */
    int32_t dtype;           /* kpm_dtype of the stored values and of the vector blocks */
    int32_t sell_C;          /* chunk height C: 1, 2, 4, 8, 16, 32 or 64; 0 = 8 */
    int32_t sell_sigma;      /* sorting window sigma in rows: 1 (no sorting) or a multiple of C
                                (>= N sorts globally); 0 = 128 C */
    double margin;           /* as in kpm_lattice_desc */
    int32_t fixed_scale;
    double a, b;
} kpm_csr_desc;

/* Layout of a CRS sparsity pattern in SELL-C-sigma (the unified storage
 * format the paper builds on, section "Related Work"; C = 1 without sorting
 * is CRS, the format of section "Testbed and Implementation").  Rows are
 * sorted by decreasing length (stable) inside consecutive windows of sigma
 * rows; sorted position p holds row perm[p] and lies in chunk p / C of
 * nchunks = ceil(N / C); chunk c is stored column-major, width[c] (its
 * longest row) entries deep, from entry start[c] (start[nchunks] = stored
 * entries, padding included), so entry j of position p sits at
 * start[p / C] + j*C + p mod C.  Host only (no device, no stream).
 * perm [N], width [nchunks], start [nchunks+1]: host, any may be NULL.
 * Errors: KPM_EINVAL (N < 1, a NULL rowptr, a decreasing rowptr or one not
 * starting at 0, C not a power of two in 1..64, sigma neither 1 nor a
 * multiple of C), KPM_ENOMEM (more than 2^31 - 1 rows). */
kpm_status kpm_sell_layout(int64_t N, const int64_t* rowptr, int32_t C, int32_t sigma, int32_t* perm,
                           int32_t* width, int64_t* start);

/* H from a general sparse Hermitian matrix in host CRS, stored on the
 * device in SELL-C-sigma (layout of kpm_sell_layout; padding entries hold
 * value 0 and column N), with the Gershgorin scaling of kpm_build_hamiltonian
 * computed on the device from the stored values (section "Problem
 * Description").  The vector blocks keep the matrix's own row order: the
 * sorting only reorders the work of a sweep.  kpm_aug_spmmv, kpm_moments,
 * kpm_moments_naive and kpm_lanczos_bounds accept the result; the lattice
 * entry points (kpm_moments_batched) do not.  H must be Hermitian for the
 * moments to mean anything; the library does not check it (kpm_moments
 * with check reports KPM_ESPECTRUM when moments leave [-mu_0, mu_0]).
 * Synchronises `stream`.  Errors: KPM_EINVAL (a NULL desc, out, col or val
 * with nnz > 0, a bad layout argument, a column out of range, a
 * non-finite value, margin < 1, a zero-width Gershgorin interval),
 * KPM_ENOMEM (stored values reaching 4 GiB: the sweep addresses them with
 * 32-bit offsets), KPM_EDEVICE.  *out is NULL on error.  The sweeps over
 * this storage take blocks of up to 4 GiB as well: kpm_aug_spmmv and
 * kpm_moments return KPM_ENOTSUP for an [N+1][R] block that reaches it. */
kpm_status kpm_import_csr(const kpm_csr_desc* desc, void* stream, kpm_hamiltonian** out);

/* SELL-C-sigma parameters of H: C and sigma (0 and 0 for a lattice H built
 * by kpm_build_hamiltonian), chunks, stored entries (padding included) and
 * the imported nonzero count.  Any output may be NULL.  Errors: KPM_EINVAL. */
kpm_status kpm_sell_info(const kpm_hamiltonian* H, int32_t* C, int32_t* sigma, int64_t* nchunks,
                         int64_t* stored, int64_t* nnz);

/* One augmented sweep (Alg. "kpm_improved_blocked", the fused body):
 *   W <- alpha * H V + beta * V + gamma * W            (variant FULL / NODOT)
 *   eta[0][r] = <V_r|V_r>,  eta[1][r] = <W_r|V_r>     (FULL only, new W)
 *   W <- H V                                           (variant PLAIN)
 * V, W: device [N][R] blocks of H's dtype, V read-only, W updated in place;
 * V and W must not overlap.  eta: device [2][R] complex double, written for
 * FULL when non-NULL (it is reduced on the device, deterministically).
 * R in {1, 2, 4, 8, 16, 32, 64}.  Blocks of any size on a lattice H (the
 * lattice sweep addresses arrays of 4 GiB or more plane by plane; the
 * index-reading sweeps fall back to 64-bit addressing there); on an
 * imported H an [N+1][R] block must stay below 4 GiB (kpm_moments splits
 * larger ones into column groups).  Errors: KPM_EINVAL, KPM_ENOTSUP. */
kpm_status kpm_aug_spmmv(const kpm_hamiltonian* H, const void* V, void* W, int32_t R,
                         double alpha, double beta, double gamma, int32_t variant,
                         double* eta, void* stream);

/* Options of kpm_moments.  A NULL opts pointer means all fields zero.
 * (struct kpm_sweep_tuning is defined with kpm_set_sweep_tuning below.) */
struct kpm_sweep_tuning;
typedef struct {
    int32_t check;       /* nonzero: synchronise `stream` and return KPM_ESPECTRUM when a moment is
                            non-finite or |mu_n| > mu_0 (1 + 1e-6) */
    int32_t use_graph;   /* nonzero: the launch sequence (copy of V0, the M/2 sweeps, the reductions
                            and eta -> mu) is captured once in a HIP graph and replayed by later calls
                            on the same stream with the same H, V0, R, M, mu, eta_out, variant,
                            scaling and tuning (any change captures again) */
    int32_t variant;     /* KPM_FULL (moments), or KPM_NODOT: the same M/2 sweeps of the recurrence
                            without the scalar products, for timing; mu is then not written */
    int32_t mu_on_host;  /* nonzero: mu is host memory (the call synchronises `stream`) */
    const struct kpm_sweep_tuning* tuning;   /* launch shape for this call only (NULL: the process-wide
                                         kpm_set_sweep_tuning setting, read once at entry) */
    double* eta_out;     /* optional device [M][R] complex double: the raw products eta_n */
    int32_t group;       /* column groups: 0 = the library's choice: on a lattice the lattice sweep
                            takes 32 columns at a time (R = 64 runs as two 32-column recurrences,
                            unless eta_out is set); otherwise the whole block in one recurrence,
                            unless the sweeps could not address it (an [N+1][R] block of 4 GiB or
                            more: then the widest supported width whose block fits, at least 32
                            on a lattice); else a supported width dividing R: the R columns run as
                            R / group independent recurrences of that width, one after the other,
                            on work blocks of N x group (the matrix is read once per group and
                            sweep).  Not with eta_out. */
} kpm_run_opts;

/* Chebyshev moments for R start vectors (eq. "eq:kpm_iter", scalar products
 * eta_{2m} = <nu_m|nu_m>, eta_{2m+1} = <nu_{m+1}|nu_m>, blocked algorithm):
 * M/2 fused sweeps on the device give eta_0 .. eta_{M-1}, then
 *   mu_0 = eta_0, mu_1 = Re eta_1, mu_{2m} = 2 eta_{2m} - mu_0,
 *   mu_{2m+1} = 2 Re eta_{2m+1} - mu_1      (per start vector r).
 * V0: device [N][R] block in H's dtype (read-only).  mu: [R][M] double,
 * device (or host with opts->mu_on_host).  M even and >= 2, R in {1, 2, 4,
 * 8, 16, 32, 64}.  (|<v|T_n(Htilde)|v>| <= <v|v> holds whenever the
 * spectrum of Htilde lies in [-1, 1], which the check tests.)
 * Workspaces (two blocks, the partial sums, the graph) are cached on H per
 * stream: calls on one stream reuse them in order, calls on different
 * streams (also from different threads) use separate sets and may overlap.
 * The start vectors' recurrences are independent (the columns of a block
 * share only the matrix), so a block split into column groups (opts->group)
 * gives the same moments up to the order of the scalar products' sums.
 * Errors: KPM_EINVAL, KPM_ENOTSUP, KPM_ENOMEM, KPM_ESPECTRUM, KPM_EDEVICE. */
kpm_status kpm_moments(const kpm_hamiltonian* H, const void* V0, int32_t R, int32_t M, double* mu,
                       const kpm_run_opts* opts, void* stream);

/* The naive KPM-DOS algorithm (Alg. "kpm_naive"), for measuring what the
 * fused and blocked sweeps save (Table "kpm_analysis": 13 N S_d vector bytes
 * per step and vector against 3 R N S_d per blocked sweep).  The trace is an
 * outer loop over the R start vectors; per vector the initialisation
 * w = nu_1 = (H v - b v) / a, eta_0 = <v|v>, eta_1 = <w|v>, then for
 * m = 1 .. M/2 - 1, with v and w swapping roles, one kernel per call:
 *   u <- H v (SpMV: the plain sweep at R = 1),  u <- u - b v (axpy),
 *   w <- -w (scal),  w <- w + (2/a) u (axpy),
 *   eta_2m = <v|v> (nrm2),  eta_2m+1 = <w|v> (dot),
 * and at the end the eta -> mu identity of kpm_moments.  Arguments, layout,
 * check and errors as kpm_moments (mu: device [R][M] double); three [N]
 * vectors and the scalar-product partials are cached on H.  The moments
 * equal kpm_moments' to rounding. */
kpm_status kpm_moments_naive(const kpm_hamiltonian* H, const void* V0, int32_t R, int32_t M,
                             double* mu, int32_t check, void* stream);

/* The BLAS level-1 kernels of the naive algorithm on device vectors of n
 * complex elements of storage type dtype (KPM_C128 or KPM_C64), 16-byte
 * aligned, enqueued on `stream`:
 *   kpm_axpy: y <- y + alpha x;   kpm_scal: x <- alpha x;
 *   kpm_dot:  out[0] + i out[1] = sum_i conj(x_i) y_i, accumulated in FP64
 *             (out: device, 2 doubles; x == y gives the squared norm with
 *             out[1] = 0).  The sum is reduced in a fixed order through a
 *             32 KiB partials buffer per (device, stream), allocated on the
 *             first call on that stream and held until the process ends:
 *             calls on one stream reuse it in order, calls on different
 *             streams (or threads using different streams) do not share it.
 * Errors: KPM_EINVAL (dtype, n < 0, NULL or misaligned vector). */
kpm_status kpm_axpy(int32_t dtype, int64_t n, double alpha, const void* x, void* y, void* stream);
kpm_status kpm_scal(int32_t dtype, int64_t n, double alpha, void* x, void* stream);
kpm_status kpm_dot(int32_t dtype, int64_t n, const void* x, const void* y, double* out, void* stream);

/* kpm_dot for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same result, computed by the same kernels in the same order, so it equals
 * kpm_dot bit for bit.  Its partial sums live in a 32 KiB array the library
 * holds in each GPU's memory from load to process exit (2048 workgroup
 * partials of two doubles: the dot grid never has more workgroups, so every
 * n fits and no size is rejected).  The call allocates nothing: no hipMalloc,
 * no hipFree, no allocating library routine; its first call on a device only
 * looks up that device's array address.  Every call on one GPU shares the
 * array: calls that overlap on one GPU (other streams, other threads) race
 * and may return wrong sums; calls ordered on one stream are safe.  Nothing
 * in the array needs clearing (each launch writes every partial it reads).
 * Errors: as kpm_dot; KPM_EDEVICE if the array's address cannot be found. */
kpm_status kpm_dot_noalloc(int32_t dtype, int64_t n, const void* x, const void* y, double* out, void* stream);

/* Density of states per unit energy from moments (the reconstruction step
 * the paper leaves to the KPM literature):
 *   mubar_n = (1/R) sum_r mu[r][n]                 (stochastic trace)
 *   rho(E) = [g_0 mubar_0 + 2 sum_{n=1}^{M-1} g_n mubar_n T_n(x)]
 *            / (pi a sqrt(1 - x^2)),  x = (E - b)/a,  rho = 0 for |x| >= 1
 * so that the integral of rho over E is mubar_0.  g_n: Jackson
 * ((M-n+1) cos(pi n/(M+1)) + sin(pi n/(M+1)) cot(pi/(M+1)))/(M+1),
 * Dirichlet 1, Lorentz sinh(kparam (1 - n/M))/sinh(kparam).
 * mu: device [R][M]; E: device [K]; rho: device [K] (all double).
 * Errors: KPM_EINVAL (null pointer, R/M/K <= 0, a <= 0, kernel unknown,
 * Lorentz kparam <= 0). */
kpm_status kpm_dos(const double* mu, int32_t R, int32_t M, int32_t kernel, double kparam,
                   double a, double b, const double* E, int32_t K, double* rho, void* stream);

/* Random-phase start block for the stochastic trace (section "Problem
 * Description"; the distribution of the random vectors is not fixed by the
 * paper, this is the library's reading): V device [N][R] in dtype,
 *   V[i][r] = exp(2 pi i u_ir) / sqrt(N),
 * u_ir = (top 53 bits of SplitMix64 output) / 2^53 at counter c = i R + r:
 * state key + (c + 1) * 0x9E3779B97F4A7C15 with key = mix(seed +
 * 0x9E3779B97F4A7C15), mix the SplitMix64 finaliser (Steele, Lea, Flood,
 * OOPSLA 2014).  Computed in FP64, rounded to the storage precision; every
 * column has unit norm up to rounding.  Errors: KPM_EINVAL. */
kpm_status kpm_random_phase_block(void* V, int64_t N, int32_t R, int32_t dtype, uint64_t seed, void* stream);

/* Spectral bounds from `steps` Lanczos steps (section "Problem Description":
 * a, b from Gershgorin's theorem or from Lanczos iterations).  Starting from
 * the random-phase unit vector of kpm_random_phase_block(seed, R = 1), the
 * recurrence w = H q_j - alpha_j q_j - beta_{j-1} q_{j-1}, alpha_j =
 * Re <q_j|H q_j>, beta_j = |w|, q_{j+1} = w / beta_j runs on the device
 * (one SpMV and four vector kernels per step, no reorthogonalisation); the
 * smallest and largest eigenvalues of the resulting tridiagonal matrix (the
 * extreme Ritz values, by bisection on Sturm counts) are written to *emin and
 * *emax (host).  Ritz values lie inside the spectrum, so these are not
 * rigorous bounds: enlarge them (kpm_set_scaling) and keep the moment check
 * of kpm_moments, which reports a scaling that does not contain the spectrum.
 * 2 <= steps <= 1024.  Uses H's cached [N] vectors; synchronises `stream`.
 * Errors: KPM_EINVAL, KPM_ENOMEM, KPM_EDEVICE. */
kpm_status kpm_lanczos_bounds(const kpm_hamiltonian* H, int32_t steps, uint64_t seed, double* emin, double* emax,
                              void* stream);

/* Replace the scaling of H: the sweeps apply Htilde = (H - b) / a from now on
 * (a > 0 finite, b finite).  Errors: KPM_EINVAL. */
kpm_status kpm_set_scaling(kpm_hamiltonian* H, double a, double b);

/* Deterministic start blocks for local and momentum-resolved spectra (the
 * local DOS and the spectral function A(k, E) of Fig. "topi_demo"; the paper
 * shows them without formulas, these follow the standard KPM reading: the
 * moments of one start vector |phi> are <phi|T_n(Htilde)|phi>, with no
 * trace average).  V: device [N][R] in dtype, 0 < R <= 64, written in full.
 * kpm_site_block: column r is the unit vector of row rows[r] (host [R],
 *   0 <= rows[r] < N); row 4 n + o is orbital o of site n.
 * kpm_plane_wave_block: column r is the plane wave of momentum k[r] (host
 *   [R][3], radians per lattice spacing) on orbital orbital[r] (host [R],
 *   0..3) of the Lx x Ly x Lz lattice L (host [3], N = 4 Lx Ly Lz):
 *   V[4 n + o][r] = delta(o, orbital[r]) exp(i k[r] . (x, y, z)_n) / sqrt(Lx Ly Lz),
 *   site n = x + Lx (y + Ly z); the phase is computed in FP64.
 * Errors: KPM_EINVAL (NULL, dtype, R, a row, orbital or momentum out of range). */
kpm_status kpm_site_block(void* V, int64_t N, int32_t R, const int64_t* rows, int32_t dtype, void* stream);
kpm_status kpm_plane_wave_block(void* V, const int32_t* L, int32_t R, const double* k, const int32_t* orbital,
                                int32_t dtype, void* stream);

/* kpm_dos for n_inst instances in one launch, from a prefix of their
 * moments: instance i uses mu[i][r][n] = mu[(i R + r) ld + n] for n < M
 * (ld >= M; a prefix of an M'-moment run equals an M-moment run with the
 * same start vectors), the damping kernel for M moments and its own
 * scaling a[i], b[i] (device arrays), on the shared energy grid E [K].
 * masses = 0: rho [n_inst][K] is the density per unit energy; masses != 0:
 * each row is divided by its sum (in index order), i.e. the DOS mass per
 * bin of a uniform grid.  All pointers device.  n_inst <= 65535.
 * Errors: KPM_EINVAL. */
kpm_status kpm_dos_batched(const double* mu, int32_t n_inst, int32_t R, int32_t ld, int32_t M, int32_t kernel,
                           double kparam, const double* a, const double* b, const double* E, int32_t K,
                           int32_t masses, double* rho, void* stream);

/* Input features of the learned reconstruction: x[i][f] = (1/R) sum_r
 * mu[(i R + r) ld + f] (FP32) for f < n_mom (the stochastic trace of the
 * first n_mom moments), then x[i][n_mom] = extra[i] when extra is non-NULL
 * (e.g. the disorder strength).  All pointers device.  Errors: KPM_EINVAL. */
kpm_status kpm_moment_features(const double* mu, int32_t n_inst, int32_t R, int32_t ld, int32_t n_mom,
                               const float* extra, float* x, void* stream);

/* Launch shape of the fused sweep kernel (process-wide, guarded by a lock:
 * every call reads it once at entry, so a change from another thread takes
 * effect from the next call on; kpm_run_opts.tuning overrides it for one
 * kpm_moments call).  Results do not depend on it beyond the order of
 * floating-point sums:
 *   wg_per_cu    workgroups per compute unit in the persistent grid; 0
 *                selects 8 for the scalar-operand sweep (4-wave workgroups,
 *                32 resident waves per CU) and 16 waves per CU for the
 *                staged-gather sweep
 *   xcd_ways     row tiles are split into this many contiguous ranges, one
 *                per accelerator die, matching the round-robin dispatch of
 *                workgroups to the 8 XCDs; 1 disables it; default 8
 *   chunk_tiles  consecutive row tiles a workgroup takes per grab (dynamic)
 *                or before striding (static); default 8
 *   dynamic      nonzero: each workgroup reads the id of the die it runs on
 *                and takes tiles from that die's range through an atomic
 *                counter, then helps the other ranges; the rows a workgroup
 *                sums then vary between runs, so the scalar products agree
 *                between runs only to rounding.  Zero: static mapping
 *                (workgroup g takes range g % xcd_ways), bitwise
 *                reproducible; default 0
 *   prefetch     0, 1 or 2.  Generic sweep: 1 = before a wave streams its
 *                tiles it touches every line of their matrix rows and old
 *                W rows (0 and 2: no touch pass).  Lattice sweep: how the
 *                matrix rows of a site reach the FMAs: 2 one vector load a
 *                step ahead, handed over lane by lane (complex128) or
 *                written to the wave's slot in LDS and read back by all
 *                lanes at once (complex64); 1 scalar loads whose lines a
 *                vector load pulled into L2 a step ahead; 0 scalar loads
 *                when the row is computed; default 2
 *   lattice      1 (default): at R = 32 and 64, on lattices with at least
 *                128 4 x 4-site pencils, use the cache-blocked sweep that
 *                keeps a ring of z-planes of V in LDS (of the other fields
 *                only prefetch, stream, tile_order and wg_per_cu apply to it;
 *                wg_per_cu is capped at the 1 (complex128) or 2 (complex64)
 *                workgroups whose LDS fits on a CU, default 1; at R = 64 it
 *                sweeps the two 32-column halves of the block one after the
 *                other, reading the matrix once per half, and always takes
 *                prefetch 2); 2: use it whenever R is 32 or 64; 0: the
 *                generic gather sweep
 *   stream       bit 0: old-W loads, bit 1: new-W stores carry the
 *                non-temporal hint (W is touched once per sweep, unlike the
 *                V rows, which are gathered 13 times), so that L2 keeps the
 *                planes of V that neighbouring tiles gather; default 3
 *   pencil       processing order of the lattice sites: pencils of
 *                pencil x pencil sites spanning the whole z extent, each
 *                walked plane by plane (x fastest), so that the rows a sweep
 *                gathers for the z neighbours were fetched one plane
 *                earlier; 0 keeps the natural row order; default 16.  The
 *                storage order of H and of the vector blocks never changes.
 *   gather       which generic sweep runs where the lattice sweep does not:
 *                0 the staged-gather sweep for R != 32 and the
 *                scalar-operand sweep for R = 32; 1 (default) the
 *                staged-gather sweep for every R, as its LDS-window variant
 *                where that exists (complex128 R >= 16, complex64 R >= 32)
 *                and the lattice gives at least one run of z-planes of a
 *                tile per CU; 2 the scalar-operand sweep for every R; 3 the
 *                window variant wherever it exists (any lattice size); 4
 *                the staged-gather sweep without the window variant.  The
 *                window variant walks the lattice in pencils (one
 *                workgroup per run of z-planes of a 4 x 4-site tile, 2 x 2
 *                at complex128 R = 64), keeps the tile's planes z - 1, z,
 *                z + 1 of V in an LDS ring and gathers only the other
 *                neighbours from memory; it still reads the column indices
 *                (each is decoded once, when the matrix rows of a pass are
 *                staged), so any matrix over the lattice's rows gives the
 *                staged-gather result (on 64^3 at R = 32: 426 us per sweep
 *                against 573 us; its matrix and W streams ignore `stream`
 *                and go through L2 with the default policy).  The
 *                staged-gather sweep (one lane per 16 bytes of a block row,
 *                matrix rows copied into LDS a pass ahead) uses only
 *                wg_per_cu and xcd_ways of the fields above, and needs the
 *                vector block and the matrix to stay below 4 GiB (otherwise
 *                the scalar-operand sweep runs).
 *   tile_order   lattice sweep: how pencils are dealt to the 8 dies: 0
 *                each die a 2-D block of tiles (so that most edge rows a
 *                tile gathers belong to tiles of its own die, in its own
 *                L2), 1 each die a contiguous run of tile rows, 2 no die
 *                mapping (pencils dealt round-robin to all workgroups), 3
 *                (default) 2 when there are more pencils than workgroups,
 *                else 0 (measured: 2 is 1-12 % faster on 128 x 128 x 64 and
 *                on 100 x 100 x 40 and 200 x 100 x 40 slabs; at one pencil
 *                per workgroup, as on 64^3, 0 is as fast or faster).  Only the
 *                work distribution changes.
 *   slab         staged-gather sweep at R <= 16: the passes walk the lattice
 *                in blocks of this many y-lines, each block plane by plane,
 *                so that the rows gathered for z neighbours were touched a
 *                few lines earlier (3-8 % at R = 2..16 on 64^3; at larger R
 *                the index arithmetic costs more occupancy than it saves,
 *                and the natural order runs); 0 = natural row order;
 *                default 4
 *   gather_tile  staged-gather sweep with passes of at most one site (R >= 16
 *                in complex128, R >= 32 in complex64) on a lattice: pencil
 *                order, one workgroup per run of z-planes of a tile of
 *                gather_tile x gather_tile sites, its waves sharing each
 *                plane of the tile, so that the V rows a pass gathers were
 *                fetched at most a plane earlier by the same workgroup or by
 *                the adjacent tile's on the same die (tiles dealt to the
 *                dies in 2-D blocks where the tile grid allows); the matrix
 *                and W streams then carry the non-temporal hint when
 *                `stream` is nonzero.  0: the natural (or slab) order;
 *                default 0
 * kpm_set_sweep_tuning(NULL) restores the defaults.  Errors: KPM_EINVAL
 * (negative field). */
typedef struct kpm_sweep_tuning {
    int32_t wg_per_cu;
    int32_t xcd_ways;
    int32_t chunk_tiles;
    int32_t pencil;
    int32_t dynamic;
    int32_t prefetch;
    int32_t stream;
    int32_t lattice;
    int32_t gather;
    int32_t tile_order;
    int32_t slab;
    int32_t gather_tile;
} kpm_sweep_tuning;
kpm_status kpm_set_sweep_tuning(const kpm_sweep_tuning* tuning);
kpm_status kpm_get_sweep_tuning(kpm_sweep_tuning* tuning);

/* Which sweep kernel kpm_moments / kpm_aug_spmmv launch for H at block
 * width R under the current tuning: *kernel = 0 scalar-operand gather
 * sweep, 1 cache-blocked lattice sweep, 2 staged-gather sweep, 3 its
 * LDS-window variant, 4 the SELL-C-sigma sweep (H from kpm_import_csr).
 * Errors: KPM_EINVAL. */
kpm_status kpm_sweep_kernel(const kpm_hamiltonian* H, int32_t R, int32_t* kernel);

/* The launch a sweep of H at block width R gets under `tuning` (NULL: the
 * process-wide setting): kernel as kpm_sweep_kernel; grid = workgroups;
 * tile_order = the lattice sweep's pencil-to-die mapping after resolving
 * the automatic choice (0 2-D blocks per die, 1 runs of tile rows, 2
 * round-robin; -1 for the other kernels); pieces = z-pieces per pencil
 * (1 = whole pencils; -1 for the other kernels); halves = 32-column passes
 * of the lattice sweep over the block (-1 for the other kernels); group =
 * the column-group width kpm_moments takes for this block by default (R:
 * one recurrence; less where the block reaches 4 GiB), in which case the
 * other fields describe a sweep of one group.  Errors: KPM_EINVAL. */
typedef struct {
    int32_t kernel, grid, tile_order, pieces, halves, group;
} kpm_sweep_plan_info;
kpm_status kpm_sweep_plan(const kpm_hamiltonian* H, int32_t R, const struct kpm_sweep_tuning* tuning,
                          kpm_sweep_plan_info* out);

/* Sweep-kernel timing for measurement tools.  kpm_sweep_profile_enable(n),
 * n > 0 (process-wide, guarded by a lock): every n-th fused sweep launched by
 * kpm_moments and kpm_aug_spmmv from then on (the first, the (n+1)-th, ...)
 * is bracketed by a pair of HIP events on its own stream; each pair costs a
 * few microseconds of stream time, so sampling (n > 1) keeps a timed run
 * close to an untimed one.  n = 0 turns it off.  kpm_sweep_profile_read
 * waits for the recorded events, returns the count, total, minimum and
 * maximum kernel time in milliseconds of the timed launches (any output may
 * be NULL) and clears the record.  Sweeps captured into a HIP graph
 * (kpm_run_opts.use_graph) are not timed.  Errors: KPM_EINVAL (n < 0),
 * KPM_EDEVICE. */
kpm_status kpm_sweep_profile_enable(int32_t enable);
kpm_status kpm_sweep_profile_read(int64_t* count, double* total_ms, double* min_ms, double* max_ms);

/* Batched moments: n_inst independent problems in one persistent launch.
 * Instance i is exactly kpm_moments(H[i], V0[i], R, M) (section
 * "Algorithm" / Alg. "kpm_improved_blocked" per instance; the paper's
 * outlook combines loosely coupled outer iterations into one launch, here
 * the independent disorder realisations and lattice sizes of a study):
 * M/2 fused sweeps, the scalar products eta_0 .. eta_{M-1} and the doubling
 * identity to mu_0 .. mu_{M-1}.  One workgroup owns one instance from the
 * first sweep to its moments; instances are taken longest-first, so the
 * result of an instance is bitwise independent of the batch it is in and
 * of the tuning's mapping (it depends on `waves` and `slab`, which fix the
 * order of the sums).
 *   H:   host array [n_inst] of handles, all of one dtype, built on the
 *        current device; the same handle may appear more than once.
 *   V0:  host array [n_inst] of device start blocks [N_i][R] in that dtype
 *        (read-only).
 *   mu:  device [n_inst][R][M] doubles.
 * R in {1, 2, 4, 8, 16, 32, 64}; M even and >= 2; per instance the block
 * and the matrix arrays must each be smaller than 4 GiB.
 * flags: KPM_BATCH_CHECK synchronises `stream` and returns KPM_ESPECTRUM if
 * any instance has a moment that is non-finite or |mu_n| > mu_0 (1 + 1e-6);
 * KPM_BATCH_GRAPH captures the launch sequence (counter reset and the
 * persistent kernel) in a HIP graph and, while the next call repeats the
 * same handles, start blocks, mu, R, M and tuning, replays it instead of
 * re-uploading the instance table.
 * Workspaces (two blocks per instance, the per-sweep products, the instance
 * table, the graph) are library-owned, one set per (device, stream): calls
 * on one stream reuse them in order, calls on different streams (also from
 * different threads) use separate sets and may overlap.
 * Errors: KPM_EINVAL, KPM_ENOTSUP, KPM_ENOMEM, KPM_ESPECTRUM, KPM_EDEVICE. */
enum { KPM_BATCH_CHECK = 1, KPM_BATCH_GRAPH = 2 };
kpm_status kpm_moments_batched(const kpm_hamiltonian* const* H, const void* const* V0, int32_t n_inst,
                               int32_t R, int32_t M, double* mu, int32_t flags, void* stream);

/* Launch shape of the batched solver (process-wide, guarded by a lock and
 * read once per call):
 *   waves      waves per workgroup (4, 8 or 16, capped by what the
 *              workgroup's LDS and registers allow: 16 in complex64, 8 in
 *              complex128, fewer for R <= 2); 0 = 8 (or the cap if lower).
 *              The order of the floating-point sums of a sweep depends on it.
 *   wg_per_cu  workgroups per compute unit in the persistent grid; 0 = 1
 *   dynamic    nonzero (default): workgroups take instances from the
 *              longest-first list through an atomic counter (greedy
 *              longest-processing-time); zero: workgroup g takes entries
 *              g, g + grid, ... of that list.
 *   slab       a workgroup walks its instance's lattice in blocks of this
 *              many y-lines, each block plane by plane (0 = natural row
 *              order, the default: fastest on the 512-instance family
 *              since the solver derives its gather offsets from the
 *              lattice).  Only the order of work changes.
 * kpm_set_batch_tuning(NULL) restores the defaults.  Errors: KPM_EINVAL. */
typedef struct {
    int32_t waves;
    int32_t wg_per_cu;
    int32_t dynamic;
    int32_t slab;
} kpm_batch_tuning;
kpm_status kpm_set_batch_tuning(const kpm_batch_tuning* tuning);
kpm_status kpm_get_batch_tuning(kpm_batch_tuning* tuning);

/* ---- Learned DOS reconstruction (a small MLP; not part of the paper) ----
 * Network, for one sample x of n_in features (the first n_in - 1 Chebyshev
 * moments of the stochastic average plus the disorder strength):
 *   h1 = gelu(x W1 + b1), h2 = gelu(h1 W2 + b2), h3 = gelu(h2 W3 + b3)
 *   q = softmax(h3 W4 + b4)           n_out DOS masses on a fixed energy grid
 *   e = softplus(h3 w5 + b5)          predicted L1 error of q
 * with gelu(x) = x Phi(x) (exact, erf form).  Training loss for a batch of B
 * samples with target masses p (rows sum to 1) and error targets t:
 *   L = (1/B) sum_b [ -sum_k p_bk log q_bk + lam (e_b - t_b)^2 ].
 * All matrix products run on the matrix cores in BF16 with FP32
 * accumulation (weights are BF16 copies of FP32 masters; activations are
 * rounded to BF16 when stored); biases, softmax, loss and Adam are FP32.
 * Parameter vectors on the host are FP32 in the order W1 [n_in][hidden],
 * b1, W2 [hidden][hidden], b2, W3, b3, W4 [hidden][n_out], b4, w5 [hidden],
 * b5 (row-major).  The network, its weights, Adam state and activations
 * are library-owned device memory for batches up to max_batch.  Calls on
 * one network must not overlap.  Errors: KPM_EINVAL (NULL, sizes out of
 * range, non-finite parameters), KPM_ENOMEM, KPM_EDEVICE. */
typedef struct kpm_mlp kpm_mlp;
kpm_status kpm_mlp_create(int32_t n_in, int32_t hidden, int32_t n_out, int32_t max_batch, kpm_mlp** out);
void       kpm_mlp_destroy(kpm_mlp* net);
/* Number of parameters (floats) in the host parameter vector. */
kpm_status kpm_mlp_param_count(const kpm_mlp* net, int64_t* count);
/* Load parameters (host, FP32) and reset the Adam state.  Synchronous. */
kpm_status kpm_mlp_set_params(kpm_mlp* net, const float* params);
/* Copy the FP32 master parameters / the last computed gradients to the
 * host (same order).  Synchronous. */
kpm_status kpm_mlp_get_params(const kpm_mlp* net, float* params);
kpm_status kpm_mlp_get_grads(const kpm_mlp* net, float* grads);
/* Inference: x device [B][n_in] FP32 -> q device [B][n_out], e device [B]
 * (either may be NULL).  1 <= B <= max_batch. */
kpm_status kpm_mlp_forward(kpm_mlp* net, const float* x, int32_t B, float* q, float* e, void* stream);
/* Forward and backward pass: gradients of L (kept on the device, see
 * kpm_mlp_get_grads) for x [B][n_in], p [B][n_out], t [B] (device FP32;
 * t NULL: each sample's error target is its own current L1 error
 * sum_k |q_k - p_k|, treated as a constant); loss (device [1], may be NULL)
 * receives L.  lam >= 0. */
kpm_status kpm_mlp_backward(kpm_mlp* net, const float* x, const float* p, const float* t, int32_t B, float lam,
                            float* loss, void* stream);
/* One Adam step (bias-corrected) on the masters from the last gradients. */
kpm_status kpm_mlp_adam_step(kpm_mlp* net, float lr, float beta1, float beta2, float eps, void* stream);
/* kpm_mlp_backward followed by kpm_mlp_adam_step(lr, 0.9, 0.999, 1e-8). */
kpm_status kpm_mlp_train_step(kpm_mlp* net, const float* x, const float* p, const float* t, int32_t B, float lam,
                              float lr, float* loss, void* stream);
/* The network's GEMM on its own: C [M][N] FP32 = op(A) op(B), BF16 bits in
 * A (row-major [M][K], or [K][M] if trans_a) and B ([K][N], or [N][K] if
 * trans_b), all device; not both transposed. */
kpm_status kpm_mlp_gemm_bf16(const uint16_t* A, const uint16_t* B, int32_t M, int32_t N, int32_t K, int32_t trans_a,
                             int32_t trans_b, float* C, void* stream);

/* Attainable-bandwidth reference for the roofline (the paper bounds every
 * kernel by a measured attainable bandwidth b, Table "tab:architectures" and
 * eq. "eq:roofline_mem"): STREAM-style kernels over `bytes` (a multiple of
 * 16) of 16-byte-aligned device arrays,
 *   KPM_STREAM_COPY:   c = a              (traffic 2 x bytes)
 *   KPM_STREAM_TRIAD:  c = a + scalar b   (FP64 elements; traffic 3 x bytes)
 *   KPM_STREAM_READ:   c[g] = sum of the FP64 values of a that workgroup g
 *                      read (traffic 1 x bytes); c must hold one double per
 *                      workgroup, at most (compute units x wg_per_cu), and
 *                      the sum of c[0 .. grid-1] is the sum of a's values
 *                      (c beyond the grid is not written)
 * with wg_per_cu workgroups of 256 threads per compute unit (1 .. 32; fewer
 * when the array has fewer 4 KiB pieces than that), each thread keeping four
 * (read: eight) 16-byte loads in flight.  `nontemporal` nonzero: copy and
 * triad store, and read loads, with the non-temporal hint.  c must not
 * overlap a or b; b is unused by copy and read.  Errors: KPM_EINVAL. */
enum { KPM_STREAM_COPY = 0, KPM_STREAM_TRIAD = 1, KPM_STREAM_READ = 2 };
kpm_status kpm_stream(int32_t kind, void* c, const void* a, const void* b, double scalar, int64_t bytes,
                      int32_t wg_per_cu, int32_t nontemporal, void* stream);

/* Thread-local message for the last failing call on this thread ("" if none). */
const char* kpm_last_error(void);

/* Library version string. */
const char* kpm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* KPM_H */
