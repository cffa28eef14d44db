/*
 * kpm_oracle.c -- plain CPU oracle for the Kernel Polynomial Method (KPM)
 * density-of-states path of Kreutzer, Hager, Wellein, Pieper, Alvermann and
 * Fehske, "Performance Engineering of the Kernel Polynomial Method on
 * Large-Scale CPU-GPU Systems" (arXiv:1410.5242).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library. It includes nothing from
 * the GPU library and the GPU library includes nothing from it.
 *
 * Everything is IEEE double / double complex in compressed row storage (CRS).
 * There is no blocking, fusion or reordering beyond what the paper's
 * algorithms state: each step is written the obvious way so that it can be
 * checked against the paper by eye. The only parallelism is an OpenMP
 * "parallel for" over independent matrix rows in the sparse products and over
 * the independent columns of a block scalar product. Each scalar product is
 * a pairwise sum over the rows (error bound independent of N up to a
 * log2 N factor, so the oracle certifies moments to ~1e-14 even at 10^6
 * rows); the Gershgorin extremum is a sequential loop.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex zc;

/* Number of OpenMP threads the row loops use. */
int oracle_threads(void) { return omp_get_max_threads(); }

/* Set the number of OpenMP threads of later row loops (n >= 1).  Results do
 * not depend on it: every row and every column sum is computed by one thread
 * in a fixed order. */
void oracle_set_threads(int n) { if (n >= 1) omp_set_num_threads(n); }

/* ------------------------------------------------------------------------- */
/* Dirac matrices of the topological-insulator Hamiltonian (eq. "Ham").      */
/* Orbital index o = 2*tau + s: the first Kronecker factor (tau) is the      */
/* outer one.  Gamma^1 = tau_z (x) s_0, Gamma^{2,3,4} = tau_x (x) s_{x,y,z}. */
/* Gamma^0 is the 4x4 identity (the onsite potential multiplies it).         */
/* ------------------------------------------------------------------------- */
static void pauli(int which, zc p[2][2])
{
    /* which: 0 = identity, 1 = x, 2 = y, 3 = z */
    p[0][0] = p[0][1] = p[1][0] = p[1][1] = 0;
    switch (which) {
    case 0: p[0][0] = 1; p[1][1] = 1; break;
    case 1: p[0][1] = 1; p[1][0] = 1; break;
    case 2: p[0][1] = -I; p[1][0] = I; break;
    case 3: p[0][0] = 1; p[1][1] = -1; break;
    }
}

static void kron2(zc a[2][2], zc b[2][2], zc out[4][4])
{
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int k = 0; k < 2; ++k)
                for (int l = 0; l < 2; ++l)
                    out[2 * i + k][2 * j + l] = a[i][j] * b[k][l];
}

/* gamma(a): a = 0..4 as in eq. "Ham" (a = 0 is the identity). */
static void gamma_matrix(int a, zc g[4][4])
{
    zc tau[2][2], sig[2][2];
    if (a == 0) { pauli(0, tau); pauli(0, sig); }
    else if (a == 1) { pauli(3, tau); pauli(0, sig); }
    else { pauli(1, tau); pauli(a - 1, sig); }
    kron2(tau, sig, g);
}

/* ------------------------------------------------------------------------- */
/* Hamiltonian builder (eq. "Ham"), CRS with columns sorted and duplicate    */
/* (row, col) pairs summed.                                                  */
/*                                                                           */
/* Site n = x + Lx*(y + Ly*z); row index 4*n + o.                            */
/* Hopping term  -t * Psi^dag_{n+e_j} (Gamma^1 - i Gamma^{j+1})/2 Psi_n      */
/* puts the block T_j = -t (Gamma^1 - i Gamma^{j+1}) / 2 at                  */
/* (rows of n+e_j, columns of n); its Hermitian conjugate puts T_j^dagger at */
/* (rows of n, columns of n+e_j).  Onsite block: V_n * Gamma^0 + 2 Gamma^1.  */
/* A neighbour outside a non-periodic side is dropped (open boundary).       */
/* An entry is structural when its Gamma pattern is nonzero, independent of */
/* t and V_n, and the diagonal is always stored.                            */
/* ------------------------------------------------------------------------- */
typedef struct { int64_t col; zc v; } entry;

static int cmp_entry(const void* pa, const void* pb)
{
    const entry* a = (const entry*)pa;
    const entry* b = (const entry*)pb;
    return (a->col > b->col) - (a->col < b->col);
}

static int64_t wrap(int64_t x, int64_t L, int periodic, int* ok)
{
    if (x >= 0 && x < L) { *ok = 1; return x; }
    if (!periodic) { *ok = 0; return 0; }
    *ok = 1;
    return ((x % L) + L) % L;
}

/* The blocks of eq. "Ham" for one lattice: Gamma matrices, hopping blocks
 * T_j and their structural patterns. */
typedef struct {
    int64_t L[3];
    int periodic[3];
    zc g[5][4][4];
    zc T[3][4][4];      /* T_j = -t (Gamma^1 - i Gamma^{j+1}) / 2 */
    int Tpat[3][4][4];  /* structural pattern of Gamma^1 - i Gamma^{j+1} */
} ti_blocks;

static void make_blocks(int Lx, int Ly, int Lz, const int* periodic, double t, ti_blocks* B)
{
    B->L[0] = Lx; B->L[1] = Ly; B->L[2] = Lz;
    for (int j = 0; j < 3; ++j) B->periodic[j] = periodic[j];
    for (int a = 0; a < 5; ++a) gamma_matrix(a, B->g[a]);
    for (int j = 0; j < 3; ++j)
        for (int o = 0; o < 4; ++o)
            for (int p = 0; p < 4; ++p) {
                zc pat = B->g[1][o][p] - I * B->g[j + 2][o][p];
                B->Tpat[j][o][p] = (pat != 0);
                B->T[j][o][p] = -t * pat / 2.0;
            }
}

/* Entries of row (n, o), columns sorted and duplicates summed, into buf;
 * returns their number (at most 13 + 12 duplicates before merging). */
static int build_row(const ti_blocks* B, const double* pot, int64_t n, int o, entry buf[64])
{
    const int64_t Lx = B->L[0], Ly = B->L[1];
    const int64_t xyz[3] = {n % Lx, (n / Lx) % Ly, n / (Lx * Ly)};
    int cnt = 0;
    /* onsite block: V_n Gamma^0 + 2 Gamma^1 (diagonal always stored) */
    for (int p = 0; p < 4; ++p) {
        zc v = pot[n] * B->g[0][o][p] + 2.0 * B->g[1][o][p];
        if (p == o || v != 0) { buf[cnt].col = 4 * n + p; buf[cnt].v = v; ++cnt; }
    }
    for (int j = 0; j < 3; ++j) {
        /* row (n, o) as the n+e_j side: partner site m = n - e_j,
         * entry T_j[o][p] at column (m, p). */
        int ok;
        int64_t c[3] = {xyz[0], xyz[1], xyz[2]};
        c[j] = wrap(xyz[j] - 1, B->L[j], B->periodic[j], &ok);
        if (ok) {
            int64_t m = c[0] + Lx * (c[1] + Ly * c[2]);
            for (int p = 0; p < 4; ++p)
                if (B->Tpat[j][o][p]) { buf[cnt].col = 4 * m + p; buf[cnt].v = B->T[j][o][p]; ++cnt; }
        }
        /* row (n, o) as the n side of the conjugate term: partner
         * m = n + e_j, entry (T_j^dagger)[o][p] = conj(T_j[p][o]). */
        c[0] = xyz[0]; c[1] = xyz[1]; c[2] = xyz[2];
        c[j] = wrap(xyz[j] + 1, B->L[j], B->periodic[j], &ok);
        if (ok) {
            int64_t m = c[0] + Lx * (c[1] + Ly * c[2]);
            for (int p = 0; p < 4; ++p)
                if (B->Tpat[j][p][o]) { buf[cnt].col = 4 * m + p; buf[cnt].v = conj(B->T[j][p][o]); ++cnt; }
        }
    }
    qsort(buf, (size_t)cnt, sizeof(entry), cmp_entry);
    int out = 0;
    for (int k = 0; k < cnt; ++k) {
        if (out > 0 && buf[out - 1].col == buf[k].col) buf[out - 1].v += buf[k].v;
        else buf[out++] = buf[k];
    }
    return out;
}

/* Returns the number of stored entries, or -1 if cap is too small or the
 * arguments are invalid.  With rowptr == NULL only the count is returned.
 * Rows are independent: one pass counts each row's entries, a prefix sum
 * gives the row pointers, a second pass writes the entries. */
int64_t oracle_ti_build(int Lx, int Ly, int Lz, const int* periodic, double t,
                        const double* pot, int64_t* rowptr, int32_t* col,
                        double* val_ri, int64_t cap)
{
    if (Lx <= 0 || Ly <= 0 || Lz <= 0) return -1;
    const int64_t nsite = (int64_t)Lx * Ly * Lz;
    const int64_t N = 4 * nsite;
    ti_blocks B;
    make_blocks(Lx, Ly, Lz, periodic, t, &B);
    int64_t* cnt = rowptr ? rowptr + 1 : (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    if (!cnt) return -1;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        entry buf[64];
        cnt[i] = build_row(&B, pot, i / 4, (int)(i % 4), buf);
    }
    int64_t nnz = 0;
    for (int64_t i = 0; i < N; ++i) nnz += cnt[i];
    if (!rowptr) {
        free(cnt);
        return nnz;
    }
    if (nnz > cap) return -1;
    rowptr[0] = 0;
    for (int64_t i = 0; i < N; ++i) rowptr[i + 1] += rowptr[i];
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        entry buf[64];
        const int c = build_row(&B, pot, i / 4, (int)(i % 4), buf);
        for (int k = 0; k < c; ++k) {
            col[rowptr[i] + k] = (int32_t)buf[k].col;
            val_ri[2 * (rowptr[i] + k)] = creal(buf[k].v);
            val_ri[2 * (rowptr[i] + k) + 1] = cimag(buf[k].v);
        }
    }
    return nnz;
}

/* ------------------------------------------------------------------------- */
/* Gershgorin circles: every eigenvalue lies in some disc centred at Re H_ii */
/* with radius sum_{j != i} |H_ij|.  Returns the outer bounds.               */
/* ------------------------------------------------------------------------- */
void oracle_gershgorin(int64_t N, const int64_t* rowptr, const int32_t* col,
                       const double* val_ri, double* emin, double* emax)
{
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = 0; i < N; ++i) {
        double c = 0.0, r = 0.0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            zc h = val_ri[2 * k] + I * val_ri[2 * k + 1];
            if (col[k] == i) c += creal(h);
            else r += cabs(h);
        }
        if (c - r < lo) lo = c - r;
        if (c + r > hi) hi = c + r;
    }
    *emin = lo;
    *emax = hi;
}

/* y = Htilde x for an N x R block stored row-major (element (i, r) at
 * i*R + r), Htilde = (H - b)/a. */
static void apply_htilde(int64_t N, const int64_t* rowptr, const int32_t* col,
                         const double* val_ri, double a, double b, int R,
                         const zc* x, zc* y)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        for (int r = 0; r < R; ++r) {
            zc s = 0;
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                zc h = val_ri[2 * k] + I * val_ri[2 * k + 1];
                s += h * x[(int64_t)col[k] * R + r];
            }
            y[i * R + r] = (s - b * x[i * R + r]) / a;
        }
    }
}

/* Sum of conj(x_ir) y_ir over rows lo <= i < hi of column r by pairwise
 * (cascade) summation: ranges of at most PAIRWISE_LEAF rows are summed in
 * row order, longer ranges are halved and the two half sums added.  The
 * rounding error of the result is at most about
 * (PAIRWISE_LEAF - 1 + ceil(log2(n / PAIRWISE_LEAF))) u sum_i |x_ir| |y_ir|
 * for n = hi - lo terms and unit roundoff u = 2^-53 (Higham, "Accuracy and
 * Stability of Numerical Algorithms", 2nd ed., section 4.2), i.e. below
 * 25 u = 2.8e-15 of sum |x||y| for n <= 2^20 rows, whereas a running sum
 * is only bounded by (n - 1) u.  The tree depends on (lo, hi) alone, so the
 * result does not depend on the number of threads.                        */
#define PAIRWISE_LEAF 8

static zc pairwise_dot(int64_t lo, int64_t hi, int64_t R, int r, const zc* x, const zc* y)
{
    if (hi - lo <= PAIRWISE_LEAF) {
        zc s = 0;
        for (int64_t i = lo; i < hi; ++i) s += conj(x[i * R + r]) * y[i * R + r];
        return s;
    }
    const int64_t mid = lo + (hi - lo) / 2;
    return pairwise_dot(lo, mid, R, r, x, y) + pairwise_dot(mid, hi, R, r, x, y);
}

/* column-wise <x_r | y_r> = sum_i conj(x_ir) y_ir (pairwise in i; the
 * columns are independent sums and run on separate threads) */
static void block_dot(int64_t N, int R, const zc* x, const zc* y, zc* out)
{
    #pragma omp parallel for schedule(static)
    for (int r = 0; r < R; ++r) out[r] = pairwise_dot(0, N, R, r, x, y);
}

/* Exported for the oracle's own pins: out[2 r], out[2 r + 1] = re, im of
 * <x_r | y_r> for [N][R] blocks x, y (interleaved re, im doubles).        */
void oracle_block_dot(int64_t N, int R, const double* x_ri, const double* y_ri, double* out_ri)
{
    block_dot(N, R, (const zc*)x_ri, (const zc*)y_ri, (zc*)out_ri);
}

/* ------------------------------------------------------------------------- */
/* KPM moments by the blocked algorithm (Alg. "kpm_improved_blocked",        */
/* recurrence eq. "eq:kpm_iter").                                            */
/*   nu_0 = v0, nu_1 = Htilde nu_0, nu_{m+1} = 2 Htilde nu_m - nu_{m-1}      */
/*   eta_{2m} = <nu_m | nu_m>,  eta_{2m+1} = <nu_{m+1} | nu_m>               */
/* M/2 sweeps in total (the initialisation sweep and M/2-1 recurrence        */
/* sweeps) give eta_0 .. eta_{M-1}.  eta is [M][R] complex, stored as        */
/* interleaved (re, im) doubles.  v0 is [N][R] complex, row-major.           */
/* ------------------------------------------------------------------------- */
int oracle_kpm_eta(int64_t N, const int64_t* rowptr, const int32_t* col,
                   const double* val_ri, double a, double b, const double* v0_ri,
                   int R, int M, double* eta_ri)
{
    if (N <= 0 || R <= 0 || M < 2 || (M % 2) != 0 || a == 0.0) return -1;
    zc* V = (zc*)malloc(sizeof(zc) * (size_t)N * R);
    zc* W = (zc*)malloc(sizeof(zc) * (size_t)N * R);
    zc* d = (zc*)malloc(sizeof(zc) * (size_t)R);
    if (!V || !W || !d) { free(V); free(W); free(d); return -2; }
    zc* eta = (zc*)eta_ri;
    for (int64_t i = 0; i < N * R; ++i) V[i] = v0_ri[2 * i] + I * v0_ri[2 * i + 1];

    /* initialisation: W = nu_1 = Htilde nu_0; eta_0, eta_1 */
    apply_htilde(N, rowptr, col, val_ri, a, b, R, V, W);
    block_dot(N, R, V, V, d);
    for (int r = 0; r < R; ++r) eta[0 * R + r] = d[r];
    block_dot(N, R, W, V, d);
    for (int r = 0; r < R; ++r) eta[1 * R + r] = d[r];

    zc* U = (zc*)malloc(sizeof(zc) * (size_t)N * R);
    if (!U) { free(V); free(W); free(d); return -2; }
    for (int m = 1; m < M / 2; ++m) {
        zc* tmp = V; V = W; W = tmp;          /* V = nu_m, W = nu_{m-1} */
        apply_htilde(N, rowptr, col, val_ri, a, b, R, V, U);
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N * R; ++i) W[i] = 2.0 * U[i] - W[i];  /* nu_{m+1} */
        block_dot(N, R, V, V, d);
        for (int r = 0; r < R; ++r) eta[(2 * m) * R + r] = d[r];
        block_dot(N, R, W, V, d);
        for (int r = 0; r < R; ++r) eta[(2 * m + 1) * R + r] = d[r];
    }
    free(U); free(V); free(W); free(d);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Second, independent path to the moments: mu_n = <nu_0 | nu_n> for every   */
/* n < M straight from the recurrence (M-1 products, no doubling identity).  */
/* out is [R][M] complex (interleaved doubles).                              */
/* ------------------------------------------------------------------------- */
int oracle_kpm_direct(int64_t N, const int64_t* rowptr, const int32_t* col,
                      const double* val_ri, double a, double b, const double* v0_ri,
                      int R, int M, double* out_ri)
{
    if (N <= 0 || R <= 0 || M < 1 || a == 0.0) return -1;
    zc* nu0 = (zc*)malloc(sizeof(zc) * (size_t)N * R);
    zc* prev = (zc*)malloc(sizeof(zc) * (size_t)N * R);
    zc* cur = (zc*)malloc(sizeof(zc) * (size_t)N * R);
    zc* nxt = (zc*)malloc(sizeof(zc) * (size_t)N * R);
    zc* d = (zc*)malloc(sizeof(zc) * (size_t)R);
    if (!nu0 || !prev || !cur || !nxt || !d) {
        free(nu0); free(prev); free(cur); free(nxt); free(d); return -2;
    }
    zc* out = (zc*)out_ri;
    for (int64_t i = 0; i < N * R; ++i) nu0[i] = v0_ri[2 * i] + I * v0_ri[2 * i + 1];
    memcpy(cur, nu0, sizeof(zc) * (size_t)N * R);
    block_dot(N, R, nu0, cur, d);
    for (int r = 0; r < R; ++r) out[(int64_t)r * M + 0] = d[r];
    for (int n = 1; n < M; ++n) {
        apply_htilde(N, rowptr, col, val_ri, a, b, R, cur, nxt);
        if (n >= 2)
            for (int64_t i = 0; i < N * R; ++i) nxt[i] = 2.0 * nxt[i] - prev[i];
        zc* tmp = prev; prev = cur; cur = nxt; nxt = tmp;
        block_dot(N, R, nu0, cur, d);
        for (int r = 0; r < R; ++r) out[(int64_t)r * M + n] = d[r];
    }
    free(nu0); free(prev); free(cur); free(nxt); free(d);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Random-phase start block from a counter-based generator (reading of the
 * start-vector step of the stochastic trace, section "Problem Description",
 * whose distribution the paper does not fix).  Generator: SplitMix64
 * (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014): state advances by the odd constant 0x9E3779B97F4A7C15 and
 * each output is the state passed through the 64-bit finaliser below.
 * Element (i, r) of an [N][R] block (counter c = i R + r) draws the output
 * for state key + (c + 1) * gamma with key = mix(seed + gamma); u is its top
 * 53 bits over 2^53 and the element is exp(2 pi i u) / sqrt(N).            */
#define SM_GAMMA 0x9E3779B97F4A7C15ULL

static uint64_t sm_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t oracle_splitmix64_next(uint64_t* state)
{
    *state += SM_GAMMA;
    return sm_mix(*state);
}

void oracle_phase_block(int64_t N, int R, uint64_t seed, double* out_ri)
{
    const uint64_t key = sm_mix(seed + SM_GAMMA);
    const double scale = 1.0 / sqrt((double)N);
    for (int64_t c = 0; c < N * (int64_t)R; ++c) {
        const uint64_t z = sm_mix(key + (uint64_t)(c + 1) * SM_GAMMA);
        const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
        const double phi = 6.283185307179586476925286766559 * u;   /* 2 pi */
        out_ri[2 * c] = cos(phi) * scale;
        out_ri[2 * c + 1] = sin(phi) * scale;
    }
}

/* Disorder potential V_n = gamma (u_n - 1/2) ~ U[-gamma/2, gamma/2) of the
 * onsite term of eq. "Ham", drawn from the same counter-based SplitMix64 for
 * Hamiltonians built without a caller array: site n takes counter n under
 * the key mix(seed + 2 gamma_sm), the second output of SplitMix64 started at
 * `seed` (the start block takes the first).                               */
void oracle_potential_counter(int64_t nsite, double gamma, uint64_t seed, double* out)
{
    const uint64_t key = sm_mix(seed + 2 * SM_GAMMA);
    for (int64_t n = 0; n < nsite; ++n) {
        const uint64_t z = sm_mix(key + (uint64_t)(n + 1) * SM_GAMMA);
        const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
        out[n] = gamma * (u - 0.5);
    }
}
