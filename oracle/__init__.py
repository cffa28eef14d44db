"""Plain CPU oracle for the KPM density-of-states path (arXiv:1410.5242).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_1410_5242_amd``) and never imports it.

The heavy loops (Hamiltonian construction, Chebyshev recurrence, scalar
products) live in ``kpm_oracle.c`` (plain C, double complex, CRS).  This
module wraps them with ctypes and adds the cheap steps that turn moments into
a spectrum (section "Problem Description"): the moment doubling identity, the
damping kernels and the density-of-states reconstruction, plus the dense
brute-force and closed-form references used to pin the oracle.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import build_oracle

_LIB = None


def lib():
    """Load (building once if absent) the compiled oracle."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(build_oracle.LIB):
            build_oracle.build()
        L = ctypes.CDLL(build_oracle.LIB)
        p = ctypes.c_void_p
        L.oracle_ti_build.restype = ctypes.c_int64
        L.oracle_ti_build.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, p,
                                      ctypes.c_double, p, p, p, p, ctypes.c_int64]
        L.oracle_gershgorin.restype = None
        L.oracle_gershgorin.argtypes = [ctypes.c_int64, p, p, p, p, p]
        L.oracle_kpm_eta.restype = ctypes.c_int
        L.oracle_kpm_eta.argtypes = [ctypes.c_int64, p, p, p, ctypes.c_double,
                                     ctypes.c_double, p, ctypes.c_int, ctypes.c_int, p]
        L.oracle_kpm_direct.restype = ctypes.c_int
        L.oracle_kpm_direct.argtypes = L.oracle_kpm_eta.argtypes
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_threads.argtypes = []
        L.oracle_set_threads.restype = None
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_splitmix64_next.restype = ctypes.c_uint64
        L.oracle_splitmix64_next.argtypes = [p]
        L.oracle_phase_block.restype = None
        L.oracle_phase_block.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, p]
        L.oracle_potential_counter.restype = None
        L.oracle_potential_counter.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, p]
        L.oracle_block_dot.restype = None
        L.oracle_block_dot.argtypes = [ctypes.c_int64, ctypes.c_int, p, p, p]
        _LIB = L
    return _LIB


def splitmix64_sequence(state: int, n: int) -> list:
    """First n outputs of SplitMix64 (Steele, Lea, Flood 2014) from the given state."""
    st = np.array([state], dtype=np.uint64)
    return [int(lib().oracle_splitmix64_next(_ptr(st))) for _ in range(n)]


def phase_block_counter(N: int, R: int, seed: int) -> np.ndarray:
    """[N][R] random-phase start block exp(2 pi i u_ir)/sqrt(N), u from SplitMix64 at counter
    i R + r (reading of the start-vector step; see kpm_oracle.c)."""
    out = np.zeros(2 * N * R, dtype=np.float64)
    lib().oracle_phase_block(int(N), int(R), int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(out))
    return out.view(np.complex128).reshape(N, R)


def potential_counter(L, gamma: float, seed: int) -> np.ndarray:
    """Site potentials V_n = gamma (u_n - 1/2) from the counter generator (x fastest), for
    Hamiltonians built without a caller potential (see kpm_oracle.c)."""
    n = int(L[0]) * int(L[1]) * int(L[2])
    out = np.zeros(n, dtype=np.float64)
    lib().oracle_potential_counter(n, float(gamma), int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(out))
    return out


def block_dot(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Column scalar products <x_r|y_r> = sum_i conj(x_ir) y_ir of two [N][R] blocks, by the
    pairwise summation the moment recurrence uses (complex [R])."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.ascontiguousarray(y, dtype=np.complex128)
    if x.ndim == 1:
        x, y = x[:, None], y[:, None]
    if x.shape != y.shape:
        raise ValueError("blocks differ in shape")
    N, R = x.shape
    out = np.zeros(R, dtype=np.complex128)
    lib().oracle_block_dot(N, R, _ptr(x.view(np.float64)), _ptr(y.view(np.float64)), _ptr(out.view(np.float64)))
    return out


def lib_threads() -> int:
    """OpenMP threads the oracle's row loops run on."""
    return int(lib().oracle_threads())


def set_lib_threads(n: int) -> None:
    """Run the oracle's later row loops on n OpenMP threads (results do not depend on n)."""
    lib().oracle_set_threads(int(n))


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


class CSR:
    """Complex CRS matrix: rowptr int64 [N+1], col int32 [nnz], val complex128 [nnz]."""

    def __init__(self, rowptr, col, val):
        self.rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.complex128)

    @property
    def n(self) -> int:
        return len(self.rowptr) - 1

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def dense(self) -> np.ndarray:
        H = np.zeros((self.n, self.n), dtype=np.complex128)
        for i in range(self.n):
            for k in range(self.rowptr[i], self.rowptr[i + 1]):
                H[i, self.col[k]] += self.val[k]
        return H


# --------------------------------------------------------------------------
# Hamiltonian (eq. "Ham") and spectral scaling (Problem Description section)
# --------------------------------------------------------------------------
def ti_hamiltonian(L, potential, t: float = 1.0, periodic=(1, 1, 1)) -> CSR:
    """Topological-insulator Hamiltonian of eq. "Ham" on an Lx x Ly x Lz lattice.

    ``potential`` holds V_n for site n = x + Lx*(y + Ly*z).  Row 4*n + o with
    orbital o = 2*tau + s.  Duplicate entries (sides <= 2) are summed.
    """
    Lx, Ly, Lz = (int(v) for v in L)
    pot = np.ascontiguousarray(potential, dtype=np.float64).reshape(-1)
    if pot.size != Lx * Ly * Lz:
        raise ValueError("potential has the wrong number of sites")
    per = np.ascontiguousarray([int(bool(p)) for p in periodic], dtype=np.int32)
    Lb = lib()
    nnz = Lb.oracle_ti_build(Lx, Ly, Lz, _ptr(per), float(t), _ptr(pot),
                             None, None, None, 0)
    if nnz < 0:
        raise ValueError("invalid lattice")
    N = 4 * Lx * Ly * Lz
    rowptr = np.zeros(N + 1, dtype=np.int64)
    col = np.zeros(nnz, dtype=np.int32)
    val = np.zeros(2 * nnz, dtype=np.float64)
    got = Lb.oracle_ti_build(Lx, Ly, Lz, _ptr(per), float(t), _ptr(pot),
                             _ptr(rowptr), _ptr(col), _ptr(val), nnz)
    assert got == nnz
    return CSR(rowptr, col, val.view(np.complex128))


def gershgorin(H: CSR):
    """Outer Gershgorin bounds (E_min, E_max) of a Hermitian CRS matrix."""
    emin = np.zeros(1)
    emax = np.zeros(1)
    val = np.ascontiguousarray(H.val).view(np.float64)
    lib().oracle_gershgorin(H.n, _ptr(H.rowptr), _ptr(H.col), _ptr(val), _ptr(emin), _ptr(emax))
    return float(emin[0]), float(emax[0])


def scaling(emin: float, emax: float, margin: float = 1.01):
    """(a, b) with Htilde = (H - b)/a: b the centre, a the half-width times ``margin``."""
    b = 0.5 * (emax + emin)
    a = margin * 0.5 * (emax - emin)
    return a, b


# --------------------------------------------------------------------------
# Moments (eq. "eq:kpm_iter" and the blocked algorithm)
# --------------------------------------------------------------------------
def kpm_eta(H: CSR, a: float, b: float, v0: np.ndarray, M: int) -> np.ndarray:
    """Raw scalar products eta[M][R] (complex) of the blocked KPM algorithm.

    ``v0`` is the [N][R] start block (row-major), complex128.
    """
    v0 = np.ascontiguousarray(v0, dtype=np.complex128)
    if v0.ndim == 1:
        v0 = v0[:, None]
    N, R = v0.shape
    if N != H.n:
        raise ValueError("start block has the wrong number of rows")
    eta = np.zeros((M, R), dtype=np.complex128)
    rc = lib().oracle_kpm_eta(H.n, _ptr(H.rowptr), _ptr(H.col),
                              _ptr(np.ascontiguousarray(H.val).view(np.float64)),
                              float(a), float(b), _ptr(v0.view(np.float64)), R, M,
                              _ptr(eta.view(np.float64)))
    if rc != 0:
        raise ValueError(f"oracle_kpm_eta failed ({rc})")
    return eta


def mu_from_eta(eta: np.ndarray) -> np.ndarray:
    """Chebyshev moments mu[R][M] from eta[M][R].

    T_m T_n = (T_{m+n} + T_{|m-n|})/2 gives <nu_m|nu_m> = (mu_{2m} + mu_0)/2 and
    <nu_{m+1}|nu_m> = (mu_{2m+1} + mu_1)/2, hence
    mu_{2m} = 2 eta_{2m} - mu_0 and mu_{2m+1} = 2 Re eta_{2m+1} - mu_1.
    """
    M, R = eta.shape
    mu = np.zeros((R, M))
    mu0 = eta[0].real
    mu1 = eta[1].real
    for m in range(M // 2):
        mu[:, 2 * m] = 2.0 * eta[2 * m].real - mu0
        mu[:, 2 * m + 1] = 2.0 * eta[2 * m + 1].real - mu1
    return mu


def kpm_moments(H: CSR, a: float, b: float, v0: np.ndarray, M: int) -> np.ndarray:
    """mu[R][M] for each start vector (no average over R)."""
    return mu_from_eta(kpm_eta(H, a, b, v0, M))


def kpm_direct(H: CSR, a: float, b: float, v0: np.ndarray, M: int) -> np.ndarray:
    """<nu_0|T_n(Htilde)|nu_0> for n < M by the plain recurrence, complex [R][M]."""
    v0 = np.ascontiguousarray(v0, dtype=np.complex128)
    if v0.ndim == 1:
        v0 = v0[:, None]
    N, R = v0.shape
    out = np.zeros((R, M), dtype=np.complex128)
    rc = lib().oracle_kpm_direct(H.n, _ptr(H.rowptr), _ptr(H.col),
                                 _ptr(np.ascontiguousarray(H.val).view(np.float64)),
                                 float(a), float(b), _ptr(v0.view(np.float64)), R, M,
                                 _ptr(out.view(np.float64)))
    if rc != 0:
        raise ValueError(f"oracle_kpm_direct failed ({rc})")
    return out


# --------------------------------------------------------------------------
# Reconstruction: damping kernels and density of states
# --------------------------------------------------------------------------
def jackson(M: int) -> np.ndarray:
    """Jackson damping factors g_n, n < M (the KPM review's standard form)."""
    q = math.pi / (M + 1)
    n = np.arange(M, dtype=np.float64)
    return ((M - n + 1) * np.cos(q * n) + np.sin(q * n) / math.tan(q)) / (M + 1)


def lorentz(M: int, lam: float) -> np.ndarray:
    """Lorentz damping factors g_n = sinh(lam (1 - n/M)) / sinh(lam)."""
    n = np.arange(M, dtype=np.float64)
    return np.sinh(lam * (1.0 - n / M)) / math.sinh(lam)


def dirichlet(M: int) -> np.ndarray:
    """No damping: g_n = 1 (plain truncation)."""
    return np.ones(M)


def chebyshev_t(n: int, x: np.ndarray) -> np.ndarray:
    """T_n(x) = cos(n arccos x) for |x| <= 1."""
    return np.cos(n * np.arccos(x))


def dos(mu: np.ndarray, g: np.ndarray, a: float, b: float, E: np.ndarray) -> np.ndarray:
    """Density of states per unit energy, normalised so that its integral is mean_r mu_0.

    rho(E) = [g_0 mu_0 + 2 sum_{n>=1} g_n mu_n T_n(x)] / (pi a sqrt(1 - x^2)),
    x = (E - b)/a, with mu averaged over the R start vectors (stochastic
    trace); rho = 0 where |x| >= 1.
    """
    mu = np.atleast_2d(np.asarray(mu, dtype=np.float64))
    mbar = mu.mean(axis=0)
    M = mbar.size
    E = np.asarray(E, dtype=np.float64)
    x = (E - b) / a
    inside = np.abs(x) < 1.0
    xi = x[inside]
    s = g[0] * mbar[0] * np.ones_like(xi)
    for n in range(1, M):
        s += 2.0 * g[n] * mbar[n] * chebyshev_t(n, xi)
    rho = np.zeros_like(x)
    rho[inside] = s / (math.pi * a * np.sqrt(1.0 - xi * xi))
    return rho


def midpoint_grid(K: int, a: float, b: float) -> np.ndarray:
    """K energies at the midpoints of K equal cells of the scaled interval [-1, 1]."""
    k = np.arange(K, dtype=np.float64)
    return b + a * (-1.0 + (2.0 * k + 1.0) / K)


# --------------------------------------------------------------------------
# Dense and closed-form references (used only to pin the oracle)
# --------------------------------------------------------------------------
def dense_moments(Hd: np.ndarray, a: float, b: float, v0: np.ndarray, M: int) -> np.ndarray:
    """mu_n^(r) = sum_k |<k|v_r>|^2 T_n(lambda_k~) from a dense eigendecomposition."""
    lam, U = np.linalg.eigh(Hd)
    lt = (lam - b) / a
    v0 = np.asarray(v0, dtype=np.complex128)
    if v0.ndim == 1:
        v0 = v0[:, None]
    w = np.abs(U.conj().T @ v0) ** 2          # [k][r]
    n = np.arange(M)
    Tn = np.cos(np.outer(n, np.arccos(np.clip(lt, -1.0, 1.0))))  # [n][k]
    return (Tn @ w).T


def lanczos(H: CSR, v0: np.ndarray, steps: int):
    """Lanczos recurrence (section "Problem Description": the scaling may come from
    Lanczos iterations) from the start vector v0, without reorthogonalisation:
    w = H q_j - alpha_j q_j - beta_{j-1} q_{j-1}, alpha_j = Re <q_j|H q_j>,
    beta_j = |w|, q_{j+1} = w / beta_j.  Returns (alpha [steps], beta [steps])."""
    Hd = H.dense()
    q = np.asarray(v0, dtype=np.complex128).reshape(-1)
    q = q / np.linalg.norm(q)
    qp = np.zeros_like(q)
    alpha, beta = np.zeros(steps), np.zeros(steps)
    b_prev = 0.0
    for j in range(steps):
        w = Hd @ q
        alpha[j] = np.vdot(q, w).real
        w = w - alpha[j] * q - b_prev * qp
        beta[j] = np.linalg.norm(w)
        qp, q = q, (w / beta[j] if beta[j] > 0 else np.zeros_like(w))
        b_prev = beta[j]
    return alpha, beta


def tridiagonal_extremes(alpha: np.ndarray, beta: np.ndarray):
    """Smallest and largest eigenvalue of the tridiagonal matrix with diagonal
    alpha and off-diagonal beta[:-1] (the extreme Ritz values)."""
    k = len(alpha)
    T = np.diag(alpha) + np.diag(beta[:k - 1], 1) + np.diag(beta[:k - 1], -1)
    lam = np.linalg.eigvalsh(T)
    return lam[0], lam[-1]


def site_block(N: int, rows) -> np.ndarray:
    """Start block for local quantities: column r is the unit vector of row rows[r]."""
    rows = [int(r) for r in rows]
    v = np.zeros((N, len(rows)), dtype=np.complex128)
    for r, i in enumerate(rows):
        v[i, r] = 1.0
    return v


def plane_wave_block(L, momenta, orbitals) -> np.ndarray:
    """Start block for momentum-resolved quantities: column r is the plane wave
    sum_n exp(i k_r . (x, y, z)_n) |n, orbital_r> / sqrt(sites), site n = x + Lx (y + Ly z)."""
    Lx, Ly, Lz = (int(v) for v in L)
    n = np.arange(Lx * Ly * Lz)
    x, y, z = n % Lx, (n // Lx) % Ly, n // (Lx * Ly)
    v = np.zeros((4 * n.size, len(orbitals)), dtype=np.complex128)
    for r, (k, o) in enumerate(zip(momenta, orbitals)):
        ph = k[0] * x + k[1] * y + k[2] * z
        v[4 * n + int(o), r] = np.exp(1j * ph) / math.sqrt(n.size)
    return v


def clean_ti_spectrum(L: int, t: float = 1.0) -> np.ndarray:
    """Eigenvalues of the clean (V = 0) periodic L^3 lattice from the Bloch form.

    H(k) = (2 - t sum_j cos k_j) Gamma^1 + t sum_j sin k_j Gamma^{j+1}; the
    Gamma matrices anticommute, so E = +-sqrt((2 - t sum cos)^2 + t^2 sum sin^2),
    each twice.
    """
    k = 2.0 * math.pi * np.arange(L) / L
    kx, ky, kz = np.meshgrid(k, k, k, indexing="ij")
    m = 2.0 - t * (np.cos(kx) + np.cos(ky) + np.cos(kz))
    s2 = t * t * (np.sin(kx) ** 2 + np.sin(ky) ** 2 + np.sin(kz) ** 2)
    e = np.sqrt(m * m + s2).reshape(-1)
    return np.sort(np.concatenate([e, e, -e, -e]))


# --------------------------------------------------------------------------
# Traffic and flop model (Table "tab:kpm_analysis", eqs. for V_KPM, B_min)
# --------------------------------------------------------------------------
def flops_per_row_vector(nnzr: float = 13, Fa: int = 2, Fm: int = 6) -> float:
    """Flops per matrix row and vector of the fused sweep: Nnzr (Fa+Fm) + ceil(7Fa/2) + ceil(9Fm/2)."""
    return nnzr * (Fa + Fm) + math.ceil(7 * Fa / 2) + math.ceil(9 * Fm / 2)


def code_balance(R: float, nnzr: float = 13, Sd: int = 16, Si: int = 4, Fa: int = 2, Fm: int = 6) -> float:
    """Minimum code balance B_min(R) in bytes per flop of the blocked sweep."""
    return (nnzr / R * (Sd + Si) + 3 * Sd) / flops_per_row_vector(nnzr, Fa, Fm)


def sweep_bytes(N: int, nnz: int, R: int, Sd: int = 16, Si: int = 4) -> int:
    """Minimum bytes per blocked sweep: Nnz (Sd + Si) + 3 R Sd N."""
    return nnz * (Sd + Si) + 3 * R * Sd * N
