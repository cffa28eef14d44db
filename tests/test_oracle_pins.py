"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own code path: a Kronecker
construction of eq. "Ham", the Bloch-band closed form of the clean lattice,
dense eigendecomposition, the diagonal (t = 0) closed form, the exact trace
with an identity start block, the Chebyshev product identity checked against
the direct recurrence, the sum rule and positivity of the Jackson kernel, the
closed form of the Lorentz-damped delta function and its Fejer limit, exactly
rounded sums (math.fsum) for the pairwise scalar products, and the
code-balance numbers printed in the paper.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_1410_5242_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# eq. "Ham": independent construction with Kronecker products
# --------------------------------------------------------------------------
def _pauli():
    s0 = np.eye(2, dtype=complex)
    sx = np.array([[0, 1], [1, 0]], dtype=complex)
    sy = np.array([[0, -1j], [1j, 0]], dtype=complex)
    sz = np.array([[1, 0], [0, -1]], dtype=complex)
    return s0, sx, sy, sz


def _gammas():
    s0, sx, sy, sz = _pauli()
    return [np.eye(4, dtype=complex), np.kron(sz, s0), np.kron(sx, sx),
            np.kron(sx, sy), np.kron(sx, sz)]


def _shift(L, periodic):
    """S[m, n] = 1 where m = n + 1 along one axis of length L."""
    S = np.zeros((L, L))
    for n in range(L):
        m = n + 1
        if m == L:
            if not periodic:
                continue
            m = 0
        S[m, n] += 1.0
    return S


def kron_hamiltonian(L, pot, t, periodic):
    """H = sum_n V_n |n><n| (x) G0 + 1 (x) 2 G1 - t sum_j [S_j (x) (G1 - i G_{j+1})/2 + h.c.]."""
    Lx, Ly, Lz = L
    G = _gammas()
    ns = Lx * Ly * Lz
    H = np.kron(np.diag(pot), G[0]) + np.kron(np.eye(ns), 2.0 * G[1])
    eye = [np.eye(Lx), np.eye(Ly), np.eye(Lz)]
    for j in range(3):
        parts = list(eye)
        parts[j] = _shift(L[j], periodic[j])
        # site index n = x + Lx*(y + Ly*z): z is the slowest factor
        Ssite = np.kron(parts[2], np.kron(parts[1], parts[0]))
        hop = -t * np.kron(Ssite, (G[1] - 1j * G[j + 2]) / 2.0)
        H = H + hop + hop.conj().T
    return H


@pytest.mark.parametrize("L,periodic,t", [
    ((3, 4, 5), (1, 1, 1), 1.0),
    ((3, 3, 4), (1, 1, 0), 1.3),
    ((4, 3, 3), (0, 1, 1), 0.7),
    ((2, 3, 3), (1, 1, 1), 1.0),
    ((1, 3, 2), (1, 0, 1), 1.0),
])
def test_builder_matches_kronecker_form(L, periodic, t):
    pot = inputs.potential(L, 1.5, 7)
    H = O.ti_hamiltonian(L, pot, t=t, periodic=periodic)
    ref = kron_hamiltonian(L, pot, t, periodic)
    assert np.abs(H.dense() - ref).max() <= 1e-15


def test_builder_invariants():
    L = (5, 4, 3)
    pot = inputs.potential(L, 2.0, 3)
    t = 1.0
    H = O.ti_hamiltonian(L, pot, t=t)
    Hd = H.dense()
    N = H.n
    assert N == 4 * 5 * 4 * 3
    assert np.array_equal(Hd, Hd.conj().T)               # exactly Hermitian
    assert np.all(np.diff(H.rowptr) == 13)               # 13 entries per row, sides >= 3
    assert abs(np.trace(Hd).real / N - pot.mean()) < 1e-14
    # tr(H^2)/N = mean(V^2) + 4 + 3 t^2 (onsite 2 Gamma^1, six hop blocks of Frobenius norm^2 2 t^2 per site)
    assert abs(np.trace(Hd @ Hd).real / N - (np.mean(pot ** 2) + 4 + 3 * t * t)) < 1e-12
    # values are exactly V_n +- 2, +-t/2 and +-i t/2
    mags = np.unique(np.round(np.abs(H.val[H.col != np.repeat(np.arange(N), 13)]), 15))
    assert np.allclose(mags, [t / 2])


def test_builder_side_two_cancels():
    # forward and backward hops land on the same block; the Gamma^{j+1} parts cancel
    H = O.ti_hamiltonian((2, 2, 2), np.zeros(8))
    assert np.all(np.abs(H.val[np.abs(H.val) > 0]) > 0)
    nz = np.array([np.count_nonzero(np.abs(H.dense()[i]) > 0) for i in range(H.n)])
    assert np.all(nz == 4)


def test_clean_spectrum_closed_form():
    for L in (3, 4, 6):
        H = O.ti_hamiltonian((L, L, L), np.zeros(L ** 3))
        ev = np.linalg.eigvalsh(H.dense())
        assert np.abs(ev - O.clean_ti_spectrum(L)).max() < 1e-12
    # band edges of the clean t = 1 lattice: |E| in [1, 5] (k = 0 gives 1, k = (pi,pi,pi) gives 5)
    ev = np.linalg.eigvalsh(O.ti_hamiltonian((4, 4, 4), np.zeros(64)).dense())
    assert abs(ev.max() - 5.0) < 1e-12 and abs(ev.min() + 5.0) < 1e-12
    assert abs(np.abs(ev).min() - 1.0) < 1e-12


def test_gershgorin_and_scaling():
    H = O.ti_hamiltonian((4, 4, 4), np.zeros(64))
    emin, emax = O.gershgorin(H)
    assert emin == -8.0 and emax == 8.0        # |diag| = 2, twelve hops of size t/2
    a, b = O.scaling(emin, emax)
    assert b == 0.0 and abs(a - 8.08) < 1e-15
    pot = inputs.potential((4, 4, 4), 1.0, 0)
    emin, emax = O.gershgorin(O.ti_hamiltonian((4, 4, 4), pot))
    assert abs(emin - (pot.min() - 8.0)) < 1e-14 and abs(emax - (pot.max() + 8.0)) < 1e-14


# --------------------------------------------------------------------------
# eq. "eq:kpm_iter", moments and the doubling identity
# --------------------------------------------------------------------------
def _setup(L, gamma, seed, R, t=1.0):
    pot = inputs.potential(L, gamma, seed)
    H = O.ti_hamiltonian(L, pot, t=t)
    a, b = O.scaling(*O.gershgorin(H))
    v0 = inputs.phase_block(H.n, R, seed)
    return H, a, b, v0


def test_moments_match_dense_eigendecomposition_small():
    H, a, b, v0 = _setup((3, 3, 3), 1.0, 1, 3)
    mu = O.kpm_moments(H, a, b, v0, 64)
    ref = O.dense_moments(H.dense(), a, b, v0, 64)
    assert np.abs(mu - ref).max() <= 1e-12
    assert np.abs(mu[:, 0] - 1.0).max() <= 1e-14


def test_moments_of_an_irregular_matrix_match_its_eigendecomposition():
    # a general Hermitian matrix with empty rows and a long tail of row
    # lengths (the SELL-C-sigma workloads): the oracle's recurrence against
    # mu_n = sum_k |<k|v>|^2 cos(n arccos x_k) from eigh, and its Gershgorin
    # interval against the spectrum
    N, R, M = 120, 3, 96
    rowptr, col, val = inputs.random_hermitian_csr(N, mean_offdiag=8.0, empty_frac=0.05, seed=9)
    H = O.CSR(rowptr, col, val)
    lam, U = np.linalg.eigh(H.dense())
    emin, emax = O.gershgorin(H)
    assert emin <= lam[0] and lam[-1] <= emax
    a, b = O.scaling(emin, emax)
    v0 = inputs.phase_block(N, R, 1)
    mu = O.kpm_moments(H, a, b, v0, M)
    x = np.clip((lam - b) / a, -1.0, 1.0)
    w = np.abs(U.conj().T @ v0) ** 2                               # [N eigenvalues][R]
    T = np.cos(np.arange(M)[:, None] * np.arccos(x)[None, :])      # [M][N]
    assert np.abs(mu - (T @ w).T).max() <= 1e-12


@pytest.mark.slow
def test_moments_match_dense_eigendecomposition_8cubed():
    # 8^3 lattice, gamma = 1, seed 0, R = 1, M = 128 (N = 2048)
    H, a, b, v0 = _setup((8, 8, 8), 1.0, 0, 1)
    mu = O.kpm_moments(H, a, b, v0, 128)
    ref = O.dense_moments(H.dense(), a, b, v0, 128)
    assert np.abs(mu - ref).max() <= 1e-11


def test_doubling_identity_against_direct_recurrence():
    H, a, b, v0 = _setup((4, 3, 5), 2.0, 5, 4)
    M = 200
    eta = O.kpm_eta(H, a, b, v0, M)
    mu = O.mu_from_eta(eta)
    direct = O.kpm_direct(H, a, b, v0, M)
    assert np.abs(mu - direct.real).max() <= 1e-13
    assert np.abs(direct.imag).max() <= 1e-14      # <v|T_n(H)|v> is real for Hermitian H
    assert np.all(eta[0::2].imag == 0.0)           # <v|v> has an exactly zero imaginary part
    assert np.abs(eta[1::2].imag).max() <= 1e-15
    assert np.all(eta[0::2].real >= 0.0)
    assert np.abs(mu).max() <= 1.0 + 1e-12


def test_diagonal_hamiltonian_closed_form():
    # t = 0: H is diagonal, nu_m = T_m(Htilde) v elementwise, and with |v_i|^2 = 1/N
    # every start vector gives mu_n = (1/N) sum_i T_n(h_ii~) exactly
    L = (3, 4, 2)
    pot = inputs.potential(L, 3.0, 11)
    H = O.ti_hamiltonian(L, pot, t=0.0)
    a, b = O.scaling(*O.gershgorin(H))
    v0 = inputs.phase_block(H.n, 3, 2)
    M = 100
    mu = O.kpm_moments(H, a, b, v0, M)
    h = (np.real(np.diag(H.dense())) - b) / a
    n = np.arange(M)
    ref = np.cos(np.outer(n, np.arccos(h))).mean(axis=1)
    assert np.abs(mu - ref[None, :]).max() <= 1e-13


def test_identity_block_gives_exact_trace():
    # R = N with V0 = identity: sum_r mu_n^(r) = tr T_n(Htilde) = sum over the Bloch bands
    L = 3
    H = O.ti_hamiltonian((L, L, L), np.zeros(L ** 3))
    a, b = O.scaling(*O.gershgorin(H))
    N = H.n
    v0 = np.eye(N, dtype=complex)
    M = 40
    mu = O.kpm_moments(H, a, b, v0, M)
    tr = mu.sum(axis=0)
    E = O.clean_ti_spectrum(L)
    n = np.arange(M)
    ref = np.cos(np.outer(n, np.arccos(E / a))).sum(axis=1)
    assert np.abs(tr - ref).max() <= 1e-10
    assert np.abs(tr[1::2]).max() <= 1e-10         # symmetric spectrum, b = 0
    assert abs(tr[0] - N) <= 1e-10


# --------------------------------------------------------------------------
# Local and momentum-resolved moments (deterministic start vectors)
# --------------------------------------------------------------------------
def _bloch(k, t=1.0):
    """4 x 4 Bloch matrix of the clean lattice from eq. "Ham": a plane wave
    exp(i k . r) u is mapped to exp(i k . r) H(k) u with
    H(k) = 2 Gamma^1 + sum_j [T_j exp(-i k_j) + T_j^dagger exp(i k_j)],
    T_j = -t (Gamma^1 - i Gamma^{j+1}) / 2."""
    G = _gammas()
    Hk = 2.0 * G[1]
    for j in range(3):
        T = -0.5 * t * (G[1] - 1j * G[j + 2])
        Hk = Hk + T * np.exp(-1j * k[j]) + T.conj().T * np.exp(1j * k[j])
    return Hk


def test_plane_wave_moments_match_bloch_closed_form():
    # on the clean periodic lattice a plane wave of a lattice momentum stays in
    # the 4-dimensional Bloch subspace: mu_n = [T_n((H(k) - b) / a)]_oo
    L = (4, 6, 5)
    H = O.ti_hamiltonian(L, np.zeros(4 * 6 * 5))
    a, b = O.scaling(*O.gershgorin(H))
    ks = [(0.0, 0.0, 0.0), (2 * math.pi / 4, 0.0, 0.0), (math.pi, 2 * math.pi / 6 * 2, 2 * math.pi / 5),
          (2 * math.pi * 3 / 4, 2 * math.pi * 5 / 6, 2 * math.pi * 4 / 5)]
    kk = [k for k in ks for _ in range(4)]
    oo = [o for _ in ks for o in range(4)]
    M = 64
    mu = O.kpm_moments(H, a, b, O.plane_wave_block(L, kk, oo), M)
    n = np.arange(M)
    for i, k in enumerate(ks):
        lam, U = np.linalg.eigh((_bloch(k) - b * np.eye(4)) / a)
        Tn = np.cos(np.outer(n, np.arccos(np.clip(lam, -1, 1))))   # [n][band]
        for o in range(4):
            ref = Tn @ (np.abs(U[o, :]) ** 2)
            assert np.abs(mu[4 * i + o] - ref).max() <= 1e-12, (k, o)


def test_site_moments_match_eigendecomposition():
    # local moments <e_i|T_n(Htilde)|e_i> = sum_k |U_ik|^2 T_n(lambda_k)
    L = (3, 4, 3)
    pot = inputs.potential(L, 2.0, 5)
    H = O.ti_hamiltonian(L, pot, periodic=(1, 1, 0))
    a, b = O.scaling(*O.gershgorin(H))
    rows = [0, 5, 17, H.n - 1]
    M = 48
    mu = O.kpm_moments(H, a, b, O.site_block(H.n, rows), M)
    lam, U = np.linalg.eigh((H.dense() - b * np.eye(H.n)) / a)
    Tn = np.cos(np.outer(np.arange(M), np.arccos(np.clip(lam, -1, 1))))
    for r, i in enumerate(rows):
        assert np.abs(mu[r] - Tn @ (np.abs(U[i, :]) ** 2)).max() <= 1e-12


def test_lanczos_extremes_converge_inside_the_spectrum():
    # Ritz values lie inside [lambda_min, lambda_max] and the extreme ones
    # converge to the extreme eigenvalues (dense eigvalsh; clean lattice: +-5)
    for L, pot in (((3, 4, 3), inputs.potential((3, 4, 3), 2.0, 1)), ((4, 4, 4), np.zeros(64))):
        H = O.ti_hamiltonian(L, pot, periodic=(1, 1, 1))
        lam = np.linalg.eigvalsh(H.dense())
        v0 = inputs.phase_block(H.n, 1, 7)[:, 0]
        lo10, hi10 = O.tridiagonal_extremes(*O.lanczos(H, v0, 10))
        lo, hi = O.tridiagonal_extremes(*O.lanczos(H, v0, 80))
        assert lam[0] - 1e-10 <= lo <= lo10 and hi10 <= hi <= lam[-1] + 1e-10
        assert abs(lo - lam[0]) <= 1e-8 and abs(hi - lam[-1]) <= 1e-8
        if not pot.any():
            assert abs(hi - 5.0) <= 1e-8 and abs(lo + 5.0) <= 1e-8


# --------------------------------------------------------------------------
# Reconstruction: damping kernels and density of states
# --------------------------------------------------------------------------
def test_jackson_kernel_properties():
    for M in (16, 128, 2000):
        g = O.jackson(M)
        assert abs(g[0] - 1.0) < 1e-14
        assert np.all(np.diff(g) < 0) and g[-1] > 0
    assert np.allclose(O.dirichlet(7), 1.0)
    gl = O.lorentz(64, 4.0)
    assert abs(gl[0] - 1.0) < 1e-15 and np.all(np.diff(gl) < 0)


def _lorentz_cosine_sum(M, lam, phi):
    """C(phi) = sum_{n<M} g_n cos(n phi) for g_n = sinh(lam (1 - n/M)) / sinh(lam), in closed
    form: sinh(lam (1 - n/M)) = (e^lam q^n - e^-lam q^-n) / 2 with q = e^(-lam/M), and
    sum_{n<M} z^n = (1 - z^M) / (1 - z) for z = q^(+-1) e^(i phi)."""
    def geo(q):
        z = q * np.exp(1j * phi)
        return ((1.0 - z ** M) / (1.0 - z)).real
    q = math.exp(-lam / M)
    return (math.exp(lam) * geo(q) - math.exp(-lam) * geo(1.0 / q)) / (2.0 * math.sinh(lam))


@pytest.mark.parametrize("M,lam", [(64, 4.0), (512, 4.0), (2000, 1.5)])
def test_lorentz_delta_matches_closed_form(M, lam):
    # exact moments of one eigenvalue at x0 = cos(t0): mu_n = cos(n t0).  With
    # x = cos(t), 2 g_n cos(n t0) cos(n t) = g_n [cos(n (t + t0)) + cos(n (t - t0))], so
    # rho(x) = [C(t + t0) + C(t - t0) - g_0] / (pi sin t), C the damped cosine sum
    K = 4096
    E = O.midpoint_grid(K, 1.0, 0.0)
    th = np.arccos(E)
    for x0 in (-0.7, 0.0, 0.3):
        t0 = math.acos(x0)
        mu = np.cos(np.arange(M) * t0)[None, :]
        rho = O.dos(mu, O.lorentz(M, lam), 1.0, 0.0, E)
        ref = (_lorentz_cosine_sum(M, lam, th + t0) + _lorentz_cosine_sum(M, lam, th - t0) - 1.0) / (
            math.pi * np.sin(th))
        assert np.abs(rho - ref).max() <= 1e-9 * np.abs(ref).max()
        assert rho.min() > 0.0                      # the Lorentz kernel is positive
        assert abs(E[np.argmax(rho)] - x0) < lam / M  # within the broadening width


def test_lorentz_kernel_reduces_to_fejer():
    # sinh(lam (1 - n/M)) / sinh(lam) = (1 - n/M) (1 + O(lam^2)): as lam -> 0 the
    # Lorentz factors become the Fejer factors 1 - n/M, a positive kernel
    for M in (16, 128, 2000):
        n = np.arange(M)
        fejer = 1.0 - n / M
        assert np.abs(O.lorentz(M, 1e-5) - fejer).max() <= 1e-10
        g = O.lorentz(M, 1e-3)
        assert np.abs(g - fejer).max() <= 1e-6 and np.all(g <= fejer + 1e-15)
    M, K = 256, 4096
    E = O.midpoint_grid(K, 1.0, 0.0)
    for x0 in (-0.4, 0.5):
        mu = np.cos(np.arange(M) * np.arccos(x0))[None, :]
        assert O.dos(mu, O.lorentz(M, 1e-6), 1.0, 0.0, E).min() > -1e-9


def test_jackson_delta_is_positive_and_normalised():
    # exact moments of a single eigenvalue at x0: mu_n = T_n(x0)
    M, K = 256, 4096
    for x0 in (-0.7, 0.0, 0.3):
        mu = np.cos(np.arange(M) * np.arccos(x0))[None, :]
        E = O.midpoint_grid(K, 1.0, 0.0)
        rho = O.dos(mu, O.jackson(M), 1.0, 0.0, E)
        assert rho.min() > -1e-12                  # Jackson is a positive kernel
        assert abs(rho.sum() * (2.0 / K) - 1.0) < 1e-6
        assert abs(E[np.argmax(rho)] - x0) < 2.0 / K + 1e-12
        rho_d = O.dos(mu, O.dirichlet(M), 1.0, 0.0, E)
        assert rho_d.min() < -1e-3                 # plain truncation rings (Gibbs)


def test_dos_of_diagonal_two_level_system():
    # t = 0, gamma = 0: H = diag(+-2), so rho(E) = (delta(E-2) + delta(E+2))/2
    L = (2, 2, 2)
    H = O.ti_hamiltonian(L, np.zeros(8), t=0.0)
    a, b = O.scaling(*O.gershgorin(H))
    assert (a, b) == (2.02, 0.0)
    v0 = inputs.phase_block(H.n, 2, 0)
    M, K = 512, 8192
    mu = O.kpm_moments(H, a, b, v0, M)
    E = O.midpoint_grid(K, a, b)
    rho = O.dos(mu, O.jackson(M), a, b, E)
    dE = 2.0 * a / K
    # midpoint rule against the 1/sqrt(1-x^2) weight near x = +-0.99: error ~1e-6
    assert abs(rho.sum() * dE - 1.0) < 1e-5
    assert abs(rho[E > 0].sum() * dE - 0.5) < 1e-5
    assert rho[np.abs(np.abs(E) - 2.0) > 0.3].max() < 1e-3 * rho.max()


def test_clean_lattice_dos_gap_and_band_edges():
    L = 12
    H = O.ti_hamiltonian((L, L, L), np.zeros(L ** 3))
    a, b = O.scaling(*O.gershgorin(H))
    v0 = inputs.phase_block(H.n, 4, 3)
    M = 256
    mu = O.kpm_moments(H, a, b, v0, M)
    E = O.midpoint_grid(2048, a, b)
    rho = O.dos(mu, O.jackson(M), a, b, E)
    dE = 2.0 * a / 2048
    assert abs(rho.sum() * dE - 1.0) < 1e-6
    width = 4 * math.pi * a / M                   # a few Jackson widths
    peak = rho.max()
    assert rho[np.abs(E) < 1.0 - width].max() < 0.02 * peak
    assert rho[np.abs(E) > 5.0 + width].max() < 0.02 * peak


# --------------------------------------------------------------------------
# Traffic and flop model printed in the paper
# --------------------------------------------------------------------------
def test_code_balance_matches_printed_values():
    g = json.load(open(os.path.join(GOLDEN, "code_balance.json")))
    f = O.flops_per_row_vector(g["N_nzr"], g["F_a"], g["F_m"])
    assert f == g["flops_per_row_per_vector"]
    assert g["N_nzr"] * (g["S_d"] + g["S_i"]) == g["bytes_numerator_over_R"]
    assert 3 * g["S_d"] == g["bytes_constant"]
    d = g["printed_decimals"]
    assert round(O.code_balance(1), d) == g["B_min_R1"]
    assert round(O.code_balance(1e15), d) == g["B_min_Rinf"]
    # general SpMV, matrix traffic only: (S_d + S_i) / (F_a + F_m)
    assert (8 + 4) / (1 + 1) == g["general_spmv_min_balance_double"]
    assert (16 + 4) / (2 + 6) == g["general_spmv_min_balance_double_complex"]


def test_sweep_bytes_model():
    # V_KPM per sweep of the blocked algorithm: Nnz (S_d + S_i) + 3 R S_d N
    N, nnz, R = 1048576, 13 * 1048576, 32
    assert O.sweep_bytes(N, nnz, R) == 272629760 + 1610612736
    Bmin = O.sweep_bytes(N, nnz, R) / (R * N * O.flops_per_row_vector())
    assert abs(Bmin - O.code_balance(R)) < 1e-15


# --------------------------------------------------------------------------
# Start-block generator (counter-based SplitMix64)
# --------------------------------------------------------------------------
def test_splitmix64_matches_published_sequence():
    import json
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "splitmix64.json")))
    got = O.splitmix64_sequence(g["state"], len(g["outputs_hex"]))
    assert got == [int(h, 16) for h in g["outputs_hex"]]


def test_phase_block_counter_properties():
    N, R = 997, 6
    v = O.phase_block_counter(N, R, 11)
    # every element has modulus 1/sqrt(N); every column has unit norm
    assert np.abs(np.abs(v) - 1.0 / np.sqrt(N)).max() <= 1e-15
    assert np.abs(np.sum(np.abs(v) ** 2, axis=0) - 1.0).max() <= 1e-13
    # counter property: element (i, r) depends only on (seed, i R + r) and N
    flat = O.phase_block_counter(N * R, 1, 11).reshape(-1) * np.sqrt(N * R) / np.sqrt(N)
    assert np.abs(flat - v.reshape(-1)).max() <= 1e-15
    # deterministic, seed-dependent, phases uniform on the circle
    assert np.array_equal(v, O.phase_block_counter(N, R, 11))
    w = O.phase_block_counter(N, R, 12)
    assert np.abs(v - w).max() > 1e-3
    ph = np.angle(O.phase_block_counter(200_000, 1, 5)[:, 0]) % (2 * np.pi)
    hist, _ = np.histogram(ph, bins=16, range=(0, 2 * np.pi))
    chi2 = np.sum((hist - 12_500.0) ** 2 / 12_500.0)
    assert chi2 < 50.0            # 15 degrees of freedom: p < 1e-5 for a fair generator
    # the moment estimate of a random-phase block: mu_0 = sum |v|^2 = 1 exactly per column
    assert abs(np.vdot(v[:, 0], v[:, 0]).real - 1.0) <= 1e-13


# --------------------------------------------------------------------------
# Scalar products: pairwise summation against exactly rounded sums
# --------------------------------------------------------------------------
def _fsum_c(z):
    return complex(math.fsum(z.real.tolist()), math.fsum(z.imag.tolist()))


def test_block_dot_is_within_the_pairwise_bound_at_a_million_rows():
    # The oracle's scalar product must certify 1e-12 moments at N = 2^20 rows.
    # Its products conj(x) y are rounded exactly as NumPy rounds them; math.fsum
    # gives their exactly rounded sum, so the difference is the summation error
    # alone, which for pairwise summation with leaves of 8 rows is below
    # (7 + log2(N / 8)) u sum |x| |y| = 24 u (a running sum over these rows
    # errs by about 10x more, 2e-14 to 3e-14 here)
    N, R = 1 << 20, 2
    rng = np.random.default_rng(3)
    x = rng.standard_normal((N, R)) + 1j * rng.standard_normal((N, R))
    x /= np.sqrt((np.abs(x) ** 2).sum(axis=0))
    y = x + 1e-3 * (rng.standard_normal((N, R)) + 1j * rng.standard_normal((N, R)))
    u = 2.0 ** -53
    for a, b in ((x, x), (y, x), (x, y)):
        got = O.block_dot(a, b)
        for r in range(R):
            p = np.conj(a[:, r]) * b[:, r]
            bound = 24 * u * np.abs(p).sum()
            assert abs(got[r] - _fsum_c(p)) <= bound
    # a random-phase unit block: every column's squared norm is 1 to 1e-15
    v = O.phase_block_counter(N, 4, 9)
    assert np.abs(O.block_dot(v, v) - 1.0).max() <= 1e-15


def test_block_dot_small_cases():
    # leaves of one to nine rows, a single row, conjugation of the bra
    rng = np.random.default_rng(4)
    for N in (1, 2, 7, 8, 9, 17, 1000):
        x = rng.standard_normal((N, 3)) + 1j * rng.standard_normal((N, 3))
        y = rng.standard_normal((N, 3)) + 1j * rng.standard_normal((N, 3))
        got = O.block_dot(x, y)
        for r in range(3):
            assert abs(got[r] - np.vdot(x[:, r], y[:, r])) <= 1e-13 * max(1.0, np.abs(x[:, r] * y[:, r]).sum())
    assert O.block_dot(np.array([1j]), np.array([1.0]))[0] == -1j


def test_potential_counter_follows_the_published_generator():
    # key = second SplitMix64 output of the seed; site n takes output n + 1 of the
    # generator started at the key; V = gamma (u - 1/2) with u the top 53 bits / 2^53
    seed, gamma = 12345, 2.5
    key = O.splitmix64_sequence(seed, 2)[1]
    outs = O.splitmix64_sequence(key, 6)
    ref = [gamma * ((o >> 11) / 2.0 ** 53 - 0.5) for o in outs]
    assert O.potential_counter((6, 1, 1), gamma, seed).tolist() == ref
    v = O.potential_counter((50, 40, 30), 4.0, 7)
    assert v.min() >= -2.0 and v.max() < 2.0
    assert abs(v.mean()) < 0.02 and abs(v.var() - 16.0 / 12.0) < 0.02   # U[-2, 2): var = 4^2 / 12
    assert np.abs(v - O.potential_counter((50, 40, 30), 4.0, 8)).max() > 1.0
