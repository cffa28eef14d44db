"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerances: complex128 moments agree with the oracle to 1e-12 absolute
(relative to mu_0 = 1, since |mu_n| <= mu_0); complex64 storage with FP64
scalar products agrees with the complex128 oracle to 1e-5.  The matrix is
compared bit for bit (its entries are V_n +- 2, +-t/2, +-i t/2).
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_1410_5242_amd import inputs

pytestmark = pytest.mark.gpu

TOL_C128 = 1e-12
TOL_C64 = 1e-5


def kpm():
    from paper_1410_5242_amd import kpm as K
    return K


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch.device("cuda:0")


def oracle_problem(L, gamma, seed, t=1.0, periodic=(1, 1, 1)):
    pot = inputs.potential(L, gamma, seed)
    H = O.ti_hamiltonian(L, pot, t=t, periodic=periodic)
    a, b = O.scaling(*O.gershgorin(H))
    return pot, H, a, b


def sorted_rows(rowptr, col, val):
    out = []
    for i in range(len(rowptr) - 1):
        s, e = rowptr[i], rowptr[i + 1]
        o = np.argsort(col[s:e], kind="stable")
        out.append((col[s:e][o], val[s:e][o]))
    return out


# --------------------------------------------------------------------------
# a1-a2: Hamiltonian and Gershgorin scaling
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L,periodic,t", [
    ((3, 3, 3), (1, 1, 1), 1.0),
    ((5, 4, 7), (1, 1, 1), 0.75),
    ((4, 3, 5), (1, 1, 0), 1.0),
    ((2, 3, 1), (0, 1, 0), 1.25),
])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_hamiltonian_matches_oracle_exactly(L, periodic, t, dtype):
    say("hamiltonian", L, periodic, t, dtype)
    K = kpm()
    pot, Ho, a, b = oracle_problem(L, 2.0, 3, t=t, periodic=periodic)
    H = K.build_hamiltonian(L, pot, t=t, periodic=periodic, dtype=dtype)
    assert H.N == Ho.n and H.width == 13
    assert H.emin == pytest.approx(O.gershgorin(Ho)[0], abs=1e-14)
    assert H.emax == pytest.approx(O.gershgorin(Ho)[1], abs=1e-14)
    assert H.a == pytest.approx(a, rel=1e-15) and H.b == pytest.approx(b, abs=1e-15)
    rp, col, val = K.export_csr(H)
    assert np.array_equal(rp, Ho.rowptr)
    ref_val = Ho.val
    if dtype == "c64":
        ref_val = ref_val.astype(np.complex64).astype(np.complex128)
    for (c1, v1), (c2, v2) in zip(sorted_rows(rp, col, val), sorted_rows(Ho.rowptr, Ho.col, ref_val)):
        assert np.array_equal(c1, c2)
        assert np.array_equal(v1, v2)
    H.close()


# --------------------------------------------------------------------------
# a3-a7: moments through kpm_moments
# --------------------------------------------------------------------------
def gpu_moments(L, pot, v0, M, dtype="c128", t=1.0, periodic=(1, 1, 1), eta=False):
    K = kpm()
    H = K.build_hamiltonian(L, pot, t=t, periodic=periodic, dtype=dtype)
    V0 = torch.from_numpy(v0.astype(np.complex128 if dtype == "c128" else np.complex64)).cuda()
    et = torch.zeros((M, v0.shape[1], 2), dtype=torch.float64, device="cuda") if eta else None
    mu = K.moments(H, V0, M, eta=et)
    torch.cuda.synchronize()
    out = mu.cpu().numpy()
    e = et.cpu().numpy() if eta else None
    H.close()
    return out, e


def test_config1_matches_oracle_and_dense_eigendecomposition():
    # 8x8x8 periodic lattice, gamma = 1, seed 0, R = 1, M = 128, complex128
    L, M = (8, 8, 8), 128
    say("config1")
    pot, Ho, a, b = oracle_problem(L, 1.0, 0)
    v0 = inputs.phase_block(Ho.n, 1, 0)
    mu, _ = gpu_moments(L, pot, v0, M)
    ref = O.kpm_moments(Ho, a, b, v0, M)
    assert np.abs(mu - ref).max() <= TOL_C128
    dense = O.dense_moments(Ho.dense(), a, b, v0, M)
    assert np.abs(mu - dense).max() <= 1e-11
    assert abs(mu[0, 0] - 1.0) <= 1e-14


@pytest.mark.parametrize("R", [1, 2, 4, 8, 16, 32, 64])
def test_moments_every_block_width(R):
    # 7 x 5 x 6 sites: 840 rows, so every tile height leaves a ragged tail
    L, M = (7, 5, 6), 48
    say("moments R", R)
    pot, Ho, a, b = oracle_problem(L, 1.5, R)
    v0 = inputs.phase_block(Ho.n, R, 100 + R)
    mu, eta = gpu_moments(L, pot, v0, M, eta=True)
    ref_eta = O.kpm_eta(Ho, a, b, v0, M)
    ref = O.mu_from_eta(ref_eta)
    assert np.abs(mu - ref).max() <= TOL_C128
    got_eta = eta[..., 0] + 1j * eta[..., 1]
    assert np.abs(got_eta - ref_eta).max() <= TOL_C128
    assert np.all(eta[0::2, :, 1] == 0.0)


def test_moments_open_boundaries_and_many_tiles():
    # open z side (padding slots), 9 x 8 x 10 sites = 2880 rows, R = 32, M = 200
    L, M, R = (9, 8, 10), 200, 32
    say("open boundaries")
    pot, Ho, a, b = oracle_problem(L, 1.0, 4, periodic=(1, 1, 0))
    v0 = inputs.phase_block(Ho.n, R, 5)
    mu, _ = gpu_moments(L, pot, v0, M, periodic=(1, 1, 0))
    ref = O.kpm_moments(Ho, a, b, v0, M)
    assert np.abs(mu - ref).max() <= TOL_C128


def test_moments_minimal_sizes():
    # one site (N = 4, all sides open), M = 2 (only the initialisation sweep)
    K = kpm()
    L = (1, 1, 1)
    say("minimal sizes")
    pot, Ho, a, b = oracle_problem(L, 1.0, 9, periodic=(0, 0, 0))
    for R, M in ((1, 2), (4, 2), (32, 6)):
        v0 = inputs.phase_block(Ho.n, R, 1)
        mu, _ = gpu_moments(L, pot, v0, M, periodic=(0, 0, 0))
        ref = O.kpm_moments(Ho, a, b, v0, M)
        assert np.abs(mu - ref).max() <= TOL_C128


def test_complex64_storage_with_fp64_products():
    L, M, R = (10, 10, 8), 400, 8
    say("c64")
    pot, Ho, a, b = oracle_problem(L, 2.0, 2)
    v0 = inputs.phase_block(Ho.n, R, 2)
    mu, _ = gpu_moments(L, pot, v0, M, dtype="c64")
    ref = O.kpm_moments(Ho, a, b, v0, M)
    err = np.abs(mu - ref).max()
    say("c64 max |dmu|", err)
    assert err <= TOL_C64
    assert err > 0.0                      # it really ran in single precision
    assert np.abs(mu[:, 0] - 1.0).max() <= 1e-6


def test_moments_are_bitwise_deterministic_static_mapping():
    K = kpm()
    L, M, R = (12, 12, 12), 64, 32
    say("determinism")
    pot = inputs.potential(L, 1.0, 0)
    H = K.build_hamiltonian(L, pot)
    V0 = torch.from_numpy(inputs.phase_block(H.N, R, 0)).cuda()
    try:
        K.set_sweep_tuning(dynamic=0)
        m1 = K.moments(H, V0, M).cpu()
        m2 = K.moments(H, V0, M).cpu()
    finally:
        K.reset_sweep_tuning()
    assert torch.equal(m1, m2)
    H.close()


@pytest.mark.parametrize("tuning", [
    dict(lattice=0, dynamic=1), dict(lattice=0, dynamic=1, chunk_tiles=1),
    dict(lattice=0, dynamic=0, prefetch=0), dict(lattice=0, stream=3),
    dict(lattice=0, dynamic=0, pencil=0, xcd_ways=1, chunk_tiles=3),
    dict(lattice=0, wg_per_cu=2, dynamic=1, pencil=5), dict(lattice=2), dict(lattice=2, prefetch=0),
    dict(lattice=2, prefetch=2), dict(lattice=2, prefetch=1),
])
def test_launch_shapes_agree(tuning):
    # the launch shape and site order change only the order of the FP64 sums
    K = kpm()
    L, M, R = (11, 10, 9), 200, 32
    say("launch shape", tuning)
    pot, Ho, a, b = oracle_problem(L, 1.0, 6)
    v0 = inputs.phase_block(Ho.n, R, 6)
    ref = O.kpm_moments(Ho, a, b, v0, M)
    try:
        K.set_sweep_tuning(**tuning)
        mu, _ = gpu_moments(L, pot, v0, M)
    finally:
        K.reset_sweep_tuning()
    assert np.abs(mu - ref).max() <= TOL_C128


# --------------------------------------------------------------------------
# the cache-blocked lattice sweep (R = 32): tile edges, ragged tiles, open sides
# --------------------------------------------------------------------------
LATTICE_GEOMETRIES = [
    ((4, 4, 4), (1, 1, 1)), ((6, 7, 3), (1, 1, 1)), ((3, 3, 3), (1, 1, 1)),
    ((6, 6, 4), (0, 1, 1)), ((4, 10, 5), (1, 0, 1)), ((8, 8, 6), (1, 1, 0)),
    ((2, 3, 5), (0, 1, 1)), ((7, 6, 1), (1, 1, 0)), ((11, 6, 4), (0, 0, 0)), ((10, 3, 9), (1, 1, 1)),
]


@pytest.mark.parametrize("L,periodic", LATTICE_GEOMETRIES)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("vals", [0, 2])
def test_lattice_sweep_matches_oracle(L, periodic, dtype, vals):
    K = kpm()
    M, R = 40, 32
    say("lattice", L, periodic, dtype, "vals", vals)
    pot, Ho, a, b = oracle_problem(L, 1.5, 11, periodic=periodic)
    v0 = inputs.phase_block(Ho.n, R, 12)
    ref_eta = O.kpm_eta(Ho, a, b, v0, M)
    ref = O.mu_from_eta(ref_eta)
    try:
        K.set_sweep_tuning(lattice=2, prefetch=vals)
        H = K.build_hamiltonian(L, pot, periodic=periodic, dtype=dtype)
        assert K.sweep_kernel(H, R) == "lattice_kernel"
        H.close()
        mu, eta = gpu_moments(L, pot, v0, M, dtype=dtype, periodic=periodic, eta=True)
        K.set_sweep_tuning(lattice=0)
        mu_g, _ = gpu_moments(L, pot, v0, M, dtype=dtype, periodic=periodic)
    finally:
        K.reset_sweep_tuning()
    tol = TOL_C128 if dtype == "c128" else TOL_C64
    assert np.abs(mu - ref).max() <= tol
    assert np.abs(mu - mu_g).max() <= (1e-13 if dtype == "c128" else 1e-6)
    if dtype == "c128":
        got_eta = eta[..., 0] + 1j * eta[..., 1]
        assert np.abs(got_eta - ref_eta).max() <= TOL_C128


# blocks wider than 32 columns: the lattice sweep runs once per 32-column
# slice; every slice writes its own columns of W and of the partial sums
WIDE_GEOMETRIES = [LATTICE_GEOMETRIES[i] for i in (1, 3, 4, 6, 8, 9)]


@pytest.mark.parametrize("L,periodic", WIDE_GEOMETRIES)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_wide_lattice_sweep_matches_oracle(L, periodic, dtype):
    K = kpm()
    M, R = 32, 64
    say("wide lattice", L, periodic, dtype, "R", R)
    pot, Ho, a, b = oracle_problem(L, 1.5, 17, periodic=periodic)
    v0 = inputs.phase_block(Ho.n, R, 18)
    ref_eta = O.kpm_eta(Ho, a, b, v0, M)
    ref = O.mu_from_eta(ref_eta)
    try:
        K.set_sweep_tuning(lattice=2)
        H = K.build_hamiltonian(L, pot, periodic=periodic, dtype=dtype)
        assert K.sweep_kernel(H, R) == "lattice_kernel"
        H.close()
        mu, eta = gpu_moments(L, pot, v0, M, dtype=dtype, periodic=periodic, eta=True)
    finally:
        K.reset_sweep_tuning()
    tol = TOL_C128 if dtype == "c128" else TOL_C64
    assert np.abs(mu - ref).max() <= tol
    if dtype == "c128":
        got_eta = eta[..., 0] + 1j * eta[..., 1]
        assert np.abs(got_eta - ref_eta).max() <= TOL_C128


@pytest.mark.parametrize("lattice", [0, 2])
def test_quantum_dot_slab_matches_oracle(lattice):
    # the paper's geometry in small: periodic in x and y, open in z, a
    # superlattice of quantum dots in the top layers (rows of the two
    # surfaces carry padding slots)
    K = kpm()
    L, per, M, R = (12, 8, 6), (1, 1, 0), 40, 32
    say("quantum-dot slab, lattice", lattice)
    pot = inputs.quantum_dot_potential(L, period=6, radius=2.0, v_dot=1.5, depth=2, gamma=0.5, seed=3)
    Ho = O.ti_hamiltonian(L, pot, periodic=per)
    a, b = O.scaling(*O.gershgorin(Ho))
    v0 = inputs.phase_block(Ho.n, R, 4)
    ref = O.kpm_moments(Ho, a, b, v0, M)
    try:
        K.set_sweep_tuning(lattice=lattice)
        H = K.build_hamiltonian(L, pot, periodic=per)
        assert K.sweep_kernel(H, R) == ("lattice_kernel" if lattice else "gather_sweep_kernel")
        H.close()
        mu, _ = gpu_moments(L, pot, v0, M, periodic=per)
    finally:
        K.reset_sweep_tuning()
    assert np.abs(mu - ref).max() <= TOL_C128


@pytest.mark.parametrize("pz,dtype", [(1, "c128"), (0, "c128"), (1, "c64")])
def test_lattice_pencils_split_in_z_match_oracle(pz, dtype):
    # 17 x 16 = 272 pencils of 9 planes on 256 workgroups: the launch cuts
    # every pencil into two z-pieces (planes 0-3 and 4-8), each with its own
    # prologue; periodic and open z; complex64 (entries through LDS)
    K = kpm()
    L, per, M, R = (68, 64, 9), (1, 1, pz), 16, 32
    say("split pencils, pz", pz, dtype)
    pot = inputs.potential(L, 1.0, 6)
    Ho = O.ti_hamiltonian(L, pot, periodic=per)
    a, b = O.scaling(*O.gershgorin(Ho))
    v0 = inputs.phase_block(Ho.n, R, 7)
    ref = O.kpm_moments(Ho, a, b, v0, M)
    try:
        K.set_sweep_tuning(lattice=2, wg_per_cu=1)
        H = K.build_hamiltonian(L, pot, periodic=per, dtype=dtype)
        plan = K.sweep_plan(H, R)
        H.close()
        say("split pencils plan", plan)
        assert plan["kernel"] == "lattice_kernel"
        if plan["grid"] < 272:        # 272 pencils on fewer workgroups: the split applies
            assert plan["pieces"] == 2, plan
        mu, _ = gpu_moments(L, pot, v0, M, periodic=per, dtype=dtype)
        # the same sweep without the split (prefetch 1 never splits pencils)
        K.set_sweep_tuning(lattice=2, wg_per_cu=1, prefetch=1)
        whole, _ = gpu_moments(L, pot, v0, M, periodic=per, dtype=dtype)
    finally:
        K.reset_sweep_tuning()
    # both GPU runs form every row's products alike and reduce in tree order:
    # they agree to rounding
    assert np.abs(mu - whole).max() <= 1e-13
    assert np.abs(mu - ref).max() <= (TOL_C128 if dtype == "c128" else TOL_C64)


@pytest.mark.parametrize("L", [(5, 4, 4), (4, 9, 3), (1, 1, 7)])
def test_lattice_sweep_falls_back_for_one_site_tail_tiles(L):
    # a side with L mod 4 == 1 would leave tiles one site wide: the generic
    # (staged-gather, by default) sweep runs
    K = kpm()
    M, R = 24, 32
    pot, Ho, a, b = oracle_problem(L, 1.0, 4, periodic=(0, 0, 1))
    v0 = inputs.phase_block(Ho.n, R, 5)
    try:
        K.set_sweep_tuning(lattice=2)
        H = K.build_hamiltonian(L, pot, periodic=(0, 0, 1))
        assert K.sweep_kernel(H, R) == "gather_sweep_kernel"
        H.close()
        mu, _ = gpu_moments(L, pot, v0, M, periodic=(0, 0, 1))
    finally:
        K.reset_sweep_tuning()
    assert np.abs(mu - O.kpm_moments(Ho, a, b, v0, M)).max() <= TOL_C128


@pytest.mark.parametrize("R", [32, 64])
def test_lattice_single_sweep_variants(R):
    K = kpm()
    L = (6, 6, 7)
    pot, Ho, a, b = oracle_problem(L, 1.0, 13, periodic=(1, 0, 1))
    Hd = Ho.dense()
    H = K.build_hamiltonian(L, pot, periodic=(1, 0, 1))
    rng = np.random.default_rng(5)
    X = rng.standard_normal((Ho.n, R)) + 1j * rng.standard_normal((Ho.n, R))
    Y = rng.standard_normal((Ho.n, R)) + 1j * rng.standard_normal((Ho.n, R))
    Hx = Hd @ X
    Vt = torch.from_numpy(X).cuda()
    try:
        K.set_sweep_tuning(lattice=2)
        assert K.sweep_kernel(H, R) == "lattice_kernel"
        Wt = torch.from_numpy(Y.copy()).cuda()
        K.aug_spmmv(H, Vt, Wt, 1.0, 0.0, 0.0, variant="plain")
        assert np.abs(Wt.cpu().numpy() - Hx).max() <= 1e-12 * np.abs(Hx).max()
        Wt = torch.from_numpy(Y.copy()).cuda()
        K.aug_spmmv(H, Vt, Wt, 0.3, -0.7, -1.0, variant="nodot")
        ref = 0.3 * Hx - 0.7 * X - Y
        assert np.abs(Wt.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    finally:
        K.reset_sweep_tuning()
    H.close()


# --------------------------------------------------------------------------
# a4-a6, a14: single sweeps and the diagnostic variants
# --------------------------------------------------------------------------
@pytest.mark.parametrize("R", [1, 8, 32, 64])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_single_sweep_variants(R, dtype):
    K = kpm()
    L = (5, 6, 7)
    say("sweep variants", R, dtype)
    pot, Ho, a, b = oracle_problem(L, 1.0, 8)
    Hd = Ho.dense()
    cdt = np.complex128 if dtype == "c128" else np.complex64
    H = K.build_hamiltonian(L, pot, dtype=dtype)
    rng = np.random.default_rng(R)
    X = (rng.standard_normal((Ho.n, R)) + 1j * rng.standard_normal((Ho.n, R))).astype(cdt)
    Y = (rng.standard_normal((Ho.n, R)) + 1j * rng.standard_normal((Ho.n, R))).astype(cdt)
    Hx = Hd.astype(cdt).astype(np.complex128) @ X.astype(np.complex128)
    tol = 1e-12 if dtype == "c128" else 5e-5
    alpha, beta, gamma = 0.3, -0.7, -1.0

    Vt = torch.from_numpy(X).cuda()
    Wt = torch.from_numpy(Y.copy()).cuda()
    K.aug_spmmv(H, Vt, Wt, 1.0, 0.0, 0.0, variant="plain")
    assert np.abs(Wt.cpu().numpy() - Hx).max() <= tol * max(1.0, np.abs(Hx).max())

    Wt = torch.from_numpy(Y.copy()).cuda()
    K.aug_spmmv(H, Vt, Wt, alpha, beta, gamma, variant="nodot")
    ref = alpha * Hx + beta * X + gamma * Y
    assert np.abs(Wt.cpu().numpy() - ref).max() <= tol * max(1.0, np.abs(ref).max())

    Wt = torch.from_numpy(Y.copy()).cuda()
    eta = torch.zeros((2, R, 2), dtype=torch.float64, device="cuda")
    K.aug_spmmv(H, Vt, Wt, alpha, beta, gamma, variant="full", eta=eta)
    Wn = Wt.cpu().numpy()
    assert np.abs(Wn - ref).max() <= tol * max(1.0, np.abs(ref).max())
    e = eta.cpu().numpy()
    x64, w64 = X.astype(np.complex128), Wn.astype(np.complex128)
    vv = np.sum(np.abs(x64) ** 2, axis=0)
    wv = np.sum(w64.conj() * x64, axis=0)
    assert np.abs(e[0, :, 0] - vv).max() <= 1e-12 * vv.max()
    assert np.abs(e[1, :, 0] + 1j * e[1, :, 1] - wv).max() <= 1e-12 * np.abs(wv).max() * 10
    H.close()


# --------------------------------------------------------------------------
# a8: density of states
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kernel,kparam", [("jackson", 0.0), ("dirichlet", 0.0), ("lorentz", 4.0)])
def test_dos_matches_oracle(kernel, kparam):
    K = kpm()
    say("dos", kernel)
    L, M, R = (6, 6, 6), 300, 4
    pot, Ho, a, b = oracle_problem(L, 1.0, 1)
    v0 = inputs.phase_block(Ho.n, R, 3)
    mu = O.kpm_moments(Ho, a, b, v0, M)
    E = np.concatenate([O.midpoint_grid(777, a, b), [b - a, b + a, b + 2 * a, b - 3 * a]])
    g = {"jackson": lambda: O.jackson(M), "dirichlet": lambda: O.dirichlet(M),
         "lorentz": lambda: O.lorentz(M, kparam)}[kernel]()
    ref = O.dos(mu, g, a, b, E)
    rho = K.dos(torch.from_numpy(mu).cuda(), a, b, torch.from_numpy(E).cuda(), kernel=kernel, kparam=kparam)
    got = rho.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()
    assert np.all(got[-4:] == 0.0)       # |x| >= 1


def test_dos_long_expansion():
    # M = 5000 spans three LDS chunks of the reconstruction kernel
    K = kpm()
    M = 5000
    x0 = 0.31
    mu = np.cos(np.arange(M) * np.arccos(x0))[None, :]
    E = O.midpoint_grid(4096, 1.0, 0.0)
    ref = O.dos(mu, O.jackson(M), 1.0, 0.0, E)
    got = K.dos(torch.from_numpy(mu).cuda(), 1.0, 0.0, torch.from_numpy(E).cuda()).cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()


# --------------------------------------------------------------------------
# error paths reached from the host
# --------------------------------------------------------------------------
def test_error_paths():
    K = kpm()
    L = (4, 4, 4)
    pot = inputs.potential(L, 1.0, 0)
    H = K.build_hamiltonian(L, pot)
    V0 = torch.from_numpy(inputs.phase_block(H.N, 4, 0)).cuda()
    with pytest.raises(K.KPMError) as e:
        K.moments(H, V0, 7)
    assert e.value.status == K.KPM_EINVAL
    V3 = torch.from_numpy(inputs.phase_block(H.N, 3, 0)).cuda()
    with pytest.raises(K.KPMError) as e:
        K.moments(H, V3, 8)
    assert e.value.status == K.KPM_ENOTSUP
    with pytest.raises(K.KPMError) as e:
        K.build_hamiltonian((2, 4, 4), np.zeros(32))
    assert e.value.status == K.KPM_ENOTSUP
    with pytest.raises(K.KPMError) as e:
        K.build_hamiltonian(L, np.full(64, np.nan))
    assert e.value.status == K.KPM_EINVAL
    # a caller-fixed scale far too small: the spectrum leaves [-1, 1]
    Hs = K.build_hamiltonian(L, pot, fixed_scale=(2.0, 0.0))
    with pytest.raises(K.KPMError) as e:
        K.moments(Hs, V0, 64)
    assert e.value.status == K.KPM_ESPECTRUM
    Hs.close()
    H.close()


# --------------------------------------------------------------------------
# the benchmark workload at full size: 64^3 lattice, R = 32, M = 2000
# --------------------------------------------------------------------------
GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


def golden_moments(name):
    """Oracle moments stored by tests/golden/make_oracle_moments.py ([R][M] float64)."""
    import json
    import os
    path = os.path.join(GOLDEN, name + "_mu.npy")
    if not os.path.exists(path):
        pytest.skip(f"{path} missing (run tests/golden/make_oracle_moments.py)")
    return np.load(path, allow_pickle=False), json.load(open(os.path.join(GOLDEN, name + "_mu.json")))


@pytest.mark.slow
def test_full_size_benchmark_workload():
    # 64^3 lattice, gamma = 1, R = 32, M = 2000, complex128, in the launch shape the
    # benchmark times (its tuning cache): every one of the 64,000 moments against the
    # oracle's (pairwise scalar products: its own error is ~1e-14 at this N)
    from paper_1410_5242_amd import autotune
    K = kpm()
    ref, rec = golden_moments("ti64_r32_m2000_c128")
    L, R, M = (64, 64, 64), 32, 2000
    say("full size: build")
    pot = inputs.potential(L, rec["gamma"], rec["pot_seed"])
    H = K.build_hamiltonian(L, pot)
    assert H.N == 1048576
    assert H.a == pytest.approx(rec["a"], rel=1e-15) and H.b == pytest.approx(rec["b"], abs=1e-15)
    v0 = inputs.phase_block(H.N, R, rec["phase_seed"])
    V0 = torch.from_numpy(v0).cuda()
    try:
        K.reset_sweep_tuning()
        autotune.apply_sweep(autotune.TuningCache(), H, R, L)
        plan = K.sweep_plan(H, R)
        say("full size: plan", plan, K.get_sweep_tuning())
        assert plan["kernel"] == "lattice_kernel"
        say("full size: moments")
        mu = K.moments(H, V0, M).cpu().numpy()
        mu_short = K.moments(H, V0, 64).cpu().numpy()
    finally:
        K.reset_sweep_tuning()
    err = np.abs(mu - ref)
    say(f"full size: max |dmu| = {err.max():.3e} (even {err[:, 0::2].max():.3e}, odd {err[:, 1::2].max():.3e})")
    assert err.max() <= TOL_C128
    # properties at any size: mu_0 = 1, |mu_n| <= 1, and the Jackson DOS integrates to 1
    assert np.abs(mu[:, 0] - 1.0).max() <= 1e-13
    assert np.abs(mu).max() <= 1.0 + 1e-12
    E = O.midpoint_grid(4096, H.a, H.b)
    rho = K.dos(torch.from_numpy(mu).cuda(), H.a, H.b, torch.from_numpy(E).cuda()).cpu().numpy()
    rho_ref = O.dos(ref, O.jackson(M), H.a, H.b, E)
    assert np.abs(rho - rho_ref).max() <= 1e-10 * np.abs(rho_ref).max()
    assert abs(rho.sum() * (2 * H.a / 4096) - 1.0) < 1e-4
    # same GPU run, truncated: moments are prefix-identical
    assert np.array_equal(mu_short, mu[:, :64])
    H.close()


@pytest.mark.slow
@pytest.mark.parametrize("gather", [3, 4])
def test_full_size_workload_index_reading_sweeps(gather):
    # the benchmark workload (64^3, R = 32, M = 2000) through the index-reading
    # sweeps instead of the lattice sweep: the window sweep (gather 3: its full
    # die mapping, one 4 x 4 pencil per workgroup) and the plain staged gather
    # (gather 4), every one of the 64,000 moments against the oracle's
    K = kpm()
    ref, rec = golden_moments("ti64_r32_m2000_c128")
    L, R, M = (64, 64, 64), 32, 2000
    say("full size, index-reading sweep", gather)
    pot = inputs.potential(L, rec["gamma"], rec["pot_seed"])
    H = K.build_hamiltonian(L, pot)
    V0 = torch.from_numpy(inputs.phase_block(H.N, R, rec["phase_seed"])).cuda()
    try:
        K.set_sweep_tuning(lattice=0, gather=gather)
        plan = K.sweep_plan(H, R)
        say("plan", plan)
        assert plan["kernel"] == ("window_sweep_kernel" if gather == 3 else "gather_sweep_kernel")
        mu = K.moments(H, V0, M).cpu().numpy()
    finally:
        K.reset_sweep_tuning()
        H.close()
    err = np.abs(mu - ref)
    say(f"max |dmu| = {err.max():.3e}")
    assert err.max() <= TOL_C128


@pytest.mark.slow
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_precision_workload_prefix_against_oracle(dtype):
    # 128 x 128 x 64 lattice, gamma = 2, R = 32, start block from the device generator
    # (seed 0): the first 400 moments (200 sweeps) of the precision workload, in the
    # benchmark's tuned launch shape, against the oracle's; complex128 to 1e-12,
    # complex64 storage (FP64 products) to the stated 1e-5
    from paper_1410_5242_amd import autotune
    K = kpm()
    ref, rec = golden_moments("ti128x128x64_g2_r32_m400")
    L, R, M = tuple(rec["L"]), rec["R"], rec["M"]
    pot = inputs.potential(L, rec["gamma"], rec["pot_seed"])
    H = K.build_hamiltonian(L, pot, dtype=dtype)
    assert H.a == pytest.approx(rec["a"], rel=1e-15) and H.b == pytest.approx(rec["b"], abs=1e-15)
    try:
        K.reset_sweep_tuning()
        autotune.apply_sweep(autotune.TuningCache(), H, R, L)
        say("precision prefix", dtype, K.sweep_plan(H, R))
        V0 = K.random_phase_block(H.N, R, rec["phase_seed"], dtype)
        mu = K.moments(H, V0, M).cpu().numpy()
    finally:
        K.reset_sweep_tuning()
    err = np.abs(mu - ref).max()
    say(f"precision prefix {dtype}: max |dmu| = {err:.3e}")
    assert err <= (TOL_C128 if dtype == "c128" else TOL_C64)
    H.close()


# --------------------------------------------------------------------------
# a3: start block drawn on the device (counter-based SplitMix64)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N,R,seed", [(1, 1, 0), (2048, 1, 0), (4100, 8, 3), (1000, 32, 2**63 + 5)])
def test_random_phase_block_matches_oracle_generator(N, R, seed):
    K = kpm()
    say("phase block", N, R, seed)
    ref = O.phase_block_counter(N, R, seed)
    v = K.random_phase_block(N, R, seed, "c128")
    torch.cuda.synchronize()
    got = v.cpu().numpy()
    # same generator on both sides: values agree to the last bits of cos / sin
    assert np.abs(got - ref).max() <= 1e-14 / np.sqrt(N)
    v64 = K.random_phase_block(N, R, seed, "c64")
    torch.cuda.synchronize()
    assert np.abs(v64.cpu().numpy() - ref.astype(np.complex64)).max() <= 1e-7 / np.sqrt(N)


# --------------------------------------------------------------------------
# both generic sweeps (staged-gather and scalar-operand) at every block width
# --------------------------------------------------------------------------
@pytest.mark.parametrize("gather", [1, 2])
@pytest.mark.parametrize("R", [1, 2, 8, 32, 64])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_generic_sweeps_match_oracle(gather, R, dtype):
    K = kpm()
    L, M = (7, 6, 5), 48
    say("generic sweep gather", gather, "R", R, dtype)
    pot, Ho, a, b = oracle_problem(L, 1.0, 21, periodic=(1, 1, 0))
    v0 = inputs.phase_block(Ho.n, R, 22)
    ref = O.kpm_moments(Ho, a, b, v0, M)
    try:
        K.set_sweep_tuning(lattice=0, gather=gather)
        H = K.build_hamiltonian(L, pot, periodic=(1, 1, 0), dtype=dtype)
        assert K.sweep_kernel(H, R) == ("gather_sweep_kernel" if gather == 1 else "aug_spmmv_kernel")
        H.close()
        mu, _ = gpu_moments(L, pot, v0, M, dtype=dtype, periodic=(1, 1, 0))
    finally:
        K.reset_sweep_tuning()
    assert np.abs(mu - ref).max() <= (TOL_C128 if dtype == "c128" else TOL_C64)


@pytest.mark.parametrize("slab", [1, 2, 4])
@pytest.mark.parametrize("R", [1, 8, 64])
def test_gather_slab_order_matches_oracle(slab, R):
    # passes in blocks of `slab` y-lines, plane by plane (Ly = 7: the last
    # block is ragged for slab 2 and 4); only the order of the rows changes
    K = kpm()
    L, M = (6, 7, 5), 40
    say("gather slab order", slab, "R", R)
    pot, Ho, a, b = oracle_problem(L, 1.0, 23, periodic=(1, 1, 0))
    v0 = inputs.phase_block(Ho.n, R, 24)
    ref = O.kpm_moments(Ho, a, b, v0, M)
    try:
        K.set_sweep_tuning(lattice=0, gather=1, slab=slab)
        mu, _ = gpu_moments(L, pot, v0, M, periodic=(1, 1, 0))
    finally:
        K.reset_sweep_tuning()
    assert np.abs(mu - ref).max() <= TOL_C128


# The LDS-window variant of the staged-gather sweep (tuning gather 3 forces it on
# any lattice): pencils of 4 x 4-site tiles (2 x 2 at complex128 R = 64), tiles cut
# by the lattice edge (sides 9, 7 and 6 are not multiples of 4), open and periodic
# sides, one and several runs of z-planes per tile, both tile-to-die mappings.
WINDOW_CASES = [((9, 7, 5), (1, 1, 0)), ((6, 9, 8), (0, 1, 1)), ((4, 4, 12), (1, 1, 1)), ((3, 5, 2), (1, 0, 0))]


@pytest.mark.parametrize("L,periodic", WINDOW_CASES)
@pytest.mark.parametrize("R", [16, 32, 64])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_window_sweep_matches_oracle(L, periodic, R, dtype):
    K = kpm()
    M = 40
    say("window sweep", L, periodic, R, dtype)
    pot, Ho, a, b = oracle_problem(L, 1.0, 25, periodic=periodic)
    v0 = inputs.phase_block(Ho.n, R, 26)
    ref = O.kpm_moments(Ho, a, b, v0, M)
    exists = not (dtype == "c64" and R == 16)   # complex64 R = 16: passes span more than one site
    try:
        K.set_sweep_tuning(lattice=0, gather=3)
        H = K.build_hamiltonian(L, pot, periodic=periodic, dtype=dtype)
        assert K.sweep_kernel(H, R) == ("window_sweep_kernel" if exists else "gather_sweep_kernel")
        H.close()
        mu, _ = gpu_moments(L, pot, v0, M, dtype=dtype, periodic=periodic)
    finally:
        K.reset_sweep_tuning()
    assert np.abs(mu - ref).max() <= (TOL_C128 if dtype == "c128" else TOL_C64)


@pytest.mark.parametrize("R,dtype", [(16, "c128"), (32, "c128"), (64, "c128"), (32, "c64"), (64, "c64")])
@pytest.mark.parametrize("order", [0, 2])
def test_window_sweep_writes_the_staged_gather_result(R, dtype, order):
    # every row's products are formed in the same order from the same values, so
    # the window sweep's W equals the plain staged-gather sweep's bit for bit; the
    # scalar products differ only by summation order.  16 x 16 x 12: 16 tiles in a
    # 2 x 4 split for the dies (tile order 0) or none (2); three z-runs per tile.
    K = kpm()
    L = (16, 16, 12)
    say("window vs staged gather", R, dtype, order)
    H = K.build_hamiltonian(L, inputs.potential(L, 1.0, 27), dtype=dtype)
    V = K.random_phase_block(H.N, R, 1, dtype)
    W0 = K.random_phase_block(H.N, R, 2, dtype)
    out = {}
    try:
        for g in (4, 3):
            K.set_sweep_tuning(lattice=0, gather=g, tile_order=order)
            assert K.sweep_kernel(H, R) == ("window_sweep_kernel" if g == 3 else "gather_sweep_kernel")
            for var in ("full", "nodot", "plain"):
                W = W0.clone()
                eta = torch.zeros((2, R, 2), dtype=torch.float64, device="cuda") if var == "full" else None
                K.aug_spmmv(H, V, W, 2.0 / H.a, -2.0 * H.b / H.a, -1.0, var, eta)
                torch.cuda.synchronize()
                out[(g, var)] = (W.cpu(), None if eta is None else eta.cpu())
    finally:
        K.reset_sweep_tuning()
        H.close()
    for var in ("full", "nodot", "plain"):
        assert torch.equal(out[(3, var)][0], out[(4, var)][0]), var
    e3, e4 = out[(3, "full")][1], out[(4, "full")][1]
    assert (e3 - e4).abs().max().item() <= 1e-13 * max(1.0, e4.abs().max().item())


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_window_sweep_several_items_per_workgroup(dtype):
    # 90 x 94 x 6 (open z): 23 x 24 = 552 tiles, some cut by the lattice edge, more
    # work items than the workgroups of one per CU, so a workgroup walks several
    # tiles one after the other (a fresh ring prologue each)
    K = kpm()
    L, per, M, R = (90, 94, 6), (1, 1, 0), 12, 32
    say("window sweep, several items per workgroup", dtype)
    pot, Ho, a, b = oracle_problem(L, 1.0, 29, periodic=per)
    v0 = inputs.phase_block(Ho.n, R, 30)
    ref = O.kpm_moments(Ho, a, b, v0, M)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    try:
        K.set_sweep_tuning(lattice=0, gather=3)
        H = K.build_hamiltonian(L, pot, periodic=per, dtype=dtype)
        plan = K.sweep_plan(H, R)
        H.close()
        assert plan["kernel"] == "window_sweep_kernel" and plan["grid"] < 23 * 24, (plan, cus)
        mu, _ = gpu_moments(L, pot, v0, M, dtype=dtype, periodic=per)
    finally:
        K.reset_sweep_tuning()
    assert np.abs(mu - ref).max() <= (TOL_C128 if dtype == "c128" else TOL_C64)


@pytest.mark.parametrize("R", [16, 32, 64])
def test_window_sweep_single_sweep_variants(R):
    # FULL, NODOT, PLAIN of the window sweep against H X from the oracle's dense matrix
    K = kpm()
    L = (9, 6, 7)
    say("window sweep variants", R)
    pot, Ho, a, b = oracle_problem(L, 1.0, 28, periodic=(1, 0, 1))
    Hd = Ho.dense()
    rng = np.random.default_rng(R + 5)
    X = rng.standard_normal((Ho.n, R)) + 1j * rng.standard_normal((Ho.n, R))
    Y = rng.standard_normal((Ho.n, R)) + 1j * rng.standard_normal((Ho.n, R))
    Hx = Hd @ X
    alpha, beta, gamma = 0.3, -0.7, -1.0
    ref = alpha * Hx + beta * X + gamma * Y
    try:
        K.set_sweep_tuning(lattice=0, gather=3)
        H = K.build_hamiltonian(L, pot, periodic=(1, 0, 1))
        assert K.sweep_kernel(H, R) == "window_sweep_kernel"
        Vt = torch.from_numpy(X).cuda()
        Wt = torch.from_numpy(Y.copy()).cuda()
        K.aug_spmmv(H, Vt, Wt, 1.0, 0.0, 0.0, variant="plain")
        assert np.abs(Wt.cpu().numpy() - Hx).max() <= 1e-12 * max(1.0, np.abs(Hx).max())
        Wt = torch.from_numpy(Y.copy()).cuda()
        K.aug_spmmv(H, Vt, Wt, alpha, beta, gamma, variant="nodot")
        assert np.abs(Wt.cpu().numpy() - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
        Wt = torch.from_numpy(Y.copy()).cuda()
        eta = torch.zeros((2, R, 2), dtype=torch.float64, device="cuda")
        K.aug_spmmv(H, Vt, Wt, alpha, beta, gamma, variant="full", eta=eta)
        Wn = Wt.cpu().numpy()
        assert np.abs(Wn - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
        e = eta.cpu().numpy()
        vv = np.sum(np.abs(X) ** 2, axis=0)
        wv = np.sum(Wn.conj() * X, axis=0)
        assert np.abs(e[0, :, 0] - vv).max() <= 1e-12 * vv.max()
        assert np.abs(e[1, :, 0] + 1j * e[1, :, 1] - wv).max() <= 1e-12 * np.abs(wv).max() * 10
        H.close()
    finally:
        K.reset_sweep_tuning()


def test_window_sweep_is_the_default_generic_sweep_on_large_lattices():
    # gather 1 (default): the window variant where the lattice gives a run of
    # z-planes of a tile per CU, the plain staged gather on small lattices
    K = kpm()
    say("window default selection")
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    big = K.build_hamiltonian((64, 64, 64), None, gamma=1.0, seed=0)
    small = K.build_hamiltonian((8, 8, 8), None, gamma=1.0, seed=0)
    try:
        assert K.sweep_kernel(big, 16) == "window_sweep_kernel"
        assert K.sweep_kernel(big, 8) == "gather_sweep_kernel"
        assert K.sweep_kernel(small, 16) == "gather_sweep_kernel"
        p = K.sweep_plan(big, 16)
        assert p["kernel"] == "window_sweep_kernel" and p["grid"] == cus - cus % 8
    finally:
        big.close()
        small.close()


@pytest.mark.parametrize("order", [0, 1, 2, 3])
@pytest.mark.parametrize("L", [(8, 16, 5), (16, 16, 3)])
def test_lattice_tile_orders_match_oracle(order, L):
    # 2-D tile blocks per die, runs of tile rows, or no die mapping: same moments
    K = kpm()
    M, R = 24, 32
    say("lattice tile order", order, L)
    pot, Ho, a, b = oracle_problem(L, 1.0, 31)
    v0 = inputs.phase_block(Ho.n, R, 32)
    try:
        K.set_sweep_tuning(lattice=2, tile_order=order)
        mu, _ = gpu_moments(L, pot, v0, M)
    finally:
        K.reset_sweep_tuning()
    assert np.abs(mu - O.kpm_moments(Ho, a, b, v0, M)).max() <= TOL_C128


@pytest.mark.parametrize("period", [1, 3])
def test_sweep_profile_times_every_nth_launch(period):
    # kpm_sweep_profile_enable(n): launches 1, n + 1, 2n + 1, ... are timed
    K = kpm()
    L, R, M = (8, 8, 8), 32, 20   # 10 sweeps
    say("sweep profile period", period)
    pot = inputs.potential(L, 1.0, 41)
    H = K.build_hamiltonian(L, pot)
    V0 = torch.from_numpy(inputs.phase_block(H.N, R, 42)).cuda()
    try:
        K.sweep_profile_read()
        K.sweep_profile_enable(period)
        K.moments(H, V0, M)
        torch.cuda.synchronize()
        K.sweep_profile_enable(False)
        n, tot, lo, hi = K.sweep_profile_read()
    finally:
        K.sweep_profile_enable(False)
        H.close()
    assert n == (M // 2 + period - 1) // period
    assert 0.0 < lo <= hi and tot >= n * lo * 0.999
