"""GPU parity of the SELL-C-sigma path (kpm_import_csr + the SELL sweep)
against the CPU oracle, on general sparse Hermitian matrices: an irregular
random matrix with empty rows and a long tail of row lengths, and the
topological-insulator lattice handed over as plain CRS.

Tolerances as for the lattice path: complex128 moments within 1e-12 of the
oracle's (|mu_n| <= mu_0 = 1), complex64 storage with FP64 products within
1e-5; the imported matrix round-trips bit for bit in complex128.
"""
import os
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_1410_5242_amd import inputs

pytestmark = pytest.mark.gpu

TOL_C128 = 1e-12
TOL_C64 = 1e-5
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


def irregular(N, seed, **kw):
    rowptr, col, val = inputs.random_hermitian_csr(N, seed=seed, **kw)
    return rowptr, col, val, O.CSR(rowptr, col, val)


def tdtype(dtype):
    return torch.complex128 if dtype == "c128" else torch.complex64


LAYOUTS = [(1, 1), (4, 16), (32, 256), (64, 1 << 20)]


@pytest.mark.parametrize("C,sigma", LAYOUTS)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_import_round_trips_and_reports_its_layout(C, sigma, dtype):
    say("sell import", C, sigma, dtype)
    K = kpm()
    rowptr, col, val, Ho = irregular(3001, 1)
    H = K.import_csr(rowptr, col, val, dtype=dtype, C=C, sigma=sigma)
    info = K.sell_info(H)
    _, width, start = K.sell_layout(rowptr, C, sigma)
    assert info == {"C": C, "sigma": sigma, "nchunks": width.size, "stored": int(start[-1]),
                    "nnz": int(rowptr[-1])}
    assert H.N == 3001 and H.nnz_stored == int(start[-1]) and H.width == int(np.diff(rowptr).max())
    rp, c, v = K.export_csr(H)
    assert np.array_equal(rp, rowptr) and np.array_equal(c, col)
    ref = val if dtype == "c128" else val.astype(np.complex64).astype(np.complex128)
    assert np.array_equal(v, ref)
    emin, emax = O.gershgorin(Ho)
    tol = 1e-13 if dtype == "c128" else 1e-5
    assert H.emin == pytest.approx(emin, rel=tol, abs=tol) and H.emax == pytest.approx(emax, rel=tol, abs=tol)
    assert K.sweep_kernel(H, 8) == "sell_sweep_kernel"
    H.close()


@pytest.mark.parametrize("C,sigma", LAYOUTS)
@pytest.mark.parametrize("R", [1, 4, 32])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_sell_moments_match_oracle(C, sigma, R, dtype):
    say("sell moments", C, sigma, R, dtype)
    K = kpm()
    N, M = 4099, 120
    rowptr, col, val, Ho = irregular(N, 2)
    H = K.import_csr(rowptr, col, val, dtype=dtype, C=C, sigma=sigma)
    a, b = O.scaling(*O.gershgorin(Ho))
    if dtype == "c128":
        assert H.a == pytest.approx(a, rel=1e-13) and H.b == pytest.approx(b, rel=1e-12, abs=1e-13)
    K.set_scaling(H, a, b)
    v0 = inputs.phase_block(N, R, 3)
    ref = O.kpm_moments(Ho, a, b, v0, M)
    V0 = torch.from_numpy(v0.astype(np.complex128 if dtype == "c128" else np.complex64)).cuda()
    mu = K.moments(H, V0, M).cpu().numpy()
    err = np.abs(mu - ref).max()
    say(f"  max |dmu| = {err:.3e}")
    assert err <= (TOL_C128 if dtype == "c128" else TOL_C64)
    H.close()


@pytest.mark.parametrize("R", [1, 2, 8, 16, 64])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_sell_moments_every_block_width(R, dtype):
    say("sell moments R", R, dtype)
    K = kpm()
    N, M = 2500, 64
    rowptr, col, val, Ho = irregular(N, 4, tail=1.3, max_couplings=400)
    H = K.import_csr(rowptr, col, val, C=8, sigma=64, dtype=dtype)
    a, b = O.scaling(*O.gershgorin(Ho))
    K.set_scaling(H, a, b)
    v0 = inputs.phase_block(N, R, 5)
    ref = O.kpm_moments(Ho, a, b, v0, M)
    V0 = torch.from_numpy(v0.astype(np.complex128 if dtype == "c128" else np.complex64)).cuda()
    tol = TOL_C128 if dtype == "c128" else TOL_C64
    mu = K.moments(H, V0, M).cpu().numpy()
    assert np.abs(mu - ref).max() <= tol
    if R >= 16:   # the same block as column groups (staged passes of a narrower width)
        mu_g = K.moments(H, V0, M, group=R // 8).cpu().numpy()
        assert np.abs(mu_g - ref).max() <= tol
    H.close()


@pytest.mark.parametrize("R", [1, 4, 32])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_sell_single_sweep_variants(R, dtype):
    say("sell sweep variants", R, dtype)
    K = kpm()
    N = 1500
    rowptr, col, val, Ho = irregular(N, 6)
    Hd = Ho.dense()
    cdt = np.complex128 if dtype == "c128" else np.complex64
    H = K.import_csr(rowptr, col, val, dtype=dtype, C=16, sigma=128)
    rng = np.random.default_rng(R)
    X = (rng.standard_normal((N, R)) + 1j * rng.standard_normal((N, R))).astype(cdt)
    Y = (rng.standard_normal((N, R)) + 1j * rng.standard_normal((N, R))).astype(cdt)
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


def test_sell_edge_cases():
    K = kpm()
    # one row; fewer rows than a chunk; a dense row longer than many slot
    # groups next to empty rows; a zero matrix under a caller-fixed scaling
    say("sell edge: one row")
    H = K.import_csr(np.array([0, 1]), np.array([0]), np.array([0.5 + 0j]), C=64, sigma=64, fixed_scale=(1.0, 0.0))
    V0 = torch.ones((1, 4), dtype=torch.complex128, device="cuda")
    mu = K.moments(H, V0, 16).cpu().numpy()
    ref = np.cos(np.arange(16) * np.arccos(0.5))
    assert np.abs(mu - ref[None, :]).max() <= 1e-14
    H.close()

    say("sell edge: dense row, empty rows")
    N = 70
    rows, cols, vals = [], [], []
    rng = np.random.default_rng(1)
    for j in range(N):          # row/column 0 couples to everything: a 70-entry row
        h = complex(rng.standard_normal(), rng.standard_normal()) if j else complex(rng.standard_normal())
        rows.append(0); cols.append(j); vals.append(h)
        if j:
            rows.append(j); cols.append(0); vals.append(np.conj(h))
    for j in range(1, N, 3):    # a diagonal on every third row; the other rows keep only column 0
        rows.append(j); cols.append(j); vals.append(complex(rng.standard_normal()))
    import scipy.sparse as sp
    A = sp.coo_matrix((vals, (rows, cols)), shape=(N + 5, N + 5)).tocsr()   # rows N..N+4 empty
    A.sort_indices()
    rowptr, col, val = A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data
    Ho = O.CSR(rowptr, col, val)
    a, b = O.scaling(*O.gershgorin(Ho))
    for R in (2, 32):   # 32 rows per pass (direct loads), 2 rows per pass (staged, three groups of 32 slots)
        v0 = inputs.phase_block(N + 5, R, 7)
        ref = O.kpm_moments(Ho, a, b, v0, 40)
        for C, sigma in ((1, 1), (2, 2), (64, 64), (8, 1 << 20)):
            H = K.import_csr(rowptr, col, val, C=C, sigma=sigma)
            K.set_scaling(H, a, b)
            mu = K.moments(H, torch.from_numpy(v0).cuda(), 40).cpu().numpy()
            assert np.abs(mu - ref).max() <= TOL_C128, (R, C, sigma)
            H.close()

    say("sell edge: zero matrix")
    N = 33
    H = K.import_csr(np.zeros(N + 1, dtype=np.int64), np.zeros(0, np.int32), np.zeros(0, np.complex128),
                     C=8, sigma=8, fixed_scale=(1.0, 0.5))
    v0 = inputs.phase_block(N, 4, 9)
    mu = K.moments(H, torch.from_numpy(v0).cuda(), 10).cpu().numpy()
    ref = np.cos(np.arange(10) * np.arccos(-0.5))     # Htilde = -0.5 everywhere
    assert np.abs(mu - ref[None, :]).max() <= 1e-14
    H.close()


def test_lattice_as_crs_matches_the_lattice_path_and_the_oracle():
    # the topological-insulator lattice with open z (rows of 11 and 13
    # entries, so SELL pads) handed over as plain CRS
    K = kpm()
    L, R, M = (6, 5, 7), 8, 96
    say("sell lattice as CRS")
    pot = inputs.potential(L, 1.5, 2)
    Ho = O.ti_hamiltonian(L, pot, periodic=(1, 1, 0))
    a, b = O.scaling(*O.gershgorin(Ho))
    v0 = inputs.phase_block(Ho.n, R, 4)
    ref = O.kpm_moments(Ho, a, b, v0, M)
    Hl = K.build_hamiltonian(L, pot, periodic=(1, 1, 0))
    mu_l = K.moments(Hl, torch.from_numpy(v0).cuda(), M).cpu().numpy()
    for C, sigma in ((1, 1), (32, 256)):
        H = K.import_csr(Ho.rowptr, Ho.col, Ho.val, C=C, sigma=sigma)
        assert H.a == pytest.approx(Hl.a, rel=1e-14) and H.b == pytest.approx(Hl.b, abs=1e-14)
        assert K.sell_info(H)["stored"] >= Ho.nnz
        mu = K.moments(H, torch.from_numpy(v0).cuda(), M).cpu().numpy()
        assert np.abs(mu - ref).max() <= TOL_C128
        assert np.abs(mu - mu_l).max() <= TOL_C128
        H.close()
    Hl.close()


def test_naive_algorithm_and_lanczos_run_on_sell_storage():
    K = kpm()
    say("sell naive + lanczos")
    N, R, M = 2000, 2, 32
    rowptr, col, val, Ho = irregular(N, 8)
    H = K.import_csr(rowptr, col, val)
    a, b = O.scaling(*O.gershgorin(Ho))
    K.set_scaling(H, a, b)
    v0 = inputs.phase_block(N, R, 1)
    ref = O.kpm_moments(Ho, a, b, v0, M)
    mu = K.moments_naive(H, torch.from_numpy(v0).cuda(), M).cpu().numpy()
    assert np.abs(mu - ref).max() <= TOL_C128
    lo, hi = K.lanczos_bounds(H, steps=60, seed=3)
    lam = np.linalg.eigvalsh(Ho.dense())
    assert lam[0] - 1e-9 <= lo < hi <= lam[-1] + 1e-9
    assert hi - lo > 0.9 * (lam[-1] - lam[0])
    H.close()


def test_batched_solver_rejects_sell_storage():
    K = kpm()
    rowptr, col, val, _ = irregular(300, 3)
    H = K.import_csr(rowptr, col, val)
    V0 = torch.from_numpy(inputs.phase_block(300, 1, 0)).cuda()
    with pytest.raises(K.KPMError, match="imported matrix"):
        K.moments_batched([H], [V0], 8)
    H.close()


def test_sell_graph_replay_matches_eager():
    K = kpm()
    say("sell graph")
    N, R, M = 3000, 4, 80
    rowptr, col, val, Ho = irregular(N, 10)
    H = K.import_csr(rowptr, col, val, C=32, sigma=256)
    V0 = torch.from_numpy(inputs.phase_block(N, R, 2)).cuda()
    eager = K.moments(H, V0, M).cpu().numpy()
    for _ in range(3):
        g = K.moments(H, V0, M, graph=True).cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(g, eager)
    H.close()


@pytest.mark.slow
def test_full_size_workload_through_sell_storage():
    # the benchmark workload (64^3 periodic lattice, gamma = 1, R = 32,
    # M = 2000) handed over as the oracle's CRS and swept from SELL-32-256
    # storage: every one of the 64,000 moments against the oracle's
    K = kpm()
    path = os.path.join(GOLDEN, "ti64_r32_m2000_c128_mu.npy")
    if not os.path.exists(path):
        pytest.skip("golden moments missing")
    import json
    ref = np.load(path, allow_pickle=False)
    rec = json.load(open(os.path.join(GOLDEN, "ti64_r32_m2000_c128_mu.json")))
    L, R, M = tuple(rec["L"]), rec["R"], rec["M"]
    say("full size through SELL: oracle CRS")
    pot = inputs.potential(L, rec["gamma"], rec["pot_seed"])
    Ho = O.ti_hamiltonian(L, pot)
    H = K.import_csr(Ho.rowptr, Ho.col, Ho.val, C=32, sigma=256)
    assert H.a == pytest.approx(rec["a"], rel=1e-14) and H.b == pytest.approx(rec["b"], abs=1e-14)
    K.set_scaling(H, rec["a"], rec["b"])
    assert K.sweep_kernel(H, R) == "sell_sweep_kernel"
    V0 = torch.from_numpy(inputs.phase_block(H.N, R, rec["phase_seed"])).cuda()
    say("full size through SELL: moments")
    mu = K.moments(H, V0, M).cpu().numpy()
    H.close()
    err = np.abs(mu - ref)
    say(f"max |dmu| = {err.max():.3e}")
    assert err.max() <= TOL_C128


def test_default_layout_and_kernel_report():
    K = kpm()
    rowptr, col, val, _ = irregular(1000, 13)
    H = K.import_csr(rowptr, col, val)
    info = K.sell_info(H)
    assert (info["C"], info["sigma"]) == (8, 1024)
    plan = K.sweep_plan(H, 32)
    assert plan["kernel"] == "sell_sweep_kernel" and plan["grid"] >= 1
    assert plan["tile_order"] == -1 and plan["pieces"] == -1 and plan["halves"] == -1 and plan["group"] == 32
    Hl = K.build_hamiltonian((4, 4, 4), np.zeros(64))
    assert K.sell_info(Hl) == {"C": 0, "sigma": 0, "nchunks": 0, "stored": 0, "nnz": 0}
    Hl.close()
    H.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_lattice_built_into_sell_storage(dtype):
    # kpm_lattice_desc.sell_C: the builder's matrix stored in SELL-C-sigma
    # (open z, so padding slots are dropped and chunks pad), with the
    # lattice's exact bounds and scaling; moments against the oracle and the
    # lattice layout
    K = kpm()
    L, R, M = (5, 6, 7), 8, 80
    say("lattice into sell", dtype)
    pot = inputs.potential(L, 1.0, 3)
    Ho = O.ti_hamiltonian(L, pot, periodic=(1, 1, 0))
    Hl = K.build_hamiltonian(L, pot, periodic=(1, 1, 0), dtype=dtype)
    H = K.build_hamiltonian(L, pot, periodic=(1, 1, 0), dtype=dtype, sell_C=16, sell_sigma=256)
    info = K.sell_info(H)
    assert (info["C"], info["sigma"], info["nnz"]) == (16, 256, Ho.nnz)
    assert (H.a, H.b, H.emin, H.emax) == (Hl.a, Hl.b, Hl.emin, Hl.emax)
    rp, c, v = K.export_csr(H)
    rl, cl, vl = K.export_csr(Hl)
    assert np.array_equal(rp, rl) and np.array_equal(c, cl) and np.array_equal(v, vl)
    assert K.sweep_kernel(H, R) == "sell_sweep_kernel"
    a, b = O.scaling(*O.gershgorin(Ho))
    v0 = inputs.phase_block(Ho.n, R, 6)
    ref = O.kpm_moments(Ho, a, b, v0, M)
    V0 = torch.from_numpy(v0.astype(np.complex128 if dtype == "c128" else np.complex64)).cuda()
    mu = K.moments(H, V0, M).cpu().numpy()
    mu_l = K.moments(Hl, V0, M).cpu().numpy()
    tol = TOL_C128 if dtype == "c128" else TOL_C64
    assert np.abs(mu - ref).max() <= tol
    assert np.abs(mu - mu_l).max() <= (TOL_C128 if dtype == "c128" else 1e-6)
    H.close()
    Hl.close()


def test_sell_scaling_too_tight_reports_spectrum():
    # an imported matrix under a half-width of 40 % of its spectral radius:
    # the Chebyshev recurrence leaves [-1, 1] and the moment check refuses it
    K = kpm()
    N, R, M = 2000, 2, 64
    rowptr, col, val, Ho = irregular(N, 14)
    lam = np.linalg.eigvalsh(Ho.dense())
    H = K.import_csr(rowptr, col, val, fixed_scale=(0.4 * max(abs(lam[0]), abs(lam[-1])), 0.0))
    V0 = torch.from_numpy(inputs.phase_block(N, R, 1)).cuda()
    with pytest.raises(K.KPMError) as e:
        K.moments(H, V0, M, check=True)
    assert e.value.status == K.KPM_ESPECTRUM
    H.close()
