"""GPU tests of the C ABI's options and ownership rules: the counter-generated
potential, kpm_moments options (HIP-graph replay, host moments, the NODOT
variant, a per-call tuning), the launch plan query, and calls that overlap on
two streams (per-stream workspaces), each against the CPU oracle."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_1410_5242_amd import inputs

pytestmark = pytest.mark.gpu

TOL_C128 = 1e-12


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


def oracle_problem(L, pot, periodic=(1, 1, 1)):
    Ho = O.ti_hamiltonian(L, pot, periodic=periodic)
    a, b = O.scaling(*O.gershgorin(Ho))
    return Ho, a, b


@pytest.mark.parametrize("L,gamma,seed", [((5, 4, 7), 2.0, 11), ((8, 8, 8), 1.0, 0), ((3, 3, 3), 0.0, 5)])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_generated_potential_matches_oracle_generator(L, gamma, seed, dtype):
    # kpm_lattice_desc without a potential array: V_n from the device's counter
    # generator; the oracle draws the same numbers from its own implementation
    say("generated potential", L, gamma, seed, dtype)
    K = kpm()
    H = K.build_hamiltonian(L, None, gamma=gamma, seed=seed, dtype=dtype)
    pot = O.potential_counter(L, gamma, seed)
    Ho, a, b = oracle_problem(L, pot)
    rp, col, val = K.export_csr(H)
    assert np.array_equal(rp, Ho.rowptr)
    ref = Ho.val if dtype == "c128" else Ho.val.astype(np.complex64).astype(np.complex128)
    # same entries per row (the library keeps its slot order, the oracle sorts columns)
    for i in range(0, Ho.n, max(1, Ho.n // 97)):
        s, e = rp[i], rp[i + 1]
        o1, o2 = np.argsort(col[s:e]), np.argsort(Ho.col[s:e])
        assert np.array_equal(col[s:e][o1], Ho.col[s:e][o2])
        assert np.array_equal(val[s:e][o1], ref[s:e][o2])
    assert H.a == pytest.approx(a, rel=1e-15) and H.b == pytest.approx(b, abs=1e-15)
    if dtype == "c128":
        v0 = inputs.phase_block(Ho.n, 2, 1)
        mu = K.moments(H, torch.from_numpy(v0).cuda(), 64).cpu().numpy()
        assert np.abs(mu - O.kpm_moments(Ho, a, b, v0, 64)).max() <= TOL_C128
    H.close()


def test_moments_graph_replays_match_eager_and_oracle():
    # the 8^3 correctness workload (R = 1, M = 128): captured once, replayed with
    # eager work and synchronisations between replays; each replay reads the start
    # block anew, so changing its contents changes the result
    K = kpm()
    L, M = (8, 8, 8), 128
    pot = inputs.potential(L, 1.0, 0)
    Ho, a, b = oracle_problem(L, pot)
    H = K.build_hamiltonian(L, pot)
    blocks = [inputs.phase_block(Ho.n, 1, s) for s in (0, 1, 2)]
    refs = [O.kpm_moments(Ho, a, b, v, M) for v in blocks]
    V0 = torch.from_numpy(blocks[0]).cuda()
    mu = torch.empty((1, M), dtype=torch.float64, device="cuda")
    eager = K.moments(H, V0, M).cpu().numpy()
    assert np.abs(eager - refs[0]).max() <= TOL_C128
    for rep in range(6):
        k = rep % 3
        V0.copy_(torch.from_numpy(blocks[k]))
        junk = torch.randn(1 << 16, device="cuda") * 3.0     # eager work between replays
        mu.fill_(float("nan"))
        K.moments(H, V0, M, mu=mu, graph=True)
        torch.cuda.synchronize()
        got = mu.cpu().numpy()
        say("graph replay", rep, float(np.abs(got - refs[k]).max()), float(junk.sum()))
        assert np.abs(got - refs[k]).max() <= TOL_C128
        if k == 0:
            assert np.array_equal(got, eager)      # same launches, same sums
    # another M captures a new graph; the old key no longer matches
    mu2 = torch.empty((1, 64), dtype=torch.float64, device="cuda")
    K.moments(H, V0, 64, mu=mu2, graph=True)
    V0.copy_(torch.from_numpy(blocks[0]))
    K.moments(H, V0, 64, mu=mu2, graph=True)
    assert np.abs(mu2.cpu().numpy() - refs[0][:, :64]).max() <= TOL_C128
    H.close()


@pytest.mark.parametrize("L,R", [((16, 16, 12), 32), ((10, 9, 7), 8)])
def test_moments_graph_wide_blocks(L, R):
    # the graph path on the lattice sweep (R = 32) and the staged-gather sweep
    K = kpm()
    M = 40
    pot = inputs.potential(L, 1.5, 3)
    Ho, a, b = oracle_problem(L, pot)
    v0 = inputs.phase_block(Ho.n, R, 4)
    ref = O.kpm_moments(Ho, a, b, v0, M)
    H = K.build_hamiltonian(L, pot)
    V0 = torch.from_numpy(v0).cuda()
    mu = torch.empty((R, M), dtype=torch.float64, device="cuda")
    eta = torch.empty((M, R, 2), dtype=torch.float64, device="cuda")
    for rep in range(3):
        mu.zero_()
        K.moments(H, V0, M, mu=mu, eta=eta, graph=True, check=True)
        torch.cuda.synchronize()
        assert np.abs(mu.cpu().numpy() - ref).max() <= TOL_C128
    ref_eta = O.kpm_eta(Ho, a, b, v0, M)
    got_eta = eta.cpu().numpy()[..., 0] + 1j * eta.cpu().numpy()[..., 1]
    assert np.abs(got_eta - ref_eta).max() <= TOL_C128
    H.close()


def test_moments_host_output_nodot_and_per_call_tuning():
    K = kpm()
    L, R, M = (12, 12, 8), 4, 48
    pot = inputs.potential(L, 1.0, 9)
    Ho, a, b = oracle_problem(L, pot)
    v0 = inputs.phase_block(Ho.n, R, 9)
    ref = O.kpm_moments(Ho, a, b, v0, M)
    H = K.build_hamiltonian(L, pot)
    V0 = torch.from_numpy(v0).cuda()
    # host mu: filled in place, the call synchronises
    host = np.full((R, M), np.nan)
    K.moments(H, V0, M, mu=host)
    assert np.abs(host - ref).max() <= TOL_C128
    # NODOT: the recurrence without products; mu is not touched
    mu = torch.full((R, M), 7.0, dtype=torch.float64, device="cuda")
    K.moments(H, V0, M, mu=mu, variant="nodot", check=False)
    torch.cuda.synchronize()
    assert bool((mu == 7.0).all())
    # a per-call tuning gives what the same process-wide tuning gives, bit for bit,
    # and leaves the process-wide setting alone
    before = K.get_sweep_tuning()
    t = dict(gather=2, pencil=0, wg_per_cu=4)
    per_call = K.moments(H, V0, M, tuning=t).cpu().numpy()
    assert K.get_sweep_tuning() == before
    try:
        K.set_sweep_tuning(**t)
        glob = K.moments(H, V0, M).cpu().numpy()
    finally:
        K.reset_sweep_tuning()
    assert np.array_equal(per_call, glob)
    assert np.abs(per_call - ref).max() <= TOL_C128
    H.close()


def test_sweep_plan_of_the_headline_lattice():
    # 64^3, R = 32: one 4 x 4-site pencil per workgroup on the whole chip, dealt to
    # the 8 dies as 2-D blocks of pencils (tile order 0), whole pencils, one half
    K = kpm()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    H = K.build_hamiltonian((64, 64, 64), None, gamma=1.0, seed=0)
    p = K.sweep_plan(H, 32)
    say("headline plan", p, "CUs", cus)
    assert p["kernel"] == "lattice_kernel" and p["halves"] == 1 and p["pieces"] == 1
    assert p["grid"] == min(256, cus - cus % 8)
    if cus >= 256:
        assert p["tile_order"] == 0
    # R = 64: kpm_moments runs two 32-column recurrences on the lattice sweep
    p64 = K.sweep_plan(H, 64)
    assert p64["kernel"] == "lattice_kernel" and p64["group"] == 32 and p64["halves"] == 1
    g = K.sweep_plan(H, 8)
    assert g["kernel"] == "gather_sweep_kernel" and g["pieces"] == -1
    assert K.sweep_plan(H, 32, tuning={"lattice": 0})["kernel"] == "window_sweep_kernel"
    assert K.sweep_plan(H, 32, tuning={"lattice": 0, "gather": 4})["kernel"] == "gather_sweep_kernel"
    H.close()


def test_two_streams_overlap_with_separate_workspaces():
    # one Hamiltonian, two start blocks, two streams: kpm_moments and kpm_dot run
    # concurrently without a synchronisation between the streams; each result
    # matches the oracle (a shared workspace would mix the two runs)
    K = kpm()
    L, R, M = (16, 16, 16), 32, 64
    pot = inputs.potential(L, 1.0, 21)
    Ho, a, b = oracle_problem(L, pot)
    vs = [inputs.phase_block(Ho.n, R, s) for s in (21, 22)]
    refs = [O.kpm_moments(Ho, a, b, v, M) for v in vs]
    H = K.build_hamiltonian(L, pot)
    V = [torch.from_numpy(v).cuda() for v in vs]
    x = [torch.from_numpy(v[:, 0].copy()).cuda() for v in vs]
    y = [torch.from_numpy(v[:, 1].copy()).cuda() for v in vs]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    mus, dots = [None, None], [None, None]
    for rep in range(3):
        for i in (0, 1):
            with torch.cuda.stream(streams[i]):
                mus[i] = K.moments(H, V[i], M, check=False, stream=streams[i])
                dots[i] = K.dot(x[i], y[i], stream=streams[i])
        torch.cuda.synchronize()
        for i in (0, 1):
            err = float(np.abs(mus[i].cpu().numpy() - refs[i]).max())
            d = dots[i].cpu().numpy()
            ref_d = O.block_dot(vs[i][:, 0], vs[i][:, 1])[0]
            say("two streams", rep, i, err, abs(complex(d[0], d[1]) - ref_d))
            assert err <= TOL_C128
            assert abs(complex(d[0], d[1]) - ref_d) <= 1e-14
    H.close()


@pytest.mark.parametrize("kind", ["copy", "triad"])
@pytest.mark.parametrize("n", [2, 518, 3 * (1 << 20) + 14])
@pytest.mark.parametrize("wg,nt", [(1, False), (2, True), (8, True)])
def test_stream_kernels_write_every_unit(kind, n, wg, nt):
    # the attainable-bandwidth kernels on lengths that leave partial unroll groups and
    # grids smaller than the device; integer-valued inputs make the triad exact
    K = kpm()
    say("stream", kind, n, wg, nt)
    a = torch.arange(n, dtype=torch.float64, device="cuda")
    b = torch.arange(n, dtype=torch.float64, device="cuda") * 2.0 - 5.0
    c = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    K.stream_kernel(kind, c, a, b if kind == "triad" else None, 3.0, wg_per_cu=wg, nontemporal=nt)
    torch.cuda.synchronize()
    expect = a if kind == "copy" else a + 3.0 * b
    assert torch.equal(c, expect)
    # a length that is not a whole number of 16-byte units is refused
    with pytest.raises(K.KPMError):
        K.stream_kernel(kind, c[:n - 1], a[:n - 1], b[:n - 1] if kind == "triad" else None)


@pytest.mark.parametrize("n", [2, 518, 3 * (1 << 20) + 14])
@pytest.mark.parametrize("wg,nt", [(1, False), (1, True), (4, True)])
def test_stream_read_kernel_sums_every_unit(n, wg, nt):
    # the read-only bandwidth kernel: per-workgroup sums of integer values, exact in FP64
    K = kpm()
    say("stream read", n, wg, nt)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    a = torch.arange(n, dtype=torch.float64, device="cuda") - 7.0
    part = torch.zeros(cus * wg, dtype=torch.float64, device="cuda")
    K.stream_kernel("read", part, a, wg_per_cu=wg, nontemporal=nt)
    torch.cuda.synchronize()
    assert float(part.sum().item()) == float(a.sum().item()) == float(n * (n - 1) // 2 - 7 * n)
    with pytest.raises(ValueError):       # c too small for the grid
        K.stream_kernel("read", part[:cus * wg - 1], a, wg_per_cu=wg)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_column_groups_give_the_whole_block_moments(dtype):
    # kpm_run_opts.group: the R columns as independent recurrences of a
    # narrower width (the matrix read once per group) give the moments of
    # the whole block up to the order of the scalar products' sums
    from paper_1410_5242_amd import kpm as K
    L, R, M = (16, 16, 12), 64, 48
    pot = inputs.potential(L, 1.0, 5)
    H = K.build_hamiltonian(L, pot, dtype=dtype)
    v0 = inputs.phase_block(H.N, R, 8)
    V0 = torch.from_numpy(v0.astype(np.complex128 if dtype == "c128" else np.complex64)).cuda()
    whole = K.moments(H, V0, M).cpu().numpy()
    tol = 1e-13 if dtype == "c128" else 1e-6
    for g in (32, 16, 1):
        mu = K.moments(H, V0, M, group=g).cpu().numpy()
        assert np.abs(mu - whole).max() <= tol, g
    Ho = O.ti_hamiltonian(L, pot)
    a, b = O.scaling(*O.gershgorin(Ho))
    cols = [3, 40]
    ref = O.kpm_moments(Ho, a, b, v0[:, cols], M)
    mu = K.moments(H, V0, M, group=16).cpu().numpy()
    assert np.abs(mu[cols] - ref).max() <= (1e-12 if dtype == "c128" else 1e-5)
    # replayed from a graph: the whole grouped sequence, every replay equal
    g1 = K.moments(H, V0, M, group=16, graph=True).cpu().numpy()
    g2 = K.moments(H, V0, M, group=16, graph=True).cpu().numpy()
    assert np.array_equal(g1, mu) and np.array_equal(g2, mu)
    # a width that does not divide R, or a raw eta wanted from several groups
    with pytest.raises(K.KPMError) as e:
        K.moments(H, V0, M, group=3)
    assert e.value.status == K.KPM_EINVAL
    eta = torch.zeros((M, R, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(K.KPMError) as e:
        K.moments(H, V0, M, group=32, eta=eta)
    assert e.value.status == K.KPM_ENOTSUP
    H.close()


@pytest.mark.slow
@pytest.mark.parametrize("L,R,dtype,group,auto", [
    ((128, 128, 64), 64, "c128", 0, 32),     # 4 GiB block: two 32-column groups by default
    ((128, 128, 64), 64, "c128", 64, 32),    # the whole block: per-plane descriptors, two slices
    ((128, 128, 128), 32, "c128", 0, 32),    # 4 GiB even at 32 columns: per-plane descriptors
    ((128, 128, 128), 64, "c64", 64, 32),    # the whole 4 GiB block in complex64, per plane
])
def test_blocks_of_4_gib_on_the_lattice_sweep(L, R, dtype, group, auto):
    # blocks past the 32-bit offsets of one buffer descriptor: the lattice
    # sweep addresses V, W and the matrix plane by plane; two sampled
    # columns against the oracle over the first 8 moments
    from paper_1410_5242_amd import kpm as K
    M, seed = 8, 2
    say("4 GiB block", L, R, dtype, group)
    pot = inputs.potential(L, 2.0, 0)
    H = K.build_hamiltonian(L, pot, dtype=dtype)
    plan = K.sweep_plan(H, R)
    assert plan["kernel"] == "lattice_kernel" and plan["group"] == auto and plan["pieces"] == 1
    V0 = K.random_phase_block(H.N, R, seed, dtype)
    assert V0.numel() * V0.element_size() >= 1 << 32
    mu = K.moments(H, V0, M, group=group).cpu().numpy()
    del V0
    torch.cuda.empty_cache()
    H.close()
    cols = [5, R - 3]
    v0 = O.phase_block_counter(4 * L[0] * L[1] * L[2], R, seed)[:, cols].copy()
    Ho = O.ti_hamiltonian(L, pot)
    a, b = O.scaling(*O.gershgorin(Ho))
    ref = O.kpm_moments(Ho, a, b, v0, M)
    tol = 1e-12 if dtype == "c128" else 1e-5
    assert np.abs(mu[cols] - ref).max() <= tol
    assert np.abs(mu[:, 0] - 1.0).max() <= (1e-12 if dtype == "c128" else 1e-6)


@pytest.mark.slow
@pytest.mark.parametrize("R,dtype", [(32, "c128"), (64, "c64")])
def test_single_sweeps_on_4_gib_blocks_match_the_matrix(R, dtype):
    # kpm_aug_spmmv on 4 GiB blocks (128^3 sites: R = 32 in complex128, R = 64
    # in complex64, the record-in-LDS instantiation): the lattice sweep with
    # per-plane descriptors in its three variants; rows of every plane class
    # (first, last, interior planes; tile edges) against products with the
    # oracle's CRS rows (in complex64 against the rounded matrix and block)
    from paper_1410_5242_amd import kpm as K
    L = (128, 128, 128)
    say("4 GiB single sweeps", R, dtype)
    pot = inputs.potential(L, 1.0, 1)
    H = K.build_hamiltonian(L, pot, dtype=dtype)
    assert K.sweep_kernel(H, R) == "lattice_kernel"
    N = H.N
    V = K.random_phase_block(N, R, 3, dtype)
    W = K.random_phase_block(N, R, 4, dtype)
    assert V.numel() * V.element_size() >= 1 << 32
    rng = np.random.default_rng(0)
    plane = 4 * L[0] * L[1]
    rows = np.unique(np.concatenate([rng.integers(0, plane, 300), rng.integers(N - plane, N, 300),
                                     rng.integers(0, N, 600), np.arange(0, 64), N - 1 - np.arange(64)]))
    Ho = O.ti_hamiltonian(L, pot)
    cdt = np.complex128 if dtype == "c128" else np.complex64
    cols_needed = np.unique(np.concatenate([Ho.col[Ho.rowptr[i]:Ho.rowptr[i + 1]] for i in rows] + [rows]))
    Vh = V[torch.from_numpy(cols_needed).cuda()].cpu().numpy().astype(np.complex128)
    idx = {int(c): j for j, c in enumerate(cols_needed)}
    hval = Ho.val.astype(cdt).astype(np.complex128)   # the stored matrix entries

    def hx(i):
        k = np.arange(Ho.rowptr[i], Ho.rowptr[i + 1])
        return sum(hval[kk] * Vh[idx[int(Ho.col[kk])]] for kk in k)

    ref_hv = np.stack([hx(i) for i in rows])
    w0 = W[torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.complex128)
    v_rows = Vh[[idx[int(i)] for i in rows]]
    scale = np.abs(ref_hv).max()
    tol = 1e-12 if dtype == "c128" else 5e-6   # complex64: products and sums in the storage precision
    alpha, beta, gamma = 0.3, -0.7, -1.0
    K.aug_spmmv(H, V, W, alpha, beta, gamma, variant="nodot")
    got = W[torch.from_numpy(rows).cuda()].cpu().numpy()
    ref = alpha * ref_hv + beta * v_rows + gamma * w0
    assert np.abs(got - ref).max() <= tol * max(scale, np.abs(ref).max())
    K.aug_spmmv(H, V, W, 1.0, 0.0, 0.0, variant="plain")
    got = W[torch.from_numpy(rows).cuda()].cpu().numpy()
    assert np.abs(got - ref_hv).max() <= tol * scale
    eta = torch.zeros((2, R, 2), dtype=torch.float64, device="cuda")
    K.aug_spmmv(H, V, W, 1.0, 0.0, 0.0, variant="full", eta=eta)   # W = H V again; eta_0 = <V|V> = 1
    e = eta.cpu().numpy()
    assert np.abs(e[0, :, 0] - 1.0).max() <= (1e-12 if dtype == "c128" else 1e-6)
    del V, W
    torch.cuda.empty_cache()
    H.close()
