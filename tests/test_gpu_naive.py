"""GPU parity of the naive KPM-DOS algorithm (Alg. "kpm_naive": one SpMV and
separate axpy / scal / nrm2 / dot calls per step) and of its BLAS level-1
kernels.  The naive moments must reproduce the CPU oracle's (1e-12 in
complex128, 1e-5 with complex64 storage) and the fused path's to rounding."""
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
    yield torch.device("cuda:0")


# lengths: single elements, odd counts (a complex64 tail), several thousand
# workgroups' worth (grid-stride loop)
LENGTHS = [1, 2, 3, 1001, (1 << 20) + 7]


@pytest.mark.parametrize("n", LENGTHS)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_blas1_kernels_match_numpy(n, dtype):
    K = kpm()
    say("blas1", dtype, n)
    cdt = np.complex128 if dtype == "c128" else np.complex64
    rng = np.random.default_rng(n)
    x = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(cdt)
    y = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(cdt)
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    eps = np.finfo(np.float64 if dtype == "c128" else np.float32).eps
    # axpy and scal in the storage precision: within one rounding of each part
    K.axpy(-0.375, xt, yt)
    ref = y.astype(np.complex128) - 0.375 * x.astype(np.complex128)
    assert np.abs(yt.cpu().numpy() - ref).max() <= 4 * eps * np.abs(ref).max()
    K.scal(1.25, xt)
    assert np.abs(xt.cpu().numpy() - 1.25 * x.astype(np.complex128)).max() <= 2 * eps * np.abs(x).max()
    # scalar products in FP64 of the stored values
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    x64, y64 = x.astype(np.complex128), y.astype(np.complex128)
    d = K.dot(xt, yt).cpu().numpy()
    ref = np.sum(np.conj(x64) * y64)
    scale = np.sum(np.abs(x64) * np.abs(y64))
    assert abs(complex(d[0], d[1]) - ref) <= 1e-14 * scale
    nr = K.dot(xt, xt).cpu().numpy()
    assert nr[1] == 0.0
    assert abs(nr[0] - np.sum(np.abs(x64) ** 2)) <= 1e-14 * np.sum(np.abs(x64) ** 2)


def test_dot_is_deterministic():
    K = kpm()
    rng = np.random.default_rng(3)
    n = 3 << 18
    x = torch.from_numpy(rng.standard_normal(n) + 1j * rng.standard_normal(n)).cuda()
    y = torch.from_numpy(rng.standard_normal(n) + 1j * rng.standard_normal(n)).cuda()
    first = K.dot(x, y).cpu().numpy()
    for _ in range(3):
        assert np.array_equal(K.dot(x, y).cpu().numpy(), first)


NAIVE_CASES = [((8, 8, 8), (1, 1, 1), 1, 128), ((7, 5, 6), (1, 1, 1), 4, 48), ((6, 4, 5), (0, 1, 0), 2, 40),
               ((3, 3, 3), (1, 1, 1), 8, 32)]


@pytest.mark.parametrize("L,periodic,R,M", NAIVE_CASES)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_naive_moments_match_oracle(L, periodic, R, M, dtype):
    K = kpm()
    say("naive moments", L, periodic, "R", R, "M", M, dtype)
    pot = inputs.potential(L, 1.0, 0)
    Ho = O.ti_hamiltonian(L, pot, periodic=periodic)
    a, b = O.scaling(*O.gershgorin(Ho))
    v0 = inputs.phase_block(Ho.n, R, 1)
    ref = O.kpm_moments(Ho, a, b, v0, M)
    H = K.build_hamiltonian(L, pot, periodic=periodic, dtype=dtype)
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    V0 = torch.from_numpy(v0).cuda().to(tdt)
    mu = K.moments_naive(H, V0, M).cpu().numpy()
    fused = K.moments(H, V0, M).cpu().numpy()
    H.close()
    assert np.abs(mu - ref).max() <= (TOL_C128 if dtype == "c128" else TOL_C64)
    assert np.abs(mu - fused).max() <= (1e-13 if dtype == "c128" else 1e-5)


def test_naive_edge_cases():
    # minimal M (the initialisation only), the widest block, empty BLAS-1 calls
    K = kpm()
    L = (3, 4, 3)
    pot = inputs.potential(L, 1.0, 2)
    Ho = O.ti_hamiltonian(L, pot, periodic=(1, 1, 0))
    a, b = O.scaling(*O.gershgorin(Ho))
    H = K.build_hamiltonian(L, pot, periodic=(1, 1, 0))
    for R, M in ((1, 2), (64, 6)):
        v0 = inputs.phase_block(Ho.n, R, R)
        mu = K.moments_naive(H, torch.from_numpy(v0).cuda(), M).cpu().numpy()
        assert np.abs(mu - O.kpm_moments(Ho, a, b, v0, M)).max() <= TOL_C128
    H.close()
    e = torch.empty(0, dtype=torch.complex128, device="cuda")
    K.axpy(2.0, e, e)
    K.scal(2.0, e)
    assert np.array_equal(K.dot(e, e).cpu().numpy(), [0.0, 0.0])
    with pytest.raises(K.KPMError):
        K.moments_naive(K.build_hamiltonian(L, pot, periodic=(1, 1, 0)), torch.from_numpy(
            inputs.phase_block(Ho.n, 3, 0)).cuda(), 8)   # R = 3 is not a supported block width
