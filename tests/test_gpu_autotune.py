"""The autotuner on the GPU: every candidate it times is a valid launch shape,
the winner is applied from the JSON cache, and moments computed under the
tuned shapes still match the CPU oracle."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_1410_5242_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield
    from paper_1410_5242_amd import kpm as K
    K.reset_sweep_tuning()
    K.reset_batch_tuning()


def test_tune_sweep_then_moments_match_oracle(tmp_path):
    from paper_1410_5242_amd import autotune as A, kpm as K
    L, R, M = (16, 16, 12), 32, 40
    say("tune sweep", L, R)
    pot = inputs.potential(L, 1.0, 4)
    H = K.build_hamiltonian(L, pot)
    cands = [dict(wg_per_cu=wg, xcd_ways=8, chunk_tiles=ch, pencil=p, dynamic=0, prefetch=pf, stream=st, lattice=lat,
                  gather=g)
             for wg, ch, p, pf, st, lat, g in [(8, 8, 16, 2, 3, 1, 0), (4, 4, 0, 0, 0, 0, 2), (8, 16, 16, 0, 3, 0, 2),
                                               (4, 8, 0, 2, 3, 2, 0), (2, 8, 16, 0, 3, 0, 1)]]
    cache = A.TuningCache(str(tmp_path / "t.json"))
    res = A.tune_sweep(H, R, cache=cache, candidates=cands, sweeps=4, repeats=2, L=L)
    assert res.best in cands and len(res.trials) == len(cands)
    assert all(t.seconds > 0 for t in res.trials)
    cache.save()
    K.reset_sweep_tuning()
    assert A.apply_sweep(A.TuningCache(cache.path), H, R, L=L)
    got = K.get_sweep_tuning()
    assert all(got[k] == res.best[k] for k in res.best)
    Ho = O.ti_hamiltonian(L, pot)
    a, b = O.scaling(*O.gershgorin(Ho))
    v0 = inputs.phase_block(Ho.n, R, 9)
    mu = K.moments(H, torch.from_numpy(v0).cuda(), M)
    torch.cuda.synchronize()
    assert np.abs(mu.cpu().numpy() - O.kpm_moments(Ho, a, b, v0, M)).max() <= 1e-12
    K.reset_sweep_tuning()


def test_tune_batched_and_block_width(tmp_path):
    from paper_1410_5242_amd import autotune as A, kpm as K
    R, M = 8, 32
    say("tune batched")
    fam = inputs.instance_family(24, (4, 6, 8), 4.0, 3)
    Hs, V0s, hosts = [], [], []
    for f in fam:
        pot = inputs.potential(f["L"], f["gamma"], f["pot_seed"])
        H = K.build_hamiltonian(f["L"], pot, dtype="c64")
        v0 = inputs.phase_block(H.N, R, f["vec_seed"])
        Hs.append(H)
        V0s.append(torch.from_numpy(v0.astype(np.complex64)).cuda())
        hosts.append((f["L"], pot, v0))
    cands = [dict(waves=8, wg_per_cu=1, dynamic=1), dict(waves=4, wg_per_cu=2, dynamic=0),
             dict(waves=16, wg_per_cu=1, dynamic=1)]
    cache = A.TuningCache(str(tmp_path / "b.json"))
    res = A.tune_batched(Hs, V0s, M, cache=cache, candidates=cands, repeats=1)
    assert res.best in cands
    K.reset_batch_tuning()
    assert A.apply_batched(cache, Hs, R)
    got = K.get_batch_tuning()
    assert {k: got[k] for k in res.best} == res.best
    mu = K.moments_batched(Hs, V0s, M).cpu().numpy()
    for i in (0, len(fam) // 2, len(fam) - 1):
        L, pot, v0 = hosts[i]
        Ho = O.ti_hamiltonian(L, pot)
        a, b = O.scaling(*O.gershgorin(Ho))
        assert np.abs(mu[i] - O.kpm_moments(Ho, a, b, v0, M)).max() <= 1e-5
    K.reset_batch_tuning()
    say("tune block width")
    res = A.tune_block_width(Hs[-1], 16, cache=cache, sweeps=2, repeats=1)
    assert res.best["R"] in (1, 2, 4, 8, 16) and len(res.trials) == 5


def test_tune_sell_layout_then_moments_match_oracle(tmp_path):
    # the SELL-C-sigma layout of a general matrix as a tuning dimension
    from paper_1410_5242_amd import autotune as A, kpm as K
    N, R, M = 6000, 8, 48
    say("tune sell layout", N, R)
    rowptr, col, val = inputs.random_hermitian_csr(N, seed=12)
    cands = [{"C": 8, "sigma": 1024}, {"C": 1, "sigma": 1}, {"C": 32, "sigma": 1}, {"C": 64, "sigma": 4096}]
    cache = A.TuningCache(str(tmp_path / "s.json"))
    res = A.tune_sell_layout(rowptr, col, val, R, cache=cache, candidates=cands, sweeps=4, repeats=2)
    assert res.best in cands and len(res.trials) == len(cands)
    _, _, start = K.sell_layout(rowptr, 32, 1)
    assert [t.params["stored"] for t in res.trials][2] == int(start[-1])
    cache.save()
    assert A.TuningCache(cache.path).get(res.key) == res.best
    H = K.import_csr(rowptr, col, val, **res.best)
    Ho = O.CSR(rowptr, col, val)
    a, b = O.scaling(*O.gershgorin(Ho))
    K.set_scaling(H, a, b)
    v0 = inputs.phase_block(N, R, 2)
    mu = K.moments(H, torch.from_numpy(v0).cuda(), M).cpu().numpy()
    assert np.abs(mu - O.kpm_moments(Ho, a, b, v0, M)).max() <= 1e-12
    H.close()
