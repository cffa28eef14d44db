"""The learned-reconstruction pipeline on the GPU.

(1) The family data path (fixed family scaling, device start blocks,
batched solver, batched DOS masses, moment features) against the CPU oracle.
(2) The trained network against plain KPM on held-out instances: from the
first 128 moments the network's DOS is closer to the M = 4096 truth than the
Jackson DOS of 512 moments, and the fallback returns, for every instance
whose predicted error exceeds the calibrated threshold, exactly the plain
KPM DOS.
"""
import os
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


def test_family_data_path_matches_oracle():
    from paper_1410_5242_amd import learned as LN
    say("family data path")
    fam = inputs.instance_family(5, (4, 5, 6), 4.0, 9)
    R, M = 4, 160
    mu = LN.solve(fam, M, R, "c128")
    q = LN.masses(mu, 64).cpu().numpy()
    x = LN.features(mu, fam).cpu().numpy()
    mu = mu.cpu().numpy()
    E = LN.energy_grid().cpu().numpy()
    for i, f in enumerate(fam):
        pot = inputs.potential(f["L"], f["gamma"], f["pot_seed"])
        Ho = O.ti_hamiltonian(f["L"], pot)
        v0 = O.phase_block_counter(Ho.n, R, f["vec_seed"])
        ref = O.kpm_moments(Ho, LN.A_FAMILY, LN.B_FAMILY, v0, M)
        assert np.abs(mu[i] - ref).max() <= 1e-12
        rho = O.dos(ref[:, :64].mean(axis=0), O.jackson(64), LN.A_FAMILY, LN.B_FAMILY, E)
        assert np.abs(q[i] - rho / rho.sum()).max() <= 1e-12 * max(1.0, np.abs(q[i]).max())
        assert np.abs(x[i, :LN.N_MOM] - ref[:, :LN.N_MOM].mean(axis=0)).max() <= 1e-6
        assert x[i, LN.N_MOM] == np.float32(f["gamma"])


def test_trained_network_gains_over_short_kpm_and_fallback_contract():
    from paper_1410_5242_amd import learned as LN
    assert os.path.exists(LN.WEIGHTS), "trained network weights are missing"
    say("learned vs short KPM")
    net, meta = LN.load_weights()
    assert meta["n_in"] == LN.N_MOM + 1 and meta["n_out"] == LN.K_BINS
    assert meta["m_truth"] == LN.M_TRUTH
    fam = LN.family(400, LN.TEST_SEED + 100)      # instances the network never saw
    x, p, mu = LN.dataset(fam)
    q, e = LN.predict(net, x)
    l1_net = LN.l1(q, p)
    l1_128 = LN.l1(LN.masses(mu, LN.N_MOM), p)
    l1_512 = LN.l1(LN.masses(mu, 512), p)
    say("mean L1: network", float(l1_net.mean()), "Jackson KPM at M=128", float(l1_128.mean()),
        "at M=512", float(l1_512.mean()))
    # what the network gains: from 128 moments it is closer to the truth than plain KPM from
    # 128 moments (by a wide margin) and than plain KPM from 512 moments
    assert float(l1_net.mean()) < 0.75 * float(l1_128.mean())
    assert float(l1_net.mean()) < float(l1_512.mean())
    # the error head orders the instances: predicted and actual errors correlate
    assert np.corrcoef(e.double().cpu().numpy(), l1_net.cpu().numpy())[0, 1] > 0.5
    eps = 0.08
    rec = meta["fallback"][str(eps)]
    tau, M_fb = rec["tau"], rec["M"]
    out, fb = LN.reconstruct(net, fam, eps, M_fb, dtype="c64", mu_short=mu[:, :, :LN.N_MOM].contiguous(), tau=tau)
    idx = torch.nonzero(fb).flatten().tolist()
    assert torch.equal(out[~fb], q[~fb].double())
    assert bool((e[~fb] <= tau).all())
    if idx:
        ref = LN.masses(mu[idx].contiguous(), M_fb)
        assert torch.allclose(out[fb], ref, rtol=0, atol=1e-14)
    net.close()
