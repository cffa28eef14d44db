"""GPU parity of the learned-reconstruction network (BF16 MFMA kernels).

The GEMM is checked against a float64 product of the same BF16 inputs.  The
network's forward pass and gradients are checked against the FP64 oracle
(oracle/mlp.py) run on the same BF16-rounded weights and inputs: the GPU also
rounds the hidden activations and the layer gradients to BF16, so the bar is
a normwise relative error of 2e-2 per tensor.  The Adam update is checked
against the oracle's update applied to the GPU's own gradients.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import mlp as OM

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def bf16_round(x):
    """Round float values to the nearest BF16 (ties to even), returned as float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def bf16_bits(x):
    return (bf16_round(x).view(np.uint32) >> 16).astype(np.uint16)


def dev_bits(a):
    return torch.from_numpy(bf16_bits(a).view(np.int16)).cuda()


@pytest.mark.parametrize("M,N,K", [(64, 64, 32), (70, 100, 45), (129, 513, 512), (1, 17, 300)])
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True)])
def test_gemm_bf16_matches_float64_product(M, N, K, ta, tb):
    from paper_1410_5242_amd import kpm as K_
    say("gemm", M, N, K, ta, tb)
    g = np.random.default_rng(M * 7 + N + K)
    A = bf16_round(g.standard_normal((M, K)))
    B = bf16_round(g.standard_normal((K, N)))
    ref = A.astype(np.float64) @ B.astype(np.float64)
    Ad = dev_bits(A.T.copy() if ta else A)
    Bd = dev_bits(B.T.copy() if tb else B)
    C = K_.gemm_bf16(Ad, Bd, trans_a=ta, trans_b=tb)
    torch.cuda.synchronize()
    err = np.abs(C.cpu().numpy() - ref).max()
    assert err <= 1e-5 * np.sqrt(K) * max(1.0, np.abs(ref).max()), err


def make_net_and_data(B=64, seed=1, n_in=129, H=512, n_out=512):
    from paper_1410_5242_amd import kpm as K_
    P = OM.init_params(n_in, H, n_out, seed=seed)
    g = np.random.default_rng(seed + 100)
    for k in ("b1", "b2", "b3", "b4", "b5"):
        P[k] = g.uniform(-0.1, 0.1, size=P[k].shape)
    # the GPU computes with BF16 copies of the weight matrices and FP32 biases
    Pr = {k: (bf16_round(v).astype(np.float64) if k.startswith(("W", "w")) else
              np.asarray(v, dtype=np.float32).astype(np.float64)) for k, v in P.items()}
    x = np.concatenate([g.uniform(-1, 1, size=(B, n_in - 1)), g.uniform(0, 4, size=(B, 1))], axis=1)
    xr = bf16_round(x).astype(np.float64)
    p = g.dirichlet(np.ones(n_out) * 0.5, size=B)
    t = g.uniform(0.0, 0.3, size=B)
    net = K_.MLP(n_in, H, n_out, max_batch=max(B, 8))
    net.set_params(P)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    return net, P, Pr, x, xr, p, t, dev


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def test_forward_matches_oracle():
    say("mlp forward")
    net, P, Pr, x, xr, p, t, dev = make_net_and_data()
    q, e = net.forward(dev(x))
    torch.cuda.synchronize()
    q_ref, e_ref, _ = OM.forward(Pr, xr)
    assert rel(q.cpu().numpy(), q_ref) <= 2e-2
    assert rel(e.cpu().numpy(), e_ref) <= 2e-2
    assert np.allclose(q.cpu().numpy().sum(axis=1), 1.0, atol=1e-5)
    # parameters round-trip exactly through the device
    flat = net.get_params()
    from paper_1410_5242_amd import kpm as K_
    assert np.array_equal(flat, K_.flatten_params(P))


@pytest.mark.parametrize("lam", [1.0, 0.0])
def test_gradients_match_oracle(lam):
    from paper_1410_5242_amd import kpm as K_
    say("mlp gradients lam", lam)
    net, P, Pr, x, xr, p, t, dev = make_net_and_data()
    loss = net.backward(dev(x), dev(p), dev(t), lam=lam)
    torch.cuda.synchronize()
    G = K_.unflatten_params(net.get_grads(), 129, 512, 512)
    Gr = OM.backward(Pr, xr, p, t, lam=lam)
    for k in K_.MLP_PARAM_ORDER:
        if lam == 0.0 and k in ("w5", "b5"):
            assert np.abs(G[k]).max() == 0.0
            continue
        r = rel(G[k].reshape(Gr[k].shape), Gr[k])
        assert r <= 2e-2, (k, r)
    assert abs(float(loss.item()) - OM.loss(Pr, xr, p, t, lam=lam)) <= 2e-2 * abs(OM.loss(Pr, xr, p, t, lam=lam))


def test_adam_step_matches_oracle_update():
    from paper_1410_5242_amd import kpm as K_
    say("mlp adam")
    net, P, Pr, x, xr, p, t, dev = make_net_and_data(B=32)
    w0 = K_.unflatten_params(net.get_params(), 129, 512, 512)
    net.backward(dev(x), dev(p), dev(t), lam=1.0)
    G = K_.unflatten_params(net.get_grads(), 129, 512, 512)
    net.adam_step(lr=1e-3)
    w1 = K_.unflatten_params(net.get_params(), 129, 512, 512)
    m = {k: np.zeros_like(v) for k, v in w0.items()}
    v = {k: np.zeros_like(v_) for k, v_ in w0.items()}
    ref = {k: val.copy() for k, val in w0.items()}
    OM.adam_step(ref, G, m, v, 1, lr=1e-3)
    for k in K_.MLP_PARAM_ORDER:
        assert np.abs(w1[k] - ref[k]).max() <= 1e-6 + 1e-6 * np.abs(ref[k]).max(), k


def test_training_reduces_loss_and_self_target():
    say("mlp training")
    n_in, H, n_out, B = 33, 64, 48, 128
    from paper_1410_5242_amd import kpm as K_
    g = np.random.default_rng(3)
    x = g.uniform(-1, 1, size=(B, n_in))
    Wt = g.standard_normal((n_in, n_out))
    z = x @ Wt
    p = np.exp(z - z.max(axis=1, keepdims=True))
    p /= p.sum(axis=1, keepdims=True)
    net = K_.MLP(n_in, H, n_out, max_batch=B)
    net.set_params(OM.init_params(n_in, H, n_out, seed=0))
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    pd = torch.from_numpy(p.astype(np.float32)).cuda()
    first = float(net.train_step(xd, pd, None, lam=1.0, lr=3e-3).item())
    for _ in range(300):
        last = float(net.train_step(xd, pd, None, lam=1.0, lr=3e-3).item())
    assert np.isfinite(last) and last < 0.5 * first, (first, last)
    q, e = net.forward(xd)
    l1 = np.abs(q.cpu().numpy() - p).sum(axis=1)
    # the error head learned the size of its own L1 error
    assert abs(float(e.mean().item()) - float(l1.mean())) <= 0.5 * float(l1.mean()) + 0.02


def test_mlp_errors():
    from paper_1410_5242_amd import kpm as K_
    with pytest.raises(K_.KPMError):
        K_.MLP(0, 8, 8)
    net = K_.MLP(8, 16, 8, max_batch=4)
    with pytest.raises(K_.KPMError):
        net.forward(torch.zeros((5, 8), dtype=torch.float32, device="cuda"))
    bad = np.full(net.param_count, np.nan, dtype=np.float32)
    with pytest.raises(K_.KPMError):
        net.set_params(bad)
