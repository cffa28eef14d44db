"""Learned DOS reconstruction on a family of disordered lattices.

A short run of the KPM (the first 128 Chebyshev moments of the stochastic
trace) plus the disorder strength is mapped by a small network to the DOS on
a fixed energy grid; the network also predicts the L1 error of its own
output, and every instance whose predicted error exceeds the caller's target
is solved again with the plain Jackson-kernel KPM (the fallback), so that
every returned DOS either passed the predicted bound or is plain KPM.

The family shares one scaling, b = 0 and a = 10.1 (1.01 times the
Gershgorin bound 10 that holds for every disorder strength up to 4:
|V| <= 2, onsite +-2, hopping row sum 6), so that the moments of all
instances live on one energy axis and the network sees comparable inputs.
Training data are this library's own KPM runs (M = 2048 moments, R = 16
random vectors, complex128); the truth for an instance is its Jackson DOS at
M = 2048, whose first 128 moments are exactly the network's input (prefix).

Everything numerical runs in the library's kernels (batched solver, batched
DOS, feature assembly, network); this module only schedules them.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import inputs
from . import kpm as K

A_FAMILY = 10.1
B_FAMILY = 0.0
N_MOM = 128
K_BINS = 512
M_TRUTH = 2048
R_TRUTH = 16
SIDES = tuple(range(16, 25))
GAMMA_MAX = 4.0
HIDDEN = 512
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "dos_mlp.safetensors")
TRAIN_SEED = 1
TEST_SEED = 2


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def family(n: int, seed: int):
    """n instances: L uniform in 16..24 (cubes, periodic), gamma ~ U[0, 4]."""
    return inputs.instance_family(n, SIDES, GAMMA_MAX, seed)


def energy_grid(K_: int = K_BINS, device="cuda") -> torch.Tensor:
    """Midpoints of K equal bins of [b - a, b + a] (never at the band edges +-a)."""
    k = torch.arange(K_, dtype=torch.float64)
    return (B_FAMILY + A_FAMILY * (-1.0 + (2.0 * k + 1.0) / K_)).to(device)


def build(fam, dtype: str):
    """Device Hamiltonians of the family with the fixed family scaling."""
    Hs = []
    for f in fam:
        pot = inputs.potential(f["L"], f["gamma"], f["pot_seed"])
        Hs.append(K.build_hamiltonian(f["L"], pot, dtype=dtype, fixed_scale=(A_FAMILY, B_FAMILY)))
    return Hs


def start_blocks(fam, Hs, R: int, dtype: str):
    return [K.random_phase_block(H.N, R, f["vec_seed"], dtype) for f, H in zip(fam, Hs)]


def solve(fam, M: int, R: int, dtype: str, chunk_rows: int = 60_000_000, mu: torch.Tensor | None = None,
          progress: bool = False):
    """Moments [n][R][M] of every instance (batched solver, chunks of at most chunk_rows rows)."""
    n = len(fam)
    if mu is None:
        mu = torch.empty((n, R, M), dtype=torch.float64, device="cuda")
    i = 0
    t0 = time.time()
    while i < n:
        j, rows = i, 0
        while j < n and (j == i or rows + 4 * np.prod(fam[j]["L"]) <= chunk_rows):
            rows += 4 * int(np.prod(fam[j]["L"]))
            j += 1
        Hs = build(fam[i:j], dtype)
        V0s = start_blocks(fam[i:j], Hs, R, dtype)
        K.moments_batched(Hs, V0s, M, mu=mu[i:j])
        torch.cuda.synchronize()
        for H in Hs:
            H.close()
        del V0s
        if progress:
            log(f"  solved {j}/{n} instances ({rows} rows in this chunk), {time.time() - t0:.1f} s")
        i = j
    return mu


def masses(mu: torch.Tensor, M: int | None = None, E: torch.Tensor | None = None) -> torch.Tensor:
    """Jackson DOS masses per bin [n][K] from the first M moments (float64)."""
    n = mu.shape[0]
    a = torch.full((n,), A_FAMILY, dtype=torch.float64, device=mu.device)
    b = torch.full((n,), B_FAMILY, dtype=torch.float64, device=mu.device)
    return K.dos_batched(mu, a, b, E if E is not None else energy_grid(), M=M, masses=True)


def features(mu: torch.Tensor, fam) -> torch.Tensor:
    g = torch.tensor([f["gamma"] for f in fam], dtype=torch.float32, device=mu.device)
    return K.moment_features(mu, N_MOM, extra=g)


def dataset(fam, progress: bool = False):
    """(x [n][129] float32, p [n][512] float32) from M = 2048, R = 16 complex128 runs."""
    mu = solve(fam, M_TRUTH, R_TRUTH, "c128", progress=progress)
    p = masses(mu).float()
    x = features(mu, fam)
    return x, p, mu


def l1(q: torch.Tensor, p: torch.Tensor) -> torch.Tensor:
    """Per-instance L1 distance of two DOS given as bin masses (= sum |rho1 - rho2| dE)."""
    return (q.double() - p.double()).abs().sum(dim=1)


def train(net: K.MLP, x: torch.Tensor, p: torch.Tensor, epochs: int = 60, batch: int = 256, lr: float = 1e-3,
          lr_min: float = 1e-5, lam: float = 1.0, seed: int = 0, progress: bool = False):
    """Adam with a cosine learning-rate schedule; error targets are each sample's own L1 error."""
    n = x.shape[0]
    g = torch.Generator().manual_seed(seed)
    steps = epochs * max(1, n // batch)
    step = 0
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(x.device)
        tot, cnt = 0.0, 0
        for s in range(0, n - batch + 1, batch):
            idx = perm[s:s + batch]
            rate = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * step / steps))
            loss = net.train_step(x[idx].contiguous(), p[idx].contiguous(), None, lam=lam, lr=rate)
            tot += float(loss.item()) if s == 0 or s + 2 * batch > n else 0.0
            cnt += 1 if s == 0 or s + 2 * batch > n else 0
            step += 1
        hist.append(tot / max(cnt, 1))
        if progress and (ep % 5 == 0 or ep == epochs - 1):
            log(f"  epoch {ep}: loss {hist[-1]:.4f}")
    return hist


def save_weights(net: K.MLP, path: str, meta: dict):
    from safetensors.numpy import save_file
    os.makedirs(os.path.dirname(path), exist_ok=True)
    save_file({"params": net.get_params()}, path, metadata={k: json.dumps(v) for k, v in meta.items()})


def load_weights(path: str = WEIGHTS, max_batch: int = 1024) -> tuple[K.MLP, dict]:
    from safetensors import safe_open
    with safe_open(path, framework="numpy") as f:
        meta = {k: json.loads(v) for k, v in (f.metadata() or {}).items()}
        flat = f.get_tensor("params")
    net = K.MLP(meta.get("n_in", N_MOM + 1), meta.get("hidden", HIDDEN), meta.get("n_out", K_BINS), max_batch)
    net.set_params(flat)
    return net, meta


def predict(net: K.MLP, x: torch.Tensor, chunk: int = 1024):
    """Network DOS masses [n][K] and predicted L1 errors [n]."""
    qs, es = [], []
    for s in range(0, x.shape[0], chunk):
        q, e = net.forward(x[s:s + chunk].contiguous())
        qs.append(q)
        es.append(e)
    return torch.cat(qs), torch.cat(es)


def reconstruct(net: K.MLP, fam, eps: float, M_fallback: int, dtype: str = "c64", R: int = R_TRUTH,
                mu_short: torch.Tensor | None = None):
    """Learned DOS with fallback: short run (first 128 moments) -> network; instances whose
    predicted error exceeds eps are re-solved with plain KPM at M_fallback.  Returns
    (masses [n][K] float64, fallback mask [n] bool)."""
    if mu_short is None:
        mu_short = solve(fam, N_MOM, R, dtype)
    x = features(mu_short, fam)
    q, e = predict(net, x)
    out = q.double()
    fb = e > eps
    idx = torch.nonzero(fb).flatten().tolist()
    if idx:
        sub = [fam[i] for i in idx]
        mu_fb = solve(sub, M_fallback, R, dtype)
        out[fb] = masses(mu_fb, M_fallback)
    return out, fb


def main(argv=None):
    ap = argparse.ArgumentParser(description="Train the learned DOS reconstruction on KPM runs of the family.")
    ap.add_argument("--n-train", type=int, default=20_000)
    ap.add_argument("--n-test", type=int, default=1_000)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--report", default=None, help="write the held-out evaluation as JSON here")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    t0 = time.time()
    log(f"generating {args.n_train} training instances (M={M_TRUTH}, R={R_TRUTH}, c128)")
    x, p, _ = dataset(family(args.n_train, TRAIN_SEED), progress=True)
    log(f"training data ready in {time.time() - t0:.1f} s")
    test_fam = family(args.n_test, TEST_SEED)
    xt, pt, mut = dataset(test_fam, progress=True)
    net = K.MLP(N_MOM + 1, HIDDEN, K_BINS, max_batch=max(args.batch, 1024))
    net.set_params(init_params(N_MOM + 1, HIDDEN, K_BINS, seed=0))
    t1 = time.time()
    hist = train(net, x, p, epochs=args.epochs, batch=args.batch, lr=args.lr, progress=True)
    torch.cuda.synchronize()
    log(f"trained in {time.time() - t1:.1f} s")
    rep = evaluate(net, test_fam, xt, pt, mut)
    rep.update(n_train=args.n_train, n_test=args.n_test, epochs=args.epochs, batch=args.batch, lr=args.lr,
               loss_history=hist, train_seconds=time.time() - t1, total_seconds=time.time() - t0)
    meta = dict(n_in=N_MOM + 1, hidden=HIDDEN, n_out=K_BINS, a=A_FAMILY, b=B_FAMILY, m_truth=M_TRUTH,
                r_truth=R_TRUTH, sides=list(SIDES), gamma_max=GAMMA_MAX, train_seed=TRAIN_SEED,
                n_train=args.n_train, epochs=args.epochs)
    save_weights(net, args.out, meta)
    log(json.dumps({k: v for k, v in rep.items() if k != "loss_history"}))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)
    return rep


def init_params(n_in: int, hidden: int, n_out: int, seed: int = 0) -> np.ndarray:
    """He-style initial weights (flat, in the library's parameter order), zero biases."""
    rng = np.random.default_rng([seed, 0x5EED_0004])
    dims = [n_in, hidden, hidden, hidden]
    parts = []
    for i in range(3):
        parts.append(rng.standard_normal((dims[i], dims[i + 1])) * math.sqrt(2.0 / dims[i]))
        parts.append(np.zeros(dims[i + 1]))
    parts.append(rng.standard_normal((hidden, n_out)) * math.sqrt(1.0 / hidden))
    parts.append(np.zeros(n_out))
    parts.append(rng.standard_normal((hidden, 1)) * math.sqrt(1.0 / hidden))
    parts.append(np.zeros(1))
    return np.concatenate([a.reshape(-1) for a in parts]).astype(np.float32)


def evaluate(net: K.MLP, fam, x: torch.Tensor, p: torch.Tensor, mu: torch.Tensor) -> dict:
    """Held-out L1 errors: network vs plain Jackson KPM at several M (prefixes of the truth run)."""
    q, e = predict(net, x)
    err_net = l1(q, p)
    out = {"net_l1_mean": float(err_net.mean()), "net_l1_median": float(err_net.median()),
           "pred_err_mean": float(e.mean()),
           "pred_err_corr": float(np.corrcoef(e.double().cpu().numpy(), err_net.cpu().numpy())[0, 1])}
    for M in (64, 128, 256, 512, 1024):
        out[f"kpm_l1_mean_M{M}"] = float(l1(masses(mu, M), p).mean())
    for eps in (0.05, 0.02):
        fb = e > eps
        err = torch.where(fb, torch.zeros_like(err_net), err_net)
        out[f"eps{eps}"] = {"fallback_fraction": float(fb.double().mean()),
                            "accepted_l1_max": float(err.max()),
                            "accepted_over_eps": float(((err_net > eps) & ~fb).double().mean())}
    return out


if __name__ == "__main__":
    main()
