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
Training data are this library's own KPM runs (M = 4096 moments, R = 16
random vectors, complex64 storage with FP64 products, whose moments differ
from complex128 ones by about 1e-8); the truth for an instance is its
Jackson DOS at M = 4096, whose first 128 moments are exactly the network's
input (prefix).  The fallback threshold for a target error eps is
calibrated on a validation split of the training family (never on the
instances it is evaluated on): the largest threshold on the predicted error
for which the mean L1 error of the mixed output (network where accepted,
plain KPM at the eps-M elsewhere) stays within eps, the criterion the plain
KPM variants meet.

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
M_TRUTH = 4096
R_TRUTH = 16
DATA_DTYPE = "c64"
M_CHOICES = (64, 128, 256, 512, 1024, 2048)   # candidate moment counts of the plain KPM
EPS_TARGETS = (0.08, 0.05)                    # mean L1 targets of the time-to-DOS comparison
N_TRAIN, N_VAL = 20_000, 1_000
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


def dataset(fam, progress: bool = False, dtype: str = DATA_DTYPE, M: int = M_TRUTH):
    """(x [n][129] float32, p [n][512] float32, mu) from M = 4096, R = 16 runs (complex64 storage)."""
    mu = solve(fam, M, R_TRUTH, dtype, progress=progress)
    p = masses(mu).float()
    x = features(mu, fam)
    return x, p, mu


def l1(q: torch.Tensor, p: torch.Tensor) -> torch.Tensor:
    """Per-instance L1 distance of two DOS given as bin masses (= sum |rho1 - rho2| dE)."""
    return (q.double() - p.double()).abs().sum(dim=1)


def _kl(q: torch.Tensor, p: torch.Tensor) -> float:
    """Mean KL divergence sum_k p log(p / q) of network masses q from target masses p (the
    cross-entropy term of the training loss minus the entropy of p)."""
    p = p.double()
    q = q.double().clamp_min(1e-300)
    t = torch.where(p > 0, p * (p.clamp_min(1e-300).log() - q.log()), torch.zeros_like(p))
    return float(t.sum(dim=1).mean())


def train(net: K.MLP, x: torch.Tensor, p: torch.Tensor, epochs: int = 400, batch: int = 512, lr: float = 3e-3,
          lr_min: float = 1e-5, lam: float = 1.0, seed: int = 0, val=None, every: int = 10,
          progress: bool = False):
    """Adam with a cosine learning-rate schedule; error targets are each sample's own L1 error.
    Returns the history: per epoch the mean training loss (cross-entropy + lam x squared
    error-head residual), and every `every` epochs (and the last) the validation KL divergence
    and mean / median L1 error when val = (x_val, p_val) is given."""
    n = x.shape[0]
    g = torch.Generator().manual_seed(seed)
    steps = epochs * max(1, n // batch)
    step = 0
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(x.device)
        losses = []
        for s in range(0, n - batch + 1, batch):
            idx = perm[s:s + batch]
            rate = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * step / steps))
            losses.append(net.train_step(x[idx].contiguous(), p[idx].contiguous(), None, lam=lam, lr=rate))
            step += 1
        rec = {"epoch": ep, "train_loss": float(torch.stack(losses).mean().item())}
        if val is not None and (ep % every == 0 or ep == epochs - 1):
            q, _ = predict(net, val[0])
            e = l1(q, val[1])
            rec.update(val_kl=_kl(q, val[1]), val_l1_mean=float(e.mean()), val_l1_median=float(e.median()))
            if progress:
                log(f"  epoch {ep}: loss {rec['train_loss']:.4f} val KL {rec['val_kl']:.4f} "
                    f"val L1 {rec['val_l1_mean']:.4f} (median {rec['val_l1_median']:.4f})")
        hist.append(rec)
    return hist


def kpm_choice(mu: torch.Tensor, p: torch.Tensor, eps: float):
    """Smallest plain-KPM moment count in M_CHOICES whose mean L1 error over the instances is
    within eps (None if none is), and the mean errors per M."""
    err = {M: float(l1(masses(mu, M), p).mean()) for M in M_CHOICES}
    return next((M for M in M_CHOICES if err[M] <= eps), None), err


def calibrate(net: K.MLP, x: torch.Tensor, p: torch.Tensor, mu: torch.Tensor, eps_list=EPS_TARGETS) -> dict:
    """Fallback thresholds on the predicted error, one per target eps, from validation data: the
    largest tau such that the mean L1 error of (network where predicted <= tau, plain KPM at the
    eps-M elsewhere) is within eps."""
    q, e = predict(net, x)
    err_net = l1(q, p).cpu().numpy()
    pred = e.double().cpu().numpy()
    out = {}
    for eps in eps_list:
        M, _ = kpm_choice(mu, p, eps)
        if M is None:
            continue
        err_kpm = l1(masses(mu, M), p).cpu().numpy()
        order = np.argsort(pred, kind="stable")
        # mean error when the k instances of smallest predicted error take the network's DOS
        gain = np.concatenate([[0.0], np.cumsum(err_net[order] - err_kpm[order])])
        mean = (err_kpm.sum() + gain) / len(order)
        ok = np.nonzero(mean <= eps)[0]
        k = int(ok.max()) if ok.size else 0
        out[str(eps)] = {"tau": float(pred[order[k - 1]]) if k > 0 else -1.0, "M": M,
                         "val_mean_l1": float(mean[k]), "val_accepted_fraction": k / len(order)}
    return out


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
                mu_short: torch.Tensor | None = None, tau: float | None = None):
    """Learned DOS with fallback: short run (first 128 moments) -> network; instances whose
    predicted error exceeds tau (default eps) are re-solved with plain KPM at M_fallback.  Returns
    (masses [n][K] float64, fallback mask [n] bool)."""
    if mu_short is None:
        mu_short = solve(fam, N_MOM, R, dtype)
    x = features(mu_short, fam)
    q, e = predict(net, x)
    out = q.double()
    fb = e > (eps if tau is None else tau)
    idx = torch.nonzero(fb).flatten().tolist()
    if idx:
        sub = [fam[i] for i in idx]
        mu_fb = solve(sub, M_fallback, R, dtype)
        out[fb] = masses(mu_fb, M_fallback)
    return out, fb


def main(argv=None):
    ap = argparse.ArgumentParser(description="Train the learned DOS reconstruction on KPM runs of the family.")
    ap.add_argument("--n-train", type=int, default=N_TRAIN)
    ap.add_argument("--n-val", type=int, default=N_VAL)
    ap.add_argument("--n-test", type=int, default=1_000)
    ap.add_argument("--epochs", type=int, default=400)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--report", default=None, help="write the held-out evaluation as JSON here")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    t0 = time.time()
    log(f"generating {args.n_train} + {args.n_val} training / validation instances "
        f"(M={M_TRUTH}, R={R_TRUTH}, {DATA_DTYPE})")
    fam_all = family(args.n_train + args.n_val, TRAIN_SEED)
    x, p, _ = dataset(fam_all[:args.n_train], progress=True)
    xv, pv, muv = dataset(fam_all[args.n_train:])
    log(f"training data ready in {time.time() - t0:.1f} s")
    test_fam = family(args.n_test, TEST_SEED)
    xt, pt, mut = dataset(test_fam)
    net = K.MLP(N_MOM + 1, HIDDEN, K_BINS, max_batch=max(args.batch, 1024))
    net.set_params(init_params(N_MOM + 1, HIDDEN, K_BINS, seed=0))
    t1 = time.time()
    hist = train(net, x, p, epochs=args.epochs, batch=args.batch, lr=args.lr, val=(xv, pv), progress=True)
    torch.cuda.synchronize()
    train_s = time.time() - t1
    log(f"trained in {train_s:.1f} s")
    fallback = calibrate(net, xv, pv, muv)
    rep = evaluate(net, test_fam, xt, pt, mut, fallback)
    rep.update(n_train=args.n_train, n_val=args.n_val, n_test=args.n_test, epochs=args.epochs, batch=args.batch,
               lr=args.lr, m_truth=M_TRUTH, data_dtype=DATA_DTYPE, fallback=fallback, history=hist,
               train_seconds=train_s, total_seconds=time.time() - t0)
    meta = dict(n_in=N_MOM + 1, hidden=HIDDEN, n_out=K_BINS, a=A_FAMILY, b=B_FAMILY, m_truth=M_TRUTH,
                r_truth=R_TRUTH, data_dtype=DATA_DTYPE, sides=list(SIDES), gamma_max=GAMMA_MAX,
                train_seed=TRAIN_SEED, n_train=args.n_train, n_val=args.n_val, epochs=args.epochs,
                fallback=fallback)
    save_weights(net, args.out, meta)
    log(json.dumps({k: v for k, v in rep.items() if k != "history"}))
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


def evaluate(net: K.MLP, fam, x: torch.Tensor, p: torch.Tensor, mu: torch.Tensor, fallback: dict | None = None) -> dict:
    """Held-out L1 errors: network vs plain Jackson KPM at several M (prefixes of the truth run),
    against the M = 4096 truth and against the M = 2048 Jackson DOS of the same run; with the
    calibrated thresholds, the mixed output's mean error, fallback fraction and the fraction of
    instances above eps (for the network's and for the plain KPM's choice)."""
    q, e = predict(net, x)
    err_net = l1(q, p)
    p2048 = masses(mu, 2048)
    out = {"net_l1_mean": float(err_net.mean()), "net_l1_median": float(err_net.median()),
           "net_l1_mean_vs_m2048": float(l1(q, p2048).mean()),
           "pred_err_mean": float(e.mean()),
           "pred_err_corr": float(np.corrcoef(e.double().cpu().numpy(), err_net.cpu().numpy())[0, 1])}
    for M in M_CHOICES:
        out[f"kpm_l1_mean_M{M}"] = float(l1(masses(mu, M), p).mean())
        if M < 2048:
            out[f"kpm_l1_mean_M{M}_vs_m2048"] = float(l1(masses(mu, M), p2048).mean())
    out["net_gain_vs_kpm_M512"] = out["kpm_l1_mean_M512"] / out["net_l1_mean"]
    for eps_s, fb_rec in (fallback or {}).items():
        eps, M, tau = float(eps_s), fb_rec["M"], fb_rec["tau"]
        fb = e > tau
        err_kpm = l1(masses(mu, M), p)
        err = torch.where(fb, err_kpm, err_net)
        out[f"eps{eps_s}"] = {"M": M, "tau": tau, "fallback_fraction": float(fb.double().mean()),
                              "mean_l1": float(err.mean()), "over_eps_fraction": float((err > eps).double().mean()),
                              "kpm_over_eps_fraction": float((err_kpm > eps).double().mean()),
                              "accepted_l1_max": float(torch.where(fb, torch.zeros_like(err_net), err_net).max())}
    return out


if __name__ == "__main__":
    main()
