"""Autotuner for the launch shapes of the KPM kernels, with a JSON cache.

The paper generates fully unrolled kernels per (C, R) and picks the best
configuration for the hardware at hand (section "Performance Engineering",
SELL-C-sigma and the block-vector width).  Here the kernels are compiled
once for every supported block width, and what is left to choose at run
time is their launch shape and the block width itself:

* the fused sweep (``kpm_set_sweep_tuning``): grid size, die-aware tile
  ranges, chunking, site order, non-temporal streams, and whether the
  cache-blocked lattice kernel or the generic gather kernel runs;
* the batched persistent solver (``kpm_set_batch_tuning``): workgroup size,
  workgroups per CU, dynamic or static instance mapping;
* the block width R for a given number of random vectors S (S/R passes of
  kpm_moments at width R; the matrix is read once per pass and sweep);
* for a general matrix handed over as CRS (``kpm_import_csr``), its
  SELL-C-sigma layout: the chunk height C and the sorting window sigma,
  which trade padding against how the entries of a pass are laid out.

Candidates are timed on the caller's problem with HIP events around the
library calls; every candidate produces the same moments up to the order of
floating-point sums, so the choice never changes results beyond rounding.
Winners are cached per (kernel, dtype, R, size bucket) in a JSON file and
re-applied without timing on later runs.  Only host logic lives here.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time
from dataclasses import dataclass, field

DEFAULT_CACHE = os.environ.get(
    "KPM_TUNING_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "mi355x.json"))

DTYPE_NAMES = {0: "c128", 1: "c64"}

SWEEP_FIELDS = ("wg_per_cu", "xcd_ways", "chunk_tiles", "pencil", "dynamic", "prefetch", "stream", "lattice",
                "gather", "tile_order", "slab", "gather_tile")
BATCH_FIELDS = ("waves", "wg_per_cu", "dynamic", "slab")


def size_bucket(n: int) -> int:
    """Rows rounded down to a power of two: problems within a factor of two share a tuning."""
    return 1 << max(0, int(n).bit_length() - 1)


def sweep_key(dtype: int, R: int, N: int, L=None) -> str:
    lat = "x".join(str(int(v)) for v in L) if L is not None else "-"
    return f"sweep:{DTYPE_NAMES[dtype]}:R{R}:N{size_bucket(N)}:L{lat}"


def batch_key(dtype: int, R: int, n_inst: int, total_rows: int) -> str:
    return f"batched:{DTYPE_NAMES[dtype]}:R{R}:n{size_bucket(n_inst)}:N{size_bucket(total_rows)}"


def width_key(dtype: int, S: int, N: int) -> str:
    return f"width:{DTYPE_NAMES[dtype]}:S{S}:N{size_bucket(N)}"


def sell_key(dtype: int, R: int, N: int, nnz: int) -> str:
    return f"sell:{DTYPE_NAMES[dtype]}:R{R}:N{size_bucket(N)}:nnz{size_bucket(nnz)}"


def sell_candidates() -> list[dict]:
    """SELL-C-sigma layouts to time: the library default first, then chunk heights from CRS
    (C = 1) to one chunk per wave of single-row passes (C = 64), unsorted and sorted."""
    out = [{"C": 8, "sigma": 1024}]
    for C in (1, 2, 4, 8, 16, 32, 64):
        for sigma in (1, 32 * C, 1024 * C):
            if sigma == 1 and C > 1 and C != 32:
                continue
            c = {"C": C, "sigma": sigma}
            if c not in out:
                out.append(c)
    return out


def sweep_candidates(R: int, lattice_ok: bool) -> list[dict]:
    """Launch shapes of the fused sweep worth timing at block width R."""
    base = dict(wg_per_cu=0, xcd_ways=8, chunk_tiles=8, pencil=16, dynamic=0, prefetch=2, stream=3, lattice=0,
                gather=1, tile_order=0, slab=4, gather_tile=0)
    out = []
    # staged-gather sweep: workgroups per CU and die-aware ranges (from R = 16 on,
    # gather 1 runs its window variant on large lattices; gather 4 keeps the
    # plain staged gather, alone or in pencil order)
    for g in ((1, 4) if R >= 16 else (1,)):
        for wg in (0, 1, 2, 4):
            for xcd in (8, 1):
                for slab in (0, 2, 4, 8):
                    out.append(dict(base, gather=g, wg_per_cu=wg, xcd_ways=xcd, slab=slab))
    if R >= 16:
        for wg in (1, 2):
            out.append(dict(base, gather=4, wg_per_cu=wg, gather_tile=4))
        # window variant: tiles dealt to the dies in blocks or not, streams
        # cached or not (blocks with non-temporal streams is the base above)
        for order, stream in ((2, 3), (0, 0), (2, 0)):
            out.append(dict(base, gather=1, tile_order=order, stream=stream))
    # scalar-operand sweep
    for wg in (4, 8):
        for chunk in (4, 8, 16):
            for pencil in (0, 16):
                for stream in (0, 3):
                    out.append(dict(base, gather=2, prefetch=0, wg_per_cu=wg, chunk_tiles=chunk, pencil=pencil,
                                    stream=stream))
    if lattice_ok:
        # wider blocks always take the record path (prefetch 2)
        for prefetch in ((2, 1) if R == 32 else (2,)):
            for stream in (3, 0):
                for order in (0, 1, 2):
                    for wg in (0, 2):
                        out.append(dict(base, lattice=2, prefetch=prefetch, stream=stream, tile_order=order,
                                        wg_per_cu=wg))
    return out


def batch_candidates(max_waves: int = 16) -> list[dict]:
    out = []
    for waves in (4, 8, 16):
        if waves > max_waves:
            continue
        for per_cu in (1, 2, 4):
            if waves * per_cu > 32:
                continue
            for dyn in (1, 0):
                for slab in (0, 2, 4, 8):
                    out.append(dict(waves=waves, wg_per_cu=per_cu, dynamic=dyn, slab=slab))
    return out


def block_widths(S: int, supported=(1, 2, 4, 8, 16, 32, 64)) -> list[int]:
    """Block widths R that split S random vectors into whole passes."""
    return [R for R in supported if R <= S and S % R == 0]


@dataclass
class Trial:
    params: dict
    seconds: float


@dataclass
class TuneResult:
    key: str
    best: dict
    seconds: float
    trials: list = field(default_factory=list)

    def to_json(self) -> dict:
        return {"best": self.best, "seconds": self.seconds,
                "trials": [{"params": t.params, "seconds": t.seconds} for t in self.trials]}


def pick_best(trials: list[Trial], margin: float = 0.0) -> Trial:
    """Fastest trial; ties go to the earlier candidate.  The first trial (the library default) is kept
    unless the fastest beats it by more than `margin` (relative), so timing noise does not move the
    launch shape away from the default."""
    if not trials:
        raise ValueError("no trials")
    best = trials[0]
    for t in trials[1:]:
        if t.seconds < best.seconds:
            best = t
    if best is not trials[0] and best.seconds > trials[0].seconds * (1.0 - margin):
        return trials[0]
    return best


class TuningCache:
    """JSON file of tuned launch shapes, keyed by sweep_key / batch_key / width_key."""

    def __init__(self, path: str = DEFAULT_CACHE):
        self.path = path
        self.entries: dict = {}
        if os.path.exists(path):
            with open(path) as f:
                data = json.load(f)
            self.entries = data.get("entries", {})

    def get(self, key: str):
        e = self.entries.get(key)
        return None if e is None else e["best"]

    def put(self, result: TuneResult):
        self.entries[result.key] = result.to_json()

    def save(self):
        os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump({"format": 1, "entries": self.entries}, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def time_call(fn, repeats: int = 3, sync=None) -> float:
    """Best wall time of `repeats` calls of fn() (after one warm-up), with `sync` after each."""
    fn()
    if sync:
        sync()
    best = math.inf
    for _ in range(repeats):
        t0 = time.perf_counter()
        fn()
        if sync:
            sync()
        best = min(best, time.perf_counter() - t0)
    return best


# --------------------------------------------------------------------------
# GPU-side tuning (needs the library and a device)
# --------------------------------------------------------------------------
def _gpu_timer():
    import torch

    def timed(fn, repeats=3):
        fn()
        torch.cuda.synchronize()
        best = math.inf
        for _ in range(repeats):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) * 1e-3)
        return best
    return timed


def tune_sweep(H, R: int, cache: TuningCache | None = None, sweeps: int = 8, candidates=None,
               repeats: int = 3, L=None, margin: float = 0.02) -> TuneResult:
    """Time the fused sweep kernel of H at block width R under each candidate launch shape, with
    the library's HIP events around every sweep launch (kernel time only).  The first candidate is
    the library default, kept unless another shape is faster by more than `margin`."""
    import torch
    from . import kpm as K

    V = torch.zeros((H.N, R), dtype=H.torch_dtype, device="cuda")
    W = torch.zeros_like(V)
    V[:, :] = 1.0 / math.sqrt(H.N)
    eta = torch.zeros((2, R, 2), dtype=torch.float64, device="cuda")
    saved = K.get_sweep_tuning()
    trials = []
    try:
        if candidates is None:
            K.reset_sweep_tuning()
            default = K.get_sweep_tuning()
            K.set_sweep_tuning(lattice=2)
            candidates = [default] + sweep_candidates(R, K.sweep_kernel(H, R) == "lattice_kernel")
        for c in candidates:
            K.set_sweep_tuning(**c)
            K.aug_spmmv(H, V, W, 2.0 / H.a, -2.0 * H.b / H.a, -1.0, "full", eta)   # warm-up
            torch.cuda.synchronize()
            best = math.inf
            for _ in range(repeats):
                K.sweep_profile_read()
                K.sweep_profile_enable(True)
                for _ in range(sweeps):
                    K.aug_spmmv(H, V, W, 2.0 / H.a, -2.0 * H.b / H.a, -1.0, "full", eta)
                torch.cuda.synchronize()
                K.sweep_profile_enable(False)
                n, tot_ms, _, _ = K.sweep_profile_read()
                best = min(best, tot_ms * 1e-3 / max(n, 1))
            trials.append(Trial(dict(c), best))
    finally:
        K.sweep_profile_enable(False)
        K.set_sweep_tuning(**saved)
    best = pick_best(trials, margin)
    res = TuneResult(sweep_key(H.dtype, R, H.N, L), best.params, best.seconds, trials)
    if cache is not None:
        cache.put(res)
    return res


def tune_batched(Hs, V0s, M: int, cache: TuningCache | None = None, candidates=None,
                 repeats: int = 2, margin: float = 0.02) -> TuneResult:
    """Time kpm_moments_batched on the caller's batch under each candidate launch shape (the first
    candidate is the library default, kept unless another is faster by more than `margin`)."""
    import torch
    from . import kpm as K

    timed = _gpu_timer()
    R = V0s[0].shape[1]
    mu = torch.empty((len(Hs), R, M), dtype=torch.float64, device="cuda")
    saved = K.get_batch_tuning()
    if candidates is None:
        K.reset_batch_tuning()
        candidates = [K.get_batch_tuning()] + batch_candidates(8 if Hs[0].dtype == K.C128 else 16)
    trials = []
    try:
        for c in candidates:
            K.set_batch_tuning(**c)
            trials.append(Trial(dict(c), timed(lambda: K.moments_batched(Hs, V0s, M, mu=mu, check=False),
                                               repeats)))
    finally:
        K.set_batch_tuning(**saved)
    best = pick_best(trials, margin)
    res = TuneResult(batch_key(Hs[0].dtype, R, len(Hs), sum(H.N for H in Hs)), best.params, best.seconds,
                     trials)
    if cache is not None:
        cache.put(res)
    return res


def tune_block_width(H, S: int, cache: TuningCache | None = None, sweeps: int = 8,
                     repeats: int = 3) -> TuneResult:
    """Block width R minimising the time per random vector for S vectors (S/R passes)."""
    import torch
    from . import kpm as K

    timed = _gpu_timer()
    trials = []
    for R in block_widths(S):
        V = torch.zeros((H.N, R), dtype=H.torch_dtype, device="cuda")
        W = torch.zeros_like(V)
        eta = torch.zeros((2, R, 2), dtype=torch.float64, device="cuda")

        def run():
            for _ in range(sweeps):
                K.aug_spmmv(H, V, W, 2.0 / H.a, -2.0 * H.b / H.a, -1.0, "full", eta)
        per_sweep = timed(run, repeats) / sweeps
        trials.append(Trial({"R": R}, per_sweep * (S // R)))
        del V, W
    best = pick_best(trials)
    res = TuneResult(width_key(H.dtype, S, H.N), best.params, best.seconds, trials)
    if cache is not None:
        cache.put(res)
    return res


def tune_sell_layout(rowptr, col, val, R: int, dtype: str = "c128", cache: TuningCache | None = None,
                     sweeps: int = 8, candidates=None, repeats: int = 3, margin: float = 0.02) -> TuneResult:
    """Import the CRS matrix under each candidate SELL-C-sigma layout and time its fused sweep at
    block width R (the library's HIP events around every sweep).  The first candidate is the
    library default, kept unless another layout is faster by more than `margin`.  Returns the
    best {"C", "sigma"} (pass them to kpm.import_csr)."""
    import numpy as np
    import torch
    from . import kpm as K

    N = len(rowptr) - 1
    trials = []
    for c in candidates or sell_candidates():
        H = K.import_csr(rowptr, col, val, dtype=dtype, C=c["C"], sigma=c["sigma"])
        try:
            V = torch.full((N, R), 1.0 / math.sqrt(N), dtype=H.torch_dtype, device="cuda")
            W = torch.zeros_like(V)
            eta = torch.zeros((2, R, 2), dtype=torch.float64, device="cuda")
            K.aug_spmmv(H, V, W, 2.0 / H.a, -2.0 * H.b / H.a, -1.0, "full", eta)   # warm-up
            torch.cuda.synchronize()
            best = math.inf
            for _ in range(repeats):
                K.sweep_profile_read()
                K.sweep_profile_enable(True)
                for _ in range(sweeps):
                    K.aug_spmmv(H, V, W, 2.0 / H.a, -2.0 * H.b / H.a, -1.0, "full", eta)
                torch.cuda.synchronize()
                K.sweep_profile_enable(False)
                n, tot_ms, _, _ = K.sweep_profile_read()
                best = min(best, tot_ms * 1e-3 / max(n, 1))
            info = K.sell_info(H)
            trials.append(Trial({"C": c["C"], "sigma": c["sigma"], "stored": info["stored"]}, best))
            del V, W
        finally:
            K.sweep_profile_enable(False)
            H.close()
    best = pick_best(trials, margin)
    res = TuneResult(sell_key(K._DTYPES[dtype] if isinstance(dtype, str) else int(dtype), R, N,
                              int(np.asarray(rowptr)[-1])),
                     {"C": best.params["C"], "sigma": best.params["sigma"]}, best.seconds, trials)
    if cache is not None:
        cache.put(res)
    return res


def apply_sweep(cache: TuningCache, H, R: int, L=None) -> bool:
    """Set the cached sweep tuning for (H, R); False if the cache has none."""
    from . import kpm as K
    best = cache.get(sweep_key(H.dtype, R, H.N, L))
    if best is None:
        return False
    K.set_sweep_tuning(**{k: int(best[k]) for k in SWEEP_FIELDS if k in best})
    return True


def apply_batched(cache: TuningCache, Hs, R: int) -> bool:
    from . import kpm as K
    best = cache.get(batch_key(Hs[0].dtype, R, len(Hs), sum(H.N for H in Hs)))
    if best is None:
        return False
    K.set_batch_tuning(**{k: int(best[k]) for k in BATCH_FIELDS if k in best})
    return True


# --------------------------------------------------------------------------
# Command line: tune the benchmark workloads and write the cache
# --------------------------------------------------------------------------
HEADLINE_L = (64, 64, 64)
FAMILY = dict(n=512, sides=(12, 16, 20, 24), gamma_max=4.0, seed=0, R=8, M=512)
TTD_INSTANCES, TTD_M = 1000, 256   # time-to-DOS family (tuned at a mid-range number of moments)
SLABS = ((100, 100, 40), (200, 100, 40))   # the paper's slab domains (quantum dots, open z), R = 32
PRECISION_L, PRECISION_GAMMA = (128, 128, 64), 2.0   # the precision comparison, both dtypes, R = 32


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description="Tune launch shapes on the benchmark workloads (64^3 TI lattice "
                                             "at every block width; the 512-instance family) and write the cache")
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--parts", default="sweep,batched,ttd,slab,precision",
                    help="sweep, batched, ttd (the time-to-DOS family: 1,000 learned-family instances, R = 16, "
                         "complex64), slab (the quantum-dot slabs at R = 32, lattice-sweep shapes), precision "
                         "(128 x 128 x 64 in both dtypes at R = 32, lattice-sweep shapes), comma separated")
    ap.add_argument("--widths", default="1,2,4,8,16,32,64")
    args = ap.parse_args(argv)
    import numpy as np
    import torch
    from . import inputs
    from . import kpm as K

    cache = TuningCache(args.out)
    parts = set(args.parts.split(","))
    if "sweep" in parts:
        pot = inputs.potential(HEADLINE_L, 1.0, 0)
        H = K.build_hamiltonian(HEADLINE_L, pot, dtype="c128")
        for R in (int(r) for r in args.widths.split(",")):
            res = tune_sweep(H, R, cache, L=HEADLINE_L)
            print(f"[autotune] {res.key}: {res.seconds * 1e6:.1f} us/sweep with {res.best}", flush=True)
            cache.save()
        H.close()
    if "batched" in parts:
        f = FAMILY
        fam = inputs.instance_family(f["n"], f["sides"], f["gamma_max"], f["seed"])
        Hs = [K.build_hamiltonian(x["L"], inputs.potential(x["L"], x["gamma"], x["pot_seed"]), dtype="c64")
              for x in fam]
        V0s = [K.random_phase_block(H.N, f["R"], x["vec_seed"], "c64") for x, H in zip(fam, Hs)]
        torch.cuda.synchronize()
        res = tune_batched(Hs, V0s, f["M"], cache)
        print(f"[autotune] {res.key}: {res.seconds:.4f} s with {res.best}", flush=True)
        cache.save()
        for H in Hs:
            H.close()
        del np
    if "ttd" in parts:
        from . import learned as LN
        fam = LN.family(TTD_INSTANCES, LN.TEST_SEED + 7)
        Hs = LN.build(fam, "c64")
        V0s = LN.start_blocks(fam, Hs, LN.R_TRUTH, "c64")
        torch.cuda.synchronize()
        res = tune_batched(Hs, V0s, TTD_M, cache)
        print(f"[autotune] {res.key}: {res.seconds:.4f} s with {res.best}", flush=True)
        cache.save()
        for H in Hs:
            H.close()
    if "slab" in parts:
        for L in SLABS:
            H = K.build_hamiltonian(L, inputs.quantum_dot_potential(L), periodic=(1, 1, 0), dtype="c128")
            K.reset_sweep_tuning()
            default = K.get_sweep_tuning()
            cands = [default] + [c for c in sweep_candidates(32, True) if c["lattice"] == 2]
            res = tune_sweep(H, 32, cache, L=L, candidates=cands)
            print(f"[autotune] {res.key}: {res.seconds * 1e6:.1f} us/sweep with {res.best}", flush=True)
            cache.save()
            H.close()
    if "precision" in parts:
        L = PRECISION_L
        pot = inputs.potential(L, PRECISION_GAMMA, 0)
        for dt in ("c128", "c64"):
            H = K.build_hamiltonian(L, pot, dtype=dt)
            K.reset_sweep_tuning()
            default = K.get_sweep_tuning()
            cands = [default] + [c for c in sweep_candidates(32, True) if c["lattice"] == 2]
            res = tune_sweep(H, 32, cache, L=L, candidates=cands)
            print(f"[autotune] {res.key}: {res.seconds * 1e6:.1f} us/sweep with {res.best}", flush=True)
            cache.save()
            H.close()
    print(f"[autotune] wrote {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
