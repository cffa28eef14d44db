"""Write the oracle's Chebyshev moments for the full-size workloads to tests/golden/.

The GPU tests compare the library with these files element by element at
sizes whose oracle run takes minutes (too long to repeat inside a test):

* ti64_r32_m2000_c128_mu.npy -- the 64 x 64 x 64 periodic topological-insulator
  lattice (N = 1,048,576), disorder gamma = 1 (potential seed 0), R = 32
  random-phase start vectors (phase seed 0), M = 2000 moments: the whole
  benchmark workload, every moment (eq. "eq:kpm_iter", Alg.
  "kpm_improved_blocked").
* ti128x128x64_g2_r32_m400_mu.npy -- the 128 x 128 x 64 lattice (N = 4,194,304),
  gamma = 2 (potential seed 0), R = 32 start vectors from the counter-based
  SplitMix64 generator (seed 0, the block the device generator draws), the
  first 400 moments of the M = 2000 precision workload (200 of its 1000 sweeps).

Only the oracle (plain C, FP64, pairwise scalar products) and the seeded input
generators are called; nothing here touches the GPU library.  Each file is a
float64 array [R][M] (numpy .npy, no pickles); a JSON file of the same stem
records the recipe.  Run from the repository root:

    python tests/golden/make_oracle_moments.py [name ...]
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1410_5242_amd import inputs  # noqa: E402

CASES = {
    "ti64_r32_m2000_c128": dict(L=(64, 64, 64), gamma=1.0, pot_seed=0, R=32, M=2000,
                                start="inputs.phase_block(N, R, seed=0)", phase_seed=0),
    "ti128x128x64_g2_r32_m400": dict(L=(128, 128, 64), gamma=2.0, pot_seed=0, R=32, M=400,
                                     start="oracle.phase_block_counter(N, R, seed=0)", phase_seed=0),
}


def path(name: str) -> str:
    return os.path.join(HERE, name + "_mu.npy")


def make(name: str) -> None:
    c = CASES[name]
    t0 = time.perf_counter()
    pot = inputs.potential(c["L"], c["gamma"], c["pot_seed"])
    H = O.ti_hamiltonian(c["L"], pot)
    a, b = O.scaling(*O.gershgorin(H))
    if c["start"].startswith("inputs"):
        v0 = inputs.phase_block(H.n, c["R"], c["phase_seed"])
    else:
        v0 = O.phase_block_counter(H.n, c["R"], c["phase_seed"])
    print(f"{name}: N={H.n} a={a!r} b={b!r}; {c['M'] // 2} sweeps on {O.lib_threads()} threads", flush=True)
    mu = O.kpm_moments(H, a, b, v0, c["M"])
    np.save(path(name), mu, allow_pickle=False)
    rec = dict(c, name=name, N=H.n, a=a, b=b, shape=list(mu.shape), dtype="float64",
               produced_by="tests/golden/make_oracle_moments.py (oracle only)",
               seconds=round(time.perf_counter() - t0, 1))
    rec["L"] = list(c["L"])
    with open(os.path.join(HERE, name + "_mu.json"), "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(f"{name}: wrote {path(name)} in {rec['seconds']} s", flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(CASES)):
        make(n)
