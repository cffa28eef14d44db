"""Seeded synthetic inputs for the KPM path: site potentials and start blocks.

This module is shared by the tests, the benchmark and (through them) both the
GPU library and the CPU oracle.  It holds none of the method's arithmetic:
it only draws the random numbers the method consumes (the disorder potential
V_n of the Hamiltonian and the random-phase start vectors of the stochastic
trace) and lays them out, so that both sides receive identical inputs.

Random numbers come from NumPy's PCG64 generator keyed by (seed, stream).
"""
from __future__ import annotations

import numpy as np

_POT_STREAM = 0x5EED_0001
_PHASE_STREAM = 0x5EED_0002


def potential(L, gamma: float, seed: int) -> np.ndarray:
    """Disorder V_n ~ U[-gamma/2, gamma/2] for the Lx*Ly*Lz sites (x fastest), float64."""
    Lx, Ly, Lz = (int(v) for v in L)
    rng = np.random.default_rng([int(seed), _POT_STREAM])
    return rng.uniform(-0.5 * gamma, 0.5 * gamma, size=Lx * Ly * Lz)


def quantum_dot_potential(L, period: int = 25, radius: float = 6.0, v_dot: float = 1.0, depth: int = 4,
                          gamma: float = 0.2, seed: int = 0) -> np.ndarray:
    """Potential of a quantum-dot superlattice on a slab (x fastest), float64.

    Cylindrical dots of radius `radius` (sites) on a square superlattice of
    period `period` in the x-y plane, centred in each cell, reaching `depth`
    layers down from the top surface z = Lz - 1, raise the potential by v_dot;
    on top of that the uniform disorder U[-gamma/2, gamma/2] of `potential`.
    """
    Lx, Ly, Lz = (int(v) for v in L)
    n = np.arange(Lx * Ly * Lz)
    x, y, z = n % Lx, (n // Lx) % Ly, n // (Lx * Ly)
    dx = (x % period) - 0.5 * (period - 1)
    dy = (y % period) - 0.5 * (period - 1)
    dot = (dx * dx + dy * dy <= radius * radius) & (z >= Lz - depth)
    return potential(L, gamma, seed) + v_dot * dot.astype(np.float64)


def phase_block(N: int, R: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """[N][R] block of random-phase unit vectors v_ir = exp(2 pi i u_ir) / sqrt(N).

    Row-major, so column r is the r-th start vector and element (i, r) sits at
    i*R + r.  The phases are drawn in double precision; a complex64 block is the
    rounded complex128 block.
    """
    rng = np.random.default_rng([int(seed), _PHASE_STREAM])
    out = np.empty((N, R), dtype=np.complex128)
    chunk = 1 << 22
    flat = out.reshape(-1)
    scale = 1.0 / np.sqrt(float(N))
    for s in range(0, N * R, chunk):
        e = min(N * R, s + chunk)
        u = rng.random(e - s)
        ph = 2.0 * np.pi * u
        flat[s:e].real = np.cos(ph) * scale
        flat[s:e].imag = np.sin(ph) * scale
    return out.astype(dtype, copy=False)


def lattice_sites(L) -> int:
    Lx, Ly, Lz = (int(v) for v in L)
    return Lx * Ly * Lz


_BATCH_STREAM = 0x5EED_0003


def instance_family(n: int, sides, gamma_max: float, seed: int):
    """Recipe of a batch of independent disorder realisations.

    Instance i gets a cubic side L_i drawn uniformly from `sides`, a disorder
    strength gamma_i ~ U[0, gamma_max], and its own potential and start-block
    seeds.  Returns a list of dicts (L, gamma, pot_seed, vec_seed).
    """
    rng = np.random.default_rng([int(seed), _BATCH_STREAM])
    sides = np.asarray(list(sides), dtype=np.int64)
    Ls = rng.choice(sides, size=n)
    gammas = rng.uniform(0.0, gamma_max, size=n)
    return [dict(L=(int(L), int(L), int(L)), gamma=float(g), pot_seed=int(seed) * 1_000_003 + i,
                 vec_seed=int(seed) * 1_000_003 + n + i) for i, (L, g) in enumerate(zip(Ls, gammas))]
