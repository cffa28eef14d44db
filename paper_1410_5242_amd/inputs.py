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


_HERM_STREAM = 0x5EED_0004


def random_hermitian_csr(N: int, mean_offdiag: float = 12.0, tail: float = 1.5, max_couplings: int = 256,
                         local_frac: float = 0.5, band: int = 64, empty_frac: float = 0.02, seed: int = 0):
    """Seeded sparse Hermitian matrix with an irregular row-length mix, as host CRS.

    Returns (rowptr int64 [N+1], col int32 [nnz], val complex128 [nnz]), columns sorted per row.
    A fraction `empty_frac` of the rows is empty (no diagonal, no couplings).  Every other row i
    proposes k_i couplings, k_i = round(mean_offdiag / 2 * (1 + X) * (tail - 1) / tail) with X drawn
    from a Lomax law of index `tail` (a power-law tail, mean k_i about mean_offdiag / 2), capped
    at `max_couplings`; a share `local_frac` of the partners lies within `band` rows of i
    (periodically), the rest is uniform over the non-empty rows.  A coupling (i, j) adds h to
    (i, j) and conj(h) to (j, i), h = (g + i g') / 2 with g, g' standard normal, so the mean row
    holds about mean_offdiag off-diagonal entries; repeated pairs add up (in the upper triangle,
    which is then mirrored, so the result is Hermitian exactly).  The diagonal of a non-empty row
    is real, standard normal.
    """
    import scipy.sparse as sp

    N = int(N)
    rng = np.random.default_rng([int(seed), _HERM_STREAM])
    empty = rng.random(N) < empty_frac
    live = np.flatnonzero(~empty)
    if live.size == 0:
        return np.zeros(N + 1, dtype=np.int64), np.zeros(0, dtype=np.int32), np.zeros(0, dtype=np.complex128)
    x = rng.pareto(tail, size=live.size)
    k = np.rint(0.5 * mean_offdiag * (1.0 + x) * (tail - 1.0) / tail).astype(np.int64)
    k = np.minimum(k, min(max_couplings, max(live.size - 1, 0)))
    src = np.repeat(live, k)
    near = rng.random(src.size) < local_frac
    off = rng.integers(-band, band + 1, size=src.size)
    dst = np.where(near, (src + off) % N, live[rng.integers(0, live.size, size=src.size)])
    keep = (dst != src) & ~empty[dst]
    src, dst = src[keep], dst[keep]
    h = 0.5 * (rng.standard_normal(src.size) + 1j * rng.standard_normal(src.size))
    d = rng.standard_normal(live.size)
    # the strict upper triangle (repeated pairs summed once), mirrored, so
    # that the matrix is Hermitian exactly
    lo, hi = np.minimum(src, dst), np.maximum(src, dst)
    h = np.where(src < dst, h, np.conj(h))
    U = sp.coo_matrix((h, (lo, hi)), shape=(N, N)).tocsr()
    U.sum_duplicates()
    D = sp.coo_matrix((d.astype(np.complex128), (live, live)), shape=(N, N)).tocsr()
    A = (U + U.conj().T.tocsr() + D).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.complex128)
