"""Local and momentum-resolved spectra on the fused sweep (Fig. "topi_demo").

The local DOS of a site and the spectral function A(k, E) use the same
Chebyshev iteration as the DOS, with deterministic start vectors and no
trace average: the moments of a start vector |phi> are
<phi|T_n(Htilde)|phi>.  Per site (per momentum) the four orbitals are four
columns of one block, so up to 16 sites (momenta) share one blocked run at
R = 64; the reconstruction averages the four orbitals (each curve
integrates to 1).  Every step runs in the library's kernels: start block,
moments, batched Jackson reconstruction.
"""
from __future__ import annotations

import torch

from . import kpm as K

GROUP = 16   # sites or momenta per blocked run (4 orbitals each: R <= 64)


def _group_size(n: int) -> int:
    """Smallest group size >= n among 1, 2, 4, 8, 16 (R = 4 x that is a supported block width)."""
    g = 1
    while g < n:
        g *= 2
    return g


def _run(H: K.Hamiltonian, blocks, M: int, E: torch.Tensor, kernel: str):
    """blocks: list of (start block [N][4g], used columns groups u); returns mu [n][4][M], rho [n][K]."""
    mus, rhos = [], []
    for V0, used in blocks:
        mu = K.moments(H, V0, M)
        g = V0.shape[1] // 4
        a = torch.full((g,), H.a, dtype=torch.float64, device=E.device)
        b = torch.full((g,), H.b, dtype=torch.float64, device=E.device)
        mu3 = mu.view(g, 4, M)
        rho = K.dos_batched(mu3, a, b, E, kernel=kernel)
        mus.append(mu3[:used])
        rhos.append(rho[:used])
    return torch.cat(mus), torch.cat(rhos)


def local_dos(H: K.Hamiltonian, L, sites, M: int, E: torch.Tensor, kernel: str = "jackson"):
    """Local DOS of the given sites (site n = x + Lx (y + Ly z)) on the device energy grid E.

    Returns (mu [n][4][M], rho [n][K]); rho is the orbital average (integral 1).
    """
    sites = [int(s) for s in sites]
    nsites = int(L[0]) * int(L[1]) * int(L[2])
    if 4 * nsites != H.N or any(not 0 <= s < nsites for s in sites):
        raise ValueError("L must be H's lattice and every site inside it")
    blocks = []
    for i in range(0, len(sites), GROUP):
        chunk = sites[i:i + GROUP]
        g = _group_size(len(chunk))
        padded = chunk + [chunk[-1]] * (g - len(chunk))
        rows = [4 * s + o for s in padded for o in range(4)]
        blocks.append((K.site_block(H.N, rows, _dtype_name(H)), len(chunk)))
    return _run(H, blocks, M, E, kernel)


def spectral_function(H: K.Hamiltonian, L, momenta, M: int, E: torch.Tensor, kernel: str = "jackson"):
    """A(k, E) for the given momenta (radians per lattice spacing, [n][3]) on the energy grid E.

    Returns (mu [n][4][M], rho [n][K]); rho is the orbital average (integral 1).
    """
    ks = [tuple(float(c) for c in k) for k in momenta]
    blocks = []
    for i in range(0, len(ks), GROUP):
        chunk = ks[i:i + GROUP]
        g = _group_size(len(chunk))
        padded = chunk + [chunk[-1]] * (g - len(chunk))
        kk = [k for k in padded for _ in range(4)]
        orbs = [o for _ in padded for o in range(4)]
        blocks.append((K.plane_wave_block(L, kk, orbs, _dtype_name(H)), len(chunk)))
    return _run(H, blocks, M, E, kernel)


def _dtype_name(H: K.Hamiltonian) -> str:
    return "c128" if H.dtype == 0 else "c64"
