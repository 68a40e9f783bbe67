"""Seeded synthetic inputs for the multi-group radiation-diffusion block system.

This module only DRAWS numbers: per-cell diffusion coefficients, per-cell
coupling coefficients, right-hand sides and loss targets.  It performs none of
the method's arithmetic (no face averaging, no matrix assembly, no solver
step), so both the CPU oracle and the GPU path can consume the same arrays
while sharing no solver code.

Structure follows the paper's block system (Section 2, eq. 2.2): G radiation
groups plus the electron (E) and ion (I) temperatures, each a cell-centred
scalar field on the same mesh, with diagonal couplings group<->E and E<->I.
The paper's own capsule-implosion matrices are not available, so these
synthetic fields stand in for them (sizes and coefficient ranges are the
workload definitions below).

Draw order (fixed, numpy PCG64 from ``default_rng(seed)``):
  1. u_R ~ U(-3, 3) over the 8^d patch grid (radiation base log10 kappa)
  2. u_s ~ U(-2, 2), one per group, only when G > 1 (per-group log10 scale)
  3. u_E, u_I ~ U(-3, 3) over the patch grid
  4. c_gE, c_Eg ~ U(0.1, 10) of shape (G, N); c_EI ~ U(0.1, 10) of shape (N,)
  5. b ~ U(0, 1) of length (G+2) N
  6. x_target ~ U(0, 1) of length (G+2) N
  7. (only if ``nonsym``) xi ~ U(0, 1) of shape (G+2, N, 2d): one factor per
     directed face, used by the nonsymmetric test variant.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = ["Workload", "WORKLOADS", "Inputs", "generate", "workload"]


@dataclass(frozen=True)
class Workload:
    """A synthetic problem shape: G groups on an n^dim cell mesh."""
    name: str
    G: int
    dim: int
    n: int           # cells per direction
    seed: int

    @property
    def N(self) -> int:
        return self.n ** self.dim

    @property
    def n_unknowns(self) -> int:
        return (self.G + 2) * self.N


# Named by what they are: groups, dimension, cells per direction.
WORKLOADS = {
    "g1_2d64": Workload("g1_2d64", G=1, dim=2, n=64, seed=1),
    "g1_2d1024": Workload("g1_2d1024", G=1, dim=2, n=1024, seed=2),
    "g20_2d256": Workload("g20_2d256", G=20, dim=2, n=256, seed=3),
    "g20_3d64": Workload("g20_3d64", G=20, dim=3, n=64, seed=4),
    "g20_2d512": Workload("g20_2d512", G=20, dim=2, n=512, seed=5),
    "g2_2d16": Workload("g2_2d16", G=2, dim=2, n=16, seed=6),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


@dataclass
class Inputs:
    """Raw per-cell fields.  Cell index is x-fastest: c = i + n*j (+ n*n*l)."""
    G: int
    dim: int
    n: int
    kappa: np.ndarray           # (G+2, N) float64, order [groups..., E, I]
    c_gE: np.ndarray            # (G, N)   coupling magnitude in row g, column E
    c_Eg: np.ndarray            # (G, N)   coupling magnitude in row E, column g
    c_EI: np.ndarray            # (N,)     E<->I exchange magnitude (symmetric)
    b: np.ndarray               # ((G+2) N,)
    x_target: np.ndarray        # ((G+2) N,)
    mass: float = 1.0
    xi: Optional[np.ndarray] = None   # (G+2, N, 2*dim) or None
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.n ** self.dim


def _patch_index(n: int, dim: int) -> np.ndarray:
    """Patch id (8^d patch grid) of every cell, x-fastest cell order."""
    p1 = (8 * np.arange(n)) // n
    if dim == 2:
        pj, pi = np.meshgrid(p1, p1, indexing="ij")
        return (pi + 8 * pj).reshape(-1)
    pl, pj, pi = np.meshgrid(p1, p1, p1, indexing="ij")
    return (pi + 8 * pj + 64 * pl).reshape(-1)


def generate(G: int, dim: int, n: int, seed: int, *, nonsym: bool = False,
             zero_row_sum: bool = False, c_scale=(1.0, 1.0, 1.0),
             log_kappa_shift=(0.0, 0.0, 0.0)) -> Inputs:
    """Draw one synthetic instance.

    ``zero_row_sum`` keeps the draws but sets the mass term and all couplings
    to zero (the zero-flux Laplacian test variant).

    ``c_scale`` = (s_gE, s_Eg, s_EI) multiplies the drawn coupling magnitudes
    after all draws (s_gE and s_Eg may be per-group arrays of length G), and
    ``log_kappa_shift`` = (radiation, E, I) is added to the drawn log10 kappa
    exponents: the weakly coupled and strongly diagonally dominant test
    variants.  The draws themselves are unchanged.
    """
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    if G < 1 or n < 1:
        raise ValueError("G and n must be positive")
    rng = np.random.default_rng(seed)
    npatch = 8 ** dim
    N = n ** dim
    u_R = rng.uniform(-3.0, 3.0, size=npatch)
    u_s = rng.uniform(-2.0, 2.0, size=G) if G > 1 else np.zeros(1)
    u_E = rng.uniform(-3.0, 3.0, size=npatch)
    u_I = rng.uniform(-3.0, 3.0, size=npatch)
    c_gE = rng.uniform(0.1, 10.0, size=(G, N))
    c_Eg = rng.uniform(0.1, 10.0, size=(G, N))
    c_EI = rng.uniform(0.1, 10.0, size=N)
    b = rng.uniform(0.0, 1.0, size=(G + 2) * N)
    x_target = rng.uniform(0.0, 1.0, size=(G + 2) * N)
    xi = rng.uniform(0.0, 1.0, size=(G + 2, N, 2 * dim)) if nonsym else None

    sgE, sEg, sEI = c_scale
    c_gE = c_gE * np.reshape(np.asarray(sgE, dtype=np.float64), (-1, 1))
    c_Eg = c_Eg * np.reshape(np.asarray(sEg, dtype=np.float64), (-1, 1))
    c_EI = c_EI * float(sEI)
    kR, kE, kI = log_kappa_shift
    patch = _patch_index(n, dim)
    kappa = np.empty((G + 2, N))
    for g in range(G):
        kappa[g] = 10.0 ** (u_R[patch] + u_s[g] + kR)
    kappa[G] = 10.0 ** (u_E[patch] + kE)
    kappa[G + 1] = 10.0 ** (u_I[patch] + kI)
    mass = 1.0
    if zero_row_sum:
        c_gE[:] = 0.0
        c_Eg[:] = 0.0
        c_EI[:] = 0.0
        mass = 0.0
    return Inputs(G=G, dim=dim, n=n, kappa=kappa, c_gE=c_gE, c_Eg=c_Eg,
                  c_EI=c_EI, b=b, x_target=x_target, mass=mass, xi=xi,
                  seed=seed)


def generate_workload(name: str, **kw) -> Inputs:
    w = WORKLOADS[name]
    return generate(w.G, w.dim, w.n, w.seed, **kw)
