"""Adaptive block preconditioning (oracle; test infrastructure only).

Two indicators decide, per system, how much of a block preconditioner is
needed:

  Definition 1 (weak coupling factor).  For a coupling block D_ab (a != b)
  relative to the diagonal block A_a of its row:
      gamma_wc^{ab}(theta_wc) = |{k : -d_kk^{ab} <= theta_wc a_kk^{(a)}}| / N.
  Section 3.5: a coupling with gamma_wc > sigma_wc is neglected in the
  preconditioning matrix (theta_wc = 1e-2, sigma_wc = 0.5 in the paper).

  Definition 2 (weak diagonal dominance factor).  For a matrix A:
      gamma_wd(theta_wd) = |{k : sum_j a_kj < theta_wd a_kk}| / N.
  Section 3.4: an inverse whose matrix has gamma_wd = 0 is approximated by a
  fixed number of Jacobi iterations (option #1), otherwise by V-cycles
  (option #2); theta_wd = 0.9.

Readings (where the paper leaves the details open):
  * Each coupling block of eq. 2.2 (D_gE, D_Eg for every g, D_EI, D_IE) is
    evaluated on its own; the neglected ones are set to zero and the chosen
    preconditioner (PCTL, Schur1, Schur2) is formed from the modified matrix,
    hats included (a hat update whose product involves a neglected coupling
    leaves the block unchanged).
  * A row block whose coupling to E is neglected no longer depends on E: it is
    solved independently first and enters E's equation through the couplings
    still kept (block Gauss-Seidel).  When every row block's coupling to E is
    neglected, the two E-inverses of Schur2 (steps 1 and 3) and of Schur1
    (its second and fourth steps) are one inverse applied after the
    independent solves; by linearity of the inverse approximations this is the
    same operator.  When every coupling into E's row is neglected, the
    correction step that uses them is skipped, and PCTL skips its coarse-grid
    correction (the Remark after Definition 1).
  * Row sums for Definition 2 are added left to right in ascending column
    order; a row counts as weakly dominant when that sum is below theta_wd
    times its diagonal, both in FP64.  A factor is compared with sigma_wc as
    count > sigma_wc * N in FP64.
  * Option #1 uses `jacobi_sweeps` Jacobi iterations (default 2) from the
    zero vector with the plain diagonal:  w <- w + diag(M)^{-1} (b - M w).
  * PCTL's interpolation weights stay on option #3 (V-cycles to tolerance),
    which the paper prescribes for them.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict

import numpy as np
import scipy.sparse as sp

from . import amg
from .assemble import BlockSystem


def weak_coupling_count(d: np.ndarray, a_diag: np.ndarray, theta_wc: float) -> int:
    """Definition 1 numerator: rows k with -d_kk <= theta_wc a_kk."""
    return int(np.count_nonzero(-d <= theta_wc * a_diag))


def weak_dominance_count(A: sp.csr_matrix, theta_wd: float) -> int:
    """Definition 2 numerator: rows k with sum_j a_kj < theta_wd a_kk."""
    lens = np.diff(A.indptr)
    rs = amg.seq_segment_sum(A.indptr[:-1].astype(np.int64), lens, A.data)
    return int(np.count_nonzero(rs < theta_wd * amg.diagonal_of(A)))


def is_weak(count: int, N: int, sigma_wc: float) -> bool:
    return float(count) > sigma_wc * float(N)


@dataclass
class CouplingPlan:
    """Which coupling blocks are neglected, with their Definition 1 counts."""
    gE: np.ndarray       # (G,) bool: D_gE neglected
    Eg: np.ndarray       # (G,) bool: D_Eg neglected
    EI: bool
    IE: bool
    counts: Dict[str, np.ndarray]

    @property
    def all_into_E_rows_weak(self) -> bool:
        """Every coupling in E's row (D_Eg for all g, D_EI) is neglected."""
        return bool(np.all(self.Eg)) and self.EI

    @property
    def all_from_E_weak(self) -> bool:
        """Every row block's coupling to E (D_gE for all g, D_IE) is neglected."""
        return bool(np.all(self.gE)) and self.IE


def coupling_plan(sys: BlockSystem, theta_wc: float = 1e-2,
                  sigma_wc: float = 0.5) -> CouplingPlan:
    """Definition 1 for every coupling block of eq. 2.2, each relative to the
    diagonal block of its own row."""
    G, N = sys.G, sys.N
    dg = [amg.diagonal_of(B) for B in sys.blocks]
    c_gE = np.array([weak_coupling_count(sys.d_gE[g], dg[g], theta_wc) for g in range(G)])
    c_Eg = np.array([weak_coupling_count(sys.d_Eg[g], dg[G], theta_wc) for g in range(G)])
    c_EI = weak_coupling_count(sys.d_EI, dg[G], theta_wc)
    c_IE = weak_coupling_count(sys.d_IE, dg[G + 1], theta_wc)
    return CouplingPlan(
        gE=np.array([is_weak(int(c), N, sigma_wc) for c in c_gE], dtype=bool),
        Eg=np.array([is_weak(int(c), N, sigma_wc) for c in c_Eg], dtype=bool),
        EI=is_weak(c_EI, N, sigma_wc), IE=is_weak(c_IE, N, sigma_wc),
        counts={"gE": c_gE, "Eg": c_Eg, "EI": np.array([c_EI]), "IE": np.array([c_IE])})


def drop_weak(sys: BlockSystem, plan: CouplingPlan) -> BlockSystem:
    """The preconditioning matrix: eq. 2.2 with the neglected couplings zeroed."""
    d_gE = sys.d_gE.copy()
    d_Eg = sys.d_Eg.copy()
    d_gE[plan.gE] = 0.0
    d_Eg[plan.Eg] = 0.0
    d_EI = np.zeros_like(sys.d_EI) if plan.EI else sys.d_EI.copy()
    d_IE = np.zeros_like(sys.d_IE) if plan.IE else sys.d_IE.copy()
    return BlockSystem(sys.G, sys.N, list(sys.blocks), d_gE, d_Eg, d_EI, d_IE)


def jacobi(M: sp.csr_matrix, b: np.ndarray, sweeps: int) -> np.ndarray:
    """Option #1: `sweeps` Jacobi iterations from the zero vector."""
    d = amg.diagonal_of(M)
    w = np.zeros_like(b)
    for _ in range(sweeps):
        w = w + (b - M @ w) / d
    return w
