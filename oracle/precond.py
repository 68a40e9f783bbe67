"""Block preconditioners of Section 3 (oracle).

Each preconditioner acts as w = M^{-1} b on a Krylov vector b of length
(G+2) N ordered [groups..., E, I].  The scalar inverses inside are
"Inverse" objects; the paper's practical form uses a fixed number of AMG
V-cycles (option #2 of Section 3.4) on:

  monolithic   one hierarchy on the whole matrix (Section 3.1)
  bdiag        A_1..A_G, A_E, A_I (block-diagonal special case, Section 3.5)
  pctl         A_1..A_G, A_E, A_I for the block relaxation and A_c of eq. 3.1
               for the coarse correction (Section 3.2); the diagonal
               interpolation weights p_g = -A_g^{-1} D_gE 1, p_I = -A_I^{-1} D_IE 1
               are computed by V-cycles to a relative residual below
               pctl_p_tol (option #3)
  schur1       A_I, C^_E, C^_g (Section 3.3, five steps; Section 3.4 hats)
  schur2       A_E, S^_g, S^_I (Section 3.3, three steps; Section 3.4 hats)
  schur2_lower Schur2 steps 1-2 only (the elimination factor of eq. 3.3)

With `adaptive` (PCTL, Schur1, Schur2: the alpha-variants of Section 3.5)
the preconditioner is formed from the system with its weak couplings
neglected (Definition 1) and each inverse whose matrix is strongly
diagonally dominant (Definition 2) is a fixed number of Jacobi iterations;
see oracle/adaptive.py for the rules and their readings.

Diagonal ("hat") approximations of Section 3.4, each one entry update per
row, evaluated as t = (d1 * d2) / diag, new = a_ii - t:
  S^_g = A_g - D_gE diag(A_E)^-1 D_Eg       S^_I = A_I - D_IE diag(A_E)^-1 D_EI
  C^_E = A_E - D_EI diag(A_I)^-1 D_IE       C^_g = A_g - D_gE diag(C^_E)^-1 D_Eg
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import adaptive as adp
from . import amg
from .assemble import BlockSystem

KINDS = ("amg", "bdiag", "pctl", "schur1", "schur2", "schur2_lower")


@dataclass
class BlockParams:
    kind: str = "schur2"
    amg: amg.AMGParams = field(default_factory=amg.AMGParams)
    cycles_rad: int = 1
    cycles_E: int = 1
    cycles_I: int = 1
    pctl_p_tol: float = 1e-2           # inner tolerance, Section 4
    pctl_p_maxcycles: int = 100
    inner_tol: float = 0.0             # > 0: option #3 for the inverses the paper's runs solve to a tolerance
    inner_maxcycles: int = 100
    option4_steps: int = 0             # > 0: option #4 for S_I (Schur2) / C_E (Schur1)
    adaptive: bool = False             # Section 3.5 strategy + options #1/#2
    theta_wc: float = 1e-2             # Definition 1
    sigma_wc: float = 0.5
    theta_wd: float = 0.9              # Definition 2
    jacobi_sweeps: int = 2             # option #1


class Counters:
    def __init__(self):
        self.inverses = 0
        self.matvecs = 0


class Inverse:
    """Approximate action of a scalar matrix inverse."""

    def __init__(self, M: sp.csr_matrix, fn: Callable[[np.ndarray], np.ndarray],
                 counters: Counters):
        self.M = M
        self._fn = fn
        self._c = counters

    def __call__(self, b: np.ndarray) -> np.ndarray:
        self._c.inverses += 1
        return self._fn(b)


def amg_inverse(M, params: amg.AMGParams, cycles: int, counters: Counters,
                hier: Optional[amg.Hierarchy] = None) -> Inverse:
    H = hier if hier is not None else amg.setup(M, params)
    inv = Inverse(M, lambda b: amg.apply_cycles(H, b, cycles), counters)
    inv.hierarchy = H
    return inv


def exact_inverse(M, counters: Counters) -> Inverse:
    """Direct sparse LU: for the exactness tests of Section 3.3."""
    lu = spla.splu(sp.csc_matrix(M))
    return Inverse(M, lambda b: lu.solve(b), counters)


def diag_update(A: sp.csr_matrix, d1: np.ndarray, d2: np.ndarray,
                diag: np.ndarray) -> sp.csr_matrix:
    """A - diag(d1 * d2 / diag) on A's own pattern."""
    B = A.copy()
    rows = amg.csr_rows(B)
    isd = B.indices == rows
    t = (d1 * d2) / diag
    B.data[isd] = B.data[isd] - t[rows[isd]]
    return B


def hatted(sys: BlockSystem, kind: str):
    """The explicit scalar matrices whose inverses a kind needs, keyed by
    role: ('g', g) radiation groups, 'E', 'I', 'c' (PCTL coarse)."""
    G = sys.G
    A = sys.blocks
    dE = amg.diagonal_of(A[G])
    dI = amg.diagonal_of(A[G + 1])
    out = {}
    if kind in ("bdiag", "pctl"):
        for g in range(G):
            out[("g", g)] = A[g]
        out["E"] = A[G]
        out["I"] = A[G + 1]
    elif kind == "schur1":
        CE = diag_update(A[G], sys.d_EI, sys.d_IE, dI)
        dCE = amg.diagonal_of(CE)
        for g in range(G):
            out[("g", g)] = diag_update(A[g], sys.d_gE[g], sys.d_Eg[g], dCE)
        out["E"] = CE
        out["I"] = A[G + 1]
    elif kind in ("schur2", "schur2_lower"):
        for g in range(G):
            out[("g", g)] = diag_update(A[g], sys.d_gE[g], sys.d_Eg[g], dE)
        out["E"] = A[G]
        out["I"] = diag_update(A[G + 1], sys.d_IE, sys.d_EI, dE)
    else:
        raise ValueError(kind)
    return out


def pctl_coarse(sys: BlockSystem, p: np.ndarray, pI: np.ndarray) -> sp.csr_matrix:
    """A_c of eq. 3.1 on the shared stencil pattern.  Entry order:
    a^E_ij, then (p_g,i a^g_ij) p_g,j for g ascending, then the ion term,
    then on the diagonal d_Eg p_g and p_g d_gE for g ascending, d_EI p_I,
    p_I d_IE."""
    G = sys.G
    AE = sys.blocks[G]
    for B in sys.blocks:
        if not (np.array_equal(B.indptr, AE.indptr)
                and np.array_equal(B.indices, AE.indices)):
            raise ValueError("PCTL needs all diagonal blocks on one pattern")
    rows = amg.csr_rows(AE)
    cols = AE.indices
    acc = AE.data.copy()
    for g in range(G):
        acc = acc + (p[g][rows] * sys.blocks[g].data) * p[g][cols]
    acc = acc + (pI[rows] * sys.blocks[G + 1].data) * pI[cols]
    isd = rows == cols
    r = rows[isd]
    dg = acc[isd]
    for g in range(G):
        dg = dg + sys.d_Eg[g][r] * p[g][r]
        dg = dg + p[g][r] * sys.d_gE[g][r]
    dg = dg + sys.d_EI[r] * pI[r]
    dg = dg + pI[r] * sys.d_IE[r]
    acc[isd] = dg
    Ac = sp.csr_matrix((acc, AE.indices.copy(), AE.indptr.copy()), shape=AE.shape)
    return Ac


def adaptive_decisions(sys: BlockSystem, kind: str, params: "BlockParams"):
    """Both levels of the adaptive strategy without building any inverse:
    the Definition 1 plan, the modified system, the matrices of the kind's
    inverses on it, and their Definition 2 counts (option #1 where zero)."""
    if kind not in ("pctl", "schur1", "schur2"):
        raise ValueError("the adaptive strategy applies to pctl, schur1 and schur2")
    plan = adp.coupling_plan(sys, params.theta_wc, params.sigma_wc)
    At = adp.drop_weak(sys, plan)
    mats = hatted(At, kind)
    wd = {key: adp.weak_dominance_count(M, params.theta_wd) for key, M in mats.items()}
    return plan, At, mats, wd


class BlockPreconditioner:
    """M^{-1} for one of KINDS built on a BlockSystem."""

    def __init__(self, sys: BlockSystem, params: BlockParams,
                 inverse_factory: Optional[Callable] = None):
        self.sys = sys
        self.params = params
        self.kind = params.kind
        self.counters = Counters()
        G = sys.G
        self.G, self.N = G, sys.N
        fac = inverse_factory or self._amg_factory
        self.inv = {}
        self.setup_info = {}
        self.plan = None
        self.jacobi_roles = set()
        if self.kind == "amg":
            self.Amono = sys.monolithic()
            self.inv["mono"] = fac(self.Amono, "mono")
            return
        wd = None
        if params.adaptive:
            self.plan, sys, mats, wd = adaptive_decisions(sys, self.kind, params)
            self.sys = sys
        else:
            mats = hatted(sys, self.kind)
        if params.option4_steps > 0:
            if self.kind not in ("schur1", "schur2"):
                raise ValueError("option #4 applies to schur1 (C_E) and schur2 (S_I)")
            # the iteration works on the original blocks, not on the hat
            mats = dict(mats)
            mats["I" if self.kind == "schur2" else "E"] = sys.blocks[
                G + 1 if self.kind == "schur2" else G]
        self.mats = mats
        for key, M in mats.items():
            self.inv[key] = fac(M, key)
        if self.kind == "pctl":
            self._pctl_setup(fac)
        if params.adaptive:
            # second level: option #1 where the matrix is strongly diagonally dominant
            if params.option4_steps > 0:
                key4 = "I" if self.kind == "schur2" else "E"
                wd = dict(wd)
                wd[key4] = adp.weak_dominance_count(mats[key4], params.theta_wd)
            self.setup_info["wd_counts"] = wd
            for key, M in mats.items():
                if wd[key] == 0:
                    self.jacobi_roles.add(key)
                    sweeps = params.jacobi_sweeps
                    self.inv[key] = Inverse(M, lambda b, M=M, k=sweeps: adp.jacobi(M, b, k),
                                            self.counters)
        if params.option4_steps > 0:
            self._option4_setup()

    # -- scalar inverse construction -----------------------------------------
    def tolerance_roles(self):
        """The inverses Section 4 approximates to a relative tolerance (option
        #3): the hatted matrices of the Schur preconditioners (C^_E, C^_g for
        Schur1; S^_g, S^_I for Schur2) and PCTL's block relaxations (A_E, A_g,
        A_I); the others (A_I for Schur1, A_E for Schur2, PCTL's A_c) keep the
        fixed number of V-cycles."""
        G = self.G
        groups = {("g", g) for g in range(G)}
        roles = {"schur1": groups | {"E"}, "schur2": groups | {"I"},
                 "schur2_lower": groups | {"I"}, "pctl": groups | {"E", "I"}}.get(self.kind, set())
        if self.params.option4_steps > 0:
            roles = roles - {"I" if self.kind == "schur2" else "E"}
        return roles

    def _amg_factory(self, M, key):
        """key: ('g', g), 'E', 'I', 'c' (PCTL coarse) or 'mono'."""
        role = "g" if isinstance(key, tuple) else key
        cyc = {"g": self.params.cycles_rad, "E": self.params.cycles_E,
               "I": self.params.cycles_I, "c": self.params.cycles_E,
               "mono": 1}[role]
        inv = amg_inverse(M, self.params.amg, cyc, self.counters)
        if self.params.inner_tol > 0 and key in self.tolerance_roles() and not (
                self.params.option4_steps > 0
                and key == ("I" if self.kind == "schur2" else "E")):
            H, tol, maxc = inv.hierarchy, self.params.inner_tol, self.params.inner_maxcycles
            inv.last_cycles = 0

            def fn(b, inv=inv):
                z, k = amg.solve_to_tolerance(H, b, tol, maxc)
                inv.last_cycles = k
                return z
            inv._fn = fn
        return inv

    def _option4_setup(self):
        """Option #4 of Section 3.4: the exact Schur complement's inverse by a
        fixed number of steps from zero,
            Schur2: w <- A_I^{-1}(q + D_IE A_E^{-1}(D_EI w))   (S_I)
            Schur1: w <- A_E^{-1}(q + D_EI A_I^{-1}(D_IE w))   (C_E)
        with the blocks' own inverses inside (the first step is A^{-1} q)."""
        sys = self.sys
        k = self.params.option4_steps
        if self.kind == "schur2":
            outer, inner, d_out, d_in, key = self.inv["I"], self.inv["E"], sys.d_IE, sys.d_EI, "I"
        else:
            outer, inner, d_out, d_in, key = self.inv["E"], self.inv["I"], sys.d_EI, sys.d_IE, "E"

        def fn(q):
            w = outer(q)
            for _ in range(k - 1):
                w = outer(q + d_out * inner(d_in * w))
            return w
        self.inv[key + "4"] = Inverse(outer.M, fn, Counters())
        self.option4_key = key

    def _pctl_setup(self, fac):
        G, N = self.G, self.N
        sys = self.sys
        p = np.empty((G, N))
        cycles = []
        for g in range(G):
            p[g], k = self._p_solve(self.inv[("g", g)], -sys.d_gE[g])
            cycles.append(k)
        pI, k = self._p_solve(self.inv["I"], -sys.d_IE)
        cycles.append(k)
        self.p, self.pI = p, pI
        self.setup_info["p_cycles"] = cycles
        self.Ac = pctl_coarse(sys, p, pI)
        self.inv["c"] = fac(self.Ac, "c")

    def _p_solve(self, inv, rhs):
        """Option #3 with AMG (V-cycles to pctl_p_tol); exact inverses solve once."""
        H = getattr(inv, "hierarchy", None)
        if H is None:
            return inv._fn(rhs), 1
        return amg.solve_to_tolerance(H, rhs, self.params.pctl_p_tol,
                                      self.params.pctl_p_maxcycles)

    # -- application -----------------------------------------------------------
    def __call__(self, b: np.ndarray) -> np.ndarray:
        G, N = self.G, self.N
        sys = self.sys
        if self.kind == "amg":
            return self.inv["mono"](b)
        B = b.reshape(G + 2, N)
        W = np.empty_like(B)
        inv = self.inv
        if self.kind == "bdiag":
            for g in range(G):
                W[g] = inv[("g", g)](B[g])
            W[G] = inv["E"](B[G])
            W[G + 1] = inv["I"](B[G + 1])
        elif self.kind == "pctl":
            W[G] = inv["E"](B[G])
            for g in range(G):
                W[g] = inv[("g", g)](B[g] - sys.d_gE[g] * W[G])
            W[G + 1] = inv["I"](B[G + 1] - sys.d_IE * W[G])
            if self.plan is not None and self.plan.all_into_E_rows_weak:
                return W.reshape(-1)   # no coarse-grid correction needed
            self.counters.matvecs += G + 2
            Rr = (b - sys.matvec(W.reshape(-1))).reshape(G + 2, N)
            rc = Rr[G].copy()
            for g in range(G):
                rc = rc + self.p[g] * Rr[g]
            rc = rc + self.pI * Rr[G + 1]
            wc = inv["c"](rc)
            W[G] = W[G] + wc
            for g in range(G):
                W[g] = W[g] + self.p[g] * wc
            W[G + 1] = W[G + 1] + self.pI * wc
        elif self.kind == "schur1":
            plan = self.plan
            CE = inv["E4"] if "E4" in inv else inv["E"]
            wI = inv["I"](B[G + 1])
            if plan is not None and bool(np.all(plan.gE)):
                # groups independent of E: one C^_E inverse after them
                for g in range(G):
                    W[g] = inv[("g", g)](B[g])
                s = np.zeros(N)
                for g in range(G):
                    s = s + sys.d_Eg[g] * W[g]
                W[G] = CE((B[G] - sys.d_EI * wI) - s)
            else:
                wE = CE(B[G] - sys.d_EI * wI)
                for g in range(G):
                    W[g] = inv[("g", g)](B[g] - sys.d_gE[g] * wE)
                if plan is not None and bool(np.all(plan.Eg)):
                    W[G] = wE
                else:
                    s = np.zeros(N)
                    for g in range(G):
                        s = s + sys.d_Eg[g] * W[g]
                    W[G] = wE - CE(s)
            if plan is not None and plan.IE:
                W[G + 1] = wI
            else:
                W[G + 1] = wI - inv["I"](sys.d_IE * W[G])
        elif self.kind in ("schur2", "schur2_lower"):
            plan = self.plan
            SI = inv["I4"] if "I4" in inv else inv["I"]
            if plan is not None and plan.all_from_E_weak:
                # every row block independent of E: block lower triangular
                for g in range(G):
                    W[g] = inv[("g", g)](B[g])
                W[G + 1] = SI(B[G + 1])
                s = np.zeros(N)
                for g in range(G):
                    s = s + sys.d_Eg[g] * W[g]
                s = s + sys.d_EI * W[G + 1]
                W[G] = inv["E"](B[G] - s)
                return W.reshape(-1)
            wE = inv["E"](B[G])
            for g in range(G):
                W[g] = inv[("g", g)](B[g] - sys.d_gE[g] * wE)
            W[G + 1] = SI(B[G + 1] - sys.d_IE * wE)
            if self.kind == "schur2" and not (plan is not None and plan.all_into_E_rows_weak):
                s = np.zeros(N)
                for g in range(G):
                    s = s + sys.d_Eg[g] * W[g]
                s = s + sys.d_EI * W[G + 1]
                W[G] = wE - inv["E"](s)
            else:
                W[G] = wE
        else:
            raise ValueError(self.kind)
        return W.reshape(-1)

    def dense_operator(self) -> np.ndarray:
        """M^{-1} as a dense matrix (tiny systems only)."""
        n = (self.G + 2) * self.N
        return np.column_stack([self(e) for e in np.eye(n)])
