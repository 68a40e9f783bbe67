"""Restarted GMRES(m) with right preconditioning (oracle).

The paper solves eq. 2.2 with GMRES(m), m = 30, and stops on the Euclidean
norm of the relative residual (Section 4).  Readings taken here:
  * right preconditioning, so the Arnoldi residual estimate |g_{j+1}| is the
    residual of the current iterate;
  * modified Gram-Schmidt, Givens rotations;
  * stop when |g_{j+1}| <= rtol ||b||; at every stop or restart the true
    residual ||b - A x|| is computed and the iteration continues if it is
    above rtol ||b||;
  * N_it counts Arnoldi steps over all restart cycles;
  * flexible=True stores Z = [M^{-1} v_j] and updates x += Z y (FGMRES);
    flexible=False updates x += M^{-1} (V y) (one extra apply per cycle).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla


@dataclass
class GmresInfo:
    iters: int = 0
    restarts: int = 0
    converged: bool = False
    relres_est: float = float("nan")
    relres_true: float = float("nan")
    history: List[float] = field(default_factory=list)
    precond_applies: int = 0


def gmres(matvec: Callable[[np.ndarray], np.ndarray],
          prec: Optional[Callable[[np.ndarray], np.ndarray]],
          b: np.ndarray, x0: Optional[np.ndarray] = None, restart: int = 30,
          max_iters: int = 1000, rtol: float = 1e-8, flexible: bool = True):
    n = len(b)
    M = prec if prec is not None else (lambda v: v.copy())
    info = GmresInfo()

    def apply_M(v):
        info.precond_applies += 1
        return M(v)

    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        info.converged = True
        info.relres_est = info.relres_true = 0.0
        return np.zeros(n), info
    tol = rtol * bnorm
    r = b - matvec(x)
    beta = float(np.linalg.norm(r))
    info.relres_true = info.relres_est = beta / bnorm
    if beta <= tol:
        info.converged = True
        return x, info
    m = restart
    while info.iters < max_iters:
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n)) if flexible else None
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            z = apply_M(V[j])
            if flexible:
                Z[j] = z
            w = matvec(z)
            for i in range(j + 1):
                H[i, j] = float(np.dot(w, V[i]))
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            breakdown = H[j + 1, j] == 0.0
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.sqrt(H[j, j] * H[j, j] + H[j + 1, j] * H[j + 1, j])
            if den == 0.0:
                raise FloatingPointError("GMRES breakdown: singular Hessenberg")
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            info.iters += 1
            k = j + 1
            info.relres_est = abs(g[j + 1]) / bnorm
            info.history.append(info.relres_est)
            if abs(g[j + 1]) <= tol or info.iters >= max_iters or breakdown:
                break
        y = sla.solve_triangular(H[:k, :k], g[:k], lower=False)
        if flexible:
            x = x + Z[:k].T @ y
        else:
            x = x + apply_M(V[:k].T @ y)
        info.restarts += 1
        r = b - matvec(x)
        beta = float(np.linalg.norm(r))
        info.relres_true = beta / bnorm
        if beta <= tol:
            info.converged = True
            break
    return x, info
