"""Adjoint solve and coefficient gradients (oracle).

For x = A(theta)^{-1} b and a loss L(x) with g = dL/dx:
  A^T lambda = g,   dL/db = lambda,   dL/dtheta = -lambda^T (dA/dtheta) x.

A^T of eq. 2.2 has the same block structure with every diagonal block
transposed and the group couplings swapped (D_gE^T = D_gE sits where D_Eg
was); the preconditioner of the requested kind is built on it.

Derivatives of the assembly (unit cells, harmonic face means, see assemble):
  face f = (i, j) of block alpha with T_f = 2 k_i k_j / (k_i + k_j):
    dL/dT_f   = -(lambda_i - lambda_j)(x_i - x_j)
    dT_f/dk_i = 2 k_j^2 / (k_i + k_j)^2
  c_gE[g,k]  (row g: +c on the diagonal, -c in column E):
    dL/dc_gE = -lambda_gk (x_gk - x_Ek)
  c_Eg[g,k]  (row E: +c on the diagonal, -c in column g):
    dL/dc_Eg = -lambda_Ek (x_Ek - x_gk)
  c_EI[k]    (rows E and I):
    dL/dc_EI = -lambda_Ek (x_Ek - x_Ik) - lambda_Ik (x_Ik - x_Ek)
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import krylov
from .assemble import BlockSystem, _neighbours
from .precond import BlockParams, BlockPreconditioner


def gradients(inp, x: np.ndarray, lam: np.ndarray):
    """(dL/dkappa (G+2, N), dL/dc_gE (G, N), dL/dc_Eg (G, N), dL/dc_EI (N,))."""
    if inp.xi is not None:
        raise ValueError("gradients are defined for the symmetric assembly")
    G, dim, n = inp.G, inp.dim, inp.n
    N = n ** dim
    X = x.reshape(G + 2, N)
    Lm = lam.reshape(G + 2, N)
    nbrs = _neighbours(n, dim)
    dk = np.zeros((G + 2, N))
    for a in range(G + 2):
        k = inp.kappa[a]
        for nb in nbrs:
            has = nb >= 0
            i = np.nonzero(has)[0]
            j = nb[has]
            dT = -(Lm[a, i] - Lm[a, j]) * (X[a, i] - X[a, j])
            s = k[i] + k[j]
            dk[a, i] += dT * (2.0 * k[j] * k[j]) / (s * s)
    E, I = G, G + 1
    dgE = -Lm[:G] * (X[:G] - X[E])
    dEg = -Lm[E] * (X[E] - X[:G])
    dEI = -Lm[E] * (X[E] - X[I]) - Lm[I] * (X[I] - X[E])
    return dk, dgE, dEg, dEI


def adjoint_solve(inp, sys: BlockSystem, x: np.ndarray, g: np.ndarray,
                  params: BlockParams, restart=30, max_iters=1000, rtol=1e-8):
    """lambda by preconditioned GMRES on A^T, then the gradients."""
    sysT = sys.transpose()
    M = BlockPreconditioner(sysT, params)
    lam, info = krylov.gmres(sysT.matvec, M, g, restart=restart,
                             max_iters=max_iters, rtol=rtol)
    return lam, gradients(inp, x, lam), info


def adjoint_direct(inp, sys: BlockSystem, x: np.ndarray, g: np.ndarray):
    """Reference adjoint: lambda = splu(A^T) g."""
    A = sys.monolithic()
    lam = spla.splu(sp.csc_matrix(A.T)).solve(g)
    return lam, gradients(inp, x, lam)
