"""Block system of the paper's eq. 2.2 from per-cell coefficients (oracle).

Discretisation reading (Section 2 gives a cell-centred finite-volume scheme
without the details): unit cells, two-point flux with the harmonic mean of
the two cell coefficients on interior faces, zero-flux outer boundary, a mass
term m on every diagonal.  The coupling blocks are diagonal (Section 2):
D_gE = -c_gE, D_Eg = -c_Eg, D_EI = D_IE = -c_EI, and each coupling magnitude
is added to the diagonal of the row it sits in, so every row of the
monolithic matrix sums to m.

Summation order of a diagonal entry (fixed so that any other implementation
can reproduce it bit for bit): start from 0, add the face weights in the
direction order -x, +x, -y, +y, -z, +z (interior faces only), then the row's
coupling magnitudes (E rows: groups in ascending order, then c_EI), then m.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np
import scipy.sparse as sp


@dataclass
class BlockSystem:
    G: int
    N: int
    blocks: List[sp.csr_matrix]   # G+2 blocks, order [1..G, E, I]
    d_gE: np.ndarray              # (G, N) diagonal of D_gE (row g, column E)
    d_Eg: np.ndarray              # (G, N) diagonal of D_Eg (row E, column g)
    d_EI: np.ndarray              # (N,)   diagonal of D_EI
    d_IE: np.ndarray              # (N,)   diagonal of D_IE

    @property
    def n(self) -> int:
        return (self.G + 2) * self.N

    def monolithic(self) -> sp.csr_matrix:
        """The full matrix of eq. 2.2, unknowns ordered [T_1..T_G, T_E, T_I]."""
        G = self.G
        nb = G + 2
        grid = [[None] * nb for _ in range(nb)]
        for a in range(nb):
            grid[a][a] = self.blocks[a]
        for g in range(G):
            grid[g][G] = sp.diags(self.d_gE[g], format="csr")
            grid[G][g] = sp.diags(self.d_Eg[g], format="csr")
        grid[G][G + 1] = sp.diags(self.d_EI, format="csr")
        grid[G + 1][G] = sp.diags(self.d_IE, format="csr")
        M = sp.bmat(grid, format="csr")
        M.sort_indices()
        return M

    def transpose(self) -> "BlockSystem":
        """A^T as a block system: blocks transposed, D_gE and D_Eg swapped."""
        return BlockSystem(self.G, self.N,
                           [sorted_csr(B.T) for B in self.blocks],
                           self.d_Eg.copy(), self.d_gE.copy(),
                           self.d_IE.copy(), self.d_EI.copy())

    def matvec(self, x: np.ndarray) -> np.ndarray:
        """y = A x using the block form of eq. 2.2."""
        G, N = self.G, self.N
        X = x.reshape(G + 2, N)
        Y = np.empty_like(X)
        for g in range(G):
            Y[g] = self.blocks[g] @ X[g] + self.d_gE[g] * X[G]
        Y[G] = self.blocks[G] @ X[G] + self.d_EI * X[G + 1]
        for g in range(G):
            Y[G] += self.d_Eg[g] * X[g]
        Y[G + 1] = self.blocks[G + 1] @ X[G + 1] + self.d_IE * X[G]
        return Y.reshape(-1)


def sorted_csr(M) -> sp.csr_matrix:
    M = sp.csr_matrix(M)
    M.sort_indices()
    return M


def _neighbours(n: int, dim: int):
    """For each direction (-x,+x,-y,+y[,-z,+z]) the neighbour index or -1."""
    N = n ** dim
    c = np.arange(N)
    coords = []
    for ax in range(dim):
        coords.append((c // (n ** ax)) % n)
    out = []
    for ax in range(dim):
        stride = n ** ax
        out.append(np.where(coords[ax] > 0, c - stride, -1))
        out.append(np.where(coords[ax] < n - 1, c + stride, -1))
    return out


def harmonic_face(ka: np.ndarray, kb: np.ndarray) -> np.ndarray:
    """Face transmissibility 2 ka kb / (ka + kb) (unit spacing)."""
    return (2.0 * ka) * kb / (ka + kb)


def assemble(inp) -> BlockSystem:
    """Assemble eq. 2.2 from a synth_inputs.Inputs instance."""
    G, dim, n = inp.G, inp.dim, inp.n
    N = n ** dim
    nbrs = _neighbours(n, dim)
    blocks = []
    for a in range(G + 2):
        kap = inp.kappa[a]
        rows, cols, vals = [], [], []
        diag = np.zeros(N)
        for d, nb in enumerate(nbrs):
            has = nb >= 0
            i = np.nonzero(has)[0]
            j = nb[has]
            w = harmonic_face(kap[i], kap[j])
            if inp.xi is not None:
                w = w * (1.0 + 0.5 * inp.xi[a, i, d])
            rows.append(i)
            cols.append(j)
            vals.append(-w)
            diag[i] += w          # each row gets its faces in direction order
        if a < G:
            diag += inp.c_gE[a]
        elif a == G:
            for g in range(G):
                diag += inp.c_Eg[g]
            diag += inp.c_EI
        else:
            diag += inp.c_EI
        diag += inp.mass
        rows.append(np.arange(N))
        cols.append(np.arange(N))
        vals.append(diag)
        B = sp.csr_matrix((np.concatenate(vals),
                           (np.concatenate(rows), np.concatenate(cols))),
                          shape=(N, N))
        B.sort_indices()
        blocks.append(B)
    return BlockSystem(G, N, blocks, -inp.c_gE.copy(), -inp.c_Eg.copy(),
                       -inp.c_EI.copy(), -inp.c_EI.copy())
