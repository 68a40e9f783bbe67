"""Classical AMG (oracle): the scalar and monolithic AMG the paper uses as its
inner solver (Section 3.1; setup/solve phases, strength threshold 0.25,
C-then-F relaxation going down and F-then-C going up, classical modified
interpolation, Galerkin coarse operators with restriction P^T, at most 100
unknowns on the coarsest level solved by Gaussian elimination).

Components the paper names but does not define, and the readings taken here:
  * coarsening: the paper uses hypre's Falgout coarsening; this oracle uses
    PMIS (De Sterck, Yang, Heys 2006) with integer keys
    (|S^T_i| << 32 | hash32) and ties broken by the larger row index.
    hash32 is the top 32 bits of the first SplitMix64 output (Steele, Lea,
    Flood 2014) for the state seed ^ (level << 56) ^ i.
  * strength: classical, sign-aware: j is a strong dependency of i when
    -a_ij >= theta * max_{k != i}(-a_ik); a row whose maximum is <= 0, or
    whose row sum is >= dominance_theta * a_ii, has no strong dependencies
    (the complement of the counted set of Definition 2, theta_wd = 0.9).
    dominance_theta <= 0 disables that cut.
  * interpolation: classical direct + distribution with the "modified"
    treatment of strong F-F connections that share no C point (lumped into
    the diagonal) and sign-filtered distribution coefficients; no truncation.
  * aggressive coarsening (the paper applies it on the finest level): a
    second pass of the same coarsening over the first pass's C points, on
    their strength graph of distance two (one path suffices), with hash keys
    of level + 64; the long-range interpolation it needs is multipass
    interpolation (Stueben 2001), the passes summed in canonical order.
  * smoother: CF-ordered l1-Jacobi, d_i = a_ii + sum_{j != i} |a_ij|
    (in place of hybrid Gauss-Seidel, which is sequential).
  * coarsest level: dense LU with partial pivoting when it has at most
    dense_max rows; a stalled coarsening with more rows is relaxed by
    n_pre + n_post l1-Jacobi sweeps instead.

Every floating-point reduction that feeds a discrete decision or a stored
entry is written as an explicit left-to-right sum in a stated order (see
``seq_segment_sum``), so that another implementation following the same
order obtains identical bits.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

C_PT = 1
F_PT = -1
UNDECIDED = 0

_MASK64 = np.uint64(0xFFFFFFFFFFFFFFFF)


# ----------------------------------------------------------------------------
# helpers
# ----------------------------------------------------------------------------
def csr_rows(A: sp.csr_matrix) -> np.ndarray:
    """Row index of every stored entry."""
    return np.repeat(np.arange(A.shape[0], dtype=np.int64), np.diff(A.indptr))


def seq_segment_sum(starts: np.ndarray, lens: np.ndarray, vals: np.ndarray,
                    init: Optional[np.ndarray] = None) -> np.ndarray:
    """out[s] = init[s] + vals[starts[s]] + vals[starts[s]+1] + ... added
    strictly left to right (one IEEE addition per term)."""
    nseg = len(starts)
    acc = np.zeros(nseg) if init is None else np.array(init, dtype=np.float64)
    if nseg == 0:
        return acc
    maxlen = int(lens.max()) if len(lens) else 0
    for p in range(maxlen):
        m = lens > p
        acc[m] = acc[m] + vals[starts[m] + p]
    return acc


def diagonal_of(A: sp.csr_matrix) -> np.ndarray:
    rows = csr_rows(A)
    is_d = A.indices == rows
    if np.count_nonzero(is_d) != A.shape[0]:
        raise ValueError("every row must store its diagonal entry")
    d = np.empty(A.shape[0])
    d[rows[is_d]] = A.data[is_d]
    return d


def splitmix64_first(state: np.ndarray) -> np.ndarray:
    """First output of SplitMix64 seeded with ``state`` (uint64 array)."""
    with np.errstate(over="ignore"):
        z = (state + np.uint64(0x9E3779B97F4A7C15)) & _MASK64
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def hash32(seed: int, level: int, idx: np.ndarray) -> np.ndarray:
    st = (np.uint64(seed) ^ (np.uint64(level) << np.uint64(56))
          ^ idx.astype(np.uint64))
    return splitmix64_first(st) >> np.uint64(32)


# ----------------------------------------------------------------------------
# strength of connection
# ----------------------------------------------------------------------------
def strength(A: sp.csr_matrix, theta: float = 0.25,
             dominance_theta: float = 0.9) -> np.ndarray:
    """Boolean flag per stored entry of A: True when the column is a strong
    dependency of the row.  Row sums are taken left to right in ascending
    column order starting from 0."""
    n = A.shape[0]
    rows = csr_rows(A)
    cols = A.indices.astype(np.int64)
    v = A.data
    offd = cols != rows
    m = np.full(n, -np.inf)
    np.maximum.at(m, rows[offd], -v[offd])
    lens = np.diff(A.indptr)
    rs = seq_segment_sum(A.indptr[:-1].astype(np.int64), lens, v)
    diag = diagonal_of(A)
    empty = m <= 0.0
    if dominance_theta > 0.0:
        empty |= rs >= dominance_theta * diag
    S = offd & (-v >= theta * m[rows]) & ~empty[rows]
    return S


def strength_transpose_counts(A: sp.csr_matrix, S: np.ndarray) -> np.ndarray:
    """|S^T_i| = number of rows that depend strongly on i."""
    return np.bincount(A.indices[S], minlength=A.shape[0]).astype(np.int64)


# ----------------------------------------------------------------------------
# PMIS coarsening
# ----------------------------------------------------------------------------
def pmis_keys(A: sp.csr_matrix, S: np.ndarray, seed: int, level: int) -> np.ndarray:
    """PMIS measure as an integer: (|S^T_i| << 32) | hash32(seed, level, i)."""
    stc = strength_transpose_counts(A, S)
    return (stc.astype(np.uint64) << np.uint64(32)) | hash32(seed, level,
                                                            np.arange(A.shape[0]))


def pmis_with_keys(A: sp.csr_matrix, S: np.ndarray, key: np.ndarray,
                   return_rounds: bool = False, initial: Optional[np.ndarray] = None):
    """PMIS rounds (De Sterck, Yang, Heys 2006) for given integer keys.

    Rows nobody depends on (|S^T_i| = 0) start as F, all others undecided.
    Each round, simultaneously over all rows:
      1. an undecided row whose (key, index) is larger than that of every
         undecided row in S_i u S^T_i becomes C;
      2. every other undecided row with a strong dependency on a row made C
         in step 1 becomes F.
    """
    n = A.shape[0]
    rows = csr_rows(A)[S]
    cols = A.indices[S].astype(np.int64)
    stc = strength_transpose_counts(A, S)
    if initial is None:
        state = np.zeros(n, dtype=np.int8)
        state[stc == 0] = F_PT
    else:
        state = initial.astype(np.int8).copy()
    ei = np.concatenate([rows, cols])
    ej = np.concatenate([cols, rows])
    rounds = 0
    while np.any(state == UNDECIDED):
        rounds += 1
        und = state == UNDECIDED
        live = und[ei] & und[ej]
        beaten = (key[ej] > key[ei]) | ((key[ej] == key[ei]) & (ej > ei))
        lose = np.zeros(n, dtype=bool)
        lose[ei[live & beaten]] = True
        new_c = und & ~lose
        state[new_c] = C_PT
        dep = np.zeros(n, dtype=bool)
        hit = new_c[cols] & und[rows] & ~new_c[rows]
        dep[rows[hit]] = True
        state[dep] = F_PT
    if return_rounds:
        return state, rounds
    return state


def pmis(A: sp.csr_matrix, S: np.ndarray, seed: int, level: int,
         return_rounds: bool = False):
    """C/F splitting by PMIS.  Returns int8 array (1 = C, -1 = F)."""
    return pmis_with_keys(A, S, pmis_keys(A, S, seed, level), return_rounds)


# ----------------------------------------------------------------------------
# HMIS coarsening
# ----------------------------------------------------------------------------
def rs_first_pass_tiles(A: sp.csr_matrix, S: np.ndarray, seed: int, level: int,
                        tile: int) -> np.ndarray:
    """C points of the Ruge-Stueben first pass run independently on each tile
    of `tile` consecutive rows, on the strength graph restricted to the tile.

    The measure of a point is the number of undecided tile points that depend
    strongly on it (initially the tile-internal |S^T_i|).  While some undecided
    point has a positive measure, the undecided point with the largest
    (measure, hash32(seed, level, i), i) becomes C; every undecided tile point
    depending strongly on it becomes F, and for each such new F point the
    measures of its undecided tile dependencies rise by one; then the measures
    of the new C point's own undecided tile dependencies drop by one.  Points
    left undecided (measure 0) are not C.  Plain loops: small inputs only."""
    n = A.shape[0]
    rows = csr_rows(A)
    cols = A.indices.astype(np.int64)
    hk = hash32(seed, level, np.arange(n)).astype(np.int64)
    isC = np.zeros(n, dtype=bool)
    for t0 in range(0, n, tile):
        t1 = min(n, t0 + tile)
        dep = {i: [] for i in range(t0, t1)}     # S_i within the tile
        rdep = {i: [] for i in range(t0, t1)}    # S^T_i within the tile
        for e in np.nonzero(S & (rows >= t0) & (rows < t1) & (cols >= t0) & (cols < t1))[0]:
            i, j = int(rows[e]), int(cols[e])
            dep[i].append(j)
            rdep[j].append(i)
        lam = {i: len(rdep[i]) for i in range(t0, t1)}
        state = {i: 0 for i in range(t0, t1)}      # 0 undecided, 1 C, -1 F
        while True:
            cand = [i for i in range(t0, t1) if state[i] == 0 and lam[i] > 0]
            if not cand:
                break
            p = max(cand, key=lambda i: (lam[i], int(hk[i]), i))
            state[p] = 1
            isC[p] = True
            newf = [j for j in rdep[p] if state[j] == 0]
            for j in newf:
                state[j] = -1
            for j in newf:
                for k in dep[j]:
                    if state[k] == 0:
                        lam[k] += 1
            for k in dep[p]:
                if state[k] == 0:
                    lam[k] -= 1
    return isC


def hmis(A: sp.csr_matrix, S: np.ndarray, seed: int, level: int, tile: int = 1024,
         return_rounds: bool = False):
    """Hybrid MIS (De Sterck, Yang, Heys 2006): the tile-local Ruge-Stueben
    first pass fixes its C points; every other point that depends strongly on
    one of them, or that nobody depends on, is F; PMIS rounds with the usual
    keys decide the rest."""
    c0 = rs_first_pass_tiles(A, S, seed, level, tile)
    rows = csr_rows(A)[S]
    cols = A.indices[S].astype(np.int64)
    stc = strength_transpose_counts(A, S)
    state = np.zeros(A.shape[0], dtype=np.int8)
    depc = np.zeros(A.shape[0], dtype=bool)
    depc[rows[c0[cols]]] = True
    state[(stc == 0) | depc] = F_PT
    state[c0] = C_PT
    return pmis_with_keys(A, S, pmis_keys(A, S, seed, level), return_rounds, initial=state)


# ----------------------------------------------------------------------------
# aggressive coarsening (Section 3.1 applies it on the finest level)
# ----------------------------------------------------------------------------
AGGRESSIVE_SALT = 64       # level offset of the second pass's hash keys


def distance2_graph(A: sp.csr_matrix, S: np.ndarray, cand: np.ndarray) -> sp.csr_matrix:
    """Strength graph of distance two among the points of ``cand`` (boolean
    mask), numbered by ascending fine index: j depends on i (i != j) when
    j is in S_i, or j is in S_k for some k in S_i.  Pattern only (values 1)."""
    n = A.shape[0]
    rows = csr_rows(A)[S]
    cols = A.indices[S].astype(np.int64)
    Sm = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))
    reach = Sm @ (sp.identity(n, format="csr") + Sm)     # paths of length 1 or 2
    idx = np.nonzero(cand)[0]
    R = reach[idx][:, idx].tocoo()
    keep = R.row != R.col
    G2 = sp.csr_matrix((np.ones(int(keep.sum())), (R.row[keep], R.col[keep])),
                       shape=(len(idx), len(idx)))
    G2.sum_duplicates()
    G2.data[:] = 1.0
    G2.sort_indices()
    return G2


def aggressive_split(A: sp.csr_matrix, S: np.ndarray, cf1: np.ndarray, seed: int,
                     level: int, coarsening: str = "pmis", tile: int = 1024):
    """Second coarsening pass over the first pass's C points on their distance-two
    strength graph, with the same algorithm as the first pass (every edge of that
    graph is strong) and hash keys of level ``level + AGGRESSIVE_SALT``.  The
    points it keeps are C; every other point is F.  Returns (cf, rounds)."""
    isC1 = cf1 == C_PT
    G2 = distance2_graph(A, S, isC1)
    S2 = np.ones(G2.nnz, dtype=bool)
    if coarsening == "hmis":
        cf2, rounds = hmis(G2, S2, seed, level + AGGRESSIVE_SALT, tile, return_rounds=True)
    else:
        cf2, rounds = pmis(G2, S2, seed, level + AGGRESSIVE_SALT, return_rounds=True)
    cf = np.full(A.shape[0], F_PT, dtype=np.int8)
    cf[np.nonzero(isC1)[0][cf2 == C_PT]] = C_PT
    return cf, rounds


def multipass_passes(A: sp.csr_matrix, S: np.ndarray, cf: np.ndarray) -> np.ndarray:
    """Pass number of every point: 0 on C points; an F point has pass m when its
    nearest C point along strong dependencies is m steps away; -1 when no chain
    of strong dependencies reaches a C point."""
    rows = csr_rows(A)[S]
    cols = A.indices[S].astype(np.int64)
    ps = np.where(cf == C_PT, 0, -1).astype(np.int64)
    m = 0
    while True:
        new = np.unique(rows[(ps[rows] == -1) & (ps[cols] == m)])
        if len(new) == 0:
            return ps
        m += 1
        ps[new] = m


def multipass_interpolation(A: sp.csr_matrix, S: np.ndarray, cf: np.ndarray) -> sp.csr_matrix:
    """Multipass interpolation (Stueben, "An introduction to algebraic
    multigrid", 2001: direct interpolation, then passes through the points
    interpolated so far).  C rows: identity.  A point i of pass m >= 1 with
    P_i = its strong dependencies of pass m - 1:
        sN-_i = sum of its negative off-diagonal entries      (ascending column)
        sN+_i = sum of its other off-diagonal entries          (ascending column)
        sP_i  = sum_{j in P_i} a_ij                            (ascending j)
        alpha_i = sN-_i / sP_i,   d_i = a_ii + sN+_i
        w_ik = -(alpha_i * sum_{j in P_i} a_ij w_jk) / d_i     (sum over ascending j)
    Strong entries are negative, so sP_i < 0 and every positive entry is lumped
    into d_i.  Rows of points no chain reaches are empty."""
    n = A.shape[0]
    isC = cf == C_PT
    cidx = np.cumsum(isC) - 1
    nc = int(isC.sum())
    rows = csr_rows(A)
    cols = A.indices.astype(np.int64)
    v = A.data
    offd = cols != rows
    neg = offd & (v < 0.0)
    pos = offd & ~(v < 0.0)
    starts = A.indptr[:-1].astype(np.int64)
    lens = np.diff(A.indptr)
    sNn = seq_segment_sum(starts, lens, np.where(neg, v, 0.0))
    sNp = seq_segment_sum(starts, lens, np.where(pos, v, 0.0))
    d = diagonal_of(A) + sNp
    ps = multipass_passes(A, S, cf)
    pr = [np.nonzero(isC)[0]]
    pc = [cidx[isC]]
    pv = [np.ones(nc)]
    for m in range(1, int(ps.max()) + 1 if n else 1):
        cur = sp.csr_matrix((np.concatenate(pv), (np.concatenate(pr), np.concatenate(pc))),
                            shape=(n, nc))
        cur.sort_indices()
        sel = S & (ps[rows] == m) & (ps[cols] == m - 1)
        sP = seq_segment_sum(starts, lens, np.where(sel, v, 0.0))
        Am = sp.csr_matrix((v[sel], (rows[sel], cols[sel])), shape=(n, n))
        Am.sort_indices()
        s = spgemm_ordered(Am, cur)
        r = csr_rows(s)
        alpha = sNn[r] / sP[r]
        pr.append(r)
        pc.append(s.indices.astype(np.int64))
        pv.append(-(alpha * s.data) / d[r])
    P = sp.csr_matrix((np.concatenate(pv), (np.concatenate(pr), np.concatenate(pc))),
                      shape=(n, nc))
    P.sort_indices()
    return P


# ----------------------------------------------------------------------------
# classical modified interpolation
# ----------------------------------------------------------------------------
def interpolation(A: sp.csr_matrix, S: np.ndarray, cf: np.ndarray) -> sp.csr_matrix:
    """Prolongation P (n x n_c) by classical modified interpolation (Section
    3.1).  Coarse numbering: C points in ascending fine index.  C rows:
    identity.  F row i, with C_i = C & S_i, F_i = F & S_i and W_i the
    remaining off-diagonal neighbours:
        ahat_kj = a_kj if sign(a_kj) != sign(a_kk) else 0
        sigma_ik = sum_{j in C_i} ahat_kj                  (ascending j)
        L_i = {k in F_i : sigma_ik == 0}
        at_ii = a_ii + sum_{n in W_i u L_i} a_in            (ascending column)
        w_ij = -(a_ij + sum_{k in F_i \\ L_i} a_ik ahat_kj / sigma_ik) / at_ii
                                                            (ascending k)
    The rows are computed one by one by the plain C loop of ``interp.c``
    (one IEEE operation per term, no fused products)."""
    from . import cext
    A = sp.csr_matrix(A)
    A.sort_indices()
    n = A.shape[0]
    isC = cf == C_PT
    cidx = (np.cumsum(isC) - 1).astype(np.int64)
    nc = int(isC.sum())
    indptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
    indices = np.ascontiguousarray(A.indices, dtype=np.int32)
    data = np.ascontiguousarray(A.data, dtype=np.float64)
    strong = np.ascontiguousarray(S, dtype=np.uint8)
    cf8 = np.ascontiguousarray(cf, dtype=np.int8)
    maxrow = int(np.diff(indptr).max()) if n else 0
    sigma = np.zeros(max(1, maxrow))
    cap = A.nnz + n
    p_indptr = np.zeros(n + 1, dtype=np.int64)
    p_indices = np.zeros(max(1, cap), dtype=np.int32)
    p_data = np.zeros(max(1, cap))
    ptr = lambda a: a.ctypes.data  # noqa: E731
    nnz = cext.lib().oracle_interpolation(n, ptr(indptr), ptr(indices), ptr(data), ptr(strong),
                                          ptr(cf8), ptr(cidx), ptr(sigma), ptr(p_indptr),
                                          ptr(p_indices), ptr(p_data))
    P = sp.csr_matrix((p_data[:nnz].copy(), p_indices[:nnz].copy(), p_indptr), shape=(n, nc))
    return P


def interpolation_vectorised(A: sp.csr_matrix, S: np.ndarray, cf: np.ndarray) -> sp.csr_matrix:
    """The same interpolation as ``interpolation``, written with array
    operations (triplet expansion, sorted look-ups).  Kept only as an
    independent cross-check of the per-row loop in the tests."""
    n = A.shape[0]
    isC = cf == C_PT
    cidx = np.cumsum(isC) - 1
    nc = int(isC.sum())
    rows = csr_rows(A)
    cols = A.indices.astype(np.int64)
    v = A.data
    diag = diagonal_of(A)
    offd = cols != rows
    Frow = ~isC[rows]
    sC = S & isC[cols] & Frow            # strong C entries of F rows
    sF = S & ~isC[cols] & Frow           # strong F entries of F rows
    weak = offd & ~S & Frow
    ahat = np.where(np.sign(v) != np.sign(diag[rows]), v, 0.0)

    # strong-C entry lists per row
    eC = np.nonzero(sC)[0]
    cntC = np.bincount(rows[eC], minlength=n)
    startC = np.zeros(n + 1, dtype=np.int64)
    startC[1:] = np.cumsum(cntC)
    # strong-F pairs (i, k)
    eF = np.nonzero(sF)[0]
    pi = rows[eF]
    pk = cols[eF]
    tlen = cntC[pi]
    # triplets (pair p, j in C_i), pairs in CSR order, j ascending
    tp = np.repeat(np.arange(len(eF)), tlen)
    toff = np.arange(len(tp)) - np.repeat(np.cumsum(tlen) - tlen, tlen)
    tj_entry = eC[startC[pi][tp] + toff]             # entry (i, j) in A
    tj = cols[tj_entry]
    tk = pk[tp]
    # look up A(k, j)
    akey = rows * n + cols                            # sorted (CSR order)
    q = tk * n + tj
    pos = np.searchsorted(akey, q)
    pos_c = np.minimum(pos, len(akey) - 1)
    found = akey[pos_c] == q
    ahat_kj = np.where(found, ahat[pos_c], 0.0)
    # sigma per pair, ascending j
    pstart = np.cumsum(tlen) - tlen
    sigma = seq_segment_sum(pstart, tlen, ahat_kj)
    lumped = sigma == 0.0
    # modified diagonal, ascending column order, starting from a_ii
    add = np.zeros(len(v))
    add[weak] = v[weak]
    add[eF[lumped]] = v[eF[lumped]]
    lens = np.diff(A.indptr)
    at_ii = seq_segment_sum(A.indptr[:-1].astype(np.int64), lens, add, init=diag)
    # numerators per strong-C entry (i, j), contributions in ascending k
    a_ik = v[eF][tp]
    with np.errstate(divide="ignore", invalid="ignore"):
        term = np.where(lumped[tp], 0.0, (a_ik * ahat_kj) / sigma[tp])
    order = np.lexsort((tk, tj_entry))               # group by (i,j), then k
    grp = tj_entry[order]
    term_o = term[order]
    # segments: for every strong-C entry, its run in the sorted order
    cnt_e = np.bincount(grp, minlength=len(v))[eC]
    st_e = np.cumsum(cnt_e) - cnt_e
    num = seq_segment_sum(st_e, cnt_e, term_o, init=v[eC])
    w = -num / at_ii[rows[eC]]

    # assemble P
    p_rows = np.concatenate([rows[eC], np.nonzero(isC)[0]])
    p_cols = np.concatenate([cidx[cols[eC]], cidx[isC]])
    p_vals = np.concatenate([w, np.ones(nc)])
    P = sp.csr_matrix((p_vals, (p_rows, p_cols)), shape=(n, nc))
    P.sort_indices()
    return P


# ----------------------------------------------------------------------------
# Galerkin coarse operator
# ----------------------------------------------------------------------------
def spgemm_ordered(A: sp.csr_matrix, B: sp.csr_matrix) -> sp.csr_matrix:
    """C = A B with the structural pattern (every (i, j) reached by some
    a_ik b_kj is stored, even if the sum is zero) and each entry summed left
    to right over ascending k, starting from 0."""
    n = A.shape[0]
    m = B.shape[1]
    ai = csr_rows(A)
    ak = A.indices.astype(np.int64)
    cnt = np.diff(B.indptr)[ak]
    tot = int(cnt.sum())
    e_rep = np.repeat(np.arange(len(ak)), cnt)
    boff = np.arange(tot) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    bidx = B.indptr[ak][e_rep] + boff
    i_x = ai[e_rep]
    j_x = B.indices[bidx].astype(np.int64)
    prod = A.data[e_rep] * B.data[bidx]
    key = i_x * m + j_x
    order = np.argsort(key, kind="stable")           # keeps ascending k
    ks = key[order]
    uniq, first, counts = np.unique(ks, return_index=True, return_counts=True)
    vals = seq_segment_sum(first, counts, prod[order])
    C = sp.csr_matrix((vals, (uniq // m, uniq % m)), shape=(n, m))
    C.sort_indices()
    return C


def transpose_csr(P: sp.csr_matrix) -> sp.csr_matrix:
    """Explicit transpose with columns sorted (entries copied, no arithmetic)."""
    R = sp.csr_matrix(P.T)
    R.sort_indices()
    return R


def galerkin(A: sp.csr_matrix, P: sp.csr_matrix):
    """R = P^T and A_c = R (A P), both products in canonical order."""
    R = transpose_csr(P)
    AP = spgemm_ordered(A, P)
    Ac = spgemm_ordered(R, AP)
    return R, Ac


def l1_diagonal(A: sp.csr_matrix) -> np.ndarray:
    """d_i = a_ii + sum_{j != i} |a_ij| added in ascending column order."""
    rows = csr_rows(A)
    offd = A.indices != rows
    add = np.where(offd, np.abs(A.data), 0.0)
    return seq_segment_sum(A.indptr[:-1].astype(np.int64), np.diff(A.indptr),
                           add, init=diagonal_of(A))


def jp_colours(A: sp.csr_matrix, seed: int, level: int) -> np.ndarray:
    """Jones-Plassmann colouring of the structural graph of A (every stored
    off-diagonal entry is an edge, in both directions).  In round c every
    uncoloured vertex whose (hash32(seed, level, i), i) exceeds that of all its
    uncoloured neighbours gets colour c."""
    n = A.shape[0]
    rows = csr_rows(A)
    cols = A.indices.astype(np.int64)
    off = rows != cols
    ei = np.concatenate([rows[off], cols[off]])
    ej = np.concatenate([cols[off], rows[off]])
    key = hash32(seed, level, np.arange(n)).astype(np.int64)
    colour = np.full(n, -1, dtype=np.int64)
    c = 0
    while np.any(colour < 0):
        unc = colour < 0
        live = unc[ei] & unc[ej]
        beaten = (key[ej] > key[ei]) | ((key[ej] == key[ei]) & (ej > ei))
        lose = np.zeros(n, dtype=bool)
        lose[ei[live & beaten]] = True
        colour[unc & ~lose] = c
        c += 1
    return colour


def gs_sweep(A, dg, b, x, colour, descending=False):
    """Multicolour Gauss-Seidel: colour by colour (ascending, or descending),
    x_c += (b_c - (A x)_c) / a_cc with A x taken after the previous colours."""
    x = x.copy()
    ncol = int(colour.max()) + 1 if len(colour) else 0
    order = range(ncol - 1, -1, -1) if descending else range(ncol)
    for c in order:
        mask = colour == c
        r = b - A @ x
        x[mask] = x[mask] + r[mask] / dg[mask]
    return x


# ----------------------------------------------------------------------------
# hierarchy
# ----------------------------------------------------------------------------
@dataclass
class AMGParams:
    strength_theta: float = 0.25       # Section 3.1
    dominance_theta: float = 0.9       # Definition 2 threshold
    seed: int = 1
    max_levels: int = 25
    coarse_max: int = 100              # Section 3.1: at most 100 DoFs
    dense_max: int = 2000
    n_pre: int = 1
    n_post: int = 1
    coarsening: str = "pmis"           # "pmis" or "hmis"
    hmis_tile: int = 1024
    smoother: str = "cf_l1_jacobi"     # or "mc_gs" (multicolour Gauss-Seidel)
    aggressive_levels: int = 0         # finest levels coarsened aggressively (Section 3.1: 1)


@dataclass
class Level:
    A: sp.csr_matrix
    d: np.ndarray                      # l1 diagonal
    cf: Optional[np.ndarray] = None    # None on the coarsest level
    P: Optional[sp.csr_matrix] = None
    R: Optional[sp.csr_matrix] = None
    pmis_rounds: int = 0
    colour: Optional[np.ndarray] = None  # multicolour Gauss-Seidel colours
    dg: Optional[np.ndarray] = None      # a_ii, for Gauss-Seidel


@dataclass
class Hierarchy:
    levels: List[Level]
    params: AMGParams
    coarse_kind: str = "lu"            # "lu" or "jacobi"
    lu: Optional[tuple] = None
    stats: dict = field(default_factory=dict)

    @property
    def A(self) -> sp.csr_matrix:
        return self.levels[0].A

    def grid_complexity(self) -> float:
        return sum(L.A.shape[0] for L in self.levels) / self.levels[0].A.shape[0]

    def operator_complexity(self) -> float:
        return sum(L.A.nnz for L in self.levels) / self.levels[0].A.nnz


def setup(A: sp.csr_matrix, params: Optional[AMGParams] = None) -> Hierarchy:
    """AMG setup: levels stop when n <= coarse_max, when coarsening stalls
    (no C point, or more than 90% C points) or at max_levels."""
    p = params or AMGParams()
    A = sp.csr_matrix(A)
    A.sort_indices()
    levels: List[Level] = []
    lvl = 0
    while True:
        n = A.shape[0]
        d = l1_diagonal(A)
        if n <= p.coarse_max or lvl == p.max_levels - 1:
            levels.append(Level(A, d))
            break
        S = strength(A, p.strength_theta, p.dominance_theta)
        if p.coarsening == "hmis":
            cf, rounds = hmis(A, S, p.seed, lvl, p.hmis_tile, return_rounds=True)
        else:
            cf, rounds = pmis(A, S, p.seed, lvl, return_rounds=True)
        aggressive = lvl < p.aggressive_levels
        if aggressive:
            cf, rounds2 = aggressive_split(A, S, cf, p.seed, lvl, p.coarsening, p.hmis_tile)
            rounds += rounds2
        nc = int(np.count_nonzero(cf == C_PT))
        if nc == 0 or 10 * nc > 9 * n:
            levels.append(Level(A, d))
            break
        P = multipass_interpolation(A, S, cf) if aggressive else interpolation(A, S, cf)
        R, Ac = galerkin(A, P)
        levels.append(Level(A, d, cf, P, R, rounds))
        A = Ac
        lvl += 1
    if p.smoother == "mc_gs":
        for k, L in enumerate(levels):
            L.colour = jp_colours(L.A, p.seed, k)
            L.dg = diagonal_of(L.A)
    H = Hierarchy(levels, p)
    Ac = levels[-1].A
    if Ac.shape[0] <= p.dense_max:
        H.coarse_kind = "lu"
        H.lu = sla.lu_factor(Ac.toarray())
    else:
        H.coarse_kind = "jacobi"
    return H


# ----------------------------------------------------------------------------
# solve phase
# ----------------------------------------------------------------------------
def half_sweep(A, d, b, x, mask):
    """l1-Jacobi on the rows in ``mask``: x_S += (b_S - (A x)_S) / d_S, with
    A x evaluated at the values x had when the half-sweep started."""
    r = b - A @ x
    y = x.copy()
    y[mask] = x[mask] + r[mask] / d[mask]
    return y


def vcycle(H: Hierarchy, b: np.ndarray, lvl: int = 0) -> np.ndarray:
    """One V(n_pre, n_post) cycle with zero initial guess (Section 3.1)."""
    L = H.levels[lvl]
    p = H.params
    gs = p.smoother == "mc_gs"
    if lvl == len(H.levels) - 1:
        if H.coarse_kind == "lu":
            return sla.lu_solve(H.lu, b)
        x = np.zeros_like(b)
        if gs:                               # ascending, then descending colours
            for _ in range(p.n_pre):
                x = gs_sweep(L.A, L.dg, b, x, L.colour)
            for _ in range(p.n_post):
                x = gs_sweep(L.A, L.dg, b, x, L.colour, descending=True)
            return x
        allrows = np.ones(len(b), dtype=bool)
        for _ in range(p.n_pre + p.n_post):
            x = half_sweep(L.A, L.d, b, x, allrows)
        return x
    isC = L.cf == C_PT
    isF = ~isC
    x = np.zeros_like(b)
    for _ in range(p.n_pre):                 # going down: C then F (or ascending colours)
        if gs:
            x = gs_sweep(L.A, L.dg, b, x, L.colour)
        else:
            x = half_sweep(L.A, L.d, b, x, isC)
            x = half_sweep(L.A, L.d, b, x, isF)
    r = b - L.A @ x
    e = vcycle(H, L.R @ r, lvl + 1)
    x = x + L.P @ e
    for _ in range(p.n_post):                # going up: F then C (or descending colours)
        if gs:
            x = gs_sweep(L.A, L.dg, b, x, L.colour, descending=True)
        else:
            x = half_sweep(L.A, L.d, b, x, isF)
            x = half_sweep(L.A, L.d, b, x, isC)
    return x


def apply_cycles(H: Hierarchy, b: np.ndarray, k: int = 1) -> np.ndarray:
    """k V-cycles as a stationary iteration from zero: z <- z + V(b - A z)."""
    z = vcycle(H, b)
    for _ in range(k - 1):
        z = z + vcycle(H, b - H.A @ z)
    return z


def solve_to_tolerance(H: Hierarchy, b: np.ndarray, rtol: float,
                       max_cycles: int = 100):
    """V-cycles until ||b - A z|| < rtol ||b|| (option #3 of Section 3.4).
    Returns (z, cycles)."""
    nb = np.linalg.norm(b)
    z = np.zeros_like(b)
    if nb == 0.0:
        return z, 0
    k = 0
    r = b.copy()
    while k < max_cycles:
        z = z + vcycle(H, r)
        k += 1
        r = b - H.A @ z
        if np.linalg.norm(r) < rtol * nb:
            break
    return z, k
