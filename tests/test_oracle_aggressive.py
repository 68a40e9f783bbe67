"""Pins of the oracle's aggressive coarsening and multipass interpolation
(Section 3.1 names aggressive coarsening on the finest level), on the CPU.

  * the distance-two strength graph equals the boolean square of the
    strength graph computed densely;
  * the second pass keeps a subset of the first pass's C points, independent
    in the distance-two graph under PMIS, and every dropped point that some
    point depends on at distance two depends on a kept one (PMIS and HMIS);
  * pass numbers are the graph distances to the C set (scipy's shortest
    paths over the strength graph);
  * multipass weights: closed forms on 1D chains and on a row with a
    positive entry, exact interpolation of constants for zero row sums,
    non-negative weights for M-matrices;
  * the aggressive hierarchy is cheaper and still a convergent preconditioner.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse import csgraph

import synth_inputs as si
from oracle import amg, assemble, krylov


def _random_mmatrix(n, seed, zero_rowsum=False, nonsym=True):
    rng = np.random.default_rng(seed)
    dense = np.zeros((n, n))
    for i in range(n):
        for j in rng.choice(n, size=min(n - 1, 4), replace=False):
            if j != i:
                dense[i, j] = -rng.uniform(0.1, 1.0)
    if not nonsym:
        dense = np.minimum(dense, dense.T)
    off = -dense.sum(axis=1)
    d = off if zero_rowsum else off + rng.uniform(0.05, 0.5, size=n)
    d[d == 0] = 1.0
    A = sp.csr_matrix(dense + np.diag(d))
    A.sort_indices()
    return A


def _chain(n):
    A = sp.csr_matrix(sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]))
    A.sort_indices()
    return A


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_distance2_graph_is_boolean_square(seed):
    A = _random_mmatrix(40, seed)
    S = amg.strength(A)
    Sd = np.zeros(A.shape, dtype=bool)
    Sd[amg.csr_rows(A)[S], A.indices[S]] = True
    reach = Sd | ((Sd.astype(int) @ Sd.astype(int)) > 0)
    cand = np.random.default_rng(seed + 10).uniform(size=40) < 0.5
    idx = np.nonzero(cand)[0]
    want = reach[np.ix_(idx, idx)] & ~np.eye(len(idx), dtype=bool)
    G2 = amg.distance2_graph(A, S, cand)
    assert np.array_equal(G2.toarray() != 0, want)


@pytest.mark.parametrize("coarsening", ["pmis", "hmis"])
def test_second_pass_is_a_distance2_independent_cover(coarsening):
    A = oracle_block()
    S = amg.strength(A)
    cf1 = amg.pmis(A, S, 7, 0) if coarsening == "pmis" else amg.hmis(A, S, 7, 0, tile=256)
    cf, _ = amg.aggressive_split(A, S, cf1, 7, 0, coarsening, 256)
    isC1, isC = cf1 == amg.C_PT, cf == amg.C_PT
    assert np.all(isC1[isC]) and 0 < isC.sum() < isC1.sum()
    G2 = amg.distance2_graph(A, S, isC1).toarray() != 0
    keep = isC[isC1]
    if coarsening == "pmis":      # a Ruge-Stueben pass may keep a point and one it depends on
        assert not np.any(G2[np.ix_(keep, keep)])           # independent
    depended = G2.any(axis=0)                                # someone depends on it
    dropped = ~keep & depended
    assert np.all(G2[dropped][:, keep].any(axis=1))          # covered by a kept point


def oracle_block():
    return assemble.assemble(si.generate(1, 2, 20, 41)).blocks[0]


@pytest.mark.parametrize("seed", [3, 4])
def test_passes_are_graph_distances_to_C(seed):
    A = _random_mmatrix(60, seed)
    S = amg.strength(A)
    cf = amg.pmis(A, S, 5, 0)
    cf2, _ = amg.aggressive_split(A, S, cf, 5, 0)
    ps = amg.multipass_passes(A, S, cf2)
    # i -> j edge when j is a strong dependency of i; distance from i to the C set
    G = sp.csr_matrix((np.ones(int(S.sum())), (amg.csr_rows(A)[S], A.indices[S])), shape=A.shape)
    Cpts = np.nonzero(cf2 == amg.C_PT)[0]
    dist = csgraph.shortest_path(G.T, unweighted=True, indices=Cpts).min(axis=0)
    want = np.where(np.isinf(dist), -1, dist).astype(np.int64)
    assert np.array_equal(ps, want)


def test_multipass_chain_closed_forms():
    A = _chain(5)
    S = amg.strength(A)
    cf = np.array([1, -1, -1, -1, 1], dtype=np.int8)
    P = amg.multipass_interpolation(A, S, cf).toarray()
    np.testing.assert_array_equal(P, [[1, 0], [1, 0], [0.5, 0.5], [0, 1], [0, 1]])
    # one C point at the end of a chain with a Dirichlet-type last row:
    # passes 1, 2, 3 with weights 1, 1, 1/2
    A = _chain(4)
    S = amg.strength(A)
    P = amg.multipass_interpolation(A, S, np.array([1, -1, -1, -1], dtype=np.int8)).toarray()
    np.testing.assert_array_equal(P[:, 0], [1.0, 1.0, 1.0, 0.5])


def test_multipass_lumps_positive_entries_into_the_diagonal():
    A = sp.csr_matrix(np.array([[2.0, -1.0, 0.0], [-1.0, 3.0, 0.5], [0.0, -1.0, 2.0]]))
    S = amg.strength(A)
    P = amg.multipass_interpolation(A, S, np.array([1, -1, -1], dtype=np.int8)).toarray()
    # row 1: alpha = 1, d = 3 + 0.5; row 2 goes through row 1: (1/3.5) / 2
    np.testing.assert_allclose(P[:, 0], [1.0, 2.0 / 7.0, 1.0 / 7.0], rtol=1e-15)


@pytest.mark.parametrize("seed", [5, 6, 7])
def test_multipass_interpolates_constants_for_zero_row_sums(seed):
    A = _random_mmatrix(80, seed, zero_rowsum=True)
    S = amg.strength(A, dominance_theta=0.0)
    cf, _ = amg.aggressive_split(A, S, amg.pmis(A, S, 2, 0), 2, 0)
    P = amg.multipass_interpolation(A, S, cf)
    ps = amg.multipass_passes(A, S, cf)
    reached = ps >= 0
    assert np.all(P.data >= 0.0)
    np.testing.assert_allclose(P @ np.ones(P.shape[1]), np.where(reached, 1.0, 0.0), atol=1e-13)
    assert np.all(np.diff(P.indptr)[~reached] == 0)
    assert ps.max() >= 2                                     # long-range rows exist


@pytest.mark.parametrize("kind", ["block", "mono"])
def test_aggressive_hierarchy_is_cheaper_and_converges(kind):
    inp = si.generate(2, 3, 12, 42)
    sysm = assemble.assemble(inp)
    A = sysm.blocks[0] if kind == "block" else sysm.monolithic()
    H0 = amg.setup(A, amg.AMGParams(seed=7))
    H1 = amg.setup(A, amg.AMGParams(seed=7, aggressive_levels=1))
    assert H1.operator_complexity() < H0.operator_complexity()
    assert H1.levels[1].A.shape[0] < 0.5 * H0.levels[1].A.shape[0]
    S = amg.strength(A)
    np.testing.assert_array_equal(H1.levels[0].P.toarray(),
                                  amg.multipass_interpolation(A, S, H1.levels[0].cf).toarray())
    b = sysm.monolithic() @ np.ones(A.shape[0]) if kind == "mono" else A @ np.ones(A.shape[0])
    x, info = krylov.gmres(lambda v: A @ v, lambda r: amg.vcycle(H1, r), b, rtol=1e-8)
    assert info.converged
    assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b) * (1 + 1e-9)
