"""Pins of the oracle's AMG (Section 3.1) against hand-derived fixtures,
published test vectors, closed forms and invariants."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth_inputs as si
from oracle import amg, assemble

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _csr_from_rows(rows, vals):
    n = len(rows)
    r = np.concatenate([[i] * len(c) for i, c in enumerate(rows)])
    A = sp.csr_matrix((np.concatenate(vals), (r, np.concatenate(rows))), shape=(n, n))
    A.sort_indices()
    return A


def _laplace2d(n):
    T = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])
    I = sp.eye(n)
    A = sp.csr_matrix(sp.kron(I, T) + sp.kron(T, I))
    A.eliminate_zeros()
    A.sort_indices()
    return A


def _random_mmatrix(n, seed, density=0.15, nonsym=True):
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=density, random_state=rng, format="csr")
    M.data[:] = -rng.uniform(0.05, 1.0, size=M.nnz)
    if not nonsym:
        M = (M + M.T) * 0.5
    M = sp.csr_matrix(M)
    M.setdiag(0.0)
    M.eliminate_zeros()
    d = -np.asarray(M.sum(axis=1)).ravel() + rng.uniform(0.0, 0.5, size=n)
    A = sp.csr_matrix(M + sp.diags(d + 1e-3))
    A.sort_indices()
    return A


# --- hash ---------------------------------------------------------------------
def test_splitmix64_published_sequence():
    g = _load("splitmix64_seed1234567.json")
    gamma = 0x9E3779B97F4A7C15
    states = np.array([(g["seed"] + k * gamma) % 2 ** 64 for k in range(5)], dtype=np.uint64)
    out = amg.splitmix64_first(states)
    assert [int(v) for v in out] == [int(v) for v in g["first_outputs"]]


def test_hash32_is_top_half():
    idx = np.arange(10)
    h = amg.hash32(7, 3, idx)
    full = amg.splitmix64_first(np.uint64(7) ^ (np.uint64(3) << np.uint64(56)) ^ idx.astype(np.uint64))
    assert np.array_equal(h, full >> np.uint64(32))
    assert h.max() < 2 ** 32


# --- strength -------------------------------------------------------------------
def test_strength_hand_fixture():
    g = _load("strength_5x5.json")
    A = _csr_from_rows(g["rows"], g["vals"])
    S_on = amg.strength(A, 0.25, 0.9)
    S_off = amg.strength(A, 0.25, 0.0)
    exp_on = np.concatenate(g["strong_dominance_on"])
    exp_off = np.concatenate(g["strong_dominance_off"])
    assert np.array_equal(S_on, exp_on)
    assert np.array_equal(S_off, exp_off)
    assert np.array_equal(amg.strength_transpose_counts(A, S_on), g["st_counts_dominance_on"])


def test_strength_laplacian_all_neighbours_strong():
    A = _laplace2d(8)
    S = amg.strength(A, 0.25, 0.9)
    offd = A.indices != amg.csr_rows(A)
    # boundary rows of the Dirichlet Laplacian have row sum 1 or 2 < 0.9*4
    assert np.array_equal(S, offd)


# --- PMIS -----------------------------------------------------------------------
def test_pmis_chain_hand_rounds():
    # symmetric chain 0-1-2-3-4, increasing keys: rounds C{4},F{3}; C{2},F{1}; C{0}
    A = sp.csr_matrix(sp.diags([-np.ones(4), 2 * np.ones(5), -np.ones(4)], [-1, 0, 1]))
    A.sort_indices()
    S = amg.strength(A, 0.25, 0.0)
    key = np.arange(5, dtype=np.uint64) + np.uint64(1 << 32)
    cf, rounds = amg.pmis_with_keys(A, S, key, return_rounds=True)
    assert cf.tolist() == [1, -1, 1, -1, 1]
    assert rounds == 3
    key_dec = (np.uint64(10) - np.arange(5, dtype=np.uint64))
    cf2 = amg.pmis_with_keys(A, S, key_dec)
    assert cf2.tolist() == [1, -1, 1, -1, 1]


def _pmis_invariants(A, S, cf, key):
    rows = amg.csr_rows(A)
    cols = A.indices.astype(np.int64)
    n = A.shape[0]
    stc = amg.strength_transpose_counts(A, S)
    assert set(np.unique(cf)) <= {1, -1}
    isC = cf == 1
    # a C point i may depend strongly on a C point j only if i won first,
    # i.e. (key_i, i) > (key_j, j); otherwise i would have been made F
    cc = S & isC[rows] & isC[cols]
    ki, kj = key[rows[cc]], key[cols[cc]]
    assert np.all((ki > kj) | ((ki == kj) & (rows[cc] > cols[cc])))
    # every F point with |S^T| > 0 depends strongly on some C point
    hasC = np.zeros(n, dtype=bool)
    hasC[rows[S & isC[cols]]] = True
    assert np.all(hasC[(cf == -1) & (stc > 0)])
    # rows nobody depends on are F
    assert np.all(cf[stc == 0] == -1)


def _pmis_brute(A, S, key):
    """Round rule evaluated row by row with Python sets (tiny inputs)."""
    n = A.shape[0]
    Si = [set() for _ in range(n)]
    STi = [set() for _ in range(n)]
    for i in range(n):
        for e in range(A.indptr[i], A.indptr[i + 1]):
            if S[e]:
                Si[i].add(int(A.indices[e]))
                STi[int(A.indices[e])].add(i)
    state = [0 if STi[i] else -1 for i in range(n)]
    while 0 in state:
        newc = []
        for i in range(n):
            if state[i] != 0:
                continue
            nb = [j for j in Si[i] | STi[i] if state[j] == 0]
            if all((int(key[i]), i) > (int(key[j]), j) for j in nb):
                newc.append(i)
        for i in newc:
            state[i] = 1
        for j in range(n):
            if state[j] == 0 and any(c in Si[j] for c in newc):
                state[j] = -1
    return np.array(state, dtype=np.int8)


@pytest.mark.parametrize("seed", range(6))
def test_pmis_invariants_and_brute_force(seed):
    A = _random_mmatrix(60, seed)
    S = amg.strength(A, 0.25, 0.9)
    key = amg.pmis_keys(A, S, seed, 0)
    cf = amg.pmis_with_keys(A, S, key)
    _pmis_invariants(A, S, cf, key)
    assert np.array_equal(cf, _pmis_brute(A, S, key))


def test_pmis_on_generator_block():
    inp = si.generate(1, 2, 16, 11)
    A = assemble.assemble(inp).blocks[1]
    S = amg.strength(A)
    cf = amg.pmis(A, S, 11, 0)
    _pmis_invariants(A, S, cf, amg.pmis_keys(A, S, 11, 0))


# --- interpolation ----------------------------------------------------------------
def test_interpolation_hand_fixture():
    g = _load("interp_6pt.json")
    A = _csr_from_rows(g["rows"], g["vals"])
    S = amg.strength(A, 0.25, 0.9)
    cf = np.array(g["cf"], dtype=np.int8)
    P = amg.interpolation(A, S, cf).toarray()
    exp = np.zeros((6, 3))
    for i, j, num, den in g["P_entries"]:
        exp[i, j] = num / den
    assert np.array_equal(P != 0, exp != 0)
    np.testing.assert_allclose(P, exp, rtol=1e-15, atol=0)


def test_interpolation_sign_filter_hand_fixture():
    """Positive off-diagonal entries in the rows of strong F neighbours: the
    sign filter of the distribution coefficients moves a whole F-F coupling to
    one C point and lumps another into the diagonal."""
    g = _load("interp_positive_5pt.json")
    A = _csr_from_rows(g["rows"], g["vals"])
    S = amg.strength(A, 0.25, 0.9)
    strong = {i: sorted(int(j) for j in A.indices[A.indptr[i]:A.indptr[i + 1]][
        S[A.indptr[i]:A.indptr[i + 1]]]) for i in range(5)}
    assert strong[0] == [1, 2, 3, 4] and strong[2] == [0, 1] and strong[4] == [0]
    cf = np.array(g["cf"], dtype=np.int8)
    P = amg.interpolation(A, S, cf).toarray()
    exp = np.zeros((5, 2))
    for i, j, num, den in g["P_entries"]:
        exp[i, j] = num / den
    assert np.array_equal(P, exp)
    # the values an unfiltered distribution would give are not these
    for j, num, den in g["no_filter_row0"]:
        assert P[0, j] != num / den
    Pv = amg.interpolation_vectorised(A, S, cf).toarray()
    assert np.array_equal(Pv, exp)


def _mixed_sign_matrix(n, seed, density=0.12, frac_pos=0.2):
    """Random nonsymmetric matrix with a positive diagonal and off-diagonal
    entries of both signs (about frac_pos of them positive)."""
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=density, random_state=rng, format="csr")
    mag = rng.uniform(0.05, 1.0, size=M.nnz)
    pos = rng.uniform(size=M.nnz) < frac_pos
    M.data[:] = np.where(pos, mag * 0.5, -mag)
    M = sp.csr_matrix(M)
    M.setdiag(0.0)
    M.eliminate_zeros()
    d = np.asarray(abs(M).sum(axis=1)).ravel() * rng.uniform(0.6, 1.2, size=n) + 0.1
    A = sp.csr_matrix(M + sp.diags(d))
    A.sort_indices()
    return A


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_interpolation_loop_matches_vectorised_form(seed):
    """The per-row loop and the array formulation of the same formula agree
    bit for bit, on every level of a hierarchy of a matrix with off-diagonal
    entries of both signs (where the sign filter is active)."""
    A = _mixed_sign_matrix(400, seed)
    filt = 0
    for lvl in range(4):
        S = amg.strength(A, 0.25, 0.9)
        cf = amg.pmis(A, S, seed, lvl)
        if not np.any(cf == 1) or np.all(cf == 1):
            break
        P = amg.interpolation(A, S, cf)
        Pv = amg.interpolation_vectorised(A, S, cf)
        assert np.array_equal(P.indptr, Pv.indptr) and np.array_equal(P.indices, Pv.indices)
        assert np.array_equal(P.data.view(np.int64), Pv.data.view(np.int64))
        rows = amg.csr_rows(A)
        d = amg.diagonal_of(A)
        filt += int(np.count_nonzero((A.indices != rows) & (np.sign(A.data) == np.sign(d[rows]))))
        _, A = amg.galerkin(A, P)
    assert filt > 0


def test_interpolation_1d_alternating_is_half():
    n = 9
    A = sp.csr_matrix(sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]))
    A.sort_indices()
    S = amg.strength(A, 0.25, 0.0)
    cf = np.array([1 if i % 2 == 0 else -1 for i in range(n)], dtype=np.int8)
    P = amg.interpolation(A, S, cf).toarray()
    for i in range(1, n, 2):
        assert P[i, i // 2] == 0.5 and P[i, i // 2 + 1] == 0.5
    for i in range(0, n, 2):
        assert P[i, i // 2] == 1.0 and P[i].sum() == 1.0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_interpolation_exact_for_constants(seed):
    """Zero-row-sum M-matrix (zero-flux Laplacian, random kappa, no mass, no
    couplings): P 1 = 1 on every C row and every F row with a strong C point."""
    inp = si.generate(1, 2, 24, 100 + seed, zero_row_sum=True)
    inp_ns = si.generate(1, 2, 24, 100 + seed, zero_row_sum=True, nonsym=True)
    for the in (inp, inp_ns):
        A = assemble.assemble(the).blocks[0]
        S = amg.strength(A, 0.25, 0.0)
        cf = amg.pmis(A, S, seed, 0)
        P = amg.interpolation(A, S, cf)
        rows = amg.csr_rows(A)
        hasC = np.zeros(A.shape[0], dtype=bool)
        hasC[rows[S & (cf[A.indices] == 1)]] = True
        sel = (cf == 1) | hasC
        one = P @ np.ones(P.shape[1])
        np.testing.assert_allclose(one[sel], 1.0, rtol=0, atol=1e-14)
        assert np.all(one[~sel] == 0.0)


def test_interpolation_rows_sorted_and_c_identity():
    inp = si.generate(2, 2, 12, 5)
    A = assemble.assemble(inp).monolithic()
    S = amg.strength(A)
    cf = amg.pmis(A, S, 5, 0)
    P = amg.interpolation(A, S, cf)
    assert P.has_sorted_indices
    cidx = np.cumsum(cf == 1) - 1
    for i in np.nonzero(cf == 1)[0][:50]:
        assert P.indices[P.indptr[i]:P.indptr[i + 1]].tolist() == [cidx[i]]
        assert P.data[P.indptr[i]] == 1.0


# --- Galerkin -------------------------------------------------------------------
def test_spgemm_keeps_structural_zeros_and_orders():
    A = sp.csr_matrix(np.array([[1.0, 1.0], [0.0, 2.0]]))
    B = sp.csr_matrix(np.array([[1.0, 0.0], [-1.0, 3.0]]))
    C = amg.spgemm_ordered(A, B)
    # (0,0) = 1*1 + 1*(-1) = 0 is stored
    assert C.nnz == 4
    np.testing.assert_array_equal(C.toarray(), A.toarray() @ B.toarray())


@pytest.mark.parametrize("seed", [0, 1])
def test_galerkin_dense_identity(seed):
    A = _random_mmatrix(50, seed)
    S = amg.strength(A)
    cf = amg.pmis(A, S, seed, 0)
    P = amg.interpolation(A, S, cf)
    R, Ac = amg.galerkin(A, P)
    Pd, Ad = P.toarray(), A.toarray()
    np.testing.assert_allclose(Ac.toarray(), Pd.T @ Ad @ Pd, rtol=0, atol=1e-13 * np.abs(Ad).max())
    np.testing.assert_array_equal(R.toarray(), Pd.T)


def test_galerkin_every_level_64x64():
    inp = si.generate_workload("g1_2d64")
    A = assemble.assemble(inp).monolithic()
    H = amg.setup(A, amg.AMGParams(seed=1))
    assert len(H.levels) >= 3
    for lo, hi in zip(H.levels[:-1], H.levels[1:]):
        ref = (lo.P.T @ lo.A @ lo.P).tocsr()
        diff = abs(hi.A - ref).max()
        assert diff <= 1e-13 * abs(lo.A).max()


def test_l1_diagonal_closed_form():
    A = _laplace2d(5)
    d = amg.l1_diagonal(A)
    # every off-diagonal is -1: d_i = a_ii + (number of neighbours of i)
    np.testing.assert_array_equal(d, A.diagonal() + (np.diff(A.indptr) - 1))


# --- hierarchy & cycle ------------------------------------------------------------
def test_small_matrix_is_single_direct_level():
    A = _random_mmatrix(80, 3)
    H = amg.setup(A)
    assert len(H.levels) == 1 and H.coarse_kind == "lu"
    b = np.arange(80.0)
    np.testing.assert_allclose(amg.vcycle(H, b), spla.spsolve(sp.csc_matrix(A), b), rtol=1e-12)


def test_max_levels_and_coarse_max():
    inp = si.generate(1, 2, 32, 9)
    A = assemble.assemble(inp).blocks[0]
    H = amg.setup(A, amg.AMGParams(max_levels=2))
    assert len(H.levels) == 2
    H = amg.setup(A, amg.AMGParams())
    assert H.levels[-1].A.shape[0] <= 100 or H.coarse_kind == "jacobi" or len(H.levels) == 25


def _dense_vcycle_error(H, lvl=0):
    """E_l = E_post (I - P V_{l+1} R A) E_pre, V = (I - E) A^{-1}."""
    L = H.levels[lvl]
    A = L.A.toarray()
    n = A.shape[0]
    I = np.eye(n)
    if lvl == len(H.levels) - 1:
        return np.zeros((n, n))       # exact LU on the coarsest level
    Dinv = np.diag(1.0 / L.d)
    IC = np.diag((L.cf == 1).astype(float))
    IF = np.diag((L.cf == -1).astype(float))
    sC = I - IC @ Dinv @ A
    sF = I - IF @ Dinv @ A
    Ac = H.levels[lvl + 1].A.toarray()
    Ec = _dense_vcycle_error(H, lvl + 1)
    Vc = (np.eye(Ac.shape[0]) - Ec) @ np.linalg.inv(Ac)
    P, R = L.P.toarray(), L.R.toarray()
    return (sC @ sF) @ (I - P @ Vc @ R @ A) @ (sF @ sC)


def test_vcycle_equals_error_recursion():
    inp = si.generate(1, 2, 14, 21, nonsym=True)
    A = assemble.assemble(inp).blocks[0]
    H = amg.setup(A, amg.AMGParams(coarse_max=20, seed=4))
    assert len(H.levels) >= 3
    n = A.shape[0]
    V = np.column_stack([amg.vcycle(H, e) for e in np.eye(n)])
    E = np.eye(n) - V @ A.toarray()
    np.testing.assert_allclose(E, _dense_vcycle_error(H), rtol=0, atol=1e-11)


def test_stalled_coarsest_uses_jacobi():
    # strongly diagonally dominant rows: every row cut, no C point -> stall
    n = 3000
    A = sp.csr_matrix(sp.diags([-np.ones(n - 1), 30 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]))
    A.sort_indices()
    H = amg.setup(A, amg.AMGParams())
    assert len(H.levels) == 1 and H.coarse_kind == "jacobi"
    b = np.ones(n)
    x = amg.vcycle(H, b)
    d = amg.l1_diagonal(A)
    x1 = b / d
    x2 = x1 + (b - A @ x1) / d
    np.testing.assert_allclose(x, x2, rtol=1e-15)


def test_solve_to_tolerance_reaches_tolerance():
    inp = si.generate(1, 2, 32, 13)
    A = assemble.assemble(inp).blocks[0]
    H = amg.setup(A)
    b = np.ones(A.shape[0])
    z, k = amg.solve_to_tolerance(H, b, 1e-6)
    assert np.linalg.norm(b - A @ z) < 1e-6 * np.linalg.norm(b)
    z2, k2 = amg.solve_to_tolerance(H, b, 1e-2)
    assert k2 <= k


# --- HMIS ---------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(5))
def test_rs_first_pass_1d_chain_alternates(seed):
    """Ruge-Stueben coarsening of the 1D Poisson chain (textbook result): C and
    F points alternate, whichever interior point the tie-break picks first."""
    n = 17
    A = sp.csr_matrix(sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]))
    A.sort_indices()
    S = amg.strength(A, 0.25, 0.0)
    c = amg.rs_first_pass_tiles(A, S, seed, 0, 1024)
    assert not np.any(c[1:] & c[:-1])          # no two neighbouring C points
    assert not np.any(~c[1:-1] & ~c[2:] & ~c[:-2])  # no interior F run of three
    cf = amg.hmis(A, S, seed, 0, 1024)
    assert np.array_equal(cf == 1, c)           # PMIS has nothing left to decide


@pytest.mark.parametrize("seed", range(4))
def test_hmis_single_row_tiles_is_pmis(seed):
    """With one-row tiles the first pass finds no tile-internal dependency, so
    HMIS reduces to PMIS exactly."""
    A = _random_mmatrix(70, seed)
    S = amg.strength(A, 0.25, 0.9)
    assert np.array_equal(amg.hmis(A, S, seed, 1, tile=1), amg.pmis(A, S, seed, 1))


@pytest.mark.parametrize("seed", range(4))
def test_hmis_splitting_invariants(seed):
    A = _random_mmatrix(90, seed + 10)
    S = amg.strength(A, 0.25, 0.9)
    rows = amg.csr_rows(A)
    cols = A.indices.astype(np.int64)
    stc = amg.strength_transpose_counts(A, S)
    c0 = amg.rs_first_pass_tiles(A, S, seed, 0, 32)
    cf = amg.hmis(A, S, seed, 0, tile=32)
    isC = cf == 1
    assert set(np.unique(cf)) <= {1, -1}
    assert np.all(isC[c0])                      # first-pass C points stay C
    hasC = np.zeros(A.shape[0], dtype=bool)
    hasC[rows[S & isC[cols]]] = True
    assert np.all(hasC[(cf == -1) & (stc > 0)])  # F points interpolate from a C point
    assert np.all(cf[stc == 0] == -1)


def test_hmis_2d_laplacian_one_tile_halves_points():
    """On the 2D 5-point Laplacian one RS first pass over the whole grid gives
    the red-black pattern (every C point's four neighbours are F)."""
    A = _laplace2d(8)
    S = amg.strength(A, 0.25, 0.0)
    cf = amg.hmis(A, S, 2, 0, tile=1024)
    isC = cf == 1
    rows = amg.csr_rows(A)
    cols = A.indices.astype(np.int64)
    off = rows != cols
    assert not np.any(isC[rows[off]] & isC[cols[off]])   # C points independent
    assert abs(int(isC.sum()) - 32) <= 4


# --- multicolour Gauss-Seidel -------------------------------------------------
@pytest.mark.parametrize("seed", range(4))
def test_jp_colouring_is_proper_and_brute_force(seed):
    A = _random_mmatrix(60, seed)
    col = amg.jp_colours(A, seed, 0)
    rows = amg.csr_rows(A)
    cols = A.indices.astype(np.int64)
    off = rows != cols
    assert np.all(col >= 0)
    assert not np.any(col[rows[off]] == col[cols[off]])
    # round rule with Python sets
    n = A.shape[0]
    nb = [set() for _ in range(n)]
    for e in np.nonzero(off)[0]:
        nb[int(rows[e])].add(int(cols[e]))
        nb[int(cols[e])].add(int(rows[e]))
    key = [int(k) for k in amg.hash32(seed, 0, np.arange(n))]
    ref = [-1] * n
    c = 0
    while -1 in ref:
        new = [i for i in range(n) if ref[i] < 0 and
               all((key[i], i) > (key[j], j) for j in nb[i] if ref[j] < 0)]
        for i in new:
            ref[i] = c
        c += 1
    assert np.array_equal(col, np.array(ref))


def test_mc_gs_sweep_is_pointwise_gauss_seidel_in_colour_order():
    """With a proper colouring, one multicolour sweep equals point Gauss-Seidel
    visiting the rows by (colour, index), written as a plain loop."""
    A = _random_mmatrix(50, 3)
    col = amg.jp_colours(A, 7, 0)
    dg = A.diagonal()
    b = np.random.default_rng(1).uniform(size=50)
    x0 = np.random.default_rng(2).uniform(size=50)
    for desc in (False, True):
        x = x0.copy()
        order = sorted(range(50), key=lambda i: (-col[i] if desc else col[i], i))
        for i in order:
            s = sum(A.data[e] * x[A.indices[e]] for e in range(A.indptr[i], A.indptr[i + 1]))
            x[i] = x[i] + (b[i] - s) / dg[i]
        np.testing.assert_allclose(amg.gs_sweep(A, dg, b, x0, col, descending=desc), x,
                                   rtol=1e-13, atol=1e-13)


def test_mc_gs_vcycle_converges_faster_than_jacobi_on_laplacian():
    """Gauss-Seidel smoothing gives a smaller V-cycle error reduction than
    l1-Jacobi on the 2D Laplacian (both below one)."""
    A = sp.csr_matrix(_laplace2d(24) + sp.eye(576) * 1e-3)
    rates = {}
    for sm in ("cf_l1_jacobi", "mc_gs"):
        H = amg.setup(A, amg.AMGParams(seed=3, smoother=sm))
        b = np.zeros(576)
        x = np.random.default_rng(4).uniform(size=576)
        for _ in range(6):
            x = x + amg.vcycle(H, b - A @ x)
        e5 = np.linalg.norm(x)
        x = x + amg.vcycle(H, b - A @ x)
        rates[sm] = np.linalg.norm(x) / e5
    assert rates["mc_gs"] < rates["cf_l1_jacobi"] < 1.0
