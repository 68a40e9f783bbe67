"""Pins of the adaptive strategy (Section 3.5, Definitions 1-2, options #1/#2
of Section 3.4) in the oracle, on the CPU.

What pins it, independent of the oracle's own formulas:
  * the two indicators on hand-counted cases (strict vs non-strict
    comparisons, the sign of d, the diagonal of the row block);
  * Jacobi iterations against hand arithmetic and the textbook contraction
    bound for strongly diagonally dominant rows;
  * exactness: with exact inner inverses every structural case (couplings to
    E neglected, couplings into E's row neglected, all neglected) must give
    M = A~ exactly, A~ the system with the neglected couplings removed,
    because the Schur error terms of Section 3.3 then vanish; with all
    couplings neglected every kind is the block-diagonal inverse;
  * the merged E inverse equals the paper's two-inverse form by linearity;
  * the inverse counts per apply of each structural case.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synth_inputs as si
from oracle import adaptive as adp
from oracle import assemble, precond


def _sys(G=3, n=6, seed=41, **kw):
    inp = si.generate(G, 2, n, seed, **kw)
    return inp, assemble.assemble(inp)


def _exact(counters):
    return lambda M, role: precond.exact_inverse(M, counters)


def _dense_operator(M, n):
    return np.column_stack([M(e) for e in np.eye(n)])


# --- Definition 1 and 2 on hand-counted cases ---------------------------------
def test_weak_coupling_count_by_hand():
    # -d <= 0.01 a: 0.001 <= 0.01 yes; 0.5 no; 0.02 no; 0.01 <= 0.01 yes (not strict)
    d = np.array([-0.001, -0.5, -0.02, -0.01])
    a = np.array([1.0, 1.0, 1.0, 1.0])
    assert adp.weak_coupling_count(d, a, 1e-2) == 2
    # relative to the row block's diagonal: a = 100 makes -d = 0.5 weak
    assert adp.weak_coupling_count(d, np.array([1.0, 100.0, 1.0, 1.0]), 1e-2) == 3
    # Definition 1 needs more than sigma N rows (strict)
    assert not adp.is_weak(2, 4, 0.5) and adp.is_weak(3, 4, 0.5)


def test_weak_dominance_count_by_hand():
    # row 0: sum 1.0 < 0.9 * 4 counts; row 1: sum 0.9 < 0.9 * 1 is false
    # (strict); row 2: sum 9.5 >= 0.9 * 10, strongly dominant
    M = sp.csr_matrix(np.array([[4.0, -3.0, 0.0],
                                [-0.1, 1.0, 0.0],
                                [0.0, -0.5, 10.0]]))
    assert adp.weak_dominance_count(M, 0.9) == 1
    assert adp.weak_dominance_count(sp.identity(5, format="csr"), 0.9) == 0


# --- option #1 -----------------------------------------------------------------
def test_jacobi_by_hand_and_diagonal_exactness():
    M = sp.csr_matrix(np.array([[4.0, -1.0], [-2.0, 5.0]]))
    b = np.array([1.0, 2.0])
    # sweep 1: b / d = (0.25, 0.4); sweep 2: r = (0.4, 0.5), w += r / d
    np.testing.assert_allclose(adp.jacobi(M, b, 1), [0.25, 0.4], rtol=0, atol=1e-15)
    np.testing.assert_allclose(adp.jacobi(M, b, 2), [0.35, 0.5], rtol=0, atol=1e-15)
    D = sp.diags([2.0, 4.0, 8.0], format="csr")
    np.testing.assert_array_equal(adp.jacobi(D, np.array([1.0, 1.0, 1.0]), 1), [0.5, 0.25, 0.125])


def test_jacobi_contraction_on_strongly_dominant_block():
    """Rows with sum >= 0.9 a_kk of an M-matrix have off-diagonal mass <= 0.1
    a_kk, so k Jacobi sweeps from zero leave an error <= 0.1^k ||x||_inf."""
    inp, sysm = _sys(G=2, n=8, log_kappa_shift=(0.0, 0.0, -8.0))
    AI = sysm.blocks[3]
    assert adp.weak_dominance_count(AI, 0.9) == 0
    x = np.linalg.solve(AI.toarray(), inp.b[:sysm.N])
    for k in (1, 2, 3):
        err = np.abs(adp.jacobi(AI, inp.b[:sysm.N], k) - x).max()
        assert err <= 0.1 ** k * np.abs(x).max() * (1 + 1e-12)


# --- Definition 1 on generated systems --------------------------------------------
def test_plan_follows_coupling_scale():
    _, s0 = _sys()
    p0 = adp.coupling_plan(s0)
    assert not p0.gE.any() and not p0.Eg.any() and not p0.EI
    _, s1 = _sys(c_scale=(1e-6, 1.0, 1.0))
    p1 = adp.coupling_plan(s1)
    assert p1.gE.all() and not p1.Eg.any() and not p1.EI
    assert np.array_equal(p1.counts["gE"], np.full(3, s1.N))
    A1 = adp.drop_weak(s1, p1)
    assert np.all(A1.d_gE == 0.0) and np.array_equal(A1.d_Eg, s1.d_Eg)


# --- exactness of the structural cases ------------------------------------------------
def _modified_dense(sysm, plan):
    return adp.drop_weak(sysm, plan).monolithic().toarray()


CASES = {
    # every row block's coupling to E neglected (D_gE, D_IE): a large kappa_I
    # makes D_IE weak against A_I's diagonal
    "from_E": dict(c_scale=(1e-6, 1.0, 1.0), log_kappa_shift=(0.0, 0.0, 6.0)),
    # every coupling in E's row neglected (D_Eg, D_EI): a large kappa_E
    "into_E": dict(log_kappa_shift=(0.0, 6.0, 0.0)),
    "all": dict(c_scale=(1e-6, 1e-6, 1e-6)),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("kind", ["schur1", "schur2", "pctl"])
def test_adaptive_exact_inverses_give_modified_system(kind, case):
    inp, sysm = _sys(**CASES[case])
    plan = adp.coupling_plan(sysm)
    if case == "from_E":
        assert plan.all_from_E_weak and not plan.all_into_E_rows_weak
    elif case == "into_E":
        assert plan.all_into_E_rows_weak and not plan.IE
    else:
        assert plan.all_from_E_weak and plan.all_into_E_rows_weak
    cnt = precond.Counters()
    M = precond.BlockPreconditioner(sysm, precond.BlockParams(kind=kind, adaptive=True),
                                    inverse_factory=_exact(cnt))
    assert not M.jacobi_roles
    if kind == "pctl" and case == "from_E":
        pytest.skip("PCTL keeps its coarse correction when E's row is coupled")
    At = _modified_dense(sysm, plan)
    Mi = _dense_operator(M, sysm.n)
    Ai = np.linalg.inv(At)
    assert np.linalg.norm(Mi - Ai) <= 1e-10 * np.linalg.norm(Ai)
    if case == "all":
        Bd = np.zeros_like(At)
        for a in range(sysm.G + 2):
            sl = slice(a * sysm.N, (a + 1) * sysm.N)
            Bd[sl, sl] = sysm.blocks[a].toarray()
        np.testing.assert_allclose(Mi, np.linalg.inv(Bd), atol=1e-12)


@pytest.mark.parametrize("kind,case,count", [
    ("schur2", "from_E", "G+2"), ("schur2", "into_E", "G+2"), ("schur2", "all", "G+2"),
    ("schur1", "from_E", "G+2"), ("schur1", "into_E", "G+3"), ("schur1", "all", "G+2"),
    ("pctl", "into_E", "G+2"), ("pctl", "all", "G+2")])
def test_adaptive_inverse_counts(kind, case, count):
    inp, sysm = _sys(**CASES[case])
    cnt = precond.Counters()
    M = precond.BlockPreconditioner(sysm, precond.BlockParams(kind=kind, adaptive=True),
                                    inverse_factory=_exact(cnt))
    M(inp.b)
    assert cnt.inverses == eval(count, {"G": sysm.G})   # exact inverses count here
    assert M.counters.matvecs == 0


def test_merged_E_inverse_equals_two_inverse_form():
    """Schur2 with every coupling to E neglected applies one A_E inverse after
    the independent solves; the paper's three steps on the modified system
    give the same vector because the V-cycle is a linear operator."""
    inp, sysm = _sys(**CASES["from_E"])
    M = precond.BlockPreconditioner(sysm, precond.BlockParams(kind="schur2", adaptive=True))
    G, N = sysm.G, sysm.N
    At = M.sys
    B = inp.b.reshape(G + 2, N)
    wE = M.inv["E"](B[G])
    W = np.empty_like(B)
    for g in range(G):
        W[g] = M.inv[("g", g)](B[g] - At.d_gE[g] * wE)
    W[G + 1] = M.inv["I"](B[G + 1] - At.d_IE * wE)
    s = np.zeros(N)
    for g in range(G):
        s = s + At.d_Eg[g] * W[g]
    s = s + At.d_EI * W[G + 1]
    W[G] = wE - M.inv["E"](s)
    got = M(inp.b)
    assert np.linalg.norm(got - W.reshape(-1)) <= 1e-12 * np.linalg.norm(got)


def test_option1_selected_for_strongly_dominant_block():
    inp, sysm = _sys(G=2, n=8, log_kappa_shift=(0.0, 0.0, -8.0))
    M = precond.BlockPreconditioner(sysm, precond.BlockParams(kind="schur2", adaptive=True))
    assert M.jacobi_roles == {"I"}
    assert M.setup_info["wd_counts"]["I"] == 0
    assert all(M.setup_info["wd_counts"][("g", g)] > 0 for g in range(2))
    r = inp.b[3 * sysm.N:]
    np.testing.assert_array_equal(M.inv["I"](r), adp.jacobi(M.mats["I"], r, 2))


def test_adaptive_rejects_other_kinds():
    _, sysm = _sys()
    with pytest.raises(ValueError):
        precond.BlockPreconditioner(sysm, precond.BlockParams(kind="bdiag", adaptive=True))
