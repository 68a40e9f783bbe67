"""Pins of the inner solves to a tolerance (option #3 of Section 3.4 used for
the inverses Section 4 names) in the oracle, on the CPU.

  * every inverse named by Section 4 stops at the first V-cycle that brings
    its residual below inner_tol ||b|| (one cycle fewer does not);
  * the other inverses keep exactly one V-cycle;
  * with a tiny tolerance the inner solves reach the exact inverse of their
    matrix (scipy's direct solve);
  * a zero right-hand side takes no cycle;
  * FGMRES converges with the resulting nonlinear preconditioner.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth_inputs as si
from oracle import amg, assemble, krylov, precond


def _setup(kind, tol, G=3, n=10, seed=71):
    inp = si.generate(G, 2, n, seed)
    sysm = assemble.assemble(inp)
    M = precond.BlockPreconditioner(sysm, precond.BlockParams(
        kind=kind, inner_tol=tol, amg=amg.AMGParams(seed=3)))
    return inp, sysm, M


EXPECTED_ROLES = {
    "schur1": lambda G: {("g", g) for g in range(G)} | {"E"},
    "schur2": lambda G: {("g", g) for g in range(G)} | {"I"},
    "pctl": lambda G: {("g", g) for g in range(G)} | {"E", "I"},
}


@pytest.mark.parametrize("kind", ["schur1", "schur2", "pctl"])
def test_tolerance_roles_follow_section4(kind):
    _, sysm, M = _setup(kind, 1e-2)
    assert M.tolerance_roles() == EXPECTED_ROLES[kind](sysm.G)


@pytest.mark.parametrize("kind", ["schur1", "schur2", "pctl"])
def test_inner_solves_stop_at_first_cycle_below_tolerance(kind):
    inp, sysm, M = _setup(kind, 1e-2)
    rng = np.random.default_rng(2)
    for key in M.tolerance_roles():
        inv = M.inv[key]
        b = rng.standard_normal(sysm.N)
        z = inv(b)
        k = inv.last_cycles
        assert k >= 1
        assert np.linalg.norm(b - inv.M @ z) < 1e-2 * np.linalg.norm(b)
        if k > 1:
            zp, kp = amg.solve_to_tolerance(inv.hierarchy, b, 1e-2, k - 1)
            assert kp == k - 1
            assert np.linalg.norm(b - inv.M @ zp) >= 1e-2 * np.linalg.norm(b)
        zero, k0 = amg.solve_to_tolerance(inv.hierarchy, np.zeros(sysm.N), 1e-2)
        assert k0 == 0 and not zero.any()


@pytest.mark.parametrize("kind", ["schur1", "schur2", "pctl"])
def test_other_inverses_keep_one_cycle(kind):
    inp, sysm, M = _setup(kind, 1e-2)
    b = np.random.default_rng(3).standard_normal(sysm.N)
    for key, inv in M.inv.items():
        if key in M.tolerance_roles():
            continue
        np.testing.assert_array_equal(inv(b), amg.apply_cycles(inv.hierarchy, b, 1))


def test_tiny_tolerance_reaches_exact_inverse():
    inp, sysm, M = _setup("schur2", 1e-11)
    b = np.random.default_rng(4).standard_normal(sysm.N)
    for key in M.tolerance_roles():
        inv = M.inv[key]
        x = spla.spsolve(inv.M.tocsc(), b)
        assert np.linalg.norm(inv(b) - x) <= 1e-8 * np.linalg.norm(x)


@pytest.mark.parametrize("kind", ["schur1", "schur2", "pctl"])
def test_fgmres_with_inner_tolerance(kind):
    inp, sysm, M = _setup(kind, 1e-2, n=16)
    x, info = krylov.gmres(sysm.matvec, M, inp.b, rtol=1e-8, flexible=True)
    assert info.converged
    assert np.linalg.norm(inp.b - sysm.matvec(x)) <= 1e-8 * np.linalg.norm(inp.b) * (1 + 1e-9)


# --- option #4: the exact Schur complement inverse by fixed-point steps ----------
def _exact_blocks_factory():
    cnt = precond.Counters()
    return lambda M, role: precond.exact_inverse(M, cnt)


@pytest.mark.parametrize("kind,key", [("schur2", "I"), ("schur1", "E")])
def test_option4_converges_to_exact_schur_complement(kind, key):
    """With exact block inverses the steps are a fixed-point iteration with
    iteration matrix T = A_a^{-1} D_ab A_b^{-1} D_ba >= 0; for these M-matrix
    blocks ||T||_inf < 1, so the error to S^{-1} q (S = A_a - D_ab A_b^{-1}
    D_ba) falls monotonically in the max norm, and 1 step is A_a^{-1} q."""
    inp = si.generate(3, 2, 8, 81)
    sysm = assemble.assemble(inp)
    G, N = sysm.G, sysm.N
    A = {"E": sysm.blocks[G].toarray(), "I": sysm.blocks[G + 1].toarray()}
    D = {("I", "E"): np.diag(sysm.d_IE), ("E", "I"): np.diag(sysm.d_EI)}
    other = "E" if key == "I" else "I"
    S = A[key] - D[(key, other)] @ np.linalg.solve(A[other], D[(other, key)])
    q = np.random.default_rng(5).standard_normal(N)
    x = np.linalg.solve(S, q)
    errs = []
    for k in (1, 2, 3, 5, 8, 40):
        M = precond.BlockPreconditioner(sysm, precond.BlockParams(kind=kind, option4_steps=k),
                                        inverse_factory=_exact_blocks_factory())
        w = M.inv[key + "4"](q)
        if k == 1:
            np.testing.assert_allclose(w, np.linalg.solve(A[key], q), rtol=1e-12, atol=0)
        errs.append(np.abs(w - x).max())
    assert all(b <= a * (1 + 1e-12) for a, b in zip(errs, errs[1:]))
    assert errs[-1] <= 1e-10 * np.abs(x).max()


def test_option4_uses_original_blocks_and_counts_inverses():
    inp = si.generate(3, 2, 8, 82)
    sysm = assemble.assemble(inp)
    M = precond.BlockPreconditioner(sysm, precond.BlockParams(kind="schur2", option4_steps=3,
                                                              amg=amg.AMGParams(seed=3)))
    assert (M.mats["I"] != sysm.blocks[sysm.G + 1]).nnz == 0
    c0 = M.counters.inverses
    M(inp.b)
    # Schur2: A_E twice, G groups, S_I by 3 steps = 3 A_I + 2 A_E
    assert M.counters.inverses - c0 == 2 + sysm.G + 3 + 2
    x, info = krylov.gmres(sysm.matvec, M, inp.b, rtol=1e-8)
    assert info.converged
    with pytest.raises(ValueError):
        precond.BlockPreconditioner(sysm, precond.BlockParams(kind="pctl", option4_steps=2))
