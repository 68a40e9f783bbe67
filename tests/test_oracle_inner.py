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
