"""Pins of the oracle's block system, block preconditioners (Section 3),
GMRES and adjoint against hand-derived fixtures, the paper's exactness
statements and error formulas, closed forms and direct solves."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth_inputs as si
from oracle import adjoint, amg, assemble, krylov, precond

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# --- inputs & assembly -------------------------------------------------------------
def test_generator_deterministic_and_ranges():
    a = si.generate(3, 2, 16, 5)
    b = si.generate(3, 2, 16, 5)
    assert np.array_equal(a.kappa, b.kappa) and np.array_equal(a.b, b.b)
    assert a.kappa.shape == (5, 256) and a.c_gE.shape == (3, 256)
    assert a.c_EI.min() >= 0.1 and a.c_EI.max() <= 10.0
    lk = np.log10(a.kappa[3:])
    assert lk.min() >= -3 and lk.max() <= 3
    lg = np.log10(a.kappa[:3])
    assert lg.min() >= -5 and lg.max() <= 5
    # piecewise constant over 8x8 patches of 2x2 cells
    k = a.kappa[0].reshape(16, 16)
    assert np.all(k[::2, ::2] == k[1::2, 1::2])


def test_assembly_hand_fixture():
    with open(os.path.join(GOLD, "assemble_g1_2x2.json")) as f:
        g = json.load(f)
    inp = si.Inputs(G=1, dim=2, n=2, kappa=np.array(g["kappa"]), c_gE=np.array(g["c_gE"]),
                    c_Eg=np.array(g["c_Eg"]), c_EI=np.array(g["c_EI"]),
                    b=np.ones(12), x_target=np.zeros(12), mass=g["mass"])
    A = assemble.assemble(inp).monolithic().toarray()
    E = np.zeros((12, 12))
    for i, j, v in g["entries"]:
        E[i, j] = v
    np.testing.assert_array_equal(A, E)


@pytest.mark.parametrize("dim,n,G", [(2, 9, 1), (3, 5, 3), (2, 7, 4)])
def test_assembly_row_sums_and_structure(dim, n, G):
    inp = si.generate(G, dim, n, 17)
    sysm = assemble.assemble(inp)
    A = sysm.monolithic()
    np.testing.assert_allclose(A @ np.ones(A.shape[0]), 1.0, rtol=0,
                               atol=1e-12 * abs(A).max())
    for B in sysm.blocks:                     # harmonic means are symmetric
        assert abs(B - B.T).max() == 0.0
    x = np.random.default_rng(0).standard_normal(A.shape[0])
    np.testing.assert_allclose(sysm.matvec(x), A @ x, rtol=1e-14, atol=1e-12)
    np.testing.assert_array_equal(sysm.transpose().monolithic().toarray(), A.T.toarray())
    nnz_block = (2 * dim + 1) * n ** dim - 2 * dim * n ** (dim - 1)
    assert all(B.nnz == nnz_block for B in sysm.blocks)


def test_assembly_nonsym_variant_row_sums():
    inp = si.generate(2, 2, 8, 3, nonsym=True)
    sysm = assemble.assemble(inp)
    A = sysm.monolithic()
    assert abs(sysm.blocks[0] - sysm.blocks[0].T).max() > 0
    np.testing.assert_allclose(A @ np.ones(A.shape[0]), 1.0, atol=1e-12 * abs(A).max())


# --- preconditioners ---------------------------------------------------------------
def _tiny(G, n=6, seed=31):
    inp = si.generate(G, 2, n, seed)
    return inp, assemble.assemble(inp)


def _exact_factory(counters):
    return lambda M, role: precond.exact_inverse(M, counters)


def _dense_inv(M):
    return np.linalg.inv(M.toarray() if sp.issparse(M) else M)


def _exact_schur_preconditioner(sysm, kind):
    """The oracle's Schur1/Schur2 steps driven by exact inverses of the exact
    Schur complements of Section 3.3: C_E, C~_g, A_I (Schur1) or A_E, S~_g,
    S_I (Schur2)."""
    G = sysm.G
    A = [B.toarray() for B in sysm.blocks]
    D = np.diag
    AIi = _dense_inv(A[G + 1])
    AEi = _dense_inv(A[G])
    CE = A[G] - D(sysm.d_EI) @ AIi @ D(sysm.d_IE)
    CEi = _dense_inv(CE)
    if kind == "schur1":
        exact = {"E": CE, "I": A[G + 1]}
        for g in range(G):
            exact[("g", g)] = A[g] - D(sysm.d_gE[g]) @ CEi @ D(sysm.d_Eg[g])
    else:
        exact = {"E": A[G], "I": A[G + 1] - D(sysm.d_IE) @ AEi @ D(sysm.d_EI)}
        for g in range(G):
            exact[("g", g)] = A[g] - D(sysm.d_gE[g]) @ AEi @ D(sysm.d_Eg[g])
    cnt = precond.Counters()

    def factory(M, key):
        Mi = _dense_inv(exact[key])
        return precond.Inverse(M, lambda b: Mi @ b, cnt)
    return precond.BlockPreconditioner(sysm, precond.BlockParams(kind=kind),
                                       inverse_factory=factory)


def test_schur1_exact_for_one_group():
    """Section 3.3: with G = 1 the Schur1 error block set is empty."""
    inp, sysm = _tiny(1)
    Mi = _exact_schur_preconditioner(sysm, "schur1")
    A = sysm.monolithic().toarray()
    MiA = np.column_stack([Mi(c) for c in A.T])
    np.testing.assert_allclose(MiA, np.eye(A.shape[0]), atol=1e-10)
    x, info = krylov.gmres(lambda v: A @ v, Mi, inp.b, rtol=1e-10)
    assert info.iters == 1


@pytest.mark.parametrize("G", [2, 3])
@pytest.mark.parametrize("kind", ["schur1", "schur2"])
def test_schur_error_formulas(kind, G):
    """A - M equals the paper's Err_Schur1 / Err_Schur2 block pattern."""
    inp, sysm = _tiny(G, n=4)
    N = sysm.N
    Mi = _exact_schur_preconditioner(sysm, kind)
    A = sysm.monolithic().toarray()
    n = A.shape[0]
    M = np.linalg.inv(np.column_stack([Mi(e) for e in np.eye(n)]))
    Err = A - M
    Ab = [B.toarray() for B in sysm.blocks]
    if kind == "schur1":
        AIi = np.linalg.inv(Ab[G + 1])
        mid = np.linalg.inv(Ab[G] - np.diag(sysm.d_EI) @ AIi @ np.diag(sysm.d_IE))
        idx = list(range(G))
        dcol = {g: sysm.d_gE[g] for g in range(G)}
        drow = {g: sysm.d_Eg[g] for g in range(G)}
    else:
        mid = np.linalg.inv(Ab[G])
        idx = list(range(G)) + [G + 1]
        dcol = {g: sysm.d_gE[g] for g in range(G)}
        dcol[G + 1] = sysm.d_IE
        drow = {g: sysm.d_Eg[g] for g in range(G)}
        drow[G + 1] = sysm.d_EI
    Exp = np.zeros_like(A)
    for i in idx:
        for j in idx:
            if i != j:
                Exp[i * N:(i + 1) * N, j * N:(j + 1) * N] = -np.diag(dcol[i]) @ mid @ np.diag(drow[j])
    np.testing.assert_allclose(Err, Exp, atol=1e-9 * np.abs(A).max())


@pytest.mark.parametrize("kind,G,inv,mv", [
    ("pctl", 2, 5, 4), ("schur1", 2, 6, 0), ("schur2", 2, 5, 0),
    ("pctl", 3, 6, 5), ("schur1", 3, 7, 0), ("schur2", 3, 6, 0),
    ("bdiag", 3, 5, 0), ("schur2_lower", 3, 5, 0), ("amg", 3, 1, 0)])
def test_table1_operation_counts(kind, G, inv, mv):
    """Table 1: PCTL G+3 inverses and G+2 block matvecs, Schur1 G+4, Schur2 G+3."""
    inp, sysm = _tiny(G)
    M = precond.BlockPreconditioner(sysm, precond.BlockParams(kind=kind))
    c0, m0 = M.counters.inverses, M.counters.matvecs
    M(inp.b)
    assert M.counters.inverses - c0 == inv
    assert M.counters.matvecs - m0 == mv


def test_pctl_coarse_operator_is_galerkin():
    """eq. 3.1 equals P^T A P with P = [diag(p_1); ...; I; diag(p_I)], and
    A_c has A_E's pattern."""
    inp, sysm = _tiny(3)
    M = precond.BlockPreconditioner(sysm, precond.BlockParams(kind="pctl"))
    G, N = sysm.G, sysm.N
    Pb = sp.vstack([sp.diags(M.p[g]) for g in range(G)] + [sp.eye(N), sp.diags(M.pI)])
    A = sysm.monolithic()
    ref = (Pb.T @ A @ Pb).toarray()
    np.testing.assert_allclose(M.Ac.toarray(), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    AE = sysm.blocks[G]
    assert np.array_equal(M.Ac.indptr, AE.indptr) and np.array_equal(M.Ac.indices, AE.indices)


def test_pctl_p_vectors_meet_tolerance():
    """Option #3: ||A_g p_g + D_gE 1|| < tol ||D_gE 1|| (constants interpolated
    to the prescribed accuracy, Section 3.2)."""
    inp, sysm = _tiny(2, n=20)
    tol = 1e-2
    M = precond.BlockPreconditioner(sysm, precond.BlockParams(kind="pctl", pctl_p_tol=tol))
    G = sysm.G
    for g in range(G):
        r = sysm.blocks[g] @ M.p[g] + sysm.d_gE[g]
        assert np.linalg.norm(r) < tol * np.linalg.norm(sysm.d_gE[g])
    r = sysm.blocks[G + 1] @ M.pI + sysm.d_IE
    assert np.linalg.norm(r) < tol * np.linalg.norm(sysm.d_IE)


def test_pctl_operator_with_exact_inverses():
    """PCTL = block lower-triangular relaxation S, then coarse correction:
    M^{-1} = S + P A_c^{-1} P^T (I - A S)."""
    inp, sysm = _tiny(2, n=4)
    cnt = precond.Counters()
    M = precond.BlockPreconditioner(sysm, precond.BlockParams(kind="pctl"),
                                    inverse_factory=_exact_factory(cnt))
    G, N = sysm.G, sysm.N
    A = sysm.monolithic().toarray()
    n = A.shape[0]
    Ab = [B.toarray() for B in sysm.blocks]
    L = np.zeros_like(A)                      # block lower-triangular in E-first order
    for a in range(G + 2):
        L[a * N:(a + 1) * N, a * N:(a + 1) * N] = Ab[a]
    for g in range(G):
        L[g * N:(g + 1) * N, G * N:(G + 1) * N] = np.diag(sysm.d_gE[g])
    L[(G + 1) * N:, G * N:(G + 1) * N] = np.diag(sysm.d_IE)
    S = np.linalg.inv(L)
    P = np.vstack([np.diag(M.p[g]) for g in range(G)] + [np.eye(N), np.diag(M.pI)])
    Ac = P.T @ A @ P
    ref = S + P @ np.linalg.solve(Ac, P.T @ (np.eye(n) - A @ S))
    np.testing.assert_allclose(M.dense_operator(), ref, atol=1e-10)


def test_zero_coupling_reduces_to_block_diagonal():
    """Section 3.5 remark: without couplings every block preconditioner is
    the block-diagonal one."""
    inp = si.generate(2, 2, 10, 41)
    inp.c_gE[:] = 0
    inp.c_Eg[:] = 0
    inp.c_EI[:] = 0
    sysm = assemble.assemble(inp)
    ref = precond.BlockPreconditioner(sysm, precond.BlockParams(kind="bdiag"))(inp.b)
    for kind in ("schur1", "schur2", "schur2_lower"):
        z = precond.BlockPreconditioner(sysm, precond.BlockParams(kind=kind))(inp.b)
        np.testing.assert_array_equal(z, ref)
    cnt = precond.Counters()
    zb = precond.BlockPreconditioner(sysm, precond.BlockParams(kind="bdiag"),
                                     inverse_factory=_exact_factory(cnt))(inp.b)
    zp = precond.BlockPreconditioner(sysm, precond.BlockParams(kind="pctl"),
                                     inverse_factory=_exact_factory(cnt))(inp.b)
    np.testing.assert_allclose(zp, zb, atol=1e-12)


def test_hatted_diagonals_closed_form():
    inp, sysm = _tiny(2)
    G = sysm.G
    mats = precond.hatted(sysm, "schur2")
    dE = sysm.blocks[G].diagonal()
    for g in range(G):
        exp = sysm.blocks[g].diagonal() - sysm.d_gE[g] * sysm.d_Eg[g] / dE
        np.testing.assert_allclose(mats[("g", g)].diagonal(), exp, rtol=1e-15)
        off = (mats[("g", g)] - sysm.blocks[g])
        off.setdiag(0)
        assert abs(off).max() == 0
    m1 = precond.hatted(sysm, "schur1")
    dI = sysm.blocks[G + 1].diagonal()
    dCE = dE - sysm.d_EI * sysm.d_IE / dI
    np.testing.assert_allclose(m1["E"].diagonal(), dCE, rtol=1e-15)
    np.testing.assert_allclose(m1[("g", 0)].diagonal(),
                               sysm.blocks[0].diagonal() - sysm.d_gE[0] * sysm.d_Eg[0] / dCE, rtol=1e-15)


# --- Krylov ------------------------------------------------------------------------
def test_gmres_full_space_converges_in_n_steps():
    rng = np.random.default_rng(3)
    n = 25
    A = rng.standard_normal((n, n)) + n * np.eye(n)
    b = rng.standard_normal(n)
    x, info = krylov.gmres(lambda v: A @ v, None, b, restart=n, rtol=1e-13)
    assert info.converged and info.iters <= n
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-11)
    h = np.array(info.history)
    assert np.all(np.diff(h) <= 1e-15)        # monotone within one cycle


def test_gmres_restarted_matches_direct_and_flexible():
    inp = si.generate_workload("g1_2d64")
    sysm = assemble.assemble(inp)
    A = sysm.monolithic()
    xs = spla.spsolve(sp.csc_matrix(A), inp.b)
    M = precond.BlockPreconditioner(sysm, precond.BlockParams(kind="schur2"))
    x1, i1 = krylov.gmres(A.__matmul__, M, inp.b, rtol=1e-12, flexible=True)
    x2, i2 = krylov.gmres(A.__matmul__, M, inp.b, rtol=1e-12, flexible=False)
    assert i1.converged and i2.converged and abs(i1.iters - i2.iters) <= 1
    cond_est = 1e4
    for x in (x1, x2):
        assert np.linalg.norm(x - xs) <= 1e-12 * cond_est * np.linalg.norm(xs)
        assert np.linalg.norm(inp.b - A @ x) <= 1e-12 * np.linalg.norm(inp.b)


def test_gmres_manufactured_solution():
    inp = si.generate(2, 2, 32, 8)
    sysm = assemble.assemble(inp)
    A = sysm.monolithic()
    n = A.shape[0]
    t = np.linspace(0, 1, n)
    xstar = np.sin(3 * t) + np.random.default_rng(1).uniform(size=n)
    b = A @ xstar
    for kind in ("amg", "schur1"):
        M = precond.BlockPreconditioner(sysm, precond.BlockParams(kind=kind))
        x, info = krylov.gmres(sysm.matvec, M, b, rtol=1e-10)
        assert info.converged
        assert np.linalg.norm(x - xstar) <= 1e-10 * 1e4 * np.linalg.norm(xstar)


def test_gmres_edge_cases():
    A = np.diag([1.0, 2.0, 3.0])
    x, info = krylov.gmres(lambda v: A @ v, None, np.zeros(3))
    assert info.converged and info.iters == 0 and np.all(x == 0)
    x, info = krylov.gmres(lambda v: A @ v, None, np.ones(3), max_iters=1, rtol=1e-14)
    assert not info.converged and info.iters == 1
    x0 = np.array([1.0, 0.5, 1.0 / 3.0])
    x, info = krylov.gmres(lambda v: A @ v, None, np.ones(3), x0=x0)
    assert info.converged and info.iters == 0


# --- adjoint -----------------------------------------------------------------------
def test_adjoint_matches_direct_transpose_solve():
    inp = si.generate_workload("g2_2d16")
    sysm = assemble.assemble(inp)
    A = sysm.monolithic()
    x = spla.spsolve(sp.csc_matrix(A), inp.b)
    g = x - inp.x_target
    lam, grads, info = adjoint.adjoint_solve(inp, sysm, x, g,
                                             precond.BlockParams(kind="schur2"), rtol=1e-13)
    lam_d, grads_d = adjoint.adjoint_direct(inp, sysm, x, g)
    assert info.converged
    np.testing.assert_allclose(lam, lam_d, rtol=0, atol=1e-10 * np.abs(lam_d).max())
    for a, b_ in zip(grads, grads_d):
        np.testing.assert_allclose(a, b_, rtol=0, atol=1e-9 * np.abs(b_).max())


def _solve(inp):
    A = assemble.assemble(inp).monolithic()
    return spla.splu(sp.csc_matrix(A)).solve(inp.b)


def test_adjoint_gradients_central_differences():
    """Section 2 system, G = 2 on 16 x 16: gradients vs central differences
    (relative step 1e-6, direct forward solves), relative error < 1e-5.
    L(+h) - L(-h) is evaluated as 0.5 sum (x+ - x-)(x+ + x- - 2 t), which is
    the same number with far less cancellation."""
    inp = si.generate_workload("g2_2d16")
    x = _solve(inp)
    sysm = assemble.assemble(inp)
    lam, (dk, dgE, dEg, dEI) = adjoint.adjoint_direct(inp, sysm, x, x - inp.x_target)
    rng = np.random.default_rng(0)
    N = inp.N
    t = inp.x_target

    def fd(field, idx):
        arr = getattr(inp, field)
        old = arr[idx]
        h = 1e-6 * abs(old)
        arr[idx] = old + h
        xp = _solve(inp)
        arr[idx] = old - h
        xm = _solve(inp)
        arr[idx] = old
        return 0.5 * np.sum((xp - xm) * (xp + xm - 2 * t)) / (2 * h)

    def pick(grad, shape):
        cand = [tuple(int(rng.integers(0, s)) for s in shape) for _ in range(64)]
        cand.sort(key=lambda c: -abs(grad[c]))
        return cand[:3]

    checks = []
    for c in pick(dk, dk.shape):
        checks.append((dk[c], fd("kappa", c)))
    for c in pick(dgE, dgE.shape):
        checks.append((dgE[c], fd("c_gE", c)))
    for c in pick(dEg, dEg.shape):
        checks.append((dEg[c], fd("c_Eg", c)))
    for c in pick(dEI, dEI.shape):
        checks.append((dEI[c], fd("c_EI", c[0])))
    for c in pick(lam, lam.shape):
        checks.append((lam[c], fd("b", c[0])))
    for an, num in checks:
        assert abs(an - num) <= 1e-5 * abs(num), (an, num)
