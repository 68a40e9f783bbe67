"""GPU parity on the full-size workloads (2D 1024^2 G=1, 2D 256^2 G=20,
3D 64^3 G=20, 2D 512^2 G=20) against the oracle.

The oracle runs the whole method at these sizes on the host in minutes
(3D 64^3, G=20, Schur2: about 50 s of setup and 75 s of FGMRES); its results
are stored in tests/golden/fullsize_<workload>.{json,npz} by
tests/golden/make_fullsize.py, which calls only the oracle.  Compared here:
  * every AMG hierarchy of every inverse role, level by level, bit for bit
    (level sizes, entry counts, PMIS rounds, digests of C/F, A_l and P_l);
    PCTL's coarse matrix A_c depends on V-cycle results and is compared in
    structure, with its p-vector cycle counts equal;
  * FGMRES(30) to rtol 1e-8 (Section 4, stop test of reading A1): the FP64
    iteration count within +-1 of the oracle's; after exactly the oracle's
    iteration count, the solution element by element at the stored sample
    positions (to 1e-10 relative, with a floor of 1e-3 of the block
    segment's largest entry) and every block segment's 2-norm (to 1e-10);
  * the FP32-hierarchy batched form that the benchmark times: its true
    residual through the oracle's matvec and its error against the oracle's
    solution;
plus checks evaluated with the oracle's own arithmetic on the full vectors
(bit-exact assembly, true residuals, batched against sequential applies,
one V-cycle of A_E, the adjoint's gradient formulas).
"""
import json

import numpy as np
import pytest

import synth_inputs as si
from oracle import adjoint as oadj
from oracle import amg as oamg
from oracle import assemble as oasm
from oracle import precond as opc

from gpu_helpers import (assert_elementwise, gpu_modules, gpu_system, rel, to_dev, to_host)

import os
import sys
sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import fullsize_format as ff  # noqa: E402

pytestmark = pytest.mark.gpu

SOLUTION_TOL = 1e-10      # FP64, same iteration count as the oracle
SOLUTION_FLOOR = 1e-3
FP32_SOLUTION_TOL = 1e-6  # FP32 V-cycles inside FP64 FGMRES, both to rtol 1e-8


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    api = gpu_modules()
    c = api.Context(0)
    yield c
    _CACHE.clear()
    c.synchronize()


_CACHE = {}


def workload(ctx, name):
    """(inputs, oracle system, GPU coefficients, GPU system), built once; the
    previous workload is released first."""
    if name not in _CACHE:
        _CACHE.clear()
        inp = si.generate_workload(name)
        osys = oasm.assemble(inp)
        co, gsys = gpu_system(ctx, inp)
        _CACHE[name] = (inp, osys, co, gsys)
    return _CACHE[name]


def golden(name):
    jpath, npath = ff.paths(name)
    with open(jpath) as f:
        meta = json.load(f)
    with np.load(npath) as z:
        arrays = {k: z[k] for k in z.files}
    return meta, arrays


def true_relres(osys, x, b):
    return np.linalg.norm(b - osys.matvec(x)) / np.linalg.norm(b)


def assert_assembly_equal(gsys, osys):
    for a in range(osys.G + 2):
        rp, ci, v = gsys.block_arrays(a)
        B = osys.blocks[a]
        assert np.array_equal(rp, B.indptr) and np.array_equal(ci, B.indices), a
        assert np.array_equal(v, B.data), a
    dgE, dEg, dEI, dIE = gsys.couplings()
    assert np.array_equal(dgE, osys.d_gE.reshape(-1)) and np.array_equal(dEg, osys.d_Eg.reshape(-1))
    assert np.array_equal(dEI, osys.d_EI) and np.array_equal(dIE, osys.d_IE)


def role_index(role, G):
    if role == "mono":
        return 0
    if role.startswith("g"):
        return int(role[1:])
    return {"E": G, "I": G + 1, "c": G + 2}[role]


def assert_hierarchy_matches(gh, rec, label, values=True):
    """Level sizes, entry counts, PMIS rounds and C/F splittings always; the
    digests of A_l and P_l (values included) when `values`."""
    info = gh.info()
    levels = rec["levels"]
    assert info["levels"] == len(levels), (label, info["n"], [L["n"] for L in levels])
    assert info["coarse_kind"] == {"lu": 0, "jacobi": 1}[rec["coarse_kind"]], label
    for l, L in enumerate(levels):
        assert info["n"][l] == L["n"] and info["nnz"][l] == L["nnz"], (label, l)
        e = gh.export_level(l)
        if values:
            assert ff.digest_csr(*e["A"]) == L["A"], (label, l, "A")
        if "cf" in L:
            assert info["nnz_P"][l] == L["nnz_P"], (label, l)
            assert info["pmis_rounds"][l] == L["rounds"], (label, l)
            assert ff.digest_cf(e["cf"]) == L["cf"], (label, l, "cf")
            if values:
                assert ff.digest_csr(*e["P"]) == L["P"], (label, l, "P")


def assert_precond_hierarchies(M, case, G, info=None):
    roles = [r for r in case["hierarchies"] if r != "pctl_p_cycles"]
    assert roles
    for role in roles:
        # PCTL's A_c (eq. 3.1) is formed from p-vectors that V-cycles compute
        # to a tolerance, so its values equal the oracle's to rounding only:
        # its hierarchy is compared in structure (the p-cycle counts below are
        # integers and must be equal)
        assert_hierarchy_matches(M.hierarchy(role_index(role, G)), case["hierarchies"][role], role,
                                 values=(role != "c"))
    if "pctl_p_cycles" in case["hierarchies"]:
        assert (info or M.info())["pctl_p_cycles"] == case["hierarchies"]["pctl_p_cycles"]


def assert_solution_matches(x, case, arrays, key, G, N, tol, floor, what):
    """x (full GPU vector, host) against the oracle's at the sample positions,
    entry by entry with the floor taken from the oracle's full segment max,
    and the per-segment 2-norms."""
    pos = arrays["pos"]
    ref = arrays[key]
    seg_inf = np.asarray(case["x_norminf"])[pos // N]
    scale = np.maximum(np.abs(ref), floor * seg_inf)
    assert_elementwise(x[pos], ref, tol, scale=scale, what=what)
    n2 = np.linalg.norm(x.reshape(G + 2, N), axis=1)
    assert_elementwise(n2, np.asarray(case["x_norm2"]), tol, floor=1.0, what=what + " segment norms")


def fp64_solve_checks(ctx, name, kind, seed, batched, graph, rhs=None, case_key=None):
    """FP64 iteration count against the oracle's (+-1), then the solution after
    exactly the oracle's count.  Returns the same-iteration solution."""
    api = gpu_modules()
    inp, osys, co, gsys = workload(ctx, name)
    meta, arrays = golden(name)
    key = case_key or kind
    case = meta["cases"][key]
    G, N = inp.G, inp.N
    transpose = key.startswith("adjoint_")
    M = api.BlockPreconditioner(ctx, gsys, kind, amg_seed=seed, amg_precision=0,
                                batched=int(batched), use_graph=int(graph),
                                transpose=int(transpose))
    assert_precond_hierarchies(M, case, G)
    b = to_dev(ctx, inp.b if rhs is None else rhs)
    if transpose:
        solve = lambda **kw: api.adjoint(ctx, co, gsys, M, to_dev(ctx, np.zeros(osys.n)), b,  # noqa: E731
                                         flexible=1, **kw)
        lam, dk, dc, r = solve(rtol=1e-8)
    else:
        x, r = api.gmres(ctx, gsys, M, b, rtol=1e-8, flexible=1)
    want = case["gmres"]["iters"]
    assert r.converged and abs(r.iters - want) <= 1, (key, r.iters, want)
    if transpose:
        lam, dk, dc, r2 = solve(rtol=0.0, max_iters=want)
        x2 = lam
    else:
        x2, r2 = api.gmres(ctx, gsys, M, b, rtol=0.0, max_iters=want, flexible=1)
    assert r2.iters == want
    xh = to_host(x2)
    assert_solution_matches(xh, case, arrays, f"{key}/x", G, N, SOLUTION_TOL, SOLUTION_FLOOR,
                            f"{name} {key} batched={batched} same-iteration solution")
    return xh, M


# ---------------------------------------------------------------------------
# G=20, 3D 64^3 7-point (5,767,168 unknowns): the benchmark configuration
# ---------------------------------------------------------------------------
def test_g20_3d64_assembly_bit_exact(ctx):
    inp, osys, co, gsys = workload(ctx, "g20_3d64")
    assert_assembly_equal(gsys, osys)


def test_g20_3d64_schur2_fp64_plain_against_oracle(ctx):
    """All 22 hierarchies (S^_g, A_E, S^_I) bit for bit; FGMRES iteration count
    +-1 of the oracle's 38; the solution after 38 iterations to 1e-10."""
    fp64_solve_checks(ctx, "g20_3d64", "schur2", 4, batched=False, graph=False)


def test_g20_3d64_schur2_fp64_batched_graph_against_oracle(ctx):
    fp64_solve_checks(ctx, "g20_3d64", "schur2", 4, batched=True, graph=True)


@pytest.mark.parametrize("kind", ["schur1", "pctl"])
def test_g20_3d64_other_kinds_against_oracle(ctx, kind):
    """Schur1 (eq. 3.2, with C^_E, C^_g) and PCTL (Section 3.2, eq. 3.1) at the
    headline size: hierarchies as the oracle's (PCTL's A_c in structure, with
    equal p-vector cycle counts), the FGMRES iteration count +-1 of the
    oracle's, the same-iteration solution to 1e-10."""
    fp64_solve_checks(ctx, "g20_3d64", kind, 4, batched=True, graph=True)


@pytest.mark.parametrize("autotune", [0, 1])
def test_g20_3d64_schur2_fp32_batched_against_oracle(ctx, autotune):
    """The benchmark's form (FP32 hierarchies, batched, graph-replayed, FP64
    FGMRES; with autotune = 1 the level layouts it times at setup, as the
    benchmark builds them): the hierarchies are the oracle's (the setup is
    FP64), the iteration count is within +-2 of the oracle's, the true FP64
    residual meets 1e-8, and the solution agrees with the oracle's to 1e-6 of
    each block segment's largest entry."""
    api = gpu_modules()
    inp, osys, co, gsys = workload(ctx, "g20_3d64")
    meta, arrays = golden("g20_3d64")
    case = meta["cases"]["schur2"]
    M = api.BlockPreconditioner(ctx, gsys, "schur2", amg_seed=4, amg_precision=1, batched=1,
                                use_graph=1, amg_autotune=autotune)
    assert_precond_hierarchies(M, case, inp.G)
    x, r = api.gmres(ctx, gsys, M, to_dev(ctx, inp.b), rtol=1e-8, flexible=1)
    assert r.converged and abs(r.iters - case["gmres"]["iters"]) <= 2, r.iters
    xh = to_host(x)
    assert true_relres(osys, xh, inp.b) <= 1e-8 * (1 + 1e-6)
    assert_solution_matches(xh, case, arrays, "schur2/x", inp.G, inp.N, FP32_SOLUTION_TOL, 1.0,
                            "FP32 batched solution against the oracle")


@pytest.mark.parametrize("kind", ["schur1", "pctl"])
def test_g20_3d64_fp32_batched_other_kinds_against_oracle(ctx, kind):
    """Schur1 and PCTL in the benchmark's form (FP32 hierarchies, batched,
    graph-replayed, FP64 FGMRES): the iteration count within +-2 of the
    oracle's, the true FP64 residual meets 1e-8, the solution agrees with
    the oracle's to 1e-6 of each block segment's largest entry."""
    api = gpu_modules()
    inp, osys, co, gsys = workload(ctx, "g20_3d64")
    meta, arrays = golden("g20_3d64")
    case = meta["cases"][kind]
    M = api.BlockPreconditioner(ctx, gsys, kind, amg_seed=4, amg_precision=1, batched=1,
                                use_graph=1)
    x, r = api.gmres(ctx, gsys, M, to_dev(ctx, inp.b), rtol=1e-8, flexible=1)
    assert r.converged and abs(r.iters - case["gmres"]["iters"]) <= 2, (kind, r.iters)
    xh = to_host(x)
    assert true_relres(osys, xh, inp.b) <= 1e-8 * (1 + 1e-6)
    assert_solution_matches(xh, case, arrays, f"{kind}/x", inp.G, inp.N, FP32_SOLUTION_TOL, 1.0,
                            f"FP32 batched {kind} solution against the oracle")


@pytest.mark.parametrize("aggressive", [0, 1])
def test_g20_3d64_E_block_hierarchy_and_vcycle(ctx, aggressive):
    """The whole AMG hierarchy of A_E (262,144 rows) equals the oracle's bit for
    bit, also with aggressive coarsening and multipass interpolation on the
    finest level, and one FP64 V-cycle agrees element by element to 1e-12."""
    api = gpu_modules()
    inp, osys, co, gsys = workload(ctx, "g20_3d64")
    A = osys.blocks[inp.G]
    H = oamg.setup(A, oamg.AMGParams(seed=4, aggressive_levels=aggressive))
    g = api.AMG(ctx, A.indptr, A.indices, A.data, seed=4, aggressive_levels=aggressive)
    info = g.info()
    assert info["levels"] == len(H.levels)
    for l, L in enumerate(H.levels):
        e = g.export_level(l)
        rp, ci, v = e["A"]
        assert np.array_equal(rp, L.A.indptr) and np.array_equal(ci, L.A.indices), l
        assert np.array_equal(v, L.A.data), l
        if L.cf is not None:
            assert np.array_equal(e["cf"], L.cf), l
            prp, pci, pv = e["P"]
            assert np.array_equal(prp, L.P.indptr) and np.array_equal(pci, L.P.indices), l
            assert np.array_equal(pv, L.P.data), l
    bvec = np.random.default_rng(8).uniform(size=A.shape[0])
    assert_elementwise(to_host(g.apply(to_dev(ctx, bvec))), oamg.vcycle(H, bvec), 1e-12,
                       what="A_E V-cycle")


def test_g20_3d64_adaptive_schur2(ctx):
    """alpha-Schur2 (Section 3.5) at the benchmark size: the Definition 1 and 2
    counts and decisions equal the oracle's (integers), and the FP32 batched
    solve meets rtol 1e-8 against the full system."""
    api = gpu_modules()
    inp, osys, co, gsys = workload(ctx, "g20_3d64")
    plan, _, _, wd = opc.adaptive_decisions(osys, "schur2", opc.BlockParams(adaptive=True))
    M = api.BlockPreconditioner(ctx, gsys, "schur2", amg_seed=4, amg_precision=1, batched=1,
                                use_graph=1, adaptive=1)
    info = M.info()
    G = inp.G
    assert info["wc_counts"]["gE"] == [int(v) for v in plan.counts["gE"]]
    assert info["wc_counts"]["Eg"] == [int(v) for v in plan.counts["Eg"]]
    assert info["wc_counts"]["EI"] == int(plan.counts["EI"][0])
    assert info["wc_counts"]["IE"] == int(plan.counts["IE"][0])
    assert info["weak"]["gE"] == [bool(v) for v in plan.gE]
    keys = [("g", g) for g in range(G)] + ["E", "I"]
    assert info["wd_count"] == [wd[k] for k in keys]
    assert info["jacobi"] == [wd[k] == 0 for k in keys]
    b = to_dev(ctx, inp.b)
    x, r = api.gmres(ctx, gsys, M, b, rtol=1e-8, flexible=1)
    assert r.converged
    assert true_relres(osys, to_host(x), inp.b) <= 1e-8 * (1 + 1e-6)


# ---------------------------------------------------------------------------
# G=20, 2D 256^2 (1,441,792 unknowns): block-diagonal, 22 V-cycles per apply,
# batched (graph replay) against sequential launches, FP64
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("batched", [False, True])
def test_g20_2d256_block_diagonal_against_oracle(ctx, batched):
    fp64_solve_checks(ctx, "g20_2d256", "bdiag", 3, batched=batched, graph=batched)


def test_g20_2d256_block_diagonal_batched_against_sequential(ctx):
    """The same 22 V-cycles per apply; the per-level matrix layouts are tuned
    per union, so batched and sequential applies may sum row entries in a
    different order and agree to rounding, not bit for bit."""
    api = gpu_modules()
    inp, osys, co, gsys = workload(ctx, "g20_2d256")
    Ms = api.BlockPreconditioner(ctx, gsys, "bdiag", amg_seed=3, batched=0, use_graph=0)
    Mb = api.BlockPreconditioner(ctx, gsys, "bdiag", amg_seed=3, batched=1, use_graph=1)
    r = to_dev(ctx, np.random.default_rng(7).standard_normal(osys.n))
    assert_elementwise(to_host(Mb.apply(r)), to_host(Ms.apply(r)), 1e-12, segments=inp.G + 2,
                       what="batched against sequential apply")


# ---------------------------------------------------------------------------
# G=1, 2D 1024^2 (3,145,728 unknowns), FP64 plain
# ---------------------------------------------------------------------------
def test_g1_2d1024_assembly_bit_exact(ctx):
    inp, osys, co, gsys = workload(ctx, "g1_2d1024")
    assert_assembly_equal(gsys, osys)


@pytest.mark.parametrize("kind", ["amg", "pctl", "schur2_lower", "schur1", "schur2"])
def test_g1_2d1024_against_oracle(ctx, kind):
    xh = fp64_solve_checks(ctx, "g1_2d1024", kind, 2, batched=False, graph=False)[0]
    inp, osys, co, gsys = workload(ctx, "g1_2d1024")
    assert true_relres(osys, xh, inp.b) <= 1e-8 * (1 + 1e-6)


# ---------------------------------------------------------------------------
# G=20, 2D 512^2 (5,767,168 unknowns): forward and adjoint
# ---------------------------------------------------------------------------
def test_g20_2d512_forward_and_adjoint_against_oracle(ctx):
    """Forward Schur2 (FP64) and the adjoint on A^T (Schur2 built on the
    transposed blocks): hierarchies bit for bit, iteration counts +-1, the
    same-iteration solution and lambda to 1e-10 at the sample positions.  The
    adjoint's right-hand side x - x_target uses the GPU's same-iteration
    forward solution (equal to the oracle's to about 1e-14), and the
    gradients at the sample positions follow."""
    inp, osys, co, gsys = workload(ctx, "g20_2d512")
    meta, arrays = golden("g20_2d512")
    x, _ = fp64_solve_checks(ctx, "g20_2d512", "schur2", 5, batched=True, graph=True)
    g = x - inp.x_target
    lam, MT = fp64_solve_checks(ctx, "g20_2d512", "schur2", 5, batched=True, graph=True, rhs=g,
                                case_key="adjoint_schur2")
    api = gpu_modules()
    dk, dc = api.adjoint_gradients(ctx, co, to_dev(ctx, x), to_dev(ctx, lam))
    pos = arrays["pos"]
    assert_elementwise(to_host(dk)[pos], arrays["adjoint_schur2/dL_dkappa"], 1e-9, floor=1.0,
                       what="dL/dkappa at the sample positions")
    pc = arrays["adjoint_schur2/dL_dc_pos"]
    assert_elementwise(to_host(dc)[pc], arrays["adjoint_schur2/dL_dc"], 1e-9, floor=1.0,
                       what="dL/dc at the sample positions")


def test_g20_2d512_fp32_adjoint_gradient_formulas(ctx):
    """The FP32-hierarchy forward and adjoint solves of the adjoint workload:
    lambda solves A^T lambda = g to 1e-8 (oracle transpose matvec) and the
    gradients equal the oracle's formulas on the GPU's x and lambda."""
    api = gpu_modules()
    inp, osys, co, gsys = workload(ctx, "g20_2d512")
    b = to_dev(ctx, inp.b)
    M = api.BlockPreconditioner(ctx, gsys, "schur2", amg_seed=5, amg_precision=1, batched=1,
                                use_graph=1)
    x, r = api.gmres(ctx, gsys, M, b, rtol=1e-8, flexible=1)
    assert r.converged
    xh = to_host(x)
    g = xh - inp.x_target
    MT = api.BlockPreconditioner(ctx, gsys, "schur2", amg_seed=5, amg_precision=1, batched=1,
                                 use_graph=1, transpose=1)
    lam, dk, dc, ra = api.adjoint(ctx, co, gsys, MT, x, to_dev(ctx, g), rtol=1e-8, flexible=1)
    assert ra.converged
    lh = to_host(lam)
    ot = osys.transpose()
    assert np.linalg.norm(g - ot.matvec(lh)) / np.linalg.norm(g) <= 1e-8 * (1 + 1e-6)
    dk_o, dgE_o, dEg_o, dEI_o = oadj.gradients(inp, xh, lh)
    G, N = inp.G, inp.N
    dc = to_host(dc)
    assert_elementwise(to_host(dk), dk_o.reshape(-1), 1e-12, segments=G + 2, floor=1e-6,
                       what="dL/dkappa formula")
    assert_elementwise(dc[:G * N], dgE_o.reshape(-1), 1e-12, segments=G, floor=1e-6,
                       what="dL/dc_gE formula")
    assert_elementwise(dc[G * N:2 * G * N], dEg_o.reshape(-1), 1e-12, segments=G, floor=1e-6,
                       what="dL/dc_Eg formula")
    assert_elementwise(dc[2 * G * N:], dEI_o, 1e-12, floor=1e-6, what="dL/dc_EI formula")
    assert rel(to_host(dk), dk_o.reshape(-1)) < 1e-12
