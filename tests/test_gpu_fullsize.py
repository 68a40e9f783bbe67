"""GPU checks on the full-size workloads (2D 1024^2 G=1, 2D 256^2 G=20,
3D 64^3 G=20, 2D 512^2 G=20).

At these sizes the oracle cannot run the whole method, so the checks are
properties that hold at any size, evaluated with the oracle's own arithmetic
on the CPU (the true residual of every GPU solution through the oracle's
block matvec, bit-exact assembly, batched against sequential), plus outputs
the oracle computes directly (the full AMG hierarchy and one V-cycle of the
E block at 3D 64^3, the adjoint gradients from the GPU's x and lambda).
"""
import numpy as np
import pytest

import synth_inputs as si
from oracle import adjoint as oadj
from oracle import amg as oamg
from oracle import assemble as oasm
from oracle import precond as opc

from gpu_helpers import gpu_modules, gpu_system, rel, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    api = gpu_modules()
    return api.Context(0)


_CACHE = {}


def workload(ctx, name):
    """(inputs, oracle system, GPU coefficients, GPU system), built once per module."""
    if name not in _CACHE:
        inp = si.generate_workload(name)
        osys = oasm.assemble(inp)
        co, gsys = gpu_system(ctx, inp)
        _CACHE[name] = (inp, osys, co, gsys)
    return _CACHE[name]


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


# ---------------------------------------------------------------------------
# G=1, 2D 1024^2 (3,145,728 unknowns), FP64 plain
# ---------------------------------------------------------------------------
def test_g1_2d1024_assembly_bit_exact(ctx):
    inp, osys, co, gsys = workload(ctx, "g1_2d1024")
    assert_assembly_equal(gsys, osys)


@pytest.mark.parametrize("kind", ["amg", "pctl", "schur2_lower", "schur1", "schur2"])
def test_g1_2d1024_solves(ctx, kind):
    api = gpu_modules()
    inp, osys, co, gsys = workload(ctx, "g1_2d1024")
    M = api.BlockPreconditioner(ctx, gsys, kind, amg_seed=2)
    b = to_dev(ctx, inp.b)
    x, r = api.gmres(ctx, gsys, M, b, rtol=1e-8, flexible=1)
    assert r.converged, (kind, r)
    assert true_relres(osys, to_host(x), inp.b) <= 1e-8 * (1 + 1e-6), kind


# ---------------------------------------------------------------------------
# G=20, 2D 256^2 (1,441,792 unknowns): block-diagonal, 22 V-cycles per apply,
# batched (graph replay) against sequential launches, FP64
# ---------------------------------------------------------------------------
def test_g20_2d256_block_diagonal_batched_against_sequential(ctx):
    """The same 22 V-cycles per apply; the per-level matrix layouts are tuned
    per union, so batched and sequential applies may sum row entries in a
    different order and agree to rounding, not bit for bit."""
    api = gpu_modules()
    inp, osys, co, gsys = workload(ctx, "g20_2d256")
    Ms = api.BlockPreconditioner(ctx, gsys, "bdiag", amg_seed=3, batched=0, use_graph=0)
    Mb = api.BlockPreconditioner(ctx, gsys, "bdiag", amg_seed=3, batched=1, use_graph=1)
    r = to_dev(ctx, np.random.default_rng(7).standard_normal(osys.n))
    assert rel(to_host(Mb.apply(r)), to_host(Ms.apply(r))) < 1e-12
    b = to_dev(ctx, inp.b)
    xs, rs = api.gmres(ctx, gsys, Ms, b, rtol=1e-8)
    xb, rb = api.gmres(ctx, gsys, Mb, b, rtol=1e-8)
    assert rs.converged and rb.converged and abs(rs.iters - rb.iters) <= 1
    xs, xb = to_host(xs), to_host(xb)
    assert rel(xb, xs) < 1e-6
    assert true_relres(osys, xs, inp.b) <= 1e-8 * (1 + 1e-6)
    assert true_relres(osys, xb, inp.b) <= 1e-8 * (1 + 1e-6)


# ---------------------------------------------------------------------------
# G=20, 3D 64^3 7-point (5,767,168 unknowns): the benchmark configuration
# ---------------------------------------------------------------------------
def test_g20_3d64_assembly_bit_exact(ctx):
    inp, osys, co, gsys = workload(ctx, "g20_3d64")
    assert_assembly_equal(gsys, osys)


@pytest.mark.parametrize("aggressive", [0, 1])
def test_g20_3d64_E_block_hierarchy_and_vcycle(ctx, aggressive):
    """The whole AMG hierarchy of A_E (262,144 rows) equals the oracle's bit for
    bit, also with aggressive coarsening and multipass interpolation on the
    finest level, and one FP64 V-cycle agrees to 1e-12."""
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
    assert rel(to_host(g.apply(to_dev(ctx, bvec))), oamg.vcycle(H, bvec)) < 1e-12


def test_g20_3d64_fp32_batched_against_fp64_plain(ctx):
    api = gpu_modules()
    inp, osys, co, gsys = workload(ctx, "g20_3d64")
    b = to_dev(ctx, inp.b)
    M32 = api.BlockPreconditioner(ctx, gsys, "schur2", amg_seed=4, amg_precision=1, batched=1,
                                  use_graph=1)
    x32, r32 = api.gmres(ctx, gsys, M32, b, rtol=1e-8, flexible=1)
    del M32
    M64 = api.BlockPreconditioner(ctx, gsys, "schur2", amg_seed=4, amg_precision=0, batched=0,
                                  use_graph=0)
    x64, r64 = api.gmres(ctx, gsys, M64, b, rtol=1e-8, flexible=1)
    assert r32.converged and r64.converged
    assert abs(r32.iters - r64.iters) <= 2
    x32, x64 = to_host(x32), to_host(x64)
    assert true_relres(osys, x32, inp.b) <= 1e-8 * (1 + 1e-6)
    assert true_relres(osys, x64, inp.b) <= 1e-8 * (1 + 1e-6)
    assert rel(x32, x64) < 1e-6


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
# G=20, 2D 512^2 (5,767,168 unknowns): adjoint
# ---------------------------------------------------------------------------
def test_g20_2d512_adjoint(ctx):
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
    # lambda solves A^T lambda = g (oracle transpose matvec)
    ot = osys.transpose()
    assert np.linalg.norm(g - ot.matvec(lh)) / np.linalg.norm(g) <= 1e-8 * (1 + 1e-6)
    # gradients: the oracle's formulas on the GPU's x and lambda
    dk_o, dgE_o, dEg_o, dEI_o = oadj.gradients(inp, xh, lh)
    G, N = inp.G, inp.N
    dc = to_host(dc)
    assert rel(to_host(dk), dk_o.reshape(-1)) < 1e-12
    assert rel(dc[:G * N], dgE_o.reshape(-1)) < 1e-12
    assert rel(dc[G * N:2 * G * N], dEg_o.reshape(-1)) < 1e-12
    assert rel(dc[2 * G * N:], dEI_o) < 1e-12
