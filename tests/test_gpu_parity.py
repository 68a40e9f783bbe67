"""GPU parity against the CPU oracle, through the C ABI.

Bars: bit-exact for integer/index results (C/F splittings, sparsity
patterns) and for values computed in a fixed order without contraction
(assembly, setup); floating-point solve results within the tolerances
stated per test."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth_inputs as si
from oracle import amg as oamg
from oracle import krylov as okry
from oracle import precond as opc

from gpu_helpers import (assert_elementwise, csr_of, gpu_modules, gpu_system, matvec_scale,
                         oracle_system, small_inputs, to_dev, to_host)

# Floating-point results are compared entry by entry: |a_i - ref_i| <= tol * s_i
# with s_i = max(|ref_i|, 1e-3 * max |ref| over the block segment of i) for FP64
# results, s_i = max |ref| over the segment for FP32 V-cycle results (whose
# rounding error is absolute at the segment's scale), and
# s_i = sum_j |a_ij x_j| for matrix-vector products.
FP32_FLOOR = 1.0

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    api = gpu_modules()
    c = api.Context(0)
    yield c
    c.synchronize()


# ---------------------------------------------------------------------------
# assembly, matvec
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,inp", small_inputs() + [("g1_2d64", si.generate_workload("g1_2d64"))])
def test_assembly_bit_exact(ctx, name, inp):
    osys = oracle_system(inp)
    co, gsys = gpu_system(ctx, inp)
    for a in range(inp.G + 2):
        rp, ci, v = gsys.block_arrays(a)
        B = osys.blocks[a]
        assert np.array_equal(rp, B.indptr) and np.array_equal(ci, B.indices), (name, a)
        assert np.array_equal(v, B.data), (name, a)
    d_gE, d_Eg, d_EI, d_IE = gsys.couplings()
    assert np.array_equal(d_gE, osys.d_gE.reshape(-1)) and np.array_equal(d_Eg, osys.d_Eg.reshape(-1))
    assert np.array_equal(d_EI, osys.d_EI) and np.array_equal(d_IE, osys.d_IE)


@pytest.mark.parametrize("name,inp", small_inputs())
def test_block_matvec(ctx, name, inp):
    osys = oracle_system(inp)
    co, gsys = gpu_system(ctx, inp)
    x = np.random.default_rng(5).standard_normal(osys.n)
    y = to_host(gsys.matvec(to_dev(ctx, x)))
    A = osys.monolithic()
    assert_elementwise(y, A @ x, 1e-14, scale=matvec_scale(A, x), what="block matvec")


@pytest.mark.parametrize("name,inp", [("g2_2d37", si.generate(2, 2, 37, 31)),
                                      ("g3_3d11", si.generate(3, 3, 11, 32)),
                                      ("g2_2d37_nonsym", si.generate(2, 2, 37, 33, nonsym=True))])
def test_block_matvec_multi_tile(ctx, name, inp):
    """Assembled systems share one pattern across blocks; 1369 and 1331 rows
    span several 512-row tiles of the shared-pattern kernel with a ragged
    last tile.  The transpose keeps one pattern too."""
    osys = oracle_system(inp)
    co, gsys = gpu_system(ctx, inp)
    x = np.random.default_rng(6).standard_normal(osys.n)
    y = to_host(gsys.matvec(to_dev(ctx, x)))
    A = osys.monolithic()
    assert_elementwise(y, A @ x, 1e-14, scale=matvec_scale(A, x), what="block matvec")
    yt = to_host(gsys.transpose().matvec(to_dev(ctx, x)))
    assert_elementwise(yt, A.T @ x, 1e-14, scale=matvec_scale(A.T, x), what="transposed matvec")


def _shared_pattern_system(G, N, seed, max_len):
    """G+2 blocks on one random pattern (rows of 0..max_len sorted distinct
    columns, some rows empty), distinct values per block, random couplings."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, max_len + 1, size=N)
    lens[rng.choice(N, size=N // 10, replace=False)] = 0
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = np.concatenate([np.sort(rng.choice(N, size=int(l), replace=False)) for l in lens]
                        + [np.zeros(0, dtype=np.int64)]).astype(np.int32)
    vals = [rng.standard_normal(int(rp[-1])) for _ in range(G + 2)]
    cpl = [rng.standard_normal(G * N), rng.standard_normal(G * N), rng.standard_normal(N),
           rng.standard_normal(N)]
    return rp, ci, vals, cpl


def _monolithic(G, N, rp, ci, vals, cpl):
    from oracle import assemble as oasm
    blocks = [sp.csr_matrix((v, ci, rp), shape=(N, N)) for v in vals]
    return oasm.BlockSystem(G, N, blocks, cpl[0].reshape(G, N), cpl[1].reshape(G, N), cpl[2],
                            cpl[3]).monolithic()


@pytest.mark.parametrize("G,N,max_len", [(3, 1500, 60), (1, 1777, 5), (2, 700, 250)])
def test_block_matvec_shared_pattern_given(ctx, G, N, max_len):
    """A caller's system whose blocks point at one row_ptr / col_idx takes
    the shared-pattern kernel.  Long rows make a tile's pattern segment exceed
    the kernel's LDS capacity, so it is walked in chunks; empty rows and a
    ragged last tile are covered.  The same system with a separate pattern
    copy per block (general kernel) agrees to rounding."""
    import torch
    api = gpu_modules()
    rp, ci, vals, cpl = _shared_pattern_system(G, N, 40 + N, max_len)
    dev = ctx.device
    trp = torch.as_tensor(rp).to(dev)
    tci = torch.as_tensor(ci).to(dev)
    shared = api.BlockSystem.from_tensors(ctx, G, N, [(trp, tci, torch.as_tensor(v).to(dev))
                                                      for v in vals], *cpl)
    separate = api.BlockSystem.from_tensors(ctx, G, N, [(trp.clone(), tci.clone(),
                                                         torch.as_tensor(v).to(dev))
                                                        for v in vals], *cpl)
    M = _monolithic(G, N, rp, ci, vals, cpl)
    x = np.random.default_rng(9).standard_normal((G + 2) * N)
    ys = to_host(shared.matvec(to_dev(ctx, x)))
    yp = to_host(separate.matvec(to_dev(ctx, x)))
    ref = M @ x
    sc = matvec_scale(M, x)
    assert_elementwise(ys, ref, 1e-13, scale=sc, what="shared-pattern matvec")
    assert_elementwise(yp, ref, 1e-13, scale=sc, what="general matvec")
    assert_elementwise(ys, yp, 1e-13, scale=sc, what="shared vs general")


def test_csr_spmv_ragged(ctx):
    api = gpu_modules()
    rng = np.random.default_rng(7)
    for n, dens in ((1, 1.0), (37, 0.2), (5000, 0.002), (3000, 0.05)):
        A = sp.random(n, n + 3, density=dens, random_state=rng, format="csr")
        A.sort_indices()
        x = rng.standard_normal(n + 3)
        y = to_host(api.csr_spmv(ctx, A.indptr, A.indices, A.data, n + 3, to_dev(ctx, x)))
        assert_elementwise(y, A @ x, 1e-14, scale=matvec_scale(A, x), what=f"spmv n={n}")


# ---------------------------------------------------------------------------
# AMG setup: bit-exact C/F, P and coarse operators
# ---------------------------------------------------------------------------
def _compare_hierarchies(gamg, H, exact_values=True):
    info = gamg.info()
    assert info["levels"] == len(H.levels), (info["n"], [L.A.shape[0] for L in H.levels])
    for l, L in enumerate(H.levels):
        g = gamg.export_level(l)
        n = L.A.shape[0]
        assert info["n"][l] == n
        arp, aci, av = g["A"]
        assert np.array_equal(arp, L.A.indptr) and np.array_equal(aci, L.A.indices), l
        if exact_values:
            assert np.array_equal(av, L.A.data), (l, np.abs(av - L.A.data).max())
        else:
            np.testing.assert_allclose(av, L.A.data, rtol=1e-12, atol=1e-12 * np.abs(L.A.data).max())
        if L.cf is not None:
            assert np.array_equal(g["cf"], L.cf), l
            prp, pci, pv = g["P"]
            assert np.array_equal(prp, L.P.indptr) and np.array_equal(pci, L.P.indices), l
            if exact_values:
                assert np.array_equal(pv, L.P.data), l
            assert info["pmis_rounds"][l] == L.pmis_rounds


@pytest.mark.parametrize("which", ["mono_g1_2d64", "block_E_g2_2d16", "block_g0_3d10",
                                   "mono_g2_2d16_nonsym"])
def test_amg_setup_full_chain_bit_exact(ctx, which):
    api = gpu_modules()
    if which == "mono_g1_2d64":
        A = oracle_system(si.generate_workload("g1_2d64")).monolithic()
    elif which == "block_E_g2_2d16":
        A = oracle_system(si.generate_workload("g2_2d16")).blocks[2]
    elif which == "block_g0_3d10":
        A = oracle_system(si.generate(1, 3, 10, 31)).blocks[0]
    else:
        A = oracle_system(si.generate(2, 2, 16, 32, nonsym=True)).monolithic()
    H = oamg.setup(A, oamg.AMGParams(seed=7))
    g = api.AMG(ctx, A.indptr, A.indices, A.data, seed=7)
    _compare_hierarchies(g, H, exact_values=True)


@pytest.mark.parametrize("which,tile", [("block_E_g2_2d16", 64), ("mono_g2_2d16_nonsym", 128),
                                        ("block_g0_3d10", 1024)])
def test_amg_setup_hmis_bit_exact(ctx, which, tile):
    """HMIS (tile-local Ruge-Stueben first pass, then PMIS): the whole hierarchy
    equals the oracle's bit for bit, and one V-cycle agrees to 1e-12."""
    api = gpu_modules()
    if which == "block_E_g2_2d16":
        A = oracle_system(si.generate_workload("g2_2d16")).blocks[2]
    elif which == "block_g0_3d10":
        A = oracle_system(si.generate(1, 3, 10, 31)).blocks[0]
    else:
        A = oracle_system(si.generate(2, 2, 16, 32, nonsym=True)).monolithic()
    H = oamg.setup(A, oamg.AMGParams(seed=5, coarsening="hmis", hmis_tile=tile))
    g = api.AMG(ctx, A.indptr, A.indices, A.data, seed=5, coarsening=1, hmis_tile=tile)
    _compare_hierarchies(g, H, exact_values=True)
    b = np.random.default_rng(6).uniform(size=A.shape[0])
    assert_elementwise(to_host(g.apply(to_dev(ctx, b))), oamg.vcycle(H, b), 1e-12,
                       what="HMIS V-cycle")


@pytest.mark.parametrize("which,coarsening,levels", [("block_g0_3d10", 0, 1),
                                                     ("mono_g2_2d16_nonsym", 0, 1),
                                                     ("block_E_g2_2d16", 1, 1),
                                                     ("mono_g1_2d64", 0, 2)])
def test_amg_setup_aggressive_bit_exact(ctx, which, coarsening, levels):
    """Aggressive coarsening (a second pass over the C points on their
    distance-two strength graph, multipass interpolation) on the finest
    `levels` levels: the hierarchy equals the oracle's bit for bit, and one
    V-cycle agrees to 1e-12."""
    api = gpu_modules()
    if which == "block_E_g2_2d16":
        A = oracle_system(si.generate_workload("g2_2d16")).blocks[2]
    elif which == "block_g0_3d10":
        A = oracle_system(si.generate(1, 3, 10, 31)).blocks[0]
    elif which == "mono_g1_2d64":
        A = oracle_system(si.generate_workload("g1_2d64")).monolithic()
    else:
        A = oracle_system(si.generate(2, 2, 16, 32, nonsym=True)).monolithic()
    H = oamg.setup(A, oamg.AMGParams(seed=5, coarsening=("hmis" if coarsening else "pmis"),
                                     hmis_tile=128, aggressive_levels=levels))
    g = api.AMG(ctx, A.indptr, A.indices, A.data, seed=5, coarsening=coarsening, hmis_tile=128,
                aggressive_levels=levels)
    _compare_hierarchies(g, H, exact_values=True)
    assert H.levels[1].A.shape[0] * 4 < A.shape[0]
    b = np.random.default_rng(6).uniform(size=A.shape[0])
    assert_elementwise(to_host(g.apply(to_dev(ctx, b))), oamg.vcycle(H, b), 1e-12,
                       what="aggressive V-cycle")


def test_amg_levelwise_on_gpu_levels(ctx):
    """Binding test: the oracle's strength, PMIS and interpolation applied to
    each GPU level matrix give the GPU's C/F splitting and P bit for bit."""
    api = gpu_modules()
    A = oracle_system(si.generate(20, 2, 24, 33)).blocks[5]
    g = api.AMG(ctx, A.indptr, A.indices, A.data, seed=3)
    info = g.info()
    for l in range(info["levels"] - 1):
        e = g.export_level(l)
        Al = csr_of(e["A"], info["n"][l])
        S = oamg.strength(Al, 0.25, 0.9)
        cf = oamg.pmis(Al, S, 3, l)
        assert np.array_equal(cf, e["cf"]), l
        P = oamg.interpolation(Al, S, cf)
        prp, pci, pv = e["P"]
        assert np.array_equal(P.indptr, prp) and np.array_equal(P.indices, pci)
        assert np.array_equal(P.data, pv)


def test_amg_edge_cases(ctx):
    api = gpu_modules()
    # single row
    g = api.AMG(ctx, np.array([0, 1]), np.array([0]), np.array([2.0]))
    z = to_host(g.apply(to_dev(ctx, np.array([3.0]))))
    assert abs(z[0] - 1.5) < 1e-15
    # small system: one direct level
    A = oracle_system(si.generate(1, 2, 5, 3)).monolithic()
    g = api.AMG(ctx, A.indptr, A.indices, A.data)
    assert g.info()["levels"] == 1
    b = np.arange(A.shape[0], dtype=float)
    z = to_host(g.apply(to_dev(ctx, b)))
    assert_elementwise(z, spla.spsolve(sp.csc_matrix(A), b), 1e-12, what="one-level direct")
    # strongly dominant rows: stalled coarsening relaxed with Jacobi sweeps
    n = 3000
    A = sp.csr_matrix(sp.diags([-np.ones(n - 1), 30 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]))
    A.sort_indices()
    g = api.AMG(ctx, A.indptr, A.indices, A.data)
    inf = g.info()
    assert inf["levels"] == 1 and inf["coarse_kind"] == 1
    H = oamg.setup(A)
    b = np.ones(n)
    assert_elementwise(to_host(g.apply(to_dev(ctx, b))), oamg.vcycle(H, b), 1e-14,
                       what="stalled level relaxed")


def test_amg_rejects_invalid_csr(ctx):
    api = gpu_modules()
    from paper_2002_04958_amd._lib import MgdError
    with pytest.raises(MgdError, match="EINVAL"):  # unsorted columns
        api.AMG(ctx, np.array([0, 2, 3]), np.array([1, 0, 1]), np.array([1.0, 2.0, 3.0]))
    with pytest.raises(MgdError, match="EINVAL"):  # missing diagonal
        api.AMG(ctx, np.array([0, 1, 2]), np.array([1, 0]), np.array([1.0, 2.0]))
    with pytest.raises(MgdError, match="EINVAL"):  # column out of range
        api.AMG(ctx, np.array([0, 1, 2]), np.array([0, 5]), np.array([1.0, 2.0]))


# ---------------------------------------------------------------------------
# V-cycle
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("cycles", [1, 3])
@pytest.mark.parametrize("precision", [0, 1])
def test_vcycle_parity(ctx, cycles, precision):
    api = gpu_modules()
    A = oracle_system(si.generate_workload("g1_2d64")).monolithic()
    H = oamg.setup(A, oamg.AMGParams(seed=1))
    g = api.AMG(ctx, A.indptr, A.indices, A.data, seed=1, precision=precision)
    b = np.random.default_rng(2).uniform(size=A.shape[0])
    z = to_host(g.apply(to_dev(ctx, b), cycles=cycles))
    ref = oamg.apply_cycles(H, b, cycles)
    assert_elementwise(z, ref, (1e-12 if precision == 0 else 5e-5),
                       floor=(FP32_FLOOR if precision else 1e-3), what="V-cycles")


@pytest.mark.parametrize("sell16,span", [("1", "32767"), ("1", "40"), ("1", "0"),
                                         ("0", "32767")])
@pytest.mark.parametrize("precision", [0, 1])
def test_sliced_layouts_forced_small(ctx, monkeypatch, sell16, span, precision):
    """Sliced-ELL level layouts, with 32-bit columns or with 16-bit offsets from
    two column bases per 64-row slice (slices whose columns span more than
    `span` on a side keep 32-bit columns: none, some, all), forced on every
    level of small systems: two V-cycles and a batched Schur2 apply agree with
    the oracle."""
    monkeypatch.setenv("MGD_SELL_MIN_ROWS", "64")
    monkeypatch.setenv("MGD_SELL16", sell16)
    monkeypatch.setenv("MGD_SELL16_SPAN", span)
    api = gpu_modules()
    tol = 1e-12 if precision == 0 else 5e-5
    A = oracle_system(si.generate_workload("g1_2d64")).monolithic()
    H = oamg.setup(A, oamg.AMGParams(seed=1))
    g = api.AMG(ctx, A.indptr, A.indices, A.data, seed=1, precision=precision)
    b = np.random.default_rng(2).uniform(size=A.shape[0])
    assert_elementwise(to_host(g.apply(to_dev(ctx, b), cycles=2)), oamg.apply_cycles(H, b, 2), tol,
                       floor=(FP32_FLOOR if precision else 1e-3), what="two V-cycles")
    inp = si.generate(3, 2, 24, 41)
    osys = oracle_system(inp)
    M_o = opc.BlockPreconditioner(osys, opc.BlockParams(kind="schur2", amg=oamg.AMGParams(seed=5)))
    co, gsys = gpu_system(ctx, inp)
    M_g = api.BlockPreconditioner(ctx, gsys, "schur2", amg_seed=5, batched=1,
                                  amg_precision=precision)
    r = np.random.default_rng(4).standard_normal(osys.n)
    assert_elementwise(to_host(M_g.apply(to_dev(ctx, r))), M_o(r), (1e-10 if precision == 0 else 5e-5),
                       segments=inp.G + 2, floor=(FP32_FLOOR if precision else 1e-3), what="schur2 apply")


def test_vcycle_n_pre_n_post(ctx):
    api = gpu_modules()
    A = oracle_system(si.generate(1, 2, 20, 9)).blocks[0]
    for pre, post in ((2, 1), (0, 2), (1, 0)):
        H = oamg.setup(A, oamg.AMGParams(seed=2, n_pre=pre, n_post=post))
        g = api.AMG(ctx, A.indptr, A.indices, A.data, seed=2, n_pre=pre, n_post=post)
        b = np.random.default_rng(3).uniform(size=A.shape[0])
        assert_elementwise(to_host(g.apply(to_dev(ctx, b))), oamg.vcycle(H, b), 1e-12,
                           what=f"V({pre},{post})")


@pytest.mark.parametrize("which", ["mono_g2_2d16_nonsym", "block_g0_3d10", "mono_g1_2d64"])
@pytest.mark.parametrize("precision", [0, 1])
def test_vcycle_multicolour_gauss_seidel(ctx, which, precision):
    """Multicolour Gauss-Seidel smoothing (Jones-Plassmann colours): V-cycles
    and 3-cycle applications against the oracle."""
    api = gpu_modules()
    if which == "block_g0_3d10":
        A = oracle_system(si.generate(1, 3, 10, 31)).blocks[0]
    elif which == "mono_g1_2d64":
        A = oracle_system(si.generate_workload("g1_2d64")).monolithic()
    else:
        A = oracle_system(si.generate(2, 2, 16, 32, nonsym=True)).monolithic()
    tol = 1e-12 if precision == 0 else 5e-5
    for pre, post in ((1, 1), (2, 1), (0, 2)):
        H = oamg.setup(A, oamg.AMGParams(seed=3, smoother="mc_gs", n_pre=pre, n_post=post))
        g = api.AMG(ctx, A.indptr, A.indices, A.data, seed=3, smoother=1, n_pre=pre, n_post=post,
                    precision=precision)
        b = np.random.default_rng(9).uniform(size=A.shape[0])
        assert_elementwise(to_host(g.apply(to_dev(ctx, b))), oamg.vcycle(H, b), tol,
                           floor=(FP32_FLOOR if precision else 1e-3), what=f"GS V({pre},{post})")
        assert_elementwise(to_host(g.apply(to_dev(ctx, b), cycles=3)), oamg.apply_cycles(H, b, 3), tol,
                           floor=(FP32_FLOOR if precision else 1e-3), what="GS three cycles")


@pytest.mark.parametrize("mode", ["seq", "batched_graph"])
def test_schur2_with_multicolour_gauss_seidel(ctx, mode):
    api = gpu_modules()
    inp = si.generate(3, 2, 16, 41)
    osys = oracle_system(inp)
    M_o = opc.BlockPreconditioner(osys, opc.BlockParams(
        kind="schur2", amg=oamg.AMGParams(seed=5, smoother="mc_gs")))
    co, gsys = gpu_system(ctx, inp)
    M_g = api.BlockPreconditioner(ctx, gsys, "schur2", amg_seed=5, amg_smoother=1,
                                  batched=int(mode != "seq"), use_graph=int(mode == "batched_graph"))
    r = np.random.default_rng(4).standard_normal(osys.n)
    assert_elementwise(to_host(M_g.apply(to_dev(ctx, r))), M_o(r), 1e-10,
                       segments=inp.G + 2, what="schur2 GS apply")
    x, res = api.gmres(ctx, gsys, M_g, to_dev(ctx, inp.b), rtol=1e-8)
    xo, io = okry.gmres(osys.matvec, M_o, inp.b, rtol=1e-8)
    assert res.converged and abs(res.iters - io.iters) <= 1


# ---------------------------------------------------------------------------
# block preconditioners
# ---------------------------------------------------------------------------
KINDS = ["amg", "bdiag", "pctl", "schur1", "schur2", "schur2_lower"]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("mode", ["seq", "batched", "batched_graph"])
def test_block_preconditioner_parity(ctx, kind, mode):
    api = gpu_modules()
    inp = si.generate(3, 2, 16, 41)
    osys = oracle_system(inp)
    M_o = opc.BlockPreconditioner(osys, opc.BlockParams(kind=kind, amg=oamg.AMGParams(seed=5)))
    co, gsys = gpu_system(ctx, inp)
    M_g = api.BlockPreconditioner(ctx, gsys, kind, amg_seed=5, batched=int(mode != "seq"),
                                  use_graph=int(mode == "batched_graph"))
    r = np.random.default_rng(4).standard_normal(osys.n)
    rd = to_dev(ctx, r)
    z = to_host(M_g.apply(rd))
    ref = M_o(r)
    assert_elementwise(z, ref, 1e-10, segments=inp.G + 2, what=f"{kind} apply")
    # repeated calls on the same buffers (graph replays in graph mode), with
    # eager work and synchronisation between them, and new data in place
    import torch
    zb = torch.empty_like(rd)
    for _ in range(3):
        M_g.apply(rd, zb)
        assert np.array_equal(to_host(zb), z)
        torch.cuda.synchronize()
        assert float((rd * 2.0).sum()) == float((rd * 2.0).sum())
    r2 = np.random.default_rng(5).standard_normal(osys.n)
    rd.copy_(to_dev(ctx, r2))
    M_g.apply(rd, zb)
    assert_elementwise(to_host(zb), M_o(r2), 1e-10, segments=inp.G + 2, what=f"{kind} new data")
    info = M_g.info()
    G = inp.G
    exp_inv = {"amg": 1, "bdiag": G + 2, "pctl": G + 3, "schur1": G + 4, "schur2": G + 3,
               "schur2_lower": G + 2}[kind]
    assert info["inverses_per_apply"] == exp_inv
    assert info["matvecs_per_apply"] == (G + 2 if kind == "pctl" else 0)
    if kind == "pctl":
        assert info["pctl_p_cycles"] == M_o.setup_info["p_cycles"]


# ---------------------------------------------------------------------------
# adaptive strategy (Section 3.5; Definitions 1-2, options #1/#2)
# ---------------------------------------------------------------------------
ADAPTIVE_CASES = {
    "drawn": {},                                                     # the generator's couplings
    "from_E": dict(c_scale=(1e-6, 1.0, 1.0), log_kappa_shift=(0.0, 0.0, 6.0)),
    "into_E": dict(log_kappa_shift=(0.0, 6.0, 0.0)),
    "all": dict(c_scale=(1e-6, 1e-6, 1e-6)),
    "mixed": dict(c_scale=([1e-6, 1.0, 1e-6], 1.0, 1.0)),              # groups 1 and 3 only
    "jacobi_I": dict(log_kappa_shift=(0.0, 0.0, -8.0)),             # option #1 for the I block
}


def _role_key(role, G):
    return ("g", role) if role < G else ("E" if role == G else "I")


def assert_same_decisions(info, M_o, G):
    """Definition 1 and 2 counts are integers: GPU and oracle must agree exactly."""
    plan = M_o.plan
    assert info["wc_counts"]["gE"] == [int(v) for v in plan.counts["gE"]]
    assert info["wc_counts"]["Eg"] == [int(v) for v in plan.counts["Eg"]]
    assert info["wc_counts"]["EI"] == int(plan.counts["EI"][0])
    assert info["wc_counts"]["IE"] == int(plan.counts["IE"][0])
    assert info["weak"] == {"gE": [bool(v) for v in plan.gE], "Eg": [bool(v) for v in plan.Eg],
                            "EI": bool(plan.EI), "IE": bool(plan.IE)}
    keys = [_role_key(r, G) for r in range(G + 2)]
    assert info["wd_count"] == [M_o.setup_info["wd_counts"][k] for k in keys]
    assert info["jacobi"] == [k in M_o.jacobi_roles for k in keys]


@pytest.mark.parametrize("case", list(ADAPTIVE_CASES))
@pytest.mark.parametrize("kind", ["pctl", "schur1", "schur2"])
@pytest.mark.parametrize("mode", ["seq", "batched_graph", "fp32_batched_graph"])
def test_adaptive_preconditioner_parity(ctx, kind, case, mode):
    import torch
    api = gpu_modules()
    inp = si.generate(3, 2, 16, 41, **ADAPTIVE_CASES[case])
    osys = oracle_system(inp)
    M_o = opc.BlockPreconditioner(osys, opc.BlockParams(kind=kind, adaptive=True,
                                                        amg=oamg.AMGParams(seed=5)))
    co, gsys = gpu_system(ctx, inp)
    fp32 = mode.startswith("fp32")
    M_g = api.BlockPreconditioner(ctx, gsys, kind, amg_seed=5, adaptive=1,
                                  batched=int(mode != "seq"), use_graph=int(mode != "seq"),
                                  amg_precision=int(fp32))
    G = inp.G
    assert_same_decisions(M_g.info(), M_o, G)
    if case == "jacobi_I":
        assert M_o.jacobi_roles == {"I"}
    tol = 5e-5 if fp32 else 1e-10
    r = np.random.default_rng(4).standard_normal(osys.n)
    rd = to_dev(ctx, r)
    z = to_host(M_g.apply(rd))
    c0 = M_o.counters.inverses
    ref = M_o(r)
    assert_elementwise(z, ref, tol,
                       segments=G + 2, floor=(FP32_FLOOR if fp32 else 1e-3), what=f"adaptive {kind} apply")
    assert M_g.info()["inverses_per_apply"] == M_o.counters.inverses - c0
    assert M_g.info()["matvecs_per_apply"] == M_o.counters.matvecs
    zb = torch.empty_like(rd)
    for _ in range(3):
        M_g.apply(rd, zb)
        assert np.array_equal(to_host(zb), z)
        torch.cuda.synchronize()
    r2 = np.random.default_rng(5).standard_normal(osys.n)
    rd.copy_(to_dev(ctx, r2))
    M_g.apply(rd, zb)
    assert_elementwise(to_host(zb), M_o(r2), tol,
                       segments=G + 2, floor=(FP32_FLOOR if fp32 else 1e-3), what=f"adaptive {kind} new data")


# Structural cases for solves: the kappa-shifted apply cases above are too ill
# conditioned for GMRES(30) at 1e-8 with any of the preconditioners, so the
# same neglect patterns come from coupling scales here (scaling c_EI makes
# both D_EI and D_IE weak).
GMRES_CASES = {
    "drawn": {},
    "from_E": dict(c_scale=(1e-6, 1.0, 1e-6)),
    "into_E": dict(c_scale=(1.0, 1e-6, 1e-6)),
    "mixed": ADAPTIVE_CASES["mixed"],
    "jacobi_I": ADAPTIVE_CASES["jacobi_I"],
}


@pytest.mark.parametrize("case", list(GMRES_CASES))
def test_adaptive_schur2_gmres(ctx, case):
    """alpha-Schur2 inside FGMRES: iteration counts within one of the oracle's,
    both solutions at rtol 1e-8 against the full (unmodified) system."""
    api = gpu_modules()
    inp = si.generate(3, 2, 24, 61, **GMRES_CASES[case])
    osys = oracle_system(inp)
    M_o = opc.BlockPreconditioner(osys, opc.BlockParams(kind="schur2", adaptive=True,
                                                        amg=oamg.AMGParams(seed=6)))
    xo, io = okry.gmres(osys.matvec, M_o, inp.b, rtol=1e-8)
    co, gsys = gpu_system(ctx, inp)
    M_g = api.BlockPreconditioner(ctx, gsys, "schur2", amg_seed=6, adaptive=1, batched=1,
                                  use_graph=1)
    x, res = api.gmres(ctx, gsys, M_g, to_dev(ctx, inp.b), rtol=1e-8, flexible=1)
    assert res.converged and abs(res.iters - io.iters) <= 1, (res.iters, io.iters)
    xh = to_host(x)
    bn = np.linalg.norm(inp.b)
    assert np.linalg.norm(inp.b - osys.matvec(xh)) <= 1e-8 * bn * (1 + 1e-6)
    assert np.linalg.norm(inp.b - osys.matvec(xo)) <= 1e-8 * bn * (1 + 1e-6)


def test_adaptive_rejects_other_kinds(ctx):
    api = gpu_modules()
    inp = si.generate(2, 2, 8, 3)
    co, gsys = gpu_system(ctx, inp)
    for kind in ("amg", "bdiag", "schur2_lower"):
        with pytest.raises(RuntimeError):
            api.BlockPreconditioner(ctx, gsys, kind, adaptive=1)


# ---------------------------------------------------------------------------
# inner solves to a tolerance (option #3 for the inverses Section 4 names)
# ---------------------------------------------------------------------------
def _oracle_inner_cycles(M_o, G):
    out = []
    for r in range(G + 3):
        key = _role_key(r, G) if r < G + 2 else "c"
        inv = M_o.inv.get(key)
        out.append(getattr(inv, "last_cycles", -1) if key in M_o.tolerance_roles() else -1)
    return out


@pytest.mark.parametrize("kind", ["pctl", "schur1", "schur2"])
@pytest.mark.parametrize("mode", ["seq", "batched", "fp32_batched", "adaptive_jacobi_I"])
def test_inner_tolerance_parity(ctx, kind, mode):
    api = gpu_modules()
    extra = ADAPTIVE_CASES["jacobi_I"] if mode == "adaptive_jacobi_I" else {}
    inp = si.generate(3, 2, 16, 43, **extra)
    osys = oracle_system(inp)
    adaptive = mode.startswith("adaptive")
    M_o = opc.BlockPreconditioner(osys, opc.BlockParams(kind=kind, inner_tol=1e-2,
                                                        adaptive=adaptive,
                                                        amg=oamg.AMGParams(seed=5)))
    co, gsys = gpu_system(ctx, inp)
    fp32 = mode.startswith("fp32")
    M_g = api.BlockPreconditioner(ctx, gsys, kind, amg_seed=5, inner_tol=1e-2,
                                  adaptive=int(adaptive), batched=int(mode != "seq"),
                                  use_graph=1, amg_precision=int(fp32))
    G = inp.G
    for seed in (4, 5):
        r = np.random.default_rng(seed).standard_normal(osys.n)
        z = to_host(M_g.apply(to_dev(ctx, r)))
        ref = M_o(r)
        assert_elementwise(z, ref, (5e-5 if fp32 else 1e-10),
                           segments=G + 2, floor=(FP32_FLOOR if fp32 else 1e-3), what=f"inner-tol {kind} apply")
        got = M_g.info()["inner_cycles"]
        want = _oracle_inner_cycles(M_o, G)
        if adaptive:
            want[G + 1] = -1          # the I block uses Jacobi (option #1)
        if fp32:
            assert all(abs(a - b) <= 1 for a, b in zip(got, want)), (got, want)
        else:
            assert got == want, (got, want)
        assert max(got) >= 2


def test_inner_tolerance_fgmres(ctx):
    api = gpu_modules()
    inp = si.generate(3, 2, 24, 61)
    osys = oracle_system(inp)
    M_o = opc.BlockPreconditioner(osys, opc.BlockParams(kind="schur2", inner_tol=1e-2,
                                                        amg=oamg.AMGParams(seed=6)))
    xo, io = okry.gmres(osys.matvec, M_o, inp.b, rtol=1e-8)
    co, gsys = gpu_system(ctx, inp)
    M_g = api.BlockPreconditioner(ctx, gsys, "schur2", amg_seed=6, inner_tol=1e-2, batched=1)
    x, res = api.gmres(ctx, gsys, M_g, to_dev(ctx, inp.b), rtol=1e-8, flexible=1)
    assert res.converged and abs(res.iters - io.iters) <= 1, (res.iters, io.iters)
    bn = np.linalg.norm(inp.b)
    assert np.linalg.norm(inp.b - osys.matvec(to_host(x))) <= 1e-8 * bn * (1 + 1e-6)


# ---------------------------------------------------------------------------
# option #4: S_I (Schur2) / C_E (Schur1) by fixed-point steps
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["schur1", "schur2"])
@pytest.mark.parametrize("mode", ["seq", "batched_graph", "fp32_batched_graph", "adaptive_from_E",
                                  "inner_tol"])
def test_option4_parity(ctx, kind, mode):
    import torch
    api = gpu_modules()
    adaptive = mode == "adaptive_from_E"
    inp = si.generate(3, 2, 16, 47, **(ADAPTIVE_CASES["from_E"] if adaptive else {}))
    osys = oracle_system(inp)
    tol = 1e-2 if mode == "inner_tol" else 0.0
    M_o = opc.BlockPreconditioner(osys, opc.BlockParams(kind=kind, option4_steps=3,
                                                        adaptive=adaptive, inner_tol=tol,
                                                        amg=oamg.AMGParams(seed=5)))
    co, gsys = gpu_system(ctx, inp)
    fp32 = mode.startswith("fp32")
    M_g = api.BlockPreconditioner(ctx, gsys, kind, amg_seed=5, option4_steps=3,
                                  adaptive=int(adaptive), inner_tol=tol,
                                  batched=int(mode != "seq"), use_graph=int("graph" in mode),
                                  amg_precision=int(fp32))
    if adaptive:
        assert_same_decisions(M_g.info(), M_o, inp.G)
    tol_z = 5e-5 if fp32 else 1e-10
    r = np.random.default_rng(4).standard_normal(osys.n)
    rd = to_dev(ctx, r)
    z = to_host(M_g.apply(rd))
    c0 = M_o.counters.inverses
    ref = M_o(r)
    # the kappa-shifted case puts the I segment six decades below the others;
    # its entries carry the rounding of the O(1) terms the fixed-point steps
    # cancel into them, so the floor is taken over the whole vector there
    assert_elementwise(z, ref, tol_z, segments=1 if adaptive else inp.G + 2,
                       floor=(FP32_FLOOR if fp32 else 1e-3), what=f"option4 {kind} apply")
    assert M_g.info()["inverses_per_apply"] == M_o.counters.inverses - c0
    zb = torch.empty_like(rd)
    for _ in range(2):
        M_g.apply(rd, zb)
        assert np.array_equal(to_host(zb), z)
        torch.cuda.synchronize()


@pytest.mark.parametrize("kind", ["schur1", "schur2"])
def test_option4_fgmres(ctx, kind):
    api = gpu_modules()
    inp = si.generate(3, 2, 24, 61)
    osys = oracle_system(inp)
    M_o = opc.BlockPreconditioner(osys, opc.BlockParams(kind=kind, option4_steps=2,
                                                        amg=oamg.AMGParams(seed=6)))
    xo, io = okry.gmres(osys.matvec, M_o, inp.b, rtol=1e-8)
    co, gsys = gpu_system(ctx, inp)
    M_g = api.BlockPreconditioner(ctx, gsys, kind, amg_seed=6, option4_steps=2, batched=1,
                                  use_graph=1)
    x, res = api.gmres(ctx, gsys, M_g, to_dev(ctx, inp.b), rtol=1e-8, flexible=1)
    assert res.converged and abs(res.iters - io.iters) <= 1, (res.iters, io.iters)
    bn = np.linalg.norm(inp.b)
    assert np.linalg.norm(inp.b - osys.matvec(to_host(x))) <= 1e-8 * bn * (1 + 1e-6)


# ---------------------------------------------------------------------------
# GMRES
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["amg", "schur2", "schur1", "pctl"])
def test_gmres_parity(ctx, kind):
    api = gpu_modules()
    inp = si.generate_workload("g1_2d64")
    osys = oracle_system(inp)
    A = osys.monolithic()
    M_o = opc.BlockPreconditioner(osys, opc.BlockParams(kind=kind, amg=oamg.AMGParams(seed=1)))
    xo, io = okry.gmres(A.__matmul__, M_o, inp.b, rtol=1e-8)
    co, gsys = gpu_system(ctx, inp)
    M_g = api.BlockPreconditioner(ctx, gsys, kind, amg_seed=1)
    b = to_dev(ctx, inp.b)
    xg, rg = api.gmres(ctx, gsys, M_g, b, rtol=1e-8)
    assert rg.converged and io.converged
    assert abs(rg.iters - io.iters) <= 1, (rg.iters, io.iters)
    xg = to_host(xg)
    assert np.linalg.norm(inp.b - A @ xg) <= 1e-8 * np.linalg.norm(inp.b)
    # same number of iterations: solutions agree to 1e-10
    xo2, _ = okry.gmres(A.__matmul__, M_o, inp.b, rtol=0.0, max_iters=io.iters)
    xg2, r2 = api.gmres(ctx, gsys, M_g, b, rtol=0.0, max_iters=io.iters)
    assert r2.status == -4 and r2.iters == io.iters
    assert_elementwise(to_host(xg2), xo2, 1e-10,
                       segments=inp.G + 2, what=f"{kind} same-iteration solution")


@pytest.mark.parametrize("precision,smoother,coarsening", [(1, 0, 0), (0, 1, 0), (1, 0, 1)])
def test_aggressive_schur2_variants(ctx, precision, smoother, coarsening):
    """Aggressive coarsening combined with FP32 hierarchies, multicolour
    Gauss-Seidel and HMIS: a batched, graph-replayed Schur2 apply agrees with
    the oracle's (twice in a row), and FGMRES converges to 1e-8 in the
    oracle's iteration count (+-1 in FP64, +-2 with FP32 V-cycles)."""
    api = gpu_modules()
    inp = si.generate(3, 2, 24, 43)
    osys = oracle_system(inp)
    ap = oamg.AMGParams(seed=5, aggressive_levels=1, smoother=("mc_gs" if smoother else "cf_l1_jacobi"),
                        coarsening=("hmis" if coarsening else "pmis"), hmis_tile=128)
    M_o = opc.BlockPreconditioner(osys, opc.BlockParams(kind="schur2", amg=ap))
    co, gsys = gpu_system(ctx, inp)
    M_g = api.BlockPreconditioner(ctx, gsys, "schur2", amg_seed=5, amg_aggressive_levels=1,
                                  amg_smoother=smoother, amg_coarsening=coarsening,
                                  amg_hmis_tile=128, amg_precision=precision, batched=1,
                                  use_graph=1)
    r = np.random.default_rng(4).standard_normal(osys.n)
    tol = 1e-10 if precision == 0 else 5e-5
    for _ in range(2):
        assert_elementwise(to_host(M_g.apply(to_dev(ctx, r))), M_o(r), tol,
                           segments=inp.G + 2, floor=(FP32_FLOOR if precision else 1e-3), what="aggressive schur2 apply")
    x, res = api.gmres(ctx, gsys, M_g, to_dev(ctx, inp.b), rtol=1e-8, flexible=1)
    xo, io = okry.gmres(osys.matvec, M_o, inp.b, rtol=1e-8)
    assert res.converged and abs(res.iters - io.iters) <= (1 if precision == 0 else 2), \
        (res.iters, io.iters)
    A = osys.monolithic()
    assert np.linalg.norm(inp.b - A @ to_host(x)) <= 1e-8 * np.linalg.norm(inp.b) * (1 + 1e-6)


@pytest.mark.parametrize("kind", ["amg", "schur2"])
def test_gmres_aggressive_parity(ctx, kind):
    """Inner AMG with aggressive coarsening on the finest level: the same
    iteration count as the oracle and the same iterate after it."""
    api = gpu_modules()
    inp = si.generate_workload("g1_2d64")
    osys = oracle_system(inp)
    A = osys.monolithic()
    M_o = opc.BlockPreconditioner(osys, opc.BlockParams(
        kind=kind, amg=oamg.AMGParams(seed=1, aggressive_levels=1)))
    xo, io = okry.gmres(A.__matmul__, M_o, inp.b, rtol=1e-8)
    co, gsys = gpu_system(ctx, inp)
    M_g = api.BlockPreconditioner(ctx, gsys, kind, amg_seed=1, amg_aggressive_levels=1)
    b = to_dev(ctx, inp.b)
    xg, rg = api.gmres(ctx, gsys, M_g, b, rtol=1e-8)
    assert rg.converged and io.converged
    assert abs(rg.iters - io.iters) <= 1, (rg.iters, io.iters)
    assert np.linalg.norm(inp.b - A @ to_host(xg)) <= 1e-8 * np.linalg.norm(inp.b)
    xo2, _ = okry.gmres(A.__matmul__, M_o, inp.b, rtol=0.0, max_iters=io.iters)
    xg2, r2 = api.gmres(ctx, gsys, M_g, b, rtol=0.0, max_iters=io.iters)
    assert r2.iters == io.iters
    assert_elementwise(to_host(xg2), xo2, 1e-10,
                       segments=inp.G + 2, what=f"aggressive {kind} same-iteration solution")


@pytest.mark.parametrize("kind,precision,restart", [
    ("schur2", 0, 30), ("schur2", 1, 30), ("schur2", 1, 4), ("schur2_lower", 1, 5),
    ("pctl", 0, 4), ("schur1", 1, 30)])
def test_gmres_step_graph_matches_direct(ctx, kind, precision, restart):
    """With graph replay every flexible-GMRES step (apply, matvec, Gram-Schmidt)
    runs as one cached graph, and where the apply starts with the E solve that
    solve for the next basis vector ends the step before it (the first step of
    each restart cycle does its own); three solves in a row, with eager work
    and synchronisation between them, equal the direct launches bit for bit."""
    import torch
    api = gpu_modules()
    inp = si.generate(3, 2, 24, 61)
    co, gsys = gpu_system(ctx, inp)
    b = to_dev(ctx, inp.b)
    Md = api.BlockPreconditioner(ctx, gsys, kind, amg_seed=6, batched=1, use_graph=0,
                                 amg_precision=precision)
    xd, rd = api.gmres(ctx, gsys, Md, b, rtol=1e-9, flexible=1, restart=restart)
    xd = to_host(xd)
    Mg = api.BlockPreconditioner(ctx, gsys, kind, amg_seed=6, batched=1, use_graph=1,
                                 amg_precision=precision)
    for _ in range(3):
        xg, rg = api.gmres(ctx, gsys, Mg, b, rtol=1e-9, flexible=1, restart=restart)
        assert rg.iters == rd.iters and rg.converged
        assert np.array_equal(to_host(xg), xd)
        torch.cuda.synchronize()
        assert float((b * 2.0).sum()) == float((b * 2.0).sum())


def test_gmres_no_preconditioner_and_nonflexible(ctx):
    api = gpu_modules()
    inp = si.generate(1, 2, 12, 5)
    osys = oracle_system(inp)
    A = osys.monolithic()
    co, gsys = gpu_system(ctx, inp)
    b = to_dev(ctx, inp.b)
    xg, rg = api.gmres(ctx, gsys, None, b, rtol=1e-10, max_iters=2000)
    xo, io = okry.gmres(A.__matmul__, None, inp.b, rtol=1e-10, max_iters=2000)
    assert rg.converged and abs(rg.iters - io.iters) <= 1
    M_g = api.BlockPreconditioner(ctx, gsys, "schur2")
    M_o = opc.BlockPreconditioner(osys, opc.BlockParams(kind="schur2"))
    xg, rg = api.gmres(ctx, gsys, M_g, b, rtol=1e-10, flexible=0)
    xo, io = okry.gmres(A.__matmul__, M_o, inp.b, rtol=1e-10, flexible=False)
    assert rg.converged and abs(rg.iters - io.iters) <= 1
    assert_elementwise(to_host(xg), xo, 1e-8, segments=inp.G + 2, what="non-flexible solution")


def test_gmres_edge_cases(ctx):
    api = gpu_modules()
    import torch
    inp = si.generate(1, 2, 8, 5)
    co, gsys = gpu_system(ctx, inp)
    M = api.BlockPreconditioner(ctx, gsys, "schur2")
    x, r = api.gmres(ctx, gsys, M, ctx.zeros(gsys.n))
    assert r.converged and r.iters == 0 and float(torch.abs(x).max()) == 0.0
    x, r = api.gmres(ctx, gsys, M, to_dev(ctx, inp.b), max_iters=1, rtol=1e-14)
    assert r.status == -4 and not r.converged and r.iters == 1


# ---------------------------------------------------------------------------
# FP32 hierarchy inside FP64 FGMRES
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["schur2", "schur1", "amg"])
def test_fp32_vcycle_fgmres(ctx, kind):
    api = gpu_modules()
    inp = si.generate(4, 2, 32, 51)
    osys = oracle_system(inp)
    A = osys.monolithic()
    xs = spla.spsolve(sp.csc_matrix(A), inp.b)
    co, gsys = gpu_system(ctx, inp)
    M = api.BlockPreconditioner(ctx, gsys, kind, amg_precision=1, batched=1, use_graph=1)
    xg, r = api.gmres(ctx, gsys, M, to_dev(ctx, inp.b), rtol=1e-8)
    assert r.converged
    xg = to_host(xg)
    assert np.linalg.norm(inp.b - A @ xg) <= 1e-8 * np.linalg.norm(inp.b)
    assert_elementwise(xg, xs, 1e-6, segments=inp.G + 2, what=f"FP32 {kind} solution vs direct")


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------
def test_adjoint_parity(ctx):
    api = gpu_modules()
    from oracle import adjoint as oadj
    inp = si.generate_workload("g2_2d16")
    osys = oracle_system(inp)
    A = osys.monolithic()
    x = spla.spsolve(sp.csc_matrix(A), inp.b)
    g = x - inp.x_target
    lam_o, (dk_o, dgE_o, dEg_o, dEI_o) = oadj.adjoint_direct(inp, osys, x, g)
    co, gsys = gpu_system(ctx, inp)
    MT = api.BlockPreconditioner(ctx, gsys, "schur2", transpose=1)
    lam, dk, dc, r = api.adjoint(ctx, co, gsys, MT, to_dev(ctx, x), to_dev(ctx, g), rtol=1e-13)
    assert r.converged
    assert_elementwise(to_host(lam), lam_o, 1e-10, segments=inp.G + 2, what="lambda")
    G, N = inp.G, inp.N
    dc = to_host(dc)
    assert_elementwise(to_host(dk), dk_o.reshape(-1), 1e-9, segments=G + 2, what="dL/dkappa")
    assert_elementwise(dc[:G * N], dgE_o.reshape(-1), 1e-9, segments=G, what="dL/dc_gE")
    assert_elementwise(dc[G * N:2 * G * N], dEg_o.reshape(-1), 1e-9, segments=G, what="dL/dc_Eg")
    assert_elementwise(dc[2 * G * N:], dEI_o, 1e-9, what="dL/dc_EI")


def test_transposed_system(ctx):
    inp = si.generate(2, 2, 9, 61, nonsym=True)
    osys = oracle_system(inp)
    co, gsys = gpu_system(ctx, inp)
    gt = gsys.transpose()
    x = np.random.default_rng(1).standard_normal(osys.n)
    y = to_host(gt.matvec(to_dev(ctx, x)))
    At = osys.monolithic().T
    assert_elementwise(y, At @ x, 1e-14, scale=matvec_scale(At, x), what="transposed system")


# ---------------------------------------------------------------------------
# determinism
# ---------------------------------------------------------------------------
def test_bitwise_determinism(ctx):
    api = gpu_modules()
    inp = si.generate(3, 2, 24, 71)
    outs = []
    for _ in range(2):
        co, gsys = gpu_system(ctx, inp)
        M = api.BlockPreconditioner(ctx, gsys, "schur2", batched=1)
        x, r = api.gmres(ctx, gsys, M, to_dev(ctx, inp.b), rtol=1e-9)
        outs.append((to_host(x), r.iters))
    assert outs[0][1] == outs[1][1]
    assert np.array_equal(outs[0][0], outs[1][0])


def test_autograd_solve_matches_oracle_adjoint(ctx):
    """MGDSolve's backward against the oracle's direct adjoint (splu of A^T) on
    the G=2 2D 16x16 instance, loss 0.5 ||x - x_target||^2."""
    import torch
    gpu_modules()
    from paper_2002_04958_amd.autograd import MGDSolve
    from oracle import adjoint as oadj
    inp = si.generate_workload("g2_2d16")
    osys = oracle_system(inp)
    A = osys.monolithic()
    x_o = spla.spsolve(sp.csc_matrix(A), inp.b)
    lam_o, (dk_o, dgE_o, dEg_o, dEI_o) = oadj.adjoint_direct(inp, osys, x_o, x_o - inp.x_target)
    dev = ctx.device
    leaf = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev,  # noqa: E731
                                  requires_grad=True)
    kappa, cgE, cEg, cEI, b = (leaf(inp.kappa), leaf(inp.c_gE), leaf(inp.c_Eg), leaf(inp.c_EI),
                               leaf(inp.b))
    x = MGDSolve.apply(kappa, cgE, cEg, cEI, b, inp.dim, inp.n, "schur2", 1e-13, None)
    assert_elementwise(to_host(x), x_o, 1e-11, segments=inp.G + 2, what="x")
    xt = torch.as_tensor(inp.x_target, device=dev)
    (0.5 * torch.sum((x - xt) ** 2)).backward()
    assert_elementwise(to_host(b.grad), lam_o, 1e-9, segments=inp.G + 2, what="dL/db")
    assert_elementwise(to_host(kappa.grad), dk_o, 1e-8, segments=inp.G + 2, what="dL/dkappa")
    assert_elementwise(to_host(cgE.grad), dgE_o, 1e-8, segments=inp.G, what="dL/dc_gE")
    assert_elementwise(to_host(cEg.grad), dEg_o, 1e-8, segments=inp.G, what="dL/dc_Eg")
    assert_elementwise(to_host(cEI.grad), dEI_o, 1e-8, what="dL/dc_EI")


def test_autograd_rejects_inplace_coefficient_change(ctx):
    """The coefficients the forward solve assembled from are saved for the
    backward pass: changing one in place in between makes backward raise
    instead of returning gradients of a different system."""
    import torch
    gpu_modules()
    from paper_2002_04958_amd.autograd import MGDSolve
    inp = si.generate_workload("g2_2d16")
    dev = ctx.device
    leaf = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev,  # noqa: E731
                                  requires_grad=True)
    kappa, cgE, cEg, cEI, b = (leaf(inp.kappa), leaf(inp.c_gE), leaf(inp.c_Eg), leaf(inp.c_EI),
                               leaf(inp.b))
    x = MGDSolve.apply(kappa, cgE, cEg, cEI, b, inp.dim, inp.n, "schur2", 1e-10, None)
    with torch.no_grad():
        kappa.mul_(2.0)
    with pytest.raises(RuntimeError, match="modified by an inplace operation"):
        x.sum().backward()


def test_context_memory_comes_from_torch_allocator(ctx):
    """The default context hands the library torch's caching allocator: a
    preconditioner's device memory shows in torch's allocated bytes and
    returns to torch when the handle is destroyed; a context on hipMalloc
    gives the same apply bit for bit."""
    import torch
    api = gpu_modules()
    inp = si.generate(3, 2, 32, 41)
    co, gsys = gpu_system(ctx, inp)
    r = to_dev(ctx, np.random.default_rng(4).standard_normal(gsys.n))
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated(ctx.device)
    M = api.BlockPreconditioner(ctx, gsys, "schur2", amg_seed=5, batched=1, use_graph=1)
    z = to_host(M.apply(r))
    m1 = torch.cuda.memory_allocated(ctx.device)
    assert m1 - m0 > 8 * gsys.n
    M.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(ctx.device) < m1
    hctx = api.Context(0, allocator="hip")
    hco, hsys = gpu_system(hctx, inp)
    Mh = api.BlockPreconditioner(hctx, hsys, "schur2", amg_seed=5, batched=1, use_graph=1)
    assert np.array_equal(to_host(Mh.apply(r)), z)
    Mh.close()
    hsys.close()
    hctx.close()


# ---------------------------------------------------------------------------
# persistent tail of the batched V-cycle
# ---------------------------------------------------------------------------
def _fp32_solve_outputs(api, c, A, gsys, inp, b, r):
    """V-cycles of a sliced FP32 hierarchy, two graph replays of a batched
    Schur2 apply and an FGMRES solve, on context c."""
    import torch
    g = api.AMG(c, A.indptr, A.indices, A.data, seed=1, precision=1)
    M = api.BlockPreconditioner(c, gsys, "schur2", amg_seed=5, batched=1, use_graph=1,
                                amg_precision=1)
    v3 = to_host(g.apply(to_dev(c, b), cycles=3))
    z = [to_host(M.apply(r)) for _ in range(2)]
    torch.cuda.synchronize()
    x, res = api.gmres(c, gsys, M, to_dev(c, inp.b), rtol=1e-9, flexible=1)
    out = (v3, z, to_host(x), res.iters)
    g.close()
    M.close()
    return out


def test_chiplet_row_shares_leave_results_unchanged(monkeypatch):
    """MGD_XCD_ROWS=1 (set when a context is created) hands each chiplet a
    contiguous share of the rows of every level kernel: only the workgroup
    that handles a row changes, so V-cycles, applies and the solve are the
    same bit for bit (sliced layouts forced on a small system)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    api = gpu_modules()
    monkeypatch.setenv("MGD_SELL_MIN_ROWS", "256")
    A = oracle_system(si.generate_workload("g1_2d64")).monolithic()
    inp = si.generate(3, 2, 24, 41)
    b = np.random.default_rng(2).uniform(size=A.shape[0])
    out = {}
    try:
        for mode in ("0", "1"):
            monkeypatch.setenv("MGD_XCD_ROWS", mode)
            c = api.Context(0)
            co, gsys = gpu_system(c, inp)
            r = to_dev(c, np.random.default_rng(4).standard_normal(gsys.n))
            out[mode] = _fp32_solve_outputs(api, c, A, gsys, inp, b, r)
            gsys.close()
            c.close()
    finally:
        monkeypatch.delenv("MGD_XCD_ROWS", raising=False)
        api.Context(0).close()  # the device constant back to the default
    (a3, az, ax, ai), (b3, bz, bx, bi) = out["0"], out["1"]
    assert np.array_equal(a3, b3)
    assert np.array_equal(az[0], bz[0]) and np.array_equal(az[1], bz[1])
    assert ai == bi and np.array_equal(ax, bx)


@pytest.mark.parametrize("precision", [0, 1])
def test_step_overlap_switch_leaves_solve_unchanged(ctx, monkeypatch, precision):
    """A Schur2 GMRES step splits its block matvec so that the part without
    z_E runs beside the last E solve, and a finishing kernel adds the rest in
    the order of the one-kernel matvec: with MGD_STEP_OVERLAP=0 (one kernel
    after the apply) the solve is the same bit for bit, with graph replay
    and without."""
    api = gpu_modules()
    inp = si.generate(3, 2, 24, 61)
    co, gsys = gpu_system(ctx, inp)
    b = to_dev(ctx, inp.b)
    out = {}
    for ov in ("1", "0"):
        monkeypatch.setenv("MGD_STEP_OVERLAP", ov)
        for graph in (0, 1):
            M = api.BlockPreconditioner(ctx, gsys, "schur2", amg_seed=6, batched=1,
                                        use_graph=graph, amg_precision=precision)
            x, r = api.gmres(ctx, gsys, M, b, rtol=1e-9, flexible=1)
            assert r.converged
            out[(ov, graph)] = (to_host(x), r.iters)
            M.close()
    ref = out[("1", 1)]
    for k, v in out.items():
        assert v[1] == ref[1] and np.array_equal(v[0], ref[0]), k


@pytest.mark.parametrize("dim,n,nonsym", [(3, 16, False), (2, 40, False), (3, 16, True)])
def test_half_storage_block_matvec_is_bit_exact(ctx, monkeypatch, dim, n, nonsym):
    """An assembled system whose blocks equal their transposes bit for bit gets
    a half storage for the block matvec: each block's values on and above the
    diagonal, an entry below it reading its mirror's (from LDS inside the
    workgroup's rows, from memory across them: 16^3 and 40^2 meshes put the
    -z and -y mirrors on both sides of a 512-row tile).  y = A x, FGMRES with
    a graph-replayed batched Schur2 (the split matvec and its finishing pass)
    and the adjoint solve on the transposed system equal those of the full
    storage (MGD_SYM_MATVEC=0) bit for bit, and the profiled bytes of the
    matvec show which storage ran.  The nonsymmetric variant keeps the full
    storage."""
    api = gpu_modules()
    G = 3
    inp = si.generate(G, dim, n, 71, nonsym=nonsym)
    N = n ** dim
    A0 = sp.csr_matrix(oracle_system(inp).blocks[0])
    rows = np.repeat(np.arange(N), np.diff(A0.indptr))
    nnz0, unnz = A0.nnz, int(np.count_nonzero(A0.indices >= rows))
    rest = 4.0 * nnz0 + 4.0 * (N + 1) + 8.0 * (2 * G + 2) * N + 16.0 * (G + 2) * N
    full = 8.0 * nnz0 * (G + 2) + rest
    half = 8.0 * unnz * (G + 2) + 4.0 * nnz0 + 4.0 * (N + 1) + rest
    rng = np.random.default_rng(8)
    x = to_dev(ctx, rng.standard_normal((G + 2) * N))
    b = to_dev(ctx, inp.b)
    out = {}
    for sym in ("1", "0"):
        monkeypatch.setenv("MGD_SYM_MATVEC", sym)
        co, gsys = gpu_system(ctx, inp)
        ctx.reset_kernel_stats()
        ctx.set_profiling(True)
        y = to_host(gsys.matvec(x))
        ctx.set_profiling(False)
        name = "k_block_matvec_shared<512, false, false, %s>" % (
            "true" if sym == "1" and not nonsym else "false")
        st = ctx.kernel_symbol_stats()[name]
        M = api.BlockPreconditioner(ctx, gsys, "schur2", amg_seed=6, batched=1, use_graph=1,
                                    amg_precision=1)
        xs, r = api.gmres(ctx, gsys, M, b, rtol=1e-9, flexible=1)
        assert r.converged
        adj = (None,) * 4
        if not nonsym:  # the gradients are those of the symmetric assembly
            MT = api.BlockPreconditioner(ctx, gsys, "schur2", amg_seed=6, transpose=1)
            lam, dk, dc, ra = api.adjoint(ctx, co, gsys, MT, xs, xs - b, rtol=1e-10)
            adj = (to_host(lam), ra.iters, to_host(dk), to_host(dc))
            MT.close()
        out[sym] = (y, st["bytes"] / st["launches"], to_host(xs), r.iters) + adj
        M.close()
        gsys.close()
    on, off = out["1"], out["0"]
    assert off[1] == pytest.approx(full)
    assert on[1] == pytest.approx(full if nonsym else half)
    for k in (0, 2) if nonsym else (0, 2, 4, 6, 7):
        assert np.array_equal(on[k], off[k]), k
    assert on[3] == off[3] and on[5] == off[5]


@pytest.mark.parametrize("kind", ["schur2", "schur1", "pctl", "bdiag"])
def test_stored_order_group_output_leaves_solve_unchanged(ctx, monkeypatch, kind):
    """A batched group of single V-cycles leaves its result in the union's
    stored order (the last C half-sweep in place), and the kernel that spreads
    the members over the block vector reads each row at its stored position:
    with MGD_STORED_OUT=0 (the last half-sweep writes the natural order, the
    spreading kernel reads it there) FGMRES gives the same solution bit for
    bit, in FP64 and FP32, with graph replay and without."""
    api = gpu_modules()
    inp = si.generate(3, 2, 24, 67)
    co, gsys = gpu_system(ctx, inp)
    b = to_dev(ctx, inp.b)
    for precision in (0, 1):
        out = {}
        for so in ("1", "0"):
            monkeypatch.setenv("MGD_STORED_OUT", so)
            for graph in (0, 1):
                M = api.BlockPreconditioner(ctx, gsys, kind, amg_seed=6, batched=1,
                                            use_graph=graph, amg_precision=precision)
                x, r = api.gmres(ctx, gsys, M, b, rtol=1e-9, flexible=1)
                assert r.converged
                out[(so, graph)] = (to_host(x), r.iters)
                M.close()
        ref = out[("1", 1)]
        for k, v in out.items():
            assert v[1] == ref[1] and np.array_equal(v[0], ref[0]), (precision, k)


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("blocks", ["3", "256"])
@pytest.mark.parametrize("precision", [0, 1])
def test_persistent_tail_matches_level_launches(ctx, monkeypatch, precision, blocks):
    """The levels below MGD_TAIL_ROWS run as one persistent launch whose
    phases are separated by a grid-wide barrier.  It computes what the
    per-level launches compute, bit for bit: V-cycles of a monolithic
    hierarchy, and a batched, graph-replayed Schur2 apply and FGMRES solve
    (three workgroups make every phase loop over its rows several times)."""
    import torch
    api = gpu_modules()
    A = oracle_system(si.generate_workload("g1_2d64")).monolithic()
    inp = si.generate(3, 2, 24, 41)
    co, gsys = gpu_system(ctx, inp)
    b = np.random.default_rng(2).uniform(size=A.shape[0])
    r = to_dev(ctx, np.random.default_rng(4).standard_normal(gsys.n))
    out = {}
    for mode in ("levels", "tail"):
        monkeypatch.setenv("MGD_TAIL_ROWS", "0" if mode == "levels" else "65536")
        monkeypatch.setenv("MGD_TAIL_BLOCKS", blocks)
        g = api.AMG(ctx, A.indptr, A.indices, A.data, seed=1, precision=precision)
        M = api.BlockPreconditioner(ctx, gsys, "schur2", amg_seed=5, batched=1, use_graph=1,
                                    amg_precision=precision)
        ctx.reset_kernel_stats()
        ctx.set_profiling(True)
        v1 = to_host(g.apply(to_dev(ctx, b)))
        ctx.set_profiling(False)
        tails = [k for k in ctx.kernel_symbol_stats() if k.startswith("k_tail")]
        assert bool(tails) == (mode == "tail"), tails
        v3 = to_host(g.apply(to_dev(ctx, b), cycles=3))
        z = [to_host(M.apply(r)) for _ in range(2)]      # graph replays
        torch.cuda.synchronize()
        x, res = api.gmres(ctx, gsys, M, to_dev(ctx, inp.b), rtol=1e-9, flexible=1)
        out[mode] = (v1, v3, z, to_host(x), res.iters)
        g.close()
        M.close()
    (a1, a3, az, ax, ai), (b1, b3, bz, bx, bi) = out["levels"], out["tail"]
    assert np.array_equal(a1, b1) and np.array_equal(a3, b3)
    assert np.array_equal(az[0], bz[0]) and np.array_equal(az[1], bz[1])
    assert np.array_equal(az[0], az[1])
    assert ai == bi and np.array_equal(ax, bx)


# ---------------------------------------------------------------------------
# level-layout autotuning
# ---------------------------------------------------------------------------
_AUTOTUNE_CHILD = r"""
import sys, numpy as np, torch
sys.path.insert(0, sys.argv[1])
import synth_inputs as si
from oracle import assemble as oasm
from paper_2002_04958_amd import api
inp = si.generate(2, 2, 22, 77)
A = oasm.assemble(inp).monolithic()
ctx = api.Context(0)
g = api.AMG(ctx, A.indptr, A.indices, A.data, seed=3, precision=int(sys.argv[3]), autotune=0)
b = np.random.default_rng(5).uniform(size=A.shape[0])
z = g.apply(torch.as_tensor(b, device=ctx.device), cycles=2).cpu().numpy()
np.save(sys.argv[2], z)
"""


_DEBUG_UNION_CHILD = r"""
import sys, numpy as np, torch
sys.path.insert(0, sys.argv[1])
import synth_inputs as si
from paper_2002_04958_amd import api
inp = si.generate(3, 2, 24, 41)
ctx = api.Context(0)
co = api.Coeffs.from_inputs(ctx, inp)
sysg = api.BlockSystem.assemble(ctx, co)
M = api.BlockPreconditioner(ctx, sysg, "schur2", amg_seed=5, batched=1, use_graph=0,
                            amg_precision=1)
r = torch.as_tensor(np.random.default_rng(4).standard_normal(sysg.n), device=ctx.device)
np.save(sys.argv[2], M.apply(r).cpu().numpy())
"""


def test_debug_union_verification_passes(ctx, monkeypatch, tmp_path):
    """MGD_DEBUG_UNION=1 (read once per process) verifies every level of every
    union on the host while it is built: the stored-row map is a permutation
    and every copied row equals its source row.  A child process builds a
    batched FP32 Schur2 preconditioner with sliced layouts that way, and its
    apply equals this process's bit for bit."""
    import os
    import subprocess
    import sys
    api = gpu_modules()
    monkeypatch.setenv("MGD_SELL_MIN_ROWS", "256")
    inp = si.generate(3, 2, 24, 41)
    co, gsys = gpu_system(ctx, inp)
    M = api.BlockPreconditioner(ctx, gsys, "schur2", amg_seed=5, batched=1, use_graph=0,
                                amg_precision=1)
    r = to_dev(ctx, np.random.default_rng(4).standard_normal(gsys.n))
    z = to_host(M.apply(r))
    M.close()
    out = tmp_path / "child.npy"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, MGD_DEBUG_UNION="1")
    p = subprocess.run([sys.executable, "-c", _DEBUG_UNION_CHILD, root, str(out)],
                       capture_output=True, text=True, timeout=240, env=env)
    assert p.returncode == 0, p.stderr[-2000:]
    assert np.array_equal(np.load(out), z)


@pytest.mark.parametrize("precision", [0, 1])
def test_autotune_layouts_and_cache(ctx, monkeypatch, tmp_path, precision):
    """autotune = 1 times every level matrix's and every restriction's layouts
    (SELL, CSR with 1-32 lanes per row) with 64, 128 and 256 threads per
    workgroup and keeps the fastest (MGD_TUNE_MIN_ROWS=1: every matrix of this
    small system is timed): the tuned V-cycles agree with the oracle, the
    choices are written to MGD_AUTOTUNE_CACHE, and a fresh process that reads
    the file (autotune off) builds the same layouts, so its result equals this
    one bit for bit."""
    import json
    import os
    import subprocess
    import sys
    api = gpu_modules()
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("MGD_AUTOTUNE_CACHE", str(cache))
    monkeypatch.setenv("MGD_TUNE_MIN_ROWS", "1")
    inp = si.generate(2, 2, 22, 77)
    A = oracle_system(inp).monolithic()
    H = oamg.setup(A, oamg.AMGParams(seed=3))
    g = api.AMG(ctx, A.indptr, A.indices, A.data, seed=3, precision=precision, autotune=1)
    b = np.random.default_rng(5).uniform(size=A.shape[0])
    z = to_host(g.apply(to_dev(ctx, b), cycles=2))
    assert_elementwise(z, oamg.apply_cycles(H, b, 2), 1e-12 if precision == 0 else 5e-5,
                       floor=(FP32_FLOOR if precision else 1e-3), what="autotuned V-cycles")
    tuned = json.loads(cache.read_text())
    mine = {k: v for k, v in tuned.items() if k.startswith("f32:" if precision else "f64:")}
    levels = g.info()["levels"]
    assert len([k for k in mine if ":wt:" not in k]) >= levels - 1, tuned
    assert len([k for k in mine if ":wt:" in k]) >= levels - 2, tuned
    for v in mine.values():
        code, units = v % 100000, v // 100000
        assert units in (1, 2, 4) and (code == 1000 or code in (1, 2, 4, 8, 16, 32)), v
    out = tmp_path / "child.npy"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, "-c", _AUTOTUNE_CHILD, root, str(out), str(precision)],
                       capture_output=True, text=True, timeout=240, env=dict(os.environ))
    assert p.returncode == 0, p.stderr[-2000:]
    assert np.array_equal(np.load(out), z)
