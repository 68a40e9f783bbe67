"""gmres_solve_noalloc (the GMRES entry point that allocates nothing: its
workspace is the library's static per-device array) against gmres_solve,
through the C ABI."""
import numpy as np
import pytest

import synth_inputs as si

from gpu_helpers import assert_elementwise, gpu_modules, gpu_system, to_dev, to_host

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


def _pair(ctx, inp, kind, precision, flexible, use_graph):
    """gmres_solve, then gmres_solve_noalloc on the same system, preconditioner
    and right-hand side; the second call must not change torch's allocated
    bytes (the library's memory comes from torch's allocator)."""
    import torch
    api = gpu_modules()
    co, gsys = gpu_system(ctx, inp)
    M = api.BlockPreconditioner(ctx, gsys, kind, amg_seed=5, batched=1, use_graph=use_graph,
                                amg_precision=precision)
    b = to_dev(ctx, inp.b)
    x_ref, r_ref = api.gmres(ctx, gsys, M, b, rtol=1e-9, flexible=flexible)
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated(ctx.device)
    x, r = api.gmres_noalloc(ctx, gsys, M, b, x, rtol=1e-9, flexible=flexible)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(ctx.device) == m0
    return inp, x_ref, r_ref, x, r


@pytest.mark.parametrize("kind,precision,flexible", [("schur2", 1, 1), ("schur2", 0, 1),
                                                     ("amg", 0, 0)])
def test_noalloc_equals_gmres_solve_two_calls(ctx, kind, precision, flexible):
    """Two calls in a row, the second on a smaller system: with direct launches
    on both sides the solutions are equal bit for bit, with the same iteration
    count and residuals."""
    for inp in (si.generate(3, 2, 24, 41), si.generate(2, 2, 12, 42)):
        inp, x_ref, r_ref, x, r = _pair(ctx, inp, kind, precision, flexible, use_graph=0)
        assert r.status == r_ref.status == 0 and r.converged
        assert r.iters == r_ref.iters and r.restarts == r_ref.restarts
        assert r.relres_true == r_ref.relres_true and r.relres_est == r_ref.relres_est
        assert np.array_equal(to_host(x), to_host(x_ref))


def test_noalloc_with_a_graph_replayed_preconditioner(ctx):
    """A preconditioner made for graph replay is applied by direct launches in
    the no-allocation call: the same iteration count and the solution to the
    FP64 parity bar."""
    inp, x_ref, r_ref, x, r = _pair(ctx, si.generate(3, 2, 20, 43), "schur2", 0, 1, use_graph=1)
    assert r.converged and r.iters == r_ref.iters
    assert_elementwise(to_host(x), to_host(x_ref), 1e-10, segments=inp.G + 2,
                       what="no-allocation solution")


def test_noalloc_rejects_what_it_cannot_hold(ctx):
    """Per-phase profiling, and a system whose Krylov basis exceeds the static
    array (2D 128^2, G = 20: 360,448 unknowns, V alone 89 MB), are refused
    with MGD_EINVAL before anything is launched."""
    api = gpu_modules()
    from paper_2002_04958_amd._lib import MgdError
    inp = si.generate(2, 2, 12, 42)
    co, gsys = gpu_system(ctx, inp)
    M = api.BlockPreconditioner(ctx, gsys, "schur2", amg_seed=5, batched=1)
    with pytest.raises(MgdError, match="EINVAL.*profiling"):
        api.gmres_noalloc(ctx, gsys, M, to_dev(ctx, inp.b), rtol=1e-8, profile=1)
    big = si.generate(20, 2, 128, 45)
    co2, gsys2 = gpu_system(ctx, big)
    with pytest.raises(MgdError, match="EINVAL.*no-allocation workspace"):
        api.gmres_noalloc(ctx, gsys2, None, to_dev(ctx, big.b), rtol=1e-8)
