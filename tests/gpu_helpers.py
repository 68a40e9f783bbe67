"""Shared helpers for the GPU parity tests (oracle on the CPU, library on the GPU)."""
import json
import os

import numpy as np
import scipy.sparse as sp

import synth_inputs as si
from oracle import amg as oamg
from oracle import assemble as oasm


def gpu_modules():
    import torch  # noqa: F401
    from paper_2002_04958_amd import api
    return api


def oracle_system(inp):
    return oasm.assemble(inp)


def gpu_system(ctx, inp):
    api = gpu_modules()
    co = api.Coeffs.from_inputs(ctx, inp)
    return co, api.BlockSystem.assemble(ctx, co)


def csr_of(arrs, n):
    rp, ci, v = arrs
    A = sp.csr_matrix((v, ci, rp), shape=(n, n))
    return A


def to_dev(ctx, x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).to(ctx.device)


def to_host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    """Relative 2-norm difference; reported alongside, never the parity bar."""
    d = np.linalg.norm(a - b)
    s = np.linalg.norm(b)
    return d / s if s > 0 else d


def elementwise_ratio(a, ref, *, segments=1, floor=1e-3, scale=None):
    """max_i |a_i - ref_i| / s_i with s_i = max(|ref_i|, floor * max_{j in seg(i)} |ref_j|)
    over the block segments of the vector, or s_i = scale_i when given."""
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1)
    assert a.shape == ref.shape, (a.shape, ref.shape)
    if a.size == 0:
        return 0.0, -1
    if scale is None:
        R = np.abs(ref).reshape(segments, -1)
        s = np.maximum(R, floor * R.max(axis=1, keepdims=True)).reshape(-1)
    else:
        s = np.asarray(scale, dtype=np.float64).reshape(-1)
    err = np.abs(a - ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        q = np.where(err == 0.0, 0.0, err / s)
    i = int(np.argmax(q))
    return float(q[i]), i


def assert_elementwise(a, ref, tol, *, segments=1, floor=1e-3, scale=None, what=""):
    """Every entry within tol of the reference, relative to its own size, with
    a floor of `floor` times its block segment's largest entry (entries near a
    zero crossing are compared at that scale); `scale` overrides the
    per-entry scale (e.g. sum_j |a_ij x_j| for a matrix-vector product)."""
    q, i = elementwise_ratio(a, ref, segments=segments, floor=floor, scale=scale)
    _record(what, q, tol)
    if not q <= tol:
        a = np.asarray(a).reshape(-1)
        ref = np.asarray(ref).reshape(-1)
        raise AssertionError(f"{what}: entry {i}: {a[i]!r} vs {ref[i]!r}, scaled difference "
                             f"{q:.3e} > {tol:.1e} (2-norm rel {rel(a, ref):.3e})")


def matvec_scale(A, x):
    """sum_j |a_ij| |x_j|: the scale of the rounding error of (A x)_i."""
    return abs(A) @ np.abs(x)


def _record(what, q, tol):
    """With MGD_PARITY_LOG set, append the scaled difference of each check
    (for choosing and reviewing tolerances)."""
    path = os.environ.get("MGD_PARITY_LOG")
    if path:
        test = os.environ.get("PYTEST_CURRENT_TEST", "").split(" ")[0]
        with open(path, "a") as f:
            f.write(json.dumps({"test": test, "what": what, "ratio": q, "tol": tol}) + "\n")


def oracle_params(**kw):
    return oamg.AMGParams(**kw)


def small_inputs():
    return [("g1_2d12", si.generate(1, 2, 12, 21)),
            ("g2_2d16", si.generate_workload("g2_2d16")),
            ("g3_3d6", si.generate(3, 3, 6, 22)),
            ("g2_2d10_nonsym", si.generate(2, 2, 10, 23, nonsym=True))]
