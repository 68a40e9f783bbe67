"""Shared helpers for the GPU parity tests (oracle on the CPU, library on the GPU)."""
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
    d = np.linalg.norm(a - b)
    s = np.linalg.norm(b)
    return d / s if s > 0 else d


def oracle_params(**kw):
    return oamg.AMGParams(**kw)


def small_inputs():
    return [("g1_2d12", si.generate(1, 2, 12, 21)),
            ("g2_2d16", si.generate_workload("g2_2d16")),
            ("g3_3d6", si.generate(3, 3, 6, 22)),
            ("g2_2d10_nonsym", si.generate(2, 2, 10, 23, nonsym=True))]
