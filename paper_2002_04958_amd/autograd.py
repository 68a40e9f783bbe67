"""Differentiable solve x = A(kappa, c)^{-1} b of the block system (eq. 2.2).

Forward: assemble the system from the per-cell coefficients, build the chosen
block preconditioner (Section 3) and solve by (F)GMRES, all in libmgdamg.
Backward: one adjoint solve A^T lambda = dL/dx with the same preconditioner
kind built on A^T, then the coefficient gradients obtained by differentiating
the assembly: a face transmissibility T adds +T to both diagonal entries and
-T to both off-diagonal entries of its two cells, so dL/dT = -(lam_i - lam_j)
(x_i - x_j), carried to the two cells' kappa through the harmonic mean; a
coupling coefficient c between rows (alpha, k) and (beta, k) contributes
-lam_(alpha,k) (x_(alpha,k) - x_(beta,k)).  dL/db = lambda.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import api

_CONTEXTS: dict = {}


def _context(device: torch.device) -> api.Context:
    idx = device.index if device.index is not None else torch.cuda.current_device()
    key = (idx, torch.cuda.current_stream(idx).cuda_stream)
    ctx = _CONTEXTS.get(key)
    if ctx is None:
        ctx = api.Context(idx)
        _CONTEXTS[key] = ctx
    return ctx


class MGDSolve(torch.autograd.Function):
    """x = MGDSolve.apply(kappa, c_gE, c_Eg, c_EI, b, dim, n, kind, rtol, options)

    kappa (G+2, N), c_gE and c_Eg (G, N), c_EI (N,), b ((G+2) N,): FP64 CUDA
    tensors on one device, N = n**dim.  kind is a preconditioner name
    ("amg", "bdiag", "pctl", "schur1", "schur2", "schur2_lower"); options is
    an optional dict of block_params keywords (e.g. amg_precision=1,
    batched=1, use_graph=1; FP32 hierarchies need flexible GMRES, which is
    always used here).  Raises RuntimeError if a solve does not converge.
    """

    @staticmethod
    def forward(fctx, kappa, c_gE, c_Eg, c_EI, b, dim: int, n: int, kind: str = "schur2",
                rtol: float = 1e-8, options: Optional[dict] = None):
        if not kappa.is_cuda:
            raise ValueError("MGDSolve runs on the GPU: pass CUDA tensors")
        if any(t.dtype != torch.float64 for t in (kappa, c_gE, c_Eg, c_EI, b)):
            raise ValueError("MGDSolve takes float64 tensors")
        G = int(kappa.shape[0]) - 2
        N = n ** dim
        if kappa.numel() != (G + 2) * N or c_gE.numel() != G * N or c_Eg.numel() != G * N \
                or c_EI.numel() != N or b.numel() != (G + 2) * N:
            raise ValueError("coefficient or right-hand-side sizes do not match G, dim, n")
        ctx = _context(kappa.device)
        f64 = lambda t: t.detach().to(torch.float64).reshape(-1).contiguous()  # noqa: E731
        coeffs = api.Coeffs(dim, n, G, f64(kappa), f64(c_gE), f64(c_Eg), f64(c_EI))
        system = api.BlockSystem.assemble(ctx, coeffs)
        opts = dict(options or {})
        M = api.BlockPreconditioner(ctx, system, kind, **opts)
        x, res = api.gmres(ctx, system, M, f64(b), rtol=rtol, flexible=1)
        if not res.converged:
            raise RuntimeError(f"forward GMRES did not converge: {res}")
        fctx.state = (ctx, coeffs, system, kind, opts, rtol, G, N,
                      (kappa.shape, c_gE.shape, c_Eg.shape, c_EI.shape, b.shape))
        # the assembled system and coeffs view the caller's coefficient
        # tensors: saving them lets autograd's version check reject an
        # in-place change between forward and backward
        fctx.save_for_backward(x, kappa, c_gE, c_Eg, c_EI)
        return x

    @staticmethod
    def backward(fctx, grad_x):
        x = fctx.saved_tensors[0]
        ctx, coeffs, system, kind, opts, rtol, G, N, shapes = fctx.state
        MT = api.BlockPreconditioner(ctx, system, kind, transpose=1, **opts)
        g = grad_x.detach().to(torch.float64).contiguous()
        lam, dk, dc, res = api.adjoint(ctx, coeffs, system, MT, x, g, rtol=rtol, flexible=1)
        if not res.converged:
            raise RuntimeError(f"adjoint GMRES did not converge: {res}")
        need = fctx.needs_input_grad
        d_kappa = dk.reshape(shapes[0]) if need[0] else None
        d_gE = dc[:G * N].reshape(shapes[1]) if need[1] else None
        d_Eg = dc[G * N:2 * G * N].reshape(shapes[2]) if need[2] else None
        d_EI = dc[2 * G * N:].reshape(shapes[3]) if need[3] else None
        d_b = lam.reshape(shapes[4]) if need[4] else None
        return d_kappa, d_gE, d_Eg, d_EI, d_b, None, None, None, None, None


def solve(kappa, c_gE, c_Eg, c_EI, b, dim: int, n: int, kind: str = "schur2",
          rtol: float = 1e-8, **options):
    """Functional form of MGDSolve.apply."""
    return MGDSolve.apply(kappa, c_gE, c_Eg, c_EI, b, dim, n, kind, rtol, options or None)
