"""Python binding of libmgdamg: the C ABI with torch tensors as device memory.

Only argument marshalling happens here; every numerical step runs in the
library's HIP kernels.  There is no CPU fallback: without the built library
every entry point raises LibraryMissing.
"""
from __future__ import annotations

import atexit
import ctypes
import weakref
from ctypes import byref, c_double, c_int64, c_void_p
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L

__all__ = ["Context", "Coeffs", "BlockSystem", "AMG", "BlockPreconditioner", "GmresResult",
           "gmres", "gmres_noalloc", "adjoint", "adjoint_gradients", "csr_spmv", "PC_KINDS"]

PC_KINDS = L.PC_KINDS


def _p(t: Optional[torch.Tensor]):
    return c_void_p(t.data_ptr()) if t is not None else None


def _dev_f64(x, device) -> torch.Tensor:
    t = torch.as_tensor(x)
    return t.to(device=device, dtype=torch.float64).contiguous()


def _dev_i32(x, device) -> torch.Tensor:
    t = torch.as_tensor(x)
    return t.to(device=device, dtype=torch.int32).contiguous()


def _torch_allocator(device: int):
    """mgd_allocator callbacks that take the library's device memory from
    torch's caching allocator on the context stream (memory the library frees
    returns to torch's pool, ordered on that stream)."""
    def alloc(nbytes, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, int(stream or 0))
        except Exception:
            return None          # the library reports MGD_ENOMEM

    def free(ptr, stream, user):
        try:
            torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:
            pass                 # interpreter shutdown: the process frees it

    cbs = (L.ALLOC_FN(alloc), L.FREE_FN(free))
    return cbs, L.mgd_allocator(cbs[0], cbs[1], None)


_LIVE_CONTEXTS = weakref.WeakSet()


@atexit.register
def _close_all_contexts():
    """Release every handle and context while the interpreter and torch are
    still whole (finalizers at shutdown run in no defined order)."""
    for c in list(_LIVE_CONTEXTS):
        try:
            c.close()
        except Exception:
            pass


class Context:
    """Device, stream and library context.  The stream defaults to torch's
    current stream on the device, so library work and torch work are ordered.
    allocator="torch" (default) hands the library torch's caching allocator
    for all device memory it owns; "hip" leaves it on hipMalloc/hipFree."""

    def __init__(self, device: int = 0, stream: Optional[torch.cuda.Stream] = None,
                 allocator: str = "torch"):
        self.lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device is visible")
        if allocator not in ("torch", "hip"):
            raise ValueError("allocator must be 'torch' or 'hip'")
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._alloc_cbs, alloc = (_torch_allocator(device) if allocator == "torch"
                                  else (None, None))
        h = c_void_p()
        L.check(self.lib.mgd_ctx_create(device, c_void_p(self.stream.cuda_stream),
                                        byref(alloc) if alloc is not None else None, byref(h)))
        self.h = h
        self._children = weakref.WeakSet()
        _LIVE_CONTEXTS.add(self)

    def _adopt(self, obj):
        """Handles made on this context are closed before it (preconditioners,
        then hierarchies, then systems), whatever order their finalizers run in."""
        self._children.add(obj)

    def synchronize(self):
        L.check(self.lib.mgd_ctx_synchronize(self.h))

    def close(self):
        if getattr(self, "h", None):
            order = {"BlockPreconditioner": 0, "AMG": 1, "BlockSystem": 2}
            for ch in sorted(list(getattr(self, "_children", ())),
                             key=lambda o: order.get(type(o).__name__, 3)):
                ch.close()
            self.lib.mgd_ctx_destroy(self.h)
            self.h = None

    @property
    def alive(self) -> bool:
        return bool(getattr(self, "h", None))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- kernel-class timing ------------------------------------------------------
    def set_profiling(self, on: bool):
        L.check(self.lib.mgd_ctx_set_profiling(self.h, 1 if on else 0))

    def reset_kernel_stats(self):
        L.check(self.lib.mgd_ctx_reset_kernel_stats(self.h))

    def kernel_stats(self) -> dict:
        out = {}
        for c in range(self.lib.mgd_kernel_class_count()):
            n, ms, by = c_int64(), c_double(), c_double()
            L.check(self.lib.mgd_ctx_kernel_stats(self.h, c, byref(n), byref(ms), byref(by)))
            out[self.lib.mgd_kernel_class_name(c).decode()] = {
                "launches": n.value, "ms": ms.value, "bytes": by.value}
        return out

    def kernel_symbol_stats(self) -> dict:
        """Per-kernel-symbol launches, total ms and algorithmic bytes (stored
        layout, and the same launches priced as plain CSR)."""
        cnt = ctypes.c_int()
        L.check(self.lib.mgd_ctx_kernel_symbol_count(self.h, byref(cnt)))
        out = {}
        buf = ctypes.create_string_buffer(256)
        for i in range(cnt.value):
            n, ms, by, bc = c_int64(), c_double(), c_double(), c_double()
            L.check(self.lib.mgd_ctx_kernel_symbol_stats(self.h, i, buf, 256, byref(n), byref(ms),
                                                         byref(by), byref(bc)))
            out[buf.value.decode()] = {"launches": n.value, "ms": ms.value, "bytes": by.value,
                                       "bytes_csr": bc.value}
        return out

    def empty(self, n, dtype=torch.float64):
        return torch.empty(n, dtype=dtype, device=self.device)

    def zeros(self, n, dtype=torch.float64):
        return torch.zeros(n, dtype=dtype, device=self.device)


@dataclass
class Coeffs:
    """Per-cell coefficients on the device (see mgd_coeffs)."""
    dim: int
    n: int
    G: int
    kappa: torch.Tensor
    c_gE: torch.Tensor
    c_Eg: torch.Tensor
    c_EI: torch.Tensor
    mass: float = 1.0
    xi: Optional[torch.Tensor] = None

    @staticmethod
    def from_inputs(ctx: Context, inp) -> "Coeffs":
        d = ctx.device
        return Coeffs(inp.dim, inp.n, inp.G, _dev_f64(inp.kappa.reshape(-1), d),
                      _dev_f64(inp.c_gE.reshape(-1), d), _dev_f64(inp.c_Eg.reshape(-1), d),
                      _dev_f64(inp.c_EI, d), float(inp.mass),
                      None if inp.xi is None else _dev_f64(inp.xi.reshape(-1), d))

    @property
    def N(self):
        return self.n ** self.dim

    def c_struct(self) -> L.mgd_coeffs:
        return L.mgd_coeffs(self.dim, self.n, self.G, _p(self.kappa), _p(self.c_gE),
                            _p(self.c_Eg), _p(self.c_EI), self.mass, _p(self.xi))


class BlockSystem:
    """The block system of eq. 2.2 (library-owned after assemble, or a view of
    caller tensors)."""

    def __init__(self, ctx: Context):
        self.ctx = ctx
        self.s = L.mgd_block_system()
        self._owned = False
        self._keep = []
        ctx._adopt(self)

    @staticmethod
    def assemble(ctx: Context, coeffs: Coeffs) -> "BlockSystem":
        bs = BlockSystem(ctx)
        cs = coeffs.c_struct()
        L.check(ctx.lib.mgd_assemble(ctx.h, byref(cs), byref(bs.s)))
        bs._owned = True
        bs._keep = [coeffs]
        return bs

    @staticmethod
    def from_tensors(ctx: Context, G: int, N: int, blocks: Sequence, d_gE, d_Eg, d_EI,
                     d_IE) -> "BlockSystem":
        """blocks: G+2 tuples (row_ptr, col_idx, val) of device tensors."""
        bs = BlockSystem(ctx)
        arr = (L.mgd_csr * (G + 2))()
        keep = []
        for a, (rp, ci, v) in enumerate(blocks):
            rp, ci, v = _dev_i32(rp, ctx.device), _dev_i32(ci, ctx.device), _dev_f64(v, ctx.device)
            keep += [rp, ci, v]
            arr[a] = L.mgd_csr(N, N, int(v.numel()), _p(rp), _p(ci), _p(v))
        cpl = [_dev_f64(x, ctx.device).reshape(-1) for x in (d_gE, d_Eg, d_EI, d_IE)]
        keep += cpl + [arr]
        bs.s = L.mgd_block_system(G, N, ctypes.cast(arr, ctypes.POINTER(L.mgd_csr)),
                                  _p(cpl[0]), _p(cpl[1]), _p(cpl[2]), _p(cpl[3]))
        bs._keep = keep
        return bs

    def transpose(self) -> "BlockSystem":
        bt = BlockSystem(self.ctx)
        L.check(self.ctx.lib.mgd_block_system_transpose(self.ctx.h, byref(self.s), byref(bt.s)))
        bt._owned = True
        return bt

    @property
    def G(self):
        return self.s.G

    @property
    def N(self):
        return self.s.N

    @property
    def n(self):
        return (self.s.G + 2) * self.s.N

    def block_arrays(self, a: int):
        """(row_ptr, col_idx, val) of block a copied to host numpy arrays."""
        b = self.s.blocks[a]
        rp = _copy_from_ptr(b.row_ptr, b.n_rows + 1, torch.int32, self.ctx)
        ci = _copy_from_ptr(b.col_idx, b.nnz, torch.int32, self.ctx)
        v = _copy_from_ptr(b.val, b.nnz, torch.float64, self.ctx)
        return rp, ci, v

    def couplings(self):
        G, N = self.G, self.N
        return tuple(_copy_from_ptr(p, m, torch.float64, self.ctx)
                     for p, m in ((self.s.d_gE, G * N), (self.s.d_Eg, G * N),
                                  (self.s.d_EI, N), (self.s.d_IE, N)))

    def matvec(self, x: torch.Tensor, y: Optional[torch.Tensor] = None) -> torch.Tensor:
        y = self.ctx.empty(self.n) if y is None else y
        L.check(self.ctx.lib.mgd_block_matvec(self.ctx.h, byref(self.s), _p(x), _p(y)))
        return y

    def close(self):
        if self._owned and self.s.blocks and self.ctx.alive:
            self.ctx.lib.mgd_block_system_free(self.ctx.h, byref(self.s))
        self._owned = False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _copy_from_ptr(ptr, count, dtype, ctx) -> np.ndarray:
    """Device array at a raw pointer -> host numpy copy (via the HIP runtime)."""
    out = torch.empty(int(count), dtype=dtype)
    if count:
        ctx.synchronize()
        nbytes = int(count) * out.element_size()
        hip = _hip()
        st = hip.hipMemcpy(c_void_p(out.data_ptr()), c_void_p(ptr), ctypes.c_size_t(nbytes), 2)
        if st != 0:
            raise RuntimeError(f"hipMemcpy failed with {st}")
    return out.numpy()


_HIP = None


def _hip():
    global _HIP
    if _HIP is None:
        _HIP = ctypes.CDLL("libamdhip64.so")
        _HIP.hipMemcpy.restype = ctypes.c_int
        _HIP.hipMemcpy.argtypes = [c_void_p, c_void_p, ctypes.c_size_t, ctypes.c_int]
    return _HIP


def csr_spmv(ctx: Context, rp, ci, v, n_cols: int, x: torch.Tensor) -> torch.Tensor:
    rp, ci, v = _dev_i32(rp, ctx.device), _dev_i32(ci, ctx.device), _dev_f64(v, ctx.device)
    n = rp.numel() - 1
    A = L.mgd_csr(n, n_cols, v.numel(), _p(rp), _p(ci), _p(v))
    y = ctx.empty(n)
    L.check(ctx.lib.mgd_csr_spmv(ctx.h, byref(A), _p(x), _p(y)))
    ctx.synchronize()
    return y


def amg_params(**kw) -> L.amg_params:
    p = L.amg_params()
    L.load().amg_params_default(byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


class AMG:
    """A classical AMG hierarchy built on the device."""

    def __init__(self, ctx: Context, rp, ci, v, n: Optional[int] = None, *, _handle=None,
                 _owner=None, **params):
        self.ctx = ctx
        self._owner = _owner
        if _handle is not None:
            self.h = _handle
            self._owned = False
            return
        rp, ci, v = _dev_i32(rp, ctx.device), _dev_i32(ci, ctx.device), _dev_f64(v, ctx.device)
        n = rp.numel() - 1 if n is None else n
        A = L.mgd_csr(n, n, v.numel(), _p(rp), _p(ci), _p(v))
        self.params = amg_params(**params)
        h = c_void_p()
        L.check(ctx.lib.amg_setup(ctx.h, byref(A), byref(self.params), byref(h)))
        self.h = h
        self._owned = True
        ctx._adopt(self)

    def apply(self, r: torch.Tensor, z: Optional[torch.Tensor] = None, cycles: int = 1):
        z = torch.empty_like(r) if z is None else z
        L.check(self.ctx.lib.amg_apply(self.ctx.h, self.h, _p(r), _p(z), cycles))
        return z

    def info(self) -> dict:
        i = L.amg_info()
        L.check(self.ctx.lib.amg_get_info(self.h, byref(i)))
        nl = i.levels
        return {"levels": nl, "coarse_kind": i.coarse_kind, "n": list(i.n[:nl]),
                "nnz": list(i.nnz[:nl]), "nnz_P": list(i.nnz_P[:nl]),
                "pmis_rounds": list(i.pmis_rounds[:nl]),
                "grid_complexity": i.grid_complexity,
                "operator_complexity": i.operator_complexity}

    def export_level(self, level: int) -> dict:
        inf = self.info()
        n, nnz, nnzp = inf["n"][level], inf["nnz"][level], inf["nnz_P"][level]
        cf = np.zeros(n, dtype=np.int8)
        arp = np.zeros(n + 1, dtype=np.int32)
        aci = np.zeros(nnz, dtype=np.int32)
        av = np.zeros(nnz, dtype=np.float64)
        has_p = level < inf["levels"] - 1
        prp = np.zeros(n + 1, dtype=np.int32) if has_p else None
        pci = np.zeros(max(nnzp, 1), dtype=np.int32)
        pv = np.zeros(max(nnzp, 1), dtype=np.float64)

        def ptr(a):
            return None if a is None else a.ctypes.data_as(c_void_p)
        L.check(self.ctx.lib.amg_export_level(self.ctx.h, self.h, level, ptr(cf), ptr(arp),
                                              ptr(aci), ptr(av), ptr(prp), ptr(pci), ptr(pv)))
        out = {"cf": cf, "A": (arp, aci, av)}
        if has_p:
            out["P"] = (prp, pci[:nnzp], pv[:nnzp])
        return out

    def close(self):
        if self._owned and self.h and self.ctx.alive:
            self.ctx.lib.amg_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def block_params(kind="schur2", **kw) -> L.block_params:
    p = L.block_params()
    L.load().block_params_default(byref(p))
    p.kind = PC_KINDS[kind] if isinstance(kind, str) else int(kind)
    amg_kw = {k[4:]: v for k, v in kw.items() if k.startswith("amg_")}
    for k, v in amg_kw.items():
        setattr(p.amg, k, v)
    for k, v in kw.items():
        if k.startswith("amg_"):
            continue
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


class BlockPreconditioner:
    """z = M^{-1} r for the Section 3 preconditioners."""

    def __init__(self, ctx: Context, system: BlockSystem, kind: str = "schur2", **kw):
        self.ctx = ctx
        self.system = system
        self.params = block_params(kind, **kw)
        h = c_void_p()
        L.check(ctx.lib.block_precond_create(ctx.h, byref(system.s), byref(self.params), byref(h)))
        self.h = h
        self.G, self.N = system.G, system.N
        ctx._adopt(self)

    def apply(self, r: torch.Tensor, z: Optional[torch.Tensor] = None) -> torch.Tensor:
        z = torch.empty_like(r) if z is None else z
        L.check(self.ctx.lib.block_precond_apply(self.ctx.h, self.h, _p(r), _p(z)))
        return z

    def info(self) -> dict:
        i = L.block_precond_info()
        L.check(self.ctx.lib.block_precond_get_info(self.h, byref(i)))
        G = self.G
        return {"kind": i.kind, "n_hierarchies": i.n_hierarchies,
                "inverses_per_apply": i.inverses_per_apply,
                "matvecs_per_apply": i.matvecs_per_apply,
                "pctl_p_cycles": list(i.pctl_p_cycles[:G + 1]), "setup_ms": i.setup_ms,
                # adaptive strategy: Definition 1 counts and neglected couplings,
                # Definition 2 counts per inverse role and the Jacobi roles
                "wc_counts": {"gE": list(i.wc_count_gE[:G]), "Eg": list(i.wc_count_Eg[:G]),
                              "EI": i.wc_count_EI, "IE": i.wc_count_IE},
                "weak": {"gE": [bool(v) for v in i.weak_gE[:G]],
                         "Eg": [bool(v) for v in i.weak_Eg[:G]],
                         "EI": bool(i.weak_EI), "IE": bool(i.weak_IE)},
                "wd_count": list(i.wd_count[:G + 2]),
                "jacobi": [bool(v) for v in i.jacobi[:G + 2]],
                "inner_cycles": list(i.inner_cycles[:G + 3])}

    def hierarchy(self, index: int) -> AMG:
        h = c_void_p()
        L.check(self.ctx.lib.block_precond_get_hierarchy(self.h, index, byref(h)))
        return AMG(self.ctx, None, None, None, _handle=h, _owner=self)

    def close(self):
        if getattr(self, "h", None) and self.ctx.alive:
            self.ctx.lib.block_precond_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class GmresResult:
    status: int
    iters: int
    restarts: int
    converged: bool
    precond_applies: int
    relres_est: float
    relres_true: float
    t_total_ms: float
    t_precond_ms: float
    t_matvec_ms: float
    t_orth_ms: float
    reorths: int = 0


def gmres_params(**kw) -> L.gmres_params:
    p = L.gmres_params()
    L.load().gmres_params_default(byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _result(st, r) -> GmresResult:
    return GmresResult(st, r.iters, r.restarts, bool(r.converged), r.precond_applies,
                       r.relres_est, r.relres_true, r.t_total_ms, r.t_precond_ms,
                       r.t_matvec_ms, r.t_orth_ms, r.reorths)


def gmres(ctx: Context, system: BlockSystem, M: Optional[BlockPreconditioner], b: torch.Tensor,
          x: Optional[torch.Tensor] = None, **kw):
    """Solve A x = b; x (initial guess, default 0) is updated in place.
    Returns (x, GmresResult).  Non-convergence is reported in the result."""
    x = torch.zeros_like(b) if x is None else x
    p = gmres_params(**kw)
    r = L.gmres_result()
    st = ctx.lib.gmres_solve(ctx.h, byref(system.s), M.h if M is not None else None, _p(b), _p(x),
                             byref(p), byref(r))
    L.check(st, allow=(-4,))
    return x, _result(st, r)


def gmres_noalloc(ctx: Context, system: BlockSystem, M: Optional[BlockPreconditioner],
                  b: torch.Tensor, x: Optional[torch.Tensor] = None, **kw):
    """gmres_solve_noalloc: the same solve with no device allocation (the
    workspace is the library's static per-device array).  x must be given or
    is allocated here, outside the call.  Returns (x, GmresResult)."""
    x = torch.zeros_like(b) if x is None else x
    p = gmres_params(**kw)
    r = L.gmres_result()
    st = ctx.lib.gmres_solve_noalloc(ctx.h, byref(system.s), M.h if M is not None else None,
                                     _p(b), _p(x), byref(p), byref(r))
    L.check(st, allow=(-4,))
    return x, _result(st, r)


def adjoint(ctx: Context, coeffs: Coeffs, system: BlockSystem,
            M_T: Optional[BlockPreconditioner], x: torch.Tensor, g: torch.Tensor, **kw):
    """lambda = A^{-T} g and the coefficient gradients.
    Returns (lambda, dL_dkappa, dL_dc, GmresResult)."""
    lam = torch.empty_like(g)
    dk = ctx.empty(coeffs.kappa.numel())
    dc = ctx.empty((2 * coeffs.G + 1) * coeffs.N)
    p = gmres_params(**kw)
    r = L.gmres_result()
    cs = coeffs.c_struct()
    st = ctx.lib.adjoint_solve(ctx.h, byref(cs), byref(system.s), M_T.h if M_T else None, _p(x),
                               _p(g), _p(lam), _p(dk), _p(dc), byref(p), byref(r))
    L.check(st, allow=(-4,))
    return lam, dk, dc, _result(st, r)


def adjoint_gradients(ctx: Context, coeffs: Coeffs, x: torch.Tensor, lam: torch.Tensor):
    dk = ctx.empty(coeffs.kappa.numel())
    dc = ctx.empty((2 * coeffs.G + 1) * coeffs.N)
    cs = coeffs.c_struct()
    L.check(ctx.lib.mgd_adjoint_gradients(ctx.h, byref(cs), _p(x), _p(lam), _p(dk), _p(dc)))
    return dk, dc
