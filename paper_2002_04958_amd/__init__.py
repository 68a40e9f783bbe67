"""mgdamg for MI355X: AMG block-preconditioned GMRES for the multi-group
radiation diffusion block system (Yue, Zhang, Xu, Shu, Shi, arXiv 2002.04958).

The numerical work runs in libmgdamg.so (hand-written HIP for gfx950) behind
the C ABI in include/mgdamg.h; this package is its Python binding.
"""
import importlib

from ._lib import LibraryMissing, MgdError, load as load_library  # noqa: F401

_API_NAMES = {"Context", "Coeffs", "BlockSystem", "AMG", "BlockPreconditioner", "GmresResult",
              "gmres", "gmres_noalloc", "adjoint", "adjoint_gradients", "csr_spmv", "PC_KINDS",
              "MGDSolve"}


def __getattr__(name):
    # the torch-based binding is imported lazily so that `build` and the ABI
    # checks work without initialising the GPU runtime
    if name in _API_NAMES:
        mod = "autograd" if name == "MGDSolve" else "api"
        return getattr(importlib.import_module(f"{__name__}.{mod}"), name)
    raise AttributeError(name)
