"""ctypes declarations for libmgdamg (include/mgdamg.h).  Marshalling only."""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, c_char_p, c_double, c_int, c_int8, c_int32, c_int64,
                    c_uint8, c_uint64, c_void_p, CFUNCTYPE)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmgdamg.so")

MGD_OK = 0
STATUS = {0: "MGD_OK", -1: "MGD_EINVAL", -2: "MGD_ENOMEM", -3: "MGD_EHIP", -4: "MGD_ENOTCONV",
          -5: "MGD_EBREAKDOWN", -6: "MGD_ESINGULAR", -7: "MGD_ESTATE"}
MGD_MAX_LEVELS = 32

PC_KINDS = {"amg": 0, "bdiag": 1, "pctl": 2, "schur1": 3, "schur2": 4, "schur2_lower": 5,
            "identity": 6}


class mgd_csr(Structure):
    _fields_ = [("n_rows", c_int32), ("n_cols", c_int32), ("nnz", c_int64),
                ("row_ptr", c_void_p), ("col_idx", c_void_p), ("val", c_void_p)]


class amg_params(Structure):
    _fields_ = [("strength_theta", c_double), ("dominance_theta", c_double), ("seed", c_uint64),
                ("max_levels", c_int32), ("coarse_max", c_int32), ("dense_max", c_int32),
                ("n_pre", c_int32), ("n_post", c_int32), ("precision", c_int32),
                ("autotune", c_int32), ("coarsening", c_int32), ("hmis_tile", c_int32),
                ("smoother", c_int32), ("aggressive_levels", c_int32)]


class amg_info(Structure):
    _fields_ = [("levels", c_int32), ("coarse_kind", c_int32),
                ("n", c_int64 * MGD_MAX_LEVELS), ("nnz", c_int64 * MGD_MAX_LEVELS),
                ("nnz_P", c_int64 * MGD_MAX_LEVELS), ("pmis_rounds", c_int32 * MGD_MAX_LEVELS),
                ("grid_complexity", c_double), ("operator_complexity", c_double)]


class mgd_block_system(Structure):
    _fields_ = [("G", c_int32), ("N", c_int32), ("blocks", POINTER(mgd_csr)),
                ("d_gE", c_void_p), ("d_Eg", c_void_p), ("d_EI", c_void_p), ("d_IE", c_void_p)]


class mgd_coeffs(Structure):
    _fields_ = [("dim", c_int32), ("n", c_int32), ("G", c_int32), ("kappa", c_void_p),
                ("c_gE", c_void_p), ("c_Eg", c_void_p), ("c_EI", c_void_p), ("mass", c_double),
                ("xi", c_void_p)]


class block_params(Structure):
    _fields_ = [("kind", c_int32), ("amg", amg_params), ("cycles_rad", c_int32),
                ("cycles_E", c_int32), ("cycles_I", c_int32), ("pctl_p_tol", c_double),
                ("pctl_p_maxcycles", c_int32), ("batched", c_int32), ("use_graph", c_int32),
                ("transpose", c_int32), ("adaptive", c_int32), ("theta_wc", c_double),
                ("sigma_wc", c_double), ("theta_wd", c_double), ("jacobi_sweeps", c_int32),
                ("inner_tol", c_double), ("inner_maxcycles", c_int32), ("option4_steps", c_int32)]


class block_precond_info(Structure):
    _fields_ = [("kind", c_int32), ("n_hierarchies", c_int32), ("inverses_per_apply", c_int32),
                ("matvecs_per_apply", c_int32), ("pctl_p_cycles", c_int32 * 66),
                ("setup_ms", c_double), ("wc_count_gE", c_int32 * 64),
                ("wc_count_Eg", c_int32 * 64), ("wc_count_EI", c_int32), ("wc_count_IE", c_int32),
                ("weak_gE", c_uint8 * 64), ("weak_Eg", c_uint8 * 64), ("weak_EI", c_int32),
                ("weak_IE", c_int32), ("wd_count", c_int32 * 66), ("jacobi", c_uint8 * 66),
                ("inner_cycles", c_int32 * 66)]


class gmres_params(Structure):
    _fields_ = [("restart", c_int32), ("max_iters", c_int32), ("rtol", c_double),
                ("flexible", c_int32), ("profile", c_int32)]


class gmres_result(Structure):
    _fields_ = [("iters", c_int32), ("restarts", c_int32), ("converged", c_int32),
                ("precond_applies", c_int32), ("relres_est", c_double),
                ("relres_true", c_double), ("t_total_ms", c_double), ("t_precond_ms", c_double),
                ("t_matvec_ms", c_double), ("t_orth_ms", c_double), ("reorths", c_int32)]


ALLOC_FN = CFUNCTYPE(c_void_p, ctypes.c_size_t, c_void_p, c_void_p)
FREE_FN = CFUNCTYPE(None, c_void_p, c_void_p, c_void_p)


class mgd_allocator(Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", c_void_p)]


# (name, restype, argtypes) for every exported function of include/mgdamg.h
SIGNATURES = [
    ("mgd_last_error", c_char_p, []),
    ("mgd_version", c_char_p, []),
    ("mgd_ctx_create", c_int32, [c_int, c_void_p, POINTER(mgd_allocator), POINTER(c_void_p)]),
    ("mgd_ctx_destroy", c_int32, [c_void_p]),
    ("mgd_ctx_synchronize", c_int32, [c_void_p]),
    ("mgd_ctx_set_profiling", c_int32, [c_void_p, c_int]),
    ("mgd_ctx_reset_kernel_stats", c_int32, [c_void_p]),
    ("mgd_kernel_class_count", c_int, []),
    ("mgd_kernel_class_name", c_char_p, [c_int]),
    ("mgd_ctx_kernel_stats", c_int32, [c_void_p, c_int, POINTER(c_int64), POINTER(c_double),
                                       POINTER(c_double)]),
    ("mgd_ctx_kernel_symbol_count", c_int32, [c_void_p, POINTER(c_int)]),
    ("mgd_ctx_kernel_symbol_stats", c_int32, [c_void_p, c_int, ctypes.c_char_p, c_int,
                                              POINTER(c_int64), POINTER(c_double),
                                              POINTER(c_double), POINTER(c_double)]),
    ("mgd_csr_spmv", c_int32, [c_void_p, POINTER(mgd_csr), c_void_p, c_void_p]),
    ("gmres_solve_noalloc", c_int32, [c_void_p, POINTER(mgd_block_system), c_void_p, c_void_p,
                                      c_void_p, POINTER(gmres_params), POINTER(gmres_result)]),
    ("amg_params_default", None, [POINTER(amg_params)]),
    ("amg_setup", c_int32, [c_void_p, POINTER(mgd_csr), POINTER(amg_params), POINTER(c_void_p)]),
    ("amg_apply", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int]),
    ("amg_get_info", c_int32, [c_void_p, POINTER(amg_info)]),
    ("amg_export_level", c_int32, [c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_void_p, c_void_p, c_void_p]),
    ("amg_destroy", c_int32, [c_void_p]),
    ("mgd_block_matvec", c_int32, [c_void_p, POINTER(mgd_block_system), c_void_p, c_void_p]),
    ("mgd_assemble", c_int32, [c_void_p, POINTER(mgd_coeffs), POINTER(mgd_block_system)]),
    ("mgd_block_system_transpose", c_int32, [c_void_p, POINTER(mgd_block_system),
                                             POINTER(mgd_block_system)]),
    ("mgd_block_system_free", c_int32, [c_void_p, POINTER(mgd_block_system)]),
    ("block_params_default", None, [POINTER(block_params)]),
    ("block_precond_create", c_int32, [c_void_p, POINTER(mgd_block_system),
                                       POINTER(block_params), POINTER(c_void_p)]),
    ("block_precond_apply", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    ("block_precond_get_info", c_int32, [c_void_p, POINTER(block_precond_info)]),
    ("block_precond_get_hierarchy", c_int32, [c_void_p, c_int, POINTER(c_void_p)]),
    ("block_precond_destroy", c_int32, [c_void_p]),
    ("gmres_params_default", None, [POINTER(gmres_params)]),
    ("gmres_solve", c_int32, [c_void_p, POINTER(mgd_block_system), c_void_p, c_void_p, c_void_p,
                              POINTER(gmres_params), POINTER(gmres_result)]),
    ("adjoint_solve", c_int32, [c_void_p, POINTER(mgd_coeffs), POINTER(mgd_block_system),
                                c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                POINTER(gmres_params), POINTER(gmres_result)]),
    ("mgd_adjoint_gradients", c_int32, [c_void_p, POINTER(mgd_coeffs), c_void_p, c_void_p,
                                        c_void_p, c_void_p]),
]

_LIB = None


class LibraryMissing(RuntimeError):
    pass


class MgdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


def load(path: str = LIB_PATH):
    """Load libmgdamg.so; raises LibraryMissing when it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise LibraryMissing(
            f"{path} not found: build it with `python -m paper_2002_04958_amd.build` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def check(status: int, allow=()):
    if status == MGD_OK or status in allow:
        return status
    msg = load().mgd_last_error()
    raise MgdError(status, msg.decode() if msg else "")
