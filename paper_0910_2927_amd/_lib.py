"""ctypes declarations of the libsignkrylov C ABI (include/signkrylov.h).

Loading fails loudly when the shared library has not been built: there is
no fallback implementation of any step.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsignkrylov.so")

SK_OK = 0
SK_ERR_ARG = -1
SK_ERR_HIP = -2
SK_ERR_NOCONV = -3
SK_ERR_SINGULAR = -4
SK_ERR_NAN = -5
SK_ERR_WORKSPACE = -6

SK_C128 = 0
SK_C64 = 1
SK_PREC_FP64 = 0
SK_PREC_MIXED = 1
SK_METHOD_FOM = 0
SK_METHOD_GMRES = 1

STATUS_NAMES = {
    SK_OK: "SK_OK", SK_ERR_ARG: "SK_ERR_ARG", SK_ERR_HIP: "SK_ERR_HIP",
    SK_ERR_NOCONV: "SK_ERR_NOCONV", SK_ERR_SINGULAR: "SK_ERR_SINGULAR",
    SK_ERR_NAN: "SK_ERR_NAN", SK_ERR_WORKSPACE: "SK_ERR_WORKSPACE",
}


class SkOperator(C.Structure):
    _fields_ = [("dims", C.c_int32 * 4), ("t_antiperiodic", C.c_int32),
                ("kappa", C.c_double), ("mu", C.c_double),
                ("links", C.c_void_p), ("links_c64", C.c_void_p)]


class SkSignParams(C.Structure):
    _fields_ = [("npoles", C.c_int32), ("sigma", C.POINTER(C.c_double)),
                ("omega", C.POINTER(C.c_double)), ("k", C.c_int32),
                ("max_cycles", C.c_int32), ("tol", C.c_double), ("m", C.c_int32),
                ("R", C.c_void_p), ("L", C.c_void_p), ("F", C.c_void_p),
                ("project_each_cycle", C.c_int32), ("precision", C.c_int32),
                ("mixed_switch", C.c_double), ("X_shift", C.c_void_p),
                ("method", C.c_int32), ("seed", C.c_int32), ("resid_tol", C.c_double)]


SK_KERNEL_CLASSES = ["stencil", "gs_dot", "gs_upd_dot", "gs_upd_norm", "small", "sol_update",
                     "project", "gs_reduce"]


class SkKernelTimes(C.Structure):
    _fields_ = [("ms", C.c_double * 8), ("bytes", C.c_double * 8), ("launches", C.c_int64 * 8)]


class SkStats(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("cycles_c64", C.c_int32), ("matvecs", C.c_int32),
                ("converged", C.c_int32),
                ("breakdown", C.c_int32), ("final_update_norm", C.c_double),
                ("x_norm", C.c_double), ("hist_update", C.POINTER(C.c_double)),
                ("hist_beta", C.POINTER(C.c_double)), ("hist_leak", C.POINTER(C.c_double)),
                ("hist_cap", C.c_int32), ("times", C.POINTER(SkKernelTimes)),
                ("hist_rho", C.POINTER(C.c_double)), ("shift_resid", C.POINTER(C.c_double)),
                ("shift_resid_implicit", C.POINTER(C.c_double)), ("resid_checked", C.c_int32),
                ("resid_ok", C.c_int32), ("seconds", C.c_double)]


class SkBatchSystem(C.Structure):
    _fields_ = [("op", SkOperator), ("b", C.c_void_p), ("x", C.c_void_p), ("k", C.c_int32),
                ("m", C.c_int32), ("R", C.c_void_p), ("L", C.c_void_p), ("F", C.c_void_p),
                ("sigma", C.POINTER(C.c_double)), ("omega", C.POINTER(C.c_double))]


class SkDirectStats(C.Structure):
    _fields_ = [("k_done", C.c_int32), ("breakdown", C.c_int32), ("newton_iters", C.c_int32),
                ("pad", C.c_int32), ("newton_change", C.c_double), ("seconds", C.c_double)]


class SkOverlapStats(C.Structure):
    _fields_ = [("outer_iters", C.c_int32), ("restarts", C.c_int32), ("sign_calls", C.c_int64),
                ("inner_matvecs", C.c_int64), ("rel_residual", C.c_double), ("converged", C.c_int32),
                ("pad", C.c_int32), ("seconds", C.c_double)]


class SkEigParams(C.Structure):
    _fields_ = [("m", C.c_int32), ("nev_extra", C.c_int32), ("ncv", C.c_int32), ("key", C.c_int32),
                ("tol", C.c_double), ("max_restarts", C.c_int32), ("keep", C.c_int32)]


class SkEigStats(C.Structure):
    _fields_ = [("converged", C.c_int32), ("restarts", C.c_int32 * 2), ("matvecs", C.c_int64),
                ("resid", C.c_double * 2), ("gap", C.c_double), ("key_window", C.c_double)]


# (name, restype, argtypes) of every exported symbol
SIGNATURES = [
    ("sk_volume", C.c_int64, [C.POINTER(SkOperator)]),
    ("kl_poles", C.c_int, [C.c_int, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("sk_links_to_c64", C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    ("sk_last_error", C.c_char_p, []),
    ("wilson_apply", C.c_int, [C.POINTER(SkOperator), C.c_int, C.c_void_p, C.c_void_p, C.c_int,
                               C.c_void_p]),
    ("arnoldi_cycle_workspace_bytes", C.c_size_t, [C.POINTER(SkOperator), C.c_int]),
    ("arnoldi_cycle", C.c_int, [C.POINTER(SkOperator), C.c_int, C.c_void_p, C.c_void_p, C.c_int,
                                C.POINTER(C.c_int), C.c_void_p, C.c_size_t, C.c_void_p]),
    ("multishift_fom_restart_workspace_bytes", C.c_size_t, [C.c_int, C.c_int]),
    ("multishift_fom_restart", C.c_int, [C.c_int, C.c_int64, C.c_int, C.c_void_p, C.c_int,
                                         C.POINTER(C.c_double), C.POINTER(C.c_double),
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.POINTER(C.c_double), C.c_void_p,
                                         C.c_size_t, C.c_void_p]),
    ("deflate_project_workspace_bytes", C.c_size_t, [C.c_int, C.c_int64]),
    ("deflate_project", C.c_int, [C.c_int, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_size_t, C.c_void_p]),
    ("deflate_project_noalloc", C.c_int, [C.c_int, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("sign_apply_workspace_bytes", C.c_size_t, [C.POINTER(SkOperator), C.POINTER(SkSignParams)]),
    ("sign_apply", C.c_int, [C.POINTER(SkOperator), C.POINTER(SkSignParams), C.c_void_p,
                             C.c_void_p, C.POINTER(SkStats), C.c_void_p, C.c_size_t, C.c_void_p]),
    ("deflation_eigensolve_workspace_bytes", C.c_size_t, [C.POINTER(SkOperator),
                                                          C.POINTER(SkEigParams)]),
    ("deflation_eigensolve", C.c_int, [C.POINTER(SkOperator), C.POINTER(SkEigParams), C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                       C.POINTER(SkEigStats), C.c_void_p, C.c_size_t, C.c_void_p]),
    ("sk_dense_schur", C.c_int, [C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                 C.POINTER(C.c_double), C.c_int, C.c_int]),
    ("sk_dense_sign", C.c_int, [C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("sign_apply_batched_workspace_bytes", C.c_size_t, [C.c_int, C.POINTER(SkBatchSystem),
                                                        C.POINTER(SkSignParams)]),
    ("sign_apply_batched", C.c_int, [C.c_int, C.POINTER(SkBatchSystem), C.POINTER(SkSignParams),
                                     C.POINTER(SkStats), C.c_void_p, C.c_size_t, C.c_void_p]),
    ("sk_batched_last_tile", C.c_int, [C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    ("sk_batched_set_tile", C.c_int, [C.c_int, C.c_int, C.c_int]),
    ("direct_sign_workspace_bytes", C.c_size_t, [C.POINTER(SkOperator), C.c_int, C.c_int, C.c_int]),
    ("direct_sign_apply", C.c_int, [C.POINTER(SkOperator), C.c_int, C.c_int, C.c_int, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.POINTER(SkDirectStats), C.c_void_p, C.c_size_t, C.c_void_p]),
    ("overlap_workspace_bytes", C.c_size_t, [C.POINTER(SkOperator), C.POINTER(SkSignParams), C.c_int]),
    ("overlap_apply", C.c_int, [C.POINTER(SkOperator), C.POINTER(SkSignParams), C.c_double, C.c_void_p,
                                C.c_void_p, C.POINTER(SkStats), C.c_void_p, C.c_size_t, C.c_void_p]),
    ("overlap_solve", C.c_int, [C.POINTER(SkOperator), C.POINTER(SkSignParams), C.c_double, C.c_int,
                                C.c_int, C.c_double, C.c_void_p, C.c_void_p, C.POINTER(SkOverlapStats),
                                C.c_void_p, C.c_size_t, C.c_void_p]),
    ("sign_apply_backward_workspace_bytes", C.c_size_t, [C.POINTER(SkOperator),
                                                         C.POINTER(SkSignParams)]),
    ("sign_apply_backward", C.c_int, [C.POINTER(SkOperator), C.POINTER(SkSignParams), C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                      C.POINTER(SkStats), C.c_void_p, C.c_size_t, C.c_void_p]),
]

_lib = None


def load(path: str | None = None):
    """Load the library (once) and declare every signature."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"libsignkrylov is not built ({p} missing); run "
                          f"`python -m paper_0910_2927_amd.build`")
    lib = C.CDLL(p)
    for name, res, args in SIGNATURES:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


class SkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int):
    if status != SK_OK:
        raise SkError(status, load().sk_last_error().decode(errors="replace"))
    return status
