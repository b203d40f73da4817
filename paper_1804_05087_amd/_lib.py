"""ctypes binding of libsp.so (argument marshalling only).

Every numerical step runs in the HIP library; this module converts torch
tensors to device pointers and checks status codes. If the library is not
built it raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsp.so")

SP_OK = 0
SP_ERR_NOT_CONVERGED = -5
SP_ERR_NONFINITE = -6
SP_FP64 = 0
SP_MIXED = 1
SP_OP_PHI = 0
SP_OP_RESIDUAL = 1
SP_STAGE_SYNTH, SP_STAGE_XINV, SP_STAGE_ZLINE, SP_STAGE_XFWD, SP_STAGE_SOLVE = 0, 1, 2, 3, 4


class sp_params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("lx", C.c_double), ("lz", C.c_double), ("re", C.c_double), ("dt", C.c_double),
        ("wall_upper", C.c_double), ("wall_lower", C.c_double),
        ("precision", C.c_int32),
    ]


class sp_newton_opts(C.Structure):
    _fields_ = [
        ("max_newton", C.c_int32), ("max_krylov", C.c_int32),
        ("gmres_rtol", C.c_double), ("newton_tol", C.c_double),
        ("jvp_mode", C.c_int32), ("fd_eps", C.c_double),
        ("krylov_fp32", C.c_int32),
    ]


class sp_newton_report(C.Structure):
    _fields_ = [
        ("converged", C.c_int32), ("newton_iters", C.c_int32),
        ("total_krylov", C.c_int32), ("total_actions", C.c_int32),
        ("seconds", C.c_double),
        ("res_norm", C.c_double * 65),
        ("krylov", C.c_int32 * 64),
        ("gmres_relres", C.c_double * 64),
    ]


class sp_hook_opts(C.Structure):
    _fields_ = [
        ("max_trials", C.c_int32), ("delta_init", C.c_double),
        ("delta_min", C.c_double), ("delta_max", C.c_double),
    ]


class sp_hook_report(C.Structure):
    _fields_ = [
        ("trials", C.c_int32 * 64), ("delta", C.c_double * 64), ("mu", C.c_double * 64),
        ("step_norm", C.c_double * 64), ("rho", C.c_double * 64),
    ]


# name -> (restype, argtypes); every exported entry point of include/sp.h
SIGNATURES = {
    "sp_plan_create": (C.c_int, [C.POINTER(sp_params), C.c_void_p, C.POINTER(C.c_void_p)]),
    "sp_plan_destroy": (C.c_int, [C.c_void_p]),
    "sp_plan_set_dt": (C.c_int, [C.c_void_p, C.c_double]),
    "sp_plan_set_precision": (C.c_int, [C.c_void_p, C.c_int32]),
    "sp_plan_set_steps": (C.c_int, [C.c_void_p, C.c_int32]),
    "sp_plan_set_scheme": (C.c_int, [C.c_void_p, C.c_int32]),
    "sp_plan_set_advection": (C.c_int, [C.c_void_p, C.c_int32]),
    "sp_advected_mode_operator": (C.c_int, [C.c_int32, C.c_double, C.c_double, C.c_double,
                                            C.c_double, C.c_void_p]),
    "sp_state_shape": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "sp_plan_workspace_bytes": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_size_t)]),
    "sp_plan_set_workspace": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "sp_nonlinear": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "sp_stokes_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "sp_befe_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "sp_befe_step_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "sp_residual": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "sp_norm": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "sp_linearize": (C.c_int, [C.c_void_p, C.c_void_p]),
    "sp_jvp_lin": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "sp_jvp": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sp_vjp_lin": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "sp_vjp": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sp_pack": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "sp_jacobian_columns": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int64, C.c_void_p,
                                      C.c_int64]),
    "sp_befe_step_batch": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    "sp_jvp_lin_batch": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                   C.c_void_p]),
    "sp_unpack": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "sp_newton_gmres": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(sp_newton_opts),
                                  C.POINTER(sp_newton_report)]),
    "sp_newton_hookstep": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(sp_newton_opts),
                                     C.POINTER(sp_hook_opts), C.POINTER(sp_newton_report),
                                     C.POINTER(sp_hook_report)]),
    "sp_symmetrize": (C.c_int, [C.c_void_p, C.c_void_p]),
    "sp_plan_set_symmetry": (C.c_int, [C.c_void_p, C.c_int32]),
    "sp_hook_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_double,
                               C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "sp_profile_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "sp_time_stage": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                C.POINTER(C.c_double)]),
    "sp_profile_read": (C.c_int, [C.c_void_p, C.c_int32, C.c_char_p, C.POINTER(C.c_int64),
                                  C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_int32]),
    "sp_status_string": (C.c_char_p, [C.c_int]),
    "sp_last_error": (C.c_char_p, [C.c_void_p]),
}

_lib = None


def load() -> C.CDLL:
    """Load libsp.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1804_05087_amd.build` "
            "(the HIP library is required; there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class SPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"status {status}: {msg}")
        self.status = status
