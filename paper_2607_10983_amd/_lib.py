"""ctypes declarations of the C ABI in ``include/mg.h`` (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MG_LIBRARY") or os.path.join(HERE, "libmg.so")

MG_OK = 0
MG_ERR_INVALID = 1
MG_ERR_INVALID_COEFF = 2
MG_ERR_NOMEM = 3
MG_ERR_HIP = 4
MG_ERR_NONFINITE = 5
MG_ERR_NOT_CONVERGED = 6

MG_FP64, MG_MIXED, MG_FP32 = 0, 1, 2
MG_CHEBYSHEV, MG_JACOBI = 0, 1
MG_DTYPE_F32, MG_DTYPE_F64 = 0, 1
MG_NOALLOC_MAX_N = 512
MG_PREDICT_RECYCLE, MG_PREDICT_GROWTH, MG_PREDICT_LINEAR, MG_PREDICT_QUADRATIC = 0, 1, 2, 3
MG_TIME_STEP, MG_TIME_PAIR, MG_TIME_TRIPLE, MG_TIME_OUTER, MG_TIME_TRANSFER = 1, 2, 4, 8, 16
MG_OPT_NO_PAIR, MG_OPT_NO_VISIT, MG_OPT_NO_TAIL, MG_OPT_NO_FUSED_SUMS, MG_OPT_GRAPH = 1, 2, 4, 8, 16
(MG_STEP_SMOOTH, MG_STEP_SMOOTH_ZERO, MG_STEP_PROLONG_SMOOTH, MG_STEP_RESIDUAL_RESTRICT, MG_STEP_PROLONG,
 MG_STEP_VCYCLE) = range(6)


class MgParams(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int),
        ("levels", ctypes.c_int),
        ("cheb_degree", ctypes.c_int),
        ("cheb_alpha", ctypes.c_double),
        ("h", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("smoother", ctypes.c_int),
        ("jacobi_omega", ctypes.c_double),
        ("jacobi_sweeps", ctypes.c_int),
        ("options", ctypes.c_int),
    ]


class MgSolveInfo(ctypes.Structure):
    _fields_ = [
        ("cycles", ctypes.c_int),
        ("rel_res0", ctypes.c_double),
        ("rel_res", ctypes.c_double),
        ("history", ctypes.POINTER(ctypes.c_double)),
        ("history_cap", ctypes.c_int),
    ]


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_PD = ctypes.POINTER(ctypes.c_double)
_PI = ctypes.POINTER(ctypes.c_int)

# name -> (restype, argtypes); the set of names is exactly the ABI of mg.h
SIGNATURES = {
    "mg_params_default": (_I, [ctypes.POINTER(MgParams), _I]),
    "mg_validate_params": (_I, [ctypes.POINTER(MgParams)]),
    "mg_create": (_I, [ctypes.POINTER(MgParams), _P, _I, _P, ctypes.POINTER(_P)]),
    "mg_create_psi": (_I, [ctypes.POINTER(MgParams), _P, _P, ctypes.POINTER(_P)]),
    "mg_destroy": (_I, [_P]),
    "mg_set_stream": (_I, [_P, _P]),
    "mg_vcycle": (_I, [_P, _P, _P, _PD]),
    "mg_solve": (_I, [_P, _P, _P, _D, _I, ctypes.POINTER(MgSolveInfo)]),
    "mg_solve_adjoint": (_I, [_P, _P, _P, _D, _I, ctypes.POINTER(MgSolveInfo)]),
    "mg_solve_pcg": (_I, [_P, _P, _P, _D, _I, ctypes.POINTER(MgSolveInfo)]),
    "mg_cycles": (_I, [_P, _P, _P, _I, _PD]),
    "mg_inner_step": (_I, [_P, _I, _I, _P, _P, _P, _P]),
    "mg_coeff_grad": (_I, [_P, _P, _P, _P, _I]),
    "mg_geometry": (_I, [_I, _D, _P, _P, _I, _P, _P]),
    "mg_geometry_bwd": (_I, [_I, _D, _P, _P, _P, _P, _P]),
    "mg_geometry_bwd_noalloc": (_I, [_I, _D, _P, _P, _P, _P, _P]),
    "mg_predict": (_I, [_I, _I, _P, _P, _P, _D, _P, _P]),
    "mg_accel": (_I, [_I, _D, _P, _P, _D, _P, _I, _P]),
    "mg_apply": (_I, [_P, _I, _P, _P]),
    "mg_smooth": (_I, [_P, _I, _P, _P]),
    "mg_residual_restrict": (_I, [_P, _I, _P, _P, _P]),
    "mg_prolong_add": (_I, [_P, _I, _P, _P]),
    "mg_coarse_solve": (_I, [_P, _P, _P]),
    "mg_level_lmax": (_I, [_P, _PD]),
    "mg_enable_kernel_timing": (_I, [_P, _I]),
    "mg_kernel_timing": (_I, [_P, _PI, _PD, _PD]),
    "mg_status_string": (ctypes.c_char_p, [_I]),
    "mg_last_error": (ctypes.c_char_p, [_P]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load ``libmg.so``.  Raises if it has not been built: there is no
    fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`"
        )
    # torch first, so the library binds to the HIP runtime torch already loaded
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class MGError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        lib = load()
        msg = lib.mg_status_string(status).decode()
        super().__init__(f"{where}: {msg}" + (f" ({detail})" if detail else ""))
