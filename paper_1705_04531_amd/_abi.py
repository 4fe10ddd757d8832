"""ctypes declarations of the C ABI in include/ieti.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libieti.so")

IETI_OK = 0
IETI_EINVAL = -1
IETI_ENONCONFORMING = -2
IETI_EGEOM = -3
IETI_ENOMEM = -4
IETI_ENOCONV = -5
IETI_EDEVICE = -6
IETI_ENOTSUP = -7
IETI_PENDING = 1

IETI_LOCAL_MG = 0
IETI_LOCAL_EXACT = 1
IETI_LOCAL_EXACT_MG = 2
IETI_LOCAL_MG_SADDLE = 3
IETI_PRIMAL_VERTICES = 1
IETI_PRIMAL_EDGES = 2
IETI_SMOOTHER_CHEBYSHEV = 0
IETI_SMOOTHER_TENSOR = 1

IETI_ARR_STENCIL = 1
IETI_ARR_STENCIL_OFFS = 2
IETI_ARR_PROLONG = 3
IETI_ARR_SHAPE = 4
IETI_ARR_MASKS = 5
IETI_ARR_LAMBDA_MAP = 6
IETI_ARR_QP_WEIGHT = 7
IETI_ARR_LMAX = 8
IETI_ARR_PRIMAL_MAP = 9
IETI_ARR_BAND = 10
IETI_ARR_TENSOR_U = 11
IETI_ARR_TENSOR_LAMBDA = 12
IETI_ARR_TENSOR_PARAMS = 13

IETI_KPROF_SMOOTH_FINE = 0
IETI_KPROF_APPLY64 = 1
IETI_KPROF_RESID_FINE = 2
IETI_KPROF_FAPPLY = 3
IETI_KPROF_PREC = 4
IETI_KPROF_COARSE = 5
IETI_KPROF_COUNT = 6


class IetiPatch(C.Structure):
    _fields_ = [
        ("dim", C.c_int32),
        ("degree", C.c_int32 * 3),
        ("n_knots", C.c_int32 * 3),
        ("knots", C.POINTER(C.c_double) * 3),
        ("ctrl", C.POINTER(C.c_double)),
    ]


class IetiOptions(C.Structure):
    _fields_ = [
        ("local_solver", C.c_int32),
        ("mg_precision", C.c_int32),
        ("primal", C.c_int32),
        ("cheb_degree", C.c_int32),
        ("cheb_degree_coarse", C.c_int32),
        ("cheb_lower", C.c_double),
        ("prec_vcycles", C.c_int32),
        ("max_it", C.c_int32),
        ("inner_max_it", C.c_int32),
        ("tol", C.c_double),
        ("inner_tol", C.c_double),
        ("basis_tol", C.c_double),
        ("check_every", C.c_int32),
        ("use_graph", C.c_int32),
        ("device", C.c_int32),
        ("stream", C.c_void_p),
        ("hbm_budget", C.c_size_t),
        ("coarse_level", C.c_int32),
        ("autotune", C.c_int32),
        ("coarse_dofs", C.c_int32),
        ("smoother", C.c_int32),
        ("smoother_sigma", C.c_double),
        ("tune_cache", C.c_char_p),
        ("batch_dofs", C.c_int64),
        ("coarse_degree", C.c_int32),
    ]


class IetiStats(C.Structure):
    _fields_ = [
        ("outer_iterations", C.c_int32),
        ("inner_iterations_max", C.c_int32),
        ("inner_iterations_mean", C.c_double),
        ("residual_initial", C.c_double),
        ("residual_final", C.c_double),
        ("global_residual", C.c_double),
        ("time_rhs_ms", C.c_double),
        ("time_pcg_ms", C.c_double),
        ("time_recovery_ms", C.c_double),
        ("time_total_ms", C.c_double),
        ("ndof_torn", C.c_int64),
        ("ndof_global", C.c_int64),
        ("n_lambda", C.c_int64),
        ("n_primal", C.c_int64),
        ("breakdown", C.c_int32),
        ("cheb_degree", C.c_int32),
        ("cheb_degree_coarse", C.c_int32),
        ("cheb_lower", C.c_double),
        ("saddle_omega", C.c_double),
        ("fine_tile_staged", C.c_int32),
        ("tune_cached", C.c_int32),
        ("inner_unconverged", C.c_int32),
        ("inner_nonfinite", C.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


# every symbol include/ieti.h declares, with (restype, argtypes)
_P = C.c_void_p
_I64P = C.POINTER(C.c_int64)
SIGNATURES = {
    "ieti_default_options": (None, [C.POINTER(IetiOptions)]),
    "ieti_plan_create": (C.c_int, [C.POINTER(IetiPatch), C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                   C.POINTER(IetiOptions), C.POINTER(_P)]),
    "ieti_plan_destroy": (None, [_P]),
    "ieti_plan_sizes": (C.c_int, [_P, _I64P, _I64P, _I64P, _I64P, _I64P, C.POINTER(C.c_int32)]),
    "ieti_plan_array": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, _P, _I64P]),
    "ieti_plan_quadrature": (C.c_int, [_P, C.POINTER(C.c_double)]),
    "ieti_setup": (C.c_int, [C.POINTER(IetiPatch), C.c_int32, C.POINTER(C.c_double), C.c_int32,
                             C.POINTER(IetiOptions), C.POINTER(_P)]),
    "ieti_quadrature": (C.c_int, [_P, _P, C.c_int32, _I64P]),
    "ieti_solve": (C.c_int, [_P, _P, _P, C.POINTER(IetiStats)]),
    "ieti_solve_noalloc": (C.c_int, [_P, _P, _P, C.POINTER(IetiStats)]),
    "ieti_sizes": (C.c_int, [_P, _I64P, _I64P, _I64P]),
    "ieti_destroy": (None, [_P]),
    "ieti_profile_enable": (C.c_int, [_P, C.c_int32]),
    "ieti_profile_query": (C.c_int, [_P, C.c_int32, _I64P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "ieti_quadrature_points": (C.c_int, [C.POINTER(IetiPatch), C.c_int32, C.POINTER(C.c_double), _I64P]),
    "ieti_plan_device_bytes": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
    "ieti_server_create": (C.c_int, [C.POINTER(IetiOptions), C.c_int32, C.POINTER(_P)]),
    "ieti_server_submit": (C.c_int, [_P, C.POINTER(IetiPatch), C.c_int32, C.POINTER(C.c_double), C.c_int64,
                                     C.POINTER(C.c_double), _I64P]),
    "ieti_server_poll": (C.c_int, [_P, C.c_int64, C.c_int32, C.POINTER(IetiStats), C.POINTER(C.c_double)]),
    "ieti_server_load": (C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_size_t)]),
    "ieti_server_destroy": (None, [_P]),
    "ieti_strerror": (C.c_char_p, [C.c_int]),
    "ieti_last_error": (C.c_char_p, []),
}

_lib = None


def lib():
    """The loaded libieti.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libieti.so not built ({LIB_PATH}); run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class IetiError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        L = lib()
        msg = L.ieti_strerror(code).decode()
        detail = L.ieti_last_error().decode()
        super().__init__(f"{what}: {msg} ({code}){': ' + detail if detail else ''}")
        self.code = code


def check(code: int, what: str = ""):
    if code != IETI_OK:
        raise IetiError(code, what)
    return code
