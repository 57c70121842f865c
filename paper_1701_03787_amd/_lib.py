"""ctypes loader for libshenhip.so (the in-tree HIP library).

Fails loudly if the library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libshenhip.so")

SHEN_OK = 0
SHEN_EINVAL = -1
SHEN_ELAUNCH = -2
SHEN_ENOTSUP = -3
SHEN_EDEVICE = -4
SHEN_ESCRATCH = -5
SHEN_INFO_REFINE_FALLBACK = -2

SHEN_FP64 = 0
SHEN_FP32_REFINE = 1
SHEN_QUAD_GC = 0
SHEN_QUAD_GL = 1
SHEN_HELMHOLTZ = 0
SHEN_BIHARMONIC = 1
SHEN_SPACE = {"chebyshev": 0, "dirichlet": 1, "biharmonic": 2}


class ShenOpts(C.Structure):
    _fields_ = [
        ("stream", C.c_void_p),
        ("precision", C.c_int32),
        ("transpose", C.c_int32),
        ("quad", C.c_int32),
        ("refine_max", C.c_int32),
        ("refine_tol", C.c_double),
        ("info", C.c_void_p),
        ("variant", C.c_int32),
        ("chunk", C.c_int32),
        ("iters", C.c_void_p),
        ("work", C.c_void_p),
        ("work_bytes", C.c_int64),
    ]


class ShenProblem(C.Structure):
    _fields_ = [
        ("family", C.c_int32),
        ("N", C.c_int32),
        ("nsys", C.c_int64),
        ("c0", C.c_void_p),
        ("c1", C.c_void_p),
        ("f", C.c_void_p),
        ("u", C.c_void_p),
        ("info", C.c_void_p),
        ("tile_begin", C.c_int64),
        ("sys_per_tile", C.c_int32),
        ("chunk", C.c_int32),
    ]


# (name, restype, argtypes) of every exported entry point, in header order
_VP = C.c_void_p
SIGNATURES = [
    ("shen_opts_default", None, [C.POINTER(ShenOpts)]),
    ("shen_abi_version", C.c_int, []),
    ("shen_status_string", C.c_char_p, [C.c_int]),
    ("shen_max_n", C.c_int32, [C.c_int32, C.c_int32]),
    ("shen_wave_config", C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    ("helmholtz_solve", C.c_int, [C.c_int32, C.c_int64, _VP, _VP, _VP, C.POINTER(ShenOpts)]),
    ("biharmonic_solve", C.c_int, [C.c_int32, C.c_int64, _VP, _VP, _VP, _VP, C.POINTER(ShenOpts)]),
    ("helmholtz_adjoint", C.c_int, [C.c_int32, C.c_int64, _VP, _VP, _VP, _VP, _VP, C.POINTER(ShenOpts)]),
    ("biharmonic_adjoint", C.c_int, [C.c_int32, C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP, _VP, C.POINTER(ShenOpts)]),
    ("shen_factor_bytes", C.c_int64, [C.c_int32, C.c_int32, C.POINTER(ShenOpts)]),
    ("helmholtz_factor", C.c_int, [C.c_int32, C.c_int64, _VP, _VP, C.POINTER(ShenOpts)]),
    ("biharmonic_factor", C.c_int, [C.c_int32, C.c_int64, _VP, _VP, _VP, C.POINTER(ShenOpts)]),
    ("helmholtz_solve_factored", C.c_int, [C.c_int32, C.c_int64, _VP, _VP, _VP, _VP, C.POINTER(ShenOpts)]),
    ("biharmonic_solve_factored", C.c_int, [C.c_int32, C.c_int64, _VP, _VP, _VP, _VP, _VP, C.POINTER(ShenOpts)]),
    ("helmholtz_adjoint_factored", C.c_int, [C.c_int32, C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP, C.POINTER(ShenOpts)]),
    ("biharmonic_adjoint_factored", C.c_int,
     [C.c_int32, C.c_int64, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, C.POINTER(ShenOpts)]),
    ("helmholtz_matvec", C.c_int, [C.c_int32, C.c_int64, _VP, _VP, _VP, C.POINTER(ShenOpts)]),
    ("biharmonic_matvec", C.c_int, [C.c_int32, C.c_int64, _VP, _VP, _VP, _VP, C.POINTER(ShenOpts)]),
    ("dirichlet_mass_solve", C.c_int, [C.c_int32, C.c_int64, _VP, _VP, C.POINTER(ShenOpts)]),
    ("biharmonic_mass_solve", C.c_int, [C.c_int32, C.c_int64, _VP, _VP, C.POINTER(ShenOpts)]),
    ("dirichlet_derivative_solve", C.c_int, [C.c_int32, C.c_int64, _VP, _VP, C.POINTER(ShenOpts)]),
    ("helmholtz_rhs", C.c_int, [C.c_int32, C.c_int64, _VP, C.c_double, C.c_double, _VP, _VP, _VP, C.POINTER(ShenOpts)]),
    ("biharmonic_rhs", C.c_int, [C.c_int32, C.c_int64, _VP, C.c_double, C.c_double, _VP, _VP, _VP, C.POINTER(ShenOpts)]),
    ("shen_scalar_product", C.c_int, [C.c_int32, C.c_int64, C.c_int32, _VP, _VP, C.POINTER(ShenOpts)]),
    ("shen_forward_transform", C.c_int, [C.c_int32, C.c_int64, C.c_int32, _VP, _VP, C.POINTER(ShenOpts)]),
    ("shen_backward_transform", C.c_int, [C.c_int32, C.c_int64, C.c_int32, _VP, _VP, C.POINTER(ShenOpts)]),
    ("shen_batched_plan", C.c_int64, [C.POINTER(ShenProblem), C.c_int32, C.POINTER(ShenOpts)]),
    ("shen_batched_work_bytes", C.c_int64, [C.c_int32]),
    ("batched_solve", C.c_int, [C.POINTER(ShenProblem), C.c_int32, _VP, C.POINTER(ShenOpts)]),
    ("shen_batched_static_bytes", C.c_int64, []),
    ("batched_solve_static", C.c_int, [C.POINTER(ShenProblem), C.c_int32, C.POINTER(ShenOpts)]),
]

_lib = None


def lib() -> C.CDLL:
    """The loaded library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                "(there is no CPU fallback)")
        handle = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


class ShenError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib().shen_status_string(code).decode()
        super().__init__(f"{where}: {msg} (code {code})")
        self.code = code


def check(code: int, where: str) -> None:
    if code != SHEN_OK:
        raise ShenError(code, where)


def default_opts() -> ShenOpts:
    o = ShenOpts()
    lib().shen_opts_default(C.byref(o))
    return o
