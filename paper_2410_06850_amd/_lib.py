"""ctypes binding of libmsmg.so (argument marshalling only).

Names and arguments mirror include/msmg.h.  Device pointers are passed as
integers (e.g. ``tensor.data_ptr()``), streams as ``hipStream_t`` handles
(``torch.cuda.current_stream().cuda_stream``).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsmg.so")

MSMG_F64, MSMG_F32, MSMG_BF16 = 0, 1, 2
MSMG_PC_MULTIGRID, MSMG_PC_SMOOTHER = 0, 1
MSMG_OK, MSMG_MAXIT, MSMG_BREAKDOWN, MSMG_NONFINITE = 0, 1, 2, 3
MSMG_EINVAL, MSMG_ENOMEM, MSMG_EHIP, MSMG_ESETUP, MSMG_ESINGULAR, MSMG_ESTATE, MSMG_ETIMEOUT = -1, -2, -3, -4, -5, -6, -7

MSMG_Q1, MSMG_TPFA = 0, 1
EXPORT_LOCAL_EVALS, EXPORT_RC, EXPORT_AC, EXPORT_CC_EVALS, EXPORT_ACC, EXPORT_CELL_STATUS = range(6)


class Options(ctypes.Structure):
    _fields_ = [
        ("H", ctypes.c_int),
        ("sd", ctypes.c_int),
        ("Lc", ctypes.c_int),
        ("Lcc", ctypes.c_int),
        ("cheb_degree", ctypes.c_int),
        ("cheb_lo", ctypes.c_double),
        ("cheb_hi", ctypes.c_double),
        ("vcycle_dtype", ctypes.c_int),
        ("rho_v_dtype", ctypes.c_int),
        ("basis_dtype", ctypes.c_int),
        ("pc_kind", ctypes.c_int),
        ("check_interval", ctypes.c_int),
        ("eig_block", ctypes.c_int),
        ("eig_degree", ctypes.c_int),
        ("eig_maxit", ctypes.c_int),
        ("eig_tol", ctypes.c_double),
        ("cc_block", ctypes.c_int),
        ("cc_degree", ctypes.c_int),
        ("cc_maxit", ctypes.c_int),
        ("autotune", ctypes.c_int),
        ("tune_cache", ctypes.c_char_p),
        ("timing", ctypes.c_int),
        ("eig_warm_start", ctypes.c_int),
        ("rho_storage", ctypes.c_int),
        ("lean_memory", ctypes.c_int),
        ("cc_group", ctypes.c_int),
        ("coarse_fused", ctypes.c_int),
        ("pair_rhs", ctypes.c_int),
        ("discretisation", ctypes.c_int),
        ("lc_threshold", ctypes.c_double),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("iterations", ctypes.c_int),
        ("restarts", ctypes.c_int),
        ("rel_res", ctypes.c_double),
        ("solve_ms", ctypes.c_double),
        ("setup_ms", ctypes.c_double),
        ("n_c", ctypes.c_int),
        ("n_cc", ctypes.c_int),
        ("eig_unconverged", ctypes.c_int),
        ("cc_unconverged", ctypes.c_int),
        ("eig_ties", ctypes.c_int),
        ("timed", ctypes.c_int),
        ("apply_ms", ctypes.c_double),
        ("precond_ms", ctypes.c_double),
        ("setup_phase_ms", ctypes.c_double * 4),
        ("setup_dense_ms", ctypes.c_double),
        ("setup_dense_gflop", ctypes.c_double),
    ]


class Plan(ctypes.Structure):
    _fields_ = [
        ("ncx", ctypes.c_int), ("ncy", ctypes.c_int), ("ncz", ctypes.c_int), ("ncells", ctypes.c_int),
        ("nccx", ctypes.c_int), ("nccy", ctypes.c_int), ("nccz", ctypes.c_int), ("ncc", ctypes.c_int),
        ("n_c", ctypes.c_int), ("n_cc", ctypes.c_int),
        ("max_cell_nodes", ctypes.c_int), ("max_cc_dofs", ctypes.c_int),
        ("nodes", ctypes.c_longlong), ("elements", ctypes.c_longlong),
        ("device_bytes", ctypes.c_longlong),
    ]


# (name, restype, argtypes) of every exported symbol declared in include/msmg.h
_VP, _I, _D, _SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
SIGNATURES = [
    ("msmg_default_options", None, [ctypes.POINTER(Options)]),
    ("msmg_query_plan", _I, [_I, _I, _I, ctypes.POINTER(Options), ctypes.POINTER(Plan)]),
    ("msmg_create", _I, [ctypes.POINTER(_VP), _I, _I, _I, _D, _D, _D, ctypes.POINTER(Options)]),
    ("msmg_setup", _I, [_VP, _VP, _I, _D, _D, _I, _VP, _VP, _VP]),
    ("msmg_solve", _I, [_VP, _VP, _VP, _VP, _I, _D, _I, ctypes.POINTER(Info), _VP]),
    ("msmg_solve_adjoint", _I, [_VP, _VP, _VP, _VP, _I, _D, _I, ctypes.POINTER(Info), _VP]),
    ("msmg_solve_pair", _I, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _D, _I, ctypes.POINTER(Info), ctypes.POINTER(Info),
                             _VP]),
    ("msmg_sensitivity", _I, [_VP, _VP, _VP, _VP, _VP]),
    ("msmg_apply", _I, [_VP, _VP, _VP, _VP]),
    ("msmg_precondition", _I, [_VP, _VP, _VP, _VP]),
    ("msmg_element_load", _I, [_VP, _VP, _D, _VP, _VP]),
    ("msmg_sensitivity_heat_source", _I, [_VP, _VP, _VP, _D, _VP, _VP]),
    ("msmg_heat_source_load", _I, [_VP, _D, _VP, _VP]),
    ("msmg_stream_ceiling", _I, [_VP, _VP, _VP, ctypes.c_longlong, ctypes.c_longlong, _I, ctypes.POINTER(_D), _VP]),
    ("msmg_time_apply", _I, [_VP, _VP, _I, ctypes.POINTER(_D), _VP]),
    ("msmg_dot", _I, [_VP, _VP, _VP, ctypes.c_longlong, _VP, _VP]),
    ("msmg_scale", _I, [_VP, ctypes.c_longlong, _D, _VP, _VP, _VP]),
    ("msmg_prolong_nodal", _I, [_I, _I, _I, _VP, _VP, _VP]),
    ("msmg_prolong_element", _I, [_I, _I, _I, _VP, _VP, _I, _VP]),
    ("msmg_density_filter", _I, [_I, _I, _I, _D, _VP, _VP, _I, _VP]),
    ("msmg_oc_update", _I, [_VP, _VP, _VP, _VP, _D, _D, _D, _D, _VP, _VP, _VP]),
    ("msmg_mma_update", _I, [_VP, _I, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _D, _D, _D, _VP, _VP, _VP]),
    ("msmg_oc_update_noalloc", _I, [_I, _I, _I, _VP, _VP, _VP, _D, _D, _D, _D, _VP, _VP, _VP]),
    ("msmg_export", _I, [_VP, _I, _VP, _SZ]),
    ("msmg_destroy", None, [_VP]),
    ("msmg_last_error", ctypes.c_char_p, []),
]

_lib = None


class MissingLibrary(RuntimeError):
    pass


def lib():
    """Load libmsmg.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MissingLibrary(
                f"{LIB_PATH} is missing: build it with `python -m paper_2410_06850_amd.build_lib`")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error():
    return lib().msmg_last_error().decode(errors="replace")


class MsmgError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where} failed with code {code}: {last_error()}")
        self.code = code


def check(code, where):
    if code < 0:
        raise MsmgError(code, where)
    return code


def default_options(**kw):
    o = Options()
    lib().msmg_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        if k == "tune_cache" and isinstance(v, str):
            v = v.encode()
        setattr(o, k, v)
    return o


def query_plan(nx, ny, nz, opts=None):
    p = Plan()
    check(lib().msmg_query_plan(nx, ny, nz, ctypes.byref(opts) if opts is not None else None, ctypes.byref(p)),
          "msmg_query_plan")
    return p
