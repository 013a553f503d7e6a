"""ctypes declarations of the C ABI in include/adlbr.h (libadlbr.so).

This module only loads the library and declares argument types; it does no
computation.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libadlbr.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "adlbr.h")

# adlbr.h constants
OK = 0
E_INVALID, E_NOT_SPD, E_RANGE, E_NOMEM, E_HIP, E_NOT_CONVERGED, E_UNSUPPORTED = range(-1, -8, -1)
ST_NOT_SPD, ST_RANGE, ST_ITER, ST_CLAMPED, ST_STENCIL, ST_INCOMING = 1, 2, 4, 8, 16, 32
F64, F32, BF16, F16 = 0, 1, 2, 3
NEUMANN, PERIODIC, REFLECT = 0, 1, 2
OP_WIDE = 1
OP_TILED = 2
OP_RECORDS = 4
DT_ABS, DT_CFL = 0, 1
MAP_CED, MAP_EED = 0, 1


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("boundary", ctypes.c_int32),
                ("n", ctypes.c_int64 * 3)]


class TensorParams(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("rho", ctypes.c_double),
                ("alpha", ctypes.c_double), ("C", ctypes.c_double),
                ("eig_map", ctypes.c_int32)]


class SolveParams(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("x0_zero", ctypes.c_int32),
                ("tol", ctypes.c_double), ("net", ctypes.c_void_p)]


class SolveReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("fell_back", ctypes.c_int32), ("net_iters", ctypes.c_int32),
                ("rel_res", ctypes.c_double), ("time_ms", ctypes.c_double),
                ("restarts", ctypes.c_int32), ("fallback_reason", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


SOLVE_JACOBI_PCG, SOLVE_FCG_NET = 0, 1


class NetStruct(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("width", ctypes.c_int32),
                ("hidden", ctypes.c_int32), ("nfeat", ctypes.c_int32),
                ("params", ctypes.c_void_p), ("features", ctypes.c_void_p),
                ("hidden_act", ctypes.c_void_p), ("gates", ctypes.c_void_p),
                ("gates8", ctypes.c_void_p), ("scratch", ctypes.c_void_p),
                ("layers", ctypes.c_void_p)]


class AdlbrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"adlbr error {code}: {msg}")
        self.code = code


_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_D = ctypes.c_double
_SZ = ctypes.c_size_t
_GP = ctypes.POINTER(Grid)

SIGNATURES = {
    "adlbr_last_error": ([], ctypes.c_char_p),
    "adlbr_version": ([], _I),
    "adlbr_build_stencils": ([_GP, _P, _I, _P, _P, _I, _P, _P], _I),
    "adlbr_operator_workspace": ([_GP, _I, _I, ctypes.POINTER(_SZ)], _I),
    "adlbr_operator_create": ([_GP, _P, _P, _I, _I, _I, _P, _SZ, _P, _P,
                               ctypes.POINTER(_P)], _I),
    "adlbr_operator_destroy": ([_P], _I),
    "adlbr_operator_rebuild": ([_P, _P, _P, _I, _P, _P], _I),
    "adlbr_step_multi": ([_P, _P, _P, _I, _D, _I, _I64, _P], _I),
    "adlbr_operator_dt_cfl": ([_P, ctypes.POINTER(_D), _P], _I),
    "adlbr_operator_diagonal": ([_P, _P, _I, _P], _I),
    "adlbr_apply": ([_P, _P, _P, _P], _I),
    "adlbr_step": ([_P, _P, _P, _D, _I, _I64, _P], _I),
    "adlbr_batch_workspace": ([_I, ctypes.POINTER(_SZ)], _I),
    "adlbr_batch_create": ([_I, _P, _P, _P, _P, _I, _P, _SZ, _P, ctypes.POINTER(_P)], _I),
    "adlbr_batch_tune": ([_P, _I, _I, _P], _I),
    "adlbr_batch_tune_save": ([ctypes.c_char_p], _I),
    "adlbr_batch_tune_load": ([ctypes.c_char_p], _I),
    "adlbr_batch_tune_clear": ([], _I),
    "adlbr_batch_tune_lookup": ([_I, _I64, _I, ctypes.POINTER(_I), ctypes.POINTER(_I),
                                 ctypes.POINTER(_SZ)], _I),
    "adlbr_batch_set_variant": ([_P, _I, _I, _SZ, _P], _I),
    "adlbr_batch_variant": ([_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I),
                             ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_SZ)], _I),
    "adlbr_batch_run": ([_P, _I64, _I, _P], _I),
    "adlbr_batch_destroy": ([_P], _I),
    "adlbr_tensor_workspace": ([_GP, _I, ctypes.POINTER(_SZ)], _I),
    "adlbr_solve_workspace": ([_P, _I, ctypes.POINTER(_SZ)], _I),
    "adlbr_solve": ([_P, _D, _P, _P, ctypes.POINTER(SolveParams), _P, _SZ,
                     ctypes.POINTER(SolveReport), _P], _I),
    "adlbr_structure_tensor": ([_GP, _P, _I, ctypes.POINTER(TensorParams), _P, _P, _SZ, _P], _I),
    "adlbr_structure_tensor_vec": ([_GP, _P, _I, _I, ctypes.POINTER(TensorParams), _P, _P, _SZ,
                                    _P], _I),
    "adlbr_structure_tensor_noalloc": ([_GP, _P, _I, ctypes.POINTER(TensorParams), _P, _P], _I),
    "adlbr_net_param_count": ([_I, _I, _I, ctypes.POINTER(_SZ)], _I),
    "adlbr_net_features": ([_P, _D, _P, _P], _I),
    "adlbr_net_gates": ([_P, _P, _P], _I),
    "adlbr_net_forward": ([_P, _P, _P, _P, _P, _P], _I),
    "adlbr_net_precondition": ([_P, _P, _P, _P, _P], _I),
    "adlbr_net_backward": ([_P, _P, _P, _P, _P, _P, _P, _P, _SZ, _P], _I),
    "adlbr_net_gates_backward": ([_P, _P, _P, _P, _P, _SZ, _P], _I),
    "adlbr_net_workspace": ([_P, _P, ctypes.POINTER(_SZ)], _I),
    "adlbr_net_loss_grad": ([_P, _D, _P, _P, _P, _P, _P, _SZ, _P], _I),
    "adlbr_net_adam": ([_P, _P, _P, _P, _I64, ctypes.c_int32, _D, _D, _D, _D, _D, _P], _I),
    "adlbr_residual": ([_P, _D, _P, _P, _P, _P], _I),
}

_lib = None


def load():
    """Load libadlbr.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def check(rc: int):
    if rc != OK:
        msg = load().adlbr_last_error().decode(errors="replace")
        raise AdlbrError(rc, msg)


def declared_symbols(header: str = HEADER):
    """Names of the functions declared in the public header."""
    import re
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(adlbr_[a-z0-9_]+)\s*\(", text)))
