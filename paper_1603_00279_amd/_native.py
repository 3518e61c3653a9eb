"""ctypes binding of libtsfcde.so (declarations in include/tsfcde.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  torch is imported first so that the library binds to the HIP
runtime torch has already loaded (one runtime per process).
"""
from __future__ import annotations

import ctypes
import os
import re
from ctypes import POINTER, c_double, c_int32, c_int64, c_size_t, c_void_p, c_char_p

import numpy as np
import torch  # noqa: F401  -- must precede loading the HIP library

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtsfcde.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "tsfcde.h")
HEADERS = [HEADER] + [os.path.join(os.path.dirname(PKG), "include", h) for h in ("tsfcde2d.h", "tsfcde3d.h")]

COEF_FN = ctypes.CFUNCTYPE(c_double, c_double, c_void_p)
IC_FN = ctypes.CFUNCTYPE(c_double, c_double, c_void_p)
SRC_FN = ctypes.CFUNCTYPE(c_double, c_double, c_double, c_void_p)
IC2_FN = ctypes.CFUNCTYPE(c_double, c_double, c_double, c_void_p)
SRC2_FN = ctypes.CFUNCTYPE(c_double, c_double, c_double, c_double, c_void_p)
IC3_FN = ctypes.CFUNCTYPE(c_double, c_double, c_double, c_double, c_void_p)
SRC3_FN = ctypes.CFUNCTYPE(c_double, c_double, c_double, c_double, c_double, c_void_p)

TSFCDE_OK = 0
STATUS = {0: "TSFCDE_OK", -1: "TSFCDE_EINVAL", -2: "TSFCDE_ENOMEM", -3: "TSFCDE_EDEVICE",
          -4: "TSFCDE_ENOCONV", -5: "TSFCDE_EBREAKDOWN", -6: "TSFCDE_ENONFINITE",
          -7: "TSFCDE_EDONE", -8: "TSFCDE_EUNSUPPORTED", -9: "TSFCDE_EACCEPT"}
TSFCDE_EINVAL, TSFCDE_ENOMEM, TSFCDE_EDEVICE = -1, -2, -3
TSFCDE_ENOCONV, TSFCDE_EBREAKDOWN, TSFCDE_ENONFINITE = -4, -5, -6
TSFCDE_EDONE, TSFCDE_EUNSUPPORTED, TSFCDE_EACCEPT = -7, -8, -9
TSFCDE_FP64 = 0
TSFCDE_FP32_REFINED = 1
TSFCDE_FP32_REFINED_FELL_BACK = 2
TSFCDE_WS_ZERO, TSFCDE_WS_PREV, TSFCDE_WS_EXTRAP, TSFCDE_WS_NET = 0, 1, 2, 3
TSFCDE_FLAG_TRUE_RESIDUAL = 1
TSFCDE_FLAG_VERIFY = 2
TSFCDE_FLAG_FORCE_FP32 = 4
TSFCDE_FLAG_NO_FOLD = 8
TSFCDE_FLAG_STRICT_RESIDUAL = 16
TSFCDE_FLAG_CONSTANT_GSF = 32
TSFCDE_FLAG_GRAPHS = 64
TSFCDE_FLAG_NO_TUNE = 128
TSFCDE_METHOD_PCGS, TSFCDE_METHOD_GSF, TSFCDE_METHOD_PBICGSTAB = 0, 1, 2
TSFCDE_KRYLOV_CGS, TSFCDE_KRYLOV_BICGSTAB = 0, 1
TSFCDE_PREC_STRANG, TSFCDE_PREC_TCHAN = 0, 1
TSFCDE_OP_A, TSFCDE_OP_B, TSFCDE_OP_PINV = 0, 1, 2
TSFCDE_SPEC_EMBED, TSFCDE_SPEC_STRANG = 0, 1
TSFCDE_NOALLOC_NMAX = 32768
TSFCDE_NOALLOC_SCRATCH_BYTES = 16777216


class tsfcde_problem(ctypes.Structure):
    _fields_ = [
        ("alpha", c_double), ("beta", c_double), ("a", c_double), ("b", c_double), ("T", c_double),
        ("n", c_int64), ("M", c_int64),
        ("gamma", COEF_FN), ("dplus", COEF_FN), ("dminus", COEF_FN), ("coef_user", c_void_p),
        ("gamma_at", POINTER(c_double)), ("dplus_at", POINTER(c_double)), ("dminus_at", POINTER(c_double)),
        ("phi", IC_FN), ("phi_user", c_void_p),
        ("rtol", c_double), ("maxit", c_int32), ("precision", c_int32), ("warm_start", c_int32),
        ("flags", c_int32), ("f", SRC_FN), ("f_user", c_void_p), ("krylov", c_int32), ("preconditioner", c_int32),
        ("history_tol", c_double),
    ]


class tsfcde_stats(ctypes.Structure):
    _fields_ = [
        ("iters", c_int32), ("outer_iters", c_int32), ("restarts", c_int32), ("status", c_int32),
        ("relres", c_double), ("relres_true", c_double), ("backward_err", c_double), ("seconds", c_double),
        ("precision_used", c_int32), ("guess", c_int32), ("method", c_int32), ("pad", c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# the same record as a numpy structured type (views of stats arrays)
STATS_DTYPE = np.dtype([(k, np.int32 if t is c_int32 else np.float64) for k, t in tsfcde_stats._fields_])
assert STATS_DTYPE.itemsize == ctypes.sizeof(tsfcde_stats)


class tsfcde2d_problem(ctypes.Structure):
    _fields_ = [
        ("alpha", c_double), ("beta_x", c_double), ("beta_y", c_double),
        ("a", c_double), ("b", c_double), ("c", c_double), ("d", c_double), ("T", c_double),
        ("nx", c_int64), ("ny", c_int64), ("M", c_int64),
        ("gamma_x", COEF_FN), ("gamma_y", COEF_FN), ("dplus_x", COEF_FN), ("dminus_x", COEF_FN),
        ("dplus_y", COEF_FN), ("dminus_y", COEF_FN), ("coef_user", c_void_p),
        ("phi", IC2_FN), ("phi_user", c_void_p), ("f", SRC2_FN), ("f_user", c_void_p),
        ("rtol", c_double), ("maxit", c_int32), ("warm_start", c_int32),
    ]


class tsfcde3d_problem(ctypes.Structure):
    _fields_ = [
        ("alpha", c_double), ("beta", c_double * 3), ("lo", c_double * 3), ("hi", c_double * 3), ("T", c_double),
        ("n", c_int64 * 3), ("M", c_int64),
        ("gamma", COEF_FN * 3), ("dplus", COEF_FN * 3), ("dminus", COEF_FN * 3), ("coef_user", c_void_p),
        ("phi", IC3_FN), ("phi_user", c_void_p), ("f", SRC3_FN), ("f_user", c_void_p),
        ("rtol", c_double), ("maxit", c_int32), ("warm_start", c_int32),
    ]


class tsfcde_net_sample(ctypes.Structure):
    _fields_ = [
        ("u_next", c_void_p), ("u0", c_void_p), ("u1", c_void_p), ("u2", c_void_p),
        ("feat", ctypes.c_float * 5), ("pad", ctypes.c_float),
    ]


_SIGS = {
    "tsfcde_workspace_bytes": (c_int32, [POINTER(tsfcde_problem), POINTER(c_size_t)]),
    "tsfcde_plan": (c_int32, [POINTER(tsfcde_problem), c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]),
    "tsfcde_set_state": (c_int32, [c_void_p, c_int64, c_void_p]),
    "tsfcde_step": (c_int32, [c_void_p, c_void_p, c_void_p, POINTER(tsfcde_stats)]),
    "tsfcde_solve": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, POINTER(tsfcde_stats)]),
    "tsfcde_apply": (c_int32, [c_void_p, c_int32, c_int64, c_void_p, c_void_p]),
    "tsfcde_rhs": (c_int32, [c_void_p, c_int64, c_void_p, c_void_p]),
    "tsfcde_weights": (c_int32, [c_void_p, c_void_p]),
    "tsfcde_spectrum": (c_int32, [c_void_p, c_int32, c_void_p]),
    "tsfcde_history": (c_void_p, [c_void_p]),
    "tsfcde_level": (c_int64, [c_void_p]),
    "tsfcde_history_ld": (c_int64, [c_void_p]),
    "tsfcde_embedding_length": (c_int64, [c_void_p]),
    "tsfcde_level_time": (c_double, [c_void_p, c_int64]),
    "tsfcde_nodes": (c_int32, [c_void_p, POINTER(c_double)]),
    "tsfcde_history_soe_fit": (c_int32, [c_double, c_int64, c_double, c_int32, POINTER(c_int32), c_void_p, c_void_p,
                                         c_void_p, POINTER(c_double)]),
    "tsfcde_profile": (c_int32, [c_void_p, c_int32, c_int32]),
    "tsfcde_profile_read": (c_int32, [c_void_p, c_int32, POINTER(c_int64), POINTER(c_double)]),
    "tsfcde_profile_issued": (c_int32, [c_void_p, c_int32, POINTER(c_int64)]),
    "tsfcde_destroy": (c_int32, [c_void_p]),
    "tsfcde_apply_noalloc": (c_int32, [POINTER(tsfcde_problem), c_int32, c_int64, c_void_p, c_void_p, c_void_p]),
    "tsfcde_batch_workspace_bytes": (c_int32, [POINTER(tsfcde_problem), c_int32, POINTER(c_size_t)]),
    "tsfcde_plan_batch": (c_int32, [POINTER(tsfcde_problem), c_int32, c_void_p, c_size_t, c_void_p,
                                    POINTER(c_void_p)]),
    "tsfcde_batch_member": (c_void_p, [c_void_p, c_int32]),
    "tsfcde_batch_set_level": (c_int32, [c_void_p, c_int64]),
    "tsfcde_batch_step": (c_int32, [c_void_p, POINTER(c_void_p), POINTER(tsfcde_stats)]),
    "tsfcde_batch_solve": (c_int32, [c_void_p, POINTER(c_void_p), POINTER(c_int64), POINTER(tsfcde_stats)]),
    "tsfcde_batch_destroy": (c_int32, [c_void_p]),
    "tsfcde_batch_group_count": (c_int32, [c_void_p]),
    "tsfcde_batch_group_info": (c_int32, [c_void_p, c_int32, POINTER(c_int64), POINTER(c_int32), POINTER(c_int32)]),
    "tsfcde_strerror": (c_char_p, [c_int32]),
    "tsfcde_net_param_count": (c_int32, []),
    "tsfcde_net_workspace_bytes": (c_int32, [c_int64, c_int32, POINTER(c_size_t)]),
    "tsfcde_net_create": (c_int32, [c_void_p, c_size_t, c_int64, c_int32, c_void_p, POINTER(c_void_p)]),
    "tsfcde_net_set_params": (c_int32, [c_void_p, POINTER(ctypes.c_float)]),
    "tsfcde_net_get_params": (c_int32, [c_void_p, POINTER(ctypes.c_float)]),
    "tsfcde_level_features": (c_int32, [c_void_p, c_int64, POINTER(ctypes.c_float)]),
    "tsfcde_net_train_step": (c_int32, [c_void_p, POINTER(tsfcde_net_sample), c_int32, c_int64, ctypes.c_float,
                                        POINTER(c_double), POINTER(ctypes.c_float)]),
    "tsfcde_net_predict": (c_int32, [c_void_p, POINTER(tsfcde_net_sample), c_int64, c_void_p]),
    "tsfcde_plan_set_net": (c_int32, [c_void_p, c_void_p]),
    "tsfcde_net_destroy": (c_int32, [c_void_p]),
    "tsfcde2d_workspace_bytes": (c_int32, [POINTER(tsfcde2d_problem), POINTER(c_size_t)]),
    "tsfcde2d_plan": (c_int32, [POINTER(tsfcde2d_problem), c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]),
    "tsfcde2d_set_state": (c_int32, [c_void_p, c_int64, c_void_p]),
    "tsfcde2d_step": (c_int32, [c_void_p, c_void_p, c_void_p, POINTER(tsfcde_stats)]),
    "tsfcde2d_solve": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, POINTER(tsfcde_stats)]),
    "tsfcde2d_apply": (c_int32, [c_void_p, c_int32, c_int64, c_void_p, c_void_p]),
    "tsfcde2d_nodes": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_double)]),
    "tsfcde2d_level_time": (c_double, [c_void_p, c_int64]),
    "tsfcde2d_level": (c_int64, [c_void_p]),
    "tsfcde2d_history": (c_void_p, [c_void_p]),
    "tsfcde2d_destroy": (c_int32, [c_void_p]),
    "tsfcde3d_workspace_bytes": (c_int32, [POINTER(tsfcde3d_problem), POINTER(c_size_t)]),
    "tsfcde3d_plan": (c_int32, [POINTER(tsfcde3d_problem), c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]),
    "tsfcde3d_set_state": (c_int32, [c_void_p, c_int64, c_void_p]),
    "tsfcde3d_step": (c_int32, [c_void_p, c_void_p, c_void_p, POINTER(tsfcde_stats)]),
    "tsfcde3d_solve": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, POINTER(tsfcde_stats)]),
    "tsfcde3d_apply": (c_int32, [c_void_p, c_int32, c_int64, c_void_p, c_void_p]),
    "tsfcde3d_nodes": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_double), POINTER(c_double)]),
    "tsfcde3d_level_time": (c_double, [c_void_p, c_int64]),
    "tsfcde3d_level": (c_int64, [c_void_p]),
    "tsfcde3d_history": (c_void_p, [c_void_p]),
    "tsfcde3d_destroy": (c_int32, [c_void_p]),
}

_LIB = None


def header_symbols(paths=None):
    """Names of the functions declared in include/tsfcde.h, tsfcde2d.h and tsfcde3d.h."""
    names = set()
    for path in (paths or HEADERS):
        text = open(path).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(tsfcde(?:[23]d)?_[a-z0-9_]+)\s*\(", text))
    return sorted(names - {"tsfcde_coef_fn", "tsfcde_ic_fn", "tsfcde_src_fn", "tsfcde2d_ic_fn", "tsfcde2d_src_fn",
                           "tsfcde3d_ic_fn", "tsfcde3d_src_fn"})


def lib():
    """Load libtsfcde.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1603_00279_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


class TsfcdeError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib().tsfcde_strerror(code).decode()
        super().__init__(f"{where}: {STATUS.get(code, code)} ({msg})")
        self.code = code


def check(code: int, where: str):
    if code != TSFCDE_OK:
        raise TsfcdeError(code, where)
    return code
