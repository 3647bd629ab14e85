"""ctypes binding of libprosper.so (argument marshalling only).

Every computation runs in the HIP library; this module only converts torch
tensors to device pointers, passes the current HIP stream and raises on a
non-zero status.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
# always the in-tree build: tests and the benchmark must exercise this library
LIB_PATH = os.path.join(_HERE, "libprosper.so")

MODELS = {"bsc": 0, "tsc": 1, "mca": 2, "mmca": 3, "dsc": 4}
PRECISIONS = {"fp32": 0, "bf16": 1, "bf16x1": 2}
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EBUSY",
          -5: "ENOTFOUND", -6: "ETIMEDOUT"}

MAX_HPRIME, MAX_D, MAX_H, MAX_TOPK, MAX_STATES = 32, 1024, 1024, 8, 1 << 20
MAX_VALUES = 8  # DSC value count


class ProsperError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


FLAG_FACTOR_B = 1  # PROSPER_FLAG_FACTOR_B
FLAG_ZERO_ACC = 2  # PROSPER_FLAG_ZERO_ACC


class Args(C.Structure):
    _fields_ = [("model", C.c_int32), ("precision", C.c_int32), ("N", C.c_int64),
                ("D", C.c_int32), ("H", C.c_int32), ("Hprime", C.c_int32),
                ("gamma", C.c_int32), ("pi", C.c_double), ("sigma", C.c_double),
                ("theta_dev", C.c_void_p), ("topk", C.c_int32), ("accumulate", C.c_int32),
                ("flags", C.c_uint32), ("beta", C.c_float),
                ("nvalues", C.c_int32), ("phi", C.c_float * MAX_VALUES),
                ("pv", C.c_double * MAX_VALUES)]


class PointOut(C.Structure):
    _fields_ = [("sel", C.c_void_p), ("s_mean", C.c_void_p), ("logL", C.c_void_p),
                ("top_mask", C.c_void_p), ("top_q", C.c_void_p), ("flagged", C.c_void_p),
                ("k_mean", C.c_void_p), ("res", C.c_void_p)]


class Acc(C.Structure):
    _fields_ = [("A", C.c_void_p), ("B", C.c_void_p), ("scal", C.c_void_p),
                ("vcount", C.c_void_p)]


EXPORTS = [
    "prosper_ctx_create", "prosper_ctx_destroy", "prosper_last_error",
    "prosper_validate_args", "prosper_state_count", "prosper_state_table",
    "prosper_estep", "prosper_mstep", "prosper_mstep_et", "prosper_serve", "prosper_serve_submit",
    "prosper_serve_wait", "prosper_serve_wait_stages", "prosper_serve_stop",
    "prosper_profile", "prosper_profile_only", "prosper_profile_read",
    "prosper_estep_static", "prosper_dsc_state_count", "prosper_dsc_state_table",
]

_lib: Optional[C.CDLL] = None


def load() -> C.CDLL:
    """Load libprosper.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1908_06843_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, u32, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_double
    sz = C.c_size_t
    lib.prosper_ctx_create.argtypes = [C.c_int, sz, C.POINTER(vp)]
    lib.prosper_ctx_create.restype = i32
    lib.prosper_ctx_destroy.argtypes = [vp]
    lib.prosper_ctx_destroy.restype = None
    lib.prosper_last_error.argtypes = [vp]
    lib.prosper_last_error.restype = C.c_char_p
    lib.prosper_validate_args.argtypes = [C.POINTER(Args)]
    lib.prosper_validate_args.restype = i32
    lib.prosper_state_count.argtypes = [i32, i32, i32, C.POINTER(i64)]
    lib.prosper_state_count.restype = i32
    lib.prosper_state_table.argtypes = [i32, i32, i32, vp, vp, i64]
    lib.prosper_state_table.restype = i32
    lib.prosper_dsc_state_count.argtypes = [i32, i32, i32, C.POINTER(i64)]
    lib.prosper_dsc_state_count.restype = i32
    lib.prosper_dsc_state_table.argtypes = [i32, i32, i32, vp, vp, i64]
    lib.prosper_dsc_state_table.restype = i32
    lib.prosper_estep.argtypes = [vp, C.POINTER(Args), vp, vp, C.POINTER(PointOut),
                                  C.POINTER(Acc), vp]
    lib.prosper_estep.restype = i32
    lib.prosper_estep_static.argtypes = [C.POINTER(Args), vp, vp, C.POINTER(PointOut),
                                         C.POINTER(Acc), vp]
    lib.prosper_estep_static.restype = i32
    lib.prosper_mstep.argtypes = [vp, C.POINTER(Args), C.POINTER(Acc), vp, vp, vp, vp]
    lib.prosper_mstep.restype = i32
    lib.prosper_mstep_et.argtypes = [vp, C.POINTER(Args), C.POINTER(Acc), vp, vp, vp, vp, vp, vp,
                                     vp]
    lib.prosper_mstep_et.restype = i32
    lib.prosper_serve.argtypes = [vp, vp, i32, i32, i32, i32, dbl, dbl, i32, sz, i32, i32, i32,
                                  C.POINTER(vp)]
    lib.prosper_serve.restype = i32
    lib.prosper_serve_submit.argtypes = [vp, vp, i64, i32, i32, i32, C.POINTER(PointOut),
                                         C.POINTER(C.c_uint64)]
    lib.prosper_serve_submit.restype = i32
    lib.prosper_serve_wait.argtypes = [vp, C.c_uint64, i64, C.POINTER(dbl)]
    lib.prosper_serve_wait.restype = i32
    lib.prosper_serve_wait_stages.argtypes = [vp, C.c_uint64, i64, C.POINTER(dbl)]
    lib.prosper_serve_wait_stages.restype = i32
    lib.prosper_serve_stop.argtypes = [vp]
    lib.prosper_serve_stop.restype = i32
    lib.prosper_profile.argtypes = [vp, i32]
    lib.prosper_profile.restype = i32
    lib.prosper_profile_only.argtypes = [vp, C.c_char_p]
    lib.prosper_profile_only.restype = i32
    lib.prosper_profile_read.argtypes = [vp, i32, C.POINTER(C.c_char_p), C.POINTER(dbl),
                                         C.POINTER(i64)]
    lib.prosper_profile_read.restype = i32
    _lib = lib
    return lib


def last_error(ctx=None) -> str:
    return load().prosper_last_error(ctx).decode(errors="replace")


def check(status: int, ctx=None):
    if status != 0:
        raise ProsperError(status, last_error(ctx))


def make_args(model: str, precision: str, N: int, D: int, H: int, Hprime: int, gamma: int,
              pi: float = 0.5, sigma: float = 1.0, theta_dev: Optional[int] = None,
              topk: int = 0, accumulate: int = 0, flags: int = 0, beta: float = 1.0,
              phi=None, pv=None) -> Args:
    """Argument block; `phi` and `pv` (DSC) are the value set and its prior."""
    a = Args(MODELS[model], PRECISIONS[precision], N, D, H, Hprime, gamma, float(pi),
             float(sigma), theta_dev, topk, accumulate, flags, float(beta))
    if phi is not None:
        phi = [float(x) for x in phi]
        if len(phi) > MAX_VALUES:
            raise ValueError(f"at most {MAX_VALUES} DSC values")
        a.nvalues = len(phi)
        for v, x in enumerate(phi):
            a.phi[v] = x
    if pv is not None:
        pv = [float(x) for x in pv]
        if len(pv) > MAX_VALUES:
            raise ValueError(f"at most {MAX_VALUES} DSC values")
        for v, x in enumerate(pv):
            a.pv[v] = x
    return a


def state_count(model: str, Hprime: int, gamma: int) -> int:
    n = C.c_int64(0)
    check(load().prosper_state_count(MODELS[model], Hprime, gamma, C.byref(n)))
    return n.value


def state_table(model: str, Hprime: int, gamma: int):
    """Canonical state table from the library (host-side builder)."""
    import numpy as np
    n = state_count(model, Hprime, gamma)
    act = np.zeros(n, dtype=np.uint32)
    sgn = np.zeros(n, dtype=np.uint32)
    check(load().prosper_state_table(MODELS[model], Hprime, gamma,
                                     act.ctypes.data_as(C.c_void_p),
                                     sgn.ctypes.data_as(C.c_void_p), n))
    return act, sgn


def dsc_state_count(nvalues: int, Hprime: int, gamma: int) -> int:
    n = C.c_int64(0)
    check(load().prosper_dsc_state_count(nvalues, Hprime, gamma, C.byref(n)))
    return n.value


def dsc_state_table(nvalues: int, Hprime: int, gamma: int):
    """DSC state table from the library: active masks and packed value codes."""
    import numpy as np
    n = dsc_state_count(nvalues, Hprime, gamma)
    act = np.zeros(n, dtype=np.uint32)
    codes = np.zeros(n, dtype=np.uint32)
    check(load().prosper_dsc_state_table(nvalues, Hprime, gamma,
                                         act.ctypes.data_as(C.c_void_p),
                                         codes.ctypes.data_as(C.c_void_p), n))
    return act, codes


def validate(args: Args) -> int:
    return load().prosper_validate_args(C.byref(args))
