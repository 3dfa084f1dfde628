"""ctypes binding of libmvn.so (argument marshalling only).

Every function here has the name of the C entry point it calls (see
include/mvn.h).  torch supplies device memory and the current stream; all
arithmetic happens in the library's HIP kernels.  There is no fallback: if
the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import c_double, c_int, c_size_t, c_uint64, c_void_p, POINTER

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmvn.so")

MVN_FP64, MVN_FP32, MVN_BF16, MVN_BF16X3 = 0, 1, 2, 3
MVN_CHOL_ADAPTIVE, MVN_CHOL_UNIFORM, MVN_CHOL_FP64 = 0, 1, 2


class MvnMatern(ctypes.Structure):
    _fields_ = [("sigma2", c_double), ("beta", c_double), ("nu", c_double), ("nugget", c_double)]


class MvnOptions(ctypes.Structure):
    _fields_ = [("tile", c_int), ("precision", c_int), ("periodize", c_int), ("sweep_rows", c_int),
                ("tlr_eps", c_double), ("max_rank", c_int), ("chol_mode", c_int), ("chol_tol", c_double)]


MVN_FACTOR_TLR = 1
MVN_FACTOR_TLR_COMPACT = 2


class MvnFactor(ctypes.Structure):
    _fields_ = [("n", c_int), ("ld", c_int), ("precision", c_int), ("flags", c_int),
                ("L", c_void_p), ("info", c_void_p), ("L_low", c_void_p),
                ("tile", c_int), ("rank_stride", c_int), ("U", c_void_p), ("Vt", c_void_p),
                ("ranks", c_void_p), ("tlr_eps", c_double), ("max_rank", c_int), ("chol_mode", c_int),
                ("update_counts", c_void_p)]


class MvnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mvn error {code}: {msg}")
        self.code = code


_lib = None

# name -> (restype, argtypes)
SIGNATURES = {
    "mvn_factor_bytes": (c_int, [c_int, POINTER(MvnOptions), POINTER(c_size_t)]),
    "mvn_cholesky_workspace_bytes": (c_int, [c_int, POINTER(MvnOptions), POINTER(c_size_t)]),
    "mvn_prob_workspace_bytes": (c_int, [c_int, c_int, c_int, POINTER(MvnOptions), POINTER(c_size_t)]),
    "mvn_prob_workspace_bytes_factor": (c_int, [POINTER(MvnFactor), c_int, c_int, POINTER(MvnOptions),
                                                POINTER(c_size_t), c_void_p]),
    "mvn_prob_prefix_workspace_bytes": (c_int, [POINTER(MvnFactor), c_int, c_int, POINTER(MvnOptions),
                                                 POINTER(c_size_t), c_void_p]),
    "mvn_prob_prefix": (c_int, [POINTER(MvnFactor), c_void_p, c_void_p, c_void_p, c_int, c_int, c_uint64,
                                POINTER(MvnOptions), c_void_p, c_size_t, c_void_p, c_void_p]),
    "mvn_cholesky_permuted_workspace_bytes": (c_int, [c_int, POINTER(MvnOptions), POINTER(c_size_t)]),
    "mvn_cholesky_permuted": (c_int, [c_int, c_void_p, c_int, c_void_p, POINTER(MvnOptions), c_void_p, c_size_t,
                                      c_void_p, c_size_t, POINTER(MvnFactor), c_void_p]),
    "mvn_posterior_workspace_bytes": (c_int, [c_int, c_int, POINTER(MvnOptions), POINTER(c_size_t)]),
    "mvn_posterior": (c_int, [c_int, c_void_p, c_void_p, c_int, c_void_p, c_void_p, POINTER(MvnMatern), c_double,
                              POINTER(MvnOptions), c_void_p, c_size_t, c_void_p, c_void_p, c_void_p,
                              POINTER(c_void_p), POINTER(c_int), c_void_p]),
    "mvn_mc_prefix_workspace_bytes": (c_int, [c_int, c_int, POINTER(MvnOptions), POINTER(c_size_t)]),
    "mvn_mc_prefix": (c_int, [POINTER(MvnFactor), c_void_p, c_void_p, c_void_p, c_int, c_uint64,
                              POINTER(MvnOptions), c_void_p, c_size_t, c_void_p, c_void_p, c_void_p]),
    "mvn_cholesky": (c_int, [c_int, c_void_p, c_int, c_void_p, POINTER(MvnMatern), POINTER(MvnOptions),
                             c_void_p, c_size_t, c_void_p, c_size_t, POINTER(MvnFactor), c_void_p]),
    "mvn_prob": (c_int, [POINTER(MvnFactor), c_void_p, c_void_p, c_void_p, c_int, c_int, c_uint64,
                         POINTER(MvnOptions), c_void_p, c_size_t, c_void_p, c_void_p, c_void_p]),
    "mvn_prob_static": (c_int, [POINTER(MvnFactor), c_void_p, c_void_p, c_void_p, c_int, c_int, c_uint64,
                                POINTER(MvnOptions), c_void_p, c_void_p, c_void_p]),
    "mvn_prob_grad_workspace_bytes": (c_int, [c_int, c_int, c_int, POINTER(MvnOptions), POINTER(c_size_t)]),
    "mvn_prob_grad": (c_int, [POINTER(MvnFactor), c_void_p, c_void_p, c_void_p, c_int, c_int, c_uint64,
                              POINTER(MvnOptions), c_void_p, c_size_t, c_void_p, c_void_p, c_void_p,
                              c_void_p, c_void_p]),
    "mvn_batch_plan_bytes": (c_int, [c_int, POINTER(c_size_t)]),
    "mvn_batch_plan": (c_int, [c_int, c_void_p, c_int, c_int, POINTER(MvnOptions), c_void_p, c_size_t,
                               POINTER(c_size_t), POINTER(c_size_t)]),
    "mvn_prob_batch": (c_int, [c_int, c_void_p, c_void_p, c_void_p, c_void_p, POINTER(MvnMatern), c_void_p,
                               c_void_p, c_void_p, c_int, c_int, c_uint64, POINTER(MvnOptions), c_void_p,
                               c_size_t, c_void_p, c_size_t, c_void_p, c_void_p, c_void_p]),
    "mvn_exceedance_order_workspace_bytes": (c_int, [c_int, POINTER(c_size_t)]),
    "mvn_exceedance_order": (c_int, [c_int, c_void_p, c_void_p, c_double, c_void_p, c_void_p, c_void_p, c_size_t,
                                     c_void_p]),
    "mvn_tlr_compact_bytes": (c_int, [POINTER(MvnFactor), POINTER(c_size_t), c_void_p]),
    "mvn_tlr_compact": (c_int, [POINTER(MvnFactor), c_void_p, c_size_t, POINTER(MvnFactor), c_void_p]),
    "mvn_tlr_dense_bytes": (c_int, [POINTER(MvnFactor), POINTER(c_size_t)]),
    "mvn_tlr_dense": (c_int, [POINTER(MvnFactor), c_void_p, c_size_t, POINTER(MvnFactor), c_void_p]),
    "mvn_last_error": (ctypes.c_char_p, []),
    "mvn_version": (c_int, []),
}


def lib() -> ctypes.CDLL:
    """Load libmvn.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2405_14892_amd.build`")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def check(code: int) -> None:
    if code != 0:
        raise MvnError(code, lib().mvn_last_error().decode())


def options(tile: int = 256, precision: int = MVN_FP64, periodize: bool = False,
            tlr_eps: float = 0.0, max_rank: int = 0, sweep_rows: int = 0, chol_mode: int = MVN_CHOL_ADAPTIVE,
            chol_tol: float = 0.0) -> MvnOptions:
    return MvnOptions(tile, precision, 1 if periodize else 0, sweep_rows, tlr_eps, max_rank, chol_mode, chol_tol)
