"""Build and load the oracle's plain-C elimination (``ge_rank.c``).

Test infrastructure only: compiled with gcc, loaded with ctypes, and used by the
tests and the benchmark's CPU-baseline leg.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ge_rank.c")
_LIB = os.path.join(_HERE, "_ge_rank.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ge_rank.c into a shared object next to it."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_rank_modp.restype = ctypes.c_int64
        lib.oracle_rank_modp.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]
        _lib = lib
    return _lib


def rank_modp_c(m: int, n: int, row_ptr, col_idx, val, p: int) -> int:
    """Rank over GF(p) by the plain-C sparse elimination."""
    lib = _load()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    vv = np.ascontiguousarray(val, dtype=np.int32)
    r = lib.oracle_rank_modp(int(m), int(n), rp.ctypes.data, ci.ctypes.data, vv.ctypes.data, int(p))
    if r < 0:
        raise RuntimeError("oracle_rank_modp failed (bad input or out of memory)")
    return int(r)


def rank_csr_c(A, p: int) -> int:
    return rank_modp_c(A.m, A.n, A.row_ptr, A.col_idx, A.val, p)
