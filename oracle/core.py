"""ctypes binding of oracle_core.c (test infrastructure only).

``build()`` compiles ``oracle_core.c`` with gcc into ``oracle/_oracle_core.so``
(-O2, no fast-math, OpenMP).  ``dm`` runs the plain C definition.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_core.c")
_LIB = os.path.join(_HERE, "_oracle_core.so")
_lib = None

VARIANTS = {"unweighted": 0, "weighted_normalized": 1}


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64p = ctypes.POINTER(ctypes.c_int64)
        f64p = ctypes.POINTER(ctypes.c_double)
        lib.orc_dm.argtypes = [ctypes.c_int64, i64p, f64p, ctypes.c_int64, i64p, i64p, i64p,
                               ctypes.c_int, ctypes.c_int, f64p, ctypes.POINTER(ctypes.c_int)]
        lib.orc_dm.restype = ctypes.c_int
        lib.orc_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().orc_max_threads())


def dm(tree, table, variant: str, n_threads: int = 0):
    """Condensed FP64 distance matrix; returns (dm, threads_used)."""
    lib = _load()
    parent = np.ascontiguousarray(tree.parent, dtype=np.int64)
    length = np.ascontiguousarray(tree.length, dtype=np.float64)
    indptr = np.ascontiguousarray(table.indptr, dtype=np.int64)
    tips = np.ascontiguousarray(table.tips, dtype=np.int64)
    counts = np.ascontiguousarray(table.counts, dtype=np.int64)
    n = indptr.shape[0] - 1
    out = np.zeros(max(n * (n - 1) // 2, 1), dtype=np.float64)
    used = ctypes.c_int(0)
    P = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t))  # noqa: E731
    rc = lib.orc_dm(parent.shape[0], P(parent, ctypes.c_int64), P(length, ctypes.c_double),
                    n, P(indptr, ctypes.c_int64), P(tips, ctypes.c_int64), P(counts, ctypes.c_int64),
                    VARIANTS[variant], int(n_threads), P(out, ctypes.c_double), ctypes.byref(used))
    if rc != 0:
        raise ValueError(f"oracle_core error {rc}")
    return out[: n * (n - 1) // 2], int(used.value)
