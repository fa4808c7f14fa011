"""Sequential CPU oracle for the GTaP workloads (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP runtime and
its Python binding) never imports it, and the two share no code: the oracle is
plain C compiled with gcc (``oracle/oracle.c``) plus pure numpy here.

Functions return the workload result together with the fork-join execution
counts (task calls and resumptions after a join, GTaP Sec. 5.1.2), which do not
depend on the schedule and are therefore exact targets for the GPU runtime.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


class _Counts(ctypes.Structure):
    _fields_ = [("tasks", ctypes.c_int64), ("conts", ctypes.c_int64),
                ("leaves", ctypes.c_int64), ("aux", ctypes.c_int64)]


@dataclass
class OracleResult:
    value: int
    tasks: int
    conts: int
    leaves: int
    aux: int = 0

    @property
    def executions(self) -> int:
        return self.tasks + self.conts


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # noqa: WPS433 - build on first use (CPU only)
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    lib.orc_fib.argtypes = [ctypes.c_int, P(_Counts)]
    lib.orc_fib.restype = ctypes.c_int64
    lib.orc_nqueens.argtypes = [ctypes.c_int, P(_Counts)]
    lib.orc_nqueens.restype = ctypes.c_int64
    lib.orc_uts.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, P(_Counts)]
    lib.orc_uts.restype = ctypes.c_int64
    lib.orc_uts_mix64.argtypes = [ctypes.c_uint64]
    lib.orc_uts_mix64.restype = ctypes.c_uint64
    lib.orc_uts_num_children.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64, ctypes.c_int]
    lib.orc_uts_num_children.restype = ctypes.c_int
    lib.orc_kclique.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, P(_Counts)]
    lib.orc_kclique.restype = ctypes.c_int64
    _lib = lib
    return lib


def _res(v, c: _Counts) -> OracleResult:
    return OracleResult(int(v), int(c.tasks), int(c.conts), int(c.leaves), int(c.aux))


def fib(n: int) -> OracleResult:
    """fib(n) with one task per call (Sec. 6.3, Fibonacci without cutoff)."""
    c = _Counts()
    return _res(_load().orc_fib(int(n), ctypes.byref(c)), c)


def nqueens(n: int) -> OracleResult:
    """Number of n-queens solutions by bitmask backtracking (Sec. 6.3)."""
    c = _Counts()
    return _res(_load().orc_nqueens(int(n), ctypes.byref(c)), c)


def uts_threshold(m: float) -> int:
    """Integer continue-threshold floor(2^64 * m/(m+1)) for a geometric law of mean m.

    Computed in exact rational arithmetic so every caller gets the same integer.
    """
    from fractions import Fraction
    f = Fraction(m).limit_denominator(1 << 20)
    return int((Fraction(1 << 64) * f) // (f + 1))


def uts(seed: int, thr: int, max_depth: int) -> OracleResult:
    """Node count of the unbalanced tree rooted at mix64(seed); ``aux`` = max depth."""
    c = _Counts()
    return _res(_load().orc_uts(int(seed) & (2**64 - 1), int(thr), int(max_depth), ctypes.byref(c)), c)


def uts_mix64(z: int) -> int:
    return int(_load().orc_uts_mix64(int(z) & (2**64 - 1)))


def uts_num_children(node_id: int, depth: int, thr: int, max_depth: int) -> int:
    return int(_load().orc_uts_num_children(int(node_id), int(depth), int(thr), int(max_depth)))


def kclique(row_ptr, col, k: int, range_leaf: int = 64) -> OracleResult:
    """Number of k-cliques of an oriented graph given as CSR out-lists (Sec. 6.4.2).

    ``row_ptr`` has n+1 entries, ``col`` the concatenated sorted out-lists.
    The task counts follow the vertex-range / vertex / candidate task tree
    documented in ``oracle.c``.
    """
    rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int64))
    cl = np.ascontiguousarray(np.asarray(col, dtype=np.int32))
    n = rp.shape[0] - 1
    maxdeg = int(np.max(np.diff(rp))) if n > 0 else 0
    scratch = np.zeros(max(k - 2, 1) * max(maxdeg, 1), dtype=np.int32)
    c = _Counts()
    v = _load().orc_kclique(rp.ctypes.data, cl.ctypes.data if cl.size else None, n, int(k),
                            int(range_leaf), scratch.ctypes.data, maxdeg, ctypes.byref(c))
    if v < 0:
        raise ValueError("oracle kclique: invalid arguments")
    return _res(v, c)
