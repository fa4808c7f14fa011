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
    lib.orc_cilksort.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                 ctypes.c_int64, P(_Counts)]
    lib.orc_cilksort.restype = ctypes.c_int64
    lib.orc_kclique_split.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                      ctypes.c_int64, ctypes.c_int, ctypes.c_int, P(_Counts)]
    lib.orc_kclique_split.restype = ctypes.c_int64
    lib.orc_kclique_split_roots.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                            ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                            P(_Counts)]
    lib.orc_kclique_split_roots.restype = ctypes.c_int64
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


# ---- FMM (GTaP Sec. 6.4.1) -------------------------------------------------
class _FmmStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("n_cells", "n_leaves", "max_level", "m2l_pairs", "p2p_pairs")] + \
               [("m2l_hash", ctypes.c_uint64), ("p2p_hash", ctypes.c_uint64),
                ("p2p_interactions", ctypes.c_int64), ("coincident", ctypes.c_int64)]


CELL_DTYPE = np.dtype([("level", np.int32), ("ax", np.int32), ("ay", np.int32), ("az", np.int32),
                       ("begin", np.int32), ("end", np.int32), ("child0", np.int32), ("nchild", np.int32),
                       ("parent", np.int32)])


@dataclass
class FmmResult:
    phi: np.ndarray
    stats: dict
    m2l: np.ndarray = None   # (pairs, 2) int32: (target cell, source cell)
    p2p: np.ndarray = None


def _fmm_lib():
    lib = _load()
    if not getattr(lib, "_fmm_bound", False):
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        lib.orc_fmm_tree.argtypes = [i64, vp, vp, vp, ctypes.c_int, vp, vp, i64, vp]
        lib.orc_fmm_tree.restype = i64
        lib.orc_fmm.argtypes = [i64, vp, vp, vp, vp, ctypes.c_int, i64, i64, ctypes.c_int, vp, i64, vp,
                                ctypes.POINTER(_FmmStats), vp, vp, i64]
        lib.orc_fmm.restype = ctypes.c_int
        lib.orc_direct.argtypes = [i64, vp, vp, vp, vp, vp, i64, vp]
        lib.orc_direct.restype = None
        lib._fmm_bound = True
    return lib


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def fmm_tree(x, y, z, leaf_max: int = 64):
    """Octree of the FMM reading in ``fmm.c``: (perm, cells, sorted keys)."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    n = x.size
    perm = np.zeros(max(n, 1), dtype=np.int32)
    keys = np.zeros(max(n, 1), dtype=np.uint64)
    cap = 2 * max(n, 1) + 64
    cells = np.zeros(cap, dtype=CELL_DTYPE)
    nc = _fmm_lib().orc_fmm_tree(n, x.ctypes.data, y.ctypes.data, z.ctypes.data, int(leaf_max),
                                 perm.ctypes.data, cells.ctypes.data, cap, keys.ctypes.data)
    if nc < 0:
        raise ValueError("oracle fmm_tree: point outside the root cube" if nc == -1 else "too many cells")
    return perm[:n], cells[:nc].copy(), keys[:n]


def fmm(x, y, z, q, p: int = 6, theta=(1, 2), leaf_max: int = 64, targets=None,
        lists: bool = False) -> FmmResult:
    """Potentials of the FMM pipeline (all points, or the listed targets) with
    pair counts and order-independent pair hashes."""
    x, y, z, q = _f64(x), _f64(y), _f64(z), _f64(q)
    n = x.size
    st = _FmmStats()
    if targets is None:
        tg, nt, phi = None, 0, np.zeros(max(n, 1))
    else:
        tg = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
        nt = tg.size
        phi = np.zeros(max(nt, 1))
    cap = 0
    m2l = p2p = None
    lib = _fmm_lib()
    if lists:
        # a first pass learns the list sizes
        rc = lib.orc_fmm(n, x.ctypes.data, y.ctypes.data, z.ctypes.data, q.ctypes.data, int(p), int(theta[0]),
                         int(theta[1]), int(leaf_max), np.zeros(1, np.int64).ctypes.data, 0,
                         np.zeros(1).ctypes.data, ctypes.byref(st), None, None, 0)
        if rc != 0:
            raise ValueError(f"oracle fmm: error {rc}")
        cap = max(st.m2l_pairs, st.p2p_pairs, 1)
        m2l = np.zeros((cap, 2), dtype=np.int32)
        p2p = np.zeros((cap, 2), dtype=np.int32)
    rc = lib.orc_fmm(n, x.ctypes.data, y.ctypes.data, z.ctypes.data, q.ctypes.data, int(p), int(theta[0]),
                     int(theta[1]), int(leaf_max), tg.ctypes.data if tg is not None else None, nt,
                     phi.ctypes.data, ctypes.byref(st), m2l.ctypes.data if lists else None,
                     p2p.ctypes.data if lists else None, cap)
    if rc != 0:
        raise ValueError(f"oracle fmm: error {rc}")
    stats = {f: getattr(st, f) for f, _ in _FmmStats._fields_}
    out = FmmResult(phi[: (n if targets is None else nt)], stats)
    if lists:
        out.m2l = m2l[: st.m2l_pairs]
        out.p2p = p2p[: st.p2p_pairs]
    return out


def direct(x, y, z, q, targets) -> np.ndarray:
    """Direct summation sum_{j != i} q_j / |x_i - x_j| at the listed targets."""
    x, y, z, q = _f64(x), _f64(y), _f64(z), _f64(q)
    tg = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
    phi = np.zeros(max(tg.size, 1))
    _fmm_lib().orc_direct(x.size, x.ctypes.data, y.ctypes.data, z.ctypes.data, q.ctypes.data, tg.ctypes.data,
                          tg.size, phi.ctypes.data)
    return phi[: tg.size]


KCLIQUE_ALGORITHMS = {"orient": 0, "pivot": 1}


def kclique_split(row_ptr, col, k: int, range_leaf: int = 64, threshold: int = 32,
                  algorithm: str = "orient") -> OracleResult:
    """k-clique count with cost-threshold task splitting (Sec. 6.4.2), by the
    orientation or the pivoting algorithm.  The task tree -- vertex ranges,
    vertices, edges, and the child tasks of every node whose candidate set is
    larger than ``threshold`` -- is written out in ``oracle/kclique_split.c``;
    counts.aux is the number of nodes that split."""
    rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int64))
    cl = np.ascontiguousarray(np.asarray(col, dtype=np.int32))
    n = rp.shape[0] - 1
    c = _Counts()
    v = _load().orc_kclique_split(rp.ctypes.data, cl.ctypes.data if cl.size else None, n, int(k),
                                  int(range_leaf), int(threshold), KCLIQUE_ALGORITHMS[algorithm], ctypes.byref(c))
    if v < 0:
        raise ValueError("oracle kclique_split: invalid arguments" if v == -1 else "oracle kclique_split: no memory")
    return _res(v, c)


def kclique_split_roots(row_ptr, col, k: int, stride: int, offset: int = 0, threshold: int = 32,
                        algorithm: str = "orient") -> OracleResult:
    """kclique_split restricted to the cliques whose lowest vertex is
    offset mod stride: a sample of the vertex tasks, for timing."""
    rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int64))
    cl = np.ascontiguousarray(np.asarray(col, dtype=np.int32))
    n = rp.shape[0] - 1
    c = _Counts()
    v = _load().orc_kclique_split_roots(rp.ctypes.data, cl.ctypes.data if cl.size else None, n, int(k),
                                        int(stride), int(offset), int(threshold), KCLIQUE_ALGORITHMS[algorithm],
                                        ctypes.byref(c))
    if v < 0:
        raise ValueError("oracle kclique_split_roots: invalid arguments" if v == -1 else "no memory")
    return _res(v, c)


def cilksort(keys, sort_cutoff: int = 64, merge_cutoff: int = 256):
    """Cilksort (GTaP Sec. 6.3) of uint32 keys: returns (sorted copy, counts).
    counts.aux is the number of merge tasks, counts.leaves the serial sorts and
    serial merges.  The recursion is written out in oracle/cilksort.c."""
    x = np.array(keys, dtype=np.uint32, copy=True)
    t = np.empty_like(x)
    c = _Counts()
    v = _load().orc_cilksort(x.ctypes.data, t.ctypes.data, int(x.size), int(sort_cutoff), int(merge_cutoff),
                             ctypes.byref(c))
    return x, _res(v, c)
