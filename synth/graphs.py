"""Chung-Lu power-law graphs and their degeneracy orientation (seeded).

The paper measures k-clique counting on SNAP graphs (Sec. 6.4.2); those files
are not available here, so seeded Chung-Lu graphs with the stated vertex
count, mean degree and degree exponent stand in for them.  The orientation
used is the degeneracy (smallest-last) order, ties broken by smallest vertex
id; vertices are relabelled by their position so that every out-list holds
larger ids only, and out-lists are sorted.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    lib.syn_chung_lu.argtypes = [i64, dbl, dbl, dbl, u64, vp, ctypes.POINTER(dbl)]
    lib.syn_chung_lu.restype = i64
    lib.syn_sym_csr.argtypes = [i64, vp, i64, vp, vp]
    lib.syn_sym_csr.restype = None
    lib.syn_degeneracy_order.argtypes = [i64, vp, vp, vp]
    lib.syn_degeneracy_order.restype = i64
    lib.syn_orient.argtypes = [i64, vp, vp, vp, vp, vp]
    lib.syn_orient.restype = i64
    lib.syn_draw.argtypes = [u64, u64]
    lib.syn_draw.restype = u64
    lib.syn_induced.argtypes = [i64, vp, vp, i64, u64, vp, vp, vp, vp, i64]
    lib.syn_induced.restype = i64
    _lib = lib
    return lib


def draw(seed: int, e: int) -> int:
    """Draw e of the splitmix64 stream `seed`."""
    return int(_load().syn_draw(seed & (2**64 - 1), e))


@dataclass
class OrientedGraph:
    """Acyclic orientation of an undirected simple graph as CSR out-lists."""
    n: int
    row_ptr: np.ndarray          # int64 [n+1]
    col: np.ndarray              # int32 [m]
    m_undirected: int
    max_degree: int
    degeneracy: int
    max_outdeg: int
    info: dict = field(default_factory=dict)

    @property
    def row_ptr32(self) -> np.ndarray:
        assert self.row_ptr[-1] < 2**31
        return self.row_ptr.astype(np.int32)

    def checksum(self) -> str:
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(self.row_ptr, dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.col, dtype=np.int32).tobytes())
        return h.hexdigest()[:16]


def sym_csr_from_edges(n: int, edges) -> tuple[np.ndarray, np.ndarray, int]:
    """Symmetric sorted CSR of an undirected edge list; drops loops and duplicates."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if e.size:
        e = e[e[:, 0] != e[:, 1]]
        lo = np.minimum(e[:, 0], e[:, 1]).astype(np.uint64)
        hi = np.maximum(e[:, 0], e[:, 1]).astype(np.uint64)
        keys = np.unique((lo << np.uint64(32)) | hi)
    else:
        keys = np.zeros(0, dtype=np.uint64)
    keys = np.ascontiguousarray(keys)
    rp = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(max(2 * keys.size, 1), dtype=np.int32)
    _load().syn_sym_csr(n, keys.ctypes.data, keys.size, rp.ctypes.data, col.ctypes.data)
    return rp, col[: 2 * keys.size], int(keys.size)


def orient(n: int, rp: np.ndarray, col: np.ndarray, pos: np.ndarray) -> tuple[np.ndarray, np.ndarray, int]:
    """Orient by a total order: relabel v -> pos[v], keep u->w iff pos[u] < pos[w]."""
    pos = np.ascontiguousarray(pos, dtype=np.int64)
    assert pos.shape == (n,) and (n == 0 or np.array_equal(np.sort(pos), np.arange(n)))
    m = col.size // 2
    orp = np.zeros(n + 1, dtype=np.int64)
    ocol = np.zeros(max(m, 1), dtype=np.int32)
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    maxd = _load().syn_orient(n, rp.ctypes.data, col.ctypes.data, pos.ctypes.data,
                              orp.ctypes.data, ocol.ctypes.data)
    return orp, ocol[:m], int(maxd)


def degeneracy_order(n: int, rp: np.ndarray, col: np.ndarray) -> tuple[np.ndarray, int]:
    pos = np.zeros(max(n, 1), dtype=np.int64)
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    d = _load().syn_degeneracy_order(n, rp.ctypes.data, col.ctypes.data, pos.ctypes.data)
    return pos[:n], int(d)


def oriented_from_edges(n: int, edges, order: str = "degeneracy", seed: int = 0) -> OrientedGraph:
    """Orient an explicit undirected edge list ('degeneracy', 'id' or 'random' order)."""
    rp, col, m = sym_csr_from_edges(n, edges)
    degen = -1
    if order == "degeneracy":
        pos, degen = degeneracy_order(n, rp, col)
    elif order == "id":
        pos = np.arange(n, dtype=np.int64)
    elif order == "random":
        pos = np.random.default_rng(seed).permutation(n).astype(np.int64)
    else:
        raise ValueError(order)
    orp, ocol, maxd = orient(n, rp, col, pos)
    maxdeg = int(np.max(np.diff(rp))) if n else 0
    return OrientedGraph(n, orp, ocol, m, maxdeg, degen, maxd)


def chung_lu(n: int, mean_degree: float, gamma: float, cap_frac: float, seed: int) -> OrientedGraph:
    """Seeded Chung-Lu graph, degeneracy-oriented, as sorted int CSR out-lists."""
    lib = _load()
    m_draw = int(round(n * mean_degree / 2.0))
    keys = np.zeros(max(m_draw, 1), dtype=np.uint64)
    scale = ctypes.c_double(0.0)
    m = lib.syn_chung_lu(n, float(mean_degree), float(gamma), float(cap_frac), seed & (2**64 - 1),
                         keys.ctypes.data, ctypes.byref(scale))
    if m < 0:
        raise ValueError("chung_lu: invalid parameters")
    keys = np.ascontiguousarray(keys[:m])
    rp = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(max(2 * m, 1), dtype=np.int32)
    lib.syn_sym_csr(n, keys.ctypes.data, m, rp.ctypes.data, col.ctypes.data)
    col = col[: 2 * m]
    pos, degen = degeneracy_order(n, rp, col)
    orp, ocol, maxd = orient(n, rp, col, pos)
    maxdeg = int(np.max(np.diff(rp)))
    info = {"n": n, "mean_degree_target": mean_degree, "gamma": gamma, "cap_frac": cap_frac,
            "seed": seed, "scale_c": scale.value, "m_drawn": m_draw,
            "mean_degree_realised": 2.0 * m / n}
    return OrientedGraph(n, orp, ocol, int(m), maxdeg, degen, maxd, info)


class _InducedWork:
    """Per-thread work buffers for induced(): a vertex bitmap and an id map."""

    def __init__(self, g: OrientedGraph):
        self.mark = np.zeros(g.n // 64 + 1, dtype=np.uint64)
        self.map = np.zeros(max(g.n, 1), dtype=np.int32)
        self.col = np.zeros(max(int(g.row_ptr[-1]), 1), dtype=np.int32)


def induced(g: OrientedGraph, s: int, seed: int, work: "_InducedWork | None" = None) -> OrientedGraph:
    """Subgraph induced by s vertices of g drawn uniformly without replacement
    (seeded), renumbered in increasing order: the orientation of g restricted
    to them, still acyclic with sorted out-lists."""
    lib = _load()
    s = int(min(max(s, 0), g.n))
    w = work if work is not None else _InducedWork(g)
    rp = np.zeros(s + 1, dtype=np.int64)
    m = lib.syn_induced(g.n, g.row_ptr.ctypes.data, g.col.ctypes.data, s, seed & (2**64 - 1),
                        w.mark.ctypes.data, w.map.ctypes.data, rp.ctypes.data, w.col.ctypes.data,
                        w.col.size)
    if m < 0:
        raise RuntimeError("induced: edge buffer too small")
    col = w.col[:m].copy()
    maxd = int(np.max(np.diff(rp))) if s > 0 else 0
    return OrientedGraph(s, rp, col, int(m), -1, -1, maxd, {"parent_n": g.n, "seed": seed})


def induced_many(g: OrientedGraph, specs, threads: int = 8) -> list:
    """induced() for each (s, seed) in specs on a pool of threads."""
    import concurrent.futures as cf
    import threading
    local = threading.local()

    def one(spec):
        if not hasattr(local, "w"):
            local.w = _InducedWork(g)
        return induced(g, spec[0], spec[1], local.w)

    with cf.ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        return list(ex.map(one, specs))
