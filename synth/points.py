"""Seeded point sets for the fast multipole workloads (input generation only)."""
from __future__ import annotations

import numpy as np

from . import graphs


def plummer(n: int, seed: int):
    """Plummer-sphere points (scale 1, radius <= 100) and charges in (-1, 1):
    float64 arrays x, y, z, q of length n."""
    import ctypes
    lib = graphs._load()
    if not hasattr(lib, "_plummer_bound"):
        lib.syn_plummer.argtypes = [ctypes.c_int64, ctypes.c_uint64] + [ctypes.c_void_p] * 4
        lib.syn_plummer.restype = None
        lib._plummer_bound = True
    out = [np.zeros(n, dtype=np.float64) for _ in range(4)]
    lib.syn_plummer(n, seed & (2**64 - 1), *[a.ctypes.data for a in out])
    return tuple(out)


def uniform_cube(n: int, seed: int, half: float = 1.0):
    """Points uniform in [-half, half)^3 with charges uniform in [-1, 1)."""
    rng = np.random.default_rng(seed)
    x, y, z = (rng.uniform(-half, half, n) for _ in range(3))
    q = rng.uniform(-1.0, 1.0, n)
    return x, y, z, q
