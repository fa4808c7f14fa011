"""Seeded request traces for the batching and serving measurements.

A trace mixes k-clique counting jobs on induced subgraphs of a larger graph
with unbalanced tree search jobs, so that job sizes span many orders of
magnitude.  Arrivals are Poisson.  Only job parameters and arrival times are
drawn here; nothing of the fork-join method is computed.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class JobSpec:
    kind: str          # "kclique" or "uts"
    k: int = 0         # k-clique: clique size
    s: int = 0         # k-clique: vertices in the induced subgraph
    sub_seed: int = 0  # k-clique: seed of the vertex subset
    m: float = 0.0     # UTS: mean branching factor
    depth: int = 0     # UTS: depth limit
    seed: int = 0      # UTS: root seed


def serving_mix(n_jobs: int, seed: int, p_kclique: float = 0.6, k_range=(4, 8),
                s_range=(1000, 200000), m_range=(2.0, 4.0), depth_range=(8, 14)) -> list:
    """n_jobs job specs: with probability p_kclique a k-clique job (k uniform
    in k_range, subgraph size log-uniform in s_range), else a UTS job (m
    uniform in m_range, depth uniform in depth_range, its own root seed)."""
    rng = np.random.default_rng(seed)
    is_kc = rng.random(n_jobs) < p_kclique
    ks = rng.integers(k_range[0], k_range[1] + 1, n_jobs)
    ss = np.rint(np.exp(rng.uniform(np.log(s_range[0]), np.log(s_range[1]), n_jobs))).astype(np.int64)
    subs = rng.integers(1, 2**63 - 1, n_jobs, dtype=np.int64)
    ms = rng.uniform(m_range[0], m_range[1], n_jobs)
    ds = rng.integers(depth_range[0], depth_range[1] + 1, n_jobs)
    seeds = rng.integers(1, 2**63 - 1, n_jobs, dtype=np.int64)
    out = []
    for i in range(n_jobs):
        if is_kc[i]:
            out.append(JobSpec("kclique", k=int(ks[i]), s=int(ss[i]), sub_seed=int(subs[i])))
        else:
            out.append(JobSpec("uts", m=float(ms[i]), depth=int(ds[i]), seed=int(seeds[i])))
    return out


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (seconds from the start) of a Poisson process of the given rate."""
    if n == 0:
        return np.zeros(0)
    gaps = np.random.default_rng(seed).exponential(1.0 / rate, n)
    gaps[0] = 0.0
    return np.cumsum(gaps)
