"""The CPU oracle pinned to facts that do not come from the oracle itself.

Each check is chosen so that a plausible slip in the oracle (a dropped term,
an off-by-one in a recursion, a transposed shift, a wrong threshold) fails it:
closed forms, published constants and sequences, brute force over tiny
inputs, invariants under re-orientation, and distributional checks.
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
from synth import graphs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_pairs(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                a, b = line.split()
                out.append((a, b))
    return out


# ---- Fibonacci (Sec. 6.3): closed form and the call-tree counts ------------
def _fib_closed(n):
    """F(n) by fast doubling (independent of the oracle's naive recursion)."""
    def fd(k):
        if k == 0:
            return (0, 1)
        a, b = fd(k // 2)
        c = a * (2 * b - a)
        d = a * a + b * b
        return (d, c + d) if k % 2 else (c, d)
    return fd(n)[0]


@pytest.mark.parametrize("n", [0, 1, 2, 3, 10, 20, 25])
def test_fib_closed_form_and_tree(n):
    r = oracle.fib(n)
    assert r.value == _fib_closed(n)
    # One task per call: T(n) = 1 + T(n-1) + T(n-2), T(0) = T(1) = 1, whose
    # solution is 2F(n+1) - 1; every internal call joins once: F(n+1) - 1.
    assert r.tasks == 2 * _fib_closed(n + 1) - 1
    assert r.conts == _fib_closed(n + 1) - 1
    assert r.leaves == r.tasks - r.conts


def test_fib32_headline():
    r = oracle.fib(32)
    assert r.value == 2178309
    assert r.tasks == 7049155 and r.conts == 3524577
    assert r.executions == 10573732


# ---- N-Queens (Sec. 6.3) --------------------------------------------------
def test_nqueens_matches_published_counts():
    for n, want in _read_pairs("nqueens_counts.txt"):
        n, want = int(n), int(want)
        if n > 13:
            continue
        assert oracle.nqueens(n).value == want, n


def _nq_prefixes(n):
    """All conflict-free placements of queens on the first r rows, by brute force."""
    def ok(p):
        return all(abs(p[i] - p[j]) != j - i and p[i] != p[j]
                   for i in range(len(p)) for j in range(i + 1, len(p)))
    layers = [[()]]
    for r in range(n):
        layers.append([p + (c,) for p in layers[-1] for c in range(n) if ok(p + (c,))])
    return layers


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
def test_nqueens_tree_by_brute_force(n):
    layers = _nq_prefixes(n)
    tasks = sum(len(L) for L in layers)
    # a node forks iff it is not a full board and has at least one extension
    conts = sum(1 for r in range(n) for p in layers[r]
                if any(q[:r] == p for q in layers[r + 1]))
    r = oracle.nqueens(n)
    assert r.value == len(layers[n])
    assert r.tasks == tasks
    assert r.conts == conts


def test_nqueens_permutation_brute_force():
    for n in range(1, 9):
        cnt = sum(1 for p in itertools.permutations(range(n))
                  if len({p[i] + i for i in range(n)}) == n and len({p[i] - i for i in range(n)}) == n)
        assert oracle.nqueens(n).value == cnt


# ---- UTS: hash, geometric law, size ---------------------------------------
def test_splitmix64_published_outputs():
    gamma = 0x9E3779B97F4A7C15
    for idx, hexval in _read_pairs("splitmix64_state0.txt"):
        i = int(idx)
        assert oracle.uts_mix64((i * gamma) % 2**64) == int(hexval, 16)


def test_uts_threshold_values():
    assert oracle.uts_threshold(4) == 0xCCCCCCCCCCCCCCCC
    assert oracle.uts_threshold(1) == 1 << 63
    # mean 3: floor(2^64 * 3/4)
    assert oracle.uts_threshold(3) == (3 << 62)


def test_uts_child_count_is_geometric():
    thr = oracle.uts_threshold(4)       # continue probability 4/5
    p = thr / 2.0**64
    counts = np.array([oracle.uts_num_children(oracle.uts_mix64(s), 0, thr, 5) for s in range(20000)])
    assert abs(counts.mean() - 4.0) < 4 * math.sqrt(20.0 / counts.size)   # var = p/(1-p)^2 = 20
    # chi-square against P(c = j) = (1-p) p^j, bins 0..14 and a tail bin
    obs = np.bincount(np.minimum(counts, 15), minlength=16).astype(float)
    exp = np.array([(1 - p) * p**j for j in range(15)] + [p**15]) * counts.size
    chi2 = float(((obs - exp) ** 2 / exp).sum())
    assert chi2 < 40.0          # 15 d.o.f.: P(chi2 > 40) ~ 5e-4
    # the depth limit cuts every child
    assert all(oracle.uts_num_children(oracle.uts_mix64(s), 5, thr, 5) == 0 for s in range(50))


def test_uts_mean_size_matches_galton_watson():
    thr = oracle.uts_threshold(4)
    sizes = np.array([oracle.uts(s, thr, 3).value for s in range(1, 6001)], dtype=float)
    want = sum(4**d for d in range(4))                 # E|tree| = sum_d m^d = 85
    se = sizes.std() / math.sqrt(sizes.size)
    assert abs(sizes.mean() - want) < 4.5 * se


def test_uts_structure():
    thr = oracle.uts_threshold(4)
    for s in range(1, 30):
        r = oracle.uts(s, thr, 0)
        assert r.value == 1 and r.tasks == 1 and r.conts == 0
        r1 = oracle.uts(s, thr, 1)
        assert r1.value == 1 + oracle.uts_num_children(oracle.uts_mix64(s), 0, thr, 1)
        r3 = oracle.uts(s, thr, 3)
        assert r3.value == r3.tasks and r3.leaves + r3.conts == r3.tasks and r3.aux <= 3


def test_uts_definition_transcription():
    """Sizes quoted in the build plan for seed 1, mean 4 (they pin the reading of
    the definition, not independent truth)."""
    thr = oracle.uts_threshold(4)
    assert [oracle.uts(1, thr, d).value for d in (1, 2, 4, 6)] == [7, 32, 433, 6359]


# ---- k-clique (Sec. 6.4.2) ------------------------------------------------
def _random_graph(n, p, seed):
    rng = np.random.default_rng(seed)
    return [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]


def _brute_cliques(n, edges, k):
    adj = np.zeros((n, n), dtype=bool)
    for a, b in edges:
        adj[a, b] = adj[b, a] = True
    return sum(1 for S in itertools.combinations(range(n), k)
               if all(adj[a, b] for a, b in itertools.combinations(S, 2)))


def _range_tasks(lo, hi, leaf):
    if hi - lo <= leaf:
        return 1
    mid = lo + (hi - lo) // 2
    return 1 + _range_tasks(lo, mid, leaf) + _range_tasks(mid, hi, leaf)


@pytest.mark.parametrize("seed,n,p", [(1, 14, 0.5), (2, 18, 0.4), (3, 22, 0.3), (4, 12, 0.8)])
def test_kclique_brute_force(seed, n, p):
    edges = _random_graph(n, p, seed)
    g = graphs.oriented_from_edges(n, edges, "degeneracy")
    for k in range(1, 7):
        want = _brute_cliques(n, edges, k) if k >= 2 else n
        r = oracle.kclique(g.row_ptr, g.col, k, range_leaf=4)
        assert r.value == want, (k, r.value, want)
        if k >= 3:
            # one candidate task per j-clique grown from an edge, j = 2..k-1
            cand = sum(_brute_cliques(n, edges, j) for j in range(2, k))
            assert r.tasks == _range_tasks(0, n, 4) + n + cand


def test_kclique_complete_graph():
    for n in (5, 9, 13):
        edges = [(i, j) for i in range(n) for j in range(i + 1, n)]
        g = graphs.oriented_from_edges(n, edges, "id")
        for k in range(1, n + 1):
            assert oracle.kclique(g.row_ptr, g.col, k).value == math.comb(n, k)


def test_kclique_triangles_trace():
    edges = _random_graph(40, 0.25, 9)
    A = np.zeros((40, 40), dtype=np.int64)
    for a, b in edges:
        A[a, b] = A[b, a] = 1
    g = graphs.oriented_from_edges(40, edges, "random", seed=3)
    assert oracle.kclique(g.row_ptr, g.col, 3).value == int(np.trace(A @ A @ A)) // 6


def test_kclique_orientation_invariance():
    g0 = graphs.chung_lu(400, 14, 2.5, 1.0, 11)
    # rebuild the undirected edge list from the oriented graph
    src = np.repeat(np.arange(g0.n), np.diff(g0.row_ptr))
    edges = np.stack([src, g0.col], axis=1)
    for k in (3, 4, 5):
        counts = {oracle.kclique(g0.row_ptr, g0.col, k).value}
        for order, seed in (("id", 0), ("random", 1), ("random", 2)):
            g = graphs.oriented_from_edges(g0.n, edges, order, seed=seed)
            counts.add(oracle.kclique(g.row_ptr, g.col, k).value)
        assert len(counts) == 1, (k, counts)


def test_kclique_degenerate_cases():
    g = graphs.oriented_from_edges(10, [], "id")
    assert oracle.kclique(g.row_ptr, g.col, 1).value == 10
    assert oracle.kclique(g.row_ptr, g.col, 2).value == 0
    assert oracle.kclique(g.row_ptr, g.col, 4).value == 0
    g1 = graphs.oriented_from_edges(0, [], "id")
    assert oracle.kclique(g1.row_ptr, g1.col, 3).value == 0
    edges = [(0, 1), (1, 2), (2, 0), (2, 3)]
    g2 = graphs.oriented_from_edges(4, edges, "degeneracy")
    assert oracle.kclique(g2.row_ptr, g2.col, 2).value == 4
    assert oracle.kclique(g2.row_ptr, g2.col, 3).value == 1
    assert oracle.kclique(g2.row_ptr, g2.col, 4).value == 0
