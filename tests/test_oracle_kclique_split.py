"""The k-clique oracle with cost-threshold splitting (orientation and pivoting,
Sec. 6.4.2) pinned to facts that do not come from the oracle: brute force over
k-subsets, the clique counts of complete and complete multipartite graphs, and
task-tree sizes that follow from the split rule by plain counting on graphs
whose structure fixes every candidate set."""
import itertools
import math

import numpy as np
import pytest

import oracle
from synth import graphs

ALGS = ("orient", "pivot")


def _random_graph(n, p, seed):
    rng = np.random.default_rng(seed)
    return [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]


def _brute(n, edges, k):
    if k == 1:
        return n
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


def _multipartite(t, s):
    """Complete t-partite graph with parts of s vertices (vertex v in part v % t)."""
    n = t * s
    return n, [(a, b) for a in range(n) for b in range(a + 1, n) if a % t != b % t]


@pytest.mark.parametrize("seed,n,p", [(1, 14, 0.5), (2, 18, 0.45), (3, 22, 0.35), (4, 13, 0.8), (5, 16, 0.65),
                                      (6, 22, 0.6), (7, 24, 0.55)])
def test_split_brute_force(seed, n, p):
    edges = _random_graph(n, p, seed)
    g = graphs.oriented_from_edges(n, edges, "degeneracy")
    for k in range(1, 8):
        want = _brute(n, edges, k)
        for alg in ALGS:
            for thr in (0, 1, 3, 64):
                r = oracle.kclique_split(g.row_ptr, g.col, k, range_leaf=4, threshold=thr, algorithm=alg)
                assert r.value == want, (k, alg, thr, r.value, want)


@pytest.mark.parametrize("order", ["id", "random"])
def test_split_complete_multipartite(order):
    """K_{s,...,s} with t parts has C(t, k) s^k k-cliques: many non-edges, so the
    pivoting branches over non-neighbours of every pivot."""
    for t, s in ((6, 3), (8, 2), (5, 4), (10, 1)):
        n, edges = _multipartite(t, s)
        g = graphs.oriented_from_edges(n, edges, order, seed=t * s)
        for k in range(3, min(t, 8) + 1):
            want = math.comb(t, k) * s ** k
            for alg in ALGS:
                for thr in (0, 2, 64):
                    r = oracle.kclique_split(g.row_ptr, g.col, k, threshold=thr, algorithm=alg)
                    assert r.value == want, (t, s, k, alg, thr, r.value, want)


def _orient_tree(s, l, thr):
    """Child tasks below an orientation node on a complete DAG: the child of
    the i-th candidate keeps the s-1-i candidates after it."""
    if l == 2 or s <= thr:
        return 0, 0
    tasks, splits = 0, 1
    for i in range(s):
        c = s - 1 - i
        tasks += 1
        if l - 1 >= 2 and c >= l - 1:
            t, sp = _orient_tree(c, l - 1, thr)
            tasks += t
            splits += sp
    return tasks, splits


@pytest.mark.parametrize("n", [9, 16, 24])
def test_split_complete_graph_counts_and_trees(n):
    """K_n oriented by id: C(n, k) cliques; edge (i, j) has the n-1-j later
    vertices as candidates.  Every vertex with out-neighbours forks one edge
    task per out-neighbour and resumes once.  An edge with c > t candidates
    hands its search to one child task; pivoting on a clique always picks the
    first candidate and has no non-neighbours, so that child splits into a
    chain of c - t pivot tasks."""
    edges = [(i, j) for i in range(n) for j in range(i + 1, n)]
    g = graphs.oriented_from_edges(n, edges, "id")
    for k in range(3, min(n, 9) + 1):
        kk = k - 2
        for alg in ALGS:
            for thr in (0, 3, 1000):
                base = _range_tasks(0, n, 64) + n + len(edges)
                cs = [n - 1 - j for i in range(n) for j in range(i + 1, n)]
                r = oracle.kclique_split(g.row_ptr, g.col, k, threshold=thr, algorithm=alg)
                assert r.value == math.comb(n, k)
                # an edge with more than thr candidates hands its search to one
                # child (the orientation algorithm counts k' = 2 in place)
                heavy = [c for c in cs if kk >= 2 and c >= kk and c > thr and (alg == "pivot" or kk >= 3)]
                if alg == "pivot":
                    splits = sum(c - thr for c in heavy)
                    extra = len(heavy) + splits
                else:
                    extra, splits = len(heavy), 0
                    for c in heavy:
                        t, sp = _orient_tree(c, kk, thr)
                        extra += t
                        splits += sp
                assert r.tasks == base + extra, (k, alg, thr)
                assert r.aux == splits, (k, alg, thr)
                # every task with children resumes once: ranges, vertices with
                # out-neighbours, hand-off edges and split nodes
                assert r.conts == _range_tasks(0, n, 64) + (n - 1) + len(heavy) + splits, (k, alg, thr)


def test_split_matches_plain_recursion_on_chung_lu():
    """The splitting changes the task tree, never the count: equal to the plain
    orientation recursion, which is pinned on its own by brute force."""
    g = graphs.chung_lu(1500, 18, 2.3, 1.0, 4)
    for k in (3, 4, 5, 6, 7):
        want = oracle.kclique(g.row_ptr, g.col, k).value
        for alg in ALGS:
            for thr in (0, 4, 16):
                assert oracle.kclique_split(g.row_ptr, g.col, k, threshold=thr, algorithm=alg).value == want


def test_split_no_split_tree_and_degenerate_cases():
    edges = _random_graph(30, 0.3, 7)
    g = graphs.oriented_from_edges(30, edges, "degeneracy")
    m = len(edges)
    deg = np.diff(g.row_ptr)
    rt = _range_tasks(0, 30, 8)
    for alg in ALGS:
        assert oracle.kclique_split(g.row_ptr, g.col, 1, range_leaf=8, algorithm=alg).value == 30
        r2 = oracle.kclique_split(g.row_ptr, g.col, 2, range_leaf=8, algorithm=alg)
        assert r2.value == m and r2.tasks == rt + 30
        r = oracle.kclique_split(g.row_ptr, g.col, 3, range_leaf=8, threshold=1000, algorithm=alg)
        assert r.tasks == rt + 30 + m and r.aux == 0
        assert r.conts == rt + int((deg > 0).sum())
        for k in (4, 5):
            # no split under a threshold above every out-degree: ranges,
            # vertices and one task per edge, nothing more
            r = oracle.kclique_split(g.row_ptr, g.col, k, range_leaf=8, threshold=1000, algorithm=alg)
            assert r.tasks == rt + 30 + m and r.aux == 0
            assert r.conts == rt + int((deg > 0).sum())
            # threshold 2: the same tree plus heavy edges' hand-offs and split
            # nodes, one resumption each
            r = oracle.kclique_split(g.row_ptr, g.col, k, range_leaf=8, threshold=2, algorithm=alg)
            extra = r.tasks - (rt + 30 + m)
            hand = r.conts - (rt + int((deg > 0).sum())) - r.aux
            assert 0 <= hand <= extra and (extra == 0) == (hand == 0), (k, alg, extra, hand, r.aux)
        e0 = graphs.oriented_from_edges(12, [], "id")
        assert oracle.kclique_split(e0.row_ptr, e0.col, 4, algorithm=alg).value == 0
        z = graphs.oriented_from_edges(0, [], "id")
        assert oracle.kclique_split(z.row_ptr, z.col, 3, algorithm=alg).value == 0
        with pytest.raises(ValueError):
            oracle.kclique_split(g.row_ptr, g.col, 0, algorithm=alg)
        with pytest.raises(ValueError):
            oracle.kclique_split(g.row_ptr, g.col, 4, threshold=-1, algorithm=alg)


def test_split_root_sample_sums_to_full_count():
    """The vertex-sample form (cliques whose lowest vertex is offset mod
    stride) partitions the count."""
    g = graphs.chung_lu(1500, 18, 2.3, 1.0, 4)
    for alg in ALGS:
        for k in (4, 6):
            full = oracle.kclique_split(g.row_ptr, g.col, k, threshold=8, algorithm=alg).value
            parts = [oracle.kclique_split_roots(g.row_ptr, g.col, k, 7, o, threshold=8, algorithm=alg).value
                     for o in range(7)]
            assert sum(parts) == full and all(p_ >= 0 for p_ in parts)
    with pytest.raises(ValueError):
        oracle.kclique_split_roots(g.row_ptr, g.col, 4, 3, 3)
