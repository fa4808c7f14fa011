"""Seeded synthetic inputs: shape checks of the generated graphs."""
import pytest
import numpy as np

from synth import graphs


def _check_oriented(g):
    rp, col = g.row_ptr, g.col
    assert rp[0] == 0 and rp[-1] == col.size and np.all(np.diff(rp) >= 0)
    src = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all(col > src)                     # acyclic: every arc goes up
    for v in range(g.n):                         # sorted, no duplicates
        L = col[rp[v]:rp[v + 1]]
        assert np.all(np.diff(L) > 0)


def test_chung_lu_small_config_shape():
    g = graphs.chung_lu(2000, 16, 2.5, 1.0, 1)
    _check_oriented(g)
    assert g.m_undirected == g.col.size
    assert abs(g.info["mean_degree_realised"] - 16) / 16 < 0.05
    assert g.max_outdeg <= g.degeneracy
    # the same seed gives the same graph, another seed another one
    assert graphs.chung_lu(2000, 16, 2.5, 1.0, 1).checksum() == g.checksum()
    assert graphs.chung_lu(2000, 16, 2.5, 1.0, 2).checksum() != g.checksum()


def test_chung_lu_power_law_tail():
    g = graphs.chung_lu(20000, 16, 2.5, 1.0, 5)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    deg = np.bincount(np.concatenate([src, g.col]), minlength=g.n)
    # complementary CDF slope between degree 20 and 100 is about -(gamma-1)
    ks = np.array([20, 30, 45, 70, 100])
    ccdf = np.array([(deg >= k).mean() for k in ks])
    slope = np.polyfit(np.log(ks), np.log(ccdf), 1)[0]
    assert -2.2 < slope < -0.9


def test_orientation_by_order():
    edges = [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4)]
    g = graphs.oriented_from_edges(5, edges, "degeneracy")
    _check_oriented(g)
    assert g.col.size == 5 and g.degeneracy == 2


def _floyd_subset(n, s, seed):
    """Floyd's sampling without replacement, from the same draw stream."""
    chosen = set()
    e = 0
    for j in range(n - s, n):
        t = (graphs.draw(seed, e) * (j + 1)) >> 64
        e += 1
        chosen.add(j if t in chosen else t)
    return sorted(chosen)


@pytest.mark.parametrize("s,seed", [(1, 3), (37, 4), (300, 5), (999, 6)])
def test_induced_subgraph_matches_brute_force(s, seed):
    g = graphs.chung_lu(1000, 12, 2.5, 1.0, 9)
    h = graphs.induced(g, s, seed)
    _check_oriented(h)
    sub = _floyd_subset(g.n, s, seed)
    assert h.n == len(sub) == s
    idx = {v: i for i, v in enumerate(sub)}
    want = set()
    for u in sub:
        for v in g.col[g.row_ptr[u]:g.row_ptr[u + 1]]:
            if int(v) in idx:
                want.add((idx[u], idx[int(v)]))
    got = {(u, int(v)) for u in range(h.n) for v in h.col[h.row_ptr[u]:h.row_ptr[u + 1]]}
    assert got == want


def test_induced_whole_graph_and_threads():
    g = graphs.chung_lu(2000, 16, 2.5, 1.0, 1)
    assert graphs.induced(g, g.n, 3).checksum() == g.checksum()
    assert graphs.induced(g, 0, 3).n == 0
    hs = graphs.induced_many(g, [(700, i) for i in range(12)], threads=4)
    assert [h.checksum() for h in hs] == [graphs.induced(g, 700, i).checksum() for i in range(12)]


def test_serving_mix_recipe():
    from synth import serving
    specs = serving.serving_mix(20000, 5)
    kc = [s for s in specs if s.kind == "kclique"]
    ut = [s for s in specs if s.kind == "uts"]
    assert abs(len(kc) / 20000 - 0.6) < 0.02
    assert {s.k for s in kc} == {4, 5, 6, 7, 8}
    sizes = np.array([s.s for s in kc], dtype=np.float64)
    assert sizes.min() >= 1000 and sizes.max() <= 200000
    # log-uniform: the log sizes are uniform, mean at the log midpoint
    ls = np.log(sizes)
    assert abs(ls.mean() - 0.5 * (np.log(1000) + np.log(200000))) < 0.05
    ms = np.array([s.m for s in ut])
    assert ms.min() >= 2.0 and ms.max() <= 4.0 and abs(ms.mean() - 3.0) < 0.05
    assert {s.depth for s in ut} == set(range(8, 15))
    assert serving.serving_mix(300, 5) == serving.serving_mix(300, 5)


def test_poisson_arrivals_rate():
    from synth import serving
    t = serving.poisson_arrivals(100000, 250.0, 3)
    assert t[0] == 0.0 and np.all(np.diff(t) >= 0)
    assert abs(len(t) / t[-1] - 250.0) / 250.0 < 0.02
