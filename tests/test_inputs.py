"""Seeded synthetic inputs: shape checks of the generated graphs."""
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
