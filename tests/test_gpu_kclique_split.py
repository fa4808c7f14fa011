"""GPU parity of k-clique counting with bitset candidate subgraphs and
cost-threshold task splitting (Sec. 6.4.2: orientation and pivoting).

The count must equal the oracle's (bit-exact), and the runtime's task and
continuation counts must equal those of the oracle's task tree for the same
threshold plus the runtime's own vertex level (`kernel_vertex_level`, a
closed form over the out-degrees): the split decisions depend only on the
graph, never on the schedule.  Graphs span one-word candidate sets, multi-word bit matrices
(candidate sets above 64: complete and complete multipartite graphs) and the
full 10^6-vertex Chung-Lu graph.
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle
from synth import graphs

pytestmark = pytest.mark.gpu

ALGS = ("orient", "pivot")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gtap():
    from paper_2604_05982_amd import gtap as mod
    return mod


def kernel_vertex_level(g, k, thr):
    """Tasks and continuations the runtime's vertex level adds to the task
    tree of the paper's levels (ranges, vertices, one task per edge, the
    threshold split), from the out-degrees d alone.  For k >= 4 the runtime
    decides per vertex:
      - d < k-1 (no k-clique can start there) or d <= thr (every candidate
        set of its edges is smaller than d): the vertex counts its edges in
        place -- d edge tasks and the vertex's resumption fewer;
      - otherwise it first forks d row tasks that build its bit matrix and
        resumes once more -- d tasks and one resumption more.
    k <= 3 vertices fork the paper's tree unchanged."""
    if k < 4:
        return 0, 0
    d = np.diff(np.asarray(g.row_ptr, dtype=np.int64))
    d = d[d > 0]
    inplace = (d < k - 1) | (d <= thr)
    return (int(d[~inplace].sum()) - int(d[inplace].sum()),
            int((~inplace).sum()) - int(inplace.sum()))


def assert_tree(st, want, g, k, thr, ctx=None):
    dt, dc = kernel_vertex_level(g, k, thr)
    assert (st["tasks"], st["conts"]) == (want.tasks + dt, want.conts + dc), (ctx, k, thr)


def alg_code(gtap, name):
    return gtap.GTAP_KCLIQUE_PIVOT if name == "pivot" else gtap.GTAP_KCLIQUE_ORIENT


def make_rt(gtap, max_outdeg, big_frames=1 << 16, **kw):
    kw.setdefault("timeout_ms", 60000)
    return gtap.Runtime(mode=gtap.GTAP_MODE_THREAD, waves_per_group=4, small_frames=1 << 22,
                        big_frames=big_frames,
                        big_frame_ints=max(64, gtap.kclique_split_buffer_ints(max_outdeg)), **kw)


def run_split(rt, g, k, thr, alg, gtap, range_leaf=64):
    import torch
    rp = torch.as_tensor(g.row_ptr32).cuda()
    col = torch.as_tensor(g.col if g.col.size else np.zeros(1, np.int32)).cuda()
    jid = rt.submit_kclique_split(rp, col, k, threshold=thr, algorithm=alg_code(gtap, alg),
                                  range_leaf=range_leaf, max_outdeg=g.max_outdeg)
    rt.run()
    return rt.result(jid), rt.stats()


def complete_graph(n):
    return graphs.oriented_from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)], "id")


def multipartite(t, s, order="random"):
    n = t * s
    edges = [(a, b) for a in range(n) for b in range(a + 1, n) if a % t != b % t]
    return graphs.oriented_from_edges(n, edges, order, seed=t + s)


@pytest.mark.parametrize("alg", ALGS)
def test_split_chung_lu_small_counts_and_trees(gtap, alg):
    g = graphs.chung_lu(2000, 16, 2.5, 1.0, 1)
    with make_rt(gtap, g.max_outdeg) as rt:
        for k in (3, 4, 5, 6, 7):
            for thr in (0, 4, 16, 64):
                say(f"split k-clique {alg} chung-lu n=2000 k={k} thr={thr}")
                got, st = run_split(rt, g, k, thr, alg, gtap)
                want = oracle.kclique_split(g.row_ptr, g.col, k, threshold=thr, algorithm=alg)
                assert got == want.value == oracle.kclique(g.row_ptr, g.col, k).value
                assert_tree(st, want, g, k, thr)


@pytest.mark.parametrize("alg", ALGS)
def test_split_multiword_candidate_sets(gtap, alg):
    """Candidate sets of 65..98 vertices: two-word rows, node sets that span
    both words, pivots and non-neighbours on either side of bit 64."""
    cases = {("orient", "K_100"): ((3, 4, 5), (0, 8, 40)), ("pivot", "K_100"): ((3, 4, 5, 6), (0, 40)),
             ("orient", "K_{12x8}"): ((3, 4, 5), (0, 8, 40)), ("pivot", "K_{12x8}"): ((3, 4, 5), (8, 40))}
    for name, g, closed in (("K_100", complete_graph(100), lambda k: math.comb(100, k)),
                            ("K_{12x8}", multipartite(12, 8), lambda k: math.comb(12, k) * 8 ** k)):
        assert g.max_outdeg > 64
        ks, thrs = cases[(alg, name)]
        with make_rt(gtap, g.max_outdeg, big_frames=1 << 21) as rt:
            for k in ks:
                for thr in thrs:
                    say(f"split k-clique {alg} {name} k={k} thr={thr}")
                    got, st = run_split(rt, g, k, thr, alg, gtap)
                    want = oracle.kclique_split(g.row_ptr, g.col, k, threshold=thr, algorithm=alg)
                    assert got == want.value == closed(k), (name, k, thr)
                    assert_tree(st, want, g, k, thr, name)


@pytest.mark.parametrize("alg", ALGS)
def test_split_medium_chung_lu(gtap, alg):
    """A heavier-tailed graph whose largest candidate sets span several words."""
    g = graphs.chung_lu(30000, 40, 2.1, 1.0, 9)
    say(f"medium graph: max out-degree {g.max_outdeg}")
    with make_rt(gtap, g.max_outdeg, big_frames=1 << 20) as rt:
        for k, thr in ((4, 16), (6, 16)):
            say(f"split k-clique {alg} chung-lu n=30000 k={k} thr={thr}")
            got, st = run_split(rt, g, k, thr, alg, gtap)
            want = oracle.kclique_split(g.row_ptr, g.col, k, threshold=thr, algorithm=alg)
            assert got == want.value
            assert_tree(st, want, g, k, thr)


@pytest.mark.parametrize("alg", ALGS)
def test_split_degenerate_cases(gtap, alg):
    e0 = graphs.oriented_from_edges(50, [], "id")
    tri = graphs.oriented_from_edges(4, [(0, 1), (1, 2), (2, 0), (2, 3)], "degeneracy")
    with make_rt(gtap, 64) as rt:
        say(f"split k-clique {alg}: empty graph, k = 1, 2, 4")
        assert run_split(rt, e0, 1, 4, alg, gtap)[0] == 50
        assert run_split(rt, e0, 2, 4, alg, gtap)[0] == 0
        assert run_split(rt, e0, 4, 4, alg, gtap)[0] == 0
        say(f"split k-clique {alg}: triangle with a pendant")
        assert [run_split(rt, tri, k, 0, alg, gtap)[0] for k in (1, 2, 3, 4)] == [4, 4, 1, 0]
        say(f"split k-clique {alg}: K_9, k = 9 and 10")
        k9 = complete_graph(9)
        assert run_split(rt, k9, 9, 0, alg, gtap)[0] == 1
        assert run_split(rt, k9, 10, 0, alg, gtap)[0] == 0


def test_split_config_rules(gtap):
    import torch
    g = graphs.chung_lu(500, 10, 2.5, 1.0, 3)
    rp = torch.as_tensor(g.row_ptr32).cuda()
    col = torch.as_tensor(g.col).cuda()
    say("split k-clique argument and configuration checks")
    with make_rt(gtap, g.max_outdeg) as rt:
        for kw in (dict(k=0), dict(k=33), dict(threshold=-1), dict(threshold=65), dict(algorithm=2),
                   dict(range_leaf=0), dict(max_outdeg=g.max_outdeg - 1), dict(max_outdeg=1025)):
            args = dict(k=5, threshold=16, algorithm=gtap.GTAP_KCLIQUE_ORIENT, max_outdeg=g.max_outdeg)
            args.update(kw)
            with pytest.raises(gtap.GtapError) as e:
                rt.submit_kclique_split(rp, col, **args)
            assert e.value.code == gtap.GTAP_E_INVAL, kw
        jid = rt.submit_kclique_split(rp, col, 4, max_outdeg=g.max_outdeg)
        rt.run()
        assert rt.result(jid) == oracle.kclique(g.row_ptr, g.col, 4).value
    # too small big frames, block mode, two waves per group
    for rtkw in (dict(big_frame_ints=gtap.kclique_split_buffer_ints(g.max_outdeg) - 1),
                 dict(mode=gtap.GTAP_MODE_BLOCK, waves_per_group=1), dict(waves_per_group=2)):
        opts = dict(mode=gtap.GTAP_MODE_THREAD, waves_per_group=4, small_frames=1 << 16, big_frames=1 << 10,
                    big_frame_ints=gtap.kclique_split_buffer_ints(g.max_outdeg))
        opts.update(rtkw)
        with gtap.Runtime(**opts) as rt:
            with pytest.raises(gtap.GtapError) as e:
                rt.submit_kclique_split(rp, col, 5, max_outdeg=g.max_outdeg)
            assert e.value.code == gtap.GTAP_E_INVAL, rtkw


def test_split_shares_launch_with_other_jobs(gtap):
    """Split k-clique jobs of both algorithms, a plain k-clique job, fib jobs
    and a Cilksort job in one launch."""
    import torch
    g = graphs.chung_lu(3000, 20, 2.3, 1.0, 12)
    rp = torch.as_tensor(g.row_ptr32).cuda()
    col = torch.as_tensor(g.col).cuda()
    keys = np.random.default_rng(4).integers(0, 2**32, size=20000, dtype=np.uint32)
    kt = torch.from_numpy(keys.view(np.int32)).cuda()
    with make_rt(gtap, g.max_outdeg, big_frames=1 << 19) as rt:
        say("split k-clique jobs with other kinds in one launch")
        jobs = [(rt.submit_kclique_split(rp, col, k, threshold=t, algorithm=a, max_outdeg=g.max_outdeg),
                 oracle.kclique(g.row_ptr, g.col, k).value)
                for k, t, a in ((5, 8, gtap.GTAP_KCLIQUE_ORIENT), (6, 4, gtap.GTAP_KCLIQUE_PIVOT),
                                (4, 0, gtap.GTAP_KCLIQUE_PIVOT))]
        jobs.append((rt.submit_kclique(rp, col, 5, max_outdeg=g.max_outdeg), oracle.kclique(g.row_ptr, g.col, 5).value))
        jobs += [(rt.submit_fib(n), oracle.fib(n).value) for n in (15, 20)]
        js = rt.submit_cilksort(kt)
        rt.run()
        assert [rt.result(j) for j, _ in jobs] == [w for _, w in jobs]
        assert np.array_equal(kt.cpu().numpy().view(np.uint32), np.sort(keys)) and rt.result(js) == keys.size


@pytest.mark.parametrize("alg", ALGS)
def test_split_full_size_chung_lu_1m(gtap, alg):
    """7-cliques of the 10^6-vertex Chung-Lu graph (mean degree 40, exponent
    2.1, cap 0.6, seed 2): the stored oracle count."""
    want = None
    with open(os.path.join(os.path.dirname(__file__), "golden", "kclique_chung_lu.txt")) as fh:
        for line in fh:
            f = line.split()
            if len(f) == 6 and f[0] == "n1000000_d40_g2.1_cap0.6_s2" and f[2] == "7":
                want = (f[1], int(f[3]))
    g = graphs.chung_lu(1000000, 40, 2.1, 0.6, 2)
    assert g.checksum() == want[0]
    with make_rt(gtap, g.max_outdeg, big_frames=1 << 23, deque_capacity=1 << 17) as rt:
        say(f"split k-clique {alg}: 7-cliques of the 10^6-vertex graph")
        got, st = run_split(rt, g, 7, 16, alg, gtap)
        say(f"  count {got}, tasks {st['tasks']}, kernel {st['kernel_ms']:.1f} ms")
        assert got == want[1]


@pytest.mark.parametrize("alg", ALGS)
def test_split_with_daq_queues(gtap, alg):
    """Divergence-aware queueing (4 classes by the out-degree bound of a
    vertex's or an edge's candidate set): same counts and task trees."""
    g = graphs.chung_lu(4000, 18, 2.3, 1.0, 5)
    with make_rt(gtap, g.max_outdeg, big_frames=1 << 18, num_queues=4, daq_policy=gtap.GTAP_DAQ_KCLIQUE,
                 daq_bounds=[8, 32, 128], deque_capacity=1 << 16) as rt:
        for k, thr in ((4, 8), (6, 16), (7, 64)):
            say(f"split k-clique {alg} with 4 DAQ queues, k={k} thr={thr}")
            got, st = run_split(rt, g, k, thr, alg, gtap)
            want = oracle.kclique_split(g.row_ptr, g.col, k, threshold=thr, algorithm=alg)
            assert got == want.value
            assert_tree(st, want, g, k, thr)


@pytest.mark.parametrize("alg", ALGS)
def test_split_max_outdegree_1024(gtap, alg):
    """A hub with the largest allowed out-degree (1024: 16-word rows and node
    sets) over a 40-clique and a sparse remainder: counts and task trees
    against the oracle, and the closed form C(40, k-1) + C(40, k) + (cliques
    of the remainder, none here beyond edges and triangles)."""
    rng = np.random.default_rng(17)
    n = 1025
    edges = [(0, v) for v in range(1, n)]
    edges += [(a, b) for a in range(1, 41) for b in range(a + 1, 41)]
    edges += [(int(a), int(b)) for a, b in rng.integers(41, n, size=(300, 2)) if a < b]
    edges = sorted(set(edges))
    g = graphs.oriented_from_edges(n, edges, "id")
    assert g.max_outdeg == 1024
    with make_rt(gtap, g.max_outdeg, big_frames=1 << 20) as rt:
        for k, thr in ((4, 8), (5, 8), (6, 0), (5, 64)):
            say(f"split k-clique {alg}: hub of out-degree 1024, k={k} thr={thr}")
            got, st = run_split(rt, g, k, thr, alg, gtap)
            want = oracle.kclique_split(g.row_ptr, g.col, k, threshold=thr, algorithm=alg)
            assert got == want.value == math.comb(40, k - 1) + math.comb(40, k)
            assert_tree(st, want, g, k, thr)
