"""GPU parity: the HIP fork-join runtime against the CPU oracle.

Every case compares the job result bit-exactly and, for single-job runs, the
number of first executions (tasks) and post-join re-executions (conts) with
the oracle's counts of the same recursion: equal counts mean every task ran
exactly once, whatever the schedule.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import graphs

pytestmark = pytest.mark.gpu

THR4 = oracle.uts_threshold(4)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gtap():
    from paper_2604_05982_amd import gtap as mod
    return mod


def make_rt(gtap, **kw):
    kw.setdefault("timeout_ms", 30000)
    kw.setdefault("small_frames", 1 << 23)
    kw.setdefault("big_frames", 1 << 18)
    kw.setdefault("big_frame_ints", 512)
    return gtap.Runtime(**kw)


@pytest.fixture(scope="module")
def rt(gtap):
    r = make_rt(gtap)
    yield r
    r.close()


def run_single(rt, submit, *args, **kw):
    jid = submit(*args, **kw)
    rt.run()
    return rt.result(jid), rt.stats()


def check(got, st, want):
    assert got == want.value
    assert st["tasks"] == want.tasks, (st["tasks"], want.tasks)
    assert st["conts"] == want.conts, (st["conts"], want.conts)


# ---- Fibonacci ------------------------------------------------------------
@pytest.mark.parametrize("n", [0, 1, 2, 3, 7, 15, 24])
def test_fib(rt, n):
    say(f"fib n={n}")
    got, st = run_single(rt, rt.submit_fib, n)
    check(got, st, oracle.fib(n))


def test_fib32_full_size(rt):
    say("fib n=32 (full size)")
    got, st = run_single(rt, rt.submit_fib, 32)
    check(got, st, oracle.fib(32))


# ---- N-Queens -------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 8, 10])
def test_nqueens(rt, n):
    say(f"nqueens n={n}")
    got, st = run_single(rt, rt.submit_nqueens, n)
    check(got, st, oracle.nqueens(n))


def test_nqueens13_full_size(rt):
    say("nqueens n=13 (full size)")
    got, st = run_single(rt, rt.submit_nqueens, 13)
    check(got, st, oracle.nqueens(13))


# ---- UTS ------------------------------------------------------------------
@pytest.mark.parametrize("seed,depth", [(1, 0), (1, 1), (1, 4), (7, 6), (123, 8), (5, 10)])
def test_uts(rt, seed, depth):
    say(f"uts seed={seed} depth={depth}")
    got, st = run_single(rt, rt.submit_uts, seed, THR4, depth)
    check(got, st, oracle.uts(seed, THR4, depth))


def test_uts_other_means(rt):
    for m, seed, depth in ((2, 3, 12), (3, 4, 9)):
        thr = oracle.uts_threshold(m)
        say(f"uts mean={m} seed={seed} depth={depth}")
        got, st = run_single(rt, rt.submit_uts, seed, thr, depth)
        check(got, st, oracle.uts(seed, thr, depth))


def test_uts_depth13_full_size(rt):
    say("uts seed=1 mean=4 depth=13 (full size)")
    got, st = run_single(rt, rt.submit_uts, 1, THR4, 13)
    check(got, st, oracle.uts(1, THR4, 13))


# ---- k-clique -------------------------------------------------------------
def _rand_edges(n, p, seed):
    rng = np.random.default_rng(seed)
    iu = np.triu_indices(n, 1)
    keep = rng.random(iu[0].size) < p
    return np.stack([iu[0][keep], iu[1][keep]], axis=1)


@pytest.mark.parametrize("seed,n,p,leaf", [(1, 30, 0.4, 4), (2, 60, 0.25, 8), (3, 130, 0.15, 64)])
def test_kclique_random(rt, seed, n, p, leaf):
    g = graphs.oriented_from_edges(n, _rand_edges(n, p, seed), "degeneracy")
    for k in range(1, 7):
        say(f"kclique random seed={seed} n={n} k={k} leaf={leaf}")
        got, st = run_single(rt, rt.submit_kclique, g.row_ptr32, g.col, k, range_leaf=leaf)
        check(got, st, oracle.kclique(g.row_ptr, g.col, k, range_leaf=leaf))


def test_kclique_degenerate(rt):
    say("kclique degenerate graphs")
    for n, edges in ((1, []), (10, []), (2, [(0, 1)]), (4, [(0, 1), (1, 2), (2, 0), (2, 3)])):
        g = graphs.oriented_from_edges(n, edges, "degeneracy")
        for k in (1, 2, 3, 4):
            got, st = run_single(rt, rt.submit_kclique, g.row_ptr32, g.col, k, range_leaf=2)
            check(got, st, oracle.kclique(g.row_ptr, g.col, k, range_leaf=2))


def test_kclique_chung_lu_2000_k4(rt):
    """Thread mode, single queue: 4-cliques of the n=2000, mean degree 16,
    exponent 2.5 Chung-Lu graph (seed 1)."""
    g = graphs.chung_lu(2000, 16, 2.5, 1.0, 1)
    say(f"kclique chung-lu n=2000 k=4 checksum={g.checksum()}")
    got, st = run_single(rt, rt.submit_kclique, g.row_ptr32, g.col, 4)
    check(got, st, oracle.kclique(g.row_ptr, g.col, 4))


# ---- batching: many roots of uneven size in one launch ---------------------
def test_batch_mixed(rt):
    rng = np.random.default_rng(5)
    g = graphs.chung_lu(500, 10, 2.5, 1.0, 3)
    jobs = []
    for i in range(400):
        kind = i % 4
        if kind == 0:
            n = int(rng.integers(0, 21))
            jobs.append((rt.submit_fib(n), oracle.fib(n).value))
        elif kind == 1:
            n = int(rng.integers(1, 10))
            jobs.append((rt.submit_nqueens(n), oracle.nqueens(n).value))
        elif kind == 2:
            s, d = int(rng.integers(1, 10**9)), int(rng.integers(0, 8))
            jobs.append((rt.submit_uts(s, THR4, d), oracle.uts(s, THR4, d).value))
        else:
            k = int(rng.integers(3, 6))
            jobs.append((rt.submit_kclique(g.row_ptr32, g.col, k), oracle.kclique(g.row_ptr, g.col, k).value))
    say("batch of 400 mixed jobs")
    rt.run()
    for jid, want in jobs:
        assert rt.result(jid) == want


def test_repeated_runs_same_context(rt):
    say("repeated runs")
    want = oracle.nqueens(9).value
    for _ in range(5):
        jid = rt.submit_nqueens(9)
        rt.run()
        assert rt.result(jid) == want


# ---- adversarial scheduling: the counts must not move ----------------------
@pytest.mark.parametrize("opts", [
    dict(num_waves=1, waves_per_group=1),
    dict(num_waves=4, waves_per_group=1, steal_below=1),
    dict(waves_per_group=1, steal_below=1),
    dict(waves_per_group=8),
])
def test_adversarial_configs(gtap, opts):
    say(f"adversarial config {opts}")
    with make_rt(gtap, **opts) as r:
        for sub, arg, want in ((r.submit_fib, (20,), oracle.fib(20)),
                               (r.submit_nqueens, (9,), oracle.nqueens(9)),
                               (r.submit_uts, (3, THR4, 7), oracle.uts(3, THR4, 7))):
            got, st = run_single(r, sub, *arg)
            check(got, st, want)


def test_small_deques_wrap_around(gtap):
    """Two waves with 1024-slot rings: more IDs pass through the rings than
    they hold (about 4,100 for fib(33)), so slots are reused after
    wrap-around."""
    say("small deques wrap around")
    with make_rt(gtap, num_waves=2, waves_per_group=2, deque_capacity=1024) as r:
        got, st = run_single(r, r.submit_fib, 33)
        check(got, st, oracle.fib(33))
        assert st["pushed"] > 2 * 1024
        assert st["local_pushed"] > 0


@pytest.mark.parametrize("job", ["fib", "uts", "nqueens"])
def test_private_stack_single_wave(gtap, job):
    """One wavefront: children beyond the lanes live on its LDS stack, the
    oldest are exposed to its own deque when the stack overflows or the deque
    is empty, and come back through PopBatch."""
    say(f"private stack, one wave, {job}")
    with make_rt(gtap, num_waves=1, waves_per_group=1) as r:
        if job == "fib":
            got, st = run_single(r, r.submit_fib, 23)
            check(got, st, oracle.fib(23))
        elif job == "uts":
            got, st = run_single(r, r.submit_uts, 5, THR4, 8)
            check(got, st, oracle.uts(5, THR4, 8))
        else:
            got, st = run_single(r, r.submit_nqueens, 10)
            check(got, st, oracle.nqueens(10))
        assert st["local_pushed"] > 0 and st["stolen"] == 0


# ---- capacity exhaustion is a structured error, not a hang -----------------
def test_frame_pool_exhaustion_reports(gtap):
    say("frame pool exhaustion")
    with make_rt(gtap, small_frames=1024, num_waves=64, waves_per_group=1) as r:
        r.submit_fib(27)
        with pytest.raises(gtap.GtapError) as ei:
            r.run()
        assert ei.value.code == gtap.GTAP_E_CAPACITY
        assert ei.value.report["pool"] == 0 and ei.value.report["capacity"] == 1024
        # the context stays usable
        got, st = run_single(r, r.submit_fib, 5)
        check(got, st, oracle.fib(5))


def test_deque_exhaustion_reports(gtap):
    say("deque exhaustion")
    # a star: vertex 0 points at 2000 others, one wave, 128-slot deque
    n = 2001
    edges = [(0, j) for j in range(1, n)]
    g = graphs.oriented_from_edges(n, edges, "id")
    with make_rt(gtap, num_waves=1, waves_per_group=1, deque_capacity=128, big_frame_ints=2048) as r:
        r.submit_kclique(g.row_ptr32, g.col, 3, range_leaf=(1 << 20) - 1)
        with pytest.raises(gtap.GtapError) as ei:
            r.run()
        assert ei.value.code == gtap.GTAP_E_CAPACITY and ei.value.report["pool"] == 2


def test_submit_validation(gtap, rt):
    with pytest.raises(gtap.GtapError) as ei:
        rt.submit_fib(-1)
    assert ei.value.code == gtap.GTAP_E_INVAL
    with pytest.raises(gtap.GtapError):
        rt.submit_nqueens(0)
    with pytest.raises(gtap.GtapError):
        rt.submit_uts(1, THR4, 300)


# ---- DAQ: the queue configuration changes the schedule, never the result ----
@pytest.mark.parametrize("opts", [
    dict(num_queues=4, daq_policy=2, daq_bounds=[8, 32, 128]),
    dict(num_queues=2, daq_policy=2, daq_bounds=[4]),
    dict(num_queues=3, daq_policy=1),
    dict(num_queues=8, daq_policy=1, num_waves=2, waves_per_group=1),
])
def test_daq_configs(gtap, opts):
    say(f"daq config {opts}")
    g = graphs.chung_lu(2000, 16, 2.5, 1.0, 1)
    with make_rt(gtap, **opts) as r:
        for k in (3, 4, 5):
            got, st = run_single(r, r.submit_kclique, g.row_ptr32, g.col, k)
            check(got, st, oracle.kclique(g.row_ptr, g.col, k))
        for sub, arg, want in ((r.submit_fib, (18,), oracle.fib(18)),
                               (r.submit_uts, (9, THR4, 7), oracle.uts(9, THR4, 7))):
            got, st = run_single(r, sub, *arg)
            check(got, st, want)
        # a mixed batch spreads over the classes
        jobs = [(r.submit_fib(15), oracle.fib(15).value), (r.submit_nqueens(8), oracle.nqueens(8).value),
                (r.submit_uts(4, THR4, 6), oracle.uts(4, THR4, 6).value),
                (r.submit_kclique(g.row_ptr32, g.col, 4), oracle.kclique(g.row_ptr, g.col, 4).value)]
        r.run()
        for jid, want in jobs:
            assert r.result(jid) == want


# ---- full-size k-clique: n = 10^6, mean degree 40, exponent 2.1 (cap 0.6, seed 2) ----
def _golden_kclique():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "kclique_chung_lu.txt")
    out = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, csum, k, count, tasks, conts = line.split()
            out[(name, int(k))] = (csum, int(count), int(tasks), int(conts))
    return out


@pytest.fixture(scope="module")
def big_graph():
    return graphs.chung_lu(1000000, 40, 2.1, 0.6, 2)


@pytest.mark.parametrize("queues", [1, 4])
def test_kclique_1m_k7(gtap, big_graph, queues):
    gold = _golden_kclique()
    g = big_graph
    name = "n1000000_d40_g2.1_cap0.6_s2"
    opts = dict(num_waves=1024, deque_capacity=1 << 17, small_frames=1 << 25, big_frames=1 << 23,
                big_frame_ints=max(320, g.max_outdeg), timeout_ms=60000)
    if queues > 1:
        # per-class deques hold the breadth that one LIFO deque keeps depth-first
        opts.update(num_queues=4, daq_policy=2, daq_bounds=[8, 32, 128], deque_capacity=1 << 19,
                    big_frames=1 << 24)
    with make_rt(gtap, **opts) as r:
        for k in (5, 7):
            csum, count, tasks, conts = gold[(name, k)]
            assert g.checksum() == csum
            say(f"kclique n=1e6 k={k} queues={queues}")
            got, st = run_single(r, r.submit_kclique, g.row_ptr32, g.col, k)
            assert got == count
            assert st["tasks"] == tasks and st["conts"] == conts
