"""GPU parity of the serving path: jobs admitted into a running persistent
kernel through the pinned admission ring.

Every served job's result is compared bit-exactly with the oracle, and with
the same job launched alone (one persistent launch per job): a job's result
must not depend on which other jobs share the device with it.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import graphs

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gtap():
    from paper_2604_05982_amd import gtap as mod
    return mod


@pytest.fixture(scope="module")
def graph2000():
    import torch
    g = graphs.chung_lu(2000, 16, 2.5, 1.0, 1)
    rp = torch.as_tensor(g.row_ptr32).cuda()
    col = torch.as_tensor(g.col).cuda()
    return g, rp, col


def mixed_entries(rt, gtap, graph, n, seed, spacing_s=0.0):
    """n small jobs of all four kinds with their oracle results."""
    g, rp, col = graph
    rng = np.random.default_rng(seed)
    entries, want = [], []
    for i in range(n):
        t = i * spacing_s
        c = i % 4
        if c == 0:
            k = int(rng.integers(0, 21))
            entries.append((t, rt.fib_args(k)))
            want.append(oracle.fib(k).value)
        elif c == 1:
            k = int(rng.integers(1, 10))
            entries.append((t, rt.nqueens_args(k)))
            want.append(oracle.nqueens(k).value)
        elif c == 2:
            s = int(rng.integers(1, 1 << 62))
            m = float(rng.uniform(2.0, 4.0))
            d = int(rng.integers(0, 8))
            thr = oracle.uts_threshold(m)
            entries.append((t, rt.uts_args(s, thr, d)))
            want.append(oracle.uts(s, thr, d).value)
        else:
            k = int(rng.integers(2, 6))
            entries.append((t, rt.kclique_args(rp, col, k, max_outdeg=g.max_outdeg)))
            want.append(oracle.kclique(g.row_ptr, g.col, k).value)
    return entries, want


def make_rt(gtap, **kw):
    kw.setdefault("timeout_ms", 60000)
    kw.setdefault("small_frames", 1 << 22)
    kw.setdefault("big_frames", 1 << 20)
    kw.setdefault("big_frame_ints", 512)
    kw.setdefault("max_jobs", 256)
    return gtap.Runtime(**kw)


def test_serve_all_at_once_wraps_ring(gtap, graph2000):
    """600 jobs through a 256-slot ring (slots are reused), arrivals at t=0."""
    rt = make_rt(gtap)
    try:
        entries, want = mixed_entries(rt, gtap, graph2000, 600, seed=11)
        say("serve: 600 mixed jobs, ring 256")
        rt.serve_start(max_inflight=256)
        res = rt.trace_run(rt.trace(entries), timeout_ms=60000)
        rt.serve_stop()
        got = [r.result for r in res]
        assert all(r.status == 0 for r in res)
        assert got == want
        st = rt.stats()
        assert st["admitted"] == 600
        assert all(r.done_s >= r.submit_s >= 0.0 for r in res)
    finally:
        rt.close()


def test_serve_open_loop_matches_plain(gtap, graph2000):
    """Jobs arriving 0.2 ms apart: served results equal one-launch-per-job results."""
    rt = make_rt(gtap)
    try:
        entries, want = mixed_entries(rt, gtap, graph2000, 200, seed=12, spacing_s=2e-4)
        jobs = rt.trace(entries)
        say("plain: 200 jobs, one launch each")
        plain = rt.trace_run_plain(jobs)
        assert [r.result for r in plain] == want
        say("serve: same 200 jobs, open loop")
        rt.serve_start(max_inflight=64)
        res = rt.trace_run(jobs, timeout_ms=60000)
        rt.serve_stop()
        assert [r.result for r in res] == want
        # the serving kernel stopped cleanly: batch runs work again afterwards
        j = rt.submit_fib(20)
        rt.run()
        assert rt.result(j) == 6765
    finally:
        rt.close()


def test_serve_submit_poll(gtap):
    """Explicit submit/poll; tickets complete in any order but each exactly once."""
    rt = make_rt(gtap)
    try:
        thr = oracle.uts_threshold(4)
        rt.serve_start(max_inflight=8)
        tickets = []
        want = []
        for i in range(40):
            kind, a = rt.uts_args(1000 + i, thr, 6) if i % 2 else rt.fib_args(i % 23)
            tickets.append(rt.serve_submit(kind, a))
            want.append(oracle.uts(1000 + i, thr, 6).value if i % 2 else oracle.fib(i % 23).value)
        assert tickets == list(range(40))
        got = {}
        import time
        t_end = time.time() + 60
        while len(got) < len(tickets) and time.time() < t_end:
            for t in tickets:
                if t not in got:
                    r = rt.serve_poll(t)
                    if r is not None:
                        got[t] = r[0]
        rt.serve_stop()
        assert [got.get(t) for t in tickets] == want
    finally:
        rt.close()


def test_serve_inflight_one(gtap, graph2000):
    """max_inflight=1 serialises admission; results unchanged."""
    rt = make_rt(gtap)
    try:
        entries, want = mixed_entries(rt, gtap, graph2000, 40, seed=13)
        rt.serve_start(max_inflight=1)
        res = rt.trace_run(rt.trace(entries), timeout_ms=60000)
        rt.serve_stop()
        assert [r.result for r in res] == want
    finally:
        rt.close()


def test_serve_headroom_blocks_until_frames_free(gtap):
    """Admission by free frame-pool memory: a headroom that leaves room for
    only a few roots at a time still completes every job."""
    rt = make_rt(gtap, small_frames=1 << 16, big_frames=1 << 10, num_waves=32)
    try:
        thr = oracle.uts_threshold(3)
        entries = [(0.0, rt.uts_args(77 + i, thr, 5)) for i in range(64)]
        want = [oracle.uts(77 + i, thr, 5).value for i in range(64)]
        rt.serve_start(max_inflight=64, headroom_small=(1 << 16) - 2048)
        res = rt.trace_run(rt.trace(entries), timeout_ms=60000)
        rt.serve_stop()
        assert [r.result for r in res] == want
    finally:
        rt.close()


def test_serve_state_errors(gtap):
    rt = make_rt(gtap)
    try:
        kind, a = rt.fib_args(5)
        with pytest.raises(gtap.GtapError) as e:
            rt.serve_submit(kind, a)
        assert e.value.code == gtap.GTAP_E_STATE
        rt.serve_start(max_inflight=4)
        with pytest.raises(gtap.GtapError) as e:
            rt.run()
        assert e.value.code == gtap.GTAP_E_STATE
        with pytest.raises(gtap.GtapError) as e:
            rt.serve_start(max_inflight=4)
        assert e.value.code == gtap.GTAP_E_STATE
        t = rt.serve_submit(kind, a)
        rt.serve_stop()
        assert rt.serve_poll(t)[0] == 5
        with pytest.raises(gtap.GtapError) as e:
            rt.serve_stop()
        assert e.value.code == gtap.GTAP_E_STATE
    finally:
        rt.close()
