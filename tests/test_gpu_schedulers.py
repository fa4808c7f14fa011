"""GPU parity of the thread-mode scheduler variants of the scheduler
comparison (Sec. 6.5): the batched work-stealing deques without the private
LDS stack, non-batched work stealing (one task per pop and per steal) and a
centralised FIFO queue.  They differ only in queue management, so every
variant must give the oracle's result and the oracle's task and continuation
counts exactly; the runtime counters must show the variant's queue traffic.
"""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

THR4 = oracle.uts_threshold(4)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gtap():
    from paper_2604_05982_amd import gtap as mod
    return mod


def variants(g):
    return {"nolocal": g.GTAP_FLAG_NO_PRIVATE_STACK,
            "single": g.GTAP_FLAG_SCHED_SINGLE,
            "central": g.GTAP_FLAG_SCHED_CENTRAL}


def make_rt(gtap, **kw):
    kw.setdefault("timeout_ms", 60000)
    kw.setdefault("small_frames", 1 << 23)
    kw.setdefault("big_frames", 1 << 10)
    return gtap.Runtime(**kw)


def check(rt, jid, want):
    st = rt.stats()
    assert rt.result(jid) == want.value
    assert (st["tasks"], st["conts"]) == (want.tasks, want.conts)
    return st


@pytest.mark.parametrize("name", ["nolocal", "single", "central"])
@pytest.mark.parametrize("waves", [1, 8, 0])
def test_variant_counts_match_oracle(gtap, name, waves):
    flag = variants(gtap)[name]
    say(f"scheduler variant {name}, num_waves={waves}")
    with make_rt(gtap, flags=flag, num_waves=waves) as r:
        for sub, args, want in ((r.submit_fib, (22,), oracle.fib(22)),
                                (r.submit_nqueens, (9,), oracle.nqueens(9)),
                                (r.submit_uts, (3, THR4, 8), oracle.uts(3, THR4, 8))):
            jid = sub(*args)
            r.run()
            st = check(r, jid, want)
            assert st["local_pushed"] == 0  # every variant runs without the LDS stack
            if name == "central":
                assert st["stolen"] == 0 and st["steal_attempts"] == 0
                assert st["pushed"] == st["popped"] > 0
            if name == "single":
                assert st["popped"] == st["pop_batches"]
                assert st["stolen"] == st["steal_batches"]


@pytest.mark.parametrize("name", ["single", "central"])
def test_variant_full_size_fib32_and_batch(gtap, name):
    flag = variants(gtap)[name]
    say(f"scheduler variant {name}: fib(32) and a 200-job batch")
    with make_rt(gtap, flags=flag) as r:
        jid = r.submit_fib(32)
        r.run()
        check(r, jid, oracle.fib(32))
        rng = np.random.default_rng(11)
        jobs, wants = [], []
        for i in range(200):
            if i % 2:
                s, d = int(rng.integers(1, 2**62)), int(rng.integers(0, 9))
                jobs.append(r.submit_uts(s, THR4, d))
                wants.append(oracle.uts(s, THR4, d).value)
            else:
                n = int(rng.integers(0, 20))
                jobs.append(r.submit_fib(n))
                wants.append(oracle.fib(n).value)
        r.run()
        assert [r.result(j) for j in jobs] == wants


@pytest.mark.parametrize("waves", [256, 512])
def test_central_queue_mid_grids_fib30(gtap, waves):
    """The centralised queue at grid sizes where claims often cover positions
    whose pushes have not raised the count yet (their slots, and the frames
    the slots name, must already be complete)."""
    say(f"central queue, {waves} waves, fib(30) x 2")
    with make_rt(gtap, flags=gtap.GTAP_FLAG_SCHED_CENTRAL, num_waves=waves, deque_capacity=1 << 18) as r:
        for _ in range(2):
            jid = r.submit_fib(30)
            r.run()
            check(r, jid, oracle.fib(30))


def test_variant_configs_rejected(gtap):
    say("scheduler variant configuration checks")
    bad = [dict(flags=gtap.GTAP_FLAG_SCHED_SINGLE | gtap.GTAP_FLAG_SCHED_CENTRAL),
           dict(flags=gtap.GTAP_FLAG_SCHED_CENTRAL, num_queues=4),
           dict(flags=gtap.GTAP_FLAG_SCHED_SINGLE, mode=gtap.GTAP_MODE_BLOCK, waves_per_group=1),
           dict(flags=gtap.GTAP_FLAG_NO_PRIVATE_STACK, waves_per_group=2),
           dict(flags=8)]
    for kw in bad:
        with pytest.raises(gtap.GtapError) as e:
            make_rt(gtap, **kw)
        assert e.value.code == gtap.GTAP_E_INVAL, kw
    with make_rt(gtap, flags=gtap.GTAP_FLAG_SCHED_CENTRAL, num_waves=64) as r:
        with pytest.raises(gtap.GtapError) as e:
            r.serve_start(max_inflight=16)
        assert e.value.code == gtap.GTAP_E_INVAL
        # the context is still usable for batch runs
        jid = r.submit_fib(12)
        r.run()
        check(r, jid, oracle.fib(12))
