"""The allocation-free entry point (gtap_run_static) against the allocating
path (gtap_init + gtap_submit + gtap_run + gtap_result) on the same jobs.

Two calls in a row share the device's static workspace; the second is
smaller, so anything the first left behind that the second failed to clear
would show up as a wrong result.  A configuration whose workspace does not
fit is rejected before anything runs.
"""
import sys

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
def graph():
    import torch
    g = graphs.chung_lu(2000, 16, 2.5, 1.0, 1)
    return g, torch.as_tensor(g.row_ptr32).cuda(), torch.as_tensor(g.col).cuda()


# a configuration whose workspace fits the static array
# (about 175 MB: 64 MiB of small frames, 2^15 big frames of 2,112 bytes,
# 1,024 deques of 2^13 slots)
SMALL = dict(small_frames=1 << 20, big_frames=1 << 15, big_frame_ints=512, deque_capacity=1 << 13,
             num_waves=1024, waves_per_group=4, timeout_ms=60000)


def config(gtap, **kw):
    import torch
    cfg = gtap.gtap_config_default()
    for k, v in {**SMALL, **kw}.items():
        setattr(cfg, k, v)
    cfg.stream = torch.cuda.current_stream().cuda_stream
    return cfg


def entries(gtap, graph, big):
    g, rp, col = graph
    thr = gtap.uts_threshold(4)
    rt = gtap.Runtime  # argument structs only
    if big:
        return [rt.fib_args(27), rt.nqueens_args(11), rt.uts_args(1, thr, 10), rt.uts_args(7, thr, 9),
                (gtap.GTAP_KIND_KCLIQUE, gtap.gtap_kclique_args(rp.data_ptr(), col.data_ptr(), g.n, 4, 64,
                                                                  g.max_outdeg)),
                (gtap.GTAP_KIND_KCLIQUE, gtap.gtap_kclique_args(rp.data_ptr(), col.data_ptr(), g.n, 5, 64,
                                                                  g.max_outdeg))] + \
            [rt.fib_args(k) for k in range(0, 24)]
    return [rt.fib_args(15), rt.uts_args(3, thr, 6),
            (gtap.GTAP_KIND_KCLIQUE, gtap.gtap_kclique_args(rp.data_ptr(), col.data_ptr(), g.n, 3, 64,
                                                              g.max_outdeg))]


def allocating_path(gtap, ents):
    with gtap.Runtime(**SMALL) as rt:
        ids = [gtap.gtap_submit(rt.ctx, kind, a) for kind, a in ents]
        rt.run()
        return [rt.result(j) for j in ids]


def test_static_matches_allocating_path_twice(gtap, graph):
    import torch
    cfg = config(gtap)
    for big in (True, False):
        ents = entries(gtap, graph, big)
        jobs = gtap.Runtime.trace([(0.0, e) for e in ents])
        say(f"gtap_run_static: {len(ents)} jobs ({'larger' if big else 'smaller'} batch)")
        got = gtap.gtap_run_static(cfg, jobs)
        torch.cuda.synchronize()
        say("  allocating path on the same jobs")
        want = allocating_path(gtap, ents)
        assert got == want, (big, got, want)
    g = graph[0]
    assert got[2] == oracle.kclique(g.row_ptr, g.col, 3).value


def test_static_rejects_what_does_not_fit(gtap, graph):
    jobs = gtap.Runtime.trace([(0.0, gtap.Runtime.fib_args(10))])
    with pytest.raises(gtap.GtapError) as e:
        gtap.gtap_run_static(config(gtap, small_frames=1 << 24), jobs)  # 1 GiB of frames
    assert e.value.code == gtap.GTAP_E_NOMEM
    fmm_like = gtap.Runtime.trace([(0.0, gtap.Runtime.fib_args(10))])
    fmm_like[0].kind = gtap.GTAP_KIND_CILKSORT
    with pytest.raises(gtap.GtapError) as e:
        gtap.gtap_run_static(config(gtap), fmm_like)
    assert e.value.code == gtap.GTAP_E_INVAL
    assert gtap.gtap_run_static(config(gtap), gtap.Runtime.trace([])) == []
