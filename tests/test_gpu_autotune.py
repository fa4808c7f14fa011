"""GPU check of the configuration autotuner: it explores the candidate space on
calibration jobs and returns a configuration under which the same jobs still
give the oracle's results."""
import numpy as np
import pytest

import oracle
from synth import graphs

pytestmark = pytest.mark.gpu


def test_autotune_returns_a_working_configuration():
    import torch
    from paper_2604_05982_amd import gtap
    g = graphs.chung_lu(2000, 16, 2.5, 1.0, 1)
    rp = torch.as_tensor(g.row_ptr32).cuda()
    col = torch.as_tensor(g.col).cuda()
    rt = gtap.Runtime(timeout_ms=60000, small_frames=1 << 22, big_frames=1 << 18, big_frame_ints=512)
    try:
        thr = oracle.uts_threshold(3)
        entries, want = [], []
        rng = np.random.default_rng(21)
        for i in range(120):
            if i % 3 == 0:
                entries.append((0.0, rt.fib_args(18)))
                want.append(oracle.fib(18).value)
            elif i % 3 == 1:
                s = int(rng.integers(1, 2**62))
                entries.append((0.0, rt.uts_args(s, thr, 7)))
                want.append(oracle.uts(s, thr, 7).value)
            else:
                entries.append((0.0, rt.kclique_args(rp, col, 4, max_outdeg=g.max_outdeg)))
                want.append(oracle.kclique(g.row_ptr, g.col, 4).value)
        jobs = rt.trace(entries)
        space = gtap.tune_space(num_queues=(1, 2), waves_per_group=(2, 4), num_waves=(512, 0),
                                daq_policy=gtap.GTAP_DAQ_BY_KIND, repeats=1)
        best, rep = rt.autotune(jobs, space)
        print(best, rep, flush=True)
        assert rep["candidates"] == 9 and rep["failed"] == 0
        assert rep["best_ms"] <= rep["base_ms"]
        assert best["num_queues"] in (1, 2) and best["waves_per_group"] in (2, 4)
        assert best["small_frames"] >= 1 << 20
        tuned = gtap.Runtime(timeout_ms=60000, big_frame_ints=512, **best)
        try:
            res = tuned.trace_run_plain(jobs)
            assert [r.result for r in res] == want
            ids = [gtap.gtap_submit(tuned.ctx, k.kind, _args(gtap, k)) for k in jobs]
            tuned.run()
            assert [tuned.result(j) for j in ids] == want
        finally:
            tuned.close()
    finally:
        rt.close()


def _args(gtap, job):
    """The argument struct stored in a gtap_trace_job."""
    import ctypes
    cls = {gtap.GTAP_KIND_FIB: gtap.gtap_fib_args, gtap.GTAP_KIND_UTS: gtap.gtap_uts_args,
           gtap.GTAP_KIND_KCLIQUE: gtap.gtap_kclique_args}[job.kind]
    a = cls()
    ctypes.memmove(ctypes.addressof(a), ctypes.addressof(job.args), ctypes.sizeof(a))
    return a
