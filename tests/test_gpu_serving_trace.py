"""GPU parity of the batched-serving job mix at its real sizes.

The trace is synth.serving.serving_mix(20000, 5): k-clique jobs (k 4..8) on
induced subgraphs of up to 2e5 vertices of the seeded n=10^6 Chung-Lu graph
and unbalanced tree search jobs (m 2..4, depth 8..14).  The oracle's result
for every job is stored in tests/golden/serving_trace_s5.txt (written by
tests/golden/make_serving_golden.py from oracle/ and synth/ only).

A slice of the trace -- the largest k=8 subgraphs, the largest trees, the
k-clique jobs with the most cliques, and a seeded sample of the rest -- runs
three ways: in one batched launch, served through the admission ring while
the kernel runs (staggered arrivals, so jobs join a running mix), and alone
(one launch per job).  Every result must equal the stored oracle result.
"""
import os
import sys

import numpy as np
import pytest

from synth import graphs, serving

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "serving_trace_s5.txt")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def load_golden():
    out = []
    with open(GOLDEN) as fh:
        head = fh.readline()
        for line in fh:
            if not line.startswith("#"):
                f = line.split()
                out.append((f[1], int(f[2]), int(f[3])))
    return head, out


@pytest.fixture(scope="module")
def gtap():
    from paper_2604_05982_amd import gtap as mod
    return mod


@pytest.fixture(scope="module")
def trace_slice(gtap):
    import torch
    head, gold = load_golden()
    specs = serving.serving_mix(20000, 5)
    g = graphs.chung_lu(1000000, 40, 2.1, 0.6, 2)
    assert g.checksum() in head, "the stored results were written for another graph"
    assert len(gold) == len(specs)
    for sp, (kind, par, _) in zip(specs, gold):
        assert sp.kind == kind and par == (sp.k if kind == "kclique" else sp.depth)
    kc = [i for i, sp in enumerate(specs) if sp.kind == "kclique"]
    ut = [i for i, sp in enumerate(specs) if sp.kind == "uts"]
    pick = set(sorted((i for i in kc if specs[i].k == 8), key=lambda i: -specs[i].s)[:6])
    pick |= set(sorted(ut, key=lambda i: -(specs[i].m ** specs[i].depth))[:6])
    pick |= set(sorted(kc, key=lambda i: -gold[i][2])[:8])
    rest = sorted(set(range(len(specs))) - pick)
    pick |= set(int(i) for i in np.random.default_rng(9).choice(rest, 240, replace=False))
    idx = sorted(pick)
    kci = [i for i in idx if specs[i].kind == "kclique"]
    subs = graphs.induced_many(g, [(specs[i].s, specs[i].sub_seed) for i in kci], threads=8)
    rp_off = np.cumsum([0] + [h.n + 1 for h in subs])
    col_off = np.cumsum([0] + [h.col.size for h in subs])
    rp = torch.as_tensor(np.concatenate([h.row_ptr.astype(np.int32) for h in subs])).cuda()
    col = torch.as_tensor(np.concatenate([h.col for h in subs] + [np.zeros(1, np.int32)])).cuda()
    entries, want, it = [], [], 0
    for i in idx:
        sp = specs[i]
        if sp.kind == "kclique":
            h = subs[it]
            a = gtap.gtap_kclique_args(rp.data_ptr() + 4 * int(rp_off[it]), col.data_ptr() + 4 * int(col_off[it]),
                                       h.n, sp.k, 64, h.max_outdeg)
            entries.append((gtap.GTAP_KIND_KCLIQUE, a))
            it += 1
        else:
            entries.append(gtap.Runtime.uts_args(sp.seed, gtap.uts_threshold(sp.m), sp.depth))
        want.append(gold[i][2])
    big_k8 = max(specs[i].s for i in kci if specs[i].k == 8)
    deepest = max(specs[i].m ** specs[i].depth for i in idx if specs[i].kind == "uts")
    say(f"slice: {len(idx)} jobs ({len(kci)} k-clique, largest k=8 subgraph {big_k8} vertices, "
        f"largest tree bound m^D = {deepest:.3g}, {sum(want)} total result)")
    yield g, idx, entries, want, (rp, col)


def make_rt(gtap, g):
    return gtap.Runtime(timeout_ms=100000, small_frames=1 << 26, big_frames=1 << 22,
                        big_frame_ints=max(320, g.max_outdeg), deque_capacity=1 << 18, max_jobs=1 << 12)


def test_trace_slice_batched(gtap, trace_slice):
    """All jobs of the slice in one persistent launch."""
    g, idx, entries, want, _ = trace_slice
    with make_rt(gtap, g) as rt:
        ids = [gtap.gtap_submit(rt.ctx, kind, a) for kind, a in entries]
        say(f"batched launch of {len(ids)} trace jobs")
        rt.run()
        got = [rt.result(j) for j in ids]
        say(f"  {rt.stats()['tasks']} tasks, kernel {rt.stats()['kernel_ms']:.1f} ms")
    bad = [(idx[k], got[k], want[k]) for k in range(len(want)) if got[k] != want[k]]
    assert not bad, f"{len(bad)} jobs differ from the oracle (trace index, gpu, oracle): {bad[:5]}"


def test_trace_slice_served_and_alone(gtap, trace_slice):
    """The slice served into a running kernel (arrivals 0.2 ms apart, so
    later jobs join a running mix), then each job alone."""
    g, idx, entries, want, _ = trace_slice
    with make_rt(gtap, g) as rt:
        jobs = rt.trace([(2e-4 * k, e) for k, e in enumerate(entries)])
        say(f"serving {len(entries)} trace jobs through the admission ring")
        rt.serve_start(max_inflight=512, headroom_small=1 << 22)
        res = rt.trace_run(jobs, timeout_ms=100000)
        rt.serve_stop()
        served = [r.result for r in res]
        assert all(r.status == 0 for r in res)
        say(f"  served in {max(r.done_s for r in res):.2f} s; now one launch per job")
        alone = [r.result for r in rt.trace_run_plain(rt.trace([(0.0, e) for e in entries]))]
    for name, got in (("served", served), ("alone", alone)):
        bad = [(idx[k], got[k], want[k]) for k in range(len(want)) if got[k] != want[k]]
        assert not bad, f"{name}: {len(bad)} jobs differ from the oracle (trace index, gpu, oracle): {bad[:5]}"
