"""GPU parity of the list-building FMM pipeline (the paper's FMM evaluation):
the dual-tree traversal only appends pairs to an M2L and a P2P list -- run as
thread-mode tasks of the runtime or as the level-synchronous worklist -- and
data-parallel kernels evaluate the sorted lists.

Checked against the CPU FMM oracle like the block-mode traversal: identical
lists (counts and order-independent hashes), equal P2P interaction and
coincident counts, potentials within 1e-12 relative (L2 and max norm; the two
sides differ only in the order of floating-point additions).
"""
import os
import sys

import numpy as np
import pytest

import oracle
from synth import points

pytestmark = pytest.mark.gpu

RTOL = 1e-12


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gtap():
    from paper_2604_05982_amd import gtap as mod
    return mod


def traversals(g):
    return {"lists": g.GTAP_FMM_LISTS, "worklist": g.GTAP_FMM_WORKLIST}


def run_fmm(gtap, x, y, z, q, traversal, theta=(1, 2), leaf_max=64, extra=None, **caps):
    import torch
    rt = gtap.Runtime(mode=gtap.GTAP_MODE_THREAD, waves_per_group=4, small_frames=1 << 24, big_frames=1 << 10,
                      timeout_ms=60000)
    try:
        tx, ty, tz, tq = (torch.as_tensor(np.asarray(a, dtype=np.float64)).cuda() for a in (x, y, z, q))
        phi = torch.zeros_like(tx)
        j = rt.submit_fmm(tx, ty, tz, tq, phi, leaf_max=leaf_max, theta=theta, traversal=traversal, **caps)
        others = [(rt.submit_fib(n), oracle.fib(n).value) for n in (extra or [])]
        rt.run()
        res = rt.fmm_result(j)
        for jid, want in others:
            assert rt.result(jid) == want
        return phi.cpu().numpy(), res
    finally:
        rt.close()


def check_lists(res, want):
    for k in ("n_cells", "n_leaves", "max_level", "m2l_pairs", "p2p_pairs", "m2l_hash", "p2p_hash"):
        assert res[k] == want.stats[k], (k, res[k], want.stats[k])


def check_phi(got, want):
    err = got - want
    assert np.linalg.norm(err) <= RTOL * np.linalg.norm(want), np.linalg.norm(err) / np.linalg.norm(want)
    assert np.abs(err).max() <= RTOL * np.abs(want).max(), np.abs(err).max() / np.abs(want).max()


@pytest.mark.parametrize("name", ["lists", "worklist"])
@pytest.mark.parametrize("n,seed", [(2000, 3), (20000, 5)])
def test_fmm_lists_plummer_matches_oracle(gtap, name, n, seed):
    x, y, z, q = points.plummer(n, seed)
    say(f"fmm {name} plummer n={n}")
    got, res = run_fmm(gtap, x, y, z, q, traversals(gtap)[name])
    want = oracle.fmm(x, y, z, q)
    check_lists(res, want)
    assert res["p2p_interactions"] == want.stats["p2p_interactions"]
    assert res["coincident"] == want.stats["coincident"]
    check_phi(got, want.phi)
    if name == "worklist":
        assert res["dtt_rounds"] >= res["max_level"]


@pytest.mark.parametrize("name", ["lists", "worklist"])
def test_fmm_lists_uniform_thetas(gtap, name):
    x, y, z, q = points.uniform_cube(30000, 11, half=50.0)
    for theta in ((1, 2), (1, 3), (2, 3)):
        say(f"fmm {name} uniform theta={theta}")
        got, res = run_fmm(gtap, x, y, z, q, traversals(gtap)[name], theta=theta, leaf_max=32)
        want = oracle.fmm(x, y, z, q, theta=theta, leaf_max=32)
        check_lists(res, want)
        check_phi(got, want.phi)


@pytest.mark.parametrize("name", ["lists", "worklist"])
def test_fmm_lists_degenerate_cases(gtap, name):
    tr = traversals(gtap)[name]
    say(f"fmm {name}: n=1")
    one = [np.array([v], dtype=np.float64) for v in (0.5, 0.25, -3.0, 0.7)]
    got, res = run_fmm(gtap, *one, tr)
    assert got.tolist() == [0.0] and res["n_cells"] == 1 and res["p2p_pairs"] == 1
    x, y, z, q = points.plummer(60, 4)
    say(f"fmm {name}: one leaf")
    got, res = run_fmm(gtap, x, y, z, q, tr)
    d = oracle.direct(x, y, z, q, np.arange(60))
    assert res["m2l_pairs"] == 0
    assert np.abs(got - d).max() <= 1e-13 * np.abs(d).max()
    x, y, z, q = points.plummer(3000, 6)
    say(f"fmm {name}: theta 0")
    got, res = run_fmm(gtap, x, y, z, q, tr, theta=(0, 1))
    d = oracle.direct(x, y, z, q, np.arange(3000))
    assert res["m2l_pairs"] == 0 and res["p2p_interactions"] == 3000 * 2999
    assert np.abs(got - d).max() <= 1e-13 * np.abs(d).max()
    x, y, z, q = points.plummer(5000, 7)
    x, y, z, q = (np.concatenate([a, a[:40]]) for a in (x, y, z, q))
    say(f"fmm {name}: coincident points, leaf 17")
    got, res = run_fmm(gtap, x, y, z, q, tr, leaf_max=17)
    want = oracle.fmm(x, y, z, q, leaf_max=17)
    check_lists(res, want)
    assert res["coincident"] == want.stats["coincident"] == 80
    check_phi(got, want.phi)


@pytest.mark.parametrize("name", ["lists", "worklist"])
def test_fmm_lists_overflow_is_retried(gtap, name):
    """Lists far smaller than needed: the traversal counts past the capacity,
    the library re-runs it once with lists that fit, results are unchanged."""
    x, y, z, q = points.plummer(20000, 8)
    say(f"fmm {name}: tiny list capacities")
    got, res = run_fmm(gtap, x, y, z, q, traversals(gtap)[name], m2l_capacity=1000, p2p_capacity=500,
                       extra=[10, 17])
    want = oracle.fmm(x, y, z, q)
    assert res["list_retries"] >= 1
    check_lists(res, want)
    check_phi(got, want.phi)


def test_fmm_traversal_mode_rules(gtap):
    import torch
    x = torch.zeros(4, dtype=torch.float64, device="cuda")
    say("fmm traversal / mode rules")
    for mode, wpg, tr in ((gtap.GTAP_MODE_THREAD, 4, gtap.GTAP_FMM_TASKS),
                          (gtap.GTAP_MODE_BLOCK, 1, gtap.GTAP_FMM_LISTS),
                          (gtap.GTAP_MODE_BLOCK, 1, gtap.GTAP_FMM_WORKLIST),
                          (gtap.GTAP_MODE_THREAD, 2, gtap.GTAP_FMM_LISTS)):
        rt = gtap.Runtime(mode=mode, waves_per_group=wpg, small_frames=1 << 16, big_frames=0)
        try:
            with pytest.raises(gtap.GtapError) as e:
                rt.submit_fmm(x, x, x, x, torch.zeros_like(x), traversal=tr)
            assert e.value.code == gtap.GTAP_E_INVAL
        finally:
            rt.close()


def test_fmm_lists_plummer_1m_sampled(gtap):
    """10^6 Plummer points, leaf 64, theta 1/2, order 6, thread-mode list
    traversal: lists against the oracle's (stored with the golden sample),
    potentials at 4,096 sampled targets against the oracle FMM (1e-12) and
    fp64 direct summation (truncation error of the expansion)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "fmm_plummer_1m.txt")
    lists = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("# lists:"):
                f = line.split()[2:]
                lists = {f[i]: int(f[i + 1]) for i in range(0, len(f), 2)}
    gold = np.loadtxt(path)
    tg, direct, fmm_oracle = gold[:, 0].astype(np.int64), gold[:, 1], gold[:, 2]
    x, y, z, q = points.plummer(1000000, 3)
    say("fmm lists plummer 1M on the GPU")
    got, res = run_fmm(gtap, x, y, z, q, gtap.GTAP_FMM_LISTS)
    say(f"  gpu: {res}")
    for k, v in lists.items():
        assert res[k] == v, (k, res[k], v)
    check_phi(got[tg], fmm_oracle)
    err = got[tg] - direct
    assert np.linalg.norm(err) / np.linalg.norm(direct) < 1e-4


def test_fmm_lists_several_jobs_in_one_launch(gtap):
    """Three list-building FMM jobs (two task traversals, whose wavefronts
    switch chunk owners between descriptors, and one worklist), a Cilksort job
    and fib jobs share one launch; each FMM job's lists and potentials match
    its own oracle run."""
    import torch
    rt = gtap.Runtime(mode=gtap.GTAP_MODE_THREAD, waves_per_group=4, small_frames=1 << 24, big_frames=1 << 10,
                      timeout_ms=60000)
    try:
        jobs = []
        for seed, n, tr in ((21, 8000, gtap.GTAP_FMM_LISTS), (22, 12000, gtap.GTAP_FMM_LISTS),
                            (23, 5000, gtap.GTAP_FMM_WORKLIST)):
            x, y, z, q = points.plummer(n, seed)
            ts = [torch.as_tensor(np.asarray(a, dtype=np.float64)).cuda() for a in (x, y, z, q)]
            phi = torch.zeros_like(ts[0])
            jid = rt.submit_fmm(*ts, phi, traversal=tr)
            jobs.append((jid, (x, y, z, q), ts, phi))
        keys = np.random.default_rng(2).integers(0, 2**32, size=30000, dtype=np.uint32)
        kt = torch.from_numpy(keys.view(np.int32)).cuda()
        js = rt.submit_cilksort(kt)
        fibs = [(rt.submit_fib(n), oracle.fib(n).value) for n in (12, 21)]
        say("three FMM jobs, a Cilksort job and fib jobs in one launch")
        rt.run()
        for jid, (x, y, z, q), _, phi in jobs:
            res = rt.fmm_result(jid)
            want = oracle.fmm(x, y, z, q)
            check_lists(res, want)
            check_phi(phi.cpu().numpy(), want.phi)
        assert np.array_equal(kt.cpu().numpy().view(np.uint32), np.sort(keys)) and rt.result(js) == keys.size
        for j, v in fibs:
            assert rt.result(j) == v
    finally:
        rt.close()
