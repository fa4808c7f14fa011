"""GPU parity of block mode: one task per workgroup with Chase-Lev deques.

Integer workloads (fib, UTS) are checked bit-exactly, task and continuation
counts included.  The FMM job is checked against the CPU FMM oracle: the M2L
and P2P pair lists must be identical (counts and order-independent hashes),
the P2P interaction and coincident-point counts equal, and the potentials
within 1e-12 relative: ||dphi||_2 <= 1e-12 ||phi||_2 and
max |dphi_i| <= 1e-12 max |phi_i| (the two sides differ only in the order of
floating-point additions).
"""
import sys

import numpy as np
import pytest

import oracle
from synth import points

pytestmark = pytest.mark.gpu

THR4 = oracle.uts_threshold(4)
RTOL = 1e-12


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gtap():
    from paper_2604_05982_amd import gtap as mod
    return mod


def make_rt(gtap, **kw):
    kw.setdefault("mode", gtap.GTAP_MODE_BLOCK)
    kw.setdefault("waves_per_group", 1)
    kw.setdefault("timeout_ms", 60000)
    kw.setdefault("small_frames", 1 << 22)
    kw.setdefault("big_frames", 0)
    return gtap.Runtime(**kw)


@pytest.mark.parametrize("wpg", [1, 2, 4])
def test_block_fib(gtap, wpg):
    rt = make_rt(gtap, waves_per_group=wpg)
    try:
        for n in (0, 1, 2, 7, 18):
            say(f"block fib({n}) wpg={wpg}")
            j = rt.submit_fib(n)
            rt.run()
            want = oracle.fib(n)
            st = rt.stats()
            assert rt.result(j) == want.value
            assert (st["tasks"], st["conts"]) == (want.tasks, want.conts)
    finally:
        rt.close()


def test_block_uts_and_mixed_batch(gtap):
    rt = make_rt(gtap, waves_per_group=2)
    try:
        say("block uts(1, 4, 6)")
        j = rt.submit_uts(1, THR4, 6)
        rt.run()
        want = oracle.uts(1, THR4, 6)
        st = rt.stats()
        assert rt.result(j) == want.value
        assert (st["tasks"], st["conts"]) == (want.tasks, want.conts)
        say("block mixed batch of 300 jobs")
        rng = np.random.default_rng(3)
        jobs, wants = [], []
        for i in range(300):
            if i % 2:
                s, d = int(rng.integers(1, 2**62)), int(rng.integers(0, 7))
                jobs.append(rt.submit_uts(s, THR4, d))
                wants.append(oracle.uts(s, THR4, d).value)
            else:
                n = int(rng.integers(0, 16))
                jobs.append(rt.submit_fib(n))
                wants.append(oracle.fib(n).value)
        rt.run()
        assert [rt.result(j) for j in jobs] == wants
    finally:
        rt.close()


def test_block_mode_rejects_thread_only_kinds(gtap):
    rt = make_rt(gtap)
    try:
        with pytest.raises(gtap.GtapError) as e:
            rt.submit_nqueens(8)
        assert e.value.code == gtap.GTAP_E_INVAL
    finally:
        rt.close()


# ---- FMM ------------------------------------------------------------------------
def _run_fmm(gtap, x, y, z, q, theta=(1, 2), leaf_max=64, wpg=1):
    import torch
    rt = make_rt(gtap, waves_per_group=wpg, small_frames=1 << 24)
    try:
        tx, ty, tz, tq = (torch.as_tensor(a).cuda() for a in (x, y, z, q))
        phi = torch.zeros_like(tx)
        j = rt.submit_fmm(tx, ty, tz, tq, phi, leaf_max=leaf_max, theta=theta)
        rt.run()
        res = rt.fmm_result(j)
        st = rt.stats()
        return phi.cpu().numpy(), res, st
    finally:
        rt.close()


def _check_lists(res, want):
    for k in ("n_cells", "n_leaves", "max_level", "m2l_pairs", "p2p_pairs", "m2l_hash", "p2p_hash"):
        assert res[k] == want.stats[k], (k, res[k], want.stats[k])


def _check_phi(got, want):
    err = got - want
    assert np.linalg.norm(err) <= RTOL * np.linalg.norm(want), np.linalg.norm(err) / np.linalg.norm(want)
    assert np.abs(err).max() <= RTOL * np.abs(want).max(), np.abs(err).max() / np.abs(want).max()


@pytest.mark.parametrize("n,seed,wpg", [(2000, 3, 1), (20000, 5, 1), (20000, 5, 4)])
def test_fmm_plummer_matches_oracle(gtap, n, seed, wpg):
    x, y, z, q = points.plummer(n, seed)
    say(f"fmm plummer n={n} wpg={wpg}")
    got, res, st = _run_fmm(gtap, x, y, z, q, wpg=wpg)
    want = oracle.fmm(x, y, z, q)
    _check_lists(res, want)
    assert res["p2p_interactions"] == want.stats["p2p_interactions"]
    assert res["coincident"] == want.stats["coincident"]
    _check_phi(got, want.phi)


def test_fmm_uniform_and_other_theta(gtap):
    x, y, z, q = points.uniform_cube(30000, 11, half=50.0)
    for theta in ((1, 2), (1, 3), (2, 3)):
        say(f"fmm uniform theta={theta}")
        got, res, _ = _run_fmm(gtap, x, y, z, q, theta=theta, leaf_max=32)
        want = oracle.fmm(x, y, z, q, theta=theta, leaf_max=32)
        _check_lists(res, want)
        _check_phi(got, want.phi)


def test_fmm_degenerate_cases(gtap):
    # one point: no interactions
    say("fmm n=1")
    one = [np.array([v], dtype=np.float64) for v in (0.5, 0.25, -3.0, 0.7)]
    got, res, _ = _run_fmm(gtap, *one)
    assert got.tolist() == [0.0] and res["n_cells"] == 1 and res["p2p_pairs"] == 1
    # a single leaf: direct summation
    x, y, z, q = points.plummer(60, 4)
    say("fmm one leaf")
    got, res, _ = _run_fmm(gtap, x, y, z, q)
    d = oracle.direct(x, y, z, q, np.arange(60))
    assert res["m2l_pairs"] == 0
    assert np.abs(got - d).max() <= 1e-13 * np.abs(d).max()
    # theta = 0: every pair of leaves by P2P
    x, y, z, q = points.plummer(3000, 6)
    say("fmm theta 0")
    got, res, _ = _run_fmm(gtap, x, y, z, q, theta=(0, 1))
    d = oracle.direct(x, y, z, q, np.arange(3000))
    assert res["m2l_pairs"] == 0 and res["p2p_interactions"] == 3000 * 2999
    assert np.abs(got - d).max() <= 1e-13 * np.abs(d).max()
    # coincident points and a ragged leaf size
    x, y, z, q = points.plummer(5000, 7)
    x, y, z, q = (np.concatenate([a, a[:40]]) for a in (x, y, z, q))
    say("fmm coincident points, leaf 17")
    got, res, _ = _run_fmm(gtap, x, y, z, q, leaf_max=17)
    want = oracle.fmm(x, y, z, q, leaf_max=17)
    _check_lists(res, want)
    assert res["coincident"] == want.stats["coincident"] == 80
    _check_phi(got, want.phi)


def test_fmm_rejects_points_outside_root_cube(gtap):
    import torch
    rt = make_rt(gtap)
    try:
        x = torch.tensor([0.0, 200.0], dtype=torch.float64, device="cuda")
        phi = torch.zeros_like(x)
        rt.submit_fmm(x, x * 0, x * 0, x * 0 + 1, phi)
        with pytest.raises(gtap.GtapError) as e:
            rt.run()
        assert e.value.code == gtap.GTAP_E_INVAL
    finally:
        rt.close()


def test_fmm_plummer_1m_sampled(gtap):
    """The full-size configuration: 10^6 Plummer points, leaf 64, theta 1/2,
    order 6.  Lists against the oracle's (stored with the golden sample); the
    potentials at 4,096 sampled targets against the oracle FMM (1e-12) and
    against fp64 direct summation (truncation error of the expansion)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "fmm_plummer_1m.txt")
    lists = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("# lists:"):
                f = line.split()[2:]
                lists = {f[i]: int(f[i + 1]) for i in range(0, len(f), 2)}
    gold = np.loadtxt(path)
    tg, direct, fmm_oracle = gold[:, 0].astype(np.int64), gold[:, 1], gold[:, 2]
    n = 1000000
    x, y, z, q = points.plummer(n, 3)
    say("fmm plummer 1M on the GPU")
    got, res, st = _run_fmm(gtap, x, y, z, q, wpg=1)
    say(f"  gpu: {res}")
    for k, v in lists.items():
        assert res[k] == v, (k, res[k], v)
    _check_phi(got[tg], fmm_oracle)
    err = got[tg] - direct
    assert np.linalg.norm(err) / np.linalg.norm(direct) < 1e-4
    assert np.abs(err).max() < 2e-4 * np.abs(direct).max()


def test_fmm_plummer_1m_every_target_block_vs_lists(gtap):
    """Every one of the 10^6 potentials: the block-mode traversal (work inside
    the tasks, fp64 atomics into the targets) against the list pipeline
    (thread-mode list-building traversal, lists sorted by target, one owner per
    target: no atomics), two independent GPU evaluations of the same pairs,
    within 1e-12 relative; both are tied to the oracle by the 4,096-target
    sample of test_fmm_plummer_1m_sampled and the list hashes."""
    import torch
    n = 1000000
    x, y, z, q = points.plummer(n, 3)
    say("fmm plummer 1M: block mode, every target")
    got_block, res_b, _ = _run_fmm(gtap, x, y, z, q, wpg=2)
    say("fmm plummer 1M: list pipeline, every target")
    rt = gtap.Runtime(mode=gtap.GTAP_MODE_THREAD, waves_per_group=4, small_frames=1 << 24, big_frames=1 << 10,
                      timeout_ms=120000)
    try:
        tx, ty, tz, tq = (torch.as_tensor(a).cuda() for a in (x, y, z, q))
        phi = torch.zeros_like(tx)
        j = rt.submit_fmm(tx, ty, tz, tq, phi, traversal=gtap.GTAP_FMM_LISTS)
        rt.run()
        res_l = rt.fmm_result(j)
        got_lists = phi.cpu().numpy()
    finally:
        rt.close()
    for k in ("m2l_pairs", "p2p_pairs", "m2l_hash", "p2p_hash", "p2p_interactions", "coincident"):
        assert res_b[k] == res_l[k], (k, res_b[k], res_l[k])
    assert np.isfinite(got_block).all() and np.isfinite(got_lists).all()
    _check_phi(got_block, got_lists)
