"""GPU parity of Cilksort (Sec. 6.3) in thread mode against the CPU oracle:
the sorted keys bit-exactly, and the task and continuation counts of the
recursion (which depend on the keys but not on the schedule) exactly; with
and without the three DAQ queues of the paper (recursive, serial sort, serial
merge).  At 2^24 keys: sortedness, the key sum and equality with numpy's
sort of the input."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gtap():
    from paper_2604_05982_amd import gtap as mod
    return mod


def make_rt(gtap, **kw):
    kw.setdefault("timeout_ms", 60000)
    kw.setdefault("small_frames", 1 << 23)
    kw.setdefault("big_frames", 1 << 10)
    return gtap.Runtime(**kw)


def gpu_sort(rt, keys, sc=64, mc=256):
    import torch
    t = torch.from_numpy(keys.view(np.int32)).cuda()
    jid = rt.submit_cilksort(t, sort_cutoff=sc, merge_cutoff=mc)
    rt.run()
    return t.cpu().numpy().view(np.uint32), rt.result(jid), rt.stats()


def cases():
    rng = np.random.default_rng(9)
    yield "random 100003", rng.integers(0, 2**32, size=100003, dtype=np.uint32)
    yield "random 1000", rng.integers(0, 2**32, size=1000, dtype=np.uint32)
    yield "few distinct", rng.integers(0, 4, size=30011, dtype=np.uint32)
    yield "all equal", np.full(4097, 7, dtype=np.uint32)
    yield "sorted", np.arange(20000, dtype=np.uint32)
    yield "reversed", np.arange(20000, dtype=np.uint32)[::-1].copy()
    for n in (0, 1, 2, 63, 64, 65, 257):
        yield f"n={n}", rng.integers(0, 2**32, size=n, dtype=np.uint32)


@pytest.mark.parametrize("cut", [(64, 256), (16, 64), (1, 2)])
def test_cilksort_matches_oracle(gtap, cut):
    with make_rt(gtap) as rt:
        for name, keys in cases():
            if cut == (1, 2) and keys.size > 5000:
                continue
            say(f"cilksort {name} cutoffs {cut}")
            got, res, st = gpu_sort(rt, keys, *cut)
            want, w = oracle.cilksort(keys, *cut)
            assert np.array_equal(got, want), name
            assert res == keys.size
            assert (st["tasks"], st["conts"]) == (w.tasks, w.conts), (name, st["tasks"], st["conts"], w)


def test_cilksort_daq_three_queues(gtap):
    keys = np.random.default_rng(4).integers(0, 2**32, size=200003, dtype=np.uint32)
    want, w = oracle.cilksort(keys)
    say("cilksort with DAQ, 3 queues")
    with make_rt(gtap, num_queues=3, daq_policy=gtap.GTAP_DAQ_CILKSORT, deque_capacity=1 << 18) as rt:
        got, res, st = gpu_sort(rt, keys)
        assert np.array_equal(got, want)
        assert (st["tasks"], st["conts"]) == (w.tasks, w.conts)


def test_cilksort_in_a_mixed_batch(gtap):
    import torch
    rng = np.random.default_rng(12)
    say("cilksort jobs mixed with fib jobs in one launch")
    with make_rt(gtap) as rt:
        arrays, jobs = [], []
        for i in range(6):
            keys = rng.integers(0, 2**32, size=int(rng.integers(0, 50000)), dtype=np.uint32)
            t = torch.from_numpy(keys.view(np.int32)).cuda()
            arrays.append((keys, t))
            jobs.append(rt.submit_cilksort(t))
        fibs = [(rt.submit_fib(n), oracle.fib(n).value) for n in (5, 20, 25)]
        rt.run()
        for (keys, t), j in zip(arrays, jobs):
            assert np.array_equal(t.cpu().numpy().view(np.uint32), np.sort(keys))
            assert rt.result(j) == keys.size
        for j, v in fibs:
            assert rt.result(j) == v


def test_cilksort_2p24_sampled(gtap):
    import torch
    n = 1 << 24
    say(f"cilksort {n} keys on the GPU")
    g = torch.Generator(device="cuda").manual_seed(5)
    x = torch.randint(-2**31, 2**31, (n,), dtype=torch.int64, device="cuda", generator=g).to(torch.int32)
    u = x.to(torch.int64) & 0xFFFFFFFF
    s_in = int(u.sum())
    with make_rt(gtap, small_frames=1 << 24) as rt:
        jid = rt.submit_cilksort(x)
        rt.run()
        assert rt.result(jid) == n
    v = x.to(torch.int64) & 0xFFFFFFFF
    assert bool((v[1:] >= v[:-1]).all())
    assert int(v.sum()) == s_in
    a = np.sort(u.cpu().numpy())
    assert np.array_equal(v.cpu().numpy(), a)


def test_cilksort_rejected_configs(gtap):
    import torch
    say("cilksort configuration checks")
    t = torch.zeros(10, dtype=torch.int32, device="cuda")
    for kw, args in ((dict(mode=gtap.GTAP_MODE_BLOCK, waves_per_group=1, big_frames=0), {}),
                     (dict(waves_per_group=2), {}),
                     ({}, dict(sort_cutoff=65)),
                     ({}, dict(merge_cutoff=1))):
        rt = make_rt(gtap, **kw)
        try:
            with pytest.raises(gtap.GtapError) as e:
                rt.submit_cilksort(t, **args)
            assert e.value.code == gtap.GTAP_E_INVAL
        finally:
            rt.close()
