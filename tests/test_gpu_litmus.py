"""Litmus tests and the atomic-rate probe on the GPU (platform evidence for
the runtime's ordering discipline, Sec. 5.1.3).

The runtime hands data between wavefronts with relaxed device-scope stores and
loads and orders them by waiting for completion (drain()) instead of
release/acquire fences.  Between workgroups on different XCDs:
  - message passing with the wait: a reader that sees the flag never sees
    older data;
  - store buffering with the wait: the two loads never both miss the other
    side's store.
The runs without the wait are reported, not asserted: they show how often
the hardware would reorder.  Every kernel runs a fixed number of iterations
and no wait depends on the other workgroup.
"""
import sys

import pytest

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gtap():
    from paper_2604_05982_amd import gtap as mod
    return mod


def buffer(torch, pairs, rounds):
    nbytes = pairs * (16384 + 512 * rounds) + 16384
    return torch.zeros(nbytes, dtype=torch.uint8, device="cuda"), nbytes


def test_message_passing(gtap):
    import torch
    pairs, rounds = 64, 4096
    buf, nb = buffer(torch, pairs, rounds)
    for ordered in (True, False):
        say(f"litmus message passing, ordered={ordered}, {pairs} workgroup pairs x 64 lanes, {rounds} rounds")
        r = gtap.gtap_litmus(0, ordered, pairs, rounds, buf.data_ptr(), nb,
                             torch.cuda.current_stream().cuda_stream)
        say(f"  {r}")
        assert r["instances"] == pairs * 64 and r["mp_reads"] == pairs * 64 * 4 * rounds
        if ordered:
            assert r["mp_stale"] == 0, r
            assert r["mp_overlap"] > 0, "reader and writer never overlapped: the test exercised nothing"
            assert r["pairs_on_distinct_xcds"] >= pairs // 2, r


def test_store_buffering(gtap):
    import torch
    pairs, rounds = 64, 2048
    buf, nb = buffer(torch, pairs, rounds)
    for ordered in (True, False):
        say(f"litmus store buffering, ordered={ordered}, {pairs} workgroup pairs x 64 lanes, {rounds} rounds")
        r = gtap.gtap_litmus(1, ordered, pairs, rounds, buf.data_ptr(), nb,
                             torch.cuda.current_stream().cuda_stream)
        say(f"  {r}")
        assert r["sb_rounds"] == pairs * 64 * rounds
        assert r["sb_both_new"] + r["sb_a_new_only"] + r["sb_b_new_only"] + r["sb_both_old"] == r["sb_rounds"]
        if ordered:
            assert r["sb_both_old"] == 0, r
            # rounds where one side's load came first: the two ran concurrently
            assert r["sb_a_new_only"] + r["sb_b_new_only"] > 0, r
            assert r["pairs_on_distinct_xcds"] >= pairs // 2, r


def test_litmus_rejects_bad_arguments(gtap):
    import torch
    buf, nb = buffer(torch, 2, 16)
    for args in ((2, True, 2, 16), (0, True, 0, 16), (0, True, 2, 0), (1, True, 2, 10 ** 6)):
        with pytest.raises(gtap.GtapError) as e:
            gtap.gtap_litmus(*args, buf.data_ptr(), nb)
        assert e.value.code == gtap.GTAP_E_INVAL, args
    with pytest.raises(gtap.GtapError) as e:
        gtap.gtap_litmus(1, True, 2, 64, buf.data_ptr(), nb)
    assert e.value.code == gtap.GTAP_E_NOMEM


def test_atomic_probe_rates(gtap):
    import torch
    blocks, iters = 2048, 64
    words = torch.zeros(blocks * 256 * 8 + 1, dtype=torch.int64, device="cuda")
    rates = {}
    for mode, name in ((gtap.GTAP_PROBE_DISTINCT, "distinct"), (gtap.GTAP_PROBE_PER_WAVE, "per-wave"),
                       (gtap.GTAP_PROBE_ONE_WORD, "one word")):
        say(f"atomic probe {name}: {blocks} x 256 threads, {iters} RMWs per issuing lane")
        rate, ms = gtap.gtap_probe_atomics(mode, blocks, iters, words.data_ptr(), words.numel())
        rates[name] = rate
        say(f"  {rate / 1e9:.3f} G RMW/s in {ms:.3f} ms")
        # every RMW landed: the counters hold exactly what was added
        torch.cuda.synchronize()
        w = words[:-1]
        if mode == gtap.GTAP_PROBE_DISTINCT:
            assert int(w[::8].sum()) == blocks * 256 * iters and int(w[::8].min()) == iters
        elif mode == gtap.GTAP_PROBE_PER_WAVE:
            assert int(w[:blocks * 64:16].sum()) == blocks * 4 * iters
        else:
            assert int(w[0]) == blocks * 4 * iters
    assert rates["distinct"] > rates["one word"]
