"""Pins of the Cilksort oracle (GTaP Sec. 6.3) against what the mathematics
fixes: the output is the sorted permutation of the input (numpy's sort), the
sort recursion is a binary tree (2^(k+1) - 1 sort tasks for n = cutoff * 2^k),
and the task, continuation and leaf counts satisfy the fork-join identities of
the recursion (every internal sort forks two sorts and one merge and resumes
twice, every internal merge forks two merges and resumes once)."""
import numpy as np
import pytest

import oracle


def inputs():
    rng = np.random.default_rng(7)
    yield "random", rng.integers(0, 2**32, size=100003, dtype=np.uint32)
    yield "few distinct", rng.integers(0, 5, size=20000, dtype=np.uint32)
    yield "all equal", np.full(5000, 42, dtype=np.uint32)
    yield "sorted", np.arange(7777, dtype=np.uint32)
    yield "reversed", np.arange(7777, dtype=np.uint32)[::-1].copy()
    yield "extremes", np.array([2**32 - 1, 0, 2**32 - 1, 1, 0] * 300, dtype=np.uint32)
    for n in (0, 1, 2, 63, 64, 65, 255, 256, 257, 4099):
        yield f"n={n}", rng.integers(0, 2**32, size=n, dtype=np.uint32)


def check_identities(r, n, sc):
    S = r.tasks - r.aux                      # sort tasks
    M = r.aux                                # merge tasks
    internal_s = (S - 1) // 2 if n > sc else 0
    assert S == 2 * internal_s + 1
    internal_m = r.conts - 2 * internal_s
    assert internal_m >= 0
    assert M == internal_s + 2 * internal_m
    assert r.leaves == (internal_s + 1) + (M - internal_m)
    assert r.value == n


@pytest.mark.parametrize("cut", [(64, 256), (1, 2), (16, 1000000)])
def test_output_is_sorted_permutation(cut):
    for name, x in inputs():
        got, r = oracle.cilksort(x, *cut)
        assert np.array_equal(got, np.sort(x)), name
        check_identities(r, x.size, cut[0])


@pytest.mark.parametrize("k", [0, 1, 5, 10])
def test_sort_tree_closed_form(k):
    sc = 64
    n = sc * 2**k
    x = np.random.default_rng(k).integers(0, 2**32, size=n, dtype=np.uint32)
    got, r = oracle.cilksort(x, sc, 256)
    assert r.tasks - r.aux == 2**(k + 1) - 1
    assert np.array_equal(got, np.sort(x))


def test_merges_never_split_below_cutoff():
    """merge cutoff >= n: one unsplit merge per internal sort."""
    x = np.random.default_rng(3).integers(0, 2**32, size=3000, dtype=np.uint32)
    got, r = oracle.cilksort(x, 32, 10**9)
    internal_s = (r.tasks - r.aux - 1) // 2
    assert r.aux == internal_s and r.conts == 2 * internal_s
    assert np.array_equal(got, np.sort(x))


def test_small_input_is_one_leaf():
    x = np.array([5, 3, 9], dtype=np.uint32)
    got, r = oracle.cilksort(x, 64, 256)
    assert got.tolist() == [3, 5, 9] and (r.tasks, r.conts, r.leaves, r.aux) == (1, 0, 1, 0)
