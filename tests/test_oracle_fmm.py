"""Pins of the CPU FMM oracle against what the mathematics fixes.

- the octree's structural invariants (points inside their leaf cube, children
  partition their parent, split iff more than leaf_max points);
- every (target, source) pair is covered exactly once by the interaction lists;
- accepted pairs are geometrically well separated;
- the potential equals P2P plus, per accepted pair, the Legendre series of
  1/|d + delta| truncated at degree p (a formula independent of the Cartesian
  expansion machinery);
- direct summation is matched within the rigorous truncation bound;
- theta -> 0 reduces to direct summation; negated charges negate the potential
  exactly; the error falls as the order grows.
"""
import numpy as np
import pytest
from scipy.special import eval_legendre

import oracle
from synth import points

E, BITS = 7, 21
UNIT = 2.0 ** (E - (BITS - 1))   # grid cell edge in length units


@pytest.fixture(scope="module")
def small():
    x, y, z, q = points.plummer(3000, 3)
    return x, y, z, q


def centre(cell):
    w = 2 ** (BITS - cell["level"])
    return np.array([-2.0 ** E + (cell[k] + w / 2.0) * UNIT for k in ("ax", "ay", "az")])


def width(cell):
    return 2 ** (BITS - cell["level"]) * UNIT


def test_tree_invariants(small):
    x, y, z, q = small
    perm, cells, keys = oracle.fmm_tree(x, y, z, 64)
    n = x.size
    assert sorted(perm.tolist()) == list(range(n))
    assert np.all(np.diff(keys.astype(np.float64)) >= 0)
    assert cells[0]["begin"] == 0 and cells[0]["end"] == n and cells[0]["parent"] == -1
    levels = cells["level"]
    assert np.all(np.diff(levels) >= 0)  # breadth-first numbering
    for c, cell in enumerate(cells):
        cnt = cell["end"] - cell["begin"]
        assert cnt > 0
        split = cnt > 64 and cell["level"] < BITS
        assert (cell["nchild"] > 0) == split
        if cell["nchild"]:
            ch = cells[cell["child0"]:cell["child0"] + cell["nchild"]]
            assert np.all(ch["parent"] == c) and np.all(ch["level"] == cell["level"] + 1)
            assert ch[0]["begin"] == cell["begin"] and ch[-1]["end"] == cell["end"]
            assert np.all(ch["begin"][1:] == ch["end"][:-1])
        else:
            lo = centre(cell) - width(cell) / 2
            hi = lo + width(cell)
            pts = perm[cell["begin"]:cell["end"]]
            P = np.stack([x[pts], y[pts], z[pts]], axis=1)
            assert np.all(P >= lo) and np.all(P < hi)


def _leaf_and_ancestors(cells, perm, i):
    pos = int(np.nonzero(perm == i)[0][0])
    leaves = np.nonzero((cells["nchild"] == 0) & (cells["begin"] <= pos) & (cells["end"] > pos))[0]
    assert leaves.size == 1
    chain, c = [], int(leaves[0])
    while c >= 0:
        chain.append(c)
        c = int(cells[c]["parent"])
    return chain


def test_lists_cover_every_source_once(small):
    x, y, z, q = small
    r = oracle.fmm(x, y, z, q, lists=True)
    perm, cells, _ = oracle.fmm_tree(x, y, z, 64)
    assert r.stats["m2l_pairs"] == len(r.m2l) and r.stats["p2p_pairs"] == len(r.p2p)
    for i in (0, 17, 1234, 2999):
        chain = _leaf_and_ancestors(cells, perm, i)
        cover = np.zeros(x.size, dtype=np.int64)
        for a, b in r.m2l[np.isin(r.m2l[:, 0], chain)]:
            cover[perm[cells[b]["begin"]:cells[b]["end"]]] += 1
        for a, b in r.p2p[r.p2p[:, 0] == chain[0]]:
            cover[perm[cells[b]["begin"]:cells[b]["end"]]] += 1
        assert np.all(cover == 1), (i, np.bincount(cover))


def test_accepted_pairs_are_separated(small):
    x, y, z, q = small
    r = oracle.fmm(x, y, z, q, lists=True)
    _, cells, _ = oracle.fmm_tree(x, y, z, 64)
    for a, b in r.m2l[::7]:
        R = (np.sqrt(3) / 2) * (width(cells[a]) + width(cells[b]))
        assert R < 0.5 * np.linalg.norm(centre(cells[a]) - centre(cells[b]))
    for a, b in r.p2p:
        assert cells[a]["nchild"] == 0 and cells[b]["nchild"] == 0


def _legendre_phi(x, y, z, q, r, cells, perm, i, p):
    """P2P plus the degree-p Legendre series of every accepted pair at point i."""
    xi = np.array([x[i], y[i], z[i]])
    chain = _leaf_and_ancestors(cells, perm, i)
    phi = 0.0
    bound = 0.0
    for a, b in r.m2l[np.isin(r.m2l[:, 0], chain)]:
        ca, cb = centre(cells[a]), centre(cells[b])
        js = perm[cells[b]["begin"]:cells[b]["end"]]
        Y = np.stack([x[js], y[js], z[js]], axis=1)
        d = ca - cb
        delta = (xi - ca)[None, :] - (Y - cb)
        nd, ndel = np.linalg.norm(d), np.linalg.norm(delta, axis=1)
        cosg = -(delta @ d) / (nd * np.where(ndel > 0, ndel, 1.0))
        series = sum((ndel ** k) / nd ** (k + 1) * eval_legendre(k, cosg) for k in range(p + 1))
        phi += float(np.sum(q[js] * series))
        rho = ndel / nd
        assert np.all(rho < 1)
        bound += float(np.sum(np.abs(q[js]) * rho ** (p + 1) / ((1 - rho) * nd)))
    for a, b in r.p2p[r.p2p[:, 0] == chain[0]]:
        js = perm[cells[b]["begin"]:cells[b]["end"]]
        js = js[js != i]
        dist = np.sqrt((x[js] - x[i]) ** 2 + (y[js] - y[i]) ** 2 + (z[js] - z[i]) ** 2)
        phi += float(np.sum(q[js] / dist))
    return phi, bound


def test_potential_equals_legendre_definition(small):
    x, y, z, q = small
    r = oracle.fmm(x, y, z, q, lists=True)
    perm, cells, _ = oracle.fmm_tree(x, y, z, 64)
    scale = np.abs(r.phi).max()
    for i in (3, 400, 1500, 2500, 2998):
        want, _ = _legendre_phi(x, y, z, q, r, cells, perm, i, 6)
        assert abs(r.phi[i] - want) <= 1e-13 * scale, (i, r.phi[i], want)


def test_direct_sum_within_truncation_bound(small):
    x, y, z, q = small
    r = oracle.fmm(x, y, z, q, lists=True)
    perm, cells, _ = oracle.fmm_tree(x, y, z, 64)
    tg = np.arange(0, x.size, 97)
    d = oracle.direct(x, y, z, q, tg)
    # the oracle's direct sum is itself checked against numpy
    for t, i in enumerate(tg[:5]):
        js = np.arange(x.size) != i
        dist = np.sqrt((x[js] - x[i]) ** 2 + (y[js] - y[i]) ** 2 + (z[js] - z[i]) ** 2)
        assert abs(d[t] - np.sum(q[js] / dist)) <= 1e-12 * abs(d).max()
    for t, i in enumerate(tg):
        _, bound = _legendre_phi(x, y, z, q, r, cells, perm, int(i), 6)
        assert abs(r.phi[i] - d[t]) <= bound * (1 + 1e-9) + 1e-13 * np.abs(d).max()
    assert np.linalg.norm(r.phi[tg] - d) / np.linalg.norm(d) < 1e-4


def test_theta_zero_is_direct_sum():
    x, y, z, q = points.plummer(1500, 8)
    r = oracle.fmm(x, y, z, q, theta=(0, 1))
    assert r.stats["m2l_pairs"] == 0
    tg = np.arange(1500)
    d = oracle.direct(x, y, z, q, tg)
    assert np.abs(r.phi - d).max() <= 1e-13 * np.abs(d).max()
    assert r.stats["p2p_interactions"] == 1500 * 1499


def test_negated_charges_negate_exactly(small):
    x, y, z, q = small
    a = oracle.fmm(x, y, z, q)
    b = oracle.fmm(x, y, z, -q)
    assert np.array_equal(a.phi, -b.phi)
    assert a.stats["m2l_hash"] == b.stats["m2l_hash"]


def test_error_falls_with_order():
    x, y, z, q = points.uniform_cube(4000, 4, half=10.0)
    tg = np.arange(0, 4000, 41)
    d = oracle.direct(x, y, z, q, tg)
    errs = []
    for p in (0, 2, 4, 6, 8):
        r = oracle.fmm(x, y, z, q, p=p, targets=tg)
        errs.append(np.linalg.norm(r.phi - d) / np.linalg.norm(d))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < errs[0] * 1e-3, errs


def test_sampled_targets_equal_full_pass(small):
    x, y, z, q = small
    full = oracle.fmm(x, y, z, q)
    tg = np.array([5, 77, 1999, 2718])
    part = oracle.fmm(x, y, z, q, targets=tg)
    assert np.abs(part.phi - full.phi[tg]).max() <= 1e-14 * np.abs(full.phi).max()
    assert part.stats["m2l_hash"] == full.stats["m2l_hash"]


def test_coincident_points_are_skipped_and_counted():
    x, y, z, q = points.plummer(500, 9)
    x = np.concatenate([x, x[:3]])
    y = np.concatenate([y, y[:3]])
    z = np.concatenate([z, z[:3]])
    q = np.concatenate([q, q[:3]])
    r = oracle.fmm(x, y, z, q, theta=(0, 1))
    assert r.stats["coincident"] == 6
    d = oracle.direct(x, y, z, q, np.arange(503))
    assert np.abs(r.phi - d).max() <= 1e-13 * np.abs(d).max()


def test_split_rule_keeps_levels_close(small):
    """Splitting the wider cell keeps the two cells of a pair within one level
    of each other unless the wider one is a leaf (it cannot be split)."""
    x, y, z, q = small
    r = oracle.fmm(x, y, z, q, lists=True)
    _, cells, _ = oracle.fmm_tree(x, y, z, 64)
    for lst in (r.m2l, r.p2p):
        la, lb = cells["level"][lst[:, 0]], cells["level"][lst[:, 1]]
        far = np.abs(la - lb) >= 2
        wider = np.where(la < lb, lst[:, 0], lst[:, 1])
        assert np.all(cells["nchild"][wider[far]] == 0)


def _golden_1m():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "fmm_plummer_1m.txt")
    lists = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("# lists:"):
                f = line.split()[2:]
                lists = {f[i]: int(f[i + 1]) for i in range(0, len(f), 2)}
    data = np.loadtxt(path)
    return data[:, 0].astype(np.int64), data[:, 1], data[:, 2], lists


def test_full_size_oracle_against_direct_summation():
    """10^6 Plummer points: the oracle FMM at 4,096 sampled targets (stored by
    tests/golden/make_fmm_golden.py) against fp64 direct summation."""
    idx, direct, fmm_v, lists = _golden_1m()
    assert idx.size == 4096 and len(np.unique(idx)) == 4096
    err = fmm_v - direct
    assert np.linalg.norm(err) / np.linalg.norm(direct) < 1e-4
    assert np.abs(err).max() < 2e-4 * np.abs(direct).max()
    assert lists["m2l_pairs"] > 0 and lists["p2p_pairs"] > 0
