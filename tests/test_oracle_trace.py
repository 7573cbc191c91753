"""Pins for the oracle's ray/octree intersection (SVLF sections 4.2-4.3).

* brute force over all occupied leaves equals the hierarchical traversal;
* the FP32 slab predicate agrees with an exact rational slab test except on
  rays whose exact interval is within rounding of empty;
* hand-derived hit lists for crafted degenerate rays (tests/golden);
* a textbook 3D-DDA (Amanatides & Woo 1987) on a fully occupied block;
* invariants of hit lists.
"""

from fractions import Fraction

import numpy as np
import pytest

from oracle.octree import Octree
from oracle.trace import (reciprocal, slab, trace_hits, trace_hits_bruteforce,
                          all_hits_count)
from tests.helpers import crafted_occupancy, golden_case_arrays, load_golden, random_rays


def _same_hits(a, b):
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("depth", [1, 2, 3, 4])
@pytest.mark.parametrize("kind", ["empty", "full", "single", "checker", "random30"])
def test_bruteforce_equals_hierarchical(depth, kind):
    if depth == 4 and kind in ("full", "checker", "random30"):
        n_rays = 48
    else:
        n_rays = 200
    cells = crafted_occupancy(kind, depth, seed=depth)
    oc = Octree(cells, depth)
    rng = np.random.default_rng(depth * 10 + len(kind))
    o, d = random_rays(rng, n_rays)
    for K in (1, 3, 8):
        _same_hits(trace_hits(oc, o, d, K), trace_hits_bruteforce(oc, o, d, K))


def _exact_interval(o, d, lo, hi):
    """Exact rational slab interval of a ray and a box (half-open rule on
    zero-direction axes, t_min = 0)."""
    tn, tf = Fraction(0), None
    for a in range(3):
        oa, da = Fraction(float(o[a])), Fraction(float(d[a]))
        la, ha = Fraction(float(lo[a])), Fraction(float(hi[a]))
        if da == 0:
            if not (la <= oa < ha):
                return None
            continue
        t0, t1 = (la - oa) / da, (ha - oa) / da
        tn = max(tn, min(t0, t1))
        m = max(t0, t1)
        tf = m if tf is None else min(tf, m)
    return tn, tf


def test_fp32_predicate_against_exact_rationals():
    depth = 2
    oc = Octree(crafted_occupancy("full", depth), depth)
    h = 2.0 / (1 << depth)
    lo = (-1.0 + oc.leaf_ijk * h).astype(np.float32)
    hi = (lo + np.float32(h)).astype(np.float32)
    rng = np.random.default_rng(7)
    o, d = random_rays(rng, 120, axis_frac=0.2)
    # add rays aimed (almost) at lattice vertices, the hardest case
    v = rng.integers(0, 5, (40, 3)) * h - 1.0
    o2 = rng.uniform(-3, 3, (40, 3))
    d2 = v - o2 + rng.choice([0.0, 1e-7, -1e-7], (40, 3))
    d2 /= np.linalg.norm(d2, axis=1, keepdims=True)
    o = np.concatenate([o, o2.astype(np.float32)])
    d = np.concatenate([d, d2.astype(np.float32)])
    inv = reciprocal(d)
    disagree = 0
    total = 0
    for r in range(o.shape[0]):
        rr = np.repeat(r, lo.shape[0])
        hit32, tin32, tout32 = slab(o[rr], inv[rr], lo, hi)
        for c in range(lo.shape[0]):
            iv = _exact_interval(o[r], d[r], lo[c], hi[c])
            exact_hit = iv is not None and iv[1] is not None and iv[0] < iv[1]
            if iv is not None and iv[1] is None:   # d = 0 and inside: all t
                exact_hit = True
            total += 1
            if exact_hit != bool(hit32[c]):
                disagree += 1
                # only near-degenerate intervals may differ
                width = abs(float(iv[1] - iv[0]))
                scale = max(1.0, abs(float(iv[0])), abs(float(iv[1])))
                assert width <= 1e-6 * scale, (r, c, width)
            elif exact_hit and iv[1] is not None:
                # t values are the exact ones up to two FP32 roundings
                tin_e, tout_e = float(iv[0]), float(iv[1])
                assert abs(float(tin32[c]) - tin_e) <= 4e-7 * max(1.0, abs(tin_e))
                assert abs(float(tout32[c]) - tout_e) <= 4e-7 * max(1.0, abs(tout_e))
    assert total == o.shape[0] * lo.shape[0]
    assert disagree <= 0.02 * total


@pytest.mark.parametrize("case", load_golden("degenerate_rays.json")["cases"],
                         ids=lambda c: c["name"])
def test_hand_derived_degenerate_rays(case):
    depth = load_golden("degenerate_rays.json")["depth"]
    oc = Octree(crafted_occupancy(case["occupancy"], depth), depth)
    o, d = golden_case_arrays(case)
    K = case["K"]
    for fn in (trace_hits, trace_hits_bruteforce):
        leaf, tin, tout, cnt = fn(oc, o, d, K)
        exp = case["hits"]
        assert cnt[0] == len(exp)
        for s, (i, j, k, t0, t1) in enumerate(exp):
            assert oc.leaf_ijk[leaf[0, s]].tolist() == [i, j, k]
            assert tin[0, s] == np.float32(t0)
            assert tout[0, s] == np.float32(t1)
            # t_in is +0, never -0
            assert not np.signbit(tin[0, s])
        assert np.all(leaf[0, len(exp):] == -1)


def _dda_cells(o, d, n):
    """Amanatides-Woo 3D-DDA over an n^3 grid on [-1,1]^3 in FP64: the list
    of cells crossed with positive length, and the chord length (in t)."""
    o = np.asarray(o, np.float64)
    d = np.asarray(d, np.float64)
    h = 2.0 / n
    tmin, tmax = 0.0, np.inf
    for a in range(3):
        if d[a] == 0:
            if not (-1 <= o[a] < 1):
                return [], 0.0
            continue
        t0, t1 = (-1 - o[a]) / d[a], (1 - o[a]) / d[a]
        tmin, tmax = max(tmin, min(t0, t1)), min(tmax, max(t0, t1))
    if not tmin < tmax:
        return [], 0.0
    p = o + tmin * d
    cell = np.clip(np.floor((p + 1) / h).astype(int), 0, n - 1)
    step = np.sign(d).astype(int)
    tnext = np.full(3, np.inf)
    tdelta = np.full(3, np.inf)
    for a in range(3):
        if d[a] > 0:
            tnext[a] = (-1 + (cell[a] + 1) * h - o[a]) / d[a]
            tdelta[a] = h / d[a]
        elif d[a] < 0:
            tnext[a] = (-1 + cell[a] * h - o[a]) / d[a]
            tdelta[a] = -h / d[a]
    cells = []
    t = tmin
    while True:
        a = int(np.argmin(tnext))
        t_exit = min(tnext[a], tmax)
        if t_exit > t:
            cells.append(tuple(cell))
        if tnext[a] >= tmax:
            break
        t = tnext[a]
        cell[a] += step[a]
        tnext[a] += tdelta[a]
        if not (0 <= cell[a] < n):
            break
    return cells, tmax - tmin


def test_against_textbook_dda_full_block():
    depth = 3
    n = 1 << depth
    oc = Octree(crafted_occupancy("full", depth), depth)
    rng = np.random.default_rng(11)
    o, d = random_rays(rng, 300, inside_frac=0.3, axis_frac=0.0)
    leaf, tin, tout, cnt = trace_hits(oc, o, d, 64)
    for r in range(o.shape[0]):
        cells, chord = _dda_cells(o[r], d[r], n)
        got = [tuple(oc.leaf_ijk[leaf[r, s]]) for s in range(cnt[r])]
        if got != cells:
            # cells clipped at a corner by less than rounding may differ
            assert abs(len(got) - len(cells)) <= 1, (r, got, cells)
        total = float(np.sum(tout[r, :cnt[r]].astype(np.float64) - tin[r, :cnt[r]]))
        assert abs(total - chord) <= 1e-5 * max(1.0, chord)


def test_hit_list_invariants():
    depth = 4
    oc = Octree(crafted_occupancy("random30", depth, seed=5), depth)
    rng = np.random.default_rng(3)
    o, d = random_rays(rng, 300)
    K = 5
    leaf, tin, tout, cnt = trace_hits(oc, o, d, K)
    full = all_hits_count(oc, o, d)
    assert np.all(cnt == np.minimum(K, full))
    for r in range(o.shape[0]):
        c = cnt[r]
        assert np.all(leaf[r, :c] >= 0) and np.all(leaf[r, c:] == -1)
        assert np.all(tin[r, :c] < tout[r, :c])
        assert np.all(tin[r, :c] >= 0)
        if c > 1:
            assert np.all(tout[r, :c - 1] <= tin[r, 1:c])  # disjoint, ordered
            assert np.all(tin[r, :c - 1] < tin[r, 1:c])    # strictly increasing
        assert len(set(leaf[r, :c].tolist())) == c
