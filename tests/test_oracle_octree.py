"""Pins for the oracle's octree (SVLF section 4.1, "Scene volume")."""

import itertools

import numpy as np
import pytest

from oracle.octree import Octree


def py_morton(i, j, k, bits):
    """Bit interleave written scalar-by-scalar (independent of numpy code)."""
    code = 0
    for b in range(bits):
        code |= ((i >> b) & 1) << (3 * b)
        code |= ((j >> b) & 1) << (3 * b + 1)
        code |= ((k >> b) & 1) << (3 * b + 2)
    return code


def test_two_leaf_depth1_by_hand():
    # leaves (0,0,0) and (1,1,1) of a 2^3 grid: root mask = bit 0 | bit 7
    oc = Octree([[1, 1, 1], [0, 0, 0]], 1)
    assert oc.leaf_ijk.tolist() == [[0, 0, 0], [1, 1, 1]]
    assert oc.masks[0].tolist() == [0b10000001]
    # 8 + 8 corners share exactly the centre vertex (1,1,1)
    assert oc.n_vertices == 15
    # leaf 0's corner 7 and leaf 1's corner 0 are the same vertex
    assert oc.leaf_corners[0, 7] == oc.leaf_corners[1, 0]
    assert oc.vertex_ijk[oc.leaf_corners[0, 7]].tolist() == [1, 1, 1]


@pytest.mark.parametrize("depth,frac,seed", [(1, 0.5, 0), (2, 0.3, 1), (3, 0.1, 2), (4, 0.02, 3)])
def test_structure_against_python_sets(depth, frac, seed):
    rng = np.random.default_rng(seed)
    n = 1 << depth
    cells = [c for c in itertools.product(range(n), repeat=3) if rng.random() < frac]
    if not cells:
        cells = [(0, 0, 0)]
    oc = Octree(np.array(cells), depth)
    # leaves sorted by scalar Morton code
    keys = sorted(py_morton(i, j, k, depth) for i, j, k in cells)
    got = [py_morton(*map(int, r), depth) for r in oc.leaf_ijk]
    assert got == keys
    # each level = set of ancestors, masks = which children exist
    for l in range(depth + 1):
        anc = sorted({kk >> (3 * (depth - l)) for kk in keys})
        assert oc.level_codes[l].tolist() == anc
    for l in range(depth):
        for node, code in enumerate(oc.level_codes[l]):
            kids = {c & 7 for c in oc.level_codes[l + 1].tolist() if (c >> 3) == code}
            assert int(oc.masks[l][node]) == sum(1 << c for c in kids)
    # vertices: the set of corners, ranked by Morton code of L+1 bits
    verts = {(i + dx, j + dy, k + dz) for (i, j, k) in cells
             for dx in (0, 1) for dy in (0, 1) for dz in (0, 1)}
    vsorted = sorted(verts, key=lambda v: py_morton(*v, depth + 1))
    assert [tuple(v) for v in oc.vertex_ijk.tolist()] == vsorted
    for leaf, (i, j, k) in enumerate(oc.leaf_ijk.tolist()):
        for c in range(8):
            v = oc.vertex_ijk[oc.leaf_corners[leaf, c]].tolist()
            assert v == [i + (c & 1), j + ((c >> 1) & 1), k + ((c >> 2) & 1)]


def test_rejects_bad_input():
    with pytest.raises(ValueError):
        Octree([[0, 0, 2]], 1)
    with pytest.raises(ValueError):
        Octree([[0, 0, 0], [0, 0, 0]], 2)
    with pytest.raises(ValueError):
        Octree([[0, 0, 0]], 0)


# ------------------------------------------------------------ occupancy from depth maps

def test_occupancy_from_depth_hand_cases():
    from oracle.octree import occupancy_from_depth
    L = 2                                            # cells of edge 0.5, 4 per axis
    d = np.array([[1, 0, 0]] * 7, np.float32)
    o = np.array([[-3, 0.1, 0.1],      # p = (0, .1, .1): on a face -> the upper cell
                  [-3, -0.9, 0.6],     # p = (0, -.9, .6)
                  [-4, 0.1, 0.1],      # p = (-1, .1, .1): the lowest cell on x
                  [-2, 0.1, 0.1],      # p = (1, .1, .1): outside (upper bound open)
                  [-3, 0.1, 0.1],      # t = 0: no surface
                  [-3, 0.1, 0.1],      # duplicate of the first
                  [-3, 0.1, 0.1]],     # t = NaN
                 np.float32)
    t = np.array([3, 3, 3, 3, 0, 3, np.nan], np.float32)
    got = occupancy_from_depth(o, d, t, L)
    exp = {(2, 2, 2), (2, 0, 3), (0, 2, 2)}
    assert {tuple(c) for c in got.tolist()} == exp and got.shape[0] == 3
    # Morton order: codes ascending
    from oracle.octree import morton_encode
    codes = morton_encode(got, L)
    assert np.all(np.diff(codes) > 0)


def test_occupancy_from_depth_scalar_rational_reference():
    """Per-point scalar reference: q = RN32(RN32(o + RN32(t d)) + 1) 2^(L-1)
    floored with exact rational arithmetic."""
    from fractions import Fraction
    from oracle.octree import occupancy_from_depth
    rng = np.random.default_rng(0)
    L = 4
    n = 400
    o = rng.uniform(-1.2, 1.2, (n, 3)).astype(np.float32)
    d = rng.normal(size=(n, 3)).astype(np.float32)
    t = rng.uniform(0, 0.3, n).astype(np.float32)
    # points exactly on cell faces: x = 0.25 k
    o[:40, 0] = (rng.integers(-4, 4, 40) * 0.25).astype(np.float32)
    d[:40, 0] = 0.0
    t[::17] = 0
    cells = set()
    for r in range(n):
        if not t[r] > 0:
            continue
        c = []
        for a in range(3):
            p = np.float32(o[r, a]) + np.float32(np.float32(t[r]) * np.float32(d[r, a]))
            q = Fraction(float(np.float32(p) + np.float32(1.0))) * (2 ** (L - 1))
            i = q.numerator // q.denominator
            c.append(i)
        if all(0 <= i < (1 << L) for i in c):
            cells.add(tuple(c))
    got = occupancy_from_depth(o, d, t, L)
    assert {tuple(c) for c in got.tolist()} == cells
    assert len(cells) > 20
