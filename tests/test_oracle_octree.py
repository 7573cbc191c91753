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
