"""Sparse voxel octree, by definition (SVLF section 4.1, "Scene volume").

The scene cube [-1, 1]^3 is split into a 2^L grid of leaf cells; the octree
keeps only occupied leaves and their ancestors.  Conventions (the paper leaves
them open; the library follows the same ones):

* cell (i, j, k) of level l has h_l = 2 / 2^l, lo = -1 + (i, j, k) h_l,
  hi = lo + h_l;
* the Morton code interleaves bit b of i, j, k into bits 3b, 3b+1, 3b+2;
* a node's child index is c = x | y << 1 | z << 2 for the child's low bits;
* leaf ids are ranks in ascending Morton order; nodes of each level are also
  kept in ascending Morton order (this is "level order");
* every vertex of the (2^L + 1)^3 lattice that is a corner of an occupied leaf
  carries one feature embedding (embeddings are shared by adjacent voxels);
  vertex ids are ranks of the vertices' Morton codes (L+1 bits per axis);
* corner j of a leaf is the vertex at (i + (j&1), j + (j>>1 & 1), k + (j>>2)).

Everything here is integer work written out plainly with Python/numpy loops.
"""

from __future__ import annotations

import numpy as np


def morton_encode(ijk, bits):
    """Interleave ``bits`` low bits of each axis; ijk int array (n, 3)."""
    ijk = np.asarray(ijk, dtype=np.int64)
    code = np.zeros(ijk.shape[0], dtype=np.int64)
    for b in range(bits):
        for a in range(3):
            code |= ((ijk[:, a] >> b) & 1) << (3 * b + a)
    return code


def morton_decode(code, bits):
    code = np.asarray(code, dtype=np.int64)
    ijk = np.zeros((code.shape[0], 3), dtype=np.int64)
    for b in range(bits):
        for a in range(3):
            ijk[:, a] |= ((code >> (3 * b + a)) & 1) << b
    return ijk


CORNER_OFFSETS = np.array([[j & 1, (j >> 1) & 1, (j >> 2) & 1] for j in range(8)],
                          dtype=np.int64)


class Octree:
    """The oracle's octree.

    Attributes
    ----------
    depth        L (leaves live at level L)
    level_codes  list of L+1 sorted int64 arrays: Morton codes of the nodes at
                 each level (level 0 holds the root, code 0, if any leaf exists)
    masks        list of L uint8 arrays: child mask of each node of levels 0..L-1
    leaf_ijk     int64 (n_leaves, 3), Morton order (leaf id = row)
    vertex_ijk   int64 (n_vertices, 3), vertex id = row
    leaf_corners int64 (n_leaves, 8): vertex id of corner j
    """

    def __init__(self, leaf_ijk, depth):
        leaf_ijk = np.asarray(leaf_ijk, dtype=np.int64).reshape(-1, 3)
        L = int(depth)
        if L < 1:
            raise ValueError("depth must be >= 1")
        if leaf_ijk.size and (leaf_ijk.min() < 0 or leaf_ijk.max() >= (1 << L)):
            raise ValueError("leaf coordinate out of range")
        codes = morton_encode(leaf_ijk, L)
        order = np.argsort(codes, kind="stable")
        codes = codes[order]
        if codes.size and np.any(codes[1:] == codes[:-1]):
            raise ValueError("duplicate leaf")
        self.depth = L
        self.leaf_ijk = leaf_ijk[order]
        self.level_codes = []
        for l in range(L + 1):
            self.level_codes.append(np.unique(codes >> (3 * (L - l))))
        self.masks = []
        for l in range(L):
            parents = self.level_codes[l]
            child = self.level_codes[l + 1]
            mask = np.zeros(parents.shape[0], dtype=np.int64)
            pos = np.searchsorted(parents, child >> 3)
            np.bitwise_or.at(mask, pos, 1 << (child & 7))
            self.masks.append(mask.astype(np.uint8))
        # vertices
        corners = (self.leaf_ijk[:, None, :] + CORNER_OFFSETS[None, :, :]).reshape(-1, 3)
        vcode = morton_encode(corners, L + 1)
        uniq = np.unique(vcode)
        self.vertex_ijk = morton_decode(uniq, L + 1)
        self.leaf_corners = np.searchsorted(uniq, vcode).reshape(-1, 8)

    @property
    def n_leaves(self):
        return self.leaf_ijk.shape[0]

    @property
    def n_vertices(self):
        return self.vertex_ijk.shape[0]

    def cell_bounds(self, level, ijk):
        """FP64 lo, hi of cells (exact dyadic values)."""
        h = 2.0 / (1 << level)
        lo = -1.0 + np.asarray(ijk, np.float64) * h
        return lo, lo + h

    def children(self, level, node_index):
        """Child node indices (at level+1) of nodes ``node_index`` at level."""
        parent_codes = self.level_codes[level][node_index]
        nxt = self.level_codes[level + 1]
        first = np.searchsorted(nxt, parent_codes << 3)
        last = np.searchsorted(nxt, (parent_codes << 3) + 8)
        return first, last


def occupancy_from_depth(o, d, t, depth):
    """Occupied leaves of a depth-`depth` grid from depth maps (section 4.1:
    the octree keeps the voxels that contain a surface; the surface points
    come from the dataset's depth).  For every ray with a finite target
    depth t > 0 the surface point p = o + t d is taken in binary32
    arithmetic (a product, then a sum, each rounded to nearest; no fused
    multiply-add) and its cell is floor(RN(p + 1) * 2^(depth-1)) per axis;
    points outside [0, 2^depth) on any axis are dropped.  Returns the unique
    cells, int64 (m, 3), in ascending Morton order (the leaf-id order)."""
    o = np.asarray(o, np.float32)
    d = np.asarray(d, np.float32)
    t = np.asarray(t, np.float32)
    ok = np.isfinite(t) & (t > np.float32(0))
    with np.errstate(invalid="ignore", over="ignore"):
        p = o + t[:, None] * d                       # numpy float32: RN product, RN sum
        q = (p + np.float32(1.0)) * np.float32(2.0 ** (depth - 1))
    ok &= np.all(np.isfinite(q), axis=1) & np.all((q >= 0) & (q < (1 << depth)), axis=1)
    cells = np.floor(q[ok]).astype(np.int64)
    if cells.shape[0] == 0:
        return np.zeros((0, 3), np.int64)
    codes = np.unique(morton_encode(cells, depth))
    return morton_decode(codes, depth)
