"""Analytic scenes and their occupied leaves (input generation only).

A scene lives in the cube [-1, 1]^3 (scenes normalised to a unit cube, RTMV
section 3).  Leaves of an octree of depth L are the cells of the 2^L grid;
cell (i, j, k) spans lo = -1 + (i, j, k) * h to lo + h with h = 2 / 2^L.
The SVLF octree stores only cells that contain a surface (section 4.1); here
"contains" is decided exactly against analytic objects:

* ``shell``: the closed cell meets the shell r0 <= |x| <= r1;
* ``solid``: the closed cell meets the solid object;
* ``surface``: the closed cell meets the object's boundary surface.

Cells are found by hierarchical refinement (a cell can only contain a part of
an object that its parent contains), so no dense grid is ever allocated.
"""

from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------- objects


class Ellipsoid:
    """Solid ellipsoid {x : (x-c)^T A (x-c) <= 1}, A = R diag(1/a^2) R^T."""

    def __init__(self, center, rot, semi):
        self.c = np.asarray(center, np.float64)
        self.R = np.asarray(rot, np.float64)
        self.a = np.asarray(semi, np.float64)
        self.A = self.R @ np.diag(1.0 / self.a**2) @ self.R.T
        # axis-aligned bounding box of the rotated ellipsoid
        ext = np.sqrt((self.R**2) @ (self.a**2))
        self.bb_lo = self.c - ext
        self.bb_hi = self.c + ext

    def q(self, y):
        """Quadratic form y^T A y for y = x - c, y shaped (..., 3)."""
        A = self.A
        return (A[0, 0] * y[..., 0] ** 2 + A[1, 1] * y[..., 1] ** 2
                + A[2, 2] * y[..., 2] ** 2
                + 2.0 * (A[0, 1] * y[..., 0] * y[..., 1]
                         + A[0, 2] * y[..., 0] * y[..., 2]
                         + A[1, 2] * y[..., 1] * y[..., 2]))

    def qmin_qmax(self, lo, hi):
        """Exact min and max of q over the closed boxes [lo, hi] (n, 3).

        The max of a convex function over a box is at a corner.  The min is
        found over the 27 faces of the box (interior, 6 faces, 12 edges and
        8 corners): on each face's affine hull the strictly convex q has one
        stationary point; the global minimiser is the one that lies in the
        box, and every feasible candidate is an upper bound.
        """
        l = lo - self.c
        u = hi - self.c
        n = l.shape[0]
        A = self.A
        bounds = (l, u)
        qmax = np.full(n, -np.inf)
        qmin = np.full(n, np.inf)
        # corners
        for cx in (0, 1):
            for cy in (0, 1):
                for cz in (0, 1):
                    y = np.stack([bounds[cx][:, 0], bounds[cy][:, 1],
                                  bounds[cz][:, 2]], axis=1)
                    qq = self.q(y)
                    qmax = np.maximum(qmax, qq)
                    qmin = np.minimum(qmin, qq)
        # interior: the centre lies in the box
        inside = np.all((l <= 0.0) & (u >= 0.0), axis=1)
        qmin = np.where(inside, 0.0, qmin)
        # edges: one free axis f, two fixed axes n1, n2
        for f in range(3):
            n1, n2 = [a for a in range(3) if a != f]
            for s1 in (0, 1):
                for s2 in (0, 1):
                    v1 = bounds[s1][:, n1]
                    v2 = bounds[s2][:, n2]
                    yf = -(A[f, n1] * v1 + A[f, n2] * v2) / A[f, f]
                    ok = (yf >= l[:, f]) & (yf <= u[:, f])
                    y = np.empty((n, 3))
                    y[:, f] = yf
                    y[:, n1] = v1
                    y[:, n2] = v2
                    qmin = np.where(ok, np.minimum(qmin, self.q(y)), qmin)
        # faces: two free axes f1, f2, one fixed axis m
        for m in range(3):
            f1, f2 = [a for a in range(3) if a != m]
            a, b, d = A[f1, f1], A[f1, f2], A[f2, f2]
            e1, e2 = A[f1, m], A[f2, m]
            det = a * d - b * b
            g1 = -(d * e1 - b * e2) / det
            g2 = -(a * e2 - b * e1) / det
            for s in (0, 1):
                v = bounds[s][:, m]
                y1 = g1 * v
                y2 = g2 * v
                ok = ((y1 >= l[:, f1]) & (y1 <= u[:, f1])
                      & (y2 >= l[:, f2]) & (y2 <= u[:, f2]))
                y = np.empty((n, 3))
                y[:, f1] = y1
                y[:, f2] = y2
                y[:, m] = v
                qmin = np.where(ok, np.minimum(qmin, self.q(y)), qmin)
        return qmin, qmax

    def test(self, lo, hi, rule):
        qmin, qmax = self.qmin_qmax(lo, hi)
        if rule == "solid":
            return qmin <= 1.0
        return (qmin <= 1.0) & (qmax >= 1.0)


class Box:
    """Solid axis-aligned box [c - e, c + e]."""

    def __init__(self, center, half):
        self.c = np.asarray(center, np.float64)
        self.e = np.asarray(half, np.float64)
        self.bb_lo = self.c - self.e
        self.bb_hi = self.c + self.e

    def test(self, lo, hi, rule):
        meet = np.all((lo <= self.bb_hi) & (hi >= self.bb_lo), axis=1)
        if rule == "solid":
            return meet
        strictly_inside = np.all((lo > self.bb_lo) & (hi < self.bb_hi), axis=1)
        return meet & ~strictly_inside


class Shell:
    """Spherical shell r0 <= |x| <= r1 centred at the origin."""

    def __init__(self, r0, r1):
        self.r0, self.r1 = float(r0), float(r1)
        self.bb_lo = np.full(3, -self.r1)
        self.bb_hi = np.full(3, self.r1)

    def test(self, lo, hi, rule=None):
        near = np.clip(0.0, lo, hi)
        dmin = np.sqrt(np.sum(near**2, axis=1))
        far = np.maximum(np.abs(lo), np.abs(hi))
        dmax = np.sqrt(np.sum(far**2, axis=1))
        return (dmin <= self.r1) & (dmax >= self.r0)


# ---------------------------------------------------------------- sampling


def random_rotation(rng):
    """Uniform random rotation from a normalised Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def random_ellipsoids(rng, n, semi_lo, semi_hi, scale=1.0, rotate=True):
    out = []
    for _ in range(n):
        semi = rng.uniform(semi_lo, semi_hi, 3) * scale
        rot = random_rotation(rng) if rotate else np.eye(3)
        r = semi.max()
        center = rng.uniform(-1.0 + r, 1.0 - r, 3)
        out.append(Ellipsoid(center, rot, semi))
    return out


def random_boxes(rng, n, half_lo, half_hi, scale=1.0):
    out = []
    for _ in range(n):
        half = rng.uniform(half_lo, half_hi, 3) * scale
        center = rng.uniform(-1.0 + half, 1.0 - half)
        out.append(Box(center, half))
    return out


# ---------------------------------------------------------------- occupancy

_CHILD = np.array([[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)],
                  dtype=np.int64)


def _cells_of(obj, level):
    """Grid cells at ``level`` overlapping obj's bounding box (closed)."""
    h = 2.0 / (1 << level)
    n = 1 << level
    lo = np.clip(np.floor((obj.bb_lo + 1.0) / h).astype(np.int64) - 1, 0, n - 1)
    hi = np.clip(np.floor((obj.bb_hi + 1.0) / h).astype(np.int64) + 1, 0, n - 1)
    return lo, hi


def object_leaves(obj, depth, rule, start_level=None):
    """Leaves (int64 (m, 3)) of a depth-``depth`` grid that pass obj.test."""
    if start_level is None:
        start_level = min(depth, 3)
    lo_i, hi_i = _cells_of(obj, start_level)
    g = np.stack(np.meshgrid(*[np.arange(lo_i[a], hi_i[a] + 1) for a in range(3)],
                             indexing="ij"), axis=-1).reshape(-1, 3)
    level = start_level
    cells = g
    while True:
        h = 2.0 / (1 << level)
        lo = -1.0 + cells * h
        keep = obj.test(lo, lo + h, rule)
        cells = cells[keep]
        if level == depth or cells.shape[0] == 0:
            return cells
        cells = (cells[:, None, :] * 2 + _CHILD[None, :, :]).reshape(-1, 3)
        level += 1


def _spread3(v):
    """Insert two zero bits between the low 21 bits of v (uint64)."""
    v = v & np.uint64(0x1FFFFF)
    v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
    return v


def morton_key(ijk):
    """A sort key that orders cells by Morton code (x fastest).  Used only to
    give generated leaf lists a canonical order; consumers re-derive their
    own structures."""
    ijk = np.asarray(ijk).astype(np.uint64)
    return (_spread3(ijk[:, 0]) | (_spread3(ijk[:, 1]) << np.uint64(1))
            | (_spread3(ijk[:, 2]) << np.uint64(2)))


def scene_leaves(objects, depth, rule):
    """Union over objects of their leaves, as int32 (n, 3), Morton-sorted."""
    parts = [object_leaves(o, depth, rule) for o in objects]
    parts = [p for p in parts if p.shape[0]]
    if not parts:
        return np.zeros((0, 3), np.int32)
    allc = np.concatenate(parts, axis=0)
    key = morton_key(allc)
    key, first = np.unique(key, return_index=True)
    return allc[first].astype(np.int32)


def count_vertices(leaf_ijk):
    """Number of distinct lattice points that are corners of the leaves."""
    if leaf_ijk.shape[0] == 0:
        return 0
    c = (leaf_ijk[:, None, :].astype(np.int64) + _CHILD[None, :, :]).reshape(-1, 3)
    key = (c[:, 0] << 42) | (c[:, 1] << 21) | c[:, 2]
    return int(np.unique(key).shape[0])


def occupancy_fraction(leaf_ijk, depth):
    return leaf_ijk.shape[0] / float(8**depth)
