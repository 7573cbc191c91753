"""Ray / octree intersection with an exactly specified FP32 predicate.

SVLF first lists all voxels a ray intersects, in order along the ray, each with
its entry and exit points x1, x2 (section 4.3, "Evaluating intersected voxels"),
using a ray-AABB slab test (section 4.2) inside a hierarchical sparse
ray-octree intersection (section 4.3).  The paper does not fix the
arithmetic; this oracle defines it so that hit lists are reproducible bit for
bit:

Hit predicate H(ray, cell), every operation an IEEE binary32 operation rounded
to nearest even (numpy float32 scalar/array ops; no FMA, no flush to zero):

* inv_a = 1 / d_a per axis;
* inv_a finite:   t0 = (lo_a - o_a) * inv_a, t1 = (hi_a - o_a) * inv_a,
                  tn_a = min(t0, t1), tf_a = max(t0, t1);
* inv_a infinite: (d_a = +-0 or 1/d_a overflows) tn_a = -inf, tf_a = +inf if
                  lo_a <= o_a < hi_a (half-open), else tn_a = +inf, tf_a = -inf;
* t_in = max(tn_x, tn_y, tn_z) if that is > 0, else +0 (t_min = 0);
  t_out = min(tf_x, tf_y, tf_z);
* the ray hits the cell iff t_in < t_out (strict);
* a ray with a non-finite component or with d = 0 hits nothing.

Each plane value RN(RN(b - o) * inv) depends only on the plane b, and RN is
monotone, so a child's hit implies its parent's, hit intervals of distinct
leaves are disjoint, and ordering by t_in has no ties.  The hit list of a ray
is the first K occupied leaves in ascending t_in.
"""

from __future__ import annotations

import numpy as np

from .octree import Octree, morton_decode

F32 = np.float32


def valid_rays(o, d):
    o = np.asarray(o, F32)
    d = np.asarray(d, F32)
    return (np.all(np.isfinite(o), axis=1) & np.all(np.isfinite(d), axis=1)
            & np.any(d != 0, axis=1))


def reciprocal(d):
    """inv = RN32(1 / d) per component."""
    with np.errstate(divide="ignore", over="ignore"):
        return F32(1.0) / np.asarray(d, F32)


def slab(o, inv, lo, hi):
    """The FP32 predicate H for matched rows of o, inv, lo, hi (m, 3) float32.

    Returns (hit, t_in, t_out) with t values as float32.
    """
    o = np.asarray(o, F32)
    inv = np.asarray(inv, F32)
    lo = np.asarray(lo, F32)
    hi = np.asarray(hi, F32)
    with np.errstate(over="ignore", invalid="ignore"):
        t0 = (lo - o) * inv
        t1 = (hi - o) * inv
    tn = np.minimum(t0, t1)
    tf = np.maximum(t0, t1)
    finite = np.isfinite(inv)
    inside = (lo <= o) & (o < hi)
    inf = F32(np.inf)
    tn = np.where(finite, tn, np.where(inside, -inf, inf)).astype(F32)
    tf = np.where(finite, tf, np.where(inside, inf, -inf)).astype(F32)
    t_in = np.max(tn, axis=1)
    t_in = np.where(t_in > 0, t_in, F32(0.0)).astype(F32)
    t_out = np.min(tf, axis=1).astype(F32)
    return t_in < t_out, t_in, t_out


def cell_lohi32(level, ijk):
    """Exact FP32 bounds of cells (dyadic, so exact for level <= 23)."""
    h = 2.0 / (1 << level)
    lo = -1.0 + np.asarray(ijk, np.float64) * h
    return lo.astype(F32), (lo + h).astype(F32)


def _pack_hits(n_rays, K, ray, leaf, tin, tout):
    """Keep each ray's first K hits by ascending t_in."""
    hit_leaf = np.full((n_rays, K), -1, np.int32)
    hit_tin = np.zeros((n_rays, K), F32)
    hit_tout = np.zeros((n_rays, K), F32)
    count = np.zeros(n_rays, np.int32)
    if ray.size == 0:
        return hit_leaf, hit_tin, hit_tout, count
    order = np.lexsort((tin, ray))
    ray, leaf, tin, tout = ray[order], leaf[order], tin[order], tout[order]
    start = np.searchsorted(ray, ray, side="left")
    rank = np.arange(ray.size) - start
    keep = rank < K
    hit_leaf[ray[keep], rank[keep]] = leaf[keep]
    hit_tin[ray[keep], rank[keep]] = tin[keep]
    hit_tout[ray[keep], rank[keep]] = tout[keep]
    np.add.at(count, ray[keep], 1)
    return hit_leaf, hit_tin, hit_tout, count


def trace_hits(octree: Octree, o, d, K, chunk=1 << 16):
    """Hierarchical (level-synchronous) traversal, as in the sparse
    ray-octree intersection of section 4.3: test the root, then the children
    of every hit node, level by level, and sort the hit leaves by t_in.

    Returns hit_leaf (n, K) int32 (-1 padded), hit_tin, hit_tout (n, K)
    float32 (0 padded) and hit_count (n,) int32.
    """
    o = np.ascontiguousarray(o, F32)
    d = np.ascontiguousarray(d, F32)
    n = o.shape[0]
    out_leaf = np.full((n, K), -1, np.int32)
    out_tin = np.zeros((n, K), F32)
    out_tout = np.zeros((n, K), F32)
    out_cnt = np.zeros(n, np.int32)
    if octree.n_leaves == 0 or n == 0:
        return out_leaf, out_tin, out_tout, out_cnt
    L = octree.depth
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        oc, dc = o[s:e], d[s:e]
        inv = reciprocal(dc)
        ok = valid_rays(oc, dc)
        rays = np.nonzero(ok)[0]
        # level 0: the root cell
        nodes = np.zeros(rays.size, np.int64)
        lo, hi = cell_lohi32(0, np.zeros((rays.size, 3)))
        hit, tin, tout = slab(oc[rays], inv[rays], lo, hi)
        rays, nodes = rays[hit], nodes[hit]
        for l in range(L):
            first, last = octree.children(l, nodes)
            cnt = last - first
            rr = np.repeat(rays, cnt)
            base = np.repeat(first - np.cumsum(cnt) + cnt, cnt)
            child = base + np.arange(rr.size)
            ijk = morton_decode(octree.level_codes[l + 1][child], l + 1)
            lo, hi = cell_lohi32(l + 1, ijk)
            hit, tin, tout = slab(oc[rr], inv[rr], lo, hi)
            rays, nodes = rr[hit], child[hit]
            tin, tout = tin[hit], tout[hit]
        hl, ht0, ht1, hc = _pack_hits(e - s, K, rays, nodes.astype(np.int32), tin, tout)
        out_leaf[s:e], out_tin[s:e], out_tout[s:e], out_cnt[s:e] = hl, ht0, ht1, hc
    return out_leaf, out_tin, out_tout, out_cnt


def trace_hits_bruteforce(octree: Octree, o, d, K):
    """Flat enumeration: test every occupied leaf against every ray, sort by
    t_in, keep K.  Only for small scenes and ray counts."""
    o = np.ascontiguousarray(o, F32)
    d = np.ascontiguousarray(d, F32)
    n = o.shape[0]
    nl = octree.n_leaves
    if nl == 0 or n == 0:
        return _pack_hits(n, K, np.zeros(0, np.int64), np.zeros(0, np.int32),
                          np.zeros(0, F32), np.zeros(0, F32))
    inv = reciprocal(d)
    ok = valid_rays(o, d)
    lo, hi = cell_lohi32(octree.depth, octree.leaf_ijk)
    rr = np.repeat(np.arange(n), nl)
    ll = np.tile(np.arange(nl), n)
    hit, tin, tout = slab(o[rr], inv[rr], lo[ll], hi[ll])
    hit &= ok[rr]
    return _pack_hits(n, K, rr[hit], ll[hit].astype(np.int32), tin[hit], tout[hit])


def all_hits_count(octree: Octree, o, d):
    """Total number of occupied leaves each ray hits (no K cap)."""
    big = max(1, octree.n_leaves)
    _, _, _, cnt = trace_hits(octree, o, d, big)
    return cnt
