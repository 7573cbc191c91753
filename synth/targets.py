"""Analytic ground-truth colour and depth for ellipsoid/box scenes.

Stands in for the path-traced RTMV images: the first surface point hit along
each ray over all objects, shaded Lambertian with one directional light and a
per-object albedo, no ambient term and no shadows.  Misses are black with
depth 0.  Everything is FP64 on the FP32 rays the renderer consumes.
"""

from __future__ import annotations

import numpy as np

from .scenes import Box, Ellipsoid


def _hit_ellipsoid(e, o, d):
    # (o + t d - c)^T A (o + t d - c) = 1
    y = o - e.c
    Ad = d @ e.A
    Ay = y @ e.A
    a = np.sum(d * Ad, axis=1)
    b = 2.0 * np.sum(y * Ad, axis=1)
    c = np.sum(y * Ay, axis=1) - 1.0
    disc = b * b - 4 * a * c
    ok = disc >= 0
    sq = np.sqrt(np.where(ok, disc, 0.0))
    t0 = (-b - sq) / (2 * a)
    t1 = (-b + sq) / (2 * a)
    t = np.where(t0 > 0, t0, t1)
    ok &= t > 0
    p = o + np.where(ok, t, 0.0)[:, None] * d
    n = np.where(ok[:, None], (p - e.c) @ e.A, 0.0)
    return np.where(ok, t, np.inf), n


def _hit_box(bx, o, d):
    lo, hi = bx.bb_lo, bx.bb_hi
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        t0 = (lo - o) * inv
        t1 = (hi - o) * inv
    tn = np.minimum(t0, t1)
    tf = np.maximum(t0, t1)
    # axis-parallel rays: inside the slab means unconstrained
    par = ~np.isfinite(inv)
    inside = (o >= lo) & (o <= hi)
    tn = np.where(par, np.where(inside, -np.inf, np.inf), tn)
    tf = np.where(par, np.where(inside, np.inf, -np.inf), tf)
    tin = tn.max(axis=1)
    tout = tf.min(axis=1)
    ax = tn.argmax(axis=1)
    ok = (tin <= tout) & (tin > 0)
    t = np.where(ok, tin, np.inf)
    n = np.zeros_like(o)
    idx = np.arange(o.shape[0])
    n[idx, ax] = -np.sign(d[idx, ax])
    n = np.where(ok[:, None], n, 0.0)
    return t, n


def render_targets(objects, albedo, light, o, d):
    """rgb* (n, 3) and depth* (n,) as float32 for rays (o, d)."""
    o = np.asarray(o, np.float64)
    d = np.asarray(d, np.float64)
    n_rays = o.shape[0]
    best_t = np.full(n_rays, np.inf)
    best_n = np.zeros((n_rays, 3))
    best_k = np.full(n_rays, -1)
    for k, obj in enumerate(objects):
        if isinstance(obj, Ellipsoid):
            t, nrm = _hit_ellipsoid(obj, o, d)
        elif isinstance(obj, Box):
            t, nrm = _hit_box(obj, o, d)
        else:
            raise TypeError(type(obj))
        closer = t < best_t
        best_t = np.where(closer, t, best_t)
        best_n = np.where(closer[:, None], nrm, best_n)
        best_k = np.where(closer, k, best_k)
    hit = np.isfinite(best_t)
    nn = np.linalg.norm(best_n, axis=1, keepdims=True)
    nrm = best_n / np.where(nn > 0, nn, 1.0)
    shade = np.maximum(0.0, nrm @ np.asarray(light, np.float64))
    alb = np.asarray(albedo, np.float64)[np.maximum(best_k, 0)]
    rgb = np.where(hit[:, None], alb * shade[:, None], 0.0)
    depth = np.where(hit, best_t, 0.0)
    return rgb.astype(np.float32), depth.astype(np.float32)
