"""Checks of the synthetic input generators (they hold no method arithmetic;
these tests make sure the workloads have the stated shapes)."""

import numpy as np
import pytest

from oracle.octree import Octree
from synth import scenes
from synth.cameras import Camera
from synth.configs import get_workload, get_multi, tiny_workload
from synth.targets import render_targets


def test_workload0_shell_sizes():
    sc = get_workload("shell_d4").scene()
    # exact min/max-distance shell test on the 16^3 grid
    assert sc.leaf_ijk.shape[0] == 712
    assert sc.n_vertices == 1194
    assert sc.n_vertices == Octree(sc.leaf_ijk, 4).n_vertices


def test_workload1_occupancy_about_three_percent():
    sc = get_workload("ellipsoids_d7").scene()
    assert 0.025 < sc.fraction < 0.04
    assert sc.n_vertices == Octree(sc.leaf_ijk, 7).n_vertices


def test_seeded_reproducibility():
    a = tiny_workload(3, 5, 8, (8, 32, 32, 4), 4)
    b = tiny_workload(3, 5, 8, (8, 32, 32, 4), 4)
    np.testing.assert_array_equal(a.scene().leaf_ijk, b.scene().leaf_ijk)
    np.testing.assert_array_equal(a.features(), b.features())
    np.testing.assert_array_equal(a.params(), b.params())
    c = tiny_workload(4, 5, 8, (8, 32, 32, 4), 4)
    assert not np.array_equal(a.features()[:10], c.features()[:10])


def test_multi_workload_structure():
    m = get_multi(small=True)
    assert len(m.depths) == 8 and list(m.depths) == sorted(m.depths)
    counts = m.ray_counts()
    assert all(m.ray_lo <= c <= m.ray_hi for c in counts)
    full = get_multi()
    assert full.depths == (7, 8, 8, 9, 9, 10, 10, 10)
    assert all(0.005 <= f <= 0.03 for f in full.fractions)


def test_ellipsoid_cell_test_against_dense_sampling():
    rng = np.random.default_rng(0)
    e = scenes.random_ellipsoids(rng, 1, 0.2, 0.5)[0]
    level = 4
    h = 2.0 / 16
    cells = np.stack(np.meshgrid(*[np.arange(16)] * 3, indexing="ij"), -1).reshape(-1, 3)
    lo = -1.0 + cells * h
    qmin, qmax = e.qmin_qmax(lo, lo + h)
    g = np.linspace(0, 1, 9)
    pts = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    for c in rng.choice(cells.shape[0], 300, replace=False):
        p = lo[c] + pts * h
        qs = e.q(p - e.c)
        # sampled extremes bracket the exact ones (sampling can only miss)
        assert qs.min() >= qmin[c] - 1e-12
        assert qs.max() <= qmax[c] + 1e-12
        assert np.isclose(qs.max(), qmax[c])          # max at a corner
        assert qs.min() <= qmin[c] + 0.05 * (qmax[c] - qmin[c]) + 1e-9


def test_box_surface_rule():
    b = scenes.Box(np.zeros(3), np.full(3, 0.5))
    lo = np.array([[-0.25, -0.25, -0.25], [-0.6, -0.25, -0.25], [0.6, 0.6, 0.6]])
    hi = lo + 0.1
    assert b.test(lo, hi, "surface").tolist() == [False, True, False]
    assert b.test(lo, hi, "solid").tolist() == [True, True, False]


def test_camera_geometry():
    cam = Camera([0.0, -3.0, 0.0], 65, 65, 50.0)
    o, d = cam.rays()
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-6)
    c = 32 * 65 + 32                                  # centre pixel looks at the target
    np.testing.assert_allclose(d[c], [0.0, 1.0, 0.0], atol=1e-6)
    # corner pixel is half a pixel inside the 25-degree half angle
    t = np.tan(np.deg2rad(25.0)) * (1.0 - 1.0 / 65)
    assert np.isclose(abs(d[0, 0] / d[0, 1]), t, rtol=1e-5)
    assert d[0, 2] > 0                                 # row 0 is the top row


def test_targets_against_ray_marching():
    rng = np.random.default_rng(1)
    objs = scenes.random_ellipsoids(rng, 2, 0.2, 0.4) + scenes.random_boxes(rng, 1, 0.1, 0.3)
    albedo = rng.uniform(0, 1, (3, 3))
    light = np.array([0.0, 0.0, 1.0])
    cam = Camera([2.5, -2.0, 1.0], 24, 24, 50.0)
    o, d = cam.rays()
    rgb, depth = render_targets(objs, albedo, light, o, d)

    def inside(p):
        res = np.zeros(p.shape[0], bool)
        for ob in objs:
            if isinstance(ob, scenes.Ellipsoid):
                res |= ob.q(p - ob.c) <= 1.0
            else:
                res |= np.all(np.abs(p - ob.c) <= ob.e, axis=1)
        return res

    step = 2e-3
    ts = np.arange(0.0, 8.0, step)
    for r in range(o.shape[0]):
        p = o[r][None, :].astype(np.float64) + ts[:, None] * d[r][None, :].astype(np.float64)
        ins = inside(p)
        if ins.any():
            t_hit = ts[np.argmax(ins)]
            assert depth[r] > 0 and abs(depth[r] - t_hit) <= 2 * step, r
        else:
            assert depth[r] == 0 and np.all(rgb[r] == 0)
