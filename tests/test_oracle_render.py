"""Pins for the oracle's render, backward and loss (SVLF sections 4.1-4.3,
Eq. 3, section 4 footnote on optical thickness).

* trilinear interpolation: corners, centre, partition of unity, continuity
  across a shared face;
* MLP special cases with hand-computed outputs;
* closed-form single-voxel renders, telescoping with a constant decoder,
  empty scenes, compositing invariants;
* central finite differences of the loss for features and weights, and the
  conservation identity sum(grad_features) = sum over hits of dL/dx;
* the bfloat16 rounding against torch's float32 -> bfloat16 conversion.
"""

import numpy as np
import pytest

from oracle.octree import Octree
from oracle.render import (bf16_round, decoder_input_jacobian, interpolation_weights, loss, mlp_forward,
                           render, render_backward, render_backward_hit_magnitude,
                           render_backward_weight_scale, sigma_output_term_magnitude, split_params,
                           weight_sensitivity)
from oracle.trace import trace_hits
from synth.configs import param_count, tiny_workload, xavier_params
from tests.helpers import crafted_occupancy, random_rays


def _zero_mlp(widths, out_bias):
    p = np.zeros(param_count(widths))
    p[-4:] = out_bias
    return p


# ------------------------------------------------------------ interpolation

def test_trilinear_weights_corners_centre_unity():
    rng = np.random.default_rng(0)
    u = rng.uniform(0, 1, (50, 3))
    w = interpolation_weights(u)
    np.testing.assert_allclose(w.sum(axis=1), 1.0, rtol=0, atol=1e-15)
    assert np.all(w >= 0)
    for j in range(8):
        corner = np.array([[j & 1, (j >> 1) & 1, (j >> 2) & 1]], np.float64)
        e = np.zeros(8)
        e[j] = 1.0
        np.testing.assert_array_equal(interpolation_weights(corner)[0], e)
    np.testing.assert_array_equal(interpolation_weights(np.full((1, 3), 0.5))[0], np.full(8, 0.125))


def _render_one(oc, F, params, widths, o, d, K=4, **kw):
    hits = trace_hits(oc, o, d, K)
    return hits, render(oc, F, params, widths, o, d, hits, **kw)


def test_interpolation_at_corner_centre_and_shared_face():
    """Identity-like decoder exposes x: with W1 = I (C=4 -> 4 hidden) and a
    linear read-out of hidden unit 0 into o_3, sigma = relu(x_0)."""
    depth = 1
    oc = Octree([[0, 0, 0], [1, 0, 0]], depth)   # two leaves sharing face x=0
    C = 4
    widths = (C, 4, 4)
    p = np.zeros(param_count(widths))
    W = split_params(p, widths)
    W[0][0][:] = np.eye(4)
    W[1][0][3, 0] = 1.0
    rng = np.random.default_rng(2)
    F = rng.uniform(0.1, 1.0, (oc.n_vertices, C))
    # a ray along +x at y, z chosen so that the midpoint of each leaf
    # segment is at u = (0.5, uy, uz); compare x with direct weights
    uy, uz = 0.25, 0.75
    o = np.array([[-2.0, -1.0 + uy, -1.0 + uz]], np.float32)
    d = np.array([[1.0, 0.0, 0.0]], np.float32)
    hits, (rgb, depth_, acc, st) = _render_one(oc, F, p, widths, o, d)
    assert st.X.shape[0] == 2
    for hidx in range(2):
        leaf = hits[0][0, hidx]
        w = interpolation_weights(np.array([[0.5, uy, uz]]))[0]
        np.testing.assert_allclose(st.X[hidx], w @ F[oc.leaf_corners[leaf]], rtol=1e-14)
    # continuity: a point on the shared face (x = 0) interpolates the same
    # from both leaves: u_x = 1 in leaf 0 and u_x = 0 in leaf 1
    w0 = interpolation_weights(np.array([[1.0, uy, uz]]))[0]
    w1 = interpolation_weights(np.array([[0.0, uy, uz]]))[0]
    x0 = w0 @ F[oc.leaf_corners[0]]
    x1 = w1 @ F[oc.leaf_corners[1]]
    np.testing.assert_allclose(x0, x1, rtol=1e-14)


# ------------------------------------------------------------ MLP

def test_mlp_zero_weights_constant_output():
    widths = (8, 16, 16, 4)
    p = _zero_mlp(widths, [0.3, -1.0, 2.0, 0.7])
    X = np.random.default_rng(0).normal(size=(10, 8))
    out, _, _ = mlp_forward(p, widths, X)
    np.testing.assert_array_equal(out, np.tile([0.3, -1.0, 2.0, 0.7], (10, 1)))


def test_mlp_hand_computed():
    # 2 -> 2 -> 4 with W1 = [[1,-1],[2,1]], b1 = [0, -1]; x = (3, 1)
    # z1 = (2, 6), a1 = (2, 6); W2 rows pick: o = (a0, a1, a0 - a1, -a0) + b2
    widths = (2, 2, 4)
    p = np.array([1, -1, 2, 1, 0, -1,
                  1, 0, 0, 1, 1, -1, -1, 0, 0.5, 0, 0, 0], np.float64)
    out, acts, pres = mlp_forward(p, widths, np.array([[3.0, 1.0]]))
    np.testing.assert_array_equal(pres[0], [[2.0, 6.0]])
    np.testing.assert_array_equal(out, [[2.5, 6.0, -4.0, -2.0]])
    # negative hidden pre-activation is clamped: x = (-1, 0) -> z1 = (-1, -3)
    out, _, _ = mlp_forward(p, widths, np.array([[-1.0, 0.0]]))
    np.testing.assert_array_equal(out, [[0.5, 0.0, 0.0, 0.0]])


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("tau_mode", ["voxel", "direct", "world"])
def test_single_voxel_closed_form(tau_mode):
    depth = 2
    leaf = [1, 2, 1]
    oc = Octree([leaf], depth)
    h = 0.5
    widths = (4, 8, 4)
    z = np.array([0.2, -0.4, 0.6, 0.1])
    F = np.tile(z, (oc.n_vertices, 1))          # all corners equal -> x = z
    rng = np.random.default_rng(4)
    p = xavier_params(rng, widths).astype(np.float64)
    p[-4:] = [0.1, -0.2, 0.3, 0.9]               # make sigma > 0
    out, _, _ = mlp_forward(p, widths, z[None, :])
    c = 1.0 / (1.0 + np.exp(-out[0, :3]))
    sigma = max(out[0, 3], 0.0)
    assert sigma > 0
    lo = np.array([-1.0 + 1 * h, -1.0 + 2 * h, -1.0 + 1 * h])
    ctr = lo + h / 2
    # axis-aligned ray through the centre: dt = h
    o = np.array([[-3.0, ctr[1], ctr[2]]], np.float32)
    d = np.array([[1.0, 0.0, 0.0]], np.float32)
    _, (rgb, dep, acc, _) = _render_one(oc, F, p, widths, o, d, tau_mode=tau_mode)
    dt = h
    tau = {"voxel": sigma * dt / h, "direct": sigma, "world": sigma * dt}[tau_mode]
    a = 1.0 - np.exp(-tau)
    t_mid = (lo[0] - (-3.0)) + h / 2
    np.testing.assert_allclose(rgb[0], c * a, rtol=1e-12)
    np.testing.assert_allclose(acc[0], a, rtol=1e-12)
    np.testing.assert_allclose(dep[0], a * t_mid, rtol=1e-12)
    # main diagonal through the cell: dt = h (per unit of the unnormalised
    # direction (1,1,1)), so the voxel-mode tau is sigma
    o = (ctr - 2.0).astype(np.float32)[None, :]
    d = np.array([[1.0, 1.0, 1.0]], np.float32)
    _, (rgb, dep, acc, _) = _render_one(oc, F, p, widths, o, d, tau_mode=tau_mode)
    tau = {"voxel": sigma, "direct": sigma, "world": sigma * h}[tau_mode]
    np.testing.assert_allclose(acc[0], 1.0 - np.exp(-tau), rtol=1e-12)


def test_viewdir_closed_form():
    """View-direction input: a decoder whose colour channel 0 is
    sigmoid(relu(d_x)) and whose sigma is a constant gives, for two rays
    crossing the same voxel in different directions, colours that differ
    exactly as the closed form says; zero weights on d reproduce the render
    without the direction input."""
    depth = 2
    oc = Octree([[1, 2, 1]], depth)
    C = 4
    widths = (C + 3, 4, 4)
    F = np.tile([0.3, -0.1, 0.2, 0.5], (oc.n_vertices, 1))
    p = np.zeros(param_count(widths))
    W1 = p[:4 * 7].reshape(4, 7)
    W1[0, C + 0] = 1.0                            # hidden 0 = relu(d_x)
    off = 4 * 7 + 4
    W2 = p[off:off + 16].reshape(4, 4)
    W2[0, 0] = 1.0                                # o_0 = hidden 0
    p[off + 16:off + 20] = [0.0, 0.0, 0.0, 2.0]   # sigma = 2
    ctr = np.array([-0.25, 0.25, -0.25])
    dirs = np.array([[0.6, 0.8, 0.0], [-0.28, 0.96, 0.0]], np.float32)
    o = (ctr - 3.0 * dirs).astype(np.float32)
    _, (rgb, dep, acc, st) = _render_one(oc, F, p, widths, o, dirs, viewdir=True)
    a = acc
    assert np.all(a > 0)
    dx = dirs[:, 0].astype(np.float64)
    np.testing.assert_allclose(rgb[:, 0], a / (1.0 + np.exp(-np.maximum(dx, 0.0))), rtol=1e-12)
    np.testing.assert_allclose(rgb[:, 1], 0.5 * a, rtol=1e-12)
    assert rgb[0, 0] != rgb[1, 0]
    # the same decoder with the direction weights removed is the plain render
    widths0 = (C, 4, 4)
    p0 = np.concatenate([np.zeros(4 * 4 + 4), p[off:]])
    _, (rgb0, dep0, acc0, _) = _render_one(oc, F, p0, widths0, o, dirs)
    p_vd = p.copy()
    W1[0, C] = 0.0
    _, (rgb1, dep1, acc1, _) = _render_one(oc, F, p, widths, o, dirs, viewdir=True)
    np.testing.assert_array_equal(rgb1, rgb0)
    np.testing.assert_array_equal(dep1, dep0)
    np.testing.assert_array_equal(acc1, acc0)
    # the direction takes no gradient and the feature gradient keeps C columns
    gF, gp = render_backward(st, np.ones((2, 3)), np.zeros(2))
    assert gF.shape == (oc.n_vertices, C)
    with pytest.raises(ValueError):
        _render_one(oc, F, p_vd, widths, o, dirs)     # width C + 3 without viewdir


def test_telescoping_constant_decoder():
    """Constant decoder: acc = 1 - exp(-sigma sum(dt)/h), rgb = c acc."""
    depth = 3
    oc = Octree(crafted_occupancy("random30", depth, seed=1), depth)
    widths = (4, 8, 4)
    p = _zero_mlp(widths, [0.5, -0.5, 1.0, 0.8])
    F = np.random.default_rng(1).normal(size=(oc.n_vertices, 4))
    o, d = random_rays(np.random.default_rng(5), 200)
    K = 64
    hits, (rgb, dep, acc, _) = _render_one(oc, F, p, widths, o, d, K=K)
    h = 2.0 / 8
    dt = np.where(hits[0] >= 0, hits[2].astype(np.float64) - hits[1], 0.0).sum(axis=1)
    exp_acc = 1.0 - np.exp(-0.8 * dt / h)
    np.testing.assert_allclose(acc, exp_acc, rtol=1e-12, atol=1e-15)
    c = 1.0 / (1.0 + np.exp(-np.array([0.5, -0.5, 1.0])))
    np.testing.assert_allclose(rgb, exp_acc[:, None] * c[None, :], rtol=1e-12, atol=1e-15)


def test_empty_scene_and_missing_rays():
    widths = (4, 8, 4)
    p = _zero_mlp(widths, [1, 1, 1, 1])
    oc = Octree(np.zeros((0, 3)), 2)
    o, d = random_rays(np.random.default_rng(0), 20)
    F = np.zeros((0, 4))
    hits, (rgb, dep, acc, st) = _render_one(oc, F, p, widths, o, d)
    assert np.all(hits[3] == 0)
    assert np.all(rgb == 0) and np.all(dep == 0) and np.all(acc == 0)
    gF, gp = render_backward(st, np.ones((20, 3)), np.ones(20), np.ones(20))
    assert gF.shape == (0, 4) and np.all(gp == 0)


def test_compositing_invariants():
    w = tiny_workload(3, 4, 8, (8, 16, 16, 4), 6)
    sc = w.scene()
    oc = Octree(sc.leaf_ijk, sc.depth)
    F = w.features().astype(np.float64) * 20.0      # large sigma somewhere
    p = w.params().astype(np.float64)
    p[-1] = 2.0
    o, d = random_rays(np.random.default_rng(9), 300)
    hits, (rgb, dep, acc, st) = _render_one(oc, F, p, w.widths, o, d, K=6)
    T = st.T
    assert np.all((T >= 0) & (T <= 1))
    assert np.all(np.diff(T, axis=1) <= 1e-15)
    np.testing.assert_allclose(acc, st.w.sum(axis=1), rtol=1e-14)
    assert np.all((acc >= 0) & (acc <= 1))
    assert np.all(rgb >= 0) and np.all(rgb <= acc[:, None] + 1e-15)
    cnt = hits[3]
    has = cnt > 0
    first_in = hits[1][has, 0].astype(np.float64)
    last_out = hits[2][has, cnt[has] - 1].astype(np.float64)
    assert np.all(dep[has] >= acc[has] * first_in - 1e-12)
    assert np.all(dep[has] <= acc[has] * last_out + 1e-12)
    assert np.all(dep[~has] == 0)


# ------------------------------------------------------------ gradients

def _fd_setup(seed, tau_mode="voxel", bf16=False, viewdir=False):
    w = tiny_workload(seed, 3, 8, (8, 16, 16, 4), 4, n_obj=2)
    sc = w.scene()
    oc = Octree(sc.leaf_ijk, sc.depth)
    F = w.features().astype(np.float64)
    p = w.params().astype(np.float64)
    if viewdir:
        w.widths = (11, 16, 16, 4)
        p = xavier_params(np.random.default_rng(seed + 100), w.widths).astype(np.float64)
    p[-1] = 0.5                                   # sigma mostly positive
    rng = np.random.default_rng(seed)
    o, d = random_rays(rng, 64, inside_frac=0.1, axis_frac=0.0)
    hits = trace_hits(oc, o, d, 4)
    rgb_t = rng.uniform(0, 1, (64, 3))
    dep_t = rng.uniform(0, 4, 64)
    return oc, F, p, w.widths, o, d, hits, rgb_t, dep_t


def _loss_at(oc, F, p, widths, o, d, hits, rgb_t, dep_t, tau_mode, viewdir=False):
    rgb, dep, acc, st = render(oc, F, p, widths, o, d, hits, tau_mode=tau_mode, viewdir=viewdir)
    return loss(rgb, dep, rgb_t, dep_t)[0], st, rgb, dep


def _pattern(st, dep, dep_t):
    """Which side of every kink the evaluation is on (ReLU inputs, the
    sigma ReLU and the L1 residual)."""
    return np.concatenate([np.concatenate([z.ravel() > 0 for z in st.pres]),
                           st.out[:, 3] > 0, dep - dep_t > 0])


@pytest.mark.parametrize("tau_mode,viewdir", [("voxel", False), ("world", False), ("voxel", True)])
def test_gradients_against_central_differences(tau_mode, viewdir):
    oc, F, p, widths, o, d, hits, rgb_t, dep_t = _fd_setup(12, tau_mode, viewdir=viewdir)
    L0, st, rgb, dep = _loss_at(oc, F, p, widths, o, d, hits, rgb_t, dep_t, tau_mode, viewdir)
    base = _pattern(st, dep, dep_t)
    _, g_rgb, g_dep = loss(rgb, dep, rgb_t, dep_t)
    gF, gp = render_backward(st, g_rgb, g_dep)
    assert np.count_nonzero(gF) > 0

    def fd_of(Fx_p, Fx_m, px_p, px_m, eps):
        Lp, stp, _, dp = _loss_at(oc, Fx_p, px_p, widths, o, d, hits, rgb_t, dep_t, tau_mode, viewdir)
        Lm, stm, _, dm = _loss_at(oc, Fx_m, px_m, widths, o, d, hits, rgb_t, dep_t, tau_mode, viewdir)
        # an evaluation that straddles a kink is not a derivative: skip it
        if not (np.array_equal(_pattern(stp, dp, dep_t), base)
                and np.array_equal(_pattern(stm, dm, dep_t), base)):
            return None
        return (Lp - Lm) / (2 * eps)

    def floor(eps):
        return 64 * np.finfo(np.float64).eps * abs(L0) / eps

    rng = np.random.default_rng(0)
    touched = np.unique(st.corners)
    checked = skipped = 0
    for idx in rng.choice(touched.size, min(60, touched.size), replace=False):
        v = touched[idx]
        c = rng.integers(0, F.shape[1])
        eps = 1e-5 * max(1.0, abs(F[v, c]))
        Fp = F.copy(); Fp[v, c] += eps
        Fm = F.copy(); Fm[v, c] -= eps
        fd = fd_of(Fp, Fm, p, p, eps)
        if fd is None:
            skipped += 1
            continue
        checked += 1
        # FD of an FP64 loss: relative 1e-6 plus the round-off floor of
        # the difference quotient (a few ulps of |L| over eps)
        assert abs(fd - gF[v, c]) <= 1e-6 * abs(fd) + floor(eps), (v, c, fd, gF[v, c])
    for k in rng.choice(p.size, 80, replace=False):
        eps = 1e-5 * max(1.0, abs(p[k]))
        pp = p.copy(); pp[k] += eps
        pm = p.copy(); pm[k] -= eps
        fd = fd_of(F, F, pp, pm, eps)
        if fd is None:
            skipped += 1
            continue
        checked += 1
        assert abs(fd - gp[k]) <= 1e-6 * abs(fd) + floor(eps), (k, fd, gp[k])
    assert skipped <= 0.1 * (checked + skipped)


def test_acc_gradient_and_conservation():
    oc, F, p, widths, o, d, hits, _, _ = _fd_setup(12)
    rgb, dep, acc, st = render(oc, F, p, widths, o, d, hits)
    rng = np.random.default_rng(1)
    g_acc = rng.normal(size=acc.shape)
    gF, gp = render_backward(st, np.zeros_like(rgb), np.zeros_like(dep), g_acc)
    k = 5
    eps = 1e-6
    for v in np.unique(st.corners)[:k]:
        Fp = F.copy(); Fp[v, 0] += eps
        Fm = F.copy(); Fm[v, 0] -= eps
        ap = render(oc, Fp, p, widths, o, d, hits)[2]
        am = render(oc, Fm, p, widths, o, d, hits)[2]
        fd = float(g_acc @ (ap - am)) / (2 * eps)
        assert abs(fd - gF[v, 0]) <= 1e-6 * max(1e-3, abs(fd))
    # conservation: trilinear weights of each hit sum to 1, so the total
    # feature gradient equals the total input gradient over hits
    g_rgb = rng.normal(size=rgb.shape)
    g_dep = rng.normal(size=dep.shape)
    gF, _ = render_backward(st, g_rgb, g_dep)
    # recover sum over hits of dL/dx by a second path: scale all features
    # by (1 + e) shifts x by e x, so dL/de = sum_hits <dL/dx, x>
    e = 1e-6
    Lp = float(np.sum(g_rgb * render(oc, F * (1 + e), p, widths, o, d, hits)[0])
               + g_dep @ render(oc, F * (1 + e), p, widths, o, d, hits)[1])
    Lm = float(np.sum(g_rgb * render(oc, F * (1 - e), p, widths, o, d, hits)[0])
               + g_dep @ render(oc, F * (1 - e), p, widths, o, d, hits)[1])
    fd = (Lp - Lm) / (2 * e)
    assert abs(fd - float(np.sum(gF * F))) <= 1e-6 * max(1.0, abs(fd))


def test_hit_magnitude_bounds_every_entry_and_is_homogeneous():
    """The per-hit contribution scale bounds every gradient entry (triangle
    inequality), also where the hits' terms cancel, and scales linearly with
    the upstream gradients."""
    oc, F, p, widths, o, d, hits, _, _ = _fd_setup(12)
    rgb, dep, acc, st = render(oc, F, p, widths, o, d, hits)
    rng = np.random.default_rng(3)
    ups = [rng.normal(size=rgb.shape), rng.normal(size=dep.shape), rng.normal(size=acc.shape)]
    gF, gp = render_backward(st, *ups)
    mF, mp = render_backward_hit_magnitude(st, *ups)
    assert np.all(mF >= np.abs(gF)) and np.all(mp >= np.abs(gp))
    assert np.all(mF[np.any(gF != 0, axis=1)] > 0)
    mF2, mp2 = render_backward_hit_magnitude(st, *[2 * u for u in ups])
    np.testing.assert_allclose(mF2, 2 * mF, rtol=1e-14, atol=0)
    np.testing.assert_allclose(mp2, 2 * mp, rtol=1e-14, atol=0)
    # the sign of the upstream gradients does not matter
    mF3, mp3 = render_backward_hit_magnitude(st, *[-u for u in ups])
    np.testing.assert_allclose(mF3, mF, rtol=1e-14, atol=0)
    np.testing.assert_allclose(mp3, mp, rtol=1e-14, atol=0)


def test_hit_magnitude_of_one_hit():
    """One ray with one hit: every entry receives a single contribution, so
    the scale is |gradient| plus the largest |gradient| of the entry's group
    (the vertex row; the layer's weights; the layer's biases), both read off
    the oracle's gradient itself."""
    oc, F, p, widths, o, d, _, _, _ = _fd_setup(12)
    hits = trace_hits(oc, o, d, 1)
    r = int(np.nonzero(hits[3] > 0)[0][0])
    h1 = tuple(x[r:r + 1] for x in hits)
    rgb, dep, acc, st = render(oc, F, p, widths, o[r:r + 1], d[r:r + 1], h1)
    assert st.X.shape[0] == 1
    ups = [np.array([[0.3, -1.2, 0.7]]), np.array([0.4]), np.array([-0.9])]
    gF, gp = render_backward(st, *ups)
    mF, mp = render_backward_hit_magnitude(st, *ups)
    exp_F = np.abs(gF) + np.abs(gF).max(axis=1, keepdims=True)
    np.testing.assert_allclose(mF, exp_F, rtol=1e-13, atol=0)
    exp_p, off = [], 0
    for fi, fo in zip(widths[:-1], widths[1:]):
        gW = np.abs(gp[off:off + fi * fo])
        gb = np.abs(gp[off + fi * fo:off + fi * fo + fo])
        exp_p += [gW + gW.max(), gb + gb.max()]
        off += fi * fo + fo
    np.testing.assert_allclose(mp, np.concatenate(exp_p), rtol=1e-13, atol=0)


def test_hit_magnitude_adds_over_cancelling_hits():
    """The same rays twice with opposite upstream gradients: the gradients
    cancel exactly, the scale is twice that of one copy (it adds over hits,
    whatever their signs)."""
    oc, F, p, widths, o, d, hits, _, _ = _fd_setup(12)
    rng = np.random.default_rng(5)
    ups = [rng.normal(size=(o.shape[0], 3)), rng.normal(size=o.shape[0]), rng.normal(size=o.shape[0])]
    _, _, _, st1 = render(oc, F, p, widths, o, d, hits)
    m1F, m1p = render_backward_hit_magnitude(st1, *ups)
    o2, d2 = np.concatenate([o, o]), np.concatenate([d, d])
    h2 = tuple(np.concatenate([x, x]) for x in hits)
    _, _, _, st2 = render(oc, F, p, widths, o2, d2, h2)
    ups2 = [np.concatenate([u, -u]) for u in ups]
    gF, gp = render_backward(st2, *ups2)
    m2F, m2p = render_backward_hit_magnitude(st2, *ups2)
    assert np.abs(gF).max() <= 1e-15 * np.abs(m2F).max() and np.abs(gp).max() <= 1e-15 * np.abs(m2p).max()
    np.testing.assert_allclose(m2F, 2 * m1F, rtol=1e-13, atol=0)
    np.testing.assert_allclose(m2p, 2 * m1p, rtol=1e-13, atol=0)
    assert m1F.max() > 0 and m1p.max() > 0


def test_conditioned_magnitude_bounds_and_contains_the_plain_one():
    """The conditioned scale of the feature entries bounds every entry, is
    at least the plain one (|J_k| |g_k| sums dominate |sum J_k g_k|), scales
    linearly with the upstream gradients and ignores their sign; the
    decoder-parameter scale is unchanged."""
    oc, F, p, widths, o, d, hits, _, _ = _fd_setup(12)
    rgb, dep, acc, st = render(oc, F, p, widths, o, d, hits)
    rng = np.random.default_rng(3)
    ups = [rng.normal(size=rgb.shape), rng.normal(size=dep.shape), rng.normal(size=acc.shape)]
    gF, _ = render_backward(st, *ups)
    mF, mp = render_backward_hit_magnitude(st, *ups)
    cF, cp = render_backward_hit_magnitude(st, *ups, conditioned=True)
    assert np.all(cF >= np.abs(gF)) and np.all(cF >= mF * (1 - 1e-12))
    np.testing.assert_array_equal(cp, mp)
    cF2, _ = render_backward_hit_magnitude(st, *[-2 * u for u in ups], conditioned=True)
    np.testing.assert_allclose(cF2, 2 * cF, rtol=1e-14, atol=0)


def test_decoder_input_jacobian_against_finite_differences():
    oc, F, p, widths, o, d, hits, _, _ = _fd_setup(12)
    _, _, _, st = render(oc, F, p, widths, o, d, hits)
    J = decoder_input_jacobian(st)
    X = st.X[:20]
    eps = 1e-6
    for c in range(st.C):
        e = np.zeros_like(X)
        e[:, c] = eps
        fd = (mlp_forward(p, widths, X + e)[0] - mlp_forward(p, widths, X - e)[0]) / (2 * eps)
        np.testing.assert_allclose(J[:20, :, c], fd, rtol=1e-6, atol=1e-8)


def test_sigma_term_magnitude_one_hit_and_cancellation():
    """One hit with only an opacity gradient: dL/dtau is a single term, so G
    equals |dL/do_3| and the conditioned scale equals the plain one.  Upstream
    gradients chosen so that the first hit's dL/dtau cancels exactly: its
    dL/do_3 is zero but G is not (another evaluation of the same terms is off
    by their size)."""
    oc, F, p, widths, o, d, _, _, _ = _fd_setup(12)
    hits = trace_hits(oc, o, d, 1)
    r = int(np.nonzero(hits[3] > 0)[0][0])
    h1 = tuple(x[r:r + 1] for x in hits)
    _, _, _, st = render(oc, F, p, widths, o[r:r + 1], d[r:r + 1], h1)
    assert st.out[0, 3] > 0
    ups = [np.zeros((1, 3)), np.zeros(1), np.array([-0.7])]
    T_next = st.T[0, 0] * np.exp(-st.tau[0, 0])
    G = sigma_output_term_magnitude(st, *ups)
    np.testing.assert_allclose(G, [0.7 * T_next * st.dtau[0]], rtol=1e-14)
    mF, _ = render_backward_hit_magnitude(st, *ups)
    cF, _ = render_backward_hit_magnitude(st, *ups, conditioned=True)
    np.testing.assert_allclose(cF, mF, rtol=1e-12, atol=0)
    # a ray with several hits; g_acc solves dL/dtau = 0 for its first hit
    hits = trace_hits(oc, o, d, 4)
    r = int(np.nonzero(hits[3] >= 3)[0][0])
    h1 = tuple(x[r:r + 1] for x in hits)
    _, _, _, st = render(oc, F, p, widths, o[r:r + 1], d[r:r + 1], h1)
    g_rgb = np.array([[0.5, -0.3, 0.8]])
    T_next = st.T[0] * np.exp(-st.tau[0])
    wc = st.w[0][:, None] * st.col[0]
    S_c = wc.sum(axis=0) - np.cumsum(wc, axis=0)
    S_a = st.w[0].sum() - np.cumsum(st.w[0])
    num = np.sum(g_rgb[0] * (T_next[0] * st.col[0, 0] - S_c[0]))
    ups = [g_rgb, np.zeros(1), np.array([-num / (T_next[0] - S_a[0])])]
    from oracle.render import _backward_per_hit
    per_layer, _ = _backward_per_hit(st, *ups)
    g3 = per_layer[-1][0][:, 3]
    G = sigma_output_term_magnitude(st, *ups)
    assert st.out[0, 3] > 0 and G[0] > 0 and abs(g3[0]) <= 1e-12 * G[0]
    assert np.all(G >= np.abs(g3) * (1 - 1e-12))


def test_weight_sensitivity_against_finite_differences_and_closed_forms():
    """D_j = sum over axes of |d w_j / d u_a| of the trilinear weights: central
    differences of the weights at random points, 3/4 for every corner at the
    cell centre, and (3, 1, 1, 0, 1, 0, 0, 0) at the corner u = 0."""
    rng = np.random.default_rng(0)
    u = rng.uniform(0.05, 0.95, (200, 3))
    D = weight_sensitivity(u)
    fd = np.zeros_like(D)
    for a in range(3):
        e = np.zeros(3)
        e[a] = 1e-6
        fd += np.abs((interpolation_weights(u + e) - interpolation_weights(u - e)) / 2e-6)
    np.testing.assert_allclose(D, fd, rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(weight_sensitivity(np.full((1, 3), 0.5)), 0.75, rtol=0, atol=1e-15)
    np.testing.assert_array_equal(weight_sensitivity(np.zeros((1, 3)))[0], [3, 1, 1, 0, 1, 0, 0, 0])


def test_weight_scale_of_one_hit_and_over_cancelling_hits():
    """One ray with one hit: a corner row's weight scale is D_j |dL/dx| with
    dL/dx = gradient row / w_j (read off the gradient).  The same rays twice
    with opposite upstream gradients: the scale doubles."""
    oc, F, p, widths, o, d, _, _, _ = _fd_setup(12)
    hits = trace_hits(oc, o, d, 1)
    r = int(np.nonzero(hits[3] > 0)[0][0])
    h1 = tuple(x[r:r + 1] for x in hits)
    _, _, _, st = render(oc, F, p, widths, o[r:r + 1], d[r:r + 1], h1)
    ups = [np.array([[0.3, -1.2, 0.7]]), np.array([0.4]), np.array([-0.9])]
    gF, _ = render_backward(st, *ups)
    Mw = render_backward_weight_scale(st, *ups)
    corners = st.corners[0]
    wj = interpolation_weights(st.u)[0]
    Dj = weight_sensitivity(st.u)[0]
    assert np.all(wj > 1e-6)
    np.testing.assert_allclose(Mw[corners], Dj[:, None] * np.abs(gF[corners]) / wj[:, None], rtol=1e-10)
    assert np.all(np.delete(Mw, corners, axis=0) == 0)
    # additivity
    oc, F, p, widths, o, d, hits, _, _ = _fd_setup(12)
    rng = np.random.default_rng(5)
    ups = [rng.normal(size=(o.shape[0], 3)), rng.normal(size=o.shape[0]), rng.normal(size=o.shape[0])]
    _, _, _, st1 = render(oc, F, p, widths, o, d, hits)
    m1 = render_backward_weight_scale(st1, *ups)
    h2 = tuple(np.concatenate([x, x]) for x in hits)
    _, _, _, st2 = render(oc, F, p, widths, np.concatenate([o, o]), np.concatenate([d, d]), h2)
    m2 = render_backward_weight_scale(st2, *[np.concatenate([u_, -u_]) for u_ in ups])
    np.testing.assert_allclose(m2, 2 * m1, rtol=1e-13, atol=0)
    assert m1.max() > 0


def test_loss_gradient_closed_form():
    rgb = np.array([[0.5, 0.2, 0.1], [0.0, 1.0, 0.3]])
    rgb_t = np.array([[0.4, 0.2, 0.3], [0.0, 0.5, 0.3]])
    dep = np.array([2.0, 1.0])
    dep_t = np.array([1.5, 1.0])
    L, gr, gd = loss(rgb, dep, rgb_t, dep_t, 0.1)
    assert np.isclose(L, (0.01 + 0.04 + 0.25) / 6 + 0.1 * 0.5 / 2, rtol=1e-15)
    np.testing.assert_allclose(gr, 2 * (rgb - rgb_t) / 6, rtol=1e-15)
    np.testing.assert_array_equal(gd, [0.05, 0.0])


# ------------------------------------------------------------ bfloat16

def test_bf16_round_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.integers(-30, 30, 5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3e-39, -1e-40]])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(bf16_round(x32.astype(np.float64)), ref.astype(np.float64))


def _decoder_fp32_accumulation(p, widths, X, hidden=bf16_round, round_weights=True, serial=False):
    """A BF16 decoder as a device would run it: bfloat16 operands, FP32 dot
    products (numpy's FP32 matmul, or one product at a time in reverse order
    with ``serial``), ``hidden`` applied to each ReLU output."""
    from oracle.render import split_params
    a = np.float32(bf16_round(np.asarray(X, np.float64)))
    layers = split_params(p, widths)
    for li, (W, b) in enumerate(layers):
        Wr = np.float32(bf16_round(W) if round_weights else W)
        if serial:
            z = np.zeros((a.shape[0], W.shape[0]), np.float32)
            for k in reversed(range(W.shape[1])):
                z = z + a[:, k:k + 1] * Wr[:, k][None, :]
            z = z + np.float32(b)
        else:
            z = a @ Wr.T + np.float32(b)
        if li == len(layers) - 1:
            return z.astype(np.float64)
        a = np.float32(hidden(np.maximum(z.astype(np.float64), 0.0)))


def _bf16_truncate(v):
    m, e = np.frexp(v)
    s = np.ldexp(1.0, 8 - np.maximum(e, -125))
    return np.trunc(v * s) / s


@pytest.mark.parametrize("widths", [(8, 32, 32, 4), (32, 64, 64, 64, 4)])
def test_bf16_decoder_bound_holds_for_fp32_sums_and_catches_rounding_mistakes(widths):
    """The per-entry bound the BF16 decoder parity test applies: met by FP32
    accumulation in two summation orders, broken on most entries by hidden
    activations truncated instead of rounded, left unrounded, or by weights
    left in FP32."""
    from tests.gpu_cases import bf16_decoder_bound
    rng = np.random.default_rng(5)
    p = xavier_params(rng, widths).astype(np.float64)
    X = rng.normal(0, 0.5, (2000, widths[0])).astype(np.float32).astype(np.float64)
    ref, bound = bf16_decoder_bound(p, widths, X)
    np.testing.assert_array_equal(ref, mlp_forward(p, widths, X, bf16=True)[0])
    assert np.median(bound) < 2e-4 * np.abs(ref).max()
    for serial in (False, True):
        assert np.all(np.abs(_decoder_fp32_accumulation(p, widths, X, serial=serial) - ref) <= bound)
    for kw in ({"hidden": _bf16_truncate}, {"hidden": lambda v: v}, {"round_weights": False}):
        out = _decoder_fp32_accumulation(p, widths, X, **kw)
        assert np.mean(np.abs(out - ref) > bound) > 0.5, kw


def _render_fp32_emulation(st, F, mistake=None):
    """The BF16 render as a device computes it, emulated in float32 on the
    oracle's hits: FP32 cell weights and interpolation of the bfloat16 rows,
    the decoder with FP32 sums (bfloat16 operands), FP32 sigmoid / exp and
    Eq. 3 with a running transmittance.  ``mistake`` plants one error."""
    f32 = np.float32
    Fb = f32(bf16_round(np.asarray(F, np.float64)))
    u = f32(st.u)
    one = f32(1.0)
    wx = [one - u[:, 0], u[:, 0]]
    wy = [one - u[:, 1], u[:, 1]]
    wz = [one - u[:, 2], u[:, 2]]
    X = np.zeros((u.shape[0], Fb.shape[1]), f32)
    for j in range(8):
        wj = (wx[j & 1] * wy[(j >> 1) & 1]) * wz[j >> 2]
        X = X + wj[:, None] * Fb[st.corners[:, j]]
    if mistake == "unrounded input":
        o = _decoder_no_input_rounding(st.params, st.widths, X.astype(np.float64))
    elif mistake == "truncated hidden":
        o = _decoder_fp32_accumulation(st.params, st.widths, X.astype(np.float64), hidden=_bf16_truncate)
    else:
        o = _decoder_fp32_accumulation(st.params, st.widths, X.astype(np.float64))
    o = f32(o)
    c = one / (one + np.exp(-o[:, :3]))
    tau = np.maximum(o[:, 3], f32(0.0)) * f32(st.dtau)
    e = np.exp(-tau)
    alpha = -np.expm1(-tau)
    n, K = st.n, st.K
    rgb = np.zeros((n, 3), f32)
    dep = np.zeros(n, f32)
    acc = np.zeros(n, f32)
    T = np.ones(n, f32)
    tm = f32(st.tmid)
    for k in range(K):
        sel = st.slot_i == k
        ri = st.ray_i[sel]
        w = T[ri] * (e[sel] if mistake == "alpha from transmittance" else alpha[sel])
        rgb[ri] += w[:, None] * c[sel]
        dep[ri] += w * tm[ri, k]
        acc[ri] += w
        T[ri] = T[ri] * e[sel]
    return rgb.astype(np.float64), dep.astype(np.float64), acc.astype(np.float64)


def _decoder_no_input_rounding(p, widths, X):
    a = np.float32(X)
    layers = split_params(p, widths)
    for li, (W, b) in enumerate(layers):
        z = a @ np.float32(bf16_round(W)).T + np.float32(b)
        if li == len(layers) - 1:
            return z.astype(np.float64)
        a = np.float32(bf16_round(np.maximum(z.astype(np.float64), 0.0)))


def test_bf16_render_bound_holds_for_fp32_emulation_and_catches_mistakes():
    """The per-ray bound of the BF16 render parity test: met by a float32
    emulation of the device's arithmetic on several scenes, broken by an
    input left unrounded, by truncated hidden activations and by a wrong
    opacity in Eq. 3."""
    from tests.gpu_cases import bf16_render_bound
    for seed in (12, 13, 14):
        oc, F, p, widths, o, d, hits, _, _ = _fd_setup(seed)
        p = p.copy()
        p[-1] = 1.5
        rgb, dep, acc, st = render(oc, F, p, widths, o, d, hits, bf16=True)
        drgb, ddep, dacc = bf16_render_bound(st, F)
        assert np.median(drgb[acc > 0]) < 1e-3
        er, ed, ea = _render_fp32_emulation(st, F)
        assert np.all(np.abs(er - rgb) <= drgb), seed
        assert np.all(np.abs(ed - dep) <= ddep), seed
        assert np.all(np.abs(ea - acc) <= dacc), seed
        hit = acc > 0
        for m in ("unrounded input", "truncated hidden", "alpha from transmittance"):
            mr, md, ma = _render_fp32_emulation(st, F, mistake=m)
            bad = np.any(np.abs(mr - rgb) > drgb, axis=1) | (np.abs(ma - acc) > dacc)
            assert np.mean(bad[hit]) > 0.3, (seed, m, np.mean(bad[hit]))
