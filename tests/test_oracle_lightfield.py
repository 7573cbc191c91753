"""Pins for the two-decoder light-field oracle (SVLF sections 4.1-4.3):
closed forms of the bounding-sphere ray parameterisation, of where each
decoder reads its features (x1, x2, the surface point between them), of
the surface-point depth, finite differences of the loss through every
parameter and feature (including the path eta -> x_s -> psi), and
conservation identities of the feature gradients."""

import numpy as np
import pytest

from oracle.lightfield import (n_params, render_lf, render_lf_backward, render_lf_backward_hit_magnitude,
                               render_lf_backward_weight_scale, sphere_param, weight_derivatives, widths_of)
from oracle.octree import Octree
from oracle.render import loss
from oracle.trace import trace_hits
from synth.configs import tiny_workload, xavier_params
from tests.helpers import random_rays


def _layers_flat(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def _zeros(widths):
    return [(np.zeros((b, a)), np.zeros(b)) for a, b in zip(widths[:-1], widths[1:])]


def _one_voxel():
    depth = 2
    oc = Octree([[1, 2, 1]], depth)
    h = 0.5
    lo = np.array([-0.5, 0.0, -0.5])
    return oc, h, lo


def _vertex_pos(oc, h):
    """World position of every vertex (rank of the Morton code of the
    (L+1)-bit corner lattice; corners of leaf 0 in corner order)."""
    pos = np.zeros((oc.n_vertices, 3))
    for j in range(8):
        v = oc.leaf_corners[0, j]
        off = np.array([j & 1, (j >> 1) & 1, j >> 2])
        pos[v] = -1.0 + (oc.leaf_ijk[0] + off) * h
    return pos


# ------------------------------------------------------------ ray parameterisation

def test_sphere_param_closed_forms():
    lo = np.array([[0.0, 0.0, 0.0]])
    h = 0.5
    c = lo + 0.25
    # axis ray through the centre: the sphere points are c -/+ R e_x
    o = c + np.array([[-3.0, 0.0, 0.0]])
    r, ta, tb = sphere_param(o, np.array([[1.0, 0.0, 0.0]]), lo, h)
    np.testing.assert_allclose(r, [[-1, 0, 0, 1, 0, 0]], atol=1e-15)
    R = h * np.sqrt(3) / 2
    np.testing.assert_allclose([ta[0], tb[0]], [3.0 - R, 3.0 + R], rtol=1e-15)
    # main diagonal through the centre, unnormalised direction
    s = 1.0 / np.sqrt(3)
    r, ta, tb = sphere_param(c - 2.0, np.array([[1.0, 1.0, 1.0]]), lo, h)
    np.testing.assert_allclose(r, [[-s, -s, -s, s, s, s]], atol=1e-15)
    # off-centre ray: both points on the sphere, unit vectors, symmetric about
    # the point of closest approach
    rng = np.random.default_rng(0)
    o = c + rng.uniform(-0.2, 0.2, (50, 3)) - np.array([2.0, 0, 0])
    d = np.column_stack([np.ones(50), rng.uniform(-0.05, 0.05, (50, 2))])
    r, ta, tb = sphere_param(o, d, np.repeat(lo, 50, 0), h)
    np.testing.assert_allclose(np.linalg.norm(r[:, :3], axis=1), 1.0, rtol=1e-14)
    np.testing.assert_allclose(np.linalg.norm(r[:, 3:], axis=1), 1.0, rtol=1e-14)
    p1 = o + ta[:, None] * d
    p2 = o + tb[:, None] * d
    np.testing.assert_allclose(np.linalg.norm(p1 - c, axis=1), R, rtol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(p2 - c, axis=1), R, rtol=1e-12)
    tmid = 0.5 * (ta + tb)
    closest = -np.sum((o - c) * d, axis=1) / np.sum(d * d, axis=1)
    np.testing.assert_allclose(tmid, closest, rtol=1e-12)


# ------------------------------------------------------------ closed-form renders

def _axis_ray(h, lo, y_frac=0.3, z_frac=0.6):
    """+x ray crossing the voxel at fractional (y, z); t_in = 2, t_out = 2 + h."""
    o = np.array([[lo[0] - 2.0, lo[1] + y_frac * h, lo[2] + z_frac * h]], np.float32)
    d = np.array([[1.0, 0.0, 0.0]], np.float32)
    return o, d


@pytest.mark.parametrize("beta", [-1.3, 0.0, 2.2])
def test_colour_read_at_surface_point(beta):
    """Density decoder = constants (sigma = s, eta = sigmoid(beta)); colour
    decoder = identity on the colour features; colour features a linear
    field (trilinear interpolation reproduces it exactly) -> the colour is
    sigmoid of the field at x_s = eta x1 + (1 - eta) x2."""
    oc, h, lo = _one_voxel()
    dec = (2, 3, 4, 1, 1)
    wt, wc = widths_of(dec)
    lt, lc = _zeros(wt), _zeros(wc)
    s = 0.7
    lt[-1][1][:] = [s, beta]                      # output biases of F_T
    W0, b0 = lc[0]
    W0[0, 0] = W0[1, 1] = W0[2, 2] = 1.0          # hidden k = relu(z_C,k + 10)
    b0[:3] = 10.0
    W1, b1 = lc[1]
    W1[0, 0] = W1[1, 1] = W1[2, 2] = 1.0          # o_k = hidden_k - 10
    b1[:] = -10.0
    p = np.concatenate([_layers_flat(lt), _layers_flat(lc)])
    assert p.size == n_params(dec)
    A = np.array([[0.8, -0.3, 0.5], [-0.2, 0.9, 0.1], [0.4, 0.4, -0.7]])
    pos = _vertex_pos(oc, h)
    F = np.zeros((oc.n_vertices, 5))
    F[:, :2] = 3.0                                 # Z_T: irrelevant here
    F[:, 2:] = pos @ A.T + 0.1                     # Z_C: linear field
    o, d = _axis_ray(h, lo)
    hits = trace_hits(oc, o, d, 4)
    rgb, dep, acc, st = render_lf(oc, F, p, dec, o, d, hits)
    t_in, t_out = 2.0, 2.0 + h
    np.testing.assert_allclose([hits[1][0, 0], hits[2][0, 0]], [t_in, t_out])
    eta = 1.0 / (1.0 + np.exp(-beta))
    x1 = o[0].astype(np.float64) + t_in * d[0]
    x2 = o[0].astype(np.float64) + t_out * d[0]
    xs = eta * x1 + (1.0 - eta) * x2
    alpha = 1.0 - np.exp(-s)                       # "direct": tau = sigma
    c = 1.0 / (1.0 + np.exp(-(A @ xs + 0.1)))
    np.testing.assert_allclose(rgb[0], alpha * c, rtol=1e-12)
    np.testing.assert_allclose(acc[0], alpha, rtol=1e-12)
    np.testing.assert_allclose(dep[0], alpha * (eta * t_in + (1.0 - eta) * t_out), rtol=1e-12)


def test_density_reads_entry_and_exit_features():
    """sigma from psi(x1; Z_T) channel 0, eta from psi(x2; Z_T) channel 1, with
    Z_T a linear field: closed forms for opacity and depth."""
    oc, h, lo = _one_voxel()
    dec = (2, 1, 4, 1, 1)
    wt, wc = widths_of(dec)
    lt, lc = _zeros(wt), _zeros(wc)
    W0, b0 = lt[0]
    W0[0, 0] = 1.0                                 # hidden 0 = relu(psi(x1)_0 + 5)
    b0[0] = 5.0
    W0[1, 2 + 1] = 1.0                             # hidden 1 = relu(psi(x2)_1 + 5)
    b0[1] = 5.0
    W1, b1 = lt[1]
    W1[0, 0] = 1.0
    W1[1, 1] = 1.0
    b1[:] = [-5.0, -5.0]
    p = np.concatenate([_layers_flat(lt), _layers_flat(lc)])
    pos = _vertex_pos(oc, h)
    F = np.zeros((oc.n_vertices, 3))
    F[:, 0] = pos @ [1.5, 0.2, -0.4] + 1.0
    F[:, 1] = pos @ [-0.6, 0.8, 0.3] - 0.2
    o, d = _axis_ray(h, lo, 0.4, 0.2)
    hits = trace_hits(oc, o, d, 4)
    rgb, dep, acc, st = render_lf(oc, F, p, dec, o, d, hits, tau_mode="direct")
    x1 = o[0].astype(np.float64) + 2.0 * d[0]
    x2 = o[0].astype(np.float64) + (2.0 + h) * d[0]
    sigma = max(x1 @ [1.5, 0.2, -0.4] + 1.0, 0.0)
    eta = 1.0 / (1.0 + np.exp(-(x2 @ [-0.6, 0.8, 0.3] - 0.2)))
    assert sigma > 0
    alpha = 1.0 - np.exp(-sigma)
    np.testing.assert_allclose(acc[0], alpha, rtol=1e-12)
    np.testing.assert_allclose(dep[0], alpha * (eta * 2.0 + (1 - eta) * (2.0 + h)), rtol=1e-12)
    # colour decoder with zero weights: c = 1/2
    np.testing.assert_allclose(rgb[0], 0.5 * alpha, rtol=1e-12)


def test_ray_parameterisation_reaches_the_colour_decoder():
    """Colour channel 0 = sigmoid(r_0) (x of p1~), channel 1 = sigmoid(r_3)
    (x of p2~), channel 2 = sigmoid(d_x) with the view direction: for a +x
    ray through the voxel centre r_0 = -1, r_3 = +1."""
    oc, h, lo = _one_voxel()
    dec = (1, 1, 4, 1, 1)
    wt, wc = widths_of(dec, viewdir=True)
    lt, lc = _zeros(wt), _zeros(wc)
    lt[-1][1][:] = [2.0, 0.0]
    W0, b0 = lc[0]
    W0[0, 1 + 0] = 1.0                             # input = [z_C (1) | r (6) | d (3)]
    W0[1, 1 + 3] = 1.0
    W0[2, 1 + 6] = 1.0
    b0[:3] = 10.0
    W1, b1 = lc[1]
    W1[0, 0] = W1[1, 1] = W1[2, 2] = 1.0
    b1[:] = -10.0
    p = np.concatenate([_layers_flat(lt), _layers_flat(lc)])
    F = np.zeros((oc.n_vertices, 2))
    o, d = _axis_ray(h, lo, 0.5, 0.5)
    hits = trace_hits(oc, o, d, 4)
    rgb, _, acc, st = render_lf(oc, F, p, dec, o, d, hits, viewdir=True)
    np.testing.assert_allclose(st.r[0], [-1, 0, 0, 1, 0, 0], atol=1e-12)
    sg = lambda x: 1.0 / (1.0 + np.exp(-x))
    np.testing.assert_allclose(rgb[0], acc[0] * sg(np.array([-1.0, 1.0, 1.0])), rtol=1e-12)


# ------------------------------------------------------------ gradients

def _fd_case(seed, tau_mode, viewdir=False):
    w = tiny_workload(seed, 3, 7, (8, 16, 16, 4), 4, n_obj=2)
    sc = w.scene()
    oc = Octree(sc.leaf_ijk, sc.depth)
    dec = (4, 3, 16, 1, 2)
    rng = np.random.default_rng(seed)
    F = rng.normal(0, 1.0, (oc.n_vertices, 7))
    wt, wc = widths_of(dec, viewdir)
    p = np.concatenate([xavier_params(rng, wt), xavier_params(rng, wc)]).astype(np.float64)
    nt = sum(a * b + b for a, b in zip(wt[:-1], wt[1:]))
    p[nt - 2] = 0.8                                # sigma mostly positive
    o, d = random_rays(rng, 48, inside_frac=0.1, axis_frac=0.0)
    hits = trace_hits(oc, o, d, 4)
    rgb_t = rng.uniform(0, 1, (48, 3))
    dep_t = rng.uniform(0, 4, 48)
    return oc, F, p, dec, o, d, hits, rgb_t, dep_t


def _pattern(st, dep, dep_t):
    return np.concatenate([np.concatenate([z.ravel() > 0 for z in st.presT + st.presC]),
                           st.oT[:, 0] > 0, dep - dep_t > 0,
                           ((st.us_raw >= 0) & (st.us_raw <= 1)).ravel()])


@pytest.mark.parametrize("tau_mode,viewdir", [("direct", False), ("voxel", False), ("direct", True)])
def test_lf_gradients_against_central_differences(tau_mode, viewdir):
    oc, F, p, dec, o, d, hits, rgb_t, dep_t = _fd_case(5, tau_mode, viewdir)

    def L(Fx, px):
        rgb, dep, acc, st = render_lf(oc, Fx, px, dec, o, d, hits, tau_mode=tau_mode, viewdir=viewdir)
        return loss(rgb, dep, rgb_t, dep_t)[0], st, rgb, dep

    L0, st, rgb, dep = L(F, p)
    assert st.ray_i.size > 20
    base = _pattern(st, dep, dep_t)
    _, g_rgb, g_dep = loss(rgb, dep, rgb_t, dep_t)
    gF, gp = render_lf_backward(st, g_rgb, g_dep)
    assert np.abs(gF[:, :4]).max() > 0 and np.abs(gF[:, 4:]).max() > 0

    def fd(Fp, Fm, pp, pm, eps):
        Lp, sp, _, dp = L(Fp, pp)
        Lm, sm, _, dm = L(Fm, pm)
        if not (np.array_equal(_pattern(sp, dp, dep_t), base) and np.array_equal(_pattern(sm, dm, dep_t), base)):
            return None
        return (Lp - Lm) / (2 * eps)

    floor = lambda eps: 64 * np.finfo(np.float64).eps * abs(L0) / eps
    rng = np.random.default_rng(1)
    touched = np.unique(st.corners)
    checked = skipped = 0
    for _ in range(60):
        v = touched[rng.integers(touched.size)]
        c = rng.integers(0, F.shape[1])
        eps = 1e-6
        Fp = F.copy(); Fp[v, c] += eps
        Fm = F.copy(); Fm[v, c] -= eps
        g = fd(Fp, Fm, p, p, eps)
        if g is None:
            skipped += 1
            continue
        checked += 1
        assert abs(g - gF[v, c]) <= 1e-6 * abs(g) + floor(eps), (v, c, g, gF[v, c])
    for k in rng.choice(p.size, 80, replace=False):
        eps = 1e-6
        pp = p.copy(); pp[k] += eps
        pm = p.copy(); pm[k] -= eps
        g = fd(F, F, pp, pm, eps)
        if g is None:
            skipped += 1
            continue
        checked += 1
        assert abs(g - gp[k]) <= 1e-6 * abs(g) + floor(eps), (k, g, gp[k])
    assert skipped <= 0.1 * (checked + skipped)


def test_eta_gradient_through_the_surface_point():
    """With a constant eta path only (colour features a linear field, colour
    decoder the identity), dL/dbeta (the eta output bias) equals the closed
    form sum over channels of dL/dc * c(1-c) * A (x1 - x2) * eta(1-eta)
    plus the depth term."""
    oc, h, lo = _one_voxel()
    dec = (2, 3, 4, 1, 1)
    wt, wc = widths_of(dec)
    lt, lc = _zeros(wt), _zeros(wc)
    beta, s = 0.4, 0.9
    lt[-1][1][:] = [s, beta]
    W0, b0 = lc[0]
    W0[0, 0] = W0[1, 1] = W0[2, 2] = 1.0
    b0[:3] = 10.0
    W1, b1 = lc[1]
    W1[0, 0] = W1[1, 1] = W1[2, 2] = 1.0
    b1[:] = -10.0
    p = np.concatenate([_layers_flat(lt), _layers_flat(lc)])
    A = np.array([[0.8, -0.3, 0.5], [-0.2, 0.9, 0.1], [0.4, 0.4, -0.7]])
    F = np.zeros((oc.n_vertices, 5))
    F[:, 2:] = _vertex_pos(oc, h) @ A.T + 0.1
    o, d = _axis_ray(h, lo)
    hits = trace_hits(oc, o, d, 4)
    rgb, dep, acc, st = render_lf(oc, F, p, dec, o, d, hits)
    g_rgb = np.array([[0.3, -0.7, 0.2]])
    g_dep = np.array([0.5])
    _, gp = render_lf_backward(st, g_rgb, g_dep)
    nt = sum(a * b + b for a, b in zip(wt[:-1], wt[1:]))
    eta = 1.0 / (1.0 + np.exp(-beta))
    alpha = 1.0 - np.exp(-s)
    x1 = o[0].astype(np.float64) + 2.0 * d[0]
    x2 = o[0].astype(np.float64) + (2.0 + h) * d[0]
    xs = eta * x1 + (1 - eta) * x2
    c = 1.0 / (1.0 + np.exp(-(A @ xs + 0.1)))
    dL_deta = alpha * (g_rgb[0] * c * (1 - c)) @ (A @ (x1 - x2)) + alpha * g_dep[0] * (2.0 - (2.0 + h))
    np.testing.assert_allclose(gp[nt - 1], dL_deta * eta * (1 - eta), rtol=1e-12)


def test_feature_gradient_conservation():
    oc, F, p, dec, o, d, hits, _, _ = _fd_case(9, "direct")
    rgb, dep, acc, st = render_lf(oc, F, p, dec, o, d, hits)
    rng = np.random.default_rng(2)
    g_rgb = rng.normal(size=rgb.shape)
    g_dep = rng.normal(size=dep.shape)
    gF, _ = render_lf_backward(st, g_rgb, g_dep)
    # trilinear weights sum to one: a perturbation of all of Z_C by a constant vector e shifts psi(x_s) by
    # e exactly: the directional derivative equals sum(gF_C) . e
    e = rng.normal(size=3)
    eps = 1e-6
    Fp = F.copy(); Fp[:, 4:] += eps * e
    Fm = F.copy(); Fm[:, 4:] -= eps * e
    r1 = render_lf(oc, Fp, p, dec, o, d, hits)
    r2 = render_lf(oc, Fm, p, dec, o, d, hits)
    fd = (np.sum(g_rgb * (r1[0] - r2[0])) + np.sum(g_dep * (r1[1] - r2[1]))) / (2 * eps)
    assert abs(fd - gF[:, 4:].sum(axis=0) @ e) <= 1e-6 * abs(fd) + 1e-8
    # the same for Z_T (both points share the voxel's corners)
    e = rng.normal(size=4)
    Fp = F.copy(); Fp[:, :4] += eps * e
    Fm = F.copy(); Fm[:, :4] -= eps * e
    r1 = render_lf(oc, Fp, p, dec, o, d, hits)
    r2 = render_lf(oc, Fm, p, dec, o, d, hits)
    fd = (np.sum(g_rgb * (r1[0] - r2[0])) + np.sum(g_dep * (r1[1] - r2[1]))) / (2 * eps)
    assert abs(fd - gF[:, :4].sum(axis=0) @ e) <= 1e-6 * abs(fd) + 1e-8


def test_lf_hit_magnitude_bounds_every_entry_and_is_homogeneous():
    """The per-hit contribution scale of the light-field backward bounds every
    gradient entry (triangle inequality), is linear in the upstream gradients
    and does not depend on their sign."""
    oc, F, p, dec, o, d, hits, _, _ = _fd_case(5, "voxel")
    rgb, dep, acc, st = render_lf(oc, F, p, dec, o, d, hits, tau_mode="voxel")
    rng = np.random.default_rng(3)
    ups = [rng.normal(size=rgb.shape), rng.normal(size=dep.shape), rng.normal(size=acc.shape)]
    gF, gp = render_lf_backward(st, *ups)
    mF, mp = render_lf_backward_hit_magnitude(st, *ups)
    assert np.all(mF >= np.abs(gF)) and np.all(mp >= np.abs(gp))
    assert np.all(mF[gF != 0] > 0) and np.count_nonzero(gF) > 100
    mF2, mp2 = render_lf_backward_hit_magnitude(st, *[2 * u for u in ups])
    np.testing.assert_allclose(mF2, 2 * mF, rtol=1e-14, atol=0)
    np.testing.assert_allclose(mp2, 2 * mp, rtol=1e-14, atol=0)
    mF3, mp3 = render_lf_backward_hit_magnitude(st, *[-u for u in ups])
    np.testing.assert_allclose(mF3, mF, rtol=1e-14, atol=0)
    np.testing.assert_allclose(mp3, mp, rtol=1e-14, atol=0)


def _one_hit_case():
    oc, F, p, dec, o, d, _, _, _ = _fd_case(5, "direct")
    hits = trace_hits(oc, o, d, 1)
    # a ray whose entry and exit weights differ and whose tau ReLU is on
    for r in np.nonzero(hits[3] > 0)[0]:
        h1 = tuple(x[r:r + 1] for x in hits)
        _, _, _, st = render_lf(oc, F, p, dec, o[r:r + 1], d[r:r + 1], h1)
        if (np.linalg.matrix_rank(np.stack([st.w1[0], st.w2[0]], axis=1), tol=1e-3) == 2
                and st.oT[0, 0] > 0.05):
            return oc, F, p, dec, o[r:r + 1], d[r:r + 1], h1, st
    raise AssertionError("no suitable ray")


def test_lf_hit_magnitude_of_one_hit():
    """One ray, one hit.  Colour block and decoder parameters receive one
    term per entry: the scale is |gradient| plus the largest |gradient| of
    the entry's group, read off the gradient."""
    oc, F, p, dec, o, d, h1, st = _one_hit_case()
    wt, wc = widths_of(dec)
    ct = dec[0]
    assert st.ray_i.size == 1
    ups = [np.array([[0.3, -1.2, 0.7]]), np.array([0.4]), np.array([-0.9])]
    gF, gp = render_lf_backward(st, *ups)
    mF, mp = render_lf_backward_hit_magnitude(st, *ups)
    corners = st.corners[0]
    gC = gF[corners, ct:]
    np.testing.assert_allclose(mF[corners, ct:], np.abs(gC) + np.abs(gC).max(axis=1, keepdims=True),
                               rtol=1e-13, atol=0)
    assert np.all(mF[corners, :ct] >= np.abs(gF[corners, :ct]))
    others = np.setdiff1d(np.arange(F.shape[0]), corners)
    assert np.all(mF[others] == 0)
    exp_p, off = [], 0
    for widths in (wt, wc):
        for fi, fo in zip(widths[:-1], widths[1:]):
            gW = np.abs(gp[off:off + fi * fo])
            gb = np.abs(gp[off + fi * fo:off + fi * fo + fo])
            exp_p += [gW + gW.max(), gb + gb.max()]
            off += fi * fo + fo
    np.testing.assert_allclose(mp, np.concatenate(exp_p), rtol=1e-13, atol=0)


@pytest.mark.parametrize("cancel", [False, True])
def test_lf_density_block_magnitude_closed_form(cancel):
    """One ray with one hit and no colour gradient (g_rgb = 0, so nothing
    reaches the colour decoder and the surface point carries no gradient):
    with T = 1 and no later voxel, dL/dtau = e^{-tau} (g_d t_s + g_a) and
    dL/deta = g_d w (t_in - t_out), w = 1 - e^{-tau}.  Their term magnitudes
    are e^{-tau} (|g_d| t_s + |g_a|) and |g_d| w |t_in - t_out|; the Z_T
    scale is w1_j (A1 + max A1) + w2_j (A2 + max A2) with A = |J0| G0 + |J1| G1,
    the decoder's input Jacobian J taken by central differences of its
    forward.  With g_a = -g_d t_s the tau gradient cancels exactly while its
    term magnitude does not."""
    from oracle.lightfield import _mlp
    oc, F, p, dec, o, d, h1, st = _one_hit_case()
    ct = dec[0]
    ts, tau, eta = st.ts[0, 0], st.tau[0, 0], st.eta[0]
    g_d = 0.4
    g_a = -g_d * ts if cancel else -0.9
    ups = [np.zeros((1, 3)), np.array([g_d]), np.array([g_a])]
    gF, _ = render_lf_backward(st, *ups)
    mF, _ = render_lf_backward_hit_magnitude(st, *ups)
    e = np.exp(-tau)
    w = 1.0 - e
    G0 = e * (abs(g_d) * ts + abs(g_a)) * st.dtau[0]
    G1 = abs(g_d) * w * abs(st.t0[0] - st.t1[0]) * eta * (1.0 - eta)
    X = st.actsT[0][0]
    J = np.zeros((X.size, 2))
    for i in range(X.size):
        dx = np.zeros(X.size)
        dx[i] = 1e-6
        J[i] = (_mlp(st.lt, (X + dx)[None], lambda v: v)[0][0] - _mlp(st.lt, (X - dx)[None], lambda v: v)[0][0]) / 2e-6
    A = np.abs(J[:, 0]) * G0 + np.abs(J[:, 1]) * G1
    A1, A2 = A[:ct], A[ct:2 * ct]
    exp_T = (st.w1[0][:, None] * (A1[None, :] + A1.max()) + st.w2[0][:, None] * (A2[None, :] + A2.max()))
    np.testing.assert_allclose(mF[st.corners[0], :ct], exp_T, rtol=1e-6, atol=0)
    assert np.all(mF[st.corners[0], ct:] == 0)
    if cancel:
        # the tau term cancels: the gradient comes through eta alone, while
        # the scale still holds the tau term's size
        J1_only = np.abs(J[:, 1]) * G1
        assert np.all(exp_T > st.w1[0][:, None] * J1_only[None, :ct])


def test_lf_hit_magnitude_adds_over_cancelling_hits():
    """The same rays twice with opposite upstream gradients: the gradients
    cancel exactly and the scale is twice that of one copy."""
    oc, F, p, dec, o, d, hits, _, _ = _fd_case(7, "direct")
    rng = np.random.default_rng(5)
    ups = [rng.normal(size=(o.shape[0], 3)), rng.normal(size=o.shape[0]), rng.normal(size=o.shape[0])]
    _, _, _, st1 = render_lf(oc, F, p, dec, o, d, hits)
    m1F, m1p = render_lf_backward_hit_magnitude(st1, *ups)
    o2, d2 = np.concatenate([o, o]), np.concatenate([d, d])
    h2 = tuple(np.concatenate([x, x]) for x in hits)
    _, _, _, st2 = render_lf(oc, F, p, dec, o2, d2, h2)
    ups2 = [np.concatenate([u, -u]) for u in ups]
    gF, gp = render_lf_backward(st2, *ups2)
    m2F, m2p = render_lf_backward_hit_magnitude(st2, *ups2)
    assert np.abs(gF).max() <= 1e-15 * m2F.max() and np.abs(gp).max() <= 1e-15 * m2p.max()
    np.testing.assert_allclose(m2F, 2 * m1F, rtol=1e-13, atol=0)
    np.testing.assert_allclose(m2p, 2 * m1p, rtol=1e-13, atol=0)
    assert m1F[:, :4].max() > 0 and m1F[:, 4:].max() > 0 and m1p.max() > 0


def test_lf_weight_scale_of_one_hit_and_over_cancelling_hits():
    """One ray, one hit: a Z_C row of corner j has the weight scale
    D_s,j |dL/dpsi(x_s)| with dL/dpsi(x_s) = Z_C gradient row / w_s,j, and a Z_T
    row D1_j |g1| + D2_j |g2| with g1, g2 recovered from the Z_T gradient by
    least squares over the trilinear weights (D from the weights' central
    differences).  Opposite upstream gradients on duplicated rays double it."""
    from oracle.render import interpolation_weights
    oc, F, p, dec, o, d, _, _, _ = _fd_case(5, "direct")
    hits = trace_hits(oc, o, d, 1)
    ct = dec[0]
    for r in np.nonzero(hits[3] > 0)[0]:
        h1 = tuple(x[r:r + 1] for x in hits)
        _, _, _, st = render_lf(oc, F, p, dec, o[r:r + 1], d[r:r + 1], h1)
        A = np.stack([st.w1[0], st.w2[0]], axis=1)
        if np.linalg.matrix_rank(A, tol=1e-3) == 2 and np.all(st.ws[0] > 1e-6):
            break
    ups = [np.array([[0.3, -1.2, 0.7]]), np.array([0.4]), np.array([-0.9])]
    gF, _ = render_lf_backward(st, *ups)
    Mw = render_lf_backward_weight_scale(st, *ups)

    def fd_D(u):
        D = np.zeros(8)
        for a in range(3):
            e = np.zeros(3)
            e[a] = 1e-7
            D += np.abs((interpolation_weights(u + e) - interpolation_weights(u - e))[0] / 2e-7)
        return D

    corners = st.corners[0]
    Ds = fd_D(st.us)
    np.testing.assert_allclose(Mw[corners, ct:], Ds[:, None] * np.abs(gF[corners, ct:]) / st.ws[0][:, None],
                               rtol=1e-6)
    g12, *_ = np.linalg.lstsq(A, gF[corners, :ct], rcond=None)
    exp_T = fd_D(st.u1)[:, None] * np.abs(g12[0])[None, :] + fd_D(st.u2)[:, None] * np.abs(g12[1])[None, :]
    np.testing.assert_allclose(Mw[corners, :ct], exp_T, rtol=1e-5, atol=1e-12)
    oc, F, p, dec, o, d, hits, _, _ = _fd_case(7, "direct")
    rng = np.random.default_rng(5)
    ups = [rng.normal(size=(o.shape[0], 3)), rng.normal(size=o.shape[0]), rng.normal(size=o.shape[0])]
    _, _, _, st1 = render_lf(oc, F, p, dec, o, d, hits)
    m1 = render_lf_backward_weight_scale(st1, *ups)
    h2 = tuple(np.concatenate([x, x]) for x in hits)
    _, _, _, st2 = render_lf(oc, F, p, dec, np.concatenate([o, o]), np.concatenate([d, d]), h2)
    m2 = render_lf_backward_weight_scale(st2, *[np.concatenate([u_, -u_]) for u_ in ups])
    np.testing.assert_allclose(m2, 2 * m1, rtol=1e-13, atol=0)
    assert m1[:, :ct].max() > 0 and m1[:, ct:].max() > 0
    # the derivative table used for D agrees with central differences
    u = np.random.default_rng(1).uniform(0.1, 0.9, (5, 3))
    for i in range(5):
        np.testing.assert_allclose(np.sum(np.abs(weight_derivatives(u[i:i + 1])[0]), axis=1), fd_D(u[i:i + 1]),
                                   rtol=1e-6)


# ------------------------------------------------------------ staged losses (section 4.4)

from oracle.lightfield import stage_loss, surface_slots  # noqa: E402


def _const_decoders(s, beta, bc):
    """Density decoder constant (sigma = s, eta = sigmoid(beta)), colour
    decoder constant (c = sigmoid(bc)): the dec (2, 3, 4, 1, 1) shapes."""
    dec = (2, 3, 4, 1, 1)
    wt, wc = widths_of(dec)
    lt, lc = _zeros(wt), _zeros(wc)
    lt[-1][1][:] = [s, beta]
    lc[-1][1][:] = bc
    return dec, np.concatenate([_layers_flat(lt), _layers_flat(lc)])


@pytest.mark.parametrize("kind", ["surface", "volume"])
def test_stage_loss_single_voxel_closed_form(kind):
    oc, h, lo = _one_voxel()
    s, beta, bc = 0.8, 0.3, np.array([0.2, -0.5, 1.0])
    dec, p = _const_decoders(s, beta, bc)
    F = np.zeros((oc.n_vertices, 5))
    o, d = _axis_ray(h, lo)
    hits = trace_hits(oc, o, d, 4)
    rgb, dep, acc, st = render_lf(oc, F, p, dec, o, d, hits)
    t_star = np.array([2.0 + 0.3 * h], np.float32)      # surface point inside the voxel
    c_star = np.array([[0.1, 0.7, 0.4]])
    lam_eta, lam_tau, ls = 0.5, 0.25, 0.125
    L, g_rgb, hg = stage_loss(st, hits, rgb, c_star, t_star, kind, lam_eta, lam_tau, ls)
    assert surface_slots(hits, t_star)[0] == 0
    eta = 1.0 / (1.0 + np.exp(-beta))
    eta_gt = ((2.0 + h) - float(t_star[0])) / h
    c = 1.0 / (1.0 + np.exp(-bc))
    alpha = 1.0 - np.exp(-s)
    col = c if kind == "surface" else alpha * c
    L_exp = ls * (np.sum((col - c_star[0]) ** 2) + lam_eta * (eta - eta_gt) ** 2 + lam_tau * np.exp(-2 * s))
    assert L == pytest.approx(L_exp, rel=1e-12)
    # gradient of the eta-bias and the tau-bias in closed form
    _, gp = render_lf_backward(st, g_rgb, np.zeros(1), hit_grads=hg)
    wt, _ = widths_of(dec)
    nt = sum(a * b + b for a, b in zip(wt[:-1], wt[1:]))
    assert gp[nt - 1] == pytest.approx(ls * 2 * lam_eta * (eta - eta_gt) * eta * (1 - eta), rel=1e-12)
    g_s = -2.0 * ls * lam_tau * np.exp(-2 * s)
    if kind == "volume":                                # d|alpha c - c*|^2 / ds
        g_s += ls * 2 * np.sum((alpha * c - c_star[0]) * c) * np.exp(-s)
    assert gp[nt - 2] == pytest.approx(g_s, rel=1e-12)
    # no surface voxel: a target depth beyond the voxel leaves only the
    # photometric term of the volume loss
    L2, _, hg2 = stage_loss(st, hits, rgb, c_star, np.array([5.0], np.float32), kind, lam_eta, lam_tau, ls)
    assert np.all(hg2[1] == 0) and np.all(hg2[0] == 0)
    assert L2 == pytest.approx(0.0 if kind == "surface" else ls * np.sum((alpha * c - c_star[0]) ** 2))


def test_surface_slots_half_open():
    tin = np.array([[1.0, 2.0, 0.0]], np.float32)
    tout = np.array([[2.0, 3.0, 0.0]], np.float32)
    cnt = np.array([2])
    hits = (np.array([[0, 1, -1]]), tin, tout, cnt)
    assert surface_slots(hits, np.array([2.0], np.float32))[0] == 1     # boundary -> the later voxel
    assert surface_slots(hits, np.array([1.0], np.float32))[0] == 0
    assert surface_slots(hits, np.array([3.0], np.float32))[0] == -1    # t_out is open
    assert surface_slots(hits, np.array([0.5], np.float32))[0] == -1


@pytest.mark.parametrize("kind", ["surface", "volume"])
def test_stage_loss_gradients_against_central_differences(kind):
    oc, F, p, dec, o, d, hits, rgb_t, _ = _fd_case(7, "direct")
    # target depths: the middle of a random hit of each ray (or none)
    rng = np.random.default_rng(3)
    cnt = hits[3]
    pick = np.where(cnt > 0, rng.integers(0, np.maximum(cnt, 1)), 0)
    t_d = np.where(cnt > 0, 0.5 * (hits[1][np.arange(o.shape[0]), pick] + hits[2][np.arange(o.shape[0]), pick]),
                   0.0).astype(np.float32)

    def L(Fx, px):
        rgb, dep, acc, st = render_lf(oc, Fx, px, dec, o, d, hits)
        Lv, g_rgb, hg = stage_loss(st, hits, rgb, rgb_t, t_d, kind, 0.7, 0.3, 1.0 / o.shape[0])
        return Lv, st, g_rgb, hg

    L0, st, g_rgb, hg = L(F, p)
    assert np.count_nonzero(hg[1]) > 5
    gF, gp = render_lf_backward(st, g_rgb, np.zeros(o.shape[0]), hit_grads=hg)

    def pattern(sx):
        return np.concatenate([np.concatenate([z.ravel() > 0 for z in sx.presT + sx.presC]),
                               sx.oT[:, 0] > 0, ((sx.us_raw >= 0) & (sx.us_raw <= 1)).ravel()])

    base = pattern(st)
    floor = lambda eps: 64 * np.finfo(np.float64).eps * abs(L0) / eps
    checked = skipped = 0
    for _ in range(50):
        v = np.unique(st.corners)[rng.integers(np.unique(st.corners).size)]
        c = rng.integers(0, F.shape[1])
        eps = 1e-6
        Fp = F.copy(); Fp[v, c] += eps
        Fm = F.copy(); Fm[v, c] -= eps
        (Lp, sp, _, _), (Lm, sm, _, _) = L(Fp, p), L(Fm, p)
        if not (np.array_equal(pattern(sp), base) and np.array_equal(pattern(sm), base)):
            skipped += 1
            continue
        checked += 1
        g = (Lp - Lm) / (2 * eps)
        assert abs(g - gF[v, c]) <= 1e-6 * abs(g) + floor(eps), (v, c, g, gF[v, c])
    for k in rng.choice(p.size, 60, replace=False):
        eps = 1e-6
        pp = p.copy(); pp[k] += eps
        pm = p.copy(); pm[k] -= eps
        (Lp, sp, _, _), (Lm, sm, _, _) = L(F, pp), L(F, pm)
        if not (np.array_equal(pattern(sp), base) and np.array_equal(pattern(sm), base)):
            skipped += 1
            continue
        checked += 1
        g = (Lp - Lm) / (2 * eps)
        assert abs(g - gp[k]) <= 1e-6 * abs(g) + floor(eps), (k, g, gp[k])
    assert skipped <= 0.1 * (checked + skipped)


def test_surface_point_error_scale_bounds_the_corner_weight_change():
    """The test helper's surface-point scale, given eta's change, bounds the
    change of every Z_C entry that the moved corner weights cause (with
    dL/dpsi(x_s) held fixed): eta moved through the density decoder's o_T1
    bias by delta, |d eta| = eta (1 - eta) delta to first order."""
    from oracle.lightfield import _lf_backward_per_hit
    from tests.gpu_cases import lf_surface_point_error
    for seed in (5, 6, 7):
        oc, F, p, dec, o, d, hits, _, _ = _fd_case(seed, "direct")
        _, _, _, st = render_lf(oc, F, p, dec, o, d, hits)
        rng = np.random.default_rng(9)
        g_rgb = rng.normal(size=(o.shape[0], 3))
        g_dep = rng.normal(size=o.shape[0])
        _, _, _, _, g_zC = _lf_backward_per_hit(st, g_rgb, g_dep)
        wt, _ = widths_of(dec)
        nt = sum(a * b + b for a, b in zip(wt[:-1], wt[1:]))
        delta = 1e-6
        p2 = p.copy()
        p2[nt - 1] += delta                       # bias of o_T1
        _, _, _, st2 = render_lf(oc, F, p2, dec, o, d, hits)
        dW = st2.ws - st.ws
        actual = np.zeros((st.n_vertices, g_zC.shape[1]))
        np.add.at(actual, st.corners.ravel(), (dW[:, :, None] * g_zC[:, None, :]).reshape(-1, g_zC.shape[1]))
        E = lf_surface_point_error(st, F, g_rgb, g_dep, deta=st.eta * (1.0 - st.eta) * delta)
        assert np.abs(actual).max() > 0
        assert np.all(np.abs(actual) <= E * (1 + 1e-4) + 1e-18), seed
        # tight where one hit dominates an entry (a scale too large by a
        # constant factor fails here)
        big = np.abs(actual) > 0.5 * np.abs(actual).max()
        assert np.min(E[big] / np.abs(actual[big])) < 1.1, seed
