"""Shared set-up for the GPU parity tests: one workload on the device and
the same inputs in the oracle, plus the stated tolerances.

Tolerances (FP32 path, derived from the arithmetic):
* rgb / depth / acc: per channel max|err| <= 1e-5 * max|ref| + 1e-7 S and
  elementwise |err| <= 1e-5 |ref| + 1e-6 S, S = 1 (rgb, acc) or max depth.
  FP32 MLP dot products (length <= 64) and FP32 compositing round at ~1e-7
  relative; the mixed bound covers cancellation near sigma ~ 0.
* gradients: normwise max|err| <= 1e-5 max|g| (features) or 1e-4 max|g|
  (decoder parameters, whose sums run over every hit of the batch), and
  per entry |err| <= c 2^-24 M, where M is the oracle's per-hit
  contribution scale of that entry (the sum over the hits that reach it of
  |contribution| plus each such hit's largest contribution to the entry's
  group, render_backward_hit_magnitude).  Every contribution is computed in
  FP32 along a chain of about a dozen dependent stages (interpolation, the
  decoder's dot products of length <= 64 forward and backward, Eq. 3 and its
  suffix sums), so it carries a rounding error of some hundreds of ulps of
  the hit's largest contribution; the FP32 sum over the entry's hits (atomics
  in any order, or the per-block MFMA accumulation and the reduction of the
  decoder gradient) adds at most a few ulps of S per addition.  A sample
  point's cell coordinates u carry an absolute error of a few ulps of 1
  (more in the light field, whose surface point moves with eta's error), which
  moves a corner's weight by at most that error times D_j = sum_a |dw_j/du_a|:
  for a weight near zero (a point near a face of its cell) that is no small
  relative error, so the bound adds c_w 2^-24 W, W = the sum over the hits of
  D_j |dL/dx_h[c]| (render_backward_weight_scale).  Measured on every parity
  case, the largest (|err| - c_w 2^-24 W) / (2^-24 M) was 72 for the feature
  entries (c_w = 8) and 1.0 for the decoder entries; C_FEAT = 256 and
  C_PARAM = 4 leave a margin of 3.5 and 4.  Unlike a floor relative to max|g|, the bound scales with the
  entry's own contributions, so a small or cancelling entry is checked at its
  own scale.  Gradient parity uses rays with no decoder pre-activation within
  1e-4 of a ReLU kink (there FP32 and FP64 may legitimately take different
  one-sided derivatives).  On rays with many hits Eq. 3's dL/dtau is a small
  difference of large terms; tests of such rays take M at the conditioning
  of each hit's dL/dX (render_backward_hit_magnitude(conditioned=True)), and
  where large density-decoder activations make eta's FP32 error move the
  light field's surface point by more than a few ulps, the Z_C entries add
  that error's own scale (lf_surface_point_error).
BF16 path: compared with the oracle's BF16-rounding mode; hidden activations
may round differently where FP32 and FP64 accumulations straddle a bfloat16
rounding boundary (one bfloat16 ulp = 2^-8 relative).  Single-decoder renders
are checked per ray (bf16_render_bound), light-field renders at
max|err| <= 2^-6 max|ref| + 1e-4 S, and the error against the FP64 oracle is
reported as PSNR.  The decoder alone is checked per entry
(bf16_decoder_bound): each output within the error that FP32 accumulation
can produce, carried through the layers, where a hidden activation may take
the neighbouring bfloat16 value only if its exact pre-activation lies within
that error of a rounding boundary.
"""

import numpy as np

from oracle.octree import Octree
from oracle.render import render as oracle_render, split_params
from oracle.trace import trace_hits as oracle_trace


def assert_outputs_close(got, exp, S=1.0, name="", rel=1e-5, abs_el=1e-6, abs_nw=1e-7):
    got = np.asarray(got, np.float64)
    exp = np.asarray(exp, np.float64)
    assert got.shape == exp.shape, name
    assert np.all(np.isfinite(got)), f"{name}: non-finite output"
    err = np.abs(got - exp)
    if exp.ndim == 1:
        err = err[:, None]
        ref = np.abs(exp)[:, None]
    else:
        ref = np.abs(exp)
    nw = ref.max(axis=0) if ref.size else np.zeros(ref.shape[1])
    worst = err.max(axis=0) if err.size else np.zeros(ref.shape[1])
    assert np.all(worst <= rel * nw + abs_nw * S), f"{name}: normwise {worst} vs {rel * nw + abs_nw * S}"
    bad = err > rel * ref + abs_el * S
    assert not bad.any(), f"{name}: {bad.sum()} elements outside elementwise bound, worst {err[bad].max()}"


EPS32 = 2.0 ** -24
BF16_ULP = 2.0 ** -8
C_FEAT = 2.0 ** 8
C_PARAM = 4.0
C_W = 8.0          # single decoder: the midpoint's cell coordinates to a few ulps
C_W_LF = 64.0      # light field: the surface point moves with eta's error


def bf16_decoder_bound(params, widths, X, dX=None):
    """(ref, bound): the oracle's BF16-mode decoder outputs (n, out) and, per
    entry, the largest |out - ref| of an implementation that rounds X, the
    weights and every hidden activation to bfloat16 exactly as the oracle
    does (to nearest, ties to even) but accumulates each dot product and its
    bias in FP32 in any order.  The products of two bfloat16 values are exact
    in FP32, so a layer's FP32 sum of n products and the bias is off by at
    most gamma_n sum |terms| (gamma_n = n 2^-24 / (1 - n 2^-24)), plus
    |W| times the error its inputs already carry.  ReLU and the rounding are
    monotone, so a pre-activation known to within dz rounds to a value within
    max(r(h(z + dz)) - r(h(z)), r(h(z)) - r(h(z - dz))) of the oracle's: zero
    unless a rounding boundary lies within dz of z.  ``dX`` bounds an error
    of X itself before its rounding (the same rule gives the rounded input's
    error)."""
    from oracle.render import bf16_round as r
    layers = split_params(params, widths)
    X = np.asarray(X, np.float64)
    a = r(X)
    e = np.zeros_like(a) if dX is None else np.maximum(r(X + dX) - a, a - r(X - dX))
    for li, (W, b) in enumerate(layers):
        Wr = r(W)
        absW = np.abs(Wr)
        n = W.shape[1] + 1
        gamma = 1.01 * n * EPS32 / (1.0 - n * EPS32)   # 1% covers the FP64 sum's own rounding
        z = a @ Wr.T + b
        dz = e @ absW.T + gamma * (np.abs(a) @ absW.T + np.abs(b))
        if li == len(layers) - 1:
            return z, dz
        h = lambda v: r(np.maximum(v, 0.0))
        a = h(z)
        e = np.maximum(h(z + dz) - a, a - h(z - dz))
    raise ValueError("empty MLP")


def bf16_render_bound(st, F, dX_ulps=16.0):
    """Per ray, bounds on |rgb - rgb_ref| (n, 3), |depth - depth_ref| and
    |acc - acc_ref| (n,) for a device render in the BF16 mode against the
    oracle's BF16-mode render state ``st`` (single decoder, no view
    direction).  The device interpolates the bfloat16 feature rows in FP32
    (cell coordinates and weights a few ulps off: dX = dX_ulps 2^-24
    sum_j (w_j + D_j) |F_j|, D_j = weight_sensitivity; F unrounded, its rows
    are rounded here), rounds X to bfloat16,
    runs the decoder with FP32 sums (bf16_decoder_bound) and evaluates
    sigmoid, tau, exp and Eq. 3 in FP32.  Each step's error is carried in
    absolute terms: |dc| <= |do|/4 + 4 ulps, |dtau| <= dtau |do_3| + 2 ulps,
    |d exp(-tau)| <= exp(-tau + |dtau|) |dtau| + 4 ulps (so for alpha),
    then along the ray T_{i+1} = T_i e_i, w_i = T_i alpha_i and the three
    sums, each product and sum adding one rounding."""
    from oracle.render import bf16_round, weight_sensitivity
    assert st.X.shape[1] == st.widths[0], "view-direction input not covered"
    D = weight_sensitivity(st.u)
    absF = np.abs(bf16_round(np.asarray(F[st.corners], np.float64)))      # the rows the hits read
    dX = dX_ulps * EPS32 * np.einsum("mj,mjc->mc", st.wj + D, absF)
    o, do = bf16_decoder_bound(st.params, st.widths, st.X, dX)
    c = 1.0 / (1.0 + np.exp(-o[:, :3]))
    dc = 0.25 * do[:, :3] + 4 * EPS32
    sig = np.maximum(o[:, 3], 0.0)
    tau = sig * st.dtau
    dtau = do[:, 3] * st.dtau + 2 * EPS32 * tau
    e = np.exp(-tau)
    de = np.exp(-tau + dtau) * dtau + 4 * EPS32 * e
    alpha = 1.0 - e
    dalpha = de + 4 * EPS32 * alpha
    n, K = st.n, st.K
    dense = lambda v, fill=0.0: _dense(v, st, fill)
    C_, DC = dense(c), dense(dc)
    E, DE, A, DA = dense(e, 1.0), dense(de), dense(alpha), dense(dalpha)
    TM = dense(st.tmid[st.ray_i, st.slot_i])
    T = np.ones(n)
    dT = np.zeros(n)
    rgb, drgb = np.zeros((n, 3)), np.zeros((n, 3))
    dep, ddep = np.zeros(n), np.zeros(n)
    acc, dacc = np.zeros(n), np.zeros(n)
    for k in range(K):
        w = T * A[:, k]
        dw = dT * A[:, k] + T * DA[:, k] + EPS32 * w
        rgb += w[:, None] * C_[:, k]
        drgb += dw[:, None] * C_[:, k] + w[:, None] * DC[:, k] + EPS32 * np.abs(rgb)
        dep += w * TM[:, k]
        ddep += dw * np.abs(TM[:, k]) + w * EPS32 * np.abs(TM[:, k]) + EPS32 * np.abs(dep)
        acc += w
        dacc += dw + EPS32 * acc
        Tn = T * E[:, k]
        dT = dT * E[:, k] + T * DE[:, k] + EPS32 * Tn
        T = Tn
    return drgb, ddep, dacc


def assert_bf16_render_close(rgb, dep, acc, ref, st, F, name=""):
    """Every ray's BF16 render outputs within bf16_render_bound of the
    oracle's BF16-mode render ``ref`` = (rgb, depth, acc) with state st."""
    drgb, ddep, dacc = bf16_render_bound(st, F)
    worst = 0.0
    for got, exp, b, what in ((rgb, ref[0], drgb, "rgb"), (dep, ref[1], ddep, "depth"),
                              (acc, ref[2], dacc, "acc")):
        if got is None:
            continue
        err = np.abs(np.asarray(got, np.float64) - exp)
        bad = err > b
        with np.errstate(divide="ignore", invalid="ignore"):
            worst = max(worst, float(np.max(np.where(b > 0, err / b, np.where(err > 0, np.inf, 0.0)),
                                            initial=0.0)))
        assert not bad.any(), (f"{name} {what}: {bad.sum()} of {bad.size} outside the per-ray bound, "
                               f"worst err {err[bad].max():.3g} vs bound {b[bad][np.argmax(err[bad])]:.3g}")
    print(f"{name}: BF16 render max err / bound = {worst:.3g}")


def lf_surface_point_error(st, F, grad_rgb, grad_depth, deta=None):
    """Per entry of the Z_C block of the light-field feature gradient, the
    error that the surface point's FP32 evaluation carries into it through
    the corner weights (a moved x_s also changes dL/dpsi(x_s) through the
    colour decoder; that part is relative to the entry's own contributions
    and the caller's factor 2 is meant for it, a measured margin rather than
    a derived one).  eta = sigmoid(o_T1) inherits the FP32 error of the
    density decoder's output (each layer's dot products off by gamma_n
    sum |terms| plus |W| times the error of their inputs, the inputs'
    interpolation off by 16 ulps of sum_j (w_j + D_j) |F_j|, r by 64 ulps);
    x_s = eta x1 + (1 - eta) x2 then moves by |d eta| |x1 - x2| per axis and
    each corner weight by sum_a |dw_j / du_a| |du_a|.  Where the density
    decoder's activations are large this exceeds the few ulps of a cell
    coordinate that the weight-sensitivity term assumes.  (C_C columns.)
    ``deta`` (per hit) replaces the derived bound on eta's error."""
    from oracle.lightfield import _lf_backward_per_hit, weight_derivatives
    ct = st.dec[0]
    if deta is None:
        FT = np.abs(np.asarray(F, np.float64)[st.corners][:, :, :ct])
        D1 = np.sum(np.abs(weight_derivatives(st.u1)), axis=2)
        D2 = np.sum(np.abs(weight_derivatives(st.u2)), axis=2)
        e = np.concatenate([16 * EPS32 * np.einsum("mj,mjc->mc", st.w1 + D1, FT),
                            16 * EPS32 * np.einsum("mj,mjc->mc", st.w2 + D2, FT),
                            64 * EPS32 * np.abs(st.r)], axis=1)
        for li, (W, b) in enumerate(st.lt):
            a = np.abs(st.actsT[li])
            absW = np.abs(W)
            n = W.shape[1] + 1
            gamma = 1.01 * n * EPS32 / (1.0 - n * EPS32)
            dz = e @ absW.T + gamma * (a @ absW.T + np.abs(b))
            e = dz
        deta = 0.25 * dz[:, 1] + 4 * EPS32
        dus = deta[:, None] * np.abs(st.x1 - st.x2) / st.h + 8 * EPS32
    else:
        dus = np.asarray(deta, np.float64)[:, None] * np.abs(st.x1 - st.x2) / st.h
    dwj = np.einsum("mja,ma->mj", np.abs(weight_derivatives(st.us)), dus)
    _, _, _, _, g_zC = _lf_backward_per_hit(st, grad_rgb, grad_depth)
    E = np.zeros((st.n_vertices, g_zC.shape[1]))
    np.add.at(E, st.corners.ravel(), (dwj[:, :, None] * np.abs(g_zC)[:, None, :]).reshape(-1, g_zC.shape[1]))
    return E


def _dense(v, st, fill):
    """Per-hit values (m, ...) into the dense per-ray layout (n, K, ...)."""
    v = np.asarray(v, np.float64)
    out = np.full((st.n, st.K) + v.shape[1:], fill)
    out[st.ray_i, st.slot_i] = v
    return out


def grad_error_ratio(got, exp, mag, unit=EPS32, wmag=None, c_w=C_W):
    """Largest (|got - exp| - 2^-24 c_w W) / (unit M) over the entries with
    M > 0 (W = the weight-sensitivity scale, 0 if not given), and the largest
    |got - exp| where M = W = 0 (no contribution: must be exact)."""
    got = np.asarray(got, np.float64)
    exp = np.asarray(exp, np.float64)
    mag = np.asarray(mag, np.float64)
    assert got.shape == exp.shape == mag.shape
    err = np.abs(got - exp)
    if wmag is not None:
        wmag = np.asarray(wmag, np.float64)
        assert wmag.shape == mag.shape
        err_m = err - EPS32 * c_w * wmag
        pos = (mag > 0) | (wmag > 0)
    else:
        err_m = err
        pos = mag > 0
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(mag[pos] > 0, err_m[pos] / (unit * mag[pos]), np.where(err_m[pos] > 0, np.inf, 0.0))
    return float(np.max(r, initial=0.0)), float(np.max(err[~pos], initial=0.0))


def assert_grad_close(got, exp, name="", rel_nw=1e-5, mag=None, c=C_FEAT, unit=EPS32, wmag=None, c_w=C_W):
    """Normwise max|err| <= rel_nw max|exp|; with ``mag`` (the oracle's
    per-entry contribution scale M) and ``wmag`` (its weight-sensitivity
    scale W) also |err| <= c unit M + c_w 2^-24 W for every entry."""
    got = np.asarray(got, np.float64)
    exp = np.asarray(exp, np.float64)
    m = np.abs(exp).max() if exp.size else 0.0
    err = np.abs(got - exp)
    assert np.all(np.isfinite(got)), f"{name}: non-finite gradient"
    if rel_nw is not None:
        nbad = int(np.sum(err > rel_nw * m))
        assert err.max(initial=0.0) <= rel_nw * m + 1e-30, \
            f"{name}: normwise {err.max()} vs {rel_nw * m} ({nbad} of {err.size} entries above)"
    if mag is not None:
        worst, at_zero = grad_error_ratio(got, exp, mag, unit, wmag, c_w)
        print(f"{name}: max (|err| - c_w 2^-24 W) / (unit M) = {worst:.4g} (bound {c:g})")
        assert at_zero == 0.0, f"{name}: entry without contributions differs by {at_zero}"
        assert worst <= c, f"{name}: per-entry error {worst:.4g} x unit x M exceeds {c:g}"


def residual_terms(g, value, target):
    """The gradient of a squared residual, g = k (value - target), taken at
    the size of its terms: k (|value| + |target|).  Another evaluation of the
    value (FP32 against FP64) moves g by a rounding error of the value, which
    relative to g is large where value and target nearly cancel; a bound's
    scale computed from these upstream sizes covers that.  0 where the
    residual is exactly zero (there both evaluations give 0)."""
    g = np.asarray(g, np.float64)
    v = np.asarray(value, np.float64)
    t = np.asarray(target, np.float64)
    r = v - t
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(r != 0, np.abs(g) * (np.abs(v) + np.abs(t)) / np.abs(r), 0.0)


def loss_scales(mag_fn, weight_fn, st, g_rgb, G_rgb, *rest, **kw):
    """Contribution and weight-sensitivity scales of a train step's gradient:
    the oracle's scales at the loss gradient plus those at the size of the
    loss terms (residual_terms), so that both the chain's own cancellations
    and the rounding of a nearly cancelling residual are covered.  Returns
    (M_features, M_params, W)."""
    mF, mp = mag_fn(st, g_rgb, *rest, **kw)
    mF2, mp2 = mag_fn(st, G_rgb, *rest, **kw)
    return mF + mF2, mp + mp2, weight_fn(st, g_rgb, *rest, **kw) + weight_fn(st, G_rgb, *rest, **kw)


def cosine(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))


# A pre-activation counts as at a kink when it lies within KINK_REL of the
# scale sum_k |W_ik a_k| + |b_i| of its dot product: FP32 evaluates a dot
# product of length <= 128 to within about 2^-17 of that scale, and the
# layer inputs carry errors of the same order from the layers before.
KINK_REL = 2.0 ** -16


def _dot_scales(layers, acts):
    return [np.abs(a) @ np.abs(W).T + np.abs(b) for (W, b), a in zip(layers, acts)]


def decoder_kinks(st):
    """Hits (of an oracle render state) with a decoder pre-activation at a
    kink: a hidden ReLU input or the sigma ReLU input within KINK_REL of its
    dot product's scale."""
    sc = _dot_scales(split_params(st.params, st.widths), st.acts)
    near = np.abs(st.out[:, 3]) < KINK_REL * sc[-1][:, 3]
    for z, s in zip(st.pres, sc[:-1]):
        near |= np.any(np.abs(z) < KINK_REL * s, axis=1)
    return near


def lf_kinks(st):
    """As decoder_kinks for the light-field state: both decoders' ReLUs, the
    tau ReLU, and the clamp of the surface point's cell coordinates."""
    scT, scC = _dot_scales(st.lt, st.actsT), _dot_scales(st.lc, st.actsC)
    near = np.abs(st.oT[:, 0]) < KINK_REL * scT[-1][:, 0]
    for z, s in list(zip(st.presT, scT[:-1])) + list(zip(st.presC, scC[:-1])):
        near |= np.any(np.abs(z) < KINK_REL * s, axis=1)
    # the clamp of the surface point's cell coordinates (evaluated to a few
    # ulps of the result)
    near |= np.any((np.abs(st.us_raw) < KINK_REL) | (np.abs(st.us_raw - 1.0) < KINK_REL), axis=1)
    return near


def psnr(a, b):
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else -10.0 * np.log10(mse)


class Case:
    """A scene + decoder on the device and in the oracle."""

    def __init__(self, svlf, leaf_ijk, depth, features, params, widths, K, tau_mode="voxel",
                 viewdir=False):
        import torch
        self.svlf = svlf
        self.viewdir = viewdir
        self.depth = depth
        self.widths = tuple(widths)
        self.K = K
        self.tau_mode = tau_mode
        self.F = np.ascontiguousarray(features, np.float32)
        self.p = np.ascontiguousarray(params, np.float32)
        self.oc = Octree(leaf_ijk, depth)
        self.scene = svlf.DeviceScene.from_host(leaf_ijk, depth, self.F, bf16=True)
        self.params = torch.from_numpy(self.p).cuda()

    @classmethod
    def from_workload(cls, svlf, w, feat_scale=1.0, sigma_bias=None, tau_mode="voxel",
                      viewdir=False):
        sc = w.scene()
        F = w.features() * np.float32(feat_scale)
        widths = tuple(w.widths)
        p = w.params().copy()
        if viewdir:
            from synth.configs import xavier_params
            widths = (widths[0] + 3,) + widths[1:]
            p = xavier_params(np.random.default_rng(len(widths) + widths[0]), widths)
        if sigma_bias is not None:
            p[-1] = sigma_bias
        return cls(svlf, sc.leaf_ijk, sc.depth, F, p, widths, w.K, tau_mode, viewdir)

    def opts(self, precision="fp32"):
        return self.svlf.make_opts(self.K, self.tau_mode, precision,
                                   self.svlf.FLAG_VIEWDIR if self.viewdir else 0)

    def rays(self, o, d):
        import torch
        return (torch.from_numpy(np.ascontiguousarray(o, np.float32)).cuda(),
                torch.from_numpy(np.ascontiguousarray(d, np.float32)).cuda())

    def gpu_render(self, o, d, precision="fp32"):
        import torch
        to, td = self.rays(o, d)
        rgb, dep, acc = self.svlf.render([self.scene], [o.shape[0]], self.params, self.widths,
                                         self.opts(precision), to, td)
        torch.cuda.synchronize()
        return rgb.cpu().numpy(), dep.cpu().numpy(), acc.cpu().numpy()

    def smooth_rays(self, o, d, margin=1e-4, bf16=False):
        """Indices of rays none of whose hits has a decoder pre-activation
        (hidden ReLU or the sigma ReLU) within `margin` of zero.  At such a
        kink FP32 and FP64 may take different one-sided derivatives, both of
        them valid, so gradient parity is checked on the other rays."""
        _, _, _, st = self.oracle(o, d, bf16=bf16)
        near = np.zeros(st.out.shape[0], bool)
        for z in st.pres:
            near |= np.any(np.abs(z) < margin, axis=1)
        near |= np.abs(st.out[:, 3]) < margin
        bad_rays = np.unique(st.ray_i[near])
        keep = np.ones(o.shape[0], bool)
        keep[bad_rays] = False
        return np.nonzero(keep)[0]

    def oracle(self, o, d, bf16=False):
        hits = oracle_trace(self.oc, o, d, self.K)
        return oracle_render(self.oc, self.F, self.p, self.widths, o, d, hits,
                             tau_mode=self.tau_mode, bf16=bf16, viewdir=self.viewdir)


class LfCase:
    """A scene with the two-decoder light-field model on the device and in
    the oracle (features [n_vertices][C_T + C_C])."""

    def __init__(self, svlf, leaf_ijk, depth, features, params, K, tau_mode="direct", viewdir=False):
        import torch
        from oracle.lightfield import n_params
        self.svlf = svlf
        self.K = K
        self.tau_mode = tau_mode
        self.viewdir = viewdir
        self.dec = tuple(svlf.LF_DECODERS)
        self.F = np.ascontiguousarray(features, np.float32)
        self.p = np.ascontiguousarray(params, np.float32)
        assert self.p.size == n_params(self.dec, viewdir)
        self.oc = Octree(leaf_ijk, depth)
        self.scene = svlf.DeviceScene.lf_from_host(leaf_ijk, depth, self.F, bf16=True)
        self.params = torch.from_numpy(self.p).cuda()

    def rows(self, g):
        """Device feature gradient (block layout) -> [n_vertices][C_T + C_C]."""
        return self.svlf.lf_feature_rows(g.cpu().numpy() if hasattr(g, "cpu") else g, self.F.shape[0])

    @classmethod
    def random(cls, svlf, seed, depth, n_obj=3, feat_sd=0.5, sigma_bias=0.5, K=8, tau_mode="direct",
               viewdir=False, rule="surface"):
        from synth.configs import tiny_workload, xavier_params
        from oracle.lightfield import widths_of
        w = tiny_workload(seed, depth, 8, (8, 32, 32, 4), K, n_obj=n_obj, rule=rule)
        sc = w.scene()
        rng = np.random.default_rng(seed + 1000)
        dec = tuple(svlf.LF_DECODERS)
        F = rng.normal(0, feat_sd, (sc.n_vertices, dec[0] + dec[1])).astype(np.float32)
        wt, wc = widths_of(dec, viewdir)
        pt = xavier_params(rng, wt)
        pt[-2] = sigma_bias                      # bias of o_T0 (tau)
        p = np.concatenate([pt, xavier_params(rng, wc)])
        return cls(svlf, sc.leaf_ijk, sc.depth, F, p, K, tau_mode, viewdir)

    def opts(self, precision="fp32"):
        return self.svlf.make_opts(self.K, self.tau_mode, precision,
                                   self.svlf.FLAG_VIEWDIR if self.viewdir else 0)

    def rays(self, o, d):
        import torch
        return (torch.from_numpy(np.ascontiguousarray(o, np.float32)).cuda(),
                torch.from_numpy(np.ascontiguousarray(d, np.float32)).cuda())

    def oracle(self, o, d, bf16=False):
        from oracle.lightfield import render_lf
        hits = oracle_trace(self.oc, o, d, self.K)
        return render_lf(self.oc, self.F, self.p, self.dec, o, d, hits, tau_mode=self.tau_mode,
                         bf16=bf16, viewdir=self.viewdir)

    def gpu_render(self, o, d, precision="fp32"):
        import torch
        to, td = self.rays(o, d)
        rgb, dep, acc = self.svlf.lf_render([self.scene], [o.shape[0]], self.params,
                                            self.opts(precision), to, td)
        torch.cuda.synchronize()
        return rgb.cpu().numpy(), dep.cpu().numpy(), acc.cpu().numpy()

    def gpu_backward(self, o, d, g_rgb, g_dep, g_acc=None, precision="fp32"):
        import torch
        to, td = self.rays(o, d)
        gF = torch.zeros(self.scene.features.shape, dtype=torch.float32, device="cuda")
        gp = torch.zeros(self.params.shape, dtype=torch.float32, device="cuda")
        t = lambda x: torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
        self.svlf.lf_render_backward([self.scene], [o.shape[0]], self.params, self.opts(precision),
                                     to, td, t(g_rgb), t(g_dep), None if g_acc is None else t(g_acc),
                                     [gF], gp)
        torch.cuda.synchronize()
        return self.rows(gF), gp.cpu().numpy()

    def smooth_rays(self, o, d, margin=1e-4):
        """Rays none of whose hits is within `margin` of a kink: a ReLU input
        of either decoder, the tau ReLU, or the clamp of the surface point's
        cell coordinates."""
        _, _, _, st = self.oracle(o, d)
        near = np.zeros(st.oT.shape[0], bool)
        for z in st.presT + st.presC:
            near |= np.any(np.abs(z) < margin, axis=1)
        near |= np.abs(st.oT[:, 0]) < margin
        near |= np.any((np.abs(st.us_raw) < margin) | (np.abs(st.us_raw - 1.0) < margin), axis=1)
        keep = np.ones(o.shape[0], bool)
        keep[np.unique(st.ray_i[near])] = False
        return np.nonzero(keep)[0]
