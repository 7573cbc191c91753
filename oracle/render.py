"""FP64 render, backward and loss of the SVLF per-ray path.

Follows SVLF section 4 with the single-decoder reading used by the library:

* per hit (leaf, t_in, t_out): the sample point is the segment midpoint
  t_mid = (t_in + t_out) / 2, p = o + t_mid d (the paper samples its colour
  features at a point inside the voxel between x1 and x2, section 4.2);
* x = psi(p; Z): trilinear interpolation of the leaf's 8 corner embeddings
  (section 4.1), u = clamp((p - lo) / h, 0, 1), w_j = prod_a (u_a or 1 - u_a);
* one ReLU MLP (section 4.5 "Architecture") maps x to 4 outputs o; the colour
  is sigmoid(o_0..2), the density sigma = ReLU(o_3);
* optical thickness (section 4 footnote: integral of density along the
  segment) tau = sigma * (t_out - t_in) / h ("voxel" mode: density in units of
  voxel edges); "direct" mode tau = sigma, "world" mode tau = sigma * dt;
* Eq. 3: c(r) = sum_i T_i (1 - e^{-tau_i}) c_i, T_i = prod_{j<i} e^{-tau_j},
  over the first min(N, K) voxels in order along the ray; depth and the
  accumulated opacity use the same weights (depth = sum w_i t_mid_i,
  acc = sum w_i); a ray with no hits gives zeros.

``viewdir=True`` appends the ray direction d (3 values) to the decoder input,
x_in = [psi(p; Z) | d]: the view-direction input the paper proposes for its
colour decoder to capture view-dependent appearance (section 6,
limitations); with one decoder it is an input of the whole MLP.

``bf16=True`` rounds (round to nearest even) the features, the weights, the
MLP input x and every hidden activation after ReLU to bfloat16 before use;
in the backward it also rounds each layer's incoming gradient (dL/dz) to
bfloat16 before it enters the weight, bias and input gradients.  All
accumulation stays in FP64.

No GPU code and no automatic differentiation is used; the backward is
derived by hand from the formulas above.
"""

from __future__ import annotations

import numpy as np

from .octree import Octree

TAU_MODES = ("voxel", "direct", "world")


def bf16_round(x):
    """Round FP64 values to the nearest bfloat16 (8 significant bits, ties
    to even, bfloat16 exponent range including its subnormals)."""
    x = np.asarray(x, np.float64)
    m, e = np.frexp(x)                     # x = m 2^e, 0.5 <= |m| < 1
    e = np.maximum(e, -125)                # subnormal spacing 2^-133
    scale = np.ldexp(1.0, 8 - e)
    return np.rint(x * scale) / scale


def split_params(params, widths):
    """Views W_l (out, in) and b_l (out,) of the flat FP64 parameter vector."""
    params = np.asarray(params, np.float64)
    out, off = [], 0
    for fi, fo in zip(widths[:-1], widths[1:]):
        W = params[off:off + fo * fi].reshape(fo, fi)
        off += fo * fi
        b = params[off:off + fo]
        off += fo
        out.append((W, b))
    if off != params.size:
        raise ValueError("parameter vector does not match widths")
    return out


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def mlp_forward(params, widths, X, bf16=False):
    """Returns (o, acts, pres): output pre-activations o (n, 4), the inputs
    of every layer acts[l] and hidden pre-activations pres[l]."""
    layers = split_params(params, widths)
    r = bf16_round if bf16 else (lambda v: v)
    a = r(np.asarray(X, np.float64))
    acts, pres = [], []
    for li, (W, b) in enumerate(layers):
        acts.append(a)
        z = a @ r(W).T + b
        if li < len(layers) - 1:
            pres.append(z)
            a = r(np.maximum(z, 0.0))
        else:
            return z, acts, pres
    raise ValueError("empty MLP")


def interpolation_weights(u):
    """w (n, 8): corner j weight = prod over axes of u_a if bit a of j else
    1 - u_a (textbook trilinear weights)."""
    w = np.ones((u.shape[0], 8))
    for j in range(8):
        for a in range(3):
            w[:, j] *= u[:, a] if (j >> a) & 1 else 1.0 - u[:, a]
    return w


def weight_sensitivity(u):
    """D (n, 8): sum over the axes a of |d w_j / d u_a| for the textbook
    trilinear weights, i.e. how strongly corner j's weight responds to an
    error in the cell coordinates of the sample point (d w_j / d u_a is the
    product of the other two axes' factors, with the sign of bit a of j)."""
    D = np.zeros((u.shape[0], 8))
    for j in range(8):
        for a in range(3):
            other = np.ones(u.shape[0])
            for b in range(3):
                if b != a:
                    other *= u[:, b] if (j >> b) & 1 else 1.0 - u[:, b]
            D[:, j] += other
    return D


class RenderState:
    """Everything the backward needs (dense [n_rays, K] layout)."""


def render(octree: Octree, features, params, widths, o, d, hits, tau_mode="voxel",
           bf16=False, viewdir=False):
    """Forward render.  ``hits`` = (hit_leaf, hit_tin, hit_tout, hit_count)
    from ``trace.trace_hits``.  Returns (rgb (n,3), depth (n,), acc (n,),
    state)."""
    if tau_mode not in TAU_MODES:
        raise ValueError(tau_mode)
    hit_leaf, hit_tin, hit_tout, _ = hits
    n, K = hit_leaf.shape
    o = np.asarray(o, np.float64)
    d = np.asarray(d, np.float64)
    F = np.asarray(features, np.float64)
    if bf16:
        F = bf16_round(F)
    valid = hit_leaf >= 0
    ray_i, slot_i = np.nonzero(valid)
    leaf = hit_leaf[ray_i, slot_i].astype(np.int64)
    t0 = hit_tin[ray_i, slot_i].astype(np.float64)
    t1 = hit_tout[ray_i, slot_i].astype(np.float64)
    L = octree.depth
    h = 2.0 / (1 << L)
    tm = 0.5 * (t0 + t1)
    p = o[ray_i] + tm[:, None] * d[ray_i]
    lo = -1.0 + octree.leaf_ijk[leaf].astype(np.float64) * h
    u = np.clip((p - lo) / h, 0.0, 1.0)
    wj = interpolation_weights(u)
    corners = octree.leaf_corners[leaf]                 # (m, 8)
    X = np.einsum("mj,mjc->mc", wj, F[corners])
    X_in = np.concatenate([X, d[ray_i]], axis=1) if viewdir else X
    if widths[0] != X_in.shape[1]:
        raise ValueError("decoder input width does not match the features (+3 with viewdir)")
    out, acts, pres = mlp_forward(params, widths, X_in, bf16)
    c = sigmoid(out[:, :3])
    sigma = np.maximum(out[:, 3], 0.0)
    dt = t1 - t0
    dtau = {"voxel": dt / h, "direct": np.ones_like(dt), "world": dt}[tau_mode]
    tau_h = sigma * dtau
    # dense per-ray layout, zero padded
    tau = np.zeros((n, K))
    col = np.zeros((n, K, 3))
    tmid = np.zeros((n, K))
    tau[ray_i, slot_i] = tau_h
    col[ray_i, slot_i] = c
    tmid[ray_i, slot_i] = tm
    # Eq. 3
    T = np.exp(-(np.cumsum(tau, axis=1) - tau))
    alpha = -np.expm1(-tau)
    w = T * alpha
    rgb = np.sum(w[:, :, None] * col, axis=1)
    depth = np.sum(w * tmid, axis=1)
    acc = np.sum(w, axis=1)
    st = RenderState()
    st.__dict__.update(dict(octree=octree, widths=tuple(widths), params=np.asarray(params, np.float64),
                            bf16=bf16, n=n, K=K, ray_i=ray_i, slot_i=slot_i, u=u, wj=wj,
                            corners=corners, X=X, out=out, acts=acts, pres=pres, c=c,
                            sigma=sigma, dtau=dtau, tau=tau, col=col, tmid=tmid, T=T,
                            w=w, rgb=rgb, depth=depth, acc=acc, n_vertices=F.shape[0],
                            C=F.shape[1]))
    return rgb, depth, acc, st


def _backward_per_hit(st, grad_rgb, grad_depth, grad_acc=None):
    """The backward of ``render`` up to the point where per-hit quantities
    are summed: returns, for the decoder layers (first to last), the pairs
    (dL/dz of every hit, the layer input of every hit), and dL/dX of every
    hit (the decoder input's feature part)."""
    n, K = st.n, st.K
    g_rgb = np.asarray(grad_rgb, np.float64).reshape(n, 3)
    g_d = np.asarray(grad_depth, np.float64).reshape(n)
    g_a = np.zeros(n) if grad_acc is None else np.asarray(grad_acc, np.float64).reshape(n)
    T, w, tau, col, tmid = st.T, st.w, st.tau, st.col, st.tmid
    T_next = T * np.exp(-tau)
    # suffix sums S_i = sum_{j > i} w_j x_j
    wc = w[:, :, None] * col
    S_c = np.sum(wc, axis=1, keepdims=True) - np.cumsum(wc, axis=1)
    wt = w * tmid
    S_t = np.sum(wt, axis=1, keepdims=True) - np.cumsum(wt, axis=1)
    S_a = np.sum(w, axis=1, keepdims=True) - np.cumsum(w, axis=1)
    g_tau = (np.sum(g_rgb[:, None, :] * (T_next[:, :, None] * col - S_c), axis=2)
             + g_d[:, None] * (T_next * tmid - S_t)
             + g_a[:, None] * (T_next - S_a))
    g_col = w[:, :, None] * g_rgb[:, None, :]
    ri, si = st.ray_i, st.slot_i
    g_sigma = g_tau[ri, si] * st.dtau
    g_out = np.zeros_like(st.out)
    g_out[:, 3] = np.where(st.out[:, 3] > 0.0, g_sigma, 0.0)
    c = st.c
    g_out[:, :3] = g_col[ri, si] * c * (1.0 - c)
    # MLP backward
    layers = split_params(st.params, st.widths)
    r = bf16_round if st.bf16 else (lambda v: v)
    per_layer = []
    g_z = g_out
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        g_zr = r(g_z)
        per_layer.append((g_zr, st.acts[li]))
        g_a = g_zr @ r(W)
        if li > 0:
            g_z = np.where(st.pres[li - 1] > 0.0, g_a, 0.0)
        else:
            g_X = g_a[:, :st.C]          # the view direction takes no gradient
    per_layer.reverse()
    return per_layer, g_X


def render_backward(st, grad_rgb, grad_depth, grad_acc=None):
    """Hand-derived backward of ``render`` for upstream gradients of rgb,
    depth and acc.  Returns (grad_features (n_vertices, C), grad_params)."""
    per_layer, g_X = _backward_per_hit(st, grad_rgb, grad_depth, grad_acc)
    grad_params = np.concatenate([np.concatenate([(g_zr.T @ a).ravel(), np.sum(g_zr, axis=0)])
                                  for g_zr, a in per_layer])
    grad_F = np.zeros((st.n_vertices, st.C))
    contrib = st.wj[:, :, None] * g_X[:, None, :]       # (m, 8, C)
    np.add.at(grad_F, st.corners.ravel(), contrib.reshape(-1, st.C))
    return grad_F, grad_params


def sigma_output_term_magnitude(st, grad_rgb, grad_depth, grad_acc=None):
    """Per hit, the sum of absolute values of the terms that make up dL/do_3
    (the decoder's density output; test infrastructure).  Eq. 3's backward
    gives dL/dtau = sum_ch g_ch (T_next c_ch - S_ch) + g_d (T_next t - S_t)
    + g_a (T_next - S_a) with S the suffix sums over the ray's later hits;
    on a ray with many hits these terms nearly cancel, and another
    evaluation of dL/dtau is accurate to their size, not to its own.
    G = sum_ch |g_ch| (T_next c_ch + S_ch) + |g_d| (T_next t + S_t) +
    |g_a| (T_next + S_a), times dtau where o_3 > 0.  Returns (m,)."""
    n = st.n
    g_rgb = np.asarray(grad_rgb, np.float64).reshape(n, 3)
    g_d = np.asarray(grad_depth, np.float64).reshape(n)
    g_a = np.zeros(n) if grad_acc is None else np.asarray(grad_acc, np.float64).reshape(n)
    T, w, tau, col, tmid = st.T, st.w, st.tau, st.col, st.tmid
    T_next = T * np.exp(-tau)
    wc = w[:, :, None] * col
    S_c = np.sum(wc, axis=1, keepdims=True) - np.cumsum(wc, axis=1)
    wt = w * tmid
    S_t = np.sum(wt, axis=1, keepdims=True) - np.cumsum(wt, axis=1)
    S_a = np.sum(w, axis=1, keepdims=True) - np.cumsum(w, axis=1)
    G = (np.sum(np.abs(g_rgb)[:, None, :] * (T_next[:, :, None] * col + S_c), axis=2)
         + np.abs(g_d)[:, None] * (T_next * np.abs(tmid) + np.abs(S_t)) + np.abs(g_a)[:, None] * (T_next + S_a))
    G = G[st.ray_i, st.slot_i] * st.dtau
    return np.where(st.out[:, 3] > 0.0, G, 0.0)


def decoder_input_jacobian(st):
    """Per hit, d o_k / d X for each of the decoder's 4 outputs (the feature
    part of the input; the hit's ReLU pattern; bfloat16 weights in the BF16
    mode).  Returns (m, 4, C)."""
    layers = split_params(st.params, st.widths)
    r = bf16_round if st.bf16 else (lambda v: v)
    m = st.out.shape[0]
    J = np.zeros((m, 4, st.C))
    for k in range(4):
        g_z = np.zeros((m, 4))
        g_z[:, k] = 1.0
        for li in range(len(layers) - 1, -1, -1):
            g_a = g_z @ r(layers[li][0])
            if li > 0:
                g_z = np.where(st.pres[li - 1] > 0.0, g_a, 0.0)
        J[:, k, :] = g_a[:, :st.C]
    return J


def render_backward_hit_magnitude(st, grad_rgb, grad_depth, grad_acc=None, conditioned=False):
    """Scale of the per-hit contributions behind every entry of
    ``render_backward`` (test infrastructure: the scale of per-entry rounding
    bounds of another evaluation of the same sums).

    Every gradient entry is a sum over hits: a feature row receives
    w_j dL/dx_h from each hit h that has the vertex as corner j, a decoder
    weight dL/dz_h[i] a_h[k] from every hit, a bias dL/dz_h[i].  Returns,
    per entry, S + R with
      S = the sum over those hits of |contribution|, and
      R = the sum over those hits of the largest |contribution| the same hit
          makes to the entry's group (a feature row: w_j max_c |dL/dx_h[c]|;
          a layer's weights: max_i |dL/dz_h[i]| max_k |a_h[k]|; a layer's
          biases: max_i |dL/dz_h[i]|).
    S bounds the entry (triangle inequality), also when the hits' terms
    cancel; R is the scale of a hit's own evaluation error, which arises
    over the whole group (the decoder backward mixes all its units).  With
    ``conditioned`` a hit's dL/dX is taken at its conditioning,
    sum_{k<3} |J_k| |dL/do_k| + |J_3| G (``decoder_input_jacobian``,
    ``sigma_output_term_magnitude``), in place of its absolute value, for the
    feature entries.  Returns (M_features (n_vertices, C), M_params)."""
    per_layer, g_X = _backward_per_hit(st, grad_rgb, grad_depth, grad_acc)
    mags = []
    for g_zr, a in per_layer:
        gz, aa = np.abs(g_zr), np.abs(a)
        rW = float(np.sum(gz.max(axis=1, initial=0.0) * aa.max(axis=1, initial=0.0)))
        rb = float(np.sum(gz.max(axis=1, initial=0.0)))
        mags.append(np.concatenate([(gz.T @ aa).ravel() + rW, np.sum(gz, axis=0) + rb]))
    M_params = np.concatenate(mags)
    gx = np.abs(g_X)
    if conditioned:
        J = np.abs(decoder_input_jacobian(st))
        g_out = np.abs(per_layer[-1][0])
        G = sigma_output_term_magnitude(st, grad_rgb, grad_depth, grad_acc)
        gx = np.einsum("mkc,mk->mc", J[:, :3, :], g_out[:, :3]) + J[:, 3, :] * G[:, None]
    row = st.wj[:, :, None] * (gx[:, None, :] + gx.max(axis=1, initial=0.0)[:, None, None])
    M_F = np.zeros((st.n_vertices, st.C))
    np.add.at(M_F, st.corners.ravel(), row.reshape(-1, st.C))
    return M_F, M_params


def render_backward_weight_scale(st, grad_rgb, grad_depth, grad_acc=None):
    """Per entry of the feature gradient of ``render_backward``, the sum over
    the hits that reach it of D_j |dL/dx_h[c]| (``weight_sensitivity`` of
    the hit's sample point; test infrastructure).  An error e in the cell
    coordinates of a hit's sample point moves the hit's contribution to the
    entry by at most e D_j |dL/dx_h[c]|: this is the scale of that part of a
    rounding bound, which a weight near zero (a sample point near a face of
    its cell) would otherwise make unbounded relative to the contribution."""
    _, g_X = _backward_per_hit(st, grad_rgb, grad_depth, grad_acc)
    D = weight_sensitivity(st.u)
    M_w = np.zeros((st.n_vertices, st.C))
    np.add.at(M_w, st.corners.ravel(), (D[:, :, None] * np.abs(g_X)[:, None, :]).reshape(-1, st.C))
    return M_w


def loss(rgb, depth, rgb_t, depth_t, lam_depth=0.1):
    """L = mean over rays and channels of (rgb - rgb*)^2
         + lam * mean over rays of |depth - depth*|; returns (L, dL/drgb,
    dL/ddepth) with sign(0) = 0."""
    rgb = np.asarray(rgb, np.float64)
    depth = np.asarray(depth, np.float64)
    n = rgb.shape[0]
    dr = rgb - np.asarray(rgb_t, np.float64)
    dd = depth - np.asarray(depth_t, np.float64)
    L = np.sum(dr * dr) / (3.0 * n) + lam_depth * np.sum(np.abs(dd)) / n
    return L, 2.0 * dr / (3.0 * n), lam_depth * np.sign(dd) / n


def psnr(img, ref, peak=1.0):
    mse = np.mean((np.asarray(img, np.float64) - np.asarray(ref, np.float64)) ** 2)
    return float("inf") if mse == 0 else 10.0 * np.log10(peak * peak / mse)
