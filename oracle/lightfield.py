"""FP64 oracle of the paper's voxel light-field function (SVLF sections
4.1-4.3, Eq. 1-3): two decoders, a ray parameterisation and two gathers per
crossed voxel.

TEST INFRASTRUCTURE ONLY (see the package header).

For every hit (leaf with lo, edge h; entry t_in, exit t_out) of a ray (o, d):

* ray parameterisation (section 4.1): the ray meets the smallest sphere
  around the voxel (centre c = lo + h/2, radius R = h sqrt(3)/2) at
  p1, p2 (ascending t along the ray); r = [p1~ | p2~] with
  p_i~ = (p_i - c) / |p_i - c| (vectors from the voxel centre, unit norm);
* x1 = o + t_in d, x2 = o + t_out d (the ray-voxel intersection points);
* z_T = [psi(x1; Z_T) | psi(x2; Z_T)] with psi the trilinear interpolation of
  the voxel's corner embeddings (section 4.1), u = clamp((x - lo)/h, 0, 1);
* density decoder F_T on [z_T | r] (ReLU MLP): its two outputs give the
  optical thickness tau = ReLU(o_0) (times dt/h or dt in the "voxel" /
  "world" modes; the paper's decoder outputs tau itself, the "direct" mode)
  and the mixing factor eta = sigmoid(o_1);
* surface point x_s = eta x1 + (1 - eta) x2 (at ray parameter
  t_s = eta t_in + (1 - eta) t_out), u_s = clamp((x_s - lo)/h, 0, 1);
* colour decoder F_C on [psi(x_s; Z_C) | r] (and the ray direction d when
  ``viewdir``): c = sigmoid(o_0..2);
* Eq. 3 over the first min(N, K) hits with weights w_i = T_i (1 - e^-tau_i);
  depth = sum w_i t_s,i; acc = sum w_i.

Z_T and Z_C are the two column blocks of one per-vertex table
F = [Z_T | Z_C] (C_T + C_C columns).  The parameter vector holds F_T's layers
then F_C's, each layer as W[out][in] followed by b[out].

``bf16=True`` rounds to bfloat16 the features, the weights, both decoders'
inputs and hidden activations (after ReLU), and in the backward every
layer's incoming gradient, as ``render.py`` does for the single decoder.

The backward is derived by hand (no automatic differentiation): compositing
as in ``render.render_backward``, then the colour decoder, the gradient of
the trilinear interpolation with respect to the sample point (which carries
dL/deta through x_s), the density decoder and the scatter of both feature
gradients to the corners.  The clamp of u_s passes gradient where the
unclamped coordinate lies in [0, 1].
"""

from __future__ import annotations

import numpy as np

from .octree import Octree
from .render import bf16_round, interpolation_weights, sigmoid, split_params

TAU_MODES = ("voxel", "direct", "world")


def widths_of(dec, viewdir=False):
    """(density widths, colour widths) of dec = (C_T, C_C, H, nh_T, nh_C)."""
    ct, cc, h, nht, nhc = dec
    wt = (2 * ct + 6,) + (h,) * nht + (2,)
    wc = (cc + 6 + (3 if viewdir else 0),) + (h,) * nhc + (3,)
    return wt, wc


def n_params(dec, viewdir=False):
    n = 0
    for w in widths_of(dec, viewdir):
        n += sum(a * b + b for a, b in zip(w[:-1], w[1:]))
    return n


def sphere_param(o, d, lo, h):
    """r (m, 6) and the two sphere parameters (t_a, t_b) for rays (o, d)
    against the bounding spheres of cells [lo, lo + h)."""
    c = lo + 0.5 * h
    R2 = 0.75 * h * h
    y = o - c
    a = np.sum(d * d, axis=1)
    b = 2.0 * np.sum(d * y, axis=1)
    cc = np.sum(y * y, axis=1) - R2
    sq = np.sqrt(np.maximum(b * b - 4.0 * a * cc, 0.0))
    ta = (-b - sq) / (2.0 * a)
    tb = (-b + sq) / (2.0 * a)
    p1 = o + ta[:, None] * d - c
    p2 = o + tb[:, None] * d - c
    r = np.concatenate([p1 / np.linalg.norm(p1, axis=1, keepdims=True),
                        p2 / np.linalg.norm(p2, axis=1, keepdims=True)], axis=1)
    return r, ta, tb


def _mlp(layers, X, rnd):
    """Forward of a ReLU MLP; returns (out, acts, pres)."""
    a = rnd(X)
    acts, pres = [], []
    for li, (W, b) in enumerate(layers):
        acts.append(a)
        z = a @ rnd(W).T + b
        if li < len(layers) - 1:
            pres.append(z)
            a = rnd(np.maximum(z, 0.0))
        else:
            return z, acts, pres
    raise ValueError("empty MLP")


def _mlp_backward_terms(layers, acts, pres, g_out, rnd):
    """Backward of ``_mlp`` up to the sums over hits: returns (per layer in
    order, the pair (dL/dz of every hit, the layer input of every hit)),
    gradient of the input)."""
    terms = []
    g_z = g_out
    g_in = None
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        g_zr = rnd(g_z)
        terms.append((g_zr, acts[li]))
        g_a = g_zr @ rnd(W)
        if li > 0:
            g_z = np.where(pres[li - 1] > 0.0, g_a, 0.0)
        else:
            g_in = g_a
    terms.reverse()
    return terms, g_in


def weight_derivatives(u):
    """dw (m, 8, 3): d w_j / d u_a of the trilinear weights."""
    m = u.shape[0]
    dw = np.ones((m, 8, 3))
    for j in range(8):
        for a in range(3):
            for b in range(3):
                bit = (j >> b) & 1
                if b == a:
                    dw[:, j, a] *= 1.0 if bit else -1.0
                else:
                    dw[:, j, a] *= u[:, b] if bit else 1.0 - u[:, b]
    return dw


class LFState:
    """Everything the backward needs."""


def render_lf(octree: Octree, features, params, dec, o, d, hits, tau_mode="direct", bf16=False,
              viewdir=False):
    """Forward render with the two-decoder function.  Returns (rgb, depth,
    acc, state)."""
    if tau_mode not in TAU_MODES:
        raise ValueError(tau_mode)
    ct, cc, H, nht, nhc = dec
    wt, wc = widths_of(dec, viewdir)
    rnd = bf16_round if bf16 else (lambda v: v)
    F = np.asarray(features, np.float64)
    if F.shape[1] != ct + cc:
        raise ValueError("features must have C_T + C_C columns")
    if bf16:
        F = bf16_round(F)
    p = np.asarray(params, np.float64)
    nt = sum(a * b + b for a, b in zip(wt[:-1], wt[1:]))
    if p.size != n_params(dec, viewdir):
        raise ValueError("parameter vector does not match the decoders")
    lt = split_params(p[:nt], wt)
    lc = split_params(p[nt:], wc)
    hit_leaf, hit_tin, hit_tout, _ = hits
    n, K = hit_leaf.shape
    o = np.asarray(o, np.float64)
    d = np.asarray(d, np.float64)
    ray_i, slot_i = np.nonzero(hit_leaf >= 0)
    leaf = hit_leaf[ray_i, slot_i].astype(np.int64)
    t0 = hit_tin[ray_i, slot_i].astype(np.float64)
    t1 = hit_tout[ray_i, slot_i].astype(np.float64)
    h = 2.0 / (1 << octree.depth)
    lo = -1.0 + octree.leaf_ijk[leaf].astype(np.float64) * h
    oo, dd = o[ray_i], d[ray_i]
    x1 = oo + t0[:, None] * dd
    x2 = oo + t1[:, None] * dd
    r, _, _ = sphere_param(oo, dd, lo, h)
    corners = octree.leaf_corners[leaf]
    u1 = np.clip((x1 - lo) / h, 0.0, 1.0)
    u2 = np.clip((x2 - lo) / h, 0.0, 1.0)
    w1 = interpolation_weights(u1)
    w2 = interpolation_weights(u2)
    FT = F[corners][:, :, :ct]                      # (m, 8, C_T)
    FC = F[corners][:, :, ct:]                      # (m, 8, C_C)
    zT = np.concatenate([np.einsum("mj,mjc->mc", w1, FT), np.einsum("mj,mjc->mc", w2, FT)], axis=1)
    XT = np.concatenate([zT, r], axis=1)
    oT, actsT, presT = _mlp(lt, XT, rnd)
    sigma = np.maximum(oT[:, 0], 0.0)
    eta = sigmoid(oT[:, 1])
    dt = t1 - t0
    dtau = {"voxel": dt / h, "direct": np.ones_like(dt), "world": dt}[tau_mode]
    tau_h = sigma * dtau
    xs = eta[:, None] * x1 + (1.0 - eta)[:, None] * x2
    ts = eta * t0 + (1.0 - eta) * t1
    us_raw = (xs - lo) / h
    us = np.clip(us_raw, 0.0, 1.0)
    ws = interpolation_weights(us)
    zC = np.einsum("mj,mjc->mc", ws, FC)
    XC = np.concatenate([zC, r] + ([dd] if viewdir else []), axis=1)
    oC, actsC, presC = _mlp(lc, XC, rnd)
    c = sigmoid(oC)
    tau = np.zeros((n, K))
    col = np.zeros((n, K, 3))
    tsd = np.zeros((n, K))
    tau[ray_i, slot_i] = tau_h
    col[ray_i, slot_i] = c
    tsd[ray_i, slot_i] = ts
    T = np.exp(-(np.cumsum(tau, axis=1) - tau))
    w = T * -np.expm1(-tau)
    rgb = np.sum(w[:, :, None] * col, axis=1)
    depth = np.sum(w * tsd, axis=1)
    acc = np.sum(w, axis=1)
    st = LFState()
    st.__dict__.update(dict(dec=tuple(dec), viewdir=viewdir, bf16=bf16, n=n, K=K, ray_i=ray_i,
                            slot_i=slot_i, lt=lt, lc=lc, nt=nt, corners=corners, FC=FC, h=h,
                            t0=t0, t1=t1, u1=u1, u2=u2, w1=w1, w2=w2, us_raw=us_raw, us=us,
                            ws=ws, x1=x1, x2=x2, r=r, oT=oT, actsT=actsT, presT=presT, eta=eta,
                            sigma=sigma, dtau=dtau, oC=oC, actsC=actsC, presC=presC, c=c,
                            tau=tau, col=col, ts=tsd, T=T, w=w, n_vertices=F.shape[0],
                            C=F.shape[1]))
    return rgb, depth, acc, st


def surface_slots(hits, t_depth):
    """Per ray, the slot of the hit whose [t_in, t_out) holds the target depth
    (compared in FP32, the precision of the hit list), or -1 (section 4.4:
    the voxel containing the surface point seen by the ray)."""
    _, tin, tout, cnt = hits
    t = np.asarray(t_depth, np.float32)[:, None]
    K = tin.shape[1]
    valid = np.arange(K)[None, :] < cnt[:, None]
    inside = valid & (tin <= t) & (t < tout)
    return np.where(inside.any(axis=1), np.argmax(inside, axis=1), -1)


def stage_loss(st, hits, rgb, t_rgb, t_depth, kind, lam_eta=1.0, lam_tau=0.0, loss_scale=1.0):
    """The staged loss of section 4.4 (Eq. 4).  Per ray with a surface voxel
    v (``surface_slots``), eta* = (t_out - t*) / (t_out - t_in) puts x_s on the
    target surface point; e_v = e^{-tau_v}.
      "surface": sum over rays with v of |c_v - c*|^2 + lam_eta (eta_v - eta*)^2
                 + lam_tau e_v^2;
      "volume":  sum over rays of |c(r) - c*|^2 plus the same eta and tau terms
                 of the rays that have v;
    times loss_scale.  Returns (L, dL/drgb (n, 3), per-hit direct gradients
    (dL/dc (m, 3), dL/deta (m,), dL/dtau (m,)))."""
    ls = float(loss_scale)
    n = st.n
    t_rgb = np.asarray(t_rgb, np.float64).reshape(n, 3)
    t_d = np.asarray(t_depth, np.float32).astype(np.float64)
    slot = surface_slots(hits, t_depth)
    m = st.ray_i.size
    hit_of = {(int(r_), int(s_)): i for i, (r_, s_) in enumerate(zip(st.ray_i, st.slot_i))}
    g_c = np.zeros((m, 3))
    g_eta = np.zeros(m)
    g_tau = np.zeros(m)
    L = 0.0
    g_rgb = np.zeros((n, 3))
    if kind == "volume":
        e = np.asarray(rgb, np.float64) - t_rgb
        L += ls * np.sum(e * e)
        g_rgb = 2.0 * ls * e
    elif kind != "surface":
        raise ValueError(kind)
    for r_ in np.nonzero(slot >= 0)[0]:
        i = hit_of[(int(r_), int(slot[r_]))]
        t0, t1 = st.t0[i], st.t1[i]
        eta_gt = (t1 - t_d[r_]) / (t1 - t0)
        ev = np.exp(-st.tau[r_, slot[r_]])
        if kind == "surface":
            ec = st.c[i] - t_rgb[r_]
            L += ls * np.sum(ec * ec)
            g_c[i] = 2.0 * ls * ec
        L += ls * (lam_eta * (st.eta[i] - eta_gt) ** 2 + lam_tau * ev * ev)
        g_eta[i] = 2.0 * ls * lam_eta * (st.eta[i] - eta_gt)
        g_tau[i] = -2.0 * ls * lam_tau * ev * ev
    return L, g_rgb, (g_c, g_eta, g_tau)


def _lf_backward_per_hit(st, grad_rgb, grad_depth, grad_acc=None, hit_grads=None):
    """The backward of ``render_lf`` up to the point where per-hit quantities
    are summed: returns the per-layer pairs (dL/dz of every hit, the layer
    input of every hit) of the density decoder and of the colour decoder,
    and per hit dL/dpsi(x1), dL/dpsi(x2) (Z_T part) and dL/dpsi(x_s) (Z_C
    part)."""
    ct, cc = st.dec[0], st.dec[1]
    rnd = bf16_round if st.bf16 else (lambda v: v)
    n = st.n
    g_rgb = np.asarray(grad_rgb, np.float64).reshape(n, 3)
    g_d = np.asarray(grad_depth, np.float64).reshape(n)
    g_a = np.zeros(n) if grad_acc is None else np.asarray(grad_acc, np.float64).reshape(n)
    T, w, tau, col, ts = st.T, st.w, st.tau, st.col, st.ts
    Tn = T * np.exp(-tau)
    wc = w[:, :, None] * col
    S_c = np.sum(wc, axis=1, keepdims=True) - np.cumsum(wc, axis=1)
    wt = w * ts
    S_t = np.sum(wt, axis=1, keepdims=True) - np.cumsum(wt, axis=1)
    S_a = np.sum(w, axis=1, keepdims=True) - np.cumsum(w, axis=1)
    g_tau = (np.sum(g_rgb[:, None, :] * (Tn[:, :, None] * col - S_c), axis=2)
             + g_d[:, None] * (Tn * ts - S_t) + g_a[:, None] * (Tn - S_a))
    ri, si = st.ray_i, st.slot_i
    g_c = w[ri, si][:, None] * g_rgb[ri]                 # dL/dc per hit
    g_ts = w[ri, si] * g_d[ri]                           # dL/dt_s per hit
    g_tau_hit = g_tau[ri, si]
    g_eta_direct = np.zeros(ri.size)
    if hit_grads is not None:
        g_c = g_c + hit_grads[0]
        g_eta_direct = hit_grads[1]
        g_tau_hit = g_tau_hit + hit_grads[2]
    # colour decoder
    gC_out = g_c * st.c * (1.0 - st.c)
    termsC, g_XC = _mlp_backward_terms(st.lc, st.actsC, st.presC, gC_out, rnd)
    g_zC = g_XC[:, :cc]
    # gradient through the sample point: psi(x_s) = sum_j w_j(u_s) F_j
    dw = weight_derivatives(st.us)                       # (m, 8, 3)
    proj = np.einsum("mjc,mc->mj", st.FC, g_zC)          # F_j . dL/dz_C
    g_us = np.einsum("mja,mj->ma", dw, proj)
    inside = (st.us_raw >= 0.0) & (st.us_raw <= 1.0)
    g_xs = np.where(inside, g_us, 0.0) / st.h            # dL/dx_s
    g_eta = g_ts * (st.t0 - st.t1) + np.sum(g_xs * (st.x1 - st.x2), axis=1) + g_eta_direct
    # density decoder
    gT_out = np.zeros_like(st.oT)
    gT_out[:, 0] = np.where(st.oT[:, 0] > 0.0, g_tau_hit * st.dtau, 0.0)
    gT_out[:, 1] = g_eta * st.eta * (1.0 - st.eta)
    termsT, g_XT = _mlp_backward_terms(st.lt, st.actsT, st.presT, gT_out, rnd)
    g_z1, g_z2 = g_XT[:, :ct], g_XT[:, ct:2 * ct]
    return termsT, termsC, g_z1, g_z2, g_zC


def render_lf_backward(st, grad_rgb, grad_depth, grad_acc=None, hit_grads=None):
    """Hand-derived backward of ``render_lf``.  ``hit_grads`` = per-hit
    direct gradients (dL/dc, dL/deta, dL/dtau) added to those coming through
    the compositing (``stage_loss``).  Returns (grad_features
    (n_vertices, C_T + C_C), grad_params)."""
    ct, cc = st.dec[0], st.dec[1]
    termsT, termsC, g_z1, g_z2, g_zC = _lf_backward_per_hit(st, grad_rgb, grad_depth, grad_acc,
                                                            hit_grads)
    grad_F = np.zeros((st.n_vertices, st.C))
    cT = st.w1[:, :, None] * g_z1[:, None, :] + st.w2[:, :, None] * g_z2[:, None, :]
    np.add.at(grad_F[:, :ct], st.corners.ravel(), cT.reshape(-1, ct))
    cC = st.ws[:, :, None] * g_zC[:, None, :]
    np.add.at(grad_F[:, ct:], st.corners.ravel(), cC.reshape(-1, cc))
    flat = []
    for g_zr, a in termsT + termsC:
        flat += [(g_zr.T @ a).ravel(), np.sum(g_zr, axis=0)]
    return grad_F, np.concatenate(flat)


def render_lf_backward_weight_scale(st, grad_rgb, grad_depth, grad_acc=None, hit_grads=None):
    """As ``render.render_backward_weight_scale`` for the light-field
    backward: a Z_T entry sums D1_j |dL/dpsi(x1)[c]| + D2_j |dL/dpsi(x2)[c]|
    over the hits that reach it, a Z_C entry D_s,j |dL/dpsi(x_s)[c]|, with
    D = sum over axes of |d w_j / d u_a| at the entry point, the exit point
    and the surface point (test infrastructure: the scale of the part of a
    rounding bound due to errors in those points' cell coordinates)."""
    ct = st.dec[0]
    _, _, g_z1, g_z2, g_zC = _lf_backward_per_hit(st, grad_rgb, grad_depth, grad_acc, hit_grads)
    D1, D2, Ds = (np.sum(np.abs(weight_derivatives(u)), axis=2) for u in (st.u1, st.u2, st.us))
    M_w = np.zeros((st.n_vertices, st.C))
    mT = D1[:, :, None] * np.abs(g_z1)[:, None, :] + D2[:, :, None] * np.abs(g_z2)[:, None, :]
    np.add.at(M_w[:, :ct], st.corners.ravel(), mT.reshape(-1, ct))
    mC = Ds[:, :, None] * np.abs(g_zC)[:, None, :]
    np.add.at(M_w[:, ct:], st.corners.ravel(), mC.reshape(-1, g_zC.shape[1]))
    return M_w


def density_output_term_magnitudes(st, grad_rgb, grad_depth, grad_acc=None, hit_grads=None):
    """Per hit, the sums of absolute values of the terms that make up
    dL/do_T0 and dL/do_T1 (the density decoder's output pre-activations;
    test infrastructure: where those terms cancel, the gradient is a small
    difference of large terms and another evaluation of it is accurate to
    their size, not to its own).  dL/dtau = sum_ch g_ch (T_next c_ch - S_ch)
    + g_d (T_next t_s - S_t) + g_a (T_next - S_a) (+ a direct term) gives
    G_tau = sum_ch |g_ch| (T_next c_ch + S_ch) + |g_d| (T_next t_s + S_t) +
    |g_a| (T_next + S_a) (+ |direct|), times dtau where o_T0 > 0; dL/deta =
    dL/dt_s (t_in - t_out) + dL/dx_s . (x1 - x2) (+ direct) gives
    G_eta = |dL/dt_s| |t_in - t_out| + sum_a |x1 - x2|_a G_xs,a (+ |direct|)
    with G_xs,a = sum_j |d w_j / d u_a| sum_c |F_jc| |dL/dpsi(x_s)_c| / h
    where the clamp passes, times eta (1 - eta).  Returns (G0, G1), each
    (m,)."""
    n = st.n
    g_rgb = np.asarray(grad_rgb, np.float64).reshape(n, 3)
    g_d = np.asarray(grad_depth, np.float64).reshape(n)
    g_a = np.zeros(n) if grad_acc is None else np.asarray(grad_acc, np.float64).reshape(n)
    T, w, tau, col, ts = st.T, st.w, st.tau, st.col, st.ts
    Tn = T * np.exp(-tau)
    wc = w[:, :, None] * col
    S_c = np.sum(wc, axis=1, keepdims=True) - np.cumsum(wc, axis=1)
    wt = w * ts
    S_t = np.sum(wt, axis=1, keepdims=True) - np.cumsum(wt, axis=1)
    S_a = np.sum(w, axis=1, keepdims=True) - np.cumsum(w, axis=1)
    G_tau = (np.sum(np.abs(g_rgb)[:, None, :] * (Tn[:, :, None] * col + S_c), axis=2)
             + np.abs(g_d)[:, None] * (Tn * ts + S_t) + np.abs(g_a)[:, None] * (Tn + S_a))
    ri, si = st.ray_i, st.slot_i
    G_tau = G_tau[ri, si]
    G_eta_direct = np.zeros(ri.size)
    if hit_grads is not None:
        G_tau = G_tau + np.abs(hit_grads[2])
        G_eta_direct = np.abs(hit_grads[1])
    G0 = np.where(st.oT[:, 0] > 0.0, G_tau * st.dtau, 0.0)
    _, _, _, _, g_zC = _lf_backward_per_hit(st, grad_rgb, grad_depth, grad_acc, hit_grads)
    adw = np.abs(weight_derivatives(st.us))                       # (m, 8, 3)
    fz = np.einsum("mjc,mc->mj", np.abs(st.FC), np.abs(g_zC))      # (m, 8)
    inside = (st.us_raw >= 0.0) & (st.us_raw <= 1.0)
    G_xs = np.where(inside, np.einsum("mja,mj->ma", adw, fz), 0.0) / st.h
    g_ts = np.abs(w[ri, si] * g_d[ri])
    G_eta = g_ts * np.abs(st.t0 - st.t1) + np.sum(G_xs * np.abs(st.x1 - st.x2), axis=1) + G_eta_direct
    G1 = G_eta * st.eta * (1.0 - st.eta)
    return G0, G1


def density_input_jacobian(st):
    """Per hit, the gradient of the density decoder's input with respect to
    each of its two outputs (the backward of a unit output gradient; the
    hit's ReLU pattern).  Returns (J0, J1), each (m, 2 C_T + 6 [+ 3])."""
    rnd = bf16_round if st.bf16 else (lambda v: v)
    out = []
    for k in range(2):
        e = np.zeros_like(st.oT)
        e[:, k] = 1.0
        _, g_in = _mlp_backward_terms(st.lt, st.actsT, st.presT, e, rnd)
        out.append(g_in)
    return out[0], out[1]


def render_lf_backward_hit_magnitude(st, grad_rgb, grad_depth, grad_acc=None, hit_grads=None):
    """Scale of the per-hit contributions behind every entry of
    ``render_lf_backward`` (test infrastructure: the scale of per-entry
    rounding bounds of another evaluation of the same sums), as
    ``render.render_backward_hit_magnitude`` gives it for the single decoder.

    A Z_T row receives from each hit that has the vertex as corner j the two
    terms w1_j dL/dpsi(x1) and w2_j dL/dpsi(x2), a Z_C row ws_j dL/dpsi(x_s),
    a weight of either decoder dL/dz_h[i] a_h[k], a bias dL/dz_h[i].  Per
    entry the result is S + R: S = the sum over those terms of |term|
    (it bounds the entry, also when the terms cancel); R = the sum over the
    same terms of the largest |term| of the entry's group that the hit's
    same factor makes (a feature block of the row: w_j max_c |dL/dpsi[c]|; a
    layer's weights: max_i |dL/dz_h[i]| max_k |a_h[k]|; a layer's biases:
    max_i |dL/dz_h[i]|).  For Z_T, dL/dpsi(x1) and dL/dpsi(x2) are taken at
    their conditioning: |J0| G0 + |J1| G1 (``density_input_jacobian``,
    ``density_output_term_magnitudes``) in place of their absolute values,
    as the density decoder's two output gradients are often small
    differences of large terms (Eq. 3's backward of an opaque ray).  Returns
    (M_features (n_vertices, C_T + C_C), M_params)."""
    ct = st.dec[0]
    termsT, termsC, g_z1, g_z2, g_zC = _lf_backward_per_hit(st, grad_rgb, grad_depth, grad_acc,
                                                            hit_grads)
    mags = []
    for g_zr, a in termsT + termsC:
        gz, aa = np.abs(g_zr), np.abs(a)
        gmax = gz.max(axis=1, initial=0.0)
        rW = float(np.sum(gmax * aa.max(axis=1, initial=0.0)))
        rb = float(np.sum(gmax))
        mags += [(gz.T @ aa).ravel() + rW, np.sum(gz, axis=0) + rb]
    M_F = np.zeros((st.n_vertices, st.C))

    def part(wj, g):
        ga = np.abs(g)
        return wj[:, :, None] * (ga[:, None, :] + ga.max(axis=1, initial=0.0)[:, None, None])

    G0, G1 = density_output_term_magnitudes(st, grad_rgb, grad_depth, grad_acc, hit_grads)
    J0, J1 = density_input_jacobian(st)
    A = np.abs(J0) * G0[:, None] + np.abs(J1) * G1[:, None]
    mT = part(st.w1, A[:, :ct]) + part(st.w2, A[:, ct:2 * ct])
    np.add.at(M_F[:, :ct], st.corners.ravel(), mT.reshape(-1, ct))
    mC = part(st.ws, g_zC)
    np.add.at(M_F[:, ct:], st.corners.ravel(), mC.reshape(-1, g_zC.shape[1]))
    return M_F, np.concatenate(mags)
