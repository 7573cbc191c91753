"""Shared set-up for the GPU parity tests: one workload on the device and
the same inputs in the oracle, plus the stated tolerances.

Tolerances (FP32 path, derived from the arithmetic):
* rgb / depth / acc: per channel max|err| <= 1e-5 * max|ref| + 1e-7 S and
  elementwise |err| <= 1e-5 |ref| + 1e-6 S, S = 1 (rgb, acc) or max depth.
  FP32 MLP dot products (length <= 64) and FP32 compositing round at ~1e-7
  relative; the mixed bound covers cancellation near sigma ~ 0.
* gradients (FP32 atomics, order-dependent): features max|err| <= 1e-5 max|g|
  and elementwise |err| <= 1e-4 |g| + 1e-5 max|g| (an entry sums many
  contributions whose FP32 rounding is relative to their own magnitudes, so
  a cancelling entry gets an absolute floor); MLP parameters max|err| <= 1e-4
  max|g| (their sums run over all hits of the batch).  Gradient parity uses
  rays with no decoder pre-activation within 1e-4 of a ReLU kink (there FP32
  and FP64 may legitimately take different one-sided derivatives).
BF16 path: compared with the oracle's BF16-rounding mode; hidden activations
may round differently where FP32 and FP64 accumulations straddle a bfloat16
rounding boundary (one bfloat16 ulp = 2^-8 relative), so outputs are checked
at max|err| <= 2^-6 max|ref| + 1e-4 S, and the error against the FP64 oracle
is reported as PSNR.
"""

import numpy as np

from oracle.octree import Octree
from oracle.render import render as oracle_render
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


def assert_grad_close(got, exp, name="", rel_nw=1e-5, rel_el=1e-4, abs_el=1e-5):
    got = np.asarray(got, np.float64)
    exp = np.asarray(exp, np.float64)
    m = np.abs(exp).max() if exp.size else 0.0
    err = np.abs(got - exp)
    assert np.all(np.isfinite(got)), f"{name}: non-finite gradient"
    nbad = int(np.sum(err > rel_nw * m))
    assert err.max(initial=0.0) <= rel_nw * m + 1e-30, \
        f"{name}: normwise {err.max()} vs {rel_nw * m} ({nbad} of {err.size} entries above)"
    if rel_el is not None:
        lim = rel_el * np.abs(exp) + abs_el * m
        bad = err > lim
        assert not bad.any(), \
            f"{name}: {bad.sum()} elements outside elementwise bound (worst ratio {np.max(err / lim):.3g})"


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
