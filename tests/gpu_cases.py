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
