"""torch.autograd.Function over svlf_render / svlf_render_backward.

The forward and the hand-written backward both run in libsvlf's HIP kernels;
the backward re-traces the rays and recomputes the decoder activations
instead of storing them, then scatters dL/dx into the per-vertex features
with FP32 atomics and reduces dL/dparams per block.
"""

from __future__ import annotations

import torch

from . import svlf


class _SVLFRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, features, params, ray_o, ray_d, scene, widths, K, tau_mode, precision, flags):
        sc = svlf.DeviceScene(scene.octree, features.detach(), scene.features_bf16)
        opts = svlf.make_opts(K, tau_mode, precision, flags)
        n = ray_o.shape[0]
        rgb, depth, acc = svlf.render([sc], [n], params.detach(), widths, opts, ray_o, ray_d)
        ctx.save_for_backward(features, params, ray_o, ray_d)
        ctx.scene, ctx.widths, ctx.opts = scene, widths, opts
        return rgb, depth, acc

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_acc):
        features, params, ray_o, ray_d = ctx.saved_tensors
        n = ray_o.shape[0]
        dev = ray_o.device
        g_rgb = torch.zeros((n, 3), device=dev) if g_rgb is None else g_rgb.contiguous().float()
        g_depth = torch.zeros((n,), device=dev) if g_depth is None else g_depth.contiguous().float()
        g_acc = None if g_acc is None else g_acc.contiguous().float()
        gF = torch.zeros_like(features)
        gp = torch.zeros_like(params)
        sc = svlf.DeviceScene(ctx.scene.octree, features.detach(), ctx.scene.features_bf16)
        svlf.render_backward([sc], [n], params.detach(), ctx.widths, ctx.opts, ray_o, ray_d,
                             g_rgb, g_depth, g_acc, [gF], gp)
        return gF, gp, None, None, None, None, None, None, None, None


def render(scene: "svlf.DeviceScene", params, widths, ray_o, ray_d, K, tau_mode="voxel",
           precision="fp32", features=None, viewdir=False):
    """Differentiable render: returns (rgb, depth, acc).  Gradients flow to
    ``features`` (default: scene.features) and ``params``.  In BF16 precision
    the scene's BF16 feature copy must match ``features``.  ``viewdir``
    appends the ray direction to the decoder input (widths[0] = C + 3)."""
    feats = scene.features if features is None else features
    flags = svlf.FLAG_VIEWDIR if viewdir else 0
    return _SVLFRender.apply(feats, params, ray_o, ray_d, scene, tuple(widths), K, tau_mode, precision,
                             flags)
