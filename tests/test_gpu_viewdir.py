"""GPU parity of the view-direction decoder input (SVLF_FLAG_VIEWDIR: the
decoder reads [psi(p; Z) | d], the input the paper proposes for
view-dependent appearance) against the FP64 oracle: decoder, render in both
precisions, backward and the fused train step."""

import numpy as np
import pytest

from oracle.render import (loss as oracle_loss, mlp_forward as oracle_mlp, render_backward,
                           render_backward_hit_magnitude, render_backward_weight_scale)
from synth.configs import tiny_workload, xavier_params
from tests.gpu_cases import (C_PARAM, Case, assert_grad_close, assert_outputs_close, loss_scales, psnr,
                             residual_terms)
from tests.helpers import random_rays
from tests.test_gpu_render import _gpu_backward

pytestmark = pytest.mark.gpu

VD_SHAPES = [(11, 32, 32, 4), (35, 64, 64, 64, 4)]


def _vd_cases(svlf):
    w = tiny_workload(51, 4, 8, (8, 32, 32, 4), 6, n_obj=3)
    yield "vd8", Case.from_workload(svlf, w, feat_scale=4.0, sigma_bias=0.8, viewdir=True)
    w = tiny_workload(52, 6, 32, (32, 64, 64, 64, 4), 8, n_obj=4)
    yield "vd32", Case.from_workload(svlf, w, feat_scale=5.0, sigma_bias=0.5, viewdir=True)


@pytest.mark.parametrize("widths", VD_SHAPES, ids=lambda w: "x".join(map(str, w)))
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_decoder_viewdir(gpu_lib, widths, precision):
    import torch
    rng = np.random.default_rng(widths[0])
    p = xavier_params(rng, widths)
    p[-4:] = rng.normal(size=4).astype(np.float32)
    X = rng.normal(0, 0.5, (1031, widths[0])).astype(np.float32)
    opts = gpu_lib.make_opts(4, precision=precision, flags=gpu_lib.FLAG_VIEWDIR)
    out = gpu_lib.mlp_forward(torch.from_numpy(p).cuda(), widths, opts,
                              torch.from_numpy(X).cuda()).cpu().numpy()
    ref, _, _ = oracle_mlp(p.astype(np.float64), widths, X.astype(np.float64), bf16=precision == "bf16")
    if precision == "fp32":
        assert_outputs_close(out, ref, name="viewdir decoder fp32")
    else:
        assert np.abs(out - ref).max() <= 2 ** -6 * np.abs(ref).max()


def test_render_viewdir_fp32_and_bf16(gpu_lib):
    for name, case in _vd_cases(gpu_lib):
        rng = np.random.default_rng(len(name) + 3)
        o, d = random_rays(rng, 2500, inside_frac=0.2)
        rgb, dep, acc = case.gpu_render(o, d)
        er, ed, ea, st = case.oracle(o, d)
        assert st.ray_i.size > 100, name
        assert_outputs_close(rgb, er, 1.0, f"{name} rgb")
        assert_outputs_close(acc, ea, 1.0, f"{name} acc")
        assert_outputs_close(dep, ed, max(1.0, np.abs(ed).max()), f"{name} depth")
        rgb16, _, _ = case.gpu_render(o, d, "bf16")
        br, _, _, _ = case.oracle(o, d, bf16=True)
        assert np.abs(rgb16 - br).max() <= 2 ** -6 * max(np.abs(br).max(), 1e-3) + 1e-4, name
        assert psnr(rgb16, er) > 35.0, name
        # the same rays reversed in direction through the same points see
        # other colours (the decoder input differs only in d)
        rgb_r, _, _ = case.gpu_render(o + 4.0 * d, -d)
        er_r, _, _, _ = case.oracle(o + 4.0 * d, -d)
        assert_outputs_close(rgb_r, er_r, 1.0, f"{name} reversed rgb")


def test_backward_and_train_step_viewdir_fp32(gpu_lib):
    import torch
    for name, case in _vd_cases(gpu_lib):
        rng = np.random.default_rng(61)
        o, d = random_rays(rng, 2000, inside_frac=0.1)
        keep = case.smooth_rays(o, d)
        o, d = o[keep], d[keep]
        n = o.shape[0]
        g_rgb = rng.normal(size=(n, 3)).astype(np.float32)
        g_dep = rng.normal(size=n).astype(np.float32)
        gF, gp = _gpu_backward(case, o, d, g_rgb, g_dep, None)
        _, _, _, st = case.oracle(o, d)
        eF, ep = render_backward(st, g_rgb, g_dep)
        mF, mp = render_backward_hit_magnitude(st, g_rgb, g_dep)
        mW = render_backward_weight_scale(st, g_rgb, g_dep)
        assert gF.shape == case.F.shape and np.abs(eF).max() > 0
        assert_grad_close(gF, eF, f"{name} grad_features", mag=mF, wmag=mW)
        assert_grad_close(gp, ep, f"{name} grad_params", rel_nw=1e-4, mag=mp, c=C_PARAM)
        # fused train step
        t_rgb = rng.uniform(0, 1, (n, 3)).astype(np.float32)
        t_dep = rng.uniform(0, 5, n).astype(np.float32)
        to, td = case.rays(o, d)
        gF2 = torch.zeros(case.scene.features.shape, dtype=torch.float32, device="cuda")
        gp2 = torch.zeros(case.params.shape, dtype=torch.float32, device="cuda")
        loss_t = torch.zeros(1, dtype=torch.float32, device="cuda")
        case.svlf.train_step([case.scene], [n], case.params, case.widths, case.opts(), to, td,
                             torch.from_numpy(t_rgb).cuda(), torch.from_numpy(t_dep).cuda(),
                             0.1, 1.0 / n, [gF2], gp2, loss_out=loss_t)
        torch.cuda.synchronize()
        er, ed, _, st = case.oracle(o, d)
        L, lg_rgb, lg_dep = oracle_loss(er, ed, t_rgb, t_dep, 0.1)
        eF2, ep2 = render_backward(st, lg_rgb, lg_dep)
        mF2, mp2, mW2 = loss_scales(render_backward_hit_magnitude, render_backward_weight_scale, st, lg_rgb,
                                    residual_terms(lg_rgb, er, t_rgb), lg_dep)
        assert abs(float(loss_t.item()) - L) <= 1e-5 * abs(L), name
        assert_grad_close(gF2.cpu().numpy(), eF2, f"{name} train grad_features", mag=mF2, wmag=mW2)
        assert_grad_close(gp2.cpu().numpy(), ep2, f"{name} train grad_params", rel_nw=1e-4, mag=mp2, c=C_PARAM)


def test_viewdir_bf16_backward_close(gpu_lib):
    for name, case in _vd_cases(gpu_lib):
        rng = np.random.default_rng(71)
        o, d = random_rays(rng, 2000)
        n = o.shape[0]
        g_rgb = rng.normal(size=(n, 3)).astype(np.float32)
        g_dep = rng.normal(size=n).astype(np.float32)
        gF, gp = _gpu_backward(case, o, d, g_rgb, g_dep, None, "bf16")
        _, _, _, st = case.oracle(o, d, bf16=True)
        eF, ep = render_backward(st, g_rgb, g_dep)
        cos = lambda a, b: float(np.dot(a.ravel(), b.ravel()) / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-30))
        assert cos(gF, eF) > 0.999 and cos(gp, ep) > 0.999, name
