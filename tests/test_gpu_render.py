"""GPU parity of the decoder, svlf_render, svlf_render_backward and
svlf_train_step against the FP64 oracle (SVLF sections 4.1-4.3, Eq. 3)."""

import numpy as np
import pytest

from oracle.render import (bf16_round, loss as oracle_loss, mlp_forward as oracle_mlp, render_backward,
                           render_backward_hit_magnitude,
                           render_backward_weight_scale)
from synth.configs import get_workload, scene_from_leaves, tiny_workload, xavier_params
from tests.gpu_cases import (C_PARAM, C_W_LF, EPS32, Case, assert_bf16_render_close, assert_grad_close,
                             assert_outputs_close, bf16_decoder_bound, lf_surface_point_error, psnr,
                             loss_scales, residual_terms)
from tests.helpers import random_rays

pytestmark = pytest.mark.gpu

SHAPES = [(8, 32, 32, 4), (16, 64, 64, 64, 4), (32, 64, 64, 64, 4)]


@pytest.mark.parametrize("widths", SHAPES, ids=lambda w: "x".join(map(str, w)))
@pytest.mark.parametrize("n", [1, 31, 300, 4099])
def test_decoder_fp32(gpu_lib, widths, n):
    import torch
    rng = np.random.default_rng(n)
    p = xavier_params(rng, widths)
    p[-4:] = rng.normal(size=4).astype(np.float32)
    X = rng.normal(0, 0.5, (n, widths[0])).astype(np.float32)
    out = gpu_lib.mlp_forward(torch.from_numpy(p).cuda(), widths, gpu_lib.make_opts(4),
                              torch.from_numpy(X).cuda()).cpu().numpy()
    ref, _, _ = oracle_mlp(p.astype(np.float64), widths, X.astype(np.float64))
    assert_outputs_close(out, ref, name="decoder fp32")


@pytest.mark.parametrize("widths", SHAPES, ids=lambda w: "x".join(map(str, w)))
@pytest.mark.parametrize("n", [31, 2000])
def test_decoder_bf16(gpu_lib, widths, n):
    """Every output within its own bound: the FP32-accumulation error carried
    through the layers, with a hidden activation allowed the neighbouring
    bfloat16 value only where its pre-activation lies that close to a
    rounding boundary."""
    import torch
    rng = np.random.default_rng(5 + n)
    p = xavier_params(rng, widths)
    p[-4:] = rng.normal(size=4).astype(np.float32)
    X = rng.normal(0, 0.5, (n, widths[0])).astype(np.float32)
    out = gpu_lib.mlp_forward(torch.from_numpy(p).cuda(), widths, gpu_lib.make_opts(4, precision="bf16"),
                              torch.from_numpy(X).cuda()).cpu().numpy()
    ref, bound = bf16_decoder_bound(p.astype(np.float64), widths, X.astype(np.float64))
    ref2, _, _ = oracle_mlp(p.astype(np.float64), widths, X.astype(np.float64), bf16=True)
    np.testing.assert_array_equal(ref, ref2)
    err = np.abs(out - ref)
    bad = err > bound
    print(f"decoder bf16 {widths} n={n}: max err/bound {np.max(err / np.maximum(bound, 1e-300)):.3g}")
    assert not bad.any(), f"{bad.sum()} of {err.size} outputs outside their bound, worst err {err[bad].max()}"


def _scene_cases(svlf):
    yield "shell_d4", Case.from_workload(svlf, get_workload("shell_d4"), feat_scale=4.0, sigma_bias=0.8)
    w = tiny_workload(7, 5, 16, (16, 64, 64, 64, 4), 8, n_obj=3)
    yield "tiny16", Case.from_workload(svlf, w, feat_scale=5.0, sigma_bias=1.0)
    w = tiny_workload(8, 6, 32, (32, 64, 64, 64, 4), 8, n_obj=4)
    yield "tiny32", Case.from_workload(svlf, w, feat_scale=5.0, sigma_bias=0.5)
    w = tiny_workload(9, 4, 8, (8, 32, 32, 4), 3, kind="shell")
    yield "shellK3", Case.from_workload(svlf, w, feat_scale=5.0, sigma_bias=2.0, tau_mode="world")


def test_render_fp32_against_oracle(gpu_lib):
    for name, case in _scene_cases(gpu_lib):
        rng = np.random.default_rng(len(name))
        o, d = random_rays(rng, 3001, inside_frac=0.2)
        o[:3] = [[0.1, 0.2, 0.3], [-2, 0.1, 0.1], [np.inf, 0, 0]]
        d[:3] = [[0, 0, 0], [1, np.nan, 0], [1, 0, 0]]
        rgb, dep, acc = case.gpu_render(o, d)
        er, ed, ea, st = case.oracle(o, d)
        assert np.count_nonzero(st.ray_i) > 100, name
        assert_outputs_close(rgb, er, 1.0, f"{name} rgb")
        assert_outputs_close(acc, ea, 1.0, f"{name} acc")
        assert_outputs_close(dep, ed, max(1.0, np.abs(ed).max()), f"{name} depth")


def test_render_modes_direct(gpu_lib):
    w = tiny_workload(3, 4, 8, (8, 32, 32, 4), 6)
    case = Case.from_workload(gpu_lib, w, feat_scale=3.0, sigma_bias=0.3, tau_mode="direct")
    o, d = random_rays(np.random.default_rng(0), 1000)
    rgb, dep, acc = case.gpu_render(o, d)
    er, ed, ea, _ = case.oracle(o, d)
    assert_outputs_close(rgb, er, 1.0, "direct rgb")
    assert_outputs_close(dep, ed, max(1.0, np.abs(ed).max()), "direct depth")


def test_render_bf16_against_bf16_oracle(gpu_lib):
    for name, case in _scene_cases(gpu_lib):
        o, d = random_rays(np.random.default_rng(1), 2000)
        rgb, dep, acc = case.gpu_render(o, d, "bf16")
        br, bd, ba, bst = case.oracle(o, d, bf16=True)
        er, ed, ea, _ = case.oracle(o, d)
        assert_bf16_render_close(rgb, dep, acc, (br, bd, ba), bst, case.F, name)
        assert psnr(rgb, er) > 35.0, (name, psnr(rgb, er))


def test_workload1_full_view_sampled(gpu_lib):
    """Full 800x800 view rendered in one call (the launch a bench would
    time); 4096 seeded rays compared with the oracle."""
    case = Case.from_workload(gpu_lib, get_workload("ellipsoids_d7"), feat_scale=3.0, sigma_bias=0.5)
    o, d = get_workload("ellipsoids_d7").view_rays()
    rgb, dep, acc = case.gpu_render(o, d)
    idx = np.random.default_rng(7).choice(o.shape[0], 4096, replace=False)
    er, ed, ea, st = case.oracle(o[idx], d[idx])
    assert_outputs_close(rgb[idx], er, 1.0, "ellipsoids_d7 rgb")
    assert_outputs_close(dep[idx], ed, max(1.0, np.abs(ed).max()), "ellipsoids_d7 depth")
    assert_outputs_close(acc[idx], ea, 1.0, "ellipsoids_d7 acc")
    assert np.all(acc >= 0) and np.all(acc <= 1 + 1e-6) and np.all(rgb <= acc[:, None] + 1e-6)


def test_empty_scene(gpu_lib):
    import torch
    oc_ijk = np.zeros((0, 3), np.int32)
    case = Case(gpu_lib, oc_ijk, 3, np.zeros((0, 8), np.float32),
                xavier_params(np.random.default_rng(0), (8, 32, 32, 4)), (8, 32, 32, 4), 4)
    o, d = random_rays(np.random.default_rng(0), 500)
    rgb, dep, acc = case.gpu_render(o, d)
    assert np.all(rgb == 0) and np.all(dep == 0) and np.all(acc == 0)


def _gpu_backward(case, o, d, g_rgb, g_dep, g_acc, precision="fp32"):
    import torch
    to, td = case.rays(o, d)
    gF = torch.zeros(case.scene.features.shape, dtype=torch.float32, device="cuda")
    gp = torch.zeros(case.params.shape, dtype=torch.float32, device="cuda")
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
    case.svlf.render_backward([case.scene], [o.shape[0]], case.params, case.widths,
                              case.opts(precision), to, td, t(g_rgb), t(g_dep),
                              None if g_acc is None else t(g_acc), [gF], gp)
    torch.cuda.synchronize()
    return gF.cpu().numpy(), gp.cpu().numpy()


def test_backward_fp32_against_oracle(gpu_lib):
    for name, case in _scene_cases(gpu_lib):
        rng = np.random.default_rng(11)
        o, d = random_rays(rng, 2500, inside_frac=0.2)
        keep = case.smooth_rays(o, d)
        o, d = o[keep], d[keep]
        n = o.shape[0]
        g_rgb = rng.normal(size=(n, 3)).astype(np.float32)
        g_dep = rng.normal(size=n).astype(np.float32)
        g_acc = rng.normal(size=n).astype(np.float32)
        gF, gp = _gpu_backward(case, o, d, g_rgb, g_dep, g_acc)
        _, _, _, st = case.oracle(o, d)
        eF, ep = render_backward(st, g_rgb, g_dep, g_acc)
        mF, mp = render_backward_hit_magnitude(st, g_rgb, g_dep, g_acc)
        mW = render_backward_weight_scale(st, g_rgb, g_dep, g_acc)
        assert np.abs(eF).max() > 0 and np.abs(ep).max() > 0, name
        assert_grad_close(gF, eF, f"{name} grad_features", mag=mF, wmag=mW)
        assert_grad_close(gp, ep, f"{name} grad_params", rel_nw=1e-4, mag=mp, c=C_PARAM)
        # conservation: trilinear weights sum to one per hit
        assert abs(gF.sum() - eF.sum()) <= 1e-4 * np.abs(eF).sum()


def test_backward_accumulates(gpu_lib):
    import torch
    case = next(iter(_scene_cases(gpu_lib)))[1]
    o, d = random_rays(np.random.default_rng(3), 700)
    g = np.random.default_rng(4)
    g_rgb = g.normal(size=(700, 3)).astype(np.float32)
    g_dep = g.normal(size=700).astype(np.float32)
    gF1, gp1 = _gpu_backward(case, o, d, g_rgb, g_dep, None)
    to, td = case.rays(o, d)
    gF = torch.from_numpy(gF1).cuda()
    gp = torch.from_numpy(gp1).cuda()
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
    case.svlf.render_backward([case.scene], [700], case.params, case.widths, case.opts(),
                              to, td, t(g_rgb), t(g_dep), None, [gF], gp)
    torch.cuda.synchronize()
    np.testing.assert_allclose(gF.cpu().numpy(), 2 * gF1, rtol=1e-5, atol=1e-7 * np.abs(gF1).max())
    np.testing.assert_allclose(gp.cpu().numpy(), 2 * gp1, rtol=1e-5, atol=1e-7 * np.abs(gp1).max())


def test_train_step_fp32_against_oracle(gpu_lib):
    import torch
    for name, case in list(_scene_cases(gpu_lib))[:3]:
        rng = np.random.default_rng(21)
        o, d = random_rays(rng, 2000, inside_frac=0.0)
        keep = case.smooth_rays(o, d)
        o, d = o[keep], d[keep]
        n = o.shape[0]
        t_rgb = rng.uniform(0, 1, (n, 3)).astype(np.float32)
        t_dep = rng.uniform(0, 5, n).astype(np.float32)
        to, td = case.rays(o, d)
        gF = torch.zeros(case.scene.features.shape, dtype=torch.float32, device="cuda")
        gp = torch.zeros(case.params.shape, dtype=torch.float32, device="cuda")
        loss_t = torch.zeros(1, dtype=torch.float32, device="cuda")
        out_rgb = torch.empty((n, 3), dtype=torch.float32, device="cuda")
        out_dep = torch.empty((n,), dtype=torch.float32, device="cuda")
        case.svlf.train_step([case.scene], [n], case.params, case.widths, case.opts(), to, td,
                             torch.from_numpy(t_rgb).cuda(), torch.from_numpy(t_dep).cuda(),
                             0.1, 1.0 / n, [gF], gp, out_rgb, out_dep, loss_t)
        torch.cuda.synchronize()
        er, ed, ea, st = case.oracle(o, d)
        L, g_rgb, g_dep = oracle_loss(er, ed, t_rgb, t_dep, 0.1)
        eF, ep = render_backward(st, g_rgb, g_dep)
        mF, mp, mW = loss_scales(render_backward_hit_magnitude, render_backward_weight_scale, st, g_rgb,
                                 residual_terms(g_rgb, er, t_rgb), g_dep)
        assert abs(float(loss_t.item()) - L) <= 1e-5 * abs(L), name
        assert_outputs_close(out_rgb.cpu().numpy(), er, 1.0, f"{name} rgb")
        assert_grad_close(gF.cpu().numpy(), eF, f"{name} grad_features", mag=mF, wmag=mW)
        assert_grad_close(gp.cpu().numpy(), ep, f"{name} grad_params", rel_nw=1e-4, mag=mp, c=C_PARAM)


def test_backward_bf16_against_bf16_oracle(gpu_lib):
    for name, case in list(_scene_cases(gpu_lib))[:3]:
        rng = np.random.default_rng(31)
        o, d = random_rays(rng, 2000)
        n = o.shape[0]
        g_rgb = rng.normal(size=(n, 3)).astype(np.float32)
        g_dep = rng.normal(size=n).astype(np.float32)
        gF, gp = _gpu_backward(case, o, d, g_rgb, g_dep, None, "bf16")
        _, _, _, st = case.oracle(o, d, bf16=True)
        eF, ep = render_backward(st, g_rgb, g_dep)
        assert np.abs(eF).max() > 0 and np.abs(gF).max() > 0, name
        cos = lambda a, b: float(np.dot(a.ravel(), b.ravel()) / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-30))
        assert cos(gF, eF) > 0.999, (name, cos(gF, eF))
        assert cos(gp, ep) > 0.999, (name, cos(gp, ep))
        assert np.linalg.norm(gF - eF) <= 0.05 * np.linalg.norm(eF)


def test_multi_scene_render_and_backward(gpu_lib):
    """Three scenes with different depths in one launch; each compared with
    its own oracle run."""
    import torch
    cases, rays, counts = [], [], []
    for i, (seed, depth) in enumerate([(40, 3), (41, 5), (42, 6)]):
        w = tiny_workload(seed, depth, 16, (16, 64, 64, 64, 4), 8, n_obj=2)
        sc = w.scene()
        F = w.features() * 4.0
        p = get_workload("ellipsoids_d7").params().copy()
        p[-1] = 0.7
        cases.append(Case(gpu_lib, sc.leaf_ijk, sc.depth, F, p, w.widths, 8))
        o_, d_ = random_rays(np.random.default_rng(seed), [1000, 257, 2049][i])
        keep = cases[-1].smooth_rays(o_, d_)
        rays.append((o_[keep], d_[keep]))
        counts.append(int(keep.size))
    o = np.concatenate([r[0] for r in rays])
    d = np.concatenate([r[1] for r in rays])
    to, td = cases[0].rays(o, d)
    params = cases[0].params
    rgb, dep, acc = gpu_lib.render([c.scene for c in cases], counts, params, cases[0].widths,
                                   cases[0].opts(), to, td)
    gFs = [torch.zeros(c.scene.features.shape, dtype=torch.float32, device="cuda") for c in cases]
    gp = torch.zeros(params.shape, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(0)
    g_rgb = rng.normal(size=(o.shape[0], 3)).astype(np.float32)
    g_dep = rng.normal(size=o.shape[0]).astype(np.float32)
    t = lambda x: torch.from_numpy(x).cuda()
    gpu_lib.render_backward([c.scene for c in cases], counts, params, cases[0].widths,
                            cases[0].opts(), to, td, t(g_rgb), t(g_dep), None, gFs, gp)
    torch.cuda.synchronize()
    rgb = rgb.cpu().numpy()
    dep = dep.cpu().numpy()
    ep_total = mp_total = 0
    start = 0
    for c, n, gF in zip(cases, counts, gFs):
        sl = slice(start, start + n)
        er, ed, ea, st = c.oracle(o[sl], d[sl])
        assert_outputs_close(rgb[sl], er, 1.0, "multi rgb")
        assert_outputs_close(dep[sl], ed, max(1.0, np.abs(ed).max()), "multi depth")
        eF, ep = render_backward(st, g_rgb[sl], g_dep[sl])
        mF, mp = render_backward_hit_magnitude(st, g_rgb[sl], g_dep[sl])
        mW = render_backward_weight_scale(st, g_rgb[sl], g_dep[sl])
        assert_grad_close(gF.cpu().numpy(), eF, "multi grad_features", mag=mF, wmag=mW)
        ep_total = ep_total + ep
        mp_total = mp_total + mp
        start += n
    assert_grad_close(gp.cpu().numpy(), ep_total, "multi grad_params", rel_nw=1e-4, mag=mp_total, c=C_PARAM)


def test_deterministic_feature_gradient(gpu_lib):
    """SVLF_FLAG_DETERMINISTIC: bit-identical feature gradients over repeated
    calls, equal to the atomic path within the FP32 tolerance, and to the
    oracle on kink-free rays; decoder gradients bit-identical over repeated
    calls too, and equal to the atomic path's and the oracle's within the
    decoder-gradient bound."""
    import torch
    for name, case in list(_scene_cases(gpu_lib))[:3]:
        rng = np.random.default_rng(41)
        o, d = random_rays(rng, 3000, inside_frac=0.2)
        keep = case.smooth_rays(o, d)
        o, d = o[keep], d[keep]
        n = o.shape[0]
        g_rgb = rng.normal(size=(n, 3)).astype(np.float32)
        g_dep = rng.normal(size=n).astype(np.float32)
        to, td = case.rays(o, d)
        t = lambda x: torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()

        def run(flags):
            gF = torch.zeros(case.scene.features.shape, dtype=torch.float32, device="cuda")
            gp = torch.zeros(case.params.shape, dtype=torch.float32, device="cuda")
            opts = gpu_lib.make_opts(case.K, case.tau_mode, "fp32", flags)
            gpu_lib.render_backward([case.scene], [n], case.params, case.widths, opts, to, td,
                                    t(g_rgb), t(g_dep), None, [gF], gp)
            torch.cuda.synchronize()
            return gF.cpu().numpy(), gp.cpu().numpy()

        gF1, gp1 = run(gpu_lib.FLAG_DETERMINISTIC)
        gF2, gp2 = run(gpu_lib.FLAG_DETERMINISTIC)
        assert np.array_equal(gF1.view(np.int32), gF2.view(np.int32)), name
        assert np.array_equal(gp1.view(np.int32), gp2.view(np.int32)), name
        gFa, gpa = run(0)
        _, _, _, st = case.oracle(o, d)
        eF, ep = render_backward(st, g_rgb, g_dep)
        mF, mp = render_backward_hit_magnitude(st, g_rgb, g_dep)
        mW = render_backward_weight_scale(st, g_rgb, g_dep)
        assert_grad_close(gF1, eF, f"{name} deterministic grad_features", mag=mF, wmag=mW)
        assert_grad_close(gF1, gFa, f"{name} deterministic vs atomic", mag=mF, wmag=mW)
        # without the flag the last work items go to whichever block is free,
        # so the per-block decoder-gradient partials are grouped differently
        assert_grad_close(gp1, ep, f"{name} deterministic grad_params", rel_nw=1e-4, mag=mp, c=C_PARAM)
        assert_grad_close(gpa, gp1, f"{name} atomic vs deterministic grad_params", rel_nw=1e-4, mag=mp, c=C_PARAM)


def test_deterministic_feature_gradient_hit_dense_coarse_scene(gpu_lib):
    """SVLF_FLAG_DETERMINISTIC where leaf buckets are large: every cell of a
    depth-2 grid is a leaf (64 leaves) and 2^16 rays put thousands of hits
    in each bucket.  Bit-identical repeats, the oracle on kink-free rays,
    and the atomic path, all within the per-entry bound."""
    import torch
    cells = [(i, j, k) for i in range(4) for j in range(4) for k in range(4)]
    w = scene_from_leaves(11, 2, 8, (8, 32, 32, 4), 8, cells)
    case = Case.from_workload(gpu_lib, w, feat_scale=2.0, sigma_bias=0.05)
    rng = np.random.default_rng(43)
    o, d = random_rays(rng, 1 << 16, inside_frac=0.3)
    keep = case.smooth_rays(o, d)
    o, d = o[keep], d[keep]
    n = o.shape[0]
    assert n > 30000
    _, _, _, st = case.oracle(o, d)
    # a leaf's lowest corner identifies it
    _, per_leaf = np.unique(st.corners[:, 0], return_counts=True)
    print(f"hit-dense scene: {n} rays, {per_leaf.sum()} hits, bucket sizes {per_leaf.min()}..{per_leaf.max()}")
    assert per_leaf.size == 64 and per_leaf.min() > 1000
    g_rgb = rng.normal(size=(n, 3)).astype(np.float32)
    g_dep = rng.normal(size=n).astype(np.float32)
    to, td = case.rays(o, d)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()

    def run(flags):
        gF = torch.zeros(case.scene.features.shape, dtype=torch.float32, device="cuda")
        gp = torch.zeros(case.params.shape, dtype=torch.float32, device="cuda")
        opts = gpu_lib.make_opts(case.K, case.tau_mode, "fp32", flags)
        gpu_lib.render_backward([case.scene], [n], case.params, case.widths, opts, to, td,
                                t(g_rgb), t(g_dep), None, [gF], gp)
        torch.cuda.synchronize()
        return gF.cpu().numpy(), gp.cpu().numpy()

    gF1, gp1 = run(gpu_lib.FLAG_DETERMINISTIC)
    gF2, gp2 = run(gpu_lib.FLAG_DETERMINISTIC)
    assert np.array_equal(gF1.view(np.int32), gF2.view(np.int32))
    assert np.array_equal(gp1.view(np.int32), gp2.view(np.int32))
    gFa, gpa = run(0)
    eF, ep = render_backward(st, g_rgb, g_dep)
    mF, mp = render_backward_hit_magnitude(st, g_rgb, g_dep)
    mW = render_backward_weight_scale(st, g_rgb, g_dep)
    assert_grad_close(gF1, eF, "hit-dense deterministic grad_features", mag=mF, wmag=mW)
    assert_grad_close(gF1, gFa, "hit-dense deterministic vs atomic", mag=mF, wmag=mW)
    assert_grad_close(gp1, ep, "hit-dense deterministic grad_params", rel_nw=1e-4, mag=mp, c=C_PARAM)
    assert_grad_close(gpa, gp1, "hit-dense atomic vs deterministic grad_params", rel_nw=1e-4, mag=mp, c=C_PARAM)


def test_max_K_solid_scene(gpu_lib):
    """K = 16 (the largest hit cap) on a solid scene where many rays have 16
    hits: windows hold few rays each; forward and backward against the
    oracle, and the light-field path on the same scene."""
    from tests.gpu_cases import LfCase
    from oracle.lightfield import render_lf_backward, render_lf_backward_hit_magnitude, render_lf_backward_weight_scale
    w = tiny_workload(17, 5, 16, (16, 64, 64, 64, 4), 16, n_obj=3)
    case = Case.from_workload(gpu_lib, w, feat_scale=3.0, sigma_bias=0.3)
    rng = np.random.default_rng(5)
    o, d = random_rays(rng, 2500, inside_frac=0.3)
    rgb, dep, acc = case.gpu_render(o, d)
    er, ed, ea, st = case.oracle(o, d)
    counts = np.bincount(st.ray_i, minlength=o.shape[0])
    assert counts.max() == 16 and np.mean(counts == 16) > 0.05
    assert_outputs_close(rgb, er, 1.0, "K16 rgb")
    assert_outputs_close(dep, ed, max(1.0, np.abs(ed).max()), "K16 depth")
    keep = case.smooth_rays(o, d)
    g_rgb = rng.normal(size=(keep.size, 3)).astype(np.float32)
    g_dep = rng.normal(size=keep.size).astype(np.float32)
    gF, gp = _gpu_backward(case, o[keep], d[keep], g_rgb, g_dep, None)
    _, _, _, st2 = case.oracle(o[keep], d[keep])
    eF, ep = render_backward(st2, g_rgb, g_dep)
    mF, mp = render_backward_hit_magnitude(st2, g_rgb, g_dep)
    mW = render_backward_weight_scale(st2, g_rgb, g_dep)
    assert_grad_close(gF, eF, "K16 grad_features", mag=mF, wmag=mW)
    assert_grad_close(gp, ep, "K16 grad_params", rel_nw=1e-4, mag=mp, c=C_PARAM)
    lf = LfCase(gpu_lib, w.scene().leaf_ijk, 5,
                np.random.default_rng(1).normal(0, 0.5, (w.scene().n_vertices, 96)).astype(np.float32),
                LfCase.random(gpu_lib, 17, 5, K=16).p, 16)
    lrgb, ldep, lacc = lf.gpu_render(o, d)
    lr, ld, la, lst = lf.oracle(o, d)
    assert_outputs_close(lrgb, lr, 1.0, "K16 lf rgb")
    assert_outputs_close(ldep, ld, max(1.0, np.abs(ld).max()), "K16 lf depth")
    keep = lf.smooth_rays(o, d)
    lg_rgb = rng.normal(size=(keep.size, 3)).astype(np.float32)
    lg_dep = rng.normal(size=keep.size).astype(np.float32)
    lgF, lgp = lf.gpu_backward(o[keep], d[keep], lg_rgb, lg_dep)
    _, _, _, lst2 = lf.oracle(o[keep], d[keep])
    leF, lep = render_lf_backward(lst2, lg_rgb, lg_dep)
    lmF, lmp = render_lf_backward_hit_magnitude(lst2, lg_rgb, lg_dep)
    lmW = render_lf_backward_weight_scale(lst2, lg_rgb, lg_dep)
    assert_grad_close(lgF, leF, "K16 lf grad_features", mag=lmF, wmag=lmW, c_w=C_W_LF)
    assert_grad_close(lgp, lep, "K16 lf grad_params", rel_nw=1e-4, mag=lmp, c=C_PARAM)


def test_depth_10_scene(gpu_lib):
    """The deepest supported octree (depth 10: 1024^3 leaf grid, 10-bit cell
    coordinates, plane spacing 2^-9): clusters of leaves, including cells on
    the grid's faces and corners, and rays aimed at them.  Hit lists
    bit-exact, FP32 render and gradients against the oracle."""
    from oracle.octree import Octree
    from oracle.trace import trace_hits as oracle_trace
    rng = np.random.default_rng(1010)
    depth = 10
    n = 1 << depth
    centres = rng.integers(0, n, (24, 3))
    centres[:4] = [[0, 0, 0], [n - 1, n - 1, n - 1], [0, n - 1, n // 2], [n // 2, 0, n - 1]]
    blk = np.stack(np.meshgrid(*[np.arange(-2, 3)] * 3, indexing="ij"), -1).reshape(-1, 3)
    cells = np.concatenate([np.clip(c + blk[rng.random(blk.shape[0]) < 0.5], 0, n - 1)
                            for c in centres])
    cells = np.unique(cells, axis=0).astype(np.int32)
    nv = Octree(cells, depth).n_vertices
    widths = (16, 64, 64, 64, 4)
    F = rng.normal(0.0, 1.0, (nv, 16)).astype(np.float32)
    p = xavier_params(np.random.default_rng(7), widths)
    p[-1] = 0.5
    case = Case(gpu_lib, cells, depth, F, p, widths, 8)
    # rays from a sphere of radius 3 towards the clusters (jittered by a few
    # cells), plus random rays
    m = 3000
    tgt = -1.0 + (centres[rng.integers(0, len(centres), m)] + 0.5 + rng.uniform(-3, 3, (m, 3))) * (2.0 / n)
    v = rng.standard_normal((m, 3))
    o = 3.0 * v / np.linalg.norm(v, axis=1, keepdims=True)
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o2, d2 = random_rays(rng, 1000, inside_frac=0.3)
    o = np.concatenate([o, o2]).astype(np.float32)
    d = np.concatenate([d, d2]).astype(np.float32)
    # hit lists
    import torch
    to, td = case.rays(o, d)
    leaf, tin, tout, cnt = gpu_lib.trace_hits(case.scene.octree, to, td, 8)
    torch.cuda.synchronize()
    el, ei, eo, ec = oracle_trace(case.oc, o, d, 8)
    np.testing.assert_array_equal(cnt.cpu().numpy(), ec)
    np.testing.assert_array_equal(leaf.cpu().numpy(), el)
    np.testing.assert_array_equal(tin.cpu().numpy().view(np.int32), ei.view(np.int32))
    np.testing.assert_array_equal(tout.cpu().numpy().view(np.int32), eo.view(np.int32))
    assert ec.sum() > 3000 and (ec > 0).mean() > 0.3
    # render and gradients
    rgb, dep, acc = case.gpu_render(o, d)
    er, ed, ea, _ = case.oracle(o, d)
    assert_outputs_close(rgb, er, 1.0, "depth 10 rgb")
    assert_outputs_close(dep, ed, max(1.0, np.abs(ed).max()), "depth 10 depth")
    assert_outputs_close(acc, ea, 1.0, "depth 10 acc")
    keep = case.smooth_rays(o, d)
    g_rgb = rng.normal(size=(keep.size, 3)).astype(np.float32)
    g_dep = rng.normal(size=keep.size).astype(np.float32)
    gF, gp = _gpu_backward(case, o[keep], d[keep], g_rgb, g_dep, None)
    _, _, _, st = case.oracle(o[keep], d[keep])
    eF, ep = render_backward(st, g_rgb, g_dep)
    mF, mp = render_backward_hit_magnitude(st, g_rgb, g_dep)
    mW = render_backward_weight_scale(st, g_rgb, g_dep)
    assert_grad_close(gF, eF, "depth 10 grad_features", mag=mF, wmag=mW)
    assert_grad_close(gp, ep, "depth 10 grad_params", rel_nw=1e-4, mag=mp, c=C_PARAM)
    # the light-field function on the same scene and rays
    from tests.gpu_cases import LfCase
    from oracle.lightfield import render_lf_backward, render_lf_backward_hit_magnitude, render_lf_backward_weight_scale
    lf = LfCase(gpu_lib, cells, depth, rng.normal(0.0, 0.5, (nv, 96)).astype(np.float32),
                LfCase.random(gpu_lib, 10, 5, K=8).p, 8)
    lrgb, ldep, lacc = lf.gpu_render(o, d)
    lr, ld, la, _ = lf.oracle(o, d)
    assert_outputs_close(lrgb, lr, 1.0, "depth 10 lf rgb")
    assert_outputs_close(ldep, ld, max(1.0, np.abs(ld).max()), "depth 10 lf depth")
    keep = lf.smooth_rays(o, d)
    lg_rgb = rng.normal(size=(keep.size, 3)).astype(np.float32)
    lg_dep = rng.normal(size=keep.size).astype(np.float32)
    lgF, lgp = lf.gpu_backward(o[keep], d[keep], lg_rgb, lg_dep)
    _, _, _, lst = lf.oracle(o[keep], d[keep])
    leF, lep = render_lf_backward(lst, lg_rgb, lg_dep)
    lmF, lmp = render_lf_backward_hit_magnitude(lst, lg_rgb, lg_dep)
    lmW = render_lf_backward_weight_scale(lst, lg_rgb, lg_dep)
    assert_grad_close(lgF, leF, "depth 10 lf grad_features", mag=lmF, wmag=lmW, c_w=C_W_LF)
    assert_grad_close(lgp, lep, "depth 10 lf grad_params", rel_nw=1e-4, mag=lmp, c=C_PARAM)


def _train_outputs(case, o, d, t_rgb, t_dep, precision):
    import torch
    n = o.shape[0]
    to, td = case.rays(o, d)
    gF = torch.zeros(case.scene.features.shape, dtype=torch.float32, device="cuda")
    gp = torch.zeros(case.params.shape, dtype=torch.float32, device="cuda")
    loss_t = torch.zeros(1, dtype=torch.float32, device="cuda")
    out_rgb = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    out_dep = torch.empty((n,), dtype=torch.float32, device="cuda")
    case.svlf.train_step([case.scene], [n], case.params, case.widths, case.opts(precision), to, td,
                         torch.from_numpy(t_rgb).cuda(), torch.from_numpy(t_dep).cuda(),
                         0.1, 1.0 / n, [gF], gp, out_rgb, out_dep, loss_t)
    torch.cuda.synchronize()
    return out_rgb.cpu().numpy(), out_dep.cpu().numpy(), float(loss_t.item())


def test_full_items_of_max_hits(gpu_lib):
    """A fully occupied depth-5 scene crossed by rays through its centre:
    every ray keeps K = 16 hits, so each full 256-ray work item holds the
    largest possible hit list (4,096 hits, 32 windows) and its windows end
    where the item's hit map ends.  Train-step outputs and loss on every ray
    (two full items and a ragged one, FP32 and BF16), and the gradients on
    the rays clear of decoder kinks, against the oracle."""
    from tests.helpers import crafted_occupancy
    leaves = crafted_occupancy("full", 5).astype(np.int32)
    widths = (16, 64, 64, 64, 4)
    rng = np.random.default_rng(77)
    F = (rng.normal(0.0, 1.0, (33 ** 3, 16)) * 2.0).astype(np.float32)
    p = xavier_params(rng, widths)
    p[-1] = 0.0                        # mean opacity about 0.4 over the 16 voxels
    case = Case(gpu_lib, leaves, 5, F, p, widths, 16)
    n = 2 * 256 + 37
    v = rng.standard_normal((n, 3))
    o = (3.0 * v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)
    d = rng.uniform(-0.2, 0.2, (n, 3)) - o
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    er, ed, ea, st = case.oracle(o, d)
    counts = np.bincount(st.ray_i, minlength=n)
    assert np.all(counts == 16), np.bincount(counts)
    t_rgb = rng.uniform(0, 1, (n, 3)).astype(np.float32)
    t_dep = rng.uniform(0, 5, n).astype(np.float32)
    rgb, dep, L = _train_outputs(case, o, d, t_rgb, t_dep, "fp32")
    L_ref, _, _ = oracle_loss(er, ed, t_rgb, t_dep, 0.1)
    assert abs(L - L_ref) <= 1e-5 * abs(L_ref)
    assert_outputs_close(rgb, er, 1.0, "full items rgb")
    assert_outputs_close(dep, ed, max(1.0, np.abs(ed).max()), "full items depth")
    br, bd, ba, bst = case.oracle(o, d, bf16=True)
    rgb16, dep16, _ = _train_outputs(case, o, d, t_rgb, t_dep, "bf16")
    assert_bf16_render_close(rgb16, dep16, None, (br, bd, ba), bst, case.F, "full items bf16")
    keep = case.smooth_rays(o, d)
    assert keep.size > n // 3
    g_rgb = rng.normal(size=(keep.size, 3)).astype(np.float32)
    g_dep = rng.normal(size=keep.size).astype(np.float32)
    gF, gp = _gpu_backward(case, o[keep], d[keep], g_rgb, g_dep, None)
    _, _, _, st2 = case.oracle(o[keep], d[keep])
    eF, ep = render_backward(st2, g_rgb, g_dep)
    # 16 hits on every ray: Eq. 3's dL/dtau is a difference of suffix sums
    # over up to 15 later hits, so the feature entries are checked at the
    # conditioning of each hit's dL/dX
    mF, mp = render_backward_hit_magnitude(st2, g_rgb, g_dep, conditioned=True)
    mW = render_backward_weight_scale(st2, g_rgb, g_dep)
    assert_grad_close(gF, eF, "full items grad_features", mag=mF, wmag=mW)
    assert_grad_close(gp, ep, "full items grad_params", rel_nw=1e-4, mag=mp, c=C_PARAM)
    # the deterministic reduction reads each hit's slot from the same map
    import torch
    to, td = case.rays(o[keep], d[keep])
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()
    det = []
    for _ in range(2):
        gFd = torch.zeros(case.scene.features.shape, dtype=torch.float32, device="cuda")
        gpd = torch.zeros(case.params.shape, dtype=torch.float32, device="cuda")
        opts = gpu_lib.make_opts(case.K, case.tau_mode, "fp32", gpu_lib.FLAG_DETERMINISTIC)
        gpu_lib.render_backward([case.scene], [keep.size], case.params, case.widths, opts, to, td,
                                t(g_rgb), t(g_dep), None, [gFd], gpd)
        torch.cuda.synchronize()
        det.append((gFd.cpu().numpy(), gpd.cpu().numpy()))
    assert np.array_equal(det[0][0].view(np.int32), det[1][0].view(np.int32))
    assert np.array_equal(det[0][1].view(np.int32), det[1][1].view(np.int32))
    assert_grad_close(det[0][0], eF, "full items deterministic grad_features", mag=mF, wmag=mW)
    assert_grad_close(det[0][1], ep, "full items deterministic grad_params", rel_nw=1e-4, mag=mp, c=C_PARAM)


def test_full_items_of_max_hits_light_field(gpu_lib):
    """The light-field kernels on the same fully occupied depth-5 scene: every
    ray keeps K = 16 hits, so the backward kernels' item-wide hit maps are
    full (4,096 hits per item).  Forward on every ray and gradients on the
    rays clear of decoder kinks against the oracle."""
    from tests.gpu_cases import LfCase
    from tests.helpers import crafted_occupancy
    from oracle.lightfield import render_lf_backward, render_lf_backward_hit_magnitude, render_lf_backward_weight_scale
    from oracle.lightfield import widths_of
    from oracle.render import split_params
    leaves = crafted_occupancy("full", 5).astype(np.int32)
    rng = np.random.default_rng(78)
    F = rng.normal(0, 0.5, (33 ** 3, 96)).astype(np.float32)
    # hidden biases of 0.5 keep most ReLU inputs clear of zero, so that most
    # rays (16 hits each) are free of decoder kinks and the gradient rays
    # still fill whole work items
    wt, wc = widths_of(tuple(gpu_lib.LF_DECODERS), False)
    nt = sum(a * b + b for a, b in zip(wt[:-1], wt[1:]))
    p = LfCase.random(gpu_lib, 17, 5, K=16).p.astype(np.float64)
    for _, b in split_params(p[:nt], wt)[:-1] + split_params(p[nt:], wc)[:-1]:
        b[:] = 0.5
    lf = LfCase(gpu_lib, leaves, 5, F, p.astype(np.float32), 16)
    n = 2 * 256 + 37
    v = rng.standard_normal((n, 3))
    o = (3.0 * v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)
    d = rng.uniform(-0.2, 0.2, (n, 3)) - o
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    lr, ld, la, lst = lf.oracle(o, d)
    assert np.all(np.bincount(lst.ray_i, minlength=n) == 16)
    lrgb, ldep, lacc = lf.gpu_render(o, d)
    assert_outputs_close(lrgb, lr, 1.0, "full items lf rgb")
    assert_outputs_close(ldep, ld, max(1.0, np.abs(ld).max()), "full items lf depth")
    keep = lf.smooth_rays(o, d)
    assert keep.size > 256                  # at least one full work item of kink-free rays
    g_rgb = rng.normal(size=(keep.size, 3)).astype(np.float32)
    g_dep = rng.normal(size=keep.size).astype(np.float32)
    gF, gp = lf.gpu_backward(o[keep], d[keep], g_rgb, g_dep)
    _, _, _, st2 = lf.oracle(o[keep], d[keep])
    eF, ep = render_lf_backward(st2, g_rgb, g_dep)
    mF, mp = render_lf_backward_hit_magnitude(st2, g_rgb, g_dep)
    mW = render_lf_backward_weight_scale(st2, g_rgb, g_dep)
    ct = lf.dec[0]
    assert_grad_close(gF[:, :ct], eF[:, :ct], "full items lf grad Z_T", mag=mF[:, :ct], wmag=mW[:, :ct],
                      c_w=C_W_LF)
    # Z_C: the hidden biases make the density decoder's activations large,
    # and eta's FP32 error moves the surface point by more than the few ulps
    # the weight-sensitivity term assumes; its own bound is added
    E = lf_surface_point_error(st2, lf.F, g_rgb, g_dep)
    assert_grad_close(gF[:, ct:], eF[:, ct:], "full items lf grad Z_C", mag=mF[:, ct:],
                      wmag=mW[:, ct:] + 2.0 * E / (C_W_LF * EPS32), c_w=C_W_LF)
    assert_grad_close(gp, ep, "full items lf grad_params", rel_nw=1e-4, mag=mp, c=C_PARAM)
