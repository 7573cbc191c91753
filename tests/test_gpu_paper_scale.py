"""Parity at the paper-scale workload (depth 9, 1.37M occupied leaves,
1600^2 views, 2^20-ray training batch) in the launch configuration the
benchmark times: whole-view / whole-batch launches, with seeded samples of
rays compared against the oracle and properties checked on every output."""

import numpy as np
import pytest

from oracle.octree import Octree
from oracle.render import loss as oracle_loss, render as oracle_render
from oracle.trace import trace_hits as oracle_trace
from synth.configs import get_config
from tests.gpu_cases import assert_outputs_close, psnr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def paper(gpu_lib):
    import torch
    w = get_config(3)
    sc = w.scene()
    F = w.features()
    p = w.params().copy()
    p[-1] = 0.5           # opaque enough that compositing matters
    scene = gpu_lib.DeviceScene.from_host(sc.leaf_ijk, sc.depth, F, bf16=True)
    oc = Octree(sc.leaf_ijk, sc.depth)
    return dict(w=w, sc=sc, F=F, p=p, scene=scene, params=torch.from_numpy(p).cuda(), oc=oc)


def _sample(n, k, seed):
    return np.sort(np.random.default_rng(seed).choice(n, k, replace=False))


def test_trace_full_view_sampled(gpu_lib, paper):
    import torch
    w = paper["w"]
    o, d = w.view_rays(0)
    leaf, tin, tout, cnt = gpu_lib.trace_hits(paper["scene"].octree, torch.from_numpy(o).cuda(),
                                              torch.from_numpy(d).cuda(), w.K)
    torch.cuda.synchronize()
    idx = _sample(o.shape[0], 4096, 1)
    el, ei, eo, ec = oracle_trace(paper["oc"], o[idx], d[idx], w.K)
    np.testing.assert_array_equal(cnt.cpu().numpy()[idx], ec)
    np.testing.assert_array_equal(leaf.cpu().numpy()[idx], el)
    np.testing.assert_array_equal(tin.cpu().numpy()[idx].view(np.int32), ei.view(np.int32))
    np.testing.assert_array_equal(tout.cpu().numpy()[idx].view(np.int32), eo.view(np.int32))
    c = cnt.cpu().numpy()
    assert c.max() <= w.K and 0.05 < (c > 0).mean() < 0.6


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_render_full_view_sampled(gpu_lib, paper, precision):
    import torch
    w = paper["w"]
    o, d = w.view_rays(0)
    n = o.shape[0]
    opts = gpu_lib.make_opts(w.K, "voxel", precision)
    rgb, dep, acc = gpu_lib.render([paper["scene"]], [n], paper["params"], w.widths, opts,
                                   torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda())
    torch.cuda.synchronize()
    rgb, dep, acc = rgb.cpu().numpy(), dep.cpu().numpy(), acc.cpu().numpy()
    assert np.all(np.isfinite(rgb)) and np.all(acc >= 0) and np.all(acc <= 1 + 1e-6)
    assert np.all(rgb <= acc[:, None] + 1e-6)
    idx = _sample(n, 4096, 2)
    hits = oracle_trace(paper["oc"], o[idx], d[idx], w.K)
    if precision == "fp32":
        er, ed, ea, _ = oracle_render(paper["oc"], paper["F"], paper["p"], w.widths, o[idx], d[idx], hits)
        assert_outputs_close(rgb[idx], er, 1.0, "rgb")
        assert_outputs_close(dep[idx], ed, max(1.0, np.abs(ed).max()), "depth")
        assert_outputs_close(acc[idx], ea, 1.0, "acc")
    else:
        br, bd, ba, _ = oracle_render(paper["oc"], paper["F"], paper["p"], w.widths, o[idx], d[idx], hits,
                                      bf16=True)
        er, _, _, _ = oracle_render(paper["oc"], paper["F"], paper["p"], w.widths, o[idx], d[idx], hits)
        assert np.abs(rgb[idx] - br).max() <= 2 ** -6 * np.abs(br).max() + 1e-4
        assert psnr(rgb[idx], er) > 40.0


def test_train_step_full_batch(gpu_lib, paper):
    """Forward outputs of the fused train step on the full 2^20 batch match
    the oracle on a sample; the returned loss equals the loss recomputed from
    the step's own outputs; gradients are finite and conserve mass."""
    import torch
    w = paper["w"]
    ob, db, rgb_t, dep_t = w.train_batch(w.batch, step=0)
    n = ob.shape[0]
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    gF = torch.zeros_like(paper["scene"].features)
    gp = torch.zeros_like(paper["params"])
    loss = torch.zeros(1, device="cuda")
    out_rgb = torch.empty((n, 3), device="cuda")
    out_dep = torch.empty(n, device="cuda")
    gpu_lib.train_step([paper["scene"]], [n], paper["params"], w.widths,
                       gpu_lib.make_opts(w.K, "voxel", "fp32"), T(ob), T(db), T(rgb_t), T(dep_t),
                       0.1, 1.0 / n, [gF], gp, out_rgb=out_rgb, out_depth=out_dep, loss_out=loss)
    torch.cuda.synchronize()
    r, dd = out_rgb.cpu().numpy(), out_dep.cpu().numpy()
    L_self, _, _ = oracle_loss(r, dd, rgb_t, dep_t, 0.1)
    assert abs(float(loss.item()) - L_self) <= 1e-4 * abs(L_self)
    idx = _sample(n, 2048, 3)
    hits = oracle_trace(paper["oc"], ob[idx], db[idx], w.K)
    er, ed, ea, _ = oracle_render(paper["oc"], paper["F"], paper["p"], w.widths, ob[idx], db[idx], hits)
    assert_outputs_close(r[idx], er, 1.0, "train-step rgb")
    assert_outputs_close(dd[idx], ed, max(1.0, np.abs(ed).max()), "train-step depth")
    g = gF.cpu().numpy()
    assert np.all(np.isfinite(g)) and np.abs(g).max() > 0
    assert np.all(np.isfinite(gp.cpu().numpy())) and float(gp.abs().max()) > 0


def test_lightfield_train_step_full_batch(gpu_lib, paper):
    """The two-decoder light-field train step on the full 2^20-ray batch:
    sampled rays' forward outputs against the oracle, the loss against the
    step's own outputs, finite gradients in both feature blocks."""
    import torch
    from oracle.lightfield import render_lf
    from synth.configs import lf_inputs
    w, sc = paper["w"], paper["sc"]
    F, p = lf_inputs(w.seed, sc.n_vertices)
    scene = gpu_lib.DeviceScene.lf_from_host(sc.leaf_ijk, sc.depth, F, bf16=True)
    params = torch.from_numpy(p).cuda()
    ob, db, rgb_t, dep_t = w.train_batch(w.batch, step=0)
    n = ob.shape[0]
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    gF = torch.zeros_like(scene.features)
    gp = torch.zeros_like(params)
    loss = torch.zeros(1, device="cuda")
    out_rgb = torch.empty((n, 3), device="cuda")
    out_dep = torch.empty(n, device="cuda")
    gpu_lib.lf_train_step([scene], [n], params, gpu_lib.make_opts(w.K, "direct", "fp32"), T(ob), T(db),
                          T(rgb_t), T(dep_t), 0.1, 1.0 / n, [gF], gp, out_rgb=out_rgb, out_depth=out_dep,
                          loss_out=loss)
    torch.cuda.synchronize()
    r, dd = out_rgb.cpu().numpy(), out_dep.cpu().numpy()
    L_self, _, _ = oracle_loss(r, dd, rgb_t, dep_t, 0.1)
    assert abs(float(loss.item()) - L_self) <= 1e-4 * abs(L_self)
    idx = _sample(n, 1024, 4)
    hits = oracle_trace(paper["oc"], ob[idx], db[idx], w.K)
    er, ed, _, _ = render_lf(paper["oc"], F, p, (64, 32, 128, 1, 3), ob[idx], db[idx], hits)
    assert_outputs_close(r[idx], er, 1.0, "lf train-step rgb")
    assert_outputs_close(dd[idx], ed, max(1.0, np.abs(ed).max()), "lf train-step depth")
    g = gpu_lib.lf_feature_rows(gF.cpu().numpy(), sc.n_vertices)
    assert np.all(np.isfinite(g)) and np.abs(g[:, :64]).max() > 0 and np.abs(g[:, 64:]).max() > 0
    assert np.all(np.isfinite(gp.cpu().numpy()))


def test_deterministic_train_step_paper_scale(gpu_lib, paper):
    """Full 2^20-ray BF16 train step with the deterministic feature-gradient
    reduction: two runs give bit-identical feature gradients, within FP32
    accumulation tolerance of the atomic path."""
    import torch
    w = paper["w"]
    ob, db, rgb_t, dep_t = w.train_batch(w.batch, step=0)
    n = ob.shape[0]
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    args = [T(ob), T(db), T(rgb_t), T(dep_t)]

    def run(flags):
        gF = torch.zeros_like(paper["scene"].features)
        gp = torch.zeros_like(paper["params"])
        gpu_lib.train_step([paper["scene"]], [n], paper["params"], w.widths,
                           gpu_lib.make_opts(w.K, "voxel", "bf16", flags), *args, 0.1, 1.0 / n, [gF], gp)
        torch.cuda.synchronize()
        return gF.cpu().numpy()

    a = run(gpu_lib.FLAG_DETERMINISTIC)
    b = run(gpu_lib.FLAG_DETERMINISTIC)
    assert np.array_equal(a.view(np.int32), b.view(np.int32))
    c = run(0)
    scale = np.abs(c).max()
    assert scale > 0 and np.abs(a - c).max() <= 1e-5 * scale


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_train_step_full_batch_equals_chunked_calls(gpu_lib, paper, precision):
    """The shading kernels interleave the rays of groups of 256 full work
    items (65,536 rays); calls of 60,000 rays have no full group and take
    the rays in order.  The full-batch train step must give the same per-ray
    outputs (bit-exact: each ray is composited on its own), the same loss
    and the same gradients (up to FP32 summation order) as the sum of
    chunked calls over the same rays."""
    import torch
    w = paper["w"]
    ob, db, rgb_t, dep_t = w.train_batch(w.batch, step=0)
    n = ob.shape[0]
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    o, d, tr, td = T(ob), T(db), T(rgb_t), T(dep_t)
    opts = gpu_lib.make_opts(w.K, "voxel", precision)

    def run(bounds):
        gF = torch.zeros_like(paper["scene"].features)
        gp = torch.zeros_like(paper["params"])
        rgb = torch.empty((n, 3), device="cuda")
        dep = torch.empty(n, device="cuda")
        L = 0.0
        for lo, hi in zip(bounds[:-1], bounds[1:]):
            gpc = torch.zeros_like(gp)
            loss = torch.zeros(1, device="cuda")
            gpu_lib.train_step([paper["scene"]], [hi - lo], paper["params"], w.widths, opts, o[lo:hi],
                               d[lo:hi], tr[lo:hi], td[lo:hi], 0.1, 1.0 / n, [gF], gpc,
                               out_rgb=rgb[lo:hi], out_depth=dep[lo:hi], loss_out=loss)
            gp += gpc
            L += float(loss.item())
        torch.cuda.synchronize()
        return gF.cpu().numpy(), gp.cpu().numpy(), rgb.cpu().numpy(), dep.cpu().numpy(), L

    fa, pa, ra, da, La = run([0, n])
    fb, pb, rb, db_, Lb = run(list(range(0, n, 60000)) + [n])
    assert np.array_equal(ra.view(np.int32), rb.view(np.int32))
    assert np.array_equal(da.view(np.int32), db_.view(np.int32))
    assert abs(La - Lb) <= 1e-5 * abs(Lb)
    sf, sp = np.abs(fb).max(), np.abs(pb).max()
    assert sf > 0 and np.abs(fa - fb).max() <= 1e-5 * sf
    assert sp > 0 and np.abs(pa - pb).max() <= 1e-4 * sp


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_lightfield_train_step_full_batch_equals_chunked_calls(gpu_lib, paper, precision):
    """As for the single decoder: the light-field kernels interleave the rays
    of full 65,536-ray groups, so the full-batch train step must match the
    sum of 60,000-ray calls (per-ray outputs bit-exact, loss and gradients up
    to FP32 summation order)."""
    import torch
    from synth.configs import lf_inputs
    w, sc = paper["w"], paper["sc"]
    F, p = lf_inputs(w.seed, sc.n_vertices)
    scene = gpu_lib.DeviceScene.lf_from_host(sc.leaf_ijk, sc.depth, F, bf16=True)
    params = torch.from_numpy(p).cuda()
    ob, db, rgb_t, dep_t = w.train_batch(w.batch, step=0)
    n = ob.shape[0]
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    o, d, tr, td = T(ob), T(db), T(rgb_t), T(dep_t)
    opts = gpu_lib.make_opts(w.K, "direct", precision)

    def run(bounds):
        gF = torch.zeros_like(scene.features)
        gp = torch.zeros_like(params)
        rgb = torch.empty((n, 3), device="cuda")
        dep = torch.empty(n, device="cuda")
        L = 0.0
        for lo, hi in zip(bounds[:-1], bounds[1:]):
            gpc = torch.zeros_like(gp)
            loss = torch.zeros(1, device="cuda")
            gpu_lib.lf_train_step([scene], [hi - lo], params, opts, o[lo:hi], d[lo:hi], tr[lo:hi],
                                  td[lo:hi], 0.1, 1.0 / n, [gF], gpc, out_rgb=rgb[lo:hi],
                                  out_depth=dep[lo:hi], loss_out=loss)
            gp += gpc
            L += float(loss.item())
        torch.cuda.synchronize()
        return gF.cpu().numpy(), gp.cpu().numpy(), rgb.cpu().numpy(), dep.cpu().numpy(), L

    fa, pa, ra, da, La = run([0, n])
    fb, pb, rb, db_, Lb = run(list(range(0, n, 60000)) + [n])
    assert np.array_equal(ra.view(np.int32), rb.view(np.int32))
    assert np.array_equal(da.view(np.int32), db_.view(np.int32))
    assert abs(La - Lb) <= 1e-5 * abs(Lb)
    sf, sp = np.abs(fb).max(), np.abs(pb).max()
    assert sf > 0 and np.abs(fa - fb).max() <= 1e-4 * sf
    assert sp > 0 and np.abs(pa - pb).max() <= 1e-4 * sp
