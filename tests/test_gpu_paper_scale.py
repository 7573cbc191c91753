"""Parity at the paper-scale workload (depth 9, 1.37M occupied leaves,
1600^2 views, 2^20-ray training batch) in the launch configuration the
benchmark times: whole-view / whole-batch launches, with seeded samples of
rays compared against the oracle and properties checked on every output."""

import numpy as np
import pytest

from oracle.octree import Octree
from oracle.render import (loss as oracle_loss, render as oracle_render, render_backward,
                           render_backward_hit_magnitude,
                           render_backward_weight_scale)
from oracle.trace import trace_hits as oracle_trace
from synth.configs import get_workload
from tests.gpu_cases import (BF16_ULP, C_PARAM, C_W, C_W_LF, EPS32, assert_bf16_render_close, assert_grad_close,
                             assert_outputs_close,
                             cosine, decoder_kinks as _decoder_kinks, lf_kinks as _lf_kinks, loss_scales,
                             residual_terms,
                             psnr)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def paper(gpu_lib):
    import torch
    w = get_workload("surfaces_d9")
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
        br, bd, ba, bst = oracle_render(paper["oc"], paper["F"], paper["p"], w.widths, o[idx], d[idx], hits,
                                        bf16=True)
        er, _, _, _ = oracle_render(paper["oc"], paper["F"], paper["p"], w.widths, o[idx], d[idx], hits)
        assert_bf16_render_close(rgb[idx], dep[idx], acc[idx], (br, bd, ba), bst, paper["F"], "paper-scale bf16")
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


@pytest.mark.parametrize("det", [True, False], ids=["deterministic", "atomic"])
def test_train_step_from_hip_graph(gpu_lib, paper, det):
    """The 2^20-ray BF16 train step captured in a HIP graph and replayed
    three times, with eager work between the replays, gives the eager
    call's outputs, gradients and loss: bit for bit in deterministic mode
    (which orders the hits on the library's side stream while the shading
    kernel runs: a fork / join inside the graph), within FP32 atomic-order
    rounding otherwise (per-ray outputs are exact)."""
    import torch
    w = paper["w"]
    ob, db, rgb_t, dep_t = w.train_batch(w.batch, step=1)
    n = ob.shape[0]
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    args = [T(ob), T(db), T(rgb_t), T(dep_t)]
    ws = gpu_lib.Workspace()
    opts = gpu_lib.make_opts(w.K, "voxel", "bf16", gpu_lib.FLAG_DETERMINISTIC if det else 0)
    gF = torch.zeros_like(paper["scene"].features)
    gp = torch.zeros_like(paper["params"])
    loss = torch.zeros(1, device="cuda")
    rgb = torch.empty((n, 3), device="cuda")
    dep = torch.empty(n, device="cuda")

    def work():
        gpu_lib.fill(gF, 0.0)
        gpu_lib.fill(gp, 0.0)
        gpu_lib.train_step([paper["scene"]], [n], paper["params"], w.widths, opts, *args, 0.1,
                           1.0 / n, [gF], gp, out_rgb=rgb, out_depth=dep, loss_out=loss, workspace=ws)

    def same(x, y):
        if det:
            return torch.equal(x, y)
        return float((x - y).abs().max()) <= 1e-5 * float(y.abs().max()) + 1e-30

    work()
    torch.cuda.synchronize()
    ref = (gF.clone(), gp.clone(), loss.clone())
    ref_out = (rgb.clone(), dep.clone())
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            work()
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    for rep in range(3):
        gF.fill_(-1.0)
        gp.fill_(-1.0)
        loss.fill_(-1.0)
        rgb.fill_(-1.0)
        dep.fill_(-1.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert same(gF, ref[0]), rep
        assert same(gp, ref[1]), rep
        assert same(loss, ref[2]), rep
        assert torch.equal(rgb, ref_out[0]) and torch.equal(dep, ref_out[1]), rep
        work()                                    # eager call between replays
        torch.cuda.synchronize()
        assert same(gF, ref[0]), rep


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


# ---------------------------------------------------------------------------
# Gradient parity at the size the benchmarked kernels run.  A subset of
# N_SUB rays of the 2^20-ray batch spans four full groups of 256 work items
# (65,536 rays, whose rays the shading kernels interleave) and a ragged tail;
# the persistent grid then runs several items per block, and each window's
# feature-gradient scatter is deferred behind the next window's gather and
# across items.  The rays are those away from every kink of the loss: no
# decoder pre-activation within 1e-4 of zero (FP32 and FP64 may take
# different one-sided derivatives there) and a depth residual of the L1 term
# clear of zero by more than the precision's output error.

N_SUB = 4 * 65536 + 777
def _batch(paper):
    if "batch" not in paper:
        w = paper["w"]
        paper["batch"] = w.train_batch(w.batch, step=0)
    return paper["batch"]


def _kink_free_subset(paper, render_fn, kinks, bf16, seed):
    """First N_SUB rays (in batch order) of a seeded sample of the batch that
    avoid every kink; returns (o, d, rgb*, depth*, hit lists) of those rays."""
    w = paper["w"]
    ob, db, rgb_t, dep_t = _batch(paper)
    idx = np.sort(np.random.default_rng(seed).choice(ob.shape[0], N_SUB + N_SUB // 4, replace=False))
    hits = oracle_trace(paper["oc"], ob[idx], db[idx], w.K)
    _, dep, _, st = render_fn(ob[idx], db[idx], hits, bf16)
    bad = np.zeros(idx.size, bool)
    bad[np.unique(st.ray_i[kinks(st)])] = True
    print(f"kink-free subset: {np.count_nonzero(bad)} of {idx.size} sampled rays excluded, "
          f"{st.ray_i.size} hits sampled")
    margin = (2.0 ** -6 if bf16 else 1e-4) * np.maximum(1.0, np.abs(dep_t[idx]))
    res = dep - dep_t[idx]
    bad |= (res != 0) & (np.abs(res) < margin)
    keep = np.nonzero(~bad)[0][:N_SUB]
    assert keep.size == N_SUB
    sel = idx[keep]
    return ob[sel], db[sel], rgb_t[sel], dep_t[sel], tuple(x[keep] for x in hits)


def _gpu_train(gpu_lib, scene, params, opts, o, d, rgb_t, dep_t, lf=False):
    import torch
    n = o.shape[0]
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    gF = torch.zeros_like(scene.features)
    gp = torch.zeros_like(params)
    loss = torch.zeros(1, device="cuda")
    out_rgb = torch.empty((n, 3), device="cuda")
    out_dep = torch.empty(n, device="cuda")
    step = gpu_lib.lf_train_step if lf else gpu_lib.train_step
    extra = () if lf else (paper_widths(),)
    step([scene], [n], params, *extra, opts, T(o), T(d), T(rgb_t), T(dep_t), 0.1, 1.0 / n,
         [gF], gp, out_rgb=out_rgb, out_depth=out_dep, loss_out=loss)
    torch.cuda.synchronize()
    return (gF.cpu().numpy(), gp.cpu().numpy(), out_rgb.cpu().numpy(), out_dep.cpu().numpy(),
            float(loss.item()))


def paper_widths():
    return tuple(get_workload("surfaces_d9").widths)


def _check_bf16_grads(got, exp, mag, name, wmag=None, c_w=C_W):
    """BF16 against the oracle's BF16-rounding mode: where an FP32 and an FP64
    value straddle a bfloat16 rounding boundary the two round apart by one
    bfloat16 ulp, and the decoder's chain amplifies such a step like any
    rounding error, so the comparison is by direction and size of the whole
    gradient (cosine, relative L2); the per-entry error in units of 2^-8 M
    is reported as quantiles."""
    c = cosine(got, exp)
    r = float(np.linalg.norm(got - exp) / np.linalg.norm(exp))
    err = np.abs(np.asarray(got, np.float64) - exp)
    if wmag is not None:
        err = np.maximum(err - EPS32 * c_w * wmag, 0.0)
    pos = mag > 0
    q = np.quantile(err[pos] / (BF16_ULP * mag[pos]), [0.5, 0.99, 0.999, 1.0])
    print(f"{name}: cosine {c:.8f}, relative L2 {r:.3g}, |err| / (2^-8 M) quantiles 50/99/99.9/100%: "
          f"{q[0]:.3g} {q[1]:.3g} {q[2]:.3g} {q[3]:.3g}")
    assert c >= 0.99999 and r <= 2e-3, (name, c, r)
    assert np.all(err[~pos] == 0)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_train_step_gradients_on_batch_subset(gpu_lib, paper, precision):
    """svlf_train_step on N_SUB rays of the paper-scale batch: loss, outputs
    and both gradients against the oracle (FP32: per-entry bounds; BF16:
    against the oracle's BF16-rounding mode)."""
    w = paper["w"]
    bf = precision == "bf16"
    F, p = paper["F"], paper["p"]
    rnd = lambda o, d, hits, b: oracle_render(paper["oc"], F, p, w.widths, o, d, hits, bf16=b)
    o, d, rgb_t, dep_t, hits = _kink_free_subset(paper, rnd, _decoder_kinks, bf, 11)
    gF, gp, r, dd, L = _gpu_train(gpu_lib, paper["scene"], paper["params"],
                                  gpu_lib.make_opts(w.K, "voxel", precision), o, d, rgb_t, dep_t)
    er, ed, _, st = rnd(o, d, hits, bf)
    L_ref, g_rgb, g_dep = oracle_loss(er, ed, rgb_t, dep_t, 0.1)
    eF, ep = render_backward(st, g_rgb, g_dep)
    mF, mp, mW = loss_scales(render_backward_hit_magnitude, render_backward_weight_scale, st, g_rgb,
                             residual_terms(g_rgb, er, rgb_t), g_dep)
    print(f"{precision}: {o.shape[0]} rays, {st.ray_i.size} hits, {np.count_nonzero(mF.any(axis=1))} "
          f"feature rows reached")
    if not bf:
        assert abs(L - L_ref) <= 1e-5 * abs(L_ref)
        assert_outputs_close(r, er, 1.0, "rgb")
        assert_outputs_close(dd, ed, max(1.0, np.abs(ed).max()), "depth")
        assert_grad_close(gF, eF, "grad_features", mag=mF, wmag=mW)
        assert_grad_close(gp, ep, "grad_params", rel_nw=1e-4, mag=mp, c=C_PARAM)
    else:
        assert abs(L - L_ref) <= 2 ** -8 * abs(L_ref)
        assert np.abs(r - er).max() <= 2 ** -6 * np.abs(er).max() + 1e-4
        _check_bf16_grads(gF, eF, mF, "bf16 grad_features", mW)
        _check_bf16_grads(gp, ep, mp, "bf16 grad_params")


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_render_backward_full_batch_sparse_upstream(gpu_lib, paper, precision):
    """svlf_render_backward on the whole 2^20-ray batch with upstream
    gradients that vanish except on 2,048 seeded kink-free rays: the kernel
    takes every full-size path (interleaved groups, several items per block,
    scatter deferred across items) while the oracle needs the sampled rays
    only (a ray with zero upstream gradient contributes exact zeros)."""
    import torch
    w = paper["w"]
    bf = precision == "bf16"
    ob, db, _, _ = _batch(paper)
    n = ob.shape[0]
    idx = _sample(n, 2600, 12)
    hits = oracle_trace(paper["oc"], ob[idx], db[idx], w.K)
    _, _, _, st = oracle_render(paper["oc"], paper["F"], paper["p"], w.widths, ob[idx], db[idx], hits, bf16=bf)
    bad = np.zeros(idx.size, bool)
    bad[np.unique(st.ray_i[_decoder_kinks(st)])] = True
    sel = idx[~bad][:2048]
    rng = np.random.default_rng(13)
    g_rgb = np.zeros((n, 3), np.float32)
    g_dep = np.zeros(n, np.float32)
    g_acc = np.zeros(n, np.float32)
    g_rgb[sel] = rng.normal(size=(sel.size, 3))
    g_dep[sel] = rng.normal(size=sel.size) * 0.1
    g_acc[sel] = rng.normal(size=sel.size)
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    gF = torch.zeros_like(paper["scene"].features)
    gp = torch.zeros_like(paper["params"])
    gpu_lib.render_backward([paper["scene"]], [n], paper["params"], w.widths,
                            gpu_lib.make_opts(w.K, "voxel", precision), T(ob), T(db), T(g_rgb), T(g_dep),
                            T(g_acc), [gF], gp)
    torch.cuda.synchronize()
    gF, gp = gF.cpu().numpy(), gp.cpu().numpy()
    hs = oracle_trace(paper["oc"], ob[sel], db[sel], w.K)
    _, _, _, st = oracle_render(paper["oc"], paper["F"], paper["p"], w.widths, ob[sel], db[sel], hs, bf16=bf)
    ups = (g_rgb[sel], g_dep[sel], g_acc[sel])
    eF, ep = render_backward(st, *ups)
    mF, mp = render_backward_hit_magnitude(st, *ups)
    mW = render_backward_weight_scale(st, *ups)
    assert st.ray_i.size > 1000
    if not bf:
        assert_grad_close(gF, eF, "sparse-upstream grad_features", mag=mF, wmag=mW)
        assert_grad_close(gp, ep, "sparse-upstream grad_params", rel_nw=1e-4, mag=mp, c=C_PARAM)
    else:
        _check_bf16_grads(gF, eF, mF, "sparse-upstream bf16 grad_features", mW)
        _check_bf16_grads(gp, ep, mp, "sparse-upstream bf16 grad_params")


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_lightfield_train_step_gradients_on_batch_subset(gpu_lib, paper, precision):
    """svlf_lf_train_step (the paper's two-decoder function) on N_SUB rays of
    the paper-scale batch against the light-field oracle."""
    import torch
    from oracle.lightfield import (render_lf, render_lf_backward, render_lf_backward_hit_magnitude,
                                   render_lf_backward_weight_scale)
    from synth.configs import lf_inputs
    w, sc = paper["w"], paper["sc"]
    bf = precision == "bf16"
    if "lf" not in paper:
        F, p = lf_inputs(w.seed, sc.n_vertices)
        paper["lf"] = (F, p, gpu_lib.DeviceScene.lf_from_host(sc.leaf_ijk, sc.depth, F, bf16=True),
                       torch.from_numpy(p).cuda())
    F, p, scene, params = paper["lf"]
    dec = tuple(gpu_lib.LF_DECODERS)
    rnd = lambda o, d, hits, b: render_lf(paper["oc"], F, p, dec, o, d, hits, bf16=b)
    o, d, rgb_t, dep_t, hits = _kink_free_subset(paper, rnd, _lf_kinks, bf, 14)
    gF, gp, r, dd, L = _gpu_train(gpu_lib, scene, params, gpu_lib.make_opts(w.K, "direct", precision),
                                  o, d, rgb_t, dep_t, lf=True)
    gF = gpu_lib.lf_feature_rows(gF, sc.n_vertices)
    er, ed, _, st = rnd(o, d, hits, bf)
    L_ref, g_rgb, g_dep = oracle_loss(er, ed, rgb_t, dep_t, 0.1)
    eF, ep = render_lf_backward(st, g_rgb, g_dep)
    mF, mp, mW = loss_scales(render_lf_backward_hit_magnitude, render_lf_backward_weight_scale, st, g_rgb,
                             residual_terms(g_rgb, er, rgb_t), g_dep)
    ct = dec[0]
    if not bf:
        assert abs(L - L_ref) <= 1e-5 * abs(L_ref)
        assert_outputs_close(r, er, 1.0, "lf rgb")
        assert_outputs_close(dd, ed, max(1.0, np.abs(ed).max()), "lf depth")
        assert_grad_close(gF[:, :ct], eF[:, :ct], "lf grad Z_T", mag=mF[:, :ct], wmag=mW[:, :ct], c_w=C_W_LF)
        assert_grad_close(gF[:, ct:], eF[:, ct:], "lf grad Z_C", mag=mF[:, ct:], wmag=mW[:, ct:], c_w=C_W_LF)
        assert_grad_close(gp, ep, "lf grad_params", rel_nw=1e-4, mag=mp, c=C_PARAM)
    else:
        assert abs(L - L_ref) <= 2 ** -8 * abs(L_ref)
        assert np.abs(r - er).max() <= 2 ** -6 * np.abs(er).max() + 1e-4
        _check_bf16_grads(gF, eF, mF, "lf bf16 grad_features", mW, C_W_LF)
        _check_bf16_grads(gp, ep, mp, "lf bf16 grad_params")
