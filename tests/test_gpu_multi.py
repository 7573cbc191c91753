"""Ragged multi-scene launches (8 scenes of depths 3..6 sharing one decoder,
2^8..2^12 rays each) in one call, compared scene by scene with the oracle;
the same calls captured in a HIP graph and replayed."""

import numpy as np
import pytest

from oracle.render import render_backward
from synth.configs import get_multi
from tests.gpu_cases import Case, assert_grad_close, assert_outputs_close

pytestmark = pytest.mark.gpu


def _setup(gpu_lib):
    import torch
    m = get_multi(small=True)
    counts = m.ray_counts()
    p = m.params()
    p[-1] = 0.6
    cases, os_, ds_ = [], [], []
    for i in range(len(m.depths)):
        sc = m.scene(i)
        rng = np.random.default_rng(100 + i)
        F = rng.normal(0, 0.4, (sc.n_vertices, m.C)).astype(np.float32)
        cases.append(Case(gpu_lib, sc.leaf_ijk, sc.depth, F, p, m.widths, m.K))
        o, d = m.rays(i, counts[i])
        os_.append(o)
        ds_.append(d)
    o = np.concatenate(os_)
    d = np.concatenate(ds_)
    return m, cases, counts, o, d


def test_multi_scene_forward_matches_oracle(gpu_lib):
    import torch
    m, cases, counts, o, d = _setup(gpu_lib)
    to, td = cases[0].rays(o, d)
    rgb, dep, acc = gpu_lib.render([c.scene for c in cases], counts, cases[0].params, m.widths,
                                   cases[0].opts(), to, td)
    torch.cuda.synchronize()
    rgb, dep, acc = rgb.cpu().numpy(), dep.cpu().numpy(), acc.cpu().numpy()
    start = 0
    hit_scenes = 0
    for c, n in zip(cases, counts):
        sl = slice(start, start + n)
        er, ed, ea, st = c.oracle(o[sl], d[sl])
        hit_scenes += int(st.X.shape[0] > 0)
        assert_outputs_close(rgb[sl], er, 1.0, f"scene depth {c.depth} rgb")
        assert_outputs_close(dep[sl], ed, max(1.0, np.abs(ed).max()), f"scene depth {c.depth} depth")
        assert_outputs_close(acc[sl], ea, 1.0, f"scene depth {c.depth} acc")
        start += n
    assert hit_scenes >= 6


def test_multi_scene_graph_replay(gpu_lib):
    """Render + train step over all scenes captured once in a HIP graph and
    replayed three times, with eager work and synchronisations between the
    replays; every replay must reproduce the eager results (forward bit for
    bit; gradients up to FP32 atomic ordering)."""
    import torch
    m, cases, counts, o, d = _setup(gpu_lib)
    scenes = [c.scene for c in cases]
    params = cases[0].params
    opts = cases[0].opts("bf16")
    to, td = cases[0].rays(o, d)
    n = o.shape[0]
    rng = np.random.default_rng(0)
    t_rgb = torch.from_numpy(rng.uniform(0, 1, (n, 3)).astype(np.float32)).cuda()
    t_dep = torch.from_numpy(rng.uniform(0, 6, n).astype(np.float32)).cuda()
    out = (torch.empty((n, 3), device="cuda"), torch.empty(n, device="cuda"),
           torch.empty(n, device="cuda"))
    gFs = [torch.zeros_like(s.features) for s in scenes]
    gp = torch.zeros_like(params)
    loss = torch.zeros(1, device="cuda")
    ws = gpu_lib.Workspace()

    def work():
        gpu_lib.render(scenes, counts, params, m.widths, opts, to, td, *out, workspace=ws)
        for g in gFs + [gp]:
            gpu_lib.fill(g, 0.0)
        gpu_lib.train_step(scenes, counts, params, m.widths, opts, to, td, t_rgb, t_dep, 0.1,
                           1.0 / n, gFs, gp, loss_out=loss, workspace=ws)

    work()                                   # eager reference (also sizes the workspace)
    torch.cuda.synchronize()
    ref = [x.clone() for x in out] + [g.clone() for g in gFs] + [gp.clone(), loss.clone()]
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            work()
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    for rep in range(3):
        for x in out:
            x.fill_(-1.0)                    # eager work between replays
        for g in gFs + [gp]:
            g.fill_(123.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = [x for x in out] + gFs + [gp, loss]
        for k in range(3):
            assert torch.equal(got[k], ref[k]), (rep, k)
        for gg, rr in zip(got[3:], ref[3:]):
            np.testing.assert_allclose(gg.cpu().numpy(), rr.cpu().numpy(), rtol=1e-4,
                                       atol=1e-6 * float(rr.abs().max()) + 1e-30)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_multi_scene_interleaved_groups_match_per_scene_calls(gpu_lib, precision):
    """Scenes with full 65,536-ray groups (whose rays the shading kernels
    interleave), exact and ragged multiples and a small scene after them, in
    one call: per-ray outputs bit-exact and gradients (up to FP32 summation
    order) equal to calls made scene by scene."""
    import torch
    m = get_multi(small=True)
    p = m.params()
    p[-1] = 0.6
    counts = [70000, 65536, 131149, 513]
    cases, os_, ds_ = [], [], []
    for i, n_i in enumerate(counts):
        sc = m.scene(5 + i % 3)
        rng = np.random.default_rng(200 + i)
        F = rng.normal(0, 0.4, (sc.n_vertices, m.C)).astype(np.float32)
        cases.append(Case(gpu_lib, sc.leaf_ijk, sc.depth, F, p, m.widths, m.K))
        o, d = m.rays(5 + i % 3, n_i)
        os_.append(o)
        ds_.append(d)
    o, d = np.concatenate(os_), np.concatenate(ds_)
    n = o.shape[0]
    to, td = cases[0].rays(o, d)
    rng = np.random.default_rng(1)
    t_rgb = torch.from_numpy(rng.uniform(0, 1, (n, 3)).astype(np.float32)).cuda()
    t_dep = torch.from_numpy(rng.uniform(0, 6, n).astype(np.float32)).cuda()
    params = cases[0].params
    opts = cases[0].opts(precision)

    def run(groups):
        gFs = [torch.zeros_like(c.scene.features) for c in cases]
        gp = torch.zeros_like(params)
        rgb = torch.empty((n, 3), device="cuda")
        dep = torch.empty(n, device="cuda")
        for ids in groups:
            lo = sum(counts[:ids[0]])
            hi = lo + sum(counts[i] for i in ids)
            gpc = torch.zeros_like(gp)
            gpu_lib.train_step([cases[i].scene for i in ids], [counts[i] for i in ids], params, m.widths,
                               opts, to[lo:hi], td[lo:hi], t_rgb[lo:hi], t_dep[lo:hi], 0.1, 1.0 / n,
                               [gFs[i] for i in ids], gpc, out_rgb=rgb[lo:hi], out_depth=dep[lo:hi])
            gp += gpc
        torch.cuda.synchronize()
        return [g.cpu().numpy() for g in gFs], gp.cpu().numpy(), rgb.cpu().numpy(), dep.cpu().numpy()

    fa, pa, ra, da = run([list(range(len(counts)))])
    fb, pb, rb, db = run([[i] for i in range(len(counts))])
    assert np.array_equal(ra.view(np.int32), rb.view(np.int32))
    assert np.array_equal(da.view(np.int32), db.view(np.int32))
    for k, (ga, gb) in enumerate(zip(fa, fb)):
        s = np.abs(gb).max()
        assert (s > 0 or counts[k] < 65536) and np.abs(ga - gb).max() <= 1e-5 * s
    sp = np.abs(pb).max()
    assert sp > 0 and np.abs(pa - pb).max() <= 1e-4 * sp
