#!/usr/bin/env python
"""Benchmark of the SVLF per-ray path on one MI355X.

Workload (the paper-scale one): octree depth 9 (512^3), 40 rotated
ellipsoids + 20 boxes, surface cells scaled to ~1% occupancy, 32 features per
vertex (FP32 masters + BF16 copy), decoder 32-64-64-64-4, K = 8, 1600x1600
views, training batch 2^20 rays sampled from 50 views with analytic targets.

A timed step is one training pass over the batch: traversal, gather +
trilinear interpolation, decoder, Eq. 3 compositing, MSE + L1 loss and the
hand-written backward (svlf_train_step) with the BF16 decoder.  Also
reported: the same step with the FP32 decoder, the forward render of one
1600^2 view (BF16 and FP32), whole optimisation steps with dense and with
lazy (touched-row) Adam on the features, per-kernel
durations (HIP events on the launch stream) with the roofline of the
dominant kernel, PSNR of the BF16 render against the FP64 oracle on a seeded
ray sample, and the oracle itself timed on the host.

Prints one JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the BF16 train shading kernel on this workload,
# from rocprofv3 FETCH_SIZE / WRITE_SIZE passes scaled by a 1 GiB device copy
# (profiles/shade_train_bf16_paper_scale.md).  Valid only for the kernel
# sources they were taken with (shade.hip and the two headers it includes);
# reported as null once any of them changes.
MEASURED_TRAFFIC = {"shade_src_sha256_prefix": "34798313f0d274d1", "bytes": 2 * 445378 * 1024 + 1424017 * 1024}
SHADE_SOURCES = ("shade.hip", "mfma_common.hpp", "svlf_internal.hpp")


def shade_source_prefix():
    import hashlib
    h = hashlib.sha256()
    for name in SHADE_SOURCES:
        with open(os.path.join(ROOT, "paper_2205_07058_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def bench_lightfield(torch, svlf, timer, args, w, sc, ob_t, db_t, rgb_tt, dep_tt, ov_t, dv_t,
                     hits_b, hits_v):
    """The paper's two-decoder light-field function on the same scene and
    rays: train pass (BF16, FP32) and forward render of one view."""
    from synth.configs import lf_inputs
    F, p = lf_inputs(w.seed, sc.n_vertices)
    scene = svlf.DeviceScene.lf_from_host(sc.leaf_ijk, sc.depth, F, bf16=True)
    params = torch.from_numpy(p).cuda()
    n_b, n_v = ob_t.shape[0], ov_t.shape[0]
    gF = torch.zeros_like(scene.features)
    gp = torch.zeros_like(params)
    loss = torch.zeros(1, device="cuda")
    ws = svlf.Workspace()
    out = {"model": "density 134-128-2, colour 38-128-128-128-3, features 64+32 per vertex, tau direct"}
    for prec in ("bf16", "fp32"):
        opts = svlf.make_opts(w.K, "direct", prec)
        f = lambda: svlf.lf_train_step([scene], [n_b], params, opts, ob_t, db_t, rgb_tt, dep_tt,
                                       0.1, 1.0 / n_b, [gF], gp, loss_out=loss, workspace=ws)
        ms, _ = timer.run(f, args.steps, args.warmup)
        out[f"train_{prec}_ms"] = round(ms / args.steps, 4)
        out[f"train_{prec}_rays_per_s"] = round(n_b * args.steps / ms * 1e3, 1)
        log(f"light field train step {prec}: {ms / args.steps:.3f} ms/step, "
            f"{n_b * args.steps / ms * 1e3 / 1e6:.1f} M rays/s, loss {loss.item():.5f}")
        opts = svlf.make_opts(w.K, "direct", prec)
        bufs = (torch.empty((n_v, 3), device="cuda"), torch.empty(n_v, device="cuda"),
                torch.empty(n_v, device="cuda"))
        f = lambda: svlf.lf_render([scene], [n_v], params, opts, ov_t, dv_t, *bufs, workspace=ws)
        ms, _ = timer.run(f, args.steps, args.warmup)
        out[f"fwd_view_{prec}_ms"] = round(ms / args.steps, 4)
        out[f"fwd_view_{prec}_rays_per_s"] = round(n_v * args.steps / ms * 1e3, 1)
        log(f"light field forward view {prec}: {ms / args.steps:.3f} ms/view, "
            f"{n_v * args.steps / ms * 1e3 / 1e6:.1f} M rays/s")
    # MACs per hit: density 134*128 + 128*2, colour 38*128 + 2*128*128 + 128*3
    macs = 134 * 128 + 128 * 2 + 38 * 128 + 2 * 128 * 128 + 128 * 3
    out["macs_per_hit_forward"] = macs
    out["decoder_tflops_fwd_view_bf16"] = round(2 * macs * hits_v / (out["fwd_view_bf16_ms"] * 1e-3) / 1e12, 2)
    del scene, gF
    return out


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rays", type=int, default=1 << 17,
                    help="rays of the batch the oracle trains on for the CPU baseline")
    ap.add_argument("--psnr-rays", type=int, default=16384)
    ap.add_argument("--sections", default="all",
                    help="comma list of: train_bf16,train_fp32,fwd_bf16,fwd_fp32,adam,stages,psnr,lf,occ,det,copy,"
                         "multi (the ragged 8-scene workload; not in 'all')")
    return ap.parse_args()


class Timer:
    """HIP events on torch's current stream (the stream every libsvlf call is
    queued on)."""

    def __init__(self, torch):
        self.torch = torch

    def run(self, fn, steps, warmup):
        torch = self.torch
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record()
        for i in range(steps):
            fn()
            ev[i + 1].record()
        torch.cuda.synchronize()
        per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
        return float(np.sum(per)), per


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        sys.exit("bench.py measures one GPU only: this build has no multi-GPU path "
                 "(the sharding design is described in DESIGN.md); run with --gpus 1")
    import torch

    from paper_2205_07058_amd import svlf
    from synth.configs import get_config

    sections = set(args.sections.split(",")) if args.sections != "all" else {
        "train_bf16", "train_fp32", "fwd_bf16", "fwd_fp32", "adam", "stages", "psnr", "lf", "occ", "det"}
    torch.cuda.set_device(0)
    svlf.load()
    t0 = time.time()
    w = get_config(3)
    sc = w.scene()
    log(f"scene: depth {sc.depth}, {sc.leaf_ijk.shape[0]} leaves ({100 * sc.fraction:.2f}%), "
        f"{sc.n_vertices} vertices ({time.time() - t0:.1f}s)")
    F = w.features()
    p = w.params()
    scene = svlf.DeviceScene.from_host(sc.leaf_ijk, sc.depth, F, bf16=True)
    params = torch.from_numpy(p).cuda()
    log(f"octree on device: {scene.octree.n_nodes} internal nodes")
    ob, db, rgb_t, dep_t = w.train_batch(w.batch, step=0)
    o_v, d_v = w.view_rays(0)
    log(f"inputs ready: batch {ob.shape[0]} rays, view {o_v.shape[0]} rays ({time.time() - t0:.1f}s)")
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    ob_t, db_t, rgb_tt, dep_tt = T(ob), T(db), T(rgb_t), T(dep_t)
    ov_t, dv_t = T(o_v), T(d_v)
    n_b, n_v = ob.shape[0], o_v.shape[0]
    gF = torch.zeros_like(scene.features)
    gp = torch.zeros_like(params)
    loss = torch.zeros(1, device="cuda")
    ws = svlf.Workspace()
    timer = Timer(torch)
    res = {}

    # hits per ray of both ray sets (for the algorithmic byte counts)
    _, _, _, cnt_b = svlf.trace_hits(scene.octree, ob_t, db_t, w.K)
    _, _, _, cnt_v = svlf.trace_hits(scene.octree, ov_t, dv_t, w.K)
    hits_b = int(cnt_b.sum().item())
    hits_v = int(cnt_v.sum().item())
    log(f"hits: batch {hits_b} ({hits_b / n_b:.3f}/ray), view {hits_v} ({hits_v / n_v:.3f}/ray)")

    def train_fn(prec, flags=0):
        opts = svlf.make_opts(w.K, "voxel", prec, flags)
        return lambda: svlf.train_step([scene], [n_b], params, w.widths, opts, ob_t, db_t, rgb_tt,
                                       dep_tt, 0.1, 1.0 / n_b, [gF], gp, loss_out=loss, workspace=ws)

    def fwd_fn(prec):
        opts = svlf.make_opts(w.K, "voxel", prec)
        out = (torch.empty((n_v, 3), device="cuda"), torch.empty(n_v, device="cuda"),
               torch.empty(n_v, device="cuda"))
        return lambda: svlf.render([scene], [n_v], params, w.widths, opts, ov_t, dv_t, *out, workspace=ws)

    for prec in ("bf16", "fp32"):
        if f"train_{prec}" in sections:
            ms, _ = timer.run(train_fn(prec), args.steps, args.warmup)
            res[f"train_{prec}_ms"] = ms / args.steps
            log(f"train step {prec}: {ms / args.steps:.3f} ms/step, "
                f"{n_b * args.steps / ms * 1e3 / 1e6:.1f} M rays/s, loss {loss.item():.5f}")
        if f"fwd_{prec}" in sections:
            ms, _ = timer.run(fwd_fn(prec), args.steps, args.warmup)
            res[f"fwd_{prec}_ms"] = ms / args.steps
            log(f"forward view {prec}: {ms / args.steps:.3f} ms/view, "
                f"{n_v * args.steps / ms * 1e3 / 1e6:.1f} M rays/s")

    if "adam" in sections:
        # whole optimisation steps: the BF16 train pass, then Adam on the
        # features (dense, or lazy over the touched rows) refreshing their
        # BF16 copy, and dense Adam on the decoder parameters
        m = torch.zeros_like(scene.features)
        v = torch.zeros_like(scene.features)
        mp, vp = torch.zeros_like(params), torch.zeros_like(params)
        st = [0]
        tr = train_fn("bf16")
        F_keep = scene.features.clone()
        p_keep = params.clone()

        def step_with(lazy):
            def fn():
                st[0] += 1
                tr()
                upd = svlf.lazy_adam_step if lazy else svlf.adam_step
                upd(scene.features, gF, m, v, 1e-3, 0.9, 0.999, 1e-8, st[0],
                    bf16_out=scene.features_bf16, zero_grad=True)
                svlf.adam_step(params, gp, mp, vp, 1e-3, 0.9, 0.999, 1e-8, st[0], zero_grad=True)
            return fn
        for lazy in (False, True):
            ms, _ = timer.run(step_with(lazy), args.steps, args.warmup)
            key = "lazy" if lazy else "dense"
            res[f"step_{key}_adam_ms"] = ms / args.steps
            log(f"train step + {key} Adam: {ms / args.steps:.3f} ms/step")
            scene.features.copy_(F_keep)
            params.copy_(p_keep)
            scene.refresh_bf16()
            m.zero_(), v.zero_(), mp.zero_(), vp.zero_(), gF.zero_(), gp.zero_()
            st[0] = 0
        tr()
        res["touched_rows"] = float((gF != 0).any(dim=1).float().mean().item())
        gF.zero_(), gp.zero_()
        log(f"feature rows touched by one batch: {100 * res['touched_rows']:.1f}%")

    if "lf" in sections:
        res["lightfield"] = bench_lightfield(torch, svlf, timer, args, w, sc, ob_t, db_t, rgb_tt,
                                             dep_tt, ov_t, dv_t, hits_b, hits_v)

    if "occ" in sections:
        # occupied leaves from the depth map of one view (section 4.1)
        _, dep_v = w.targets(o_v, d_v)
        dep_vt = T(dep_v)
        f = lambda: svlf.occupancy_from_depth(ov_t, dv_t, dep_vt, sc.depth)
        ms, _ = timer.run(f, args.steps, args.warmup)
        n_leaf = int(f().shape[0])
        res["occupancy"] = {"ms_per_view": round(ms / args.steps, 4),
                            "rays_per_s": round(n_v * args.steps / ms * 1e3, 1),
                            "leaves": n_leaf, "level": sc.depth}
        log(f"occupancy from one depth map: {ms / args.steps:.3f} ms, {n_leaf} leaves")

    if "copy" in sections:
        # a plain device copy of known size: calibrates the HBM byte counters
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        ms, _ = timer.run(lambda: dst.copy_(src), args.steps, args.warmup)
        res["copy_gbs"] = 2 * src.numel() * 4 / (ms / args.steps * 1e-3) / 1e9
        log(f"device copy of 1 GiB: {ms / args.steps:.3f} ms ({res['copy_gbs']:.0f} GB/s read+write)")
        del src, dst

    multi = None
    if "multi" in sections:
        multi = bench_multi(torch, svlf, timer, args)

    if "det" in sections:
        # the same BF16 train step with the deterministic feature-gradient reduction
        ms, _ = timer.run(train_fn("bf16", svlf.FLAG_DETERMINISTIC), args.steps, args.warmup)
        res["train_bf16_det_ms"] = ms / args.steps
        log(f"train step bf16, deterministic feature gradient: {ms / args.steps:.3f} ms/step, "
            f"{n_b * args.steps / ms * 1e3 / 1e6:.1f} M rays/s")

    stages = {}
    if "stages" in sections:
        # split one BF16 train step into its kernels with events between them
        trace = train_fn("bf16", svlf.FLAG_TRACE_ONLY)
        shade = train_fn("bf16", svlf.FLAG_REUSE_HITS)
        trace()
        ms_tr, _ = timer.run(trace, args.steps, args.warmup)
        ms_sh, _ = timer.run(shade, args.steps, args.warmup)
        stages = {"trace_ms": ms_tr / args.steps, "shade_reduce_ms": ms_sh / args.steps}
        log(f"stages (bf16 train): trace {stages['trace_ms']:.3f} ms, "
            f"shade+reduce {stages['shade_reduce_ms']:.3f} ms")

    psnr = None
    if "psnr" in sections:
        from oracle.octree import Octree
        from oracle.render import render as oracle_render
        from oracle.trace import trace_hits as oracle_trace
        rgb16 = torch.empty((n_v, 3), device="cuda")
        svlf.render([scene], [n_v], params, w.widths, svlf.make_opts(w.K, "voxel", "bf16"), ov_t, dv_t,
                    rgb16, torch.empty(n_v, device="cuda"), torch.empty(n_v, device="cuda"), workspace=ws)
        torch.cuda.synchronize()
        rng = np.random.default_rng(2022)
        idx = np.sort(rng.choice(n_v, args.psnr_rays, replace=False))
        t1 = time.time()
        oc = Octree(sc.leaf_ijk, sc.depth)
        log(f"oracle octree built ({time.time() - t1:.1f}s)")
        hits = oracle_trace(oc, o_v[idx], d_v[idx], w.K)
        er, _, _, _ = oracle_render(oc, F, p, w.widths, o_v[idx], d_v[idx], hits)
        got = rgb16.cpu().numpy()[idx]
        mse = float(np.mean((got.astype(np.float64) - er) ** 2))
        psnr = float("inf") if mse == 0 else -10.0 * np.log10(mse)
        log(f"PSNR bf16 render vs FP64 oracle on {args.psnr_rays} rays: {psnr:.2f} dB")
        res["oracle_octree"] = oc

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, sc, F, p, ob, db, rgb_t, dep_t, args.cpu_rays, res.get("oracle_octree"))

    # roofline of the dominant kernel (the fused shading kernel of the BF16
    # train step): algorithmic bytes per launch over its event-timed duration
    C = w.C
    n_params = p.size
    grid = 256                                    # one block per CU for the BF16 train kernel
    bytes_ray = 24 + 4 + 16                      # o, d, hit count, targets
    bytes_hit = 16 + 32 + 8 * C * 2 + 8 * C * 4 * 2   # hit record, corners, BF16 rows, FP32 grad RMW
    bytes_launch = n_b * bytes_ray + hits_b * bytes_hit + grid * n_params * 4
    roof = None
    if stages:
        sh_ms = stages["shade_reduce_ms"]
        achieved = bytes_launch / (sh_ms * 1e-3) / 1e9
        traffic = (MEASURED_TRAFFIC["bytes"] if shade_source_prefix() == MEASURED_TRAFFIC["shade_src_sha256_prefix"]
                   else None)
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_unit": "bytes per launch (FETCH_SIZE x2.0 + WRITE_SIZE x1.0, copy-calibrated)",
                "kernel": "k_shade<bf16,32,64,3,train> + k_reduce",
                "bytes_per_launch": int(bytes_launch),
                "bytes_per_hit": bytes_hit, "bytes_per_ray": bytes_ray, "hits_per_ray": round(hits_b / n_b, 4)}

    ms = res.get("train_bf16_ms")
    value = n_b / (ms * 1e-3) if ms else None
    out = {
        "metric": "rays/sec train step @1600^2 workload (BF16 decoder on MFMA); fwd render, FP32 path and PSNR vs FP64 oracle alongside",
        "value": round(value, 1) if value else None,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4) if ms else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic (seeded analytic scene and targets standing in for RTMV)",
        "config": {"workload": "depth-9 octree (512^3), 40 ellipsoids + 20 boxes, ~1% surface leaves, "
                               "C=32, MLP 32-64-64-64-4, K=8, batch 2^20 rays from 50 1600^2 views",
                   "batch": n_b, "view_rays": n_v, "leaves": int(sc.leaf_ijk.shape[0]),
                   "vertices": int(sc.n_vertices), "hits_per_ray_batch": round(hits_b / n_b, 4),
                   "hits_per_ray_view": round(hits_v / n_v, 4)},
        "step": "traversal + gather + decoder + Eq. 3 + loss + backward (svlf_train_step); optimiser steps reported separately",
        "train_fp32_rays_per_s": round(n_b / (res["train_fp32_ms"] * 1e-3), 1) if "train_fp32_ms" in res else None,
        "fwd_view_bf16_rays_per_s": round(n_v / (res["fwd_bf16_ms"] * 1e-3), 1) if "fwd_bf16_ms" in res else None,
        "fwd_view_fp32_rays_per_s": round(n_v / (res["fwd_fp32_ms"] * 1e-3), 1) if "fwd_fp32_ms" in res else None,
        "train_bf16_with_dense_adam_rays_per_s": round(n_b / (res["step_dense_adam_ms"] * 1e-3), 1)
        if "step_dense_adam_ms" in res else None,
        "train_bf16_with_lazy_adam_rays_per_s": round(n_b / (res["step_lazy_adam_ms"] * 1e-3), 1)
        if "step_lazy_adam_ms" in res else None,
        "feature_rows_touched_per_batch": round(res["touched_rows"], 4) if "touched_rows" in res else None,
        "lightfield": res.get("lightfield"),
        "occupancy_from_depth": res.get("occupancy"),
        "train_bf16_deterministic_rays_per_s": round(n_b / (res["train_bf16_det_ms"] * 1e-3), 1)
        if "train_bf16_det_ms" in res else None,
        "stages_ms": {k: round(v, 4) for k, v in stages.items()} or None,
        "psnr_bf16_render_vs_fp64_oracle_db": round(psnr, 3) if psnr is not None else None,
        "device_copy_gbs": round(res["copy_gbs"], 1) if "copy_gbs" in res else None,
        "multi_scene": multi,
        "roofline": roof,
        "cpu_baseline": cpu,
        "paper_context": "SVLF renders 0.08 s/frame on one RTX 3090 and trains 30K steps in 2.7 h on one V100 (Table 6)",
    }
    print(json.dumps(out), flush=True)


def bench_multi(torch, svlf, timer, args):
    """Ragged workload: 8 scenes (depths 7..10, 0.5-3% occupancy) sharing one
    BF16 decoder, 2^16..2^20 rays each, rendered and trained in one launch of
    each kernel; also captured once in a HIP graph and replayed.  Features
    are drawn on the device from a seeded generator."""
    from synth.configs import get_multi
    m = get_multi()
    counts = m.ray_counts()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4)
    scenes, os_, ds_ = [], [], []
    t0 = time.time()
    leaves = []
    for i in range(len(m.depths)):
        sc = m.scene(i)
        oc = svlf.DeviceOctree(sc.leaf_ijk, sc.depth)
        feats = torch.randn((sc.n_vertices, m.C), generator=gen, device="cuda") * 0.1
        ds = svlf.DeviceScene(oc, feats)
        ds.refresh_bf16()
        scenes.append(ds)
        leaves.append(int(sc.leaf_ijk.shape[0]))
        o, d = m.rays(i, counts[i])
        os_.append(o)
        ds_.append(d)
        log(f"multi scene {i}: depth {m.depths[i]}, {leaves[-1]} leaves, {counts[i]} rays ({time.time() - t0:.1f}s)")
    n = sum(counts)
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    o_t, d_t = T(np.concatenate(os_)), T(np.concatenate(ds_))
    params = torch.from_numpy(m.params()).cuda()
    opts = svlf.make_opts(m.K, "voxel", "bf16")
    ws = svlf.Workspace()
    out = (torch.empty((n, 3), device="cuda"), torch.empty(n, device="cuda"), torch.empty(n, device="cuda"))
    rng = np.random.default_rng(5)
    t_rgb, t_dep = T(rng.uniform(0, 1, (n, 3)).astype(np.float32)), T(rng.uniform(0, 6, n).astype(np.float32))
    gFs = [torch.zeros_like(s.features) for s in scenes]
    gp = torch.zeros_like(params)
    loss = torch.zeros(1, device="cuda")
    fwd = lambda: svlf.render(scenes, counts, params, m.widths, opts, o_t, d_t, *out, workspace=ws)
    trn = lambda: svlf.train_step(scenes, counts, params, m.widths, opts, o_t, d_t, t_rgb, t_dep, 0.1,
                                  1.0 / n, gFs, gp, loss_out=loss, workspace=ws)
    ms_f, _ = timer.run(fwd, args.steps, args.warmup)
    ms_t, _ = timer.run(trn, args.steps, args.warmup)
    graph = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        with torch.cuda.graph(graph, stream=st):
            trn()
    torch.cuda.current_stream().wait_stream(st)
    ms_g, _ = timer.run(graph.replay, args.steps, args.warmup)
    res = {"workload": "8 scenes, depths " + ",".join(map(str, m.depths)) + ", C=32, MLP 32-64-64-64-4, K=8",
           "leaves": leaves, "rays": counts, "total_rays": n,
           "fwd_bf16_rays_per_s": round(n / (ms_f / args.steps * 1e-3), 1),
           "train_bf16_rays_per_s": round(n / (ms_t / args.steps * 1e-3), 1),
           "train_bf16_graph_replay_rays_per_s": round(n / (ms_g / args.steps * 1e-3), 1)}
    log(f"multi: fwd {res['fwd_bf16_rays_per_s'] / 1e6:.1f} M rays/s, train {res['train_bf16_rays_per_s'] / 1e6:.1f} "
        f"M rays/s, graph replay {res['train_bf16_graph_replay_rays_per_s'] / 1e6:.1f} M rays/s")
    return res


def cpu_baseline(w, sc, F, p, ob, db, rgb_t, dep_t, n_rays, oc=None):
    """The FP64 oracle (trace + render + loss + hand-written backward) on a
    seeded sample of the training batch, timed on the host."""
    from oracle.octree import Octree
    from oracle.render import loss as oracle_loss, render as oracle_render, render_backward
    from oracle.trace import trace_hits as oracle_trace
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = 1
    if oc is None:
        t1 = time.time()
        oc = Octree(sc.leaf_ijk, sc.depth)
        log(f"oracle octree built ({time.time() - t1:.1f}s)")
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(ob.shape[0], n_rays, replace=False))
    o, d = ob[idx], db[idx]
    t0 = time.time()
    hits = oracle_trace(oc, o, d, w.K)
    rgb, dep, acc, st = oracle_render(oc, F, p, w.widths, o, d, hits)
    L, g_rgb, g_dep = oracle_loss(rgb, dep, rgb_t[idx], dep_t[idx])
    gF, gp = render_backward(st, g_rgb, g_dep)
    dt = time.time() - t0
    log(f"oracle train pass on {n_rays} rays: {dt:.2f}s ({n_rays / dt:.0f} rays/s, {threads} threads)")
    return {"value": round(n_rays / dt, 2), "unit": "rays/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n_rays} seeded rays of the 2^20-ray batch: FP64 oracle trace + render + loss + "
                      f"backward, single process (numpy, BLAS threads = {threads}); octree build excluded"}


if __name__ == "__main__":
    main()
