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
lazy (touched-row) Adam on the features, per-kernel durations (HIP events on
the launch stream) with the roofline of the dominant kernel against the HBM
peak and against the bandwidth of a plain device copy; the other workloads
(the depth-4 shell and the depth-7 ellipsoid views forward, the depth-7
2^18-ray training batch, the ragged batch of 8 scenes of depths 7-10 in one
launch and from a HIP graph); the light-field function; PSNR of the BF16
and FP32 renders of a trained network against the FP64 oracle, and the
held-out PSNR of BF16- and FP32-trained networks; the oracle itself timed on
the host cores (a process pool in a child process).

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
MEASURED_TRAFFIC = {"shade_src_sha256_prefix": "38c71d7939761e02", "bytes": 2 * 454353 * 1024 + 1424041 * 1024}
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
                    help="comma list of: " + ",".join(ALL_SECTIONS))
    ap.add_argument("--train-steps", type=int, default=200,
                    help="optimisation steps of the networks whose PSNR is reported")
    ap.add_argument("--cpu-child", default=None, help=argparse.SUPPRESS)
    return ap.parse_args()


ALL_SECTIONS = ("train_bf16", "train_fp32", "fwd_bf16", "fwd_fp32", "copy", "stages", "adam", "lf", "occ",
                "det", "small", "multi", "psnr")


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
    if args.cpu_child:
        return cpu_child(args.cpu_child)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        sys.exit("bench.py measures one GPU only: the library has no multi-GPU path; "
                 "run with --gpus 1")
    import torch

    from paper_2205_07058_amd import svlf
    from synth.configs import get_workload

    sections = set(args.sections.split(",")) if args.sections != "all" else set(ALL_SECTIONS)
    torch.cuda.set_device(0)
    svlf.load()
    t0 = time.time()
    w = get_workload("surfaces_d9")
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

    small = bench_small(torch, svlf, timer, args) if "small" in sections else None

    psnr = bench_psnr(torch, svlf, args, w, sc, F, p, ob_t, db_t, rgb_tt, dep_tt) if "psnr" in sections else None

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, ob, db, rgb_t, dep_t)

    # roofline of the dominant kernel (the fused shading kernel of the BF16
    # train step): algorithmic bytes per launch over its event-timed duration.
    # The algorithmic count of a training pass: per ray its origin and
    # direction, outputs, targets and output gradients (24 + 16 + 16 + 16 B);
    # per hit the gather of the corner ids and 8 BF16 feature rows in the
    # forward and again in the backward, the FP32 gradient read-modify-write
    # of the 8 rows, and the hit list written by the forward and read by the
    # backward (24 B per slot, K slots per ray, over the hits per ray); plus
    # the per-block decoder-gradient partials.  The fused kernel gathers once
    # and keeps the hit list on chip; its own count is reported beside it.
    C = w.C
    K = w.K
    n_params = p.size
    grid = 256                                    # one block per CU for the BF16 train kernel
    hbar = hits_b / n_b
    b_gather = 32 + 8 * C * 2
    bytes_ray = 24 + 16 + 16 + 16
    bytes_hit = 2 * b_gather + 8 * C * 4 * 2 + 24 * K / hbar
    bytes_launch = n_b * bytes_ray + hits_b * bytes_hit + grid * n_params * 4
    fused_ray = 24 + 4 + 16                       # o, d, hit count, targets
    fused_hit = 16 + b_gather + 8 * C * 4 * 2     # hit record, one gather, gradient RMW
    fused_launch = n_b * fused_ray + hits_b * fused_hit + grid * n_params * 4
    roof = None
    if stages:
        sh_ms = stages["shade_reduce_ms"]
        achieved = bytes_launch / (sh_ms * 1e-3) / 1e9
        traffic = (MEASURED_TRAFFIC["bytes"] if shade_source_prefix() == MEASURED_TRAFFIC["shade_src_sha256_prefix"]
                   else None)
        copy = res.get("copy_gbs")
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "achievable_copy_gbs": round(copy, 1) if copy else None,
                "frac_of_copy": round(achieved / copy, 4) if copy else None,
                "traffic_unit": "bytes per launch (FETCH_SIZE x2.0 + WRITE_SIZE x1.0, copy-calibrated)",
                "kernel": "k_shade<bf16,32,64,3,train> + k_reduce",
                "bytes_per_launch": int(bytes_launch),
                "bytes_per_hit": round(bytes_hit, 1), "bytes_per_ray": bytes_ray, "hits_per_ray": round(hbar, 4),
                "fused_kernel_bytes_per_launch": int(fused_launch), "fused_kernel_bytes_per_hit": fused_hit,
                "fused_kernel_frac": round(fused_launch / (sh_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

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
        "psnr_bf16_render_vs_fp64_oracle_db": psnr["bf16_render_vs_fp64_oracle_db"] if psnr else None,
        "psnr": psnr,
        "device_copy_gbs": round(res["copy_gbs"], 1) if "copy_gbs" in res else None,
        "other_workloads": small,
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


def bench_small(torch, svlf, timer, args):
    """The workloads that fit in cache: forward views of the depth-4 shell
    (64x64, K = 4, decoder 8-32-32-4) and of the depth-7 twelve-ellipsoid
    scene (800x800, K = 8, decoder 16-64-64-64-4), and the training pass on
    the depth-7 scene with a 2^18-ray batch from 50 views (FP32, the
    workload's precision, and BF16)."""
    from synth.configs import get_workload
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    out = {}
    ws = svlf.Workspace()
    for name in ("shell_d4", "ellipsoids_d7"):
        w = get_workload(name)
        sc = w.scene()
        scene = svlf.DeviceScene.from_host(sc.leaf_ijk, sc.depth, w.features(), bf16=True)
        params = T(w.params())
        o, d = w.view_rays(0)
        n = o.shape[0]
        ot, dt = T(o), T(d)
        bufs = (torch.empty((n, 3), device="cuda"), torch.empty(n, device="cuda"), torch.empty(n, device="cuda"))
        _, _, _, cnt = svlf.trace_hits(scene.octree, ot, dt, w.K)
        r = {"workload": w.description, "rays": n, "leaves": int(sc.leaf_ijk.shape[0]),
             "hits_per_ray": round(float(cnt.sum().item()) / n, 4)}
        for prec in ("fp32", "bf16"):
            opts = svlf.make_opts(w.K, "voxel", prec)
            ms, _ = timer.run(lambda: svlf.render([scene], [n], params, w.widths, opts, ot, dt, *bufs,
                                                  workspace=ws), args.steps, args.warmup)
            r[f"fwd_{prec}_ms"] = round(ms / args.steps, 4)
            r[f"fwd_{prec}_rays_per_s"] = round(n / (ms / args.steps * 1e-3), 1)
        log(f"{name} forward: fp32 {r['fwd_fp32_rays_per_s'] / 1e6:.1f} M rays/s, "
            f"bf16 {r['fwd_bf16_rays_per_s'] / 1e6:.1f} M rays/s ({n} rays)")
        out[name] = r
    w = get_workload("ellipsoids_d7_train")
    sc = w.scene()
    scene = svlf.DeviceScene.from_host(sc.leaf_ijk, sc.depth, w.features(), bf16=True)
    params = T(w.params())
    ob, db, rgb_t, dep_t = w.train_batch(w.batch, step=0)
    n = ob.shape[0]
    args_t = [T(ob), T(db), T(rgb_t), T(dep_t)]
    gF = torch.zeros_like(scene.features)
    gp = torch.zeros_like(params)
    loss = torch.zeros(1, device="cuda")
    r = {"workload": w.description, "rays": n}
    for prec in ("fp32", "bf16"):
        opts = svlf.make_opts(w.K, "voxel", prec)
        ms, _ = timer.run(lambda: svlf.train_step([scene], [n], params, w.widths, opts, *args_t, 0.1, 1.0 / n,
                                                  [gF], gp, loss_out=loss, workspace=ws),
                          args.steps, args.warmup)
        r[f"train_{prec}_ms"] = round(ms / args.steps, 4)
        r[f"train_{prec}_rays_per_s"] = round(n / (ms / args.steps * 1e-3), 1)
    log(f"ellipsoids_d7_train step: fp32 {r['train_fp32_rays_per_s'] / 1e6:.1f} M rays/s, "
        f"bf16 {r['train_bf16_rays_per_s'] / 1e6:.1f} M rays/s")
    out["ellipsoids_d7_train"] = r
    return out


def bench_psnr(torch, svlf, args, w, sc, F, p, ob_t, db_t, rgb_tt, dep_tt):
    """Networks trained on the batch (args.train_steps steps of the train
    pass + Adam, features at lr 1e-2, decoder at 1e-3) from the same initial
    values with the BF16 and with the FP32 decoder.  Reported: PSNR of the
    BF16-trained network's BF16 render (and of its FP32 render) against the
    FP64 oracle on 16,384 seeded rays of a view, the mean opacity of those
    rays that hit the scene, and the held-out PSNR (against the analytic
    targets, 2^16 seeded pixels of a held-out view) of both trained
    networks."""
    from oracle.octree import Octree
    from oracle.render import render as oracle_render
    from oracle.trace import trace_hits as oracle_trace
    from paper_2205_07058_amd.train import Trainer
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    hv = w.heldout_views()[0]
    oh, dh = w.view_rays(hv)
    sel = np.sort(np.random.default_rng(hv).choice(oh.shape[0], 1 << 16, replace=False))
    oh, dh = oh[sel], dh[sel]
    th, _ = w.targets(oh, dh)
    oht, dht = T(oh), T(dh)
    trained = {}
    t0 = time.time()
    for prec in ("bf16", "fp32"):
        scene = svlf.DeviceScene.from_host(sc.leaf_ijk, sc.depth, F, bf16=True)
        tr = Trainer(scene, T(p.copy()), w.widths, w.K, precision=prec, lr_features=1e-2, lr_params=1e-3)
        for _ in range(args.train_steps):
            tr.step(ob_t, db_t, rgb_tt, dep_tt)
        rgb, _, _ = tr.render(oht, dht)
        torch.cuda.synchronize()
        mse = float(np.mean((rgb.cpu().numpy().astype(np.float64) - th) ** 2))
        trained[prec] = (tr, -10.0 * np.log10(mse), float(tr.loss.item()))
    log(f"trained {args.train_steps} steps per precision ({time.time() - t0:.1f}s): held-out PSNR "
        f"bf16 {trained['bf16'][1]:.3f} dB, fp32 {trained['fp32'][1]:.3f} dB")
    tr = trained["bf16"][0]
    o_v, d_v = w.view_rays(0)
    idx = np.sort(np.random.default_rng(2022).choice(o_v.shape[0], args.psnr_rays, replace=False))
    ot, dt = T(o_v[idx]), T(d_v[idx])
    outs = {}
    for prec in ("bf16", "fp32"):
        rgb, _, acc = svlf.render([tr.scene], [idx.size], tr.params, w.widths, svlf.make_opts(w.K, "voxel", prec),
                                  ot, dt)
        torch.cuda.synchronize()
        outs[prec] = (rgb.cpu().numpy(), acc.cpu().numpy())
    Ft = tr.scene.features.cpu().numpy()
    pt = tr.params.cpu().numpy()
    t1 = time.time()
    oc = Octree(sc.leaf_ijk, sc.depth)
    hits = oracle_trace(oc, o_v[idx], d_v[idx], w.K)
    er, _, ea, _ = oracle_render(oc, Ft, pt, w.widths, o_v[idx], d_v[idx], hits)
    log(f"oracle render of the trained network on {idx.size} rays ({time.time() - t1:.1f}s)")
    ps = {}
    for prec in ("bf16", "fp32"):
        mse = float(np.mean((outs[prec][0].astype(np.float64) - er) ** 2))
        ps[prec] = float("inf") if mse == 0 else -10.0 * np.log10(mse)
    hit = hits[3] > 0
    res = {"steps": args.train_steps,
           "bf16_render_vs_fp64_oracle_db": round(ps["bf16"], 3),
           "fp32_render_vs_fp64_oracle_db": round(ps["fp32"], 3),
           "rays": int(idx.size), "mean_acc_of_hit_rays": round(float(ea[hit].mean()), 4),
           "rms_rgb": round(float(np.sqrt(np.mean(er ** 2))), 4),
           "heldout_psnr_bf16_trained_db": round(trained["bf16"][1], 3),
           "heldout_psnr_fp32_trained_db": round(trained["fp32"][1], 3),
           "heldout_gap_fp32_minus_bf16_db": round(trained["fp32"][1] - trained["bf16"][1], 3),
           "final_loss_bf16": round(trained["bf16"][2], 6), "final_loss_fp32": round(trained["fp32"][2], 6)}
    log(f"trained network: BF16 render vs FP64 oracle {ps['bf16']:.2f} dB, FP32 render {ps['fp32']:.2f} dB, "
        f"mean opacity of hit rays {res['mean_acc_of_hit_rays']:.3f}")
    return res


def _cpu_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def cpu_baseline(args, ob, db, rgb_t, dep_t):
    """The FP64 oracle timed on the host: run in a child process (started
    before it touches anything but numpy, with one BLAS thread per process)
    that spreads the work over a process pool on the usable host cores."""
    import subprocess
    import tempfile
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(ob.shape[0], args.cpu_rays, replace=False))
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "sample.npz")
        np.savez(path, o=ob[idx], d=db[idx], rgb_t=rgb_t[idx], dep_t=dep_t[idx])
        env = dict(os.environ)
        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            env[k] = "1"
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-child", path], env=env,
                           capture_output=True, text=True)
    sys.stderr.write(r.stderr)
    if r.returncode != 0:
        log(f"oracle timing failed (exit {r.returncode})")
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


_G = {}


def _oracle_chunk(job):
    """One chunk of the oracle work in a pool process (state inherited)."""
    from oracle.render import loss as oracle_loss, render as oracle_render, render_backward
    from oracle.trace import trace_hits as oracle_trace
    kind, lo, hi = job
    g = _G[kind]
    o, d = g["o"][lo:hi], g["d"][lo:hi]
    hits = oracle_trace(g["oc"], o, d, g["K"])
    rgb, dep, acc, st = oracle_render(g["oc"], g["F"], g["p"], g["widths"], o, d, hits)
    if kind != "train":
        return None
    _, g_rgb, g_dep = oracle_loss(rgb, dep, g["rgb_t"][lo:hi], g["dep_t"][lo:hi])
    gF, gp = render_backward(st, g_rgb, g_dep)
    rows = np.unique(st.corners.ravel())
    return rows, gF[rows], gp


def cpu_child(path):
    """Child-process half of cpu_baseline: prints one JSON line."""
    import multiprocessing as mp
    from oracle.octree import Octree
    from synth.configs import get_workload
    z = np.load(path)
    o, d, rgb_t, dep_t = z["o"], z["d"], z["rgb_t"], z["dep_t"]
    n = o.shape[0]
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        usable = os.cpu_count() or 1
    P = max(1, min(usable, 16))
    t0 = time.time()
    w = get_workload("surfaces_d9")
    sc = w.scene()
    F = w.features().astype(np.float64)
    _G["train"] = dict(o=o, d=d, rgb_t=rgb_t, dep_t=dep_t, oc=Octree(sc.leaf_ijk, sc.depth), F=F, p=w.params(),
                       widths=w.widths, K=w.K)
    fw = {}
    for name in ("shell_d4", "ellipsoids_d7"):
        wi = get_workload(name)
        sci = wi.scene()
        oi, di = wi.view_rays(0)
        _G[f"fwd_{name}"] = dict(o=oi, d=di, oc=Octree(sci.leaf_ijk, sci.depth), F=wi.features(),
                                 p=wi.params(), widths=wi.widths, K=wi.K)
        fw[name] = oi.shape[0]
    ov, dv = w.view_rays(0)
    sel = np.sort(np.random.default_rng(3).choice(ov.shape[0], 1 << 14, replace=False))
    _G["fwd_surfaces_d9"] = dict(_G["train"], o=ov[sel], d=dv[sel])
    log(f"oracle set-up ({time.time() - t0:.1f}s); {P} worker processes ({usable} usable cores)")

    def chunks(kind, m, k):
        step = (m + k - 1) // k
        return [(kind, lo, min(m, lo + step)) for lo in range(0, m, step)]

    # one process
    t1 = time.time()
    _oracle_chunk(("train", 0, 8192))
    single = 8192 / (time.time() - t1)
    res = {}
    with mp.get_context("fork").Pool(P) as pool:
        pool.map(_oracle_chunk, chunks("fwd_shell_d4", fw["shell_d4"], P))          # warm the workers
        t2 = time.time()
        parts = pool.map(_oracle_chunk, chunks("train", n, P))
        gF = np.zeros_like(F)
        gp = 0.0
        for rows, g, gpp in parts:
            gF[rows] += g
            gp = gp + gpp
        res["train"] = n / (time.time() - t2)
        for kind, m in (("fwd_shell_d4", fw["shell_d4"]), ("fwd_ellipsoids_d7", fw["ellipsoids_d7"]),
                        ("fwd_surfaces_d9", 1 << 14)):
            t3 = time.time()
            pool.map(_oracle_chunk, chunks(kind, m, P))
            res[kind] = m / (time.time() - t3)
    log(f"oracle train pass on {n} rays with {P} processes: {res['train']:.0f} rays/s "
        f"(one process: {single:.0f} rays/s); forward: depth-4 view {res['fwd_shell_d4']:.0f}, depth-7 view "
        f"{res['fwd_ellipsoids_d7']:.0f}, paper-scale view sample {res['fwd_surfaces_d9']:.0f} rays/s")
    out = {"value": round(res["train"], 2), "unit": "rays/s", "cores": P, "kind": "oracle",
           "sample": f"{n} seeded rays of the 2^20-ray batch: FP64 oracle trace + render + loss + backward "
                     f"(feature gradients reduced over the chunks), {P} worker processes with one BLAS "
                     f"thread each; octree build excluded",
           "single_process_rays_per_s": round(single, 2),
           "forward_rays_per_s": {"depth4_view_64x64": round(res["fwd_shell_d4"], 1),
                                  "depth7_view_800x800": round(res["fwd_ellipsoids_d7"], 1),
                                  "paper_scale_view_sample_2^14": round(res["fwd_surfaces_d9"], 1)},
           "nproc": os.cpu_count(), "usable_cores": usable, "cpu_model": _cpu_info()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
