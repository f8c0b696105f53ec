#!/usr/bin/env python
"""Benchmark: light-field frames/s of DirectL on one MI355X, beside the standard paradigm (all N views, then
Alg. 1) on the same GPU and the FP64 CPU oracle on the host.

Workload (the display-scale forward): 300k Gaussians (means uniform in [-2, 2]^3, log-scales U(-4, -2),
random rotations, opacity sigmoid(N(0,1)), SH degree 3), a 3840x2160 panel with 3 subpixels per pixel,
N = 45 views, slant atan(1/6), lens pitch 7.4 subpixels, baseline 0.6, FOV 40 degrees, camera at distance 3
on a +-10 degree azimuth sweep of 200 poses.  Inputs are synthetic and resident in HBM before timing.

One step = one full light-field frame through the whole path (cameras, projection + SH of all views, depth
sort, tile binning and sort, blend into the owned subpixels).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "LF frames/s & Gsubpixel/s vs 45-view render+interleave; p50/p99 frame ms"
HBM_PEAK_GBS = 8000.0
# FP32 vector, non-packed: 256 CUs x 4 SIMD x 16 lanes x 2 FLOP (FMA) x 2.4 GHz
VALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
# FLOPs of one (ray, list entry) evaluation in the blend: offset and q (11), and for a candidate inside the
# cutoff alpha (4: scale, exp, opacity, clamp), transmittance (2) and colour (7)
FLOP_Q = 11
FLOP_BLEND = 13


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * p / 100.0
    f, c = math.floor(k), math.ceil(k)
    return xs[f] if f == c else xs[f] + (xs[c] - xs[f]) * (k - f)


def run_gpu(args):
    import numpy as np
    import torch

    from paper_2407_14053_amd import api, synth

    disp = synth.make_named_display("uhd45")
    scene = synth.make_scene("uhd45")
    poses = synth.pose_sweep(200)
    ctx = api.Context(0)
    S = api.Scene(ctx, scene.arrays())
    D = api.Display(ctx, disp)
    H, W = disp.height, disp.width
    out = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    opts = api.default_opts(tile_w=args.tile, tile_h=args.tile) if args.tile else api.default_opts()

    for i in range(args.warmup):
        api.render(ctx, S, D, poses[i % len(poses)], opts=opts, out=out)
    torch.cuda.synchronize()
    print("warmup done", file=sys.stderr, flush=True)

    ctx.set_profiling(True)
    frame_ms, stages = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        api.render(ctx, S, D, poses[(args.warmup + i) % len(poses)], opts=opts, out=out)
        e1.record(stream)
        stages.append(ctx.frame_stats())
        e1.synchronize()
        frame_ms.append(e0.elapsed_time(e1))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.set_profiling(False)
    wall = t1 - t0
    fps = args.steps / wall
    print("directl: %.2f frames/s" % fps, file=sys.stderr, flush=True)

    def mean_stats(sts):
        keys = sts[0]["stage_ms"].keys()
        st = {k: sum(s["stage_ms"][k] for s in sts) / len(sts) for k in keys}
        cnt = {k: sum(s[k] for s in sts) / len(sts) for k in ("keys", "visible", "evaluations", "blends", "rays")}
        return st, cnt

    st_ms, cnt = mean_stats(stages)
    res = {
        "metric": METRIC,
        "value": round(fps, 3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * wall / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "directl_uhd45: 300k Gaussians (uniform [-2,2]^3, SH3), 3840x2160 panel x 3 "
                               "subpixels, N=45 views, slant atan(1/6), pitch 37/5 subpixels, baseline 0.6, "
                               "FOV 40 deg, 200-pose +-10 deg sweep",
                   "gaussians": scene.n, "width": W, "height": H, "views": disp.n_views,
                   "tile": [stages[0]["tile_w"], stages[0]["tile_h"]], "rays": D.num_rays()},
        "gsubpixel_per_s": round(fps * 3 * W * H / 1e9, 4),
        "p50_ms": round(percentile(frame_ms, 50), 3),
        "p99_ms": round(percentile(frame_ms, 99), 3),
        "stage_ms": {k: round(v, 4) for k, v in st_ms.items() if v > 0},
        "work": {k: int(v) for k, v in cnt.items()},
        "chunk_ms": [{k: round(sum(s_["chunk_ms"][c].get(k, 0.0) for s_ in stages) / len(stages), 4)
                      for k in stages[0]["chunk_ms"][c]} for c in range(len(stages[0]["chunk_ms"]))],
    }

    # roofline of the dominant kernel (largest per-frame stage time, one launch per frame for these)
    dom = max(st_ms, key=lambda k: st_ms[k])
    launches = max(1, stages[0]["stage_launches"][dom])
    per_launch_ms = st_ms[dom] / launches
    G, N = scene.n, disp.n_views
    if dom == "blend":
        flops = (cnt["evaluations"] * FLOP_Q + cnt["blends"] * FLOP_BLEND) / launches
        ach = flops / (per_launch_ms * 1e-3) / 1e12
        roof = {"kernel": "blend", "bound": "alu", "achieved": round(ach, 3), "peak": round(VALU_PEAK_TFLOPS, 1),
                "unit": "TFLOP/s", "frac": round(ach / VALU_PEAK_TFLOPS, 4), "traffic": None,
                "per_launch_ms": round(per_launch_ms, 4)}
    else:
        # HBM models: bytes each launch must move
        if dom == "tile_sort":
            passes = max(1, math.ceil(math.log2(max(2, N * ((W + 55) // 56) * ((H + 55) // 56)))) / 8)
            nbytes = cnt["keys"] * (8 + 8 + 4) * passes / launches   # read k+v, write k+v, histogram read
        elif dom == "bin_emit":
            nbytes = cnt["keys"] * 8 / launches + cnt["visible"] * 48 / launches
        elif dom == "depth_sort":
            nbytes = N * G * (12 + 12 + 8) * 6 / launches
        elif dom == "project":
            nbytes = (G * 236 + N * G * 12 + cnt["visible"] * 48) / launches
        elif dom == "bin_count":
            nbytes = (cnt["visible"] * (48 + 4) + N * G * 4) / launches
        else:
            nbytes = 3 * W * H * 4 / launches
        ach = nbytes / (per_launch_ms * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "per_launch_ms": round(per_launch_ms, 4)}
    res["roofline"] = roof

    if not args.no_standard:
        # the standard paradigm on the same kernels: all 45 full views at its best tile (32x32), then Alg. 1
        out_std = torch.empty_like(out)
        api.render_standard(ctx, S, D, poses[0], out=out_std)
        torch.cuda.synchronize()
        ms, sst = [], []
        ctx.set_profiling(True)
        ts0 = time.perf_counter()
        for i in range(args.std_steps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            api.render_standard(ctx, S, D, poses[(args.warmup + i) % len(poses)], out=out_std)
            e1.record(stream)
            sst.append(ctx.frame_stats())
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        torch.cuda.synchronize()
        ts1 = time.perf_counter()
        ctx.set_profiling(False)
        std_stage, std_cnt = mean_stats(sst)
        std_fps = args.std_steps / (ts1 - ts0)
        # the last standard frame and a DirectL frame of the same pose agree bit for bit
        api.render(ctx, S, D, poses[(args.warmup + args.std_steps - 1) % len(poses)], opts=opts, out=out)
        same = bool(torch.equal(out, out_std))
        res["standard"] = {"frames_per_s": round(std_fps, 4), "ms_per_frame": round(1000 * (ts1 - ts0) / args.std_steps, 2),
                           "steps": args.std_steps, "tile": [sst[0]["tile_w"], sst[0]["tile_h"]],
                           "bit_identical_to_directl": same,
                           "stage_ms": {k: round(v, 3) for k, v in std_stage.items() if v > 0},
                           "work": {k: int(v) for k, v in std_cnt.items()}}
        res["speedup_vs_standard"] = round(fps / std_fps, 2)
        print("standard: %.3f frames/s" % std_fps, file=sys.stderr, flush=True)
    S.close()
    D.close()
    ctx.close()
    return res, scene, disp, poses


def cpu_baseline(args, scene, disp, poses):
    """The FP64 oracle timed on a bounded sample of one frame: every view's projection plus a random sample
    of subpixels composited by brute force; extrapolated to a full frame."""
    import numpy as np

    from oracle import render as orender
    from oracle import viewmap as oviewmap
    c2w = poses[args.warmup]
    V = orender.view_map_of(disp)
    rng = np.random.default_rng(5)
    n = args.cpu_subpixels
    xs = rng.integers(0, disp.height, n)
    ys = rng.integers(0, disp.width, n)
    ks = rng.integers(0, 3, n)
    vs = V[xs, 3 * ys + ks].astype(np.int64)
    R, t, eye = orender.cameras_for(disp, c2w)
    f, cx, cy = orender.intrinsics(disp)
    tp0 = time.perf_counter()
    for v in range(disp.n_views):
        orender.project(scene, R[v], t[v], eye[v], f, cx, cy)
    tp = time.perf_counter() - tp0
    t0 = time.perf_counter()
    orender.render_rays(scene, disp, c2w, vs, xs, ys)
    ts = time.perf_counter() - t0
    per_frame = tp + max(ts - tp, 0.0) * (3 * disp.width * disp.height) / n
    return {"value": round(1.0 / per_frame, 8), "unit": "frames/s", "cores": int(orender.lib().dlo_num_threads()),
            "kind": "oracle",
            "sample": "one frame: FP64 projection of all %d views (%.1f s) plus %d random subpixels composited by "
                      "brute force over all Gaussians (%.1f s incl. projection), extrapolated to %d subpixels"
                      % (disp.n_views, tp, n, ts, 3 * disp.width * disp.height)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--std-steps", type=int, default=2)
    ap.add_argument("--tile", type=int, default=0, help="DirectL tile side (0 = automatic)")
    ap.add_argument("--cpu-subpixels", type=int, default=1536)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-standard", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this renderer has no multi-GPU path (requested %d GPUs)"
              % max(args.gpus, world), file=sys.stderr)
        sys.exit(2)
    res, scene, disp, poses = run_gpu(args)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(args, scene, disp, poses)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
