"""Benchmark of the splatting hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload (one GPU's share, plain method): 2M Gaussians on a 1 km x 1 km
ground plane, SH degree 3, one 1920x1080 aerial view at 150 m pitched 45
degrees down (70 degree field of view), K = 1 cell, FP32 forward + backward
with an L1 loss against a seeded random target image.  All inputs are
synthetic and resident in HBM before timing starts.

One step = preprocess -> sort -> partial render -> composition -> L1 ->
composition backward -> render backward -> preprocess backward, every stage
a HIP kernel of libsplaxel.so on torch's current stream, with no host
synchronisation inside the step (the instance capacity is sized once during
warm-up).  value = B / t_step, where B is the number of Gaussian-pixel pairs
blended in the forward pass (counted once by the renderer's per-pixel
counter; the step is deterministic, so B is the same every step).

Prints ONE JSON line.  Per-stage times, the roofline of the dominant kernel
and the CPU oracle baseline are included in it, and (unless --no-extras)
the metric's two other parts on their own workloads: views/s of the K = 8
cells training step on the 8M-Gaussian scene at 1920x1080
(views_per_s_8M_1080p, with the roofline of its reverse walk) and serving
p50/p99 latency and frames/s on the resident 30M-Gaussian scene against
plain per-view service (serve_p50_ms, serve_p99_ms, serve_30M).
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Gaussian-pixel blends/s fwd+bwd"
HBM_PEAK_GBS = 8000.0
# FP32 vector lanes: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz (non-packed)
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload():
    """The scene is stored in spatial (Morton) order of the means, the
    layout the framework keeps a resident model in."""
    import synth
    from paper_2606_18588_amd.pipeline import spatial_order
    scene = synth.g2_scene()
    scene = scene.subset(spatial_order(scene.means))
    cam = synth.g2_camera()
    target = synth.g2_target()
    return scene, cam, target


class Step:
    """Buffers + the sequence of C-ABI calls of one training step."""

    def __init__(self, scene, cam, target, settings):
        import torch
        from paper_2606_18588_amd import binding as B
        from paper_2606_18588_amd.pipeline import CellView, GaussianParams
        self.torch = torch
        self.B = B
        self.cam = cam
        self.params = GaussianParams.from_scene(scene)
        self.grads = self.params.zeros_like()
        self.view = CellView(self.params, cam, settings)
        self.box = [type("Box", (), {"lo": (-1e30,) * 3, "hi": (1e30,) * 3})()]
        self.c_cam = self.view.c_cam
        self.c_par = self.view.c_par
        H, W = cam.height, cam.width
        self.out = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
        self.dout = torch.empty_like(self.out)
        self.target = torch.as_tensor(target).cuda()
        self.view.ensure_backward_buffers()
        # size the instance buffers once (one host read-back, outside timing)
        self.view.preprocess()
        self.counts = self.view.sort(sync=True)
        self.view._alloc_sort(int(self.counts[1] * 1.05) + 4096)
        self.view.ensure_backward_buffers()  # sized for the new capacity
        self.stage_names = ["preprocess", "sort", "render", "composite_l1",
                            "render_bwd_prep", "render_bwd_walk", "render_bwd_reduce",
                            "preprocess_bwd"]

    def run(self, events=None, count=False):
        B, v = self.B, self.view
        ev = events
        if ev: ev[0].record()
        v.preprocess()
        if ev: ev[1].record()
        v.sort(sync=False)
        if ev: ev[2].record()
        v.render(None, want_nblend=count)
        if ev: ev[3].record()
        # composition (Eq. 5), L1 and the composition backward in one pass
        B.sx_composite_l1([v.partial], self.box, self.c_cam, self.c_par, self.target,
                          self.out, None, None, [v.dpartial])
        if ev: ev[4].record()
        # the three stages of sx_render_backward, called one by one so that
        # events bracket the reverse walk alone
        for i, stage in enumerate((B.SX_RB_PREPARE, B.SX_RB_WALK, B.SX_RB_REDUCE)):
            B.sx_render_backward_stages(v.c_proj, v.vals, v.ranges, v.ws, v.params.n,
                                        v.capacity, v.bwd_ws, self.c_cam, self.c_par, None,
                                        v.partial, v.last, v.dpartial, None, v.g2d, stage)
            if ev: ev[5 + i].record()
        v.preprocess_backward(self.grads)
        if ev: ev[8].record()


def cpu_baseline(scene, cam, settings, min_s=10.0, max_steps=20):
    """The FP64 oracle (as it stands, all host threads) on the same step:
    the full 1920x1080 view of the 2M-Gaussian scene, forward (projection,
    binned render, composition), L1 loss and backward, repeated until
    `min_s` seconds have passed (at most `max_steps` steps); blends/s."""
    import oracle
    import synth
    oracle.build()
    cores = oracle.num_threads()
    box = synth.Cell((-1e30,) * 3, (1e30,) * 3)
    target = synth.g2_target()
    blends, steps = 0, 0
    t0 = time.perf_counter()
    while steps < max_steps and (steps == 0 or time.perf_counter() - t0 < min_s):
        fr = oracle.forward([scene], [box], cam, settings)
        _, g = oracle.l1_loss(fr.comp["rgb"], target)
        oracle.backward([scene], [box], cam, settings, fr, g)
        blends += int(fr.parts[0]["nblend"].sum())
        steps += 1
    dt = time.perf_counter() - t0
    # one thread on the 960x540 centre crop of the same view (the whole
    # projection, a quarter of the pixels): a few seconds of work
    w, h = cam.width // 2, cam.height // 2
    x0, y0 = (cam.width - w) // 2, (cam.height - h) // 2
    crop = dataclasses.replace(cam, cx=cam.cx - x0, cy=cam.cy - y0, width=w, height=h)
    oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        fr = oracle.forward([scene], [box], crop, settings)
        _, g = oracle.l1_loss(fr.comp["rgb"], target[y0:y0 + h, x0:x0 + w])
        oracle.backward([scene], [box], crop, settings, fr, g)
        dt1 = time.perf_counter() - t1
        b1 = int(fr.parts[0]["nblend"].sum())
    finally:
        oracle.set_threads(cores)
    return {"value": blends / dt, "unit": "blends/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} full steps: the 1920x1080 view of the 2M-Gaussian scene, "
                      f"FP64 forward + L1 + backward, {blends} blends in {dt:.2f} s",
            "single_thread": {"value": b1 / dt1, "unit": "blends/s", "cores": 1,
                              "sample": f"one step on the {w}x{h} centre crop of the same "
                                        f"view, {b1} blends in {dt1:.2f} s"},
            "cpu_model": _cpu_model()}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile", default="16x16")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (a plain "
                         "copy of known size that calibrates PMC traffic counters)")
    ap.add_argument("--form", choices=("plain", "batched", "serve", "cells"), default="plain",
                    help="plain: the headline single-view step; batched: 16-view training "
                         "step (15M Gaussians) batched vs per-view; serve: request trace "
                         "(30M Gaussians) served batched vs per-view; cells: the K = 8 "
                         "composition training step (8M Gaussians, 8 views)")
    ap.add_argument("--requests", type=int, default=800,
                    help="serve: measured requests (after 200 warm-up requests)")
    ap.add_argument("--no-tune", action="store_true", help="batched: skip the autotuner")
    ap.add_argument("--streams", type=int, default=4,
                    help="cells: streams for the cells' independent forward chains")
    ap.add_argument("--cross-filter", action="store_true",
                    help="cells: per-ray cross-boundary filtering of every cell's render")
    ap.add_argument("--reeval", action="store_true",
                    help="cells: carry the saturation state with speculative re-evaluation")
    ap.add_argument("--partition", choices=("grid", "kd"), default="grid",
                    help="cells: the 4 x 2 ground grid of the configuration, or KD-tree cells")
    ap.add_argument("--bucketed", action="store_true",
                    help="cells: the 8 views scheduled by conflict-free view bucketing (one "
                         "render and one render-backward launch per bucket) against per-view "
                         "frames, with the grid cells clipped to the scene's height range")
    ap.add_argument("--repartition", action="store_true",
                    help="cells: also time one repartition of the 8M scene's 4 x 2 grid cells "
                         "into KD-tree cells (parameters and Adam moments moved on the GPU)")
    ap.add_argument("--no-extras", action="store_true",
                    help="plain: skip the K = 8 cells step and the serving trace that the "
                         "default line also reports")
    ap.add_argument("--cells-steps", type=int, default=10,
                    help="plain: timed K = 8 cells steps (8 views each) for the extra fields")
    ap.add_argument("--serve-requests", type=int, default=400,
                    help="plain: measured requests of the serving trace for the extra fields")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "exchange of partial pixels between GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    torch.cuda.set_device(0)
    if args.form == "batched":
        return bench_batched(args)
    if args.form == "serve":
        return bench_serve(args)
    if args.form == "cells" and args.bucketed:
        return bench_bucketed(args)
    if args.form == "cells":
        return bench_cells(args)
    tw, th = (int(x) for x in args.tile.split("x"))
    settings = synth.RenderSettings(tile_w=tw, tile_h=th)
    t0 = time.perf_counter()
    scene, cam, target = make_workload()
    log(f"bench: workload generated in {time.perf_counter() - t0:.1f}s")
    if args.copy_probe_mb > 0:
        n = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    st = Step(scene, cam, target, settings)
    # blend count B (deterministic per step)
    st.run(count=True)
    torch.cuda.synchronize()
    blends = int(st.view.nblend.sum().item())
    st.blends = blends
    n_vis, n_inst = st.counts
    log(f"bench: visible {n_vis} instances {n_inst} blends {blends}")
    for _ in range(args.warmup):
        st.run()
    torch.cuda.synchronize()
    # per-stage times with events on the launch stream
    nst = len(st.stage_names)
    stage_ms = np.zeros(nst)
    # the steps run back to back, as in the timed region: a synchronisation
    # between them would leave the device idle while the host launches the
    # next step's first kernel, and that wait would be charged to the first
    # stage (one untimed step ahead of them keeps the queue busy)
    reps = max(3, min(args.steps, 20))
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(nst + 1)] for _ in range(reps)]
    st.run()
    for ev in evs:
        st.run(events=ev)
    torch.cuda.synchronize()
    for ev in evs:
        stage_ms += np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(nst)])
    stage_ms /= reps
    # timed region: exactly K steps, synchronised on both sides
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    tw0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        st.run()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - tw0
    ms = e0.elapsed_time(e1) / args.steps
    value = blends / (ms / 1e3)
    stages = {k: round(float(v), 4) for k, v in zip(st.stage_names, stage_ms)}
    log("bench: stage ms " + json.dumps(stages))
    roof = roofline(st, stages)
    line = {
        "metric": METRIC, "value": value, "unit": "blends/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "one GPU's share: 2M Gaussians SH3 on a 1 km^2 ground plane, "
                               "1920x1080 aerial view, K=1, L1 fwd+bwd",
                   "gaussians": scene.n, "width": cam.width, "height": cam.height,
                   "tile": args.tile, "cells": 1, "layout": "Morton order of the means"},
        "views_per_s": 1e3 / ms, "blends_per_step": blends, "visible": n_vis,
        "instances": n_inst, "stage_ms": stages, "wall_s": wall,
        "roofline": roof, "stage_roofline": stage_rooflines(st, stages),
    }
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        line["cpu_baseline"] = cpu_baseline(scene, cam, settings)
        log(f"bench: cpu baseline {time.perf_counter() - t0:.1f}s")
    if not args.no_extras:
        # the metric's other two parts, on their own workloads
        del st
        torch.cuda.empty_cache()
        t0 = time.perf_counter()
        cells, n8 = cells_measure(args, ((1920, 1080),), args.cells_steps, 2)
        c = cells["1920x1080"]
        line["views_per_s_8M_1080p"] = c["views_per_s"]
        line["cells_8M_1080p"] = dict(c, workload=cells_workload(args), gaussians=n8,
                                      layout="each cell in Morton order of its means")
        log(f"bench: K=8 cells {c['views_per_s']:.1f} views/s at 1080p "
            f"({time.perf_counter() - t0:.1f}s)")
        t0 = time.perf_counter()
        srv, n30 = serve_measure(args.serve_requests, args.serve_requests // 4)
        b, p = srv["batched"], srv["plain"]
        line["serve_p50_ms"] = b["open_loop"]["p50_ms"]
        line["serve_p99_ms"] = b["open_loop"]["p99_ms"]
        line["serve_frames_per_s"] = b["open_loop"]["frames_per_s"]
        line["serve_30M"] = {
            "workload": SERVE_WORKLOAD, "gaussians": n30, "requests": args.serve_requests,
            "warmup_requests": args.serve_requests // 4,
            "layout": "Morton order of the means", "batched": b, "plain": p,
            "closed_loop_speedup_vs_plain": b["closed_loop_frames_per_s"] /
            p["closed_loop_frames_per_s"]}
        log(f"bench: serve p50 {line['serve_p50_ms']:.2f} ms p99 {line['serve_p99_ms']:.2f} ms "
            f"({time.perf_counter() - t0:.1f}s)")
    print(json.dumps(line), flush=True)


def bench_batched(args):
    """16 views of uneven resolution of a 15M-Gaussian scene: one training
    step = every view's forward, L1 against its target, backward, then one
    Adam update.  Batched (autotuned tile shape and views per persistent
    launch) against the plain per-view calls."""
    import torch
    import synth
    from paper_2606_18588_amd.batched import MultiViewStep, autotune, time_step
    from paper_2606_18588_amd.pipeline import GaussianParams
    t0 = time.perf_counter()
    from paper_2606_18588_amd.pipeline import spatial_order
    scene = synth.g15_scene()
    scene = scene.subset(spatial_order(scene.means))  # the resident layout
    cams = synth.g15_cameras()
    params = GaussianParams.from_scene(scene)
    del scene
    grads = params.zeros_like()
    targets = [torch.as_tensor(synth.random_image(300 + k, c.width, c.height)).cuda()
               for k, c in enumerate(cams)]
    log(f"bench: 15M scene + 16 views ready in {time.perf_counter() - t0:.1f}s")

    def settings(tw, th):
        return synth.RenderSettings(tile_w=tw, tile_h=th)
    tuned = []
    if args.no_tune:
        tw, th = (int(x) for x in args.tile.split("x"))
        best_tile, best_batch = args.tile, 16
    else:
        tuned = autotune(params, grads, cams, targets, settings, log=log)
        best_tile, best_batch = tuned[0].tile, tuned[0].batch
    tw, th = (int(x) for x in best_tile.split("x"))
    step = MultiViewStep(params, grads, cams, targets, settings(tw, th), batch=best_batch)
    blends = step.run(1e-7, count_blends=True, check=True)
    inst = sum(c[1] for c in step.counts)
    ms_b = time_step(step, reps=args.steps, warmup=args.warmup)
    step.run(1e-7, check=True)
    del step
    torch.cuda.empty_cache()
    plain = MultiViewStep(params, grads, cams, targets, settings(16, 16), plain=True)
    plain.run(1e-7, check=True)
    ms_p = time_step(plain, reps=args.steps, warmup=args.warmup)
    plain.run(1e-7, check=True)
    del plain
    V = len(cams)
    line = {
        "metric": "views/s, 16-view training step (fwd+bwd+Adam)", "value": V / (ms_b / 1e3),
        "unit": "views/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_b, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "15M Gaussians SH3 on a 1 km^2 ground plane, 16 views of "
                               "uneven resolution (960x540..2048x1365) on a 200 m orbit, "
                               "L1 fwd+bwd per view, one Adam update",
                   "gaussians": params.n, "views": V, "tile": best_tile, "batch": best_batch,
                   "pixels": int(sum(c.width * c.height for c in cams))},
        "plain_views_per_s": V / (ms_p / 1e3), "plain_ms_per_step": ms_p,
        "speedup_vs_plain": ms_p / ms_b, "blends_per_step": blends,
        "blends_per_s": blends / (ms_b / 1e3), "instances_per_step": inst,
        "autotune": [{"tile": r.tile, "batch": r.batch, "ms": r.ms} for r in tuned],
    }
    print(json.dumps(line), flush=True)


def bench_cells(args):
    """The K = 8 composition workload (cells_measure) at 1920x1080 (the
    metric's resolution) and 1600x1200 (the configuration's), printed as its
    own line."""
    out, n_gauss = cells_measure(args, ((1920, 1080), (1600, 1200)), args.steps, args.warmup)
    m = out["1920x1080"]
    line = {
        "metric": "views/s @1080p 8M G", "value": m["views_per_s"], "unit": "views/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": cells_workload(args), "gaussians": n_gauss, "cells": 8,
                   "views": 8, "layout": "each cell in Morton order of its means"},
        "resolutions": out,
    }
    print(json.dumps(line), flush=True)


def bench_bucketed(args):
    """The K = 8 training step over the 8M scene's 8 aerial views at
    1920x1080, scheduled two ways on the same cells (the 4 x 2 grid clipped
    to the height range of the scene's means, so that a view meets only the
    cells its rays cross above the ground): per-view frames (every cell's
    chain per view, cells spread over side streams) and conflict-free view
    buckets (per bucket one render and one render-backward launch over its
    (view, participant cell) items).  Both: L1 against the view's target,
    gradients summed over the views, one Adam update of every cell."""
    import torch
    import synth
    from paper_2606_18588_amd import binding as B
    from paper_2606_18588_amd.batched import BucketedCells
    from paper_2606_18588_amd.pipeline import Frame, GaussianParams, spatial_order
    t0 = time.perf_counter()
    scene = synth.g8_scene()
    part = synth.grid_partition(scene, synth.GRID_X, synth.GRID_Y)
    z0, z1 = float(scene.means[:, 2].min()), float(scene.means[:, 2].max())
    boxes = [synth.Cell((c.lo[0], c.lo[1], z0), (c.hi[0], c.hi[1], np.nextafter(z1, np.inf)))
             for c in part.cells]
    params = [GaussianParams.from_scene(c.subset(spatial_order(c.means)))
              for c in part.cell_scenes(scene)]
    del scene
    grads = [p.zeros_like() for p in params]
    moments = [(torch.zeros_like(t), torch.zeros_like(t)) for p in params for t in p.tensors()]
    st = synth.RenderSettings()
    w, h = 1920, 1080
    cams = synth.g8_cameras(w, h)
    targets = [torch.as_tensor(synth.random_image(500 + k, w, h)).cuda() for k in range(len(cams))]
    log(f"bench: 8M scene in 8 z-clipped cells ready in {time.perf_counter() - t0:.1f}s")
    t_adam = [0]

    def adam():
        t_adam[0] += 1
        k = 0
        for p, g in zip(params, grads):
            for pt, gt in zip(p.tensors(), g.tensors()):
                B.sx_adam(pt, gt, moments[k][0], moments[k][1], t_adam[0], 1e-7)
                k += 1

    frames = [Frame(params, boxes, c, st, streams=args.streams) for c in cams]
    for f in frames:
        f.init_masks(geometric=True)
        f.forward(use_masks=True, sync=True)
        for v in f.views:
            v._alloc_sort(int(v.counts[1] * 1.1) + 4096)

    def plain_step():
        for g in grads:
            for t in g.tensors():
                B.sx_fill_u32(t, 0)
        for f, tg in zip(frames, targets):
            f.train_l1(tg, grads, accumulate=True, use_masks=True, update_masks=True, sync=False)
        adam()

    bc = BucketedCells(params, boxes, cams, st, streams=args.streams)

    def bucket_step():
        bc.step(targets, grads)
        adam()

    res = {}
    for name, fn in (("plain", plain_step), ("bucketed", bucket_step)):
        for _ in range(max(args.warmup, 2)):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        res[name] = {"ms_per_step": ms, "views_per_s": len(cams) / (ms / 1e3)}
        log(f"bench: {name} {ms:.2f} ms per 8-view step, {len(cams) / (ms / 1e3):.1f} views/s")
    line = {
        "metric": "views/s @1080p 8M G, bucketed", "value": res["bucketed"]["views_per_s"],
        "unit": "views/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["bucketed"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "8M Gaussians SH3 on a 1 km^2 ground plane in a 4x2 grid of cells "
                               "clipped to the means' height range, 8 aerial views at 1920x1080, "
                               "fwd + L1 + bwd per view with geometric and saturation masks, one "
                               "Adam update per step",
                   "gaussians": int(sum(p.n for p in params)), "cells": 8, "views": 8,
                   "layout": "each cell in Morton order of its means"},
        "participants": [sorted(s) for s in bc.participants], "buckets": bc.buckets,
        "plain": res["plain"], "speedup_vs_plain": res["plain"]["ms_per_step"] /
        res["bucketed"]["ms_per_step"],
    }
    print(json.dumps(line), flush=True)


def cells_workload(args):
    return ("8M Gaussians SH3 on a 1 km^2 ground plane in K=8 cells "
            f"({'KD-tree' if args.partition == 'kd' else '4x2 grid'}), "
            "8 aerial views, fwd + L1 + bwd per view with "
            "geometric visibility and temporal saturation masks"
            + (" re-evaluated every render" if args.reeval else "")
            + (", cross-boundary filtering" if args.cross_filter else "")
            + f", cells' chains on {args.streams} stream(s)"
            + ", one Adam update per step")


def cells_measure(args, sizes, steps, warmup, walk_roofline=True):
    """The K = 8 composition workload: 8M Gaussians split by centre into a
    4 x 2 grid of cells on the ground plane, 8 views from (10, 20, 150) m.
    One training step = for every view, each cell's preprocess, sort and
    partial render (restricted to the pixels where the cell's box is
    geometrically visible and, from the view's previous step, not behind a
    saturated prefix), composition (Eq. 5, updating the masks), L1, the
    composition backward and every cell's backward; then one Adam update of
    every cell.  Returns ({"WxH": results}, Gaussians).  With walk_roofline,
    one more step runs with every cell's chain on one stream and timing
    events around each reverse walk, for the roofline of that kernel."""
    import torch
    import synth
    from paper_2606_18588_amd import binding as B
    from paper_2606_18588_amd.pipeline import Frame, GaussianParams, spatial_order
    t0 = time.perf_counter()
    scene = synth.g8_scene()
    if args.partition == "kd":  # the paper's KD-tree cells instead of the 4 x 2 grid
        boxes_t, cell_of = B.sx_kd_partition(scene.means, 8)
        cells = [synth.Cell(lo, hi) for lo, hi in boxes_t]
        cell_scenes = [scene.subset(np.nonzero(cell_of == k)[0]) for k in range(8)]
    else:
        part = synth.grid_partition(scene, synth.GRID_X, synth.GRID_Y)
        cells = part.cells
        cell_scenes = part.cell_scenes(scene)
    cell_scenes = [c.subset(spatial_order(c.means)) for c in cell_scenes]
    del scene
    params = [GaussianParams.from_scene(c) for c in cell_scenes]
    del cell_scenes
    grads = [p.zeros_like() for p in params]
    moments = [(torch.zeros_like(t), torch.zeros_like(t)) for p in params for t in p.tensors()]
    log(f"bench: 8M scene in {len(params)} cells ready in {time.perf_counter() - t0:.1f}s")
    rep = None
    if getattr(args, "repartition", False):
        from paper_2606_18588_amd.pipeline import imbalance, repartition
        states = [[m for t in range(5) for m in moments[5 * k + t]] for k in range(len(params))]
        before = imbalance(params)
        times = []
        for _ in range(3):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            new, _, new_states = repartition(params, len(params), states)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t1)
            del new, new_states
        rep = {"imbalance_before": before, "ms": 1e3 * min(times),
               "bytes_moved": int(sum(t.numel() * 4 for p in params for t in p.tensors()) * 3)}
        log(f"bench: repartition of {len(params)} cells ({before:.3f} imbalance): "
            f"{rep['ms']:.1f} ms")
    st = synth.RenderSettings()
    out = {}
    n_gauss = int(sum(p.n for p in params))
    for (w, h) in sizes:
        cams = synth.g8_cameras(w, h)
        targets = [torch.as_tensor(synth.random_image(500 + k, w, h)).cuda()
                   for k in range(len(cams))]
        frames = [Frame(params, cells, c, st, cross_filter=args.cross_filter,
                        streams=args.streams) for c in cams]
        dout = torch.empty((h, w, 4), dtype=torch.float32, device="cuda")
        for f in frames:  # size every cell's instance buffers once, with headroom
            f.init_masks(geometric=True, reeval=args.reeval)
            f.forward(use_masks=True, sync=True)
            for v in f.views:
                v._alloc_sort(int(v.counts[1] * 1.1) + 4096)
        torch.cuda.synchronize()
        t_adam = [0]
        flips = [0, 0]  # re-activated pairs, pairs pruned before the step (counted step)
        pop8 = torch.tensor([bin(i).count("1") for i in range(256)], device="cuda")

        def popcount(words):
            return int(pop8[words.contiguous().view(torch.uint8).long()].sum().item())

        def step(count=False):
            for g in grads:
                for t in g.tensors():
                    B.sx_fill_u32(t, 0)
            blends = 0
            for f, tg in zip(frames, targets):
                before = f.masks.clone() if (count and f.omega is not None) else None
                if f.budget is None:
                    # render, composition + L1 + composition backward in one
                    # pass, every cell's backward
                    f.train_l1(tg, grads, accumulate=True, use_masks=True, update_masks=True,
                               sync=False)
                else:
                    f.forward(use_masks=True, update_masks=True, sync=False)
                    B.sx_l1_loss(f.out, tg, w, h, dout, None)
                    f.backward(dout, grads, accumulate=True)
                if count:
                    blends += sum(int(v.nblend.sum().item()) for v in f.views)
                    if before is not None:
                        flips[0] += popcount(f.masks & ~before)
                        flips[1] += popcount(f.omega & ~before)
            t_adam[0] += 1
            k = 0
            for p, g in zip(params, grads):
                for pt, gt in zip(p.tensors(), g.tensors()):
                    B.sx_adam(pt, gt, moments[k][0], moments[k][1], t_adam[0], 1e-7)
                    k += 1
            return blends

        for _ in range(max(warmup, 2)):
            step()
        blends = step(count=True)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out[f"{w}x{h}"] = {"ms_per_step": ms, "views_per_s": len(cams) / (ms / 1e3),
                           "blends_per_step": blends, "blends_per_s": blends / (ms / 1e3)}
        if walk_roofline and not args.reeval:
            # every cell's chain on one stream, timing events around each
            # reverse walk (the kernel the K = 8 step spends most time in)
            walks = []
            for f in frames:
                f.walk_events, f._side_saved, f.side = walks, f.side, None
            blends_w = step(count=True)
            torch.cuda.synchronize()
            for f in frames:
                f.walk_events, f.side = None, f._side_saved
            walk_ms = sum(a.elapsed_time(b) for a, b in walks)
            ops = 53.0 * blends_w
            ach = ops / (walk_ms / 1e3) / 1e12
            out[f"{w}x{h}"]["roofline"] = {
                "bound": "alu", "kernel": "k_render_bwd<16, 16, false, false>",
                "achieved": ach, "peak": ALU_PEAK_TOPS, "unit": "T lane-op/s",
                "frac": ach / ALU_PEAK_TOPS, "traffic": None, "algorithmic_ops": ops,
                "launches": len(walks), "walk_ms_per_step": walk_ms,
                "timing": "events around each of the step's reverse walks, the cells' chains "
                          "on one stream"}
        if args.reeval:
            out[f"{w}x{h}"].update(reactivated=flips[0], pruned_before=flips[1],
                                   flip_rate=flips[0] / max(flips[1], 1))
        log(f"bench: cells {w}x{h}: {ms:.2f} ms per 8-view step, "
            f"{len(cams) / (ms / 1e3):.1f} views/s, {blends} blends"
            + (f", re-activated {flips[0]} of {flips[1]} pruned pairs" if args.reeval else ""))
        del frames
        torch.cuda.empty_cache()
    del params, grads, moments
    torch.cuda.empty_cache()
    if rep is not None:
        out["repartition"] = rep
    return out, n_gauss


def bench_serve(args):
    """The serving workload (serve_measure), printed as its own line."""
    res, n_gauss = serve_measure(args.requests, 200)
    b, p = res["batched"], res["plain"]
    line = {
        "metric": "serve p50 latency ms", "value": b["open_loop"]["p50_ms"], "unit": "ms",
        "n_gpus": 1, "steps": args.requests, "warmup": 200,
        "ms_per_step": b["open_loop"]["mean_ms"], "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": SERVE_WORKLOAD, "gaussians": n_gauss, "requests": args.requests,
                   "layout": "Morton order of the means"},
        "p99_ms": b["open_loop"]["p99_ms"], "frames_per_s": b["open_loop"]["frames_per_s"],
        "closed_loop_frames_per_s": b["closed_loop_frames_per_s"],
        "plain": p,
        "speedup_closed_loop_vs_plain": b["closed_loop_frames_per_s"] /
        p["closed_loop_frames_per_s"],
        "batched": b,
    }
    print(json.dumps(line), flush=True)


SERVE_WORKLOAD = ("resident 30M Gaussians SH3 on a 2 km x 2 km ground plane, Poisson 200 req/s, "
                  "resolutions uniform over 640x360, 1280x720, 1920x1080, 3840x2160, forward "
                  "render + composition")


def serve_measure(requests, warm_n):
    """Poisson request trace (200 req/s, resolutions 640x360..3840x2160) on a
    resident 30M-Gaussian scene: continuous batching against plain per-view
    service, open loop (latency) and closed loop (max frames/s).  Returns
    ({"batched": ..., "plain": ...}, Gaussians)."""
    import torch
    import synth
    from paper_2606_18588_amd.pipeline import GaussianParams
    from paper_2606_18588_amd.serve import Server, summarize
    t0 = time.perf_counter()
    from paper_2606_18588_amd.pipeline import spatial_order
    scene = synth.g30_scene()
    scene = scene.subset(spatial_order(scene.means))  # the resident layout
    params = GaussianParams.from_scene(scene)
    del scene
    trace = synth.serve_trace(warm_n + requests)
    log(f"bench: 30M scene + {len(trace)} requests ready in {time.perf_counter() - t0:.1f}s")
    st = synth.RenderSettings()

    def rebase(reqs):
        a0 = reqs[0].arrival_s
        return [synth.Request(r.arrival_s - a0, r.camera, r.rid) for r in reqs]
    res = {}
    for mode in ("batched", "plain"):
        srv = Server(params, st, plain=(mode == "plain"), arena_bytes=40 << 30)
        srv.calibrate(trace[0].camera)
        srv.serve(rebase(trace[:warm_n]), open_loop=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        done = srv.serve(rebase(trace[warm_n:]), open_loop=True)
        open_s = summarize(done)
        log(f"bench: serve {mode} open loop {open_s} in {time.perf_counter() - t1:.1f}s")
        t1 = time.perf_counter()
        done = srv.serve(rebase(trace[warm_n:]), open_loop=False)
        closed_wall = time.perf_counter() - t1
        closed = summarize(done, wall_s=max(d.done_s for d in done))
        log(f"bench: serve {mode} closed loop {closed['frames_per_s']:.1f} frames/s")
        res[mode] = {"open_loop": open_s, "closed_loop_frames_per_s": closed["frames_per_s"],
                     "batches": srv.n_batches, "overflows": srv.overflows}
        del srv
        torch.cuda.empty_cache()
    n_gauss = params.n
    del params
    torch.cuda.empty_cache()
    return res, n_gauss


# Single-kernel stages: (entry point's only kernel, its source file).
KERNEL_OF_STAGE = {
    "preprocess": ("k_preprocess<3>", "sx_preprocess.hip"),
    "preprocess_bwd": ("k_preprocess_backward<3, false>", "sx_preprocess.hip"),
    "render": ("k_render<16, 16, false, false>", "sx_render.hip"),
    "render_bwd_walk": ("k_render_bwd<16, 16, false, false>", "sx_render.hip"),
}
PMC_FILE = os.path.join(ROOT, "profiles", "g2_pmc_traffic.txt")


def source_sha(name):
    """Hash of a kernel's source file and the headers every kernel file
    includes (the device helpers and constants of sx_internal.h, the ABI's
    structs), so that a change to either voids the committed counters."""
    import hashlib
    h = hashlib.sha256()
    for path in (os.path.join(ROOT, "paper_2606_18588_amd", "csrc", name),
                 os.path.join(ROOT, "paper_2606_18588_amd", "csrc", "sx_internal.h"),
                 os.path.join(ROOT, "include", "splaxel.h")):
        h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def pmc_traffic(kernel, src):
    """HBM bytes per launch of `kernel` from the committed PMC summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), or None if
    there is none or the kernel's source changed since it was taken."""
    if not os.path.exists(PMC_FILE):
        return None
    for line in open(PMC_FILE):
        if line.startswith("{"):
            d = json.loads(line)
            if d.get("kernel") == kernel and d.get("source_sha") == source_sha(src):
                return d["hbm_bytes_per_launch"]
    return None


def stage_rooflines(st, stage_ms):
    """Every stage's algorithmic work (the per-unit figures of the design
    notes times this step's counts) over its event-timed duration, as a
    fraction of the bound that limits it: HBM bytes for the data-movement
    stages (the sort also against its one-pass floor of 24 B per
    instance), FP32 lane-operation slots for the two rasterizer walks."""
    n = st.params.n
    n_vis, n_inst = st.counts
    hw = st.cam.width * st.cam.height
    tiles = st.view.tiles
    sh_bytes = st.params.sh.shape[1] * 3 * 4
    pbytes = 12 + 12 + 16 + 4 + sh_bytes
    # significant key bits at this grid: tile id bits + 32 depth bits, in
    # 8-bit LSD passes (the radix-sort reference the per-unit figure uses)
    passes = -(-(max(tiles - 1, 1).bit_length() + 32) // 8)
    hbm = {
        "preprocess": 16 * n + (4 + 12 + 16 + sh_bytes + 56) * n_vis,
        "sort": n_inst * (24 * passes + 8),
        # the fused pass: partials read (16 B per cell), target read (12),
        # composed image (16) and partial gradients (16 per cell) written
        "composite_l1": (32 * 1 + 28) * hw,
        "render_bwd_prep": 4 * hw + 4 * tiles,
        "render_bwd_reduce": 40 * n_inst + (12 + 48) * n_vis,
        "preprocess_bwd": (8 + pbytes + 40 + pbytes) * n_vis,
    }
    alu = {"render": 24.0 * st.blends,
           "render_bwd_walk": 53.0 * st.blends}
    out = {}
    for k, ms in stage_ms.items():
        if ms <= 0:
            continue
        if k in hbm:
            ach = hbm[k] / (ms / 1e3) / 1e9
            out[k] = {"bound": "hbm", "algorithmic_bytes": hbm[k], "achieved": round(ach, 1),
                      "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4)}
            if k == "sort":
                out[k]["passes"] = passes
                out[k]["frac_one_pass_floor"] = round(24 * n_inst / (ms / 1e3) / 1e9 /
                                                      HBM_PEAK_GBS, 4)
        elif k in alu:
            ach = alu[k] / (ms / 1e3) / 1e12
            out[k] = {"bound": "alu", "algorithmic_ops": alu[k], "achieved": round(ach, 3),
                      "unit": "T lane-op/s", "frac": round(ach / ALU_PEAK_TOPS, 4)}
    return out


def roofline(st, stage_ms):
    """Roofline entry for the largest kernel that has an entry point of its
    own (so that events around the call time exactly that kernel).  The
    per-unit algorithmic work: HBM-bound stages count the bytes the method
    must move, the rasterizers count FP32 lane-operation slots per blended
    (pixel, Gaussian) pair (24 forward: 14 for alpha and its test, 10 for
    the blend; 53 in the reverse walk; unit "T lane-op/s"), so that the
    evaluations of pairs that do not blend count as overhead in both.  working_set_bytes is what the kernel touches: below
    the 256 MB Infinity Cache a bandwidth figure may be served from it."""
    n = st.params.n
    n_vis, n_inst = st.counts
    sh_bytes = st.params.sh.shape[1] * 3 * 4
    stage = max(KERNEL_OF_STAGE, key=lambda k: stage_ms[k])
    ms = stage_ms[stage]
    kernel, src = KERNEL_OF_STAGE[stage]
    if stage in ("render", "render_bwd_walk"):
        # FP32 lane-operation slots per blend (a transcendental or
        # reciprocal takes 4): forward 24, reverse walk 53
        if stage == "render":
            ops = 24.0 * st.blends
        else:
            ops = 53.0 * st.blends
        ach = ops / (ms / 1e3) / 1e12
        hw = st.cam.width * st.cam.height
        tiles = st.view.tiles
        if stage == "render":
            # records (48 B per visible Gaussian), values, ranges; partial,
            # last and blend count written
            ws = 48 * n_vis + 4 * n_inst + 8 * tiles + 24 * hw
        else:
            # records, values, ranges, per-tile counts; partial, last and
            # dpartial read; one 40-byte gradient row per instance written
            ws = 48 * n_vis + 44 * n_inst + 12 * tiles + 36 * hw
        return {"bound": "alu", "kernel": kernel, "achieved": ach, "peak": ALU_PEAK_TOPS,
                "unit": "T lane-op/s", "frac": ach / ALU_PEAK_TOPS,
                "traffic": pmc_traffic(kernel, src), "algorithmic_ops": ops,
                "working_set_bytes": ws}
    if stage == "preprocess":
        # every Gaussian: mean read (12 B), tile count written (4 B); the
        # visible ones also read logit, scales, rotation and SH and write the
        # 48-byte record and the 8-byte tile rectangle
        byts = 16 * n + (4 + 12 + 16 + sh_bytes + 56) * n_vis
    else:
        # per visible Gaussian: index and tile count, parameters (means,
        # scales, rotation, logit, SH) and the 40-byte screen-space gradient
        # read; parameter gradients written
        pbytes = 12 + 12 + 16 + 4 + sh_bytes
        byts = (8 + pbytes + 40 + pbytes) * n_vis
    ach = byts / (ms / 1e3) / 1e9
    tr = pmc_traffic(kernel, src)
    return {"bound": "hbm", "kernel": kernel, "achieved": ach, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": tr,
            "algorithmic_bytes": byts, "working_set_bytes": byts}


if __name__ == "__main__":
    main()
