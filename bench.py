#!/usr/bin/env python3
"""Benchmark: one partition's 3D-GS training step on one MI355X.

Workload (the realistic single-partition configuration): a
Richtmyer-Meshkov-like mixing-layer isosurface with 1M FP32 Gaussians (SH
degree 0), 64 orbital views at 1920x1080 with background masks, batch of one
view per step.  A step runs the whole hot path through libgsmi:
project -> bin/sort -> raster fwd -> masked L1 + D-SSIM -> raster bwd ->
project bwd -> Adam.

Prints ONE JSON line.  value = fwd+bwd raster Mpix/s (pixels of a step's
image over the summed durations of the two rasteriser launches, HIP events
on the launch stream); ms_per_step / iters_per_s cover the whole step.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]

--workload highres times the high-resolution partition instead: the octant
(with 2-voxel ghost cells) of the bumpy-sphere isosurface on a 2048^3 grid,
13.3M Gaussians, 64 orbital views at 3840x2160; run it with and without
--recompute to compare the stored and recomputed backward (the line reports
the step's peak device memory and the bytes of stored raster state).

--workload batched times the batched uneven partitions: the bumpy-sphere
isosurface cut into 8 ghost-padded x-slabs of 0.5, 0.8, 1.2, 1.5, 2, 2.5, 3
and 4.5M Gaussians (16M), 4 views per partition per step at 1920x1080 (32
image slots), every stage one launch for all slots, steps replayed from HIP
graphs.  value = fwd+bwd raster Mpix/s over the 32 images of a step.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd raster Mpix/s; train iters/s at 1080p; secs to 35 dB PSNR vs plain"
PEAK_VALU_OPS = 256 * 4 * 16 * 2.4e9          # FP32 lane-ops/s without packed math
PEAK_HBM = 8.0e12
# algorithmic VALU issue slots per blended (pixel, Gaussian) pair, the work
# an exact rasteriser cannot avoid (transcendentals count 4); see the design
# notes for the derivation
OPS_PER_EVAL_FWD = 22
OPS_PER_EVAL_BWD = 50
EVENT_EVERY = 5


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--tile", default=None, help="fix the bin tile (e.g. 16x16); default autotuned")
    ap.add_argument("--schedule", default=None, help="default | lpt | persistent (default autotuned)")
    ap.add_argument("--chunk", type=int, default=None, help="backward chunk (0 = whole tiles)")
    ap.add_argument("--fwd-waves", type=int, default=None, help="forward waves per tile (1, 2, 4)")
    ap.add_argument("--deterministic", type=int, default=None,
                    help="1: per-entry gradient slots summed per pair instead of atomics")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--cached-plan", action="store_true",
                    help="reuse the plan the autotuner cached for this workload (no re-tuning)")
    ap.add_argument("--recompute", action="store_true")
    ap.add_argument("--small", action="store_true", help="tiny config (smoke use)")
    ap.add_argument("--workload", choices=["realistic", "highres", "batched"],
                    default="realistic",
                    help="realistic: 1M-Gaussian mixing layer at 1920x1080 (the headline); "
                         "highres: 13.3M-Gaussian octant at 3840x2160; batched: 8 uneven "
                         "slabs (16M Gaussians), 4 views each at 1920x1080 per step")
    ap.add_argument("--scale", type=float, default=1.0,
                    help="batched workload: multiplies every slab's Gaussian count")
    ap.add_argument("--sh-degree", type=int, default=0,
                    help="view-dependent colour of this degree, active from the first step "
                         "(the headline workload is degree 0)")
    ap.add_argument("--fov", type=float, default=50.0,
                    help="horizontal field of view of the orbit in degrees (the workload: 50); "
                         "narrower views draw part of the partition")
    ap.add_argument("--order", choices=["morton", "sampled"], default="morton",
                    help="storage order of the Gaussians: Z-order of their means, or the order "
                         "they were sampled in")
    ap.add_argument("--sparse-adam", action="store_true",
                    help="visible-only Adam (the headline workload uses the dense step)")
    ap.add_argument("--trained-steps", type=int, default=None,
                    help="also time the partition after this many training steps (default 2000 "
                         "for the headline workload, 0 = skip)")
    ap.add_argument("--ttt", type=int, default=None,
                    help="1: also measure the plain trainer's time to 35 dB masked PSNR from the "
                         "plain initialisation (default on for the headline workload)")
    ap.add_argument("--ttt-steps", type=int, default=2000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device copy 5 times (HBM counter scale)")
    return ap.parse_args()


def copy_calibration():
    """A plain copy of known size: 512 MiB read + 512 MiB written per launch,
    used to scale the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    src = torch.empty(128 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4,
                      "launches": 5}))


def cpu_baseline(params, cam, target_seconds):
    """Time the FP64 oracle's raster forward + backward on a pixel window of
    the same view (a bounded sample of the workload)."""
    import oracle
    from paper_2509_12138_amd import scene
    camd = scene.camera_dict(cam)
    W, H = int(cam["width"]), int(cam["height"])
    t0 = time.perf_counter()
    proj = oracle.project(params, camd)
    t_proj = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    d_image = rng.normal(size=(3, H, W))

    def run(side):
        x0, y0 = W // 2 - side // 2, H // 2 - side // 2
        win = (x0, y0, x0 + side, y0 + side)
        t = time.perf_counter()
        oracle.render(proj, W, H, window=win)
        oracle.render_bwd(proj, W, H, d_image, window=win)
        return time.perf_counter() - t

    # fixed cost (sorting) + per-pixel cost from two small windows, then a
    # window sized so that the timed sample takes about target_seconds
    t16, t32 = run(16), run(32)
    per_px = max((t32 - t16) / (32 * 32 - 16 * 16), 1e-9)
    fixed = max(t16 - per_px * 256, 0.0)
    side = int(max(16, min(768, ((target_seconds - fixed) / per_px) ** 0.5)))
    dt = run(side)
    return {
        "value": (side * side) / dt / 1e6,
        "unit": "Mpix/s",
        "cores": oracle.max_threads(),
        "kind": "oracle",
        "sample": f"raster fwd+bwd of a {side}x{side} pixel window at the centre of view 0 "
                  f"({W}x{H}, all {params['opacity_logit'].shape[0]} Gaussians; "
                  f"FP64 projection {t_proj:.2f}s not included), {dt:.1f}s",
    }


STAGES = ["project", "bin_sort", "raster_fwd", "loss", "zero", "raster_bwd", "project_bwd",
          "adam", "end"]


def timed_steps(tr, order, first, steps):
    """Time `steps` training steps on views order[first:first + steps].
    Stage events (HIP events on the launch stream) are recorded on every
    EVENT_EVERY-th step only: an event record costs about 5 us of queue gap,
    so nine per step would inflate the step time the wall clock measures.
    Returns (ms per step, mean stage ms, summed stage ms over the event
    steps, the views of the event steps)."""
    import torch
    timing = {}
    event_views = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        ev = s % EVENT_EVERY == 0
        tr.timing = timing if ev else None
        v = int(order[first + s])
        if ev:
            event_views.append(v)
        tr.step(v)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tr.timing = None
    mean, total = {}, {}
    for a, b in zip(STAGES[:-1], STAGES[1:]):
        d = [x.elapsed_time(y) for x, y in zip(timing[a], timing[b])]
        mean[a], total[a] = float(np.mean(d)), float(np.sum(d))
    return wall * 1000.0 / steps, mean, total, event_views


def fwd_kernel_name(tile, fwd_waves, sched="default", chunk=0):
    """The forward kernel(s) the library launches for this plan."""
    if sched.endswith("+split") and chunk:
        return f"k_raster_fwd_part<{tile[0]}, {tile[1]}>+k_raster_fwd_join<{tile[0]}, {tile[1]}>"
    return f"k_raster_fwd<{tile[0]}, {tile[1]}, {fwd_waves}>"


def bwd_kernel_name(tile, chunk, recompute, deterministic):
    """The backward kernel the library launches for this plan."""
    if chunk and not recompute:
        if tuple(tile) == (8, 8) and not deterministic:
            return f"k_raster_bwd_chunked_q<{tile[0]}, {tile[1]}>"   # quadrant lane groups
        return f"k_raster_bwd_chunked<{tile[0]}, {tile[1]}>"
    return f"k_raster_bwd<{tile[0]}, {tile[1]}, {'true' if recompute else 'false'}>"


def count_work(tr, views, W, H, tile):
    """Blended (pixel, Gaussian) pairs of each view, summed, with the
    forward's decisions (gs_raster_count) on the trainer's current state;
    also the list positions each pixel visits before it stops (the work of a
    rasteriser with no culling below the tile) and the drawn fraction."""
    import torch
    from paper_2509_12138_amd import ops as _ops
    rb = tr.bufs
    if rb.n_contrib is None:
        # the recomputing backward keeps no per-pixel state: render into
        # buffers that do
        rb = _ops.RasterBuffers(tr.views, W, H, tile, dup_capacity=tr.bufs.dup_capacity)
    blended = lists = drawn = 0.0
    tx = torch.arange(W, device="cuda") // tile[0]
    ty = torch.arange(H, device="cuda") // tile[1]
    tid = ty[:, None] * rb.tiles_x + tx[None, :]
    for v in views:
        tr.views.use_cameras(tr.cams[v:v + 1])
        rb.render_checked(tr.gst, tr.bg)
        blended += float(rb.count_blended()[0].to(torch.int64).sum())
        drawn += float((rb.n_tiles > 0).float().mean())
        nc = rb.n_contrib[0].to(torch.int64)
        rng_t = rb.ranges.to(torch.int64)
        tile_len = rng_t[:, 1] - rng_t[:, 0]
        stopped = rb.T_final[0] < 2e-4
        lists += float(torch.where(stopped, torch.minimum(nc + 1, tile_len[tid]),
                                   tile_len[tid]).sum())
    return dict(blended=blended, list_positions=lists, drawn=drawn / max(len(views), 1),
                views=len(views))


def trained_state(tr, order, first, steps, total, W, H, tile, ops_per_eval):
    """Train on to `total` steps (untimed), then time `steps` more steps the
    same way as at initialisation: the throughput of a trained partition,
    whose pixels stop earlier."""
    import torch
    n = total - first
    for s in range(max(n, 0)):
        tr.step(int(order[first + s]))
        if (s + 1) % 200 == 0:
            tr.check()
    tr.check()
    psnr = tr.evaluate()
    ms, stage, sums, views = timed_steps(tr, order, max(total, first), steps)
    tr.check()
    work = count_work(tr, views, W, H, tile)
    k = "raster_bwd" if ops_per_eval[0] == "bwd" else "raster_fwd"
    per = OPS_PER_EVAL_BWD if k == "raster_bwd" else OPS_PER_EVAL_FWD
    frac = work["blended"] * per / (sums[k] * 1e-3) / PEAK_VALU_OPS
    return {"after_steps": int(max(total, first)), "masked_psnr": round(psnr, 3),
            "value": round(W * H / ((stage["raster_fwd"] + stage["raster_bwd"]) * 1e-3) / 1e6, 3),
            "ms_per_step": round(ms, 4), "iters_per_s": round(1000.0 / ms, 3),
            "stage_ms": {a: round(b, 4) for a, b in stage.items()},
            "blended": work["blended"], "list_positions": work["list_positions"],
            "roofline_frac": round(frac, 4)}


def time_to_target(wl, targets, masks, plan, target=35.0, max_steps=2000, eval_every=50):
    """The plain trainer from the plain initialisation on the device (k-NN
    scale; its time counts) until the mean masked PSNR over all views
    reaches the target, evaluated every eval_every steps with the clock
    paused; at most max_steps steps."""
    import torch
    from paper_2509_12138_amd import ttt
    part = dict(points=wl["points"], normals=wl["normals"], targets=targets, masks=masks,
                n=len(wl["points"]))
    # the initialisation's kernels run once untimed on a subset, so that the
    # clock does not include their first load
    sub = dict(points=wl["points"][:4096], normals=wl["normals"][:4096])
    ttt.plain_params(sub)
    torch.cuda.synchronize()
    r = ttt.run_plain(part, wl["cams"], target, max_steps, eval_every, plan=plan, seed=2)
    del r["trainer"]
    hist = r["history"]
    out = {"target_db": target, "seconds": None if r["seconds"] is None else round(r["seconds"], 3),
           "steps": int(r["steps"]), "init_seconds": round(r["init_seconds"], 4),
           "final_psnr": round(hist[-1][2], 3) if hist else None,
           "max_steps": max_steps, "eval_every": eval_every,
           "curve": [(int(s), round(t, 3), round(p, 2)) for s, t, p in hist[:: max(1, len(hist) // 10)]]}
    if r["seconds"] is None and hist:
        # not reached within the cap: the time to the final PSNR less 0.5 dB
        goal = hist[-1][2] - 0.5
        s_, t_, p_ = next(h for h in hist if h[2] >= goal)
        out["fallback"] = {"target_db": round(goal, 3), "steps": int(s_),
                           "seconds": round(r["init_seconds"] + t_, 3)}
    return out


# plans tried for the batched workload (tile, schedule, backward chunk,
# forward waves, deterministic gradient sums)
BATCHED_CANDIDATES = [
    ((16, 16), "lpt", 64, 4, False), ((8, 8), "lpt", 64, 1, False), ((16, 8), "lpt", 64, 2, False),
    ((8, 16), "lpt", 64, 2, False), ((32, 8), "lpt", 128, 4, False), ((16, 16), "lpt", 128, 4, False),
    ((8, 8), "lpt+split", 64, 1, False), ((8, 8), "lpt+split", 128, 1, False),
]


def batched_main(args):
    """The batched-partition workload: graph-replayed steps timed by the wall
    clock; stage times (and the raster rate) from eager steps of the same
    view groups with HIP events on the launch stream."""
    import torch
    from paper_2509_12138_amd import scene, ttt
    from paper_2509_12138_amd.train import BatchedTrainer
    scale = 0.02 if args.small else args.scale
    counts = [int(c * scale) for c in ttt.SLAB_COUNTS]
    W, H, V = (320, 180, 16) if args.small else (1920, 1080, 64)
    vpp = 4
    cams = scene.orbit_cameras(V, W, H)
    t0 = time.perf_counter()
    parts = ttt.prepare(ttt.slab_partitions(counts), cams)
    log(f"slabs and targets in {time.perf_counter() - t0:.1f}s")
    inits = [ttt.plain_params(p)[0] for p in parts]
    bp = [dict(params={k: v.cpu().numpy() for k, v in ini.items()}, targets=p["targets"],
               masks=p["masks"]) for ini, p in zip(inits, parts)]
    del inits
    tile = tuple(int(x) for x in (args.tile or "16x16").split("x"))
    sched = args.schedule or "lpt"
    chunk = 64 if args.chunk is None else args.chunk
    fwd_waves = args.fwd_waves or 4
    det = bool(args.deterministic)
    tr = BatchedTrainer(bp, cams, views_per_part=vpp, tile=tile, schedule=sched, chunk=chunk,
                        stored=not args.recompute, fwd_waves=fwd_waves, deterministic=det,
                        order_seed=7)
    plan_source = "fixed"
    if not args.no_autotune and args.tile is None:
        # the plan of the batched step, timed on eager steps of every candidate
        # (the step count and parameters are restored after each)
        saved = [t.clone() for d in (tr.params, tr.m, tr.v) for t in d.values()]
        step0 = tr.adam.step_dev.clone()
        best = None
        for cand in BATCHED_CANDIDATES:
            if args.recompute and cand[2]:
                continue
            tr.set_plan(*cand)
            for s in range(2):
                tr.step(s % tr.G, timing={})
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for s in range(4):
                tr.step((2 + s) % tr.G, timing={})
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 250.0
            tr.check()
            log(f"batched plan {cand}: {ms:.2f} ms/step (eager)")
            if best is None or ms < best[0]:
                best = (ms, cand)
        i = 0
        for d in (tr.params, tr.m, tr.v):
            for t in d.values():
                t.copy_(saved[i])
                i += 1
        tr.adam.step_dev.copy_(step0)
        tr.steps_done = 0
        del saved
        tile, sched, chunk, fwd_waves, det = best[1]
        tr.set_plan(*best[1])
        plan_source = "autotuner"
    need = tr.fit_capacity()
    tr.prepare()
    log(f"{tr.S} slots, {tr.G} view groups, max duplicates per step {need}; graphs captured")
    rng = np.random.default_rng(11)
    order = rng.permutation(np.arange(10 ** 5) % tr.G)
    for s in range(args.warmup):
        tr.step(int(order[s]))
    tr.check()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        tr.step(int(order[args.warmup + s]))
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1000.0 / args.steps
    tr.check()
    # stage times: eager steps with events over the next groups
    n_ev = min(args.steps, tr.G)
    timing = {}
    groups = [int(order[args.warmup + args.steps + i]) for i in range(n_ev)]
    for g in groups:
        tr.step(g, timing=timing)
    torch.cuda.synchronize()
    tr.check()
    mean, total = {}, {}
    # (project_bwd covers the projection backward fused with the Adam step)
    stages = [x for x in STAGES if x != "adam"]
    for a, b in zip(stages[:-1], stages[1:]):
        d = [x.elapsed_time(y) for x, y in zip(timing[a], timing[b])]
        mean[a], total[a] = float(np.mean(d)), float(np.sum(d))
    # blended pairs of exactly those groups, on the state the steps ended in
    blended = 0.0
    for g in groups:
        tr.views.use_cameras(tr.cams_g[g])
        tr.bufs.render_checked(tr.gst, tr.bg)
        blended += float(tr.bufs.count_blended().to(torch.int64).sum())
    coverage = float(tr.masks_g[groups].float().mean())
    k = "raster_bwd" if mean["raster_bwd"] >= mean["raster_fwd"] else "raster_fwd"
    per = OPS_PER_EVAL_BWD if k == "raster_bwd" else OPS_PER_EVAL_FWD
    achieved = blended * per / (total[k] * 1e-3)
    kname = (bwd_kernel_name(tile, chunk, args.recompute, False) if k == "raster_bwd"
             else fwd_kernel_name(tile, fwd_waves, sched, chunk))
    mpix = tr.S * W * H / ((mean["raster_fwd"] + mean["raster_bwd"]) * 1e-3) / 1e6
    out = {
        "metric": METRIC,
        "value": round(mpix, 3),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "iters_per_s": round(1000.0 / ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"batched uneven partitions: bumpy-sphere isosurface in 8 x-slabs with "
                         f"2-voxel ghost cells ({', '.join(str(c) for c in counts)} Gaussians, "
                         f"{sum(counts)} in all), {vpp} views per partition per step from "
                         f"{V} orbital views at {W}x{H}, masks, {tr.S} image slots per step, "
                         f"one launch per stage, graph-replayed steps"),
            "tile": f"{tile[0]}x{tile[1]}", "schedule": sched, "backward_chunk": chunk,
            "fwd_waves": fwd_waves, "deterministic_gradients": det, "plan_source": plan_source,
            "backward": "recompute" if args.recompute else "stored",
            "duplicates_per_step": need,
        },
        "stage_ms": {a: round(b, 4) for a, b in mean.items()},
        "stage_ms_source": f"{n_ev} eager steps with HIP events (the timed steps are graph replays)",
        "pairs": {"blended": blended, "steps": n_ev},
        "mask_coverage": round(coverage, 4),
        "roofline": {"kernel": kname, "bound": "alu", "achieved": achieved / 1e12,
                     "peak": PEAK_VALU_OPS / 1e12, "unit": "TOP/s",
                     "frac": achieved / PEAK_VALU_OPS, "traffic": None,
                     "units_per_launch": blended / n_ev,
                     "unit_desc": f"{per} FP32 VALU issue slots per blended (pixel, Gaussian)",
                     "launches": n_ev, "launch_ms": round(total[k] / n_ev, 4)},
    }
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a bounded sample ...")
        big = len(parts) - 1
        prm = {k: v for k, v in bp[big]["params"].items()}
        cb = cpu_baseline(prm, cams[0], args.cpu_seconds)
        cb["sample"] = f"partition {big} ({counts[big]} Gaussians): " + cb["sample"]
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs an MI355X (no GPU visible)", file=sys.stderr)
        sys.exit(3)
    if args.copy_calibration:
        copy_calibration()
        return
    from paper_2509_12138_amd import _lib, workloads
    from paper_2509_12138_amd.train import PlainTrainer
    _lib.load()
    if args.workload == "batched":
        batched_main(args)
        return
    highres = args.workload == "highres"
    if args.trained_steps is None:
        args.trained_steps = 0 if (highres or args.small) else 2000
    if args.ttt is None:
        args.ttt = 0 if (highres or args.small) else 1
    cfg = dict(n=20000, n_ref=80000, views=8, width=320, height=180) if args.small else {}
    cfg["fov"] = args.fov
    t0 = time.perf_counter()
    if highres:
        if args.small:
            cfg.update(n=200000, n_ref=200000, width=640, height=360)
        wl = workloads.highres_partition(cfg, device="cuda")
    else:
        cfg["order"] = args.order
        wl = workloads.realistic_partition(cfg)
    log(f"scene built in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    targets, masks = workloads.render_targets_gpu(wl["reference"], wl["cams"])
    log(f"targets rendered in {time.perf_counter() - t0:.1f}s; mask coverage "
        f"{float(masks.float().mean()):.3f}")
    cfgd = wl["cfg"]
    W, H = cfgd["width"], cfgd["height"]
    stored = not args.recompute

    def make(tile):
        return PlainTrainer(wl["params"], wl["cams"], targets, masks, tile=tile, stored=stored)

    tune_entry = None
    if args.no_autotune or (args.tile and args.schedule is not None and args.chunk is not None):
        plan = (tuple(int(x) for x in (args.tile or "16x16").split("x")), args.schedule or "default",
                args.chunk or 0, args.fwd_waves or 1, bool(args.deterministic))
    else:
        from paper_2509_12138_amd import autotune
        t0 = time.perf_counter()
        plan, tune_entry = autotune.tune(make, W, H, 1, cfgd["n"], stored=stored,
                                         views=list(range(0, cfgd["views"], max(1, cfgd["views"] // 8))),
                                         cache_path=os.path.join(ROOT, "_build", "autotune.json"),
                                         force=not args.cached_plan, log=log)
        log(f"autotuned plan {plan} in {time.perf_counter() - t0:.1f}s")
    tile, sched, chunk, fwd_waves, deterministic = plan
    if not stored:
        chunk = 0
    tr = PlainTrainer(wl["params"], wl["cams"], targets, masks, tile=tile, stored=stored,
                      schedule=sched, chunk=chunk, fwd_waves=fwd_waves,
                      deterministic=deterministic, sh_degree=args.sh_degree, sh_up_every=0,
                      sparse_adam=args.sparse_adam)
    need = tr.fit_capacity()
    log(f"max duplicates per view {need}, capacity {tr.bufs.dup_capacity}")
    rng = np.random.default_rng(1000 + 2)
    order = rng.permutation(np.arange(10 ** 6) % len(wl["cams"]))
    for s in range(args.warmup):
        tr.step(int(order[s]))
    tr.check()
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    ms_per_step, stage_ms, sums, timed_views = timed_steps(tr, order, args.warmup, args.steps)
    peak_mem = torch.cuda.max_memory_allocated()
    tr.check()
    b = tr.bufs
    state_bytes = sum(int(t.numel() * t.element_size()) for t in
                      (getattr(b, "T_final", None), getattr(b, "n_contrib", None),
                       getattr(b, "checkpoints", None) if b.chunk else None,
                       getattr(b, "chunk_items", None) if b.chunk else None) if t is not None)
    t_fwd, t_bwd = stage_ms["raster_fwd"], stage_ms["raster_bwd"]
    mpix = W * H / ((t_fwd + t_bwd) * 1e-3) / 1e6

    # algorithmic work of exactly the steps whose raster launches were
    # event-timed: their views' blended (pixel, Gaussian) pairs, counted with
    # the forward's decisions on the state the timed region ended in
    work = count_work(tr, timed_views, W, H, tile)
    coverage = float(masks[timed_views].float().mean())
    blended = work["blended"]
    drawn = work["drawn"]
    list_pairs = work["list_positions"]
    # the dominant single kernel is one of the two raster passes: the bin/sort
    # stage can take longer in all, but it is a chain of ~20 shorter launches
    dom = "raster_bwd" if t_bwd >= t_fwd else "raster_fwd"
    evals_fwd = evals_bwd = blended
    if dom == "raster_bwd":
        achieved = evals_bwd * OPS_PER_EVAL_BWD / (sums["raster_bwd"] * 1e-3)
        kname = bwd_kernel_name(tile, chunk, args.recompute, deterministic)
        if deterministic:
            kname += "+k_dup_reduce"          # both run inside the timed gs_raster_bwd call
        roof = {"kernel": kname, "bound": "alu", "achieved": achieved / 1e12,
                "peak": PEAK_VALU_OPS / 1e12, "unit": "TOP/s", "frac": achieved / PEAK_VALU_OPS,
                "traffic": None, "units_per_launch": evals_bwd / len(timed_views),
                "unit_desc": f"{OPS_PER_EVAL_BWD} FP32 VALU issue slots per blended (pixel, Gaussian)"}
    else:
        achieved = evals_fwd * OPS_PER_EVAL_FWD / (sums["raster_fwd"] * 1e-3)
        roof = {"kernel": fwd_kernel_name(tile, fwd_waves, sched, chunk), "bound": "alu",
                "achieved": achieved / 1e12,
                "peak": PEAK_VALU_OPS / 1e12, "unit": "TOP/s", "frac": achieved / PEAK_VALU_OPS,
                "traffic": None, "units_per_launch": evals_fwd / len(timed_views),
                "unit_desc": f"{OPS_PER_EVAL_FWD} FP32 VALU issue slots per blended (pixel, Gaussian)"}
    # HBM traffic of the dominant kernel from committed counter runs, only
    # while its source is unchanged since they were taken
    from paper_2509_12138_amd import traffic as _traffic
    plan_str = f"{tile[0]}x{tile[1]},{sched},{chunk},{fwd_waves},{int(deterministic)}"
    # (the committed counter runs cover the 1080p partition only)
    roof["traffic"] = None if highres else _traffic.lookup(
        os.path.join(ROOT, "paper_2509_12138_amd", "hbm_traffic.json"), roof["kernel"], plan_str)
    roof["launches"] = len(timed_views)
    roof["launch_ms"] = round(sums[dom] / len(timed_views), 4)
    roof["views"] = timed_views
    roof["mask_coverage"] = round(coverage, 4)
    if roof["traffic"]:
        # HBM rate of the dominant kernel: its counted bytes over this run's launch time
        roof["hbm_tbps"] = roof["traffic"] / (roof["launch_ms"] * 1e-3) / 1e12
        roof["hbm_frac"] = roof["hbm_tbps"] * 1e12 / PEAK_HBM
    # VALU, LDS and HBM rates from the committed counter passes of this plan
    # (per-dispatch counters over the same dispatches' durations), reported
    # while the kernel's source is unchanged
    from paper_2509_12138_amd import kcounters as _kc
    kc = None if highres else _kc.lookup(
        os.path.join(ROOT, "paper_2509_12138_amd", "kernel_counters.json"), roof["kernel"], plan_str)
    if kc:
        roof["counters"] = {k: kc.get(k) for k in ("mean_us", "valu_busy", "valu_lanes", "lds_tbps",
                                                   "lds_frac", "lds_busy", "lds_conflict",
                                                   "hbm_tbps", "hbm_frac")}
    out = {
        "metric": METRIC,
        "value": round(mpix, 3),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "iters_per_s": round(1000.0 / ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"high-resolution partition: octant of the bumpy-sphere isosurface on a "
                         f"{cfgd['grid']}^3 grid with {cfgd['ghost']}-voxel ghost cells, "
                         if highres else "single partition: mixing-layer isosurface, ")
                        + f"{cfgd['n']} Gaussians "
                        f"(SH {args.sh_degree}), {cfgd['views']} orbital views at {W}x{H}"
                        + (f" (field of view {args.fov:g} deg)" if args.fov != 50.0 else "")
                        + ", masks, batch 1 view",
            "optimizer": "sparse adam" if args.sparse_adam else "adam",
            "gaussian_order": "morton" if highres else args.order,
            "tile": f"{tile[0]}x{tile[1]}",
            "schedule": sched,
            "backward_chunk": chunk,
            "fwd_waves": fwd_waves,
            "deterministic_gradients": deterministic,
            "plan_source": "autotuner" if tune_entry else "fixed",
            "backward": "recompute" if args.recompute else "stored",
            "duplicates_per_view": need,
        },
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "memory": {"peak_allocated_bytes": int(peak_mem), "raster_state_bytes": state_bytes},
        "pairs": {"blended": blended, "list_positions": list_pairs, "drawn_gaussians": drawn,
                  "views": len(timed_views)},
        "mask_coverage": round(coverage, 4),
        "roofline": roof,
    }
    if args.trained_steps > 0:
        log(f"training on to {args.trained_steps} steps for the trained-state measurement ...")
        out["trained"] = trained_state(tr, order, args.warmup + args.steps, args.steps,
                                       args.trained_steps, W, H, tile,
                                       ("bwd" if dom == "raster_bwd" else "fwd",))
    if args.ttt:
        del tr
        torch.cuda.empty_cache()
        log("time to 35 dB of the plain trainer from the plain initialisation ...")
        out["time_to_35db"] = time_to_target(wl, targets, masks,
                                             (tile, sched, chunk, fwd_waves, deterministic),
                                             max_steps=args.ttt_steps)
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(wl["params"], wl["cams"][0], args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
