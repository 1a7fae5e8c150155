"""Time to a masked-PSNR target on one GPU.

Three arms on the same partitions, views and targets:

* plain    - each partition trained on its own by the plain trainer (one
             view per step, the method's per-partition training, Sec. II
             "Parallel Training"), partitions one after another;
* batched  - all partitions x ``views_per_part`` views per step in one launch
             per stage (LPT tile order, chunked backward) with captured steps;
* learned  - the plain trainer started from the learned initialisation.

Partitions are x-slabs of the bumpy-sphere field with ghost margins (Sec. II
"Data Partitioning": the dataset is cut into partitions padded with ghost
cells); every partition sees the same orbital cameras (Sec. II "Camera
Setup") and gets targets and background masks rendered from its own
reference set (Sec. II "Image Rendering and Masking").

Timing: the training wall clock, evaluation excluded (the clock pauses while
the mean masked PSNR over all views is computed every ``eval_every`` steps),
initialisation (k-NN, features, network) included in every arm.  A
partition's time is taken at its first evaluation at or above the target.

    python -m paper_2509_12138_amd.ttt probe   [--scale S]
    python -m paper_2509_12138_amd.ttt batched [--scale S] [--target 35]
    python -m paper_2509_12138_amd.ttt learned [--scale S] [--target 35]
    python -m paper_2509_12138_amd.ttt adc     [--scale S] [--steps K]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import scene, workloads

SLAB_COUNTS = (500_000, 800_000, 1_200_000, 1_500_000, 2_000_000, 2_500_000, 3_000_000, 4_500_000)
GRID = 512               # sampling grid over [-1, 1]^3
GHOST_VOXELS = 2


def log(*a):
    # progress goes to stderr: stdout carries the JSON results only
    print("[ttt]", *a, file=sys.stderr, flush=True)


SURFACE_EXTENT = 0.56    # the isosurface |x| = 0.5 +- 0.05 lies inside [-0.56, 0.56]^3


def slab_part(x0, x1, n, seed, ref_factor=2.0, grid=GRID, ghost_voxels=GHOST_VOXELS):
    """One x-slab [x0, x1) of the bumpy-sphere isosurface padded by a ghost
    margin of ghost_voxels grid voxels, sampled at n points, plus its
    ref_factor-denser reference."""
    ghost = ghost_voxels * 2.0 / grid
    box = ((x0 - ghost, -1.0, -1.0), (x1 + ghost, 1.0, 1.0))
    pts, nrm = _z_order(*scene.sample_surface(scene.field_sphere_sines, int(n), grid, seed=seed,
                                              box=box))
    rp, rn = scene.sample_surface(scene.field_sphere_sines, int(n * ref_factor), grid,
                                  seed=seed + 50, box=box)
    return dict(points=pts, normals=nrm, ref_points=rp, ref_normals=rn, x_range=(x0, x1))


def _z_order(pts, nrm):
    """The sampled points (the future Gaussians) in Z-order of position."""
    perm = scene.morton_order(pts)
    return pts[perm], nrm[perm]


def slab_partitions(counts=SLAB_COUNTS, seed=4, ref_factor=2.0, grid=GRID,
                    ghost_voxels=GHOST_VOXELS):
    """The bumpy-sphere isosurface cut into len(counts) equal-width x-slabs
    over its extent, each padded by a ghost margin of GHOST_VOXELS voxels
    beyond its faces and sampled at exactly its listed point count (so the
    partitions' densities and workloads are uneven), plus a reference set
    ref_factor times denser in the same padded slab.  Returns per partition
    points / normals / ref_points / ref_normals ([n,3] float64)."""
    P = len(counts)
    edges = np.linspace(-SURFACE_EXTENT, SURFACE_EXTENT, P + 1)
    out = []
    for p in range(P):
        out.append(slab_part(float(edges[p]), float(edges[p + 1]), counts[p], seed * 100 + p,
                             ref_factor, grid, ghost_voxels))
        log(f"slab {p}: {counts[p]} points sampled")
    return out


def slab_faces(P):
    """x of the P - 1 interior faces between the equal-width slabs."""
    return np.linspace(-SURFACE_EXTENT, SURFACE_EXTENT, P + 1)[1:-1]


def prepare(parts, cams, device="cuda", bg=(0.0, 0.0, 0.0)):
    """Reference discs -> targets and masks on the device, per partition
    (disc spacing from the library's k-NN on the device)."""
    from . import ops
    for part in parts:
        rp = torch.as_tensor(np.ascontiguousarray(part["ref_points"].T, np.float32)).to(device)
        d = ops.knn_mean_distance(rp, 3).cpu().numpy().astype(np.float64)
        del rp
        ref = workloads.reference_discs(part["ref_points"], part["ref_normals"], d)
        part["targets"], part["masks"] = workloads.render_targets_gpu(ref, cams, device=device,
                                                                      bg=bg)
        part["n"] = len(part["points"])
    return parts


def plain_params(part, device="cuda"):
    """Plain initialisation on the device (timed by the caller)."""
    from . import learned_init
    pts = torch.as_tensor(np.ascontiguousarray(part["points"].T, np.float32)).to(device)
    nrm = torch.as_tensor(np.ascontiguousarray(part["normals"].T, np.float32)).to(device)
    return learned_init.plain_init(pts, nrm), pts, nrm


def run_plain(part, cams, target, max_steps, eval_every, init="plain", mlp=None, plan=None,
              seed=0, device="cuda"):
    """Train one partition with the plain trainer until the target.
    Returns dict(seconds, steps, psnr, history, init_seconds, init_kind)."""
    from . import learned_init
    from .train import PlainTrainer
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if init == "learned":
        pts = torch.as_tensor(np.ascontiguousarray(part["points"].T, np.float32)).to(device)
        nrm = torch.as_tensor(np.ascontiguousarray(part["normals"].T, np.float32)).to(device)
        params, kind = learned_init.choose_init(mlp, pts, nrm)
    else:
        params, _, _ = plain_params(part, device)
        kind = "plain"
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    tile, sched, chunk, nw, det = plan or ((16, 16), "lpt", 64, 4, True)
    tr = PlainTrainer(params, cams, part["targets"], part["masks"], tile=tile, schedule=sched,
                      chunk=chunk, fwd_waves=nw, deterministic=det)
    tr.fit_capacity(views=range(0, len(cams), max(1, len(cams) // 8)))
    def progress(step, t, p):
        if (step // eval_every) % 10 == 0 or p >= target:
            log(f"plain step {step}: {t:.2f} s, psnr {p:.2f}")

    hist = tr.train(max_steps, order_seed=1000 + seed, eval_every=eval_every, target_psnr=target,
                    log=progress)
    reached = [h for h in hist if h[2] is not None and h[2] >= target]
    last = [h for h in hist if h[2] is not None]
    out = dict(init_seconds=t_init, init_kind=kind,
               history=[(int(s), float(t), float(p)) for s, t, p in last])
    if reached:
        out.update(seconds=t_init + reached[0][1], steps=reached[0][0], psnr=reached[0][2])
    else:
        out.update(seconds=None, steps=max_steps, psnr=last[-1][2] if last else None)
    out["trainer"] = tr
    return out


def run_batched(parts, cams, target, max_steps, eval_every, views_per_part=4, plan=None,
                device="cuda"):
    """All partitions in one batched trainer until every one reaches its
    target (a number, or one per partition); per partition the time of its
    first evaluation at the target."""
    from .train import BatchedTrainer
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    inits = [plain_params(p, device)[0] for p in parts]
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    tile, sched, chunk, nw, det = plan or ((16, 16), "lpt", 64, 4, True)
    bp = [dict(params={k: v.cpu().numpy() for k, v in ini.items()}, targets=p["targets"],
               masks=p["masks"]) for ini, p in zip(inits, parts)]
    tr = BatchedTrainer(bp, cams, views_per_part=views_per_part, tile=tile, schedule=sched,
                        chunk=chunk, fwd_waves=nw, deterministic=det, order_seed=7)
    tr.fit_capacity()
    tr.prepare()                  # graph capture is set-up, outside the clock
    P = len(parts)
    targets = list(target) if np.ndim(target) else [float(target)] * P
    reached = [None] * P
    hist = []
    train_time = 0.0
    rng = np.random.default_rng(11)
    order = []
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for s in range(max_steps):
        if not order:
            order = list(rng.permutation(tr.G))
        tr.step(order.pop())
        if (s + 1) % eval_every == 0:
            torch.cuda.synchronize()
            train_time += time.perf_counter() - t1
            tr.check()
            ps = tr.evaluate()
            hist.append((s + 1, train_time, [float(x) for x in ps]))
            log(f"batched step {s + 1}: {train_time:.2f} s, psnr min {ps.min():.2f} "
                f"mean {ps.mean():.2f}")
            for p in range(P):
                if reached[p] is None and ps[p] >= targets[p]:
                    reached[p] = (s + 1, t_init + train_time, float(ps[p]))
            if all(r is not None for r in reached):
                break
            torch.cuda.synchronize()
            t1 = time.perf_counter()
    return dict(init_seconds=t_init, reached=reached, history=hist, trainer=tr)


def _cams(views, width, height):
    return scene.orbit_cameras(views, width, height)


def cmd_probe(a):
    """Masked PSNR against training steps of the plain trainer: the octant
    partition of the bumpy-sphere field (scale x 4M Gaussians) or the
    1M-Gaussian mixing-layer partition (--field mixing)."""
    if a.field == "mixing":
        wl = workloads.realistic_partition(dict(n=int(1_000_000 * a.scale),
                                                n_ref=int(4_000_000 * a.scale)))
        cams = wl["cams"]
        part = dict(points=wl["points"], normals=wl["normals"], n=len(wl["points"]))
        part["targets"], part["masks"] = workloads.render_targets_gpu(wl["reference"], cams)
    else:
        cams = _cams(a.views, a.width, a.height)
        part = prepare([octant_partition(int(4_000_000 * a.scale), seed=5,
                                         ref_factor=a.ref_factor)], cams)[0]
    log(f"probe: {a.field} partition, n={part['n']}")
    r = run_plain(part, cams, a.target, a.steps, a.eval_every, plan=a.plan)
    for s, t, p in r["history"]:
        log(f"plain step {s}: {t:.2f} s psnr {p:.2f}")
    print(json.dumps(dict(experiment="probe", field=a.field, n=part["n"], target=a.target,
                          seconds=r["seconds"], steps=r["steps"], history=r["history"])),
          flush=True)


def cmd_batched(a):
    """Batched vs plain on the uneven slabs.  The plain arm runs first: each
    partition alone, one view per step, until 35 dB or the step cap, with the
    batched arm's rasteriser plan ("same") and/or the untuned one-work-group-
    per-tile plan ("default").  A partition that does not reach the target
    within the cap in the first plain arm gets the target (its final PSNR -
    0.5 dB) in every arm.  The batched arm then trains all partitions
    together until each reaches its target."""
    counts = [int(c * a.scale) for c in SLAB_COUNTS]
    cams = _cams(a.views, a.width, a.height)
    log(f"sampling slabs {counts}")
    parts = prepare(slab_partitions(counts, ref_factor=a.ref_factor), cams)
    log("targets ready: " + ", ".join(str(p["n"]) for p in parts))
    plans = {"same": a.plan, "default": ((16, 16), "default", 0, 1, False)}
    arms, goals = {}, None
    for name in a.plain_plan.split(","):
        plain = []
        for i, part in enumerate(parts):
            goal = a.target if goals is None else goals[i]
            r = run_plain(part, cams, goal, a.plain_steps, a.eval_every * a.vpp,
                          plan=plans[name], seed=i)
            del r["trainer"]
            torch.cuda.empty_cache()
            if goals is None and r["seconds"] is None:
                goal = r["history"][-1][2] - 0.5
            t_goal = next((r["init_seconds"] + t for s_, t, p in r["history"] if p >= goal), None)
            r.update(goal=goal, seconds_to_goal=t_goal)
            log(f"plain ({name} plan) partition {i} (n={part['n']}): goal {goal:.2f} dB at "
                f"{t_goal} s")
            plain.append(r)
        if goals is None:
            goals = [r["goal"] for r in plain]
        tp = [r["seconds_to_goal"] for r in plain]
        arms[name] = dict(plan=list(plans[name]), partitions=plain,
                          seconds_all=sum(tp) if all(t is not None for t in tp) else None)
    rb = run_batched(parts, cams, goals, a.steps, a.eval_every, a.vpp, plan=a.plan)
    del rb["trainer"]
    torch.cuda.empty_cache()
    tb = [r[1] for r in rb["reached"]] if all(rb["reached"]) else None
    res = dict(experiment="batched_vs_plain", counts=[p["n"] for p in parts], target=a.target,
               goals=goals, plan=list(a.plan), views=a.views, width=a.width, height=a.height,
               views_per_part=a.vpp, eval_every=a.eval_every,
               plain_steps_cap=a.plain_steps, batched_steps_cap=a.steps,
               batched=dict(init_seconds=rb["init_seconds"], reached=rb["reached"],
                            history=rb["history"], seconds_all=max(tb) if tb else None),
               plain=arms)
    print(json.dumps(res), flush=True)


def cmd_adc(a):
    """The 3D-GS adaptive density control (clone / split / prune / opacity
    reset) on the mixing-layer partition: the plain trainer from a sparse
    initialisation (scale x 1M Gaussians on the surface), with and without
    density control, same views, targets and steps; masked PSNR and the
    number of Gaussians against steps and training time."""
    from .train import DensityControl, PlainTrainer
    wl = workloads.realistic_partition(dict(n=int(1_000_000 * a.scale)))
    cams = wl["cams"]
    targets, masks = workloads.render_targets_gpu(wl["reference"], cams)
    tile, sched, chunk, nw, det = a.plan
    out = dict(experiment="density_control", n0=int(len(wl["points"])), steps=a.steps,
               views=len(cams), arms={})
    for arm in ("plain", "density"):
        dc = DensityControl(seed=1) if arm == "density" else None
        tr = PlainTrainer(wl["params"], cams, targets, masks, tile=tile, schedule=sched,
                          chunk=chunk, fwd_waves=nw, deterministic=det, density=dc)
        tr.fit_capacity(views=range(0, len(cams), max(1, len(cams) // 8)))
        dens_t = []
        if dc is not None:
            plain_densify = tr.densify

            def timed():
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = plain_densify()
                torch.cuda.synchronize()
                dens_t.append(time.perf_counter() - t0)
                return r
            tr.densify = timed
        hist = []

        def record(s, t, p):
            hist.append((int(s), float(t), float(p), int(tr.n)))
            log(f"{arm} step {s}: {t:.2f} s, psnr {p:.2f}, n {tr.n}")
        # Gaussians grow during training: buffers grow on overflow instead of failing
        tr.train(a.steps, order_seed=77, eval_every=a.eval_every, log=record, check_every=10,
                 grow=True)
        out["arms"][arm] = dict(history=hist, densify_calls=len(dens_t),
                                densify_seconds_mean=float(np.mean(dens_t)) if dens_t else None,
                                capacity_grown=getattr(tr, "capacity_grown", 0))
        del tr
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def octant_partition(n, seed, ref_factor=2.0, grid=GRID):
    """The octant x, y, z >= 0 of the bumpy-sphere field padded by the ghost
    margin across its three internal faces (one of eight partitions)."""
    ghost = GHOST_VOXELS * 2.0 / grid
    box = ((-ghost, -ghost, -ghost), (1.0, 1.0, 1.0))
    pts, nrm = _z_order(*scene.sample_surface(scene.field_sphere_sines, int(n), grid, seed=seed,
                                              box=box))
    rp, rn = scene.sample_surface(scene.field_sphere_sines, int(n * ref_factor), grid,
                                  seed=seed + 100, box=box)
    return dict(points=pts, normals=nrm, ref_points=rp, ref_normals=rn)


def fitted_examples(part, cams, steps, plan, seed):
    """Fit a partition with the plain trainer, return (features, targets,
    plain-initialisation outputs, final psnr) of its Gaussians."""
    from . import learned_init
    r = run_plain(part, cams, 1e9, steps, steps, plan=plan, seed=seed)
    tr = r["trainer"]
    pts = torch.as_tensor(np.ascontiguousarray(part["points"].T, np.float32)).cuda()
    nrm = torch.as_tensor(np.ascontiguousarray(part["normals"].T, np.float32)).cuda()
    x, dbar = learned_init.features(pts, nrm)
    p = tr.params
    t = learned_init.targets(p["log_scale"], p["quat"], p["opacity_logit"], nrm, dbar)
    q = learned_init.plain_init(pts, nrm)
    y_plain = learned_init.targets(q["log_scale"], q["quat"], q["opacity_logit"], nrm, dbar)
    psnr = r["history"][-1][2] if r["history"] else None
    del tr, r
    torch.cuda.empty_cache()
    return x, t, y_plain, psnr


def cmd_learned(a):
    from . import learned_init
    cams = _cams(a.views, a.width, a.height)
    # training data: Gaussians fitted on the tiny configuration (4,096
    # Gaussians, 16 views at 128^2) and on an octant partition of the field
    tiny = workloads.tiny_partition()
    tiny_part = dict(points=tiny["points"], normals=tiny["normals"], n=len(tiny["points"]))
    tiny_part["targets"], tiny_part["masks"] = workloads.render_targets_gpu(tiny["reference"],
                                                                            tiny["cams"])
    xs, ts, ys = [], [], []
    x, t, yp, ps = fitted_examples(tiny_part, tiny["cams"], a.fit_steps,
                                   ((16, 16), "lpt", 64, 1, True), 1)
    xs.append(x); ts.append(t); ys.append(yp)
    log(f"tiny fitted: psnr {ps}")
    if a.fit_source == "highres":
        # the high-resolution partition: the octant of the field on a 2048^3
        # grid with ghost cells, 13.3M Gaussians, its own 64 views at 3840x2160
        n_hr = int(a.scale * workloads.HIGHRES["n"])
        hr = workloads.highres_partition(dict(n=n_hr, n_ref=n_hr), device="cuda")
        src = dict(points=hr["points"], normals=hr["normals"], n=len(hr["points"]))
        src["targets"], src["masks"] = workloads.render_targets_gpu(hr["reference"], hr["cams"])
        src_cams = hr["cams"]
        del hr
    else:
        src = prepare([octant_partition(int(a.scale * 13_300_000), seed=3,
                                        ref_factor=a.ref_factor)], cams)[0]
        src_cams = cams
    x, t, yp, ps = fitted_examples(src, src_cams, a.fit_steps, a.plan, 3)
    xs.append(x); ts.append(t); ys.append(yp)
    log(f"{a.fit_source} partition fitted (n={src['n']}, "
        f"{src_cams[0]['width']}x{src_cams[0]['height']}): psnr {ps}")
    del src
    x = torch.cat(xs); t = torch.cat(ts); yp = torch.cat(ys)
    # held-out tenth for the fallback rule
    nh = max(1, x.shape[0] // 10)
    g = torch.Generator(device="cpu").manual_seed(505)
    perm = torch.randperm(x.shape[0], generator=g).cuda()
    xh, th = x[perm[:nh]].contiguous(), t[perm[:nh]].contiguous()
    xt, tt = x[perm[nh:]], t[perm[nh:]]
    mlp = learned_init.InitMLP.random(seed=505, out_bias=tt.mean(0).cpu().numpy())
    mt = learned_init.MLPTrainer(mlp, xt, tt, lr=2e-3, batch=65536)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = mt.train(a.mlp_steps, log_every=max(1, a.mlp_steps // 5), log=log)
    torch.cuda.synchronize()
    mlp_seconds = time.perf_counter() - t0
    held = learned_init.evaluate_loss(mlp, xh, th)
    held_plain = float(learned_init.loss(yp[perm[:nh]].contiguous(), th)[0].item())
    use_mlp = math.isfinite(held) and held < held_plain
    log(f"network: {mlp_seconds:.1f} s, held-out loss {held:.4f} vs plain init {held_plain:.4f}"
        f" -> {'learned' if use_mlp else 'fallback to plain'}")
    # a new partition of the same field: an x-slab whose extent matches none
    # of the slab partitions, other seed; learned vs plain
    tgt = prepare([slab_part(-0.21, 0.26, int(a.scale * 4_000_000), seed=5,
                             ref_factor=a.ref_factor)], cams)[0]
    out = dict(experiment="learned_vs_plain", n=tgt["n"], target=a.target,
               mlp_train_seconds=mlp_seconds, mlp_history=hist, mlp_heldout_loss=held,
               plain_heldout_loss=held_plain)
    # both initialisations once, untimed, so neither arm's clock includes a
    # kernel's first load or the first allocation of its buffers
    _, pts_w, nrm_w = plain_params(tgt)
    learned_init.choose_init(mlp, pts_w, nrm_w)
    torch.cuda.synchronize()
    del pts_w, nrm_w
    for arm in ("plain", "learned"):
        init = arm if use_mlp else "plain"
        r = run_plain(tgt, cams, a.target, a.steps, a.eval_every, init=init, mlp=mlp, plan=a.plan,
                      seed=99)
        del r["trainer"]
        log(f"{arm}: {r['seconds']} s, {r['steps']} steps, psnr {r['psnr']}, init {r['init_kind']}")
        out[arm] = r
    print(json.dumps(out), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("experiment", choices=["probe", "batched", "learned", "adc"])
    ap.add_argument("--scale", type=float, default=1.0, help="multiplies every Gaussian count")
    ap.add_argument("--target", type=float, default=35.0)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--plain-steps", type=int, default=5000,
                    help="batched experiment: step cap of each partition's plain run")
    ap.add_argument("--eval-every", type=int, default=100)
    ap.add_argument("--views", type=int, default=64)
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1080)
    ap.add_argument("--vpp", type=int, default=4)
    ap.add_argument("--ref-factor", type=float, default=2.0)
    ap.add_argument("--field", choices=["sphere", "mixing"], default="sphere")
    ap.add_argument("--plain-plan", default="same",
                    help="batched experiment: plain arms to run, 'same', 'default' or "
                         "'same,default'")
    ap.add_argument("--fit-steps", type=int, default=2000)
    ap.add_argument("--fit-source", choices=["highres", "octant"], default="highres",
                    help="learned experiment: the second fitted partition, the 4K octant on a "
                         "2048^3 grid or an octant at the experiment's views")
    ap.add_argument("--mlp-steps", type=int, default=2000)
    ap.add_argument("--tile", default="16x16")
    ap.add_argument("--schedule", default="lpt")
    ap.add_argument("--chunk", type=int, default=64)
    ap.add_argument("--fwd-waves", type=int, default=4)
    ap.add_argument("--deterministic", type=int, default=1)
    a = ap.parse_args(argv)
    tw, th = (int(v) for v in a.tile.split("x"))
    a.plan = ((tw, th), a.schedule, a.chunk, a.fwd_waves, bool(a.deterministic))
    if not torch.cuda.is_available():
        sys.exit("ttt needs a GPU")
    dict(probe=cmd_probe, batched=cmd_batched, learned=cmd_learned, adc=cmd_adc)[a.experiment](a)


if __name__ == "__main__":
    main()
