"""Global reconstruction of a partitioned model and the seam ablation.

The method trains every spatial partition on its own and then merges the
splats of all partitions for the final rendering (Sec. II "Global
Reconstruction").  Ghost cells at the partition faces and background masks
in the per-partition loss are what keep the merged model free of gaps and
streaks at the seams (Sec. II "Data Partitioning", "Image Rendering and
Masking"; Sec. III-A and its figure).  This module merges trained partitions
and measures that claim on the uneven x-slabs of the bumpy-sphere field:

* the 8 slabs are sampled twice, with a ghost margin of 2 voxels of the
  512^3 grid and with none; each partition's targets and masks come from its
  own reference set, rendered over a white background (as isosurface images
  are), while the trainer composites over black (the 3D-GS default), so an
  unmasked loss can only match the partition's empty surroundings by
  growing white splats there;
* four arms train every partition with the plain trainer for a fixed number
  of steps: ghost cells on/off x masked/unmasked loss;
* the merged model of each arm (all partitions concatenated, nothing
  trimmed) is rendered from every view and compared with renders of a
  reference set sampled over the whole surface: PSNR over the foreground,
  over the seam band (foreground pixels whose surface lies within
  ``band`` of an interior face, found from a render of the global
  reference with its x coordinate as colour), and over the background.

    python -m paper_2509_12138_amd.reconstruct --scale 0.25 --steps 300

Metrics are evaluation only (torch reductions on rendered images); every
render goes through the library's project / bin-sort / forward calls.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import ops, scene, workloads
from . import ttt
from .train import mean_over_views

WHITE = (1.0, 1.0, 1.0)
BLACK = (0.0, 0.0, 0.0)


def merge(models):
    """Concatenate partition models (dicts of planar [C][n] parameter
    arrays) into one model: the global reconstruction."""
    keys = models[0].keys()
    return {k: torch.cat([torch.as_tensor(m[k]) for m in models], dim=-1).contiguous()
            for k in keys}


def position_colour(points, lo=-ttt.SURFACE_EXTENT, hi=ttt.SURFACE_EXTENT):
    """Degree-0 colour coefficients whose rendered grey level is the point's
    x mapped from [lo, hi] to [0, 1] (rendered colour = C0 f + 1/2)."""
    u = np.clip((points[:, 0] - lo) / (hi - lo), 0.0, 1.0)
    f = (u - 0.5) * 2.0 * np.sqrt(np.pi)
    return np.ascontiguousarray(np.tile(f, (3, 1)), np.float32)


def seam_band(xmap, cover, faces, band):
    """Foreground pixels whose surface x (xmap) lies within band of a face."""
    d = torch.full_like(xmap, float("inf"))
    for f in faces:
        d = torch.minimum(d, (xmap - float(f)).abs())
    return cover & (d <= band)


def render_views(params, cams, bg, tile=(16, 16), device="cuda"):
    """Yield (view, image [3,H,W], T_final [H,W]) of a model for every camera."""
    from . import ops
    dev = {k: torch.as_tensor(v).to(device).float().contiguous() for k, v in params.items()}
    n = dev["opacity_logit"].shape[-1]
    W, H = int(cams[0]["width"]), int(cams[0]["height"])
    gst = ops.gaussians_struct(dev)
    cams_dev = ops.Views.cams_to_device(cams, device)
    views = ops.Views.single(n, cams[:1], device)
    bufs = ops.RasterBuffers(views, W, H, tile, dup_capacity=4 * n)
    for v in range(len(cams)):
        views.use_cameras(cams_dev[v:v + 1])
        bufs.render_checked(gst, tuple(bg))
        yield v, bufs.image[0], bufs.T_final[0]


def evaluate(model, cams, glob, band):
    """Masked PSNR (gs_masked_psnr, clamped images) of a merged model against
    the global reference renders over three regions of every view: the
    foreground, the seam band and the background; each region's value is the
    mean over the views in which it is not empty."""
    W, H = int(cams[0]["width"]), int(cams[0]["height"])
    psnr = ops.PsnrBuffers(1, H, W)
    vals = {k: [] for k in ("foreground", "seam", "background")}
    for v, img, _ in render_views(model, cams, WHITE):
        fg = glob["masks"][v:v + 1].contiguous()
        regions = dict(foreground=fg, seam=glob["seam"][v:v + 1].to(torch.uint8).contiguous(),
                       background=(fg == 0).to(torch.uint8))
        for k, m in regions.items():
            vals[k].append(float(psnr(img.unsqueeze(0), glob["targets"][v:v + 1], m)[0]))
    out = {}
    for k, vs in vals.items():
        r = mean_over_views(vs)
        out[k] = None if math.isnan(r) else r
    return out


def global_reference(n_ref, cams, band, seed=977):
    """Targets, masks and seam bands of a reference set sampled over the
    whole surface (white background)."""
    rp, rn = scene.sample_surface(scene.field_sphere_sines, int(n_ref), ttt.GRID, seed=seed)
    d = workloads._knn_scale(rp, "cuda")
    ref = workloads.reference_discs(rp, rn, d)
    targets, masks = workloads.render_targets_gpu(ref, cams, bg=WHITE)
    # x of the visible surface per pixel: render x as grey level, divide out
    # the coverage
    pos = dict(ref, color=position_colour(rp))
    faces = ttt.slab_faces(len(ttt.SLAB_COUNTS))
    seam = torch.zeros_like(masks, dtype=torch.bool)
    E = ttt.SURFACE_EXTENT
    for v, img, T in render_views(pos, cams, (0.0, 0.0, 0.0)):
        cover = 1.0 - T
        xmap = img[0] / cover.clamp_min(1e-6) * (2 * E) - E
        seam[v] = seam_band(xmap, masks[v].bool(), faces, band)
    return dict(targets=targets, masks=masks, seam=seam)


def train_partition(part, cams, steps, use_mask, plan, seed, train_bg=BLACK):
    """Plain-trainer fit of one partition for a fixed number of steps;
    returns its parameters (device tensors) and its own masked PSNR."""
    from .train import PlainTrainer
    params, _, _ = ttt.plain_params(part)
    tile, sched, chunk, nw, det = plan
    tr = PlainTrainer(params, cams, part["targets"], part["masks"] if use_mask else None,
                      tile=tile, bg=train_bg, schedule=sched, chunk=chunk, fwd_waves=nw,
                      deterministic=det)
    tr.fit_capacity(views=range(0, len(cams), max(1, len(cams) // 8)))
    tr.train(steps, order_seed=2000 + seed)
    tr.check()
    tr.masks = part["masks"]          # own-target PSNR is always the masked one
    own = tr.evaluate()
    out = {k: v.detach().clone() for k, v in tr.params.items()}
    del tr
    torch.cuda.empty_cache()
    return out, own


def run(a):
    counts = [int(c * a.scale) for c in ttt.SLAB_COUNTS]
    cams = ttt._cams(a.views, a.width, a.height)
    t0 = time.perf_counter()
    glob = global_reference(int(sum(counts) * a.ref_factor), cams, a.band)
    ttt.log(f"global reference: {time.perf_counter() - t0:.1f} s, seam band covers "
            f"{float(glob['seam'].float().mean()):.4f} of the pixels")
    arms = []
    for ghost in (ttt.GHOST_VOXELS, 0):
        t0 = time.perf_counter()
        parts = ttt.prepare(ttt.slab_partitions(counts, ref_factor=a.ref_factor,
                                                ghost_voxels=ghost), cams, bg=WHITE)
        ttt.log(f"slabs with {ghost} ghost voxels ready in {time.perf_counter() - t0:.1f} s")
        for use_mask in (True, False):
            models, own = [], []
            for i, part in enumerate(parts):
                m, ps = train_partition(part, cams, a.steps, use_mask, a.plan, seed=i,
                                        train_bg=WHITE if a.train_bg == "white" else BLACK)
                models.append(m)
                own.append(ps)
            res = evaluate(merge(models), cams, glob, a.band)
            arm = dict(ghost_voxels=ghost, masks=use_mask, partition_psnr=own, merged=res)
            ttt.log(f"ghost {ghost}, masks {use_mask}: merged {res}, partitions "
                    f"{np.round(own, 2).tolist()}")
            arms.append(arm)
            del models
            torch.cuda.empty_cache()
        del parts
        torch.cuda.empty_cache()
    print(json.dumps(dict(experiment="global_reconstruction", counts=counts, steps=a.steps,
                          views=a.views, width=a.width, height=a.height, band=a.band,
                          target_background="white", train_background=a.train_bg,
                          arms=arms)), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--scale", type=float, default=0.25, help="multiplies every slab count")
    ap.add_argument("--steps", type=int, default=300, help="training steps per partition")
    ap.add_argument("--views", type=int, default=64)
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1080)
    ap.add_argument("--ref-factor", type=float, default=2.0)
    ap.add_argument("--band", type=float, default=0.01, help="seam band half-width (world x)")
    ap.add_argument("--train-bg", choices=["black", "white"], default="black",
                    help="background the trainer composites over (targets are on white)")
    ap.add_argument("--tile", default="16x16")
    ap.add_argument("--schedule", default="lpt")
    ap.add_argument("--chunk", type=int, default=64)
    ap.add_argument("--fwd-waves", type=int, default=4)
    a = ap.parse_args(argv)
    tw, th = (int(v) for v in a.tile.split("x"))
    a.plan = ((tw, th), a.schedule, a.chunk, a.fwd_waves, False)
    if not torch.cuda.is_available():
        sys.exit("reconstruct needs a GPU")
    run(a)


if __name__ == "__main__":
    main()
