"""Synthetic stand-ins for the paper's per-partition training workloads.

The paper trains on isosurface point clouds of three simulation/scan
datasets (Sec. III) from 448 orbital training images (Sec. III, Sec. II
"Camera Setup"), with targets and background masks rendered per partition
(Sec. II "Image Rendering and Masking").  None of those datasets exist here;
these builders produce seeded scenes of the same structure:

* ``realistic_partition``  a Richtmyer-Meshkov-like mixing layer with
  droplets/bubbles, 1M training Gaussians, 64 orbital views at 1920x1080.
  Targets are renders of a denser reference set of surface-aligned discs
  (opacity 0.9) through the library's own forward pass; the background mask
  is where the reference covers at least half of the pixel (1 - T >= 0.5).
* ``tiny_partition``       the bumpy-sphere field on a 64^3 grid, 4,096
  Gaussians, 16 views at 128x128 (targets supplied by the caller).
* ``highres_partition``    one eighth of a ~106.7M-Gaussian scene: the
  bumpy-sphere field on a 2048^3 grid, the x, y, z >= 0 octant padded by
  2-voxel ghost cells across its three internal faces (Sec. II, partitioning
  with ghost cells), 13.3M Gaussians, 64 orbital views at 3840x2160; its
  reference set is the octant's share of the full scene, sampled with its
  own seed.
"""
from __future__ import annotations

import math

import numpy as np

from . import scene

REALISTIC = dict(n=1_000_000, n_ref=4_000_000, views=64, width=1920, height=1080, seed=2)
TINY = dict(n=4096, n_ref=32768, views=16, width=128, height=128, grid=64, seed=1)
HIGHRES = dict(n=13_300_000, n_ref=13_300_000, views=64, width=3840, height=2160, grid=2048,
               ghost=2, seed=3)


def init_gaussians(points, normals, opacity=0.1, knn_scale=None):
    """Plain initialisation: isotropic scale = mean distance to the 3 nearest
    neighbours, identity rotation, opacity 0.1, colour from the normal."""
    d = scene.knn_mean_distance(points, 3) if knn_scale is None else knn_scale
    return scene.gaussians_from_points(points, normals, np.maximum(d, 1e-6), opacity=opacity)


def reference_discs(points, normals, spacing):
    """Surface-aligned discs (scale d, d, 0.1 d along the normal), opacity 0.9."""
    return scene.gaussians_from_points(points, normals, spacing, opacity=0.9, thin=0.1)


def realistic_partition(cfg=None, with_reference=True):
    cfg = dict(REALISTIC, **(cfg or {}))
    mi = scene.MixingInterface(seed=cfg["seed"])
    pts, nrm = _chunked_sample(mi, cfg["n"], cfg["seed"] + 10)
    if cfg.get("order", "morton") == "morton":
        perm = scene.morton_order(pts)
        pts, nrm = pts[perm], nrm[perm]
    params = init_gaussians(pts, nrm)
    cams = scene.orbit_cameras(cfg["views"], cfg["width"], cfg["height"],
                               fov_x_deg=cfg.get("fov", 50.0))
    out = dict(params=params, cams=cams, cfg=cfg, points=pts, normals=nrm)
    if with_reference:
        rp, rn = _chunked_sample(mi, cfg["n_ref"], cfg["seed"] + 100)
        out["reference"] = reference_discs(rp, rn, scene.knn_mean_distance(rp, 3))
    return out


def _chunked_sample(mi, n, seed, chunk=500_000):
    rng = np.random.default_rng(seed)
    pts, nrm = [], []
    left = n
    while left > 0:
        k = min(chunk, left)
        p, q = mi.sample(k, int(rng.integers(1 << 31)))
        pts.append(p); nrm.append(q)
        left -= k
    return np.concatenate(pts), np.concatenate(nrm)


def octant_box(grid, ghost, lo=-1.0, hi=1.0):
    """The x, y, z >= 0 octant of [lo, hi]^3, padded by ``ghost`` voxels of a
    grid^3 sampling (spacing (hi - lo) / (grid - 1)) across the three faces it
    shares with the other octants."""
    g = ghost * (hi - lo) / (grid - 1)
    return ((-g, -g, -g), (hi, hi, hi))


def _knn_scale(points, device):
    """3-NN mean distance, on the device (gs_knn) when one is given."""
    if device is None:
        return scene.knn_mean_distance(points, 3)
    import torch
    from . import ops
    pd = torch.as_tensor(np.ascontiguousarray(points.T, np.float32)).to(device)
    d = ops.knn_mean_distance(pd, 3).cpu().numpy().astype(np.float64)
    del pd
    return d


def highres_partition(cfg=None, with_reference=True, device=None):
    """The high-resolution octant partition; device = a torch device runs the
    k-NN scale of the initialisation and of the reference discs there."""
    cfg = dict(HIGHRES, **(cfg or {}))
    box = octant_box(cfg["grid"], cfg["ghost"])
    f = scene.field_sphere_sines
    pts, nrm = scene.sample_surface(f, cfg["n"], cfg["grid"], seed=cfg["seed"], box=box)
    perm = scene.morton_order(pts)
    pts, nrm = pts[perm], nrm[perm]
    params = init_gaussians(pts, nrm, knn_scale=_knn_scale(pts, device))
    cams = scene.orbit_cameras(cfg["views"], cfg["width"], cfg["height"],
                               fov_x_deg=cfg.get("fov", 50.0))
    out = dict(params=params, cams=cams, cfg=cfg, points=pts, normals=nrm, box=box)
    if with_reference:
        rp, rn = scene.sample_surface(f, cfg["n_ref"], cfg["grid"], seed=100 + cfg["seed"], box=box)
        out["reference"] = reference_discs(rp, rn, _knn_scale(rp, device))
    return out


def tiny_partition(cfg=None):
    cfg = dict(TINY, **(cfg or {}))
    pts, nrm = scene.sample_surface(scene.field_sphere_sines, cfg["n"], cfg["grid"], seed=cfg["seed"])
    params = init_gaussians(pts, nrm)
    rp, rn = scene.sample_surface(scene.field_sphere_sines, cfg["n_ref"], cfg["grid"],
                                  seed=100 + cfg["seed"])
    ref = reference_discs(rp, rn, scene.knn_mean_distance(rp, 3))
    cams = scene.orbit_cameras(cfg["views"], cfg["width"], cfg["height"])
    return dict(params=params, reference=ref, cams=cams, cfg=cfg, points=pts, normals=nrm)


def render_targets_gpu(reference, cams, tile=(16, 16), device="cuda", bg=(0.0, 0.0, 0.0)):
    """Render every view of a reference set with the library's forward pass
    over background colour bg.  Returns (targets [V,3,H,W] f32, masks [V,H,W]
    u8) on the device."""
    import torch
    from . import ops
    n = reference["opacity_logit"].shape[0]
    W, H = int(cams[0]["width"]), int(cams[0]["height"])
    dev = {k: torch.as_tensor(np.ascontiguousarray(v, np.float32)).to(device)
           for k, v in reference.items()}
    gst = ops.gaussians_struct(dev)
    cams_dev = ops.Views.cams_to_device(cams, device)
    views = ops.Views.single(n, cams[:1], device)
    bufs = ops.RasterBuffers(views, W, H, tile, dup_capacity=4 * n)
    targets = torch.empty((len(cams), 3, H, W), dtype=torch.float32, device=device)
    masks = torch.empty((len(cams), H, W), dtype=torch.uint8, device=device)
    for v in range(len(cams)):
        views.use_cameras(cams_dev[v:v + 1])
        bufs.render_checked(gst, tuple(bg))
        targets[v].copy_(bufs.image[0])
        masks[v].copy_((bufs.T_final[0] <= 0.5).to(torch.uint8))
    torch.cuda.synchronize()
    return targets, masks
