"""Shared helpers of the GPU parity tests (inputs from the scene module,
expected values from the oracle)."""
import math
import sys

import numpy as np

import oracle
from paper_2509_12138_amd import scene


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def to_dev(params, torch):
    return {k: torch.as_tensor(np.ascontiguousarray(v, np.float32)).cuda() for k, v in params.items()}


def rec_to_oracle(rec, tile_bbox, n_tiles):
    """Oracle-side SoA view of FP32 projected records [m, 12] (+ bboxes)."""
    rec = np.asarray(rec, np.float64)
    tb = np.asarray(tile_bbox, np.int64).astype(np.int32) & 0xFFFF
    return dict(mean2d=rec[:, 0:2].T.copy(), conic=rec[:, 2:5].T.copy(), depth=rec[:, 9].copy(),
                opacity=rec[:, 5].copy(), rgb=rec[:, 6:9].T.copy(),
                tile_bbox=np.ascontiguousarray(tb.T), valid=(np.asarray(n_tiles) > 0).astype(np.int32))


# Relative half-width of the oracle's decision bands (alpha thresholds,
# transmittance cut-off) where the GPU computes the projected records itself:
# the projection matches FP64 to 1e-5 relative on the conic and about 1e-4 px
# on the mean, which moves the exponent -q^T Q q / 2 of a footprint about a
# pixel wide by up to about 1e-3 near the 1/255 contour.
BAND_E2E = 1e-3


def grad_tolerance_check(g, r, term_mass, amb_mass, rel=1e-3, floor=0.01):
    """|g - r| <= rel * max(|r|, floor * A) + A_amb per element, where A is the
    oracle's term mass (sum over pixels of the magnitudes of the terms of
    dL/dalpha before they cancel) and A_amb the contribution of ambiguous
    pixels.  The floor is relative to the terms, not to the cancelled
    result: an exact FP32 replay of the kernels' transmittance recovery and
    accumulation (test_fp32_gradient_bound) uses about a tenth of this bound
    and breaks one relative to the result; returns (ok, worst ratio)."""
    bound = rel * np.maximum(np.abs(r), floor * term_mass) + amb_mass + 1e-12
    ratio = np.abs(g - r) / bound
    worst = float(ratio.max(initial=0.0))
    if worst > 1.0:
        i = np.unravel_index(np.argmax(ratio), ratio.shape)
        return False, (worst, dict(index=tuple(int(x) for x in i), got=float(g[i]), ref=float(r[i]),
                                   term_mass=float(term_mass[i]), amb_mass=float(amb_mass[i]),
                                   n_bad=int((ratio > 1).sum())))
    return True, worst


def masked_image_gradient(rng, H, W, S=2):
    """Seeded image gradient that is exactly zero where a loss mask would
    cut it: on 30% of the pixels and on a solid block (whole tiles)."""
    dI = rng.normal(size=(S, 3, H, W)).astype(np.float32)
    zero = rng.uniform(size=(S, 1, H, W)) < 0.3
    zero[:, :, H // 8:H // 2, W // 6:W // 2] = True
    return np.where(zero, np.float32(0), dI)


def surface_scene(n, seed, opacity=0.1):
    """n Gaussians on the bumpy-sphere isosurface with k-NN isotropic scales."""
    pts, nrm = scene.sample_surface(scene.field_sphere_sines, n, 64, seed=seed)
    d = scene.knn_mean_distance(pts, 3)
    return scene.gaussians_from_points(pts, nrm, d, opacity=opacity)


def perturbed(params, seed, amount=0.3):
    """Anisotropic, rotated, varied-opacity version of surface Gaussians."""
    rng = np.random.default_rng(seed)
    p = {k: v.copy() for k, v in params.items()}
    n = p["opacity_logit"].shape[0]
    p["log_scale"] = (p["log_scale"] + rng.normal(0, amount, (3, n))).astype(np.float32)
    p["quat"] = (p["quat"] + rng.normal(0, 0.5, (4, n))).astype(np.float32)
    p["opacity_logit"] = rng.normal(-0.5, 1.5, n).astype(np.float32)
    p["color"] = (p["color"] + rng.normal(0, 0.5, (3, n))).astype(np.float32)
    return p


def oracle_records(params, cams, W, H, tile):
    """Projected records of every view built by the oracle (its FP64
    projection rounded to FP32) in the library's record layout
    (mean2d, conic, opacity, rgb, depth, slot bits, 0; culled pairs zero but
    depth and slot), slot-major, plus per view the oracle-side dict of the
    same FP32 values.  Both sides then rasterise identical inputs, none of
    which comes from the GPU."""
    recs, tbs, nts, views = [], [], [], []
    for s, cam in enumerate(cams):
        o = oracle.project(params, scene.camera_dict(cam), tile)
        n = o["depth"].shape[0]
        valid = o["valid"].astype(bool) & (o["n_tiles"] > 0)
        rec = np.zeros((n, 12), np.float32)
        rec[:, 0:2] = o["mean2d"].T
        rec[:, 2:5] = o["conic"].T
        rec[:, 5] = o["opacity"]
        rec[:, 6:9] = o["rgb"].T
        rec[~valid, 0:9] = 0.0
        rec[:, 9] = o["depth"]
        rec[:, 10] = np.full(n, s, np.int32).view(np.float32)
        tb = np.ascontiguousarray(np.where(valid[None], o["tile_bbox"], 0).T
                                  .astype(np.uint16).view(np.int16))
        nt = np.where(valid, o["n_tiles"], 0).astype(np.int32)
        recs.append(rec); tbs.append(tb); nts.append(nt)
        views.append(rec_to_oracle(rec, tb, nt))
    return np.concatenate(recs), np.concatenate(tbs), np.concatenate(nts), views


def raster_records(bufs, rec, tb, nt, bg, torch):
    """Load given records into the buffers, then bin/sort and rasterise."""
    bufs.ensure_capacity(int(nt.astype(np.int64).sum()) + 1024)
    bufs.rec.copy_(torch.as_tensor(rec))
    bufs.tile_bbox.copy_(torch.as_tensor(tb))
    bufs.n_tiles.copy_(torch.as_tensor(nt))
    bufs.clear_status()
    bufs.bin_sort()
    st, req = bufs.check()
    # the support listing keeps at most the bbox tiles
    assert st == 0 and req <= int(nt.astype(np.int64).sum()), (st, req)
    bufs.order_tiles()
    bufs.raster_fwd(bg)
    torch.cuda.synchronize()


def oracle_lists(rec, tb, nt, slot, tile, W, H, S):
    """The oracle's sorted tile lists of FP32 records (rec [m,12], tb [m,4]
    u16 bits, nt [m]) with the pairs whose tile listing is ambiguous culled:
    returns (nt with those pairs at 0, keys, ids, ranges).  Give the GPU the
    returned nt so that both sides list the same pairs."""
    tx, ty = math.ceil(W / tile[0]), math.ceil(H / tile[1])
    tbi = np.asarray(tb).astype(np.int32).reshape(-1, 4) & 0xFFFF
    sup = oracle.sup_from_records(rec)
    *_, amb = oracle.bin_sort(tbi, nt, rec[:, 9], slot, tx, tx * ty, S, sup=sup, tile=tile,
                              details=True)
    nt = np.where(amb, 0, nt).astype(np.int32)
    keys, ids, ranges = oracle.bin_sort(tbi, nt, rec[:, 9], slot, tx, tx * ty, S, sup=sup,
                                        tile=tile)
    return nt, keys, ids, ranges


def decision_safe_mask(mask, r, target, tol=1e-4):
    """A loss mask [H,W] (uint8) with the pixels cut where FP32 and FP64 may
    take different discrete decisions: those the oracle's render marks
    ambiguous, and those where some channel of the oracle image lies within
    the image tolerance (1e-4) of the target, since there the sign of the
    L1 term's derivative is not fixed by an image that matches to 1e-4.
    Built from the oracle's render and the target only."""
    img = np.asarray(r["image"], np.float64)
    tgt = np.asarray(target, np.float64)
    near = (np.abs(img - tgt) <= tol).any(axis=0)
    keep = ~(np.asarray(r["ambiguous"]).astype(bool) | near)
    return (np.asarray(mask) != 0) & keep
