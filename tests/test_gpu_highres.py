"""Parity and finite differences at the high-resolution partition's full
size: the x, y, z >= 0 octant of the bumpy-sphere isosurface on a 2048^3 grid
with 2-voxel ghost cells, 13.3M Gaussians, one orbital view at 3840x2160.

* the projection of all 13.3M Gaussians, checked on 20,000 sampled ones
  against the oracle (which computes each Gaussian on its own);
* bin/sort of the oracle's records, bit-exact against the oracle's sort;
* 256 Gaussians drawn with seed 303 among those the view draws: the image on
  their footprints and their record gradients, with the per-pixel state
  stored (chunked backward, the benchmark's plan) and recomputed, against the
  oracle's window render and backward over the same FP32 records (built by
  the oracle, so both sides rasterise identical inputs);
* the oracle's analytic parameter gradients of the same 256 Gaussians
  (window backward + projection backward) against FP64 central differences
  of its forward on their footprints.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2509_12138_amd import scene, workloads
from _gpu_helpers import (grad_tolerance_check, oracle_lists, oracle_records, perturbed,
                          raster_records, say, to_dev)

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

W, H = 3840, 2160
TILE = (16, 16)
VIEW = 21
SAME_RECORD_BITS = 1 | 2 | 4 | 8
SUBSET_SEED = 303


@pytest.fixture(scope="module")
def hr(gpu):
    say("building the 13.3M-Gaussian 3840x2160 octant partition")
    wl = workloads.highres_partition(with_reference=False, device="cuda")
    assert (wl["cfg"]["width"], wl["cfg"]["height"]) == (W, H)
    params = perturbed(wl["params"], 9, amount=0.2)
    cam = wl["cams"][VIEW:VIEW + 1]
    say("oracle records")
    rec, tb, nt, views = oracle_records(params, cam, W, H, TILE)
    drawn = np.nonzero(nt > 0)[0]
    subset = np.sort(np.random.default_rng(SUBSET_SEED).choice(drawn, 256, replace=False))
    rng = np.random.default_rng(SUBSET_SEED + 1)
    dI = rng.normal(size=(3, H, W)).astype(np.float32).astype(np.float64)  # both sides' values
    return dict(params=params, cam=cam, rec=rec, tb=tb, nt=nt, o=views[0], subset=subset,
                dI=dI, n=params["opacity_logit"].shape[0])


def footprint(o, i):
    """Pixel window of Gaussian i's tile bbox (all the pixels it can touch)."""
    tx0, ty0, tx1, ty1 = (int(v) for v in o["tile_bbox"][:, i])
    return (tx0 * TILE[0], ty0 * TILE[1], min((tx1 + 1) * TILE[0], W), min((ty1 + 1) * TILE[1], H))


def window_records(o, win):
    """The records whose tile bbox meets the window's tiles, in index order
    (the oracle breaks depth ties by index, so a subset in order renders the
    window as the whole set does); returns (sub-dict, indices)."""
    x0, y0, x1, y1 = win
    tb = o["tile_bbox"]
    sel = (o["valid"] > 0) & (tb[0] <= (x1 - 1) // TILE[0]) & (tb[2] >= x0 // TILE[0]) & \
        (tb[1] <= (y1 - 1) // TILE[1]) & (tb[3] >= y0 // TILE[1])
    idx = np.nonzero(sel)[0]
    sub = {k: (v[..., idx].copy() if np.ndim(v) == 2 else v[idx].copy()) for k, v in o.items()}
    return sub, idx


def test_highres_projection_matches_oracle_on_sampled_gaussians(hr):
    from paper_2509_12138_amd import ops
    n = hr["n"]
    say(f"high-res projection n={n}")
    bufs = ops.RasterBuffers(ops.Views.single(n, hr["cam"]), W, H, TILE, dup_capacity=1024)
    bufs.project(ops.gaussians_struct(to_dev(hr["params"], torch)))
    torch.cuda.synchronize()
    rng = np.random.default_rng(17)
    sample = np.sort(rng.choice(n, 20000, replace=False))
    rec = bufs.rec[torch.as_tensor(sample).cuda()].cpu().numpy()
    tb = bufs.tile_bbox[torch.as_tensor(sample).cuda()].cpu().numpy().astype(np.int64) & 0xFFFF
    nt = bufs.n_tiles[torch.as_tensor(sample).cuda()].cpu().numpy()
    sub = {k: (v[..., sample] if v.ndim == 2 else v[sample]) for k, v in hr["params"].items()}
    o = oracle.project(sub, scene.camera_dict(hr["cam"][0]), TILE)
    kappa = 2 * np.log(np.maximum(255 * o["opacity"], 1e-300))
    hx = np.sqrt(np.maximum(kappa, 0) * o["cov2d"][0])
    hy = np.sqrt(np.maximum(kappa, 0) * o["cov2d"][2])
    edges = np.stack([o["mean2d"][0] - hx, o["mean2d"][0] + hx, o["mean2d"][1] - hy,
                      o["mean2d"][1] + hy])
    # FP32 error of m +/- h stays below 5e-4 px at 3840x2160 coordinates
    near = np.any(np.abs(edges - np.round(edges)) < 5e-4, axis=0) | \
        (np.abs(255 * o["opacity"] - 1) < 1e-4)
    assert near.mean() < 5e-3
    ok = ~near
    valid = o["valid"].astype(bool) & (o["n_tiles"] > 0)
    np.testing.assert_array_equal(nt[ok] > 0, valid[ok])
    both = ok & valid
    assert both.sum() > 2000
    np.testing.assert_array_equal(tb[both], o["tile_bbox"].T[both])
    np.testing.assert_allclose(rec[both, 0:2], o["mean2d"].T[both], rtol=1e-5, atol=5e-4)
    cscale = np.abs(o["conic"]).max(0)[both][:, None]
    assert np.all(np.abs(rec[both, 2:5] - o["conic"].T[both]) <= 1e-5 * cscale + 1e-9)
    np.testing.assert_allclose(rec[both, 5], o["opacity"][both], rtol=1e-5)
    np.testing.assert_allclose(rec[both, 6:9], o["rgb"].T[both], rtol=1e-5, atol=2e-6)
    np.testing.assert_allclose(rec[both, 9], o["depth"][both], rtol=1e-6)


def test_highres_bin_sort_bit_exact(hr):
    from paper_2509_12138_amd import ops
    n, rec, tb, nt = hr["n"], hr["rec"], hr["tb"], hr["nt"]
    say("high-res bin/sort")
    nt, keys, ids, ranges = oracle_lists(rec, tb, nt, np.zeros(n, np.int32), TILE, W, H, 1)
    K = len(ids)
    assert K > 2 * 10 ** 6
    for keep in (True, False):          # 64-bit (tile, depth) keys, or 32-bit tile keys
        bufs = ops.RasterBuffers(ops.Views.single(n, hr["cam"]), W, H, TILE, dup_capacity=1024,
                                 keep_keys=keep)
        raster_records(bufs, rec, tb, nt, (0.0, 0.0, 0.0), torch)
        assert int(bufs.check()[1]) == K and K < 0.9 * int(nt.astype(np.int64).sum())
        if keep:
            np.testing.assert_array_equal(bufs.keys[:K].cpu().numpy().view(np.uint64), keys)
        np.testing.assert_array_equal(bufs.ids[:K].cpu().numpy().view(np.uint32), ids)
        np.testing.assert_array_equal(bufs.ranges.cpu().numpy().view(np.uint32), ranges)
        del bufs


_oracle_windows = {}


def oracle_subset(hr):
    """Per subset Gaussian: its footprint, the oracle's window render and
    backward (complete for that Gaussian: the window holds all its pixels)."""
    if not _oracle_windows:
        o, dI = hr["o"], hr["dI"]
        for i in hr["subset"]:
            win = footprint(o, i)
            sub, idx = window_records(o, win)
            j = int(np.searchsorted(idx, i))
            f = oracle.render(sub, W, H, tile=TILE, window=win)
            b = oracle.render_bwd(sub, W, H, dI, tile=TILE, window=win, amb_bits=SAME_RECORD_BITS)
            g = np.concatenate([b["d_mean2d"][:, j], b["d_conic"][:, j], [b["d_opacity"][j]],
                                b["d_rgb"][:, j]])
            x0, y0, x1, y1 = win
            _oracle_windows[int(i)] = dict(win=win, image=f["image"][:, y0:y1, x0:x1].copy(),
                                           amb=f["ambiguity"][y0:y1, x0:x1].copy(), grad=g,
                                           term=b["term_mass"][:, j].copy(),
                                           amb_mass=b["amb_mass"][:, j].copy())
    return _oracle_windows


@pytest.mark.parametrize("stored,sched", [(True, "lpt"), (False, "lpt"), (True, "lpt+split")],
                         ids=["stored", "recompute", "split"])
def test_highres_raster_on_subset_footprints_matches_oracle(hr, stored, sched):
    from paper_2509_12138_amd import ops
    n = hr["n"]
    say(f"high-res raster, subset footprints, stored={stored} {sched}")
    bufs = ops.RasterBuffers(ops.Views.single(n, hr["cam"]), W, H, TILE, dup_capacity=1024,
                             store_state=stored)
    bufs.set_schedule(sched, chunk=64 if stored else 0, fwd_waves=4)
    raster_records(bufs, hr["rec"], hr["tb"], hr["nt"], (0.0, 0.0, 0.0), torch)
    bufs.zero_d_rec()
    bufs.raster_bwd(torch.as_tensor(hr["dI"][None].astype(np.float32)).cuda())
    torch.cuda.synchronize()
    sub_t = torch.as_tensor(hr["subset"]).cuda()
    drec = bufs.d_rec[sub_t].cpu().numpy().astype(np.float64)
    img = bufs.image[0].cpu().numpy()
    ref = oracle_subset(hr)
    got_g, ref_g, term, amb_m = [], [], [], []
    for k, i in enumerate(hr["subset"]):
        r = ref[int(i)]
        x0, y0, x1, y1 = r["win"]
        amb = (r["amb"] & SAME_RECORD_BITS) != 0
        err = np.abs(img[:, y0:y1, x0:x1] - r["image"])[:, ~amb]
        assert err.max(initial=0.0) <= 1e-4, (int(i), r["win"], err.max())
        got_g.append(drec[k]); ref_g.append(r["grad"]); term.append(r["term"])
        amb_m.append(r["amb_mass"])
    got_g, ref_g, term, amb_m = (np.array(a) for a in (got_g, ref_g, term, amb_m))
    assert np.mean(np.any(ref_g != 0, axis=1)) > 0.5      # occluded ones get none
    ok, worst = grad_tolerance_check(got_g, ref_g, term, amb_m)
    assert ok, worst
    for c in range(9):
        nr = np.linalg.norm(got_g[:, c] - ref_g[:, c]) / max(np.linalg.norm(ref_g[:, c]), 1e-30)
        assert nr <= 1e-3, (c, nr)


def test_highres_parameter_gradients_match_finite_differences(hr):
    """Central differences of L = sum(w * image) over each subset Gaussian's
    footprint, with its record re-projected in FP64 from the perturbed
    parameter and every other record held.  h = 1e-6 max(1, |theta|), except
    1e-7 max(1, |theta|) for the mean: at this resolution a unit move of the
    mean shifts the footprint by about 1650 px, so a step of 1e-6 moves it by
    1.6e-3 px and the truncation error of the difference reaches 1e-5
    relative.  A perturbation that changes a discrete decision (a pixel's
    contributor or blend count, the Gaussian's tile bbox, its place in the
    depth order) is rejected and counted.  Bound: 1e-5 relative, plus 1e-6 of
    the Gaussian's largest gradient, plus 2e-8: the rounding of the two
    window sums (about sqrt(3000) FP64 ulps of terms below 1) divided by
    2h = 2e-7 is about 1e-8 for the mean."""
    say("high-res FD on the 256-Gaussian subset")
    o, dI, params = hr["o"], hr["dI"], hr["params"]
    camd = scene.camera_dict(hr["cam"][0])
    keys = ("mean", "log_scale", "quat", "opacity_logit", "color")
    checked = rejected = 0
    for count, i in enumerate(hr["subset"]):
        if count % 64 == 0:
            say(f"FD: Gaussian {count} of 256, checked {checked}, rejected {rejected}")
        win = footprint(o, i)
        sub, idx = window_records(o, win)
        j = int(np.searchsorted(idx, i))
        p1 = {k: np.array(v[..., i:i + 1] if v.ndim == 2 else v[i:i + 1], np.float64)
              for k, v in params.items()}

        def with_record(p):
            q = oracle.project(p, camd, TILE)
            s = {k: v.copy() for k, v in sub.items()}
            for k in ("mean2d", "conic", "rgb"):
                s[k][:, j] = q[k][:, 0]
            for k in ("depth", "opacity"):
                s[k][j] = q[k][0]
            s["tile_bbox"][:, j] = q["tile_bbox"][:, 0]
            s["valid"][j] = int(q["valid"][0] and q["n_tiles"][0] > 0)
            return s, q

        s0, q0 = with_record(p1)
        # bbox listing: the list positions then change only with the bbox
        # and the depth rank, which the step checks itself
        base = oracle.render(s0, W, H, tile=TILE, window=win, support=False)
        b = oracle.render_bwd(s0, W, H, dI, tile=TILE, window=win)
        g2 = dict(d_mean2d=b["d_mean2d"][:, j:j + 1], d_conic=b["d_conic"][:, j:j + 1],
                  d_opacity=b["d_opacity"][j:j + 1], d_rgb=b["d_rgb"][:, j:j + 1])
        an = oracle.project_bwd(p1, camd, g2, TILE)
        gmax = max(np.abs(an[k]).max() for k in keys)
        x0, y0, x1, y1 = win

        others = np.delete(sub["depth"], j)
        rank0 = int(np.sum(others < q0["depth"][0]))

        def L(p):
            s, q = with_record(p)
            r = oracle.render(s, W, H, tile=TILE, window=win, support=False)
            same = (np.array_equal(q["tile_bbox"], q0["tile_bbox"])
                    and int(np.sum(others < q["depth"][0])) == rank0
                    and np.array_equal(r["n_contrib"][y0:y1, x0:x1], base["n_contrib"][y0:y1, x0:x1])
                    and np.array_equal(r["n_blended"][y0:y1, x0:x1], base["n_blended"][y0:y1, x0:x1]))
            return float(np.sum(dI[:, y0:y1, x0:x1] * r["image"][:, y0:y1, x0:x1])), same

        for key in keys:
            arr = p1[key] if p1[key].ndim == 2 else p1[key][None, :]
            ga = an[key] if an[key].ndim == 2 else an[key][None, :]
            for r_ in range(arr.shape[0]):
                x = arr[r_, 0]
                h = (1e-7 if key == "mean" else 1e-6) * max(1.0, abs(x))
                arr[r_, 0] = x + h
                Lp, sp = L(p1)
                arr[r_, 0] = x - h
                Lm, sm = L(p1)
                arr[r_, 0] = x
                if not (sp and sm):
                    rejected += 1
                    continue
                fd = (Lp - Lm) / (2 * h)
                g = ga[r_, 0]
                assert abs(fd - g) <= 1e-5 * abs(g) + 1e-6 * gmax + 2e-8, (int(i), key, r_, fd, g)
                checked += 1
    say(f"FD checked {checked}, rejected {rejected}")
    assert checked >= 256 * 14 * 0.8 and rejected <= checked // 10
