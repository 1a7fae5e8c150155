"""Parity at the benchmark workload's full size: the 1M-Gaussian mixing-layer
partition at 1920x1080, in every rasteriser launch configuration the
autotuner can pick (bench.py times the one it picks).

* projection of all 1M Gaussians for two views against the oracle;
* bin/sort of the oracle's records, bit-exact against the oracle's sort;
* images on sampled 32x32 pixel windows (the densest tile, the image
  centre, the bottom-right corner with its ragged tiles) within 1e-4 of the
  oracle's window render;
* gradients from an image gradient that is non-zero only inside those
  windows, so that the oracle's window backward is the complete answer.

Both sides rasterise the same FP32 records, built by the oracle."""
import math

import numpy as np
import pytest

import oracle
from paper_2509_12138_amd import scene, workloads
from _gpu_helpers import (grad_tolerance_check, oracle_lists, oracle_records, perturbed,
                          raster_records, say, to_dev)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

W, H = 1920, 1080
VIEWS = [0, 37]
SAME_RECORD_BITS = 1 | 2 | 4 | 8
WIN = 32


@pytest.fixture(scope="module")
def big(gpu):
    say("building the 1M-Gaussian 1080p partition")
    wl = workloads.realistic_partition(with_reference=False)
    assert wl["cfg"]["width"] == W and wl["cfg"]["height"] == H
    params = perturbed(wl["params"], 7, amount=0.2)
    cams = wl["cams"][VIEWS]
    return params, cams


def test_fullsize_projection_matches_oracle(big):
    from paper_2509_12138_amd import ops
    params, cams = big
    n = params["opacity_logit"].shape[0]
    say(f"full-size projection n={n}")
    views = ops.Views.single(n, cams)
    bufs = ops.RasterBuffers(views, W, H, (16, 16), dup_capacity=1024)
    bufs.project(ops.gaussians_struct(to_dev(params, torch)))
    torch.cuda.synchronize()
    rec = bufs.rec.cpu().numpy()
    tb = bufs.tile_bbox.cpu().numpy().astype(np.int64) & 0xFFFF
    nt = bufs.n_tiles.cpu().numpy()
    for v in range(len(cams)):
        o = oracle.project(params, scene.camera_dict(cams[v]))
        sl = slice(v * n, (v + 1) * n)
        r, t_, ntv = rec[sl], tb[sl], nt[sl]
        kappa = 2 * np.log(np.maximum(255 * o["opacity"], 1e-300))
        hx = np.sqrt(np.maximum(kappa, 0) * o["cov2d"][0])
        hy = np.sqrt(np.maximum(kappa, 0) * o["cov2d"][2])
        edges = np.stack([o["mean2d"][0] - hx, o["mean2d"][0] + hx,
                          o["mean2d"][1] - hy, o["mean2d"][1] + hy])
        # FP32 error of m +/- h stays below 2e-4 px at 1080p coordinates
        near = np.any(np.abs(edges - np.round(edges)) < 2e-4, axis=0) | \
            (np.abs(255 * o["opacity"] - 1) < 1e-4)
        assert near.mean() < 2e-3
        ok = ~near
        valid = o["valid"].astype(bool) & (o["n_tiles"] > 0)
        np.testing.assert_array_equal(ntv[ok] > 0, valid[ok])
        both = ok & valid
        assert both.sum() > n // 4
        np.testing.assert_array_equal(t_[both], o["tile_bbox"].T[both])
        np.testing.assert_allclose(r[both, 0:2], o["mean2d"].T[both], rtol=1e-5, atol=2e-4)
        cscale = np.abs(o["conic"]).max(0)[both][:, None]
        assert np.all(np.abs(r[both, 2:5] - o["conic"].T[both]) <= 1e-5 * cscale + 1e-9)
        np.testing.assert_allclose(r[both, 5], o["opacity"][both], rtol=1e-5)
        np.testing.assert_allclose(r[both, 9], o["depth"][both], rtol=1e-6)


_records = {}


def records(big, tile):
    if tile not in _records:
        params, cams = big
        _records[tile] = oracle_records(params, cams, W, H, tile)
    return _records[tile]


def windows_for(big, v):
    """Three windows of view v: around the tile with the longest list, the
    image centre, the bottom-right corner (ragged for 16-row tiles)."""
    rec, tb, nt, _ = records(big, (16, 16))
    n = big[0]["opacity_logit"].shape[0]
    t = tb[v * n:(v + 1) * n].astype(np.int64) & 0xFFFF
    k = nt[v * n:(v + 1) * n] > 0
    cnt = np.zeros((math.ceil(H / 16), W // 16), np.int64)
    for i in np.flatnonzero(k)[::7]:                 # a subsample finds the dense area
        cnt[t[i, 1]:t[i, 3] + 1, t[i, 0]:t[i, 2] + 1] += 1
    ty, tx = np.unravel_index(np.argmax(cnt), cnt.shape)
    x0 = int(min(max(16 * tx - 8, 0), W - WIN)); y0 = int(min(max(16 * ty - 8, 0), H - WIN))
    return [(x0, y0, x0 + WIN, y0 + WIN), (W // 2 - 16, H // 2 - 16, W // 2 + 16, H // 2 + 16),
            (W - WIN, H - WIN, W, H)]


_oracle_out = {}


def oracle_windows(big, dI):
    """The oracle's window renders and backward, once: records of other tile
    shapes differ only in their tile bboxes, and neither the images nor the
    gradients depend on the tile shape (the support ellipse lies inside the
    padded bbox for every shape)."""
    tile = (16, 16)
    if tile not in _oracle_out:
        _, _, _, views = records(big, tile)
        out = []
        for v in range(len(VIEWS)):
            per = []
            for win in windows_for(big, v):
                f = oracle.render(views[v], W, H, tile=tile, window=win)
                b = oracle.render_bwd(views[v], W, H, dI[v], tile=tile, window=win,
                                      amb_bits=SAME_RECORD_BITS)
                per.append((win, f, b))
            out.append(per)
        _oracle_out[tile] = out
    return _oracle_out[tile]


_ncontrib = {}


def oracle_ncontrib(big, tile):
    """n_contrib of the oracle's window renders with this tile shape's
    records (a position in the tile's list, so it depends on the shape)."""
    if tile not in _ncontrib:
        _, _, _, views = records(big, tile)
        _ncontrib[tile] = [[_nc_and_listing_amb(oracle.render(views[v], W, H, tile=tile,
                                                             window=win))
                            for win in windows_for(big, v)] for v in range(len(VIEWS))]
    return _ncontrib[tile]


def _nc_and_listing_amb(r):
    # n_contrib, and the pixels where an ambiguous tile listing precedes the
    # last blended entry (the list positions may differ there)
    return r["n_contrib"], (r["ambiguity"] & 32) != 0


def image_gradient(big):
    rng = np.random.default_rng(11)
    dI = np.zeros((len(VIEWS), 3, H, W), np.float32)
    for v in range(len(VIEWS)):
        for (x0, y0, x1, y1) in windows_for(big, v):
            dI[v, :, y0:y1, x0:x1] = rng.normal(size=(3, y1 - y0, x1 - x0))
    return dI


def test_fullsize_bin_sort_bit_exact(big):
    from paper_2509_12138_amd import ops
    params, cams = big
    n = params["opacity_logit"].shape[0]
    for tile in [(16, 16), (8, 16)]:
        say(f"full-size bin/sort tile={tile}")
        rec, tb, nt, _ = records(big, tile)
        slot = np.repeat(np.arange(len(cams), dtype=np.int32), n)
        nt, keys, ids, ranges = oracle_lists(rec, tb, nt, slot, tile, W, H, len(cams))
        K = len(ids)
        for keep in (True, False):      # 64-bit (tile, depth) keys, or 32-bit tile keys
            bufs = ops.RasterBuffers(ops.Views.single(n, cams), W, H, tile, dup_capacity=1024,
                                     keep_keys=keep)
            raster_records(bufs, rec, tb, nt, (0.0, 0.0, 0.0), torch)
            assert int(bufs.check()[1]) == K and K < 0.9 * int(nt.astype(np.int64).sum())
            if keep:
                np.testing.assert_array_equal(bufs.keys[:K].cpu().numpy().view(np.uint64), keys)
            np.testing.assert_array_equal(bufs.ids[:K].cpu().numpy().view(np.uint32), ids)
            np.testing.assert_array_equal(bufs.ranges.cpu().numpy().view(np.uint32), ranges)
            del bufs


def _plans():
    from paper_2509_12138_amd.autotune import CANDIDATES
    plans = [(t, s, c, w, d, True) for (t, s, c, w, d) in CANDIDATES]
    plans.append(((16, 16), "lpt", 0, 1, False, False))    # transmittance recompute
    plans.append(((16, 16), "lpt", 0, 4, True, False))
    return plans


@pytest.mark.parametrize("tile,sched,chunk,fwd_waves,det,stored", _plans())
def test_fullsize_raster_matches_oracle_windows(big, tile, sched, chunk, fwd_waves, det, stored):
    from paper_2509_12138_amd import ops
    params, cams = big
    n = params["opacity_logit"].shape[0]
    say(f"full-size raster tile={tile} {sched} chunk={chunk} fwd_waves={fwd_waves} det={det} "
        f"stored={stored}")
    rec, tb, nt, _ = records(big, tile)
    dI = image_gradient(big)
    bufs = ops.RasterBuffers(ops.Views.single(n, cams), W, H, tile, dup_capacity=1024,
                             store_state=stored)
    bufs.set_schedule(sched, chunk=chunk, fwd_waves=fwd_waves, deterministic=det)
    raster_records(bufs, rec, tb, nt, (0.0, 0.0, 0.0), torch)
    bufs.zero_d_rec()
    bufs.raster_bwd(torch.as_tensor(dI).cuda())
    torch.cuda.synchronize()
    img = bufs.image.cpu().numpy()
    drec = bufs.d_rec.cpu().numpy().astype(np.float64)
    ncs = oracle_ncontrib(big, tile) if stored else None
    for v, per in enumerate(oracle_windows(big, dI)):
        grad = np.zeros((n, 9)); term = np.zeros((n, 9)); amb_m = np.zeros((n, 9))
        for w_i, ((x0, y0, x1, y1), f, b) in enumerate(per):
            amb = ((f["ambiguity"] & SAME_RECORD_BITS) != 0)[y0:y1, x0:x1]
            # measured on these windows: at most 2 of 1,024 pixels
            assert amb.mean() <= 5e-3
            err = np.abs(img[v][:, y0:y1, x0:x1] - f["image"][:, y0:y1, x0:x1])[:, ~amb]
            assert err.max() <= 1e-4, ((x0, y0), err.max())
            if stored:
                nc = bufs.n_contrib[v].cpu().numpy()[y0:y1, x0:x1]
                onc, lamb = ncs[v][w_i]
                ok = ~amb & ~lamb[y0:y1, x0:x1]
                np.testing.assert_array_equal(nc[ok], onc[y0:y1, x0:x1][ok])
            grad += np.concatenate([b["d_mean2d"], b["d_conic"], b["d_opacity"][None],
                                    b["d_rgb"]]).T
            term += b["term_mass"].T
            amb_m += b["amb_mass"].T
        sl = slice(v * n, (v + 1) * n)
        touched = np.any(grad != 0, axis=1)
        assert touched.sum() > 1000
        np.testing.assert_array_equal(drec[sl][~touched & (term.sum(1) == 0)], 0.0)
        ok, worst = grad_tolerance_check(drec[sl], grad, term, amb_m)
        assert ok, worst
        for c in range(9):
            nr = np.linalg.norm(drec[sl][:, c] - grad[:, c]) / max(np.linalg.norm(grad[:, c]), 1e-30)
            assert nr <= 1e-3, (c, nr)


def test_fullsize_sh3_colour_and_gradients_on_sampled_gaussians(big):
    """Degree-3 view-dependent colour at full size: the projection's colours
    and the projection backward's gradients of 20,000 sampled Gaussians
    (the oracle computes each Gaussian on its own) for two views, and the
    fused backward + Adam of one view (the bench's one-slot kernel, six Adam
    groups) bit for bit against the two separate calls."""
    from paper_2509_12138_amd import ops
    from paper_2509_12138_amd.train import DEFAULT_LR
    params, cams = big
    n = params["opacity_logit"].shape[0]
    say(f"full-size sh3 n={n}")
    rng = np.random.default_rng(31)
    p3 = dict(params)
    col = np.zeros((48, n), np.float32)
    col[:3] = params["color"]
    col[3:] = 0.2 * rng.normal(size=(45, n))
    p3["color"] = col
    dp = to_dev(p3, torch)
    views = ops.Views.single(n, cams)
    bufs = ops.RasterBuffers(views, W, H, (16, 16), dup_capacity=1024)
    gst = ops.gaussians_struct(dp)
    assert gst.sh_degree == 3
    bufs.project(gst)
    torch.cuda.synchronize()
    rec = bufs.rec.cpu().numpy()
    sample = np.sort(rng.choice(n, 20000, replace=False))
    sub = {k: (v[..., sample] if v.ndim == 2 else v[sample]) for k, v in p3.items()}
    drec = np.zeros((len(cams) * n, 9), np.float32)
    for v in range(len(cams)):
        o = oracle.project(sub, scene.camera_dict(cams[v]))
        r = rec[v * n:(v + 1) * n][sample]
        kappa = 2 * np.log(np.maximum(255 * o["opacity"], 1e-300))
        hx = np.sqrt(np.maximum(kappa, 0) * o["cov2d"][0])
        hy = np.sqrt(np.maximum(kappa, 0) * o["cov2d"][2])
        edges = np.stack([o["mean2d"][0] - hx, o["mean2d"][0] + hx,
                          o["mean2d"][1] - hy, o["mean2d"][1] + hy])
        near = np.any(np.abs(edges - np.round(edges)) < 2e-4, axis=0) | \
            (np.abs(255 * o["opacity"] - 1) < 1e-4)
        ok = (o["n_tiles"] > 0) & ~near
        assert ok.sum() > 5000
        np.testing.assert_allclose(r[ok, 6:9], o["rgb"].T[ok], rtol=1e-5, atol=2e-6)
        d = rng.normal(size=(len(sample), 9)) * ok[:, None]
        d[:, 6:9] *= (o["rgb"].T > 1e-4)
        drec[v * n + sample] = d
    bufs.d_rec.copy_(torch.as_tensor(drec))
    grads = {k: torch.zeros_like(v) for k, v in dp.items()}
    bufs.project_bwd(gst, ops.grads_struct(grads, n))
    torch.cuda.synchronize()
    ref = {k: np.zeros(np.shape(v)) for k, v in sub.items()}
    for v in range(len(cams)):
        d = drec[v * n + sample].astype(np.float64)
        g = oracle.project_bwd(sub, scene.camera_dict(cams[v]),
                               dict(d_mean2d=d[:, 0:2].T, d_conic=d[:, 2:5].T, d_opacity=d[:, 5],
                                    d_rgb=d[:, 6:9].T))
        for k in ref:
            ref[k] += g[k]
    for k in ref:
        got = grads[k].cpu().numpy()
        got = (got[..., sample] if got.ndim == 2 else got[sample]).astype(np.float64)
        r = ref[k]
        nr = np.linalg.norm(got - r) / max(np.linalg.norm(r), 1e-30)
        assert nr <= 1e-4, (k, nr)
        assert np.all(np.abs(got - r) <= 1e-3 * np.abs(r) + 1e-5 * np.abs(r).max()), k
    # fused one-view step against the separate calls, all 1M Gaussians
    one = ops.Views.single(n, cams[:1])
    b1 = ops.RasterBuffers(one, W, H, (16, 16), dup_capacity=1024)
    runs = []
    for fused in (False, True):
        q = to_dev(p3, torch)
        gq = ops.gaussians_struct(q)
        m = {k: torch.zeros_like(v) for k, v in q.items()}
        vv = {k: torch.zeros_like(v) for k, v in q.items()}
        gr = {k: torch.zeros_like(v) for k, v in q.items()}
        adam = ops.DeviceAdam(ops.adam_groups(q, gr, m, vv, DEFAULT_LR))
        assert len(adam.groups) == 6
        b1.project(gq)
        b1.d_rec.copy_(torch.as_tensor(drec[:n]))
        if fused:
            b1.project_bwd_adam(gq, adam)
        else:
            b1.project_bwd(gq, ops.grads_struct(gr, n))
            adam(zero_grad=True)
        torch.cuda.synchronize()
        runs.append({k: (q[k].cpu().numpy(), m[k].cpu().numpy()) for k in q})
    for k in runs[0]:
        np.testing.assert_array_equal(runs[0][k][0], runs[1][k][0], err_msg=k)
        np.testing.assert_array_equal(runs[0][k][1], runs[1][k][1], err_msg=k)
