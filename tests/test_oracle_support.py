"""Pins of the oracle's tile listing (no GPU).

A pair is listed on the tiles of its bbox whose pixel-centre rectangle meets
its support {alpha >= 1/255} widened by a small margin.  The pins: the
closed form of a circular support (listed iff the rectangle's distance to
the mean is within the support radius), a brute-force scan of each tile's
pixel-centre rectangle on anisotropic, rotated supports, the invariant that
listing changes no image (only list positions), and the per-tile listing of
the sort.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2509_12138_amd import scene


def margin_threshold(mx, my, a, b, c, o, bb, tw, th):
    """2 ln(255 o) + 0.02 + 1e-5 M, M over the bbox's pixel-centre extents."""
    tx0, ty0, tx1, ty1 = bb
    X = max(abs(tx0 * tw + 0.5 - mx), abs(tx1 * tw + tw - 0.5 - mx))
    Y = max(abs(ty0 * th + 0.5 - my), abs(ty1 * th + th - 0.5 - my))
    M = a * X * X + 2 * abs(b) * X * Y + c * Y * Y
    return 2 * math.log(255 * o) + 0.02 + 1e-5 * M


def bits(mask, span, rows):
    return [[(int(mask) >> (r * span + q)) & 1 for q in range(span)] for r in range(rows)]


def test_circle_lists_tiles_within_the_support_radius():
    # isotropic conic a = c = 1/var, b = 0: min of Q over a rectangle is
    # dist^2 / var, so a tile is listed iff the rectangle lies within
    # sqrt(var * thr) of the mean
    tw = th = 8
    var, o = 9.0, 0.4
    mx, my = 37.3, 21.8
    bb = (1, 0, 7, 5)
    thr = margin_threshold(mx, my, 1 / var, 0.0, 1 / var, o, bb, tw, th)
    r = math.sqrt(var * thr)
    mask, amb = oracle.support_tiles(np.array([[mx], [my]]), np.array([[1 / var], [0.0], [1 / var]]),
                                     np.array([o]), np.array(bb, np.int32).reshape(4, 1),
                                     np.array([1], np.int32), (tw, th))
    assert amb[0] == 0
    span = bb[2] - bb[0] + 1
    got = bits(mask[0], span, bb[3] - bb[1] + 1)
    for ty in range(bb[1], bb[3] + 1):
        for tx in range(bb[0], bb[2] + 1):
            x0, x1 = tx * tw + 0.5, tx * tw + tw - 0.5
            y0, y1 = ty * th + 0.5, ty * th + th - 0.5
            d = math.hypot(max(x0 - mx, 0, mx - x1), max(y0 - my, 0, my - y1))
            assert got[ty - bb[1]][tx - bb[0]] == int(d <= r), (tx, ty, d, r)
    # the listing is neither empty nor the whole bbox for this case
    assert 0 < sum(map(sum, got)) < span * (bb[3] - bb[1] + 1)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_listing_matches_a_brute_force_scan_of_each_rectangle(seed):
    # rotated, elongated supports: a tile with a scanned point inside the
    # widened support must be listed; a listed tile must come within a
    # grid-spacing bound of it
    rng = np.random.default_rng(seed)
    tw, th = 16, 8
    n = 60
    ang = rng.uniform(0, np.pi, n)
    s1 = rng.uniform(1.0, 9.0, n); s2 = s1 * rng.uniform(0.08, 1.0, n)
    cov = np.zeros((n, 2, 2))
    for i in range(n):
        R = np.array([[np.cos(ang[i]), -np.sin(ang[i])], [np.sin(ang[i]), np.cos(ang[i])]])
        cov[i] = R @ np.diag([s1[i] ** 2, s2[i] ** 2]) @ R.T + 0.3 * np.eye(2)
    con = np.linalg.inv(cov)
    conic = np.stack([con[:, 0, 0], con[:, 0, 1], con[:, 1, 1]])
    mean = rng.uniform(20, 100, (2, n))
    opac = rng.uniform(0.02, 0.99, n)
    tb = np.stack([np.floor((mean[0] - 30) / tw), np.floor((mean[1] - 20) / th),
                   np.floor((mean[0] + 30) / tw), np.floor((mean[1] + 20) / th)]).astype(np.int32)
    tb = np.maximum(tb, 0)
    mask, amb = oracle.support_tiles(mean, conic, opac, tb, np.ones(n, np.int32), (tw, th))
    g = 97                                             # scan points per rectangle side
    checked = listed_n = 0
    for i in range(n):
        a, b, c = conic[:, i]
        bb = tuple(tb[:, i])
        span, rows = bb[2] - bb[0] + 1, bb[3] - bb[1] + 1
        if span * rows > 64:
            assert mask[i] == 0
            continue
        thr = margin_threshold(mean[0, i], mean[1, i], a, b, c, opac[i], bb, tw, th)
        got = bits(mask[i], span, rows)
        ab = bits(amb[i], span, rows)
        for ty in range(bb[1], bb[3] + 1):
            for tx in range(bb[0], bb[2] + 1):
                if ab[ty - bb[1]][tx - bb[0]]:
                    continue
                xs = np.linspace(tx * tw + 0.5, tx * tw + tw - 0.5, g) - mean[0, i]
                ys = np.linspace(ty * th + 0.5, ty * th + th - 0.5, g) - mean[1, i]
                X, Y = np.meshgrid(xs, ys)
                q = a * X * X + 2 * b * X * Y + c * Y * Y
                qmin = q.min()
                # |grad Q| over the rectangle bounds how far the scan's
                # minimum can sit above the exact one
                gx = np.abs(2 * (a * X + b * Y)).max(); gy = np.abs(2 * (b * X + c * Y)).max()
                slack = 0.5 * (gx * (xs[1] - xs[0]) + gy * (ys[1] - ys[0]))
                on = got[ty - bb[1]][tx - bb[0]]
                if qmin <= thr:
                    assert on, (i, tx, ty, qmin, thr)
                if on:
                    assert qmin <= thr + slack, (i, tx, ty, qmin, thr, slack)
                    listed_n += 1
                checked += 1
    assert checked > 500 and 0.1 * checked < listed_n < 0.9 * checked


def test_the_mean_tile_is_always_listed_and_listing_shrinks_with_opacity():
    rng = np.random.default_rng(7)
    n = 200
    mean = rng.uniform(40, 60, (2, n))
    conic = np.stack([np.full(n, 0.2), rng.uniform(-0.05, 0.05, n), np.full(n, 0.15)])
    tw = th = 16
    tb = np.stack([np.floor((mean[0] - 25) / tw), np.floor((mean[1] - 25) / th),
                   np.floor((mean[0] + 25) / tw), np.floor((mean[1] + 25) / th)]).astype(np.int32)
    hi, _ = oracle.support_tiles(mean, conic, np.full(n, 0.9), tb, np.ones(n, np.int32), (tw, th))
    lo, _ = oracle.support_tiles(mean, conic, np.full(n, 0.02), tb, np.ones(n, np.int32), (tw, th))
    span = tb[2] - tb[0] + 1
    for i in range(n):
        own = (int(mean[1, i] // th) - tb[1, i]) * span[i] + (int(mean[0, i] // tw) - tb[0, i])
        assert (int(lo[i]) >> own) & 1 and (int(hi[i]) >> own) & 1
        assert int(lo[i]) & ~int(hi[i]) == 0                 # lower opacity, subset
    assert sum(bin(int(x)).count("1") for x in lo) < sum(bin(int(x)).count("1") for x in hi)


def test_listing_changes_no_image_only_list_positions():
    # the widened support holds every pixel where alpha >= 1/255, so the
    # pairs left off a tile never blend there: images, transmittance and
    # blend counts are identical, list positions can only drop
    W_, H_ = 96, 80
    pts, nrm = scene.sample_surface(scene.field_sphere_sines, 1500, 64, seed=3)
    rng = np.random.default_rng(3)
    n = pts.shape[0]
    p = dict(mean=pts.T.astype(np.float64),
             log_scale=np.log(rng.uniform(0.01, 0.06, (3, n))),
             quat=rng.normal(size=(4, n)),
             opacity_logit=rng.normal(-1.0, 1.5, n),
             color=rng.normal(0, 0.5, (3, n)))
    cams = scene.orbit_cameras(2, W_, H_)
    shrank = 0
    for tile in ((16, 16), (8, 8)):
        for cam in cams:
            pr = oracle.project(p, scene.camera_dict(cam), tile)
            a = oracle.render(pr, W_, H_, tile=tile, bg=(0.2, 0.1, 0.3), support=True)
            b = oracle.render(pr, W_, H_, tile=tile, bg=(0.2, 0.1, 0.3), support=False)
            np.testing.assert_array_equal(a["image"], b["image"])
            np.testing.assert_array_equal(a["T_final"], b["T_final"])
            np.testing.assert_array_equal(a["n_blended"], b["n_blended"])
            assert np.all(a["n_contrib"] <= b["n_contrib"])
            shrank += int((a["n_contrib"] < b["n_contrib"]).sum())
    assert shrank > 100


def test_bin_sort_lists_exactly_the_support_tiles():
    # the sort's per-pair entry counts and lists follow support_tiles
    rng = np.random.default_rng(11)
    m, tw, th, tiles_x, tiles_y = 400, 8, 8, 12, 9
    mean = np.stack([rng.uniform(0, tiles_x * tw, m), rng.uniform(0, tiles_y * th, m)])
    a = rng.uniform(0.02, 0.5, m); c = rng.uniform(0.02, 0.5, m)
    b = rng.uniform(-0.9, 0.9, m) * np.sqrt(a * c)
    op = rng.uniform(0.01, 1.0, m)
    tx0 = np.clip(np.floor((mean[0] - 12) / tw), 0, tiles_x - 1)
    ty0 = np.clip(np.floor((mean[1] - 12) / th), 0, tiles_y - 1)
    tx1 = np.clip(np.floor((mean[0] + 12) / tw), 0, tiles_x - 1)
    ty1 = np.clip(np.floor((mean[1] + 12) / th), 0, tiles_y - 1)
    tb = np.stack([tx0, ty0, tx1, ty1], 1).astype(np.int32)
    nt = ((tb[:, 2] - tb[:, 0] + 1) * (tb[:, 3] - tb[:, 1] + 1)).astype(np.int32)
    nt[:20] = 0
    depth = rng.uniform(1, 3, m).astype(np.float32)
    sup = np.stack([mean[0], mean[1], a, b, c, op], 1)
    keys, ids, ranges, count, amb = oracle.bin_sort(tb, nt, depth, np.zeros(m, np.int32), tiles_x,
                                                    tiles_x * tiles_y, 1, sup=sup, tile=(tw, th),
                                                    details=True)
    mask, _ = oracle.support_tiles(mean, np.stack([a, b, c]), op, tb.T.copy(),
                                   (nt > 0).astype(np.int32), (tw, th))
    np.testing.assert_array_equal(count, [bin(int(x)).count("1") for x in mask])
    assert count.sum() < 0.9 * nt.sum()
    for t in range(tiles_x * tiles_y):
        tx, ty = t % tiles_x, t // tiles_x
        members = [p for p in range(m) if nt[p] > 0 and tb[p, 0] <= tx <= tb[p, 2]
                   and tb[p, 1] <= ty <= tb[p, 3]
                   and (int(mask[p]) >> ((ty - tb[p, 1]) * (tb[p, 2] - tb[p, 0] + 1) + tx - tb[p, 0])) & 1]
        members.sort(key=lambda p: (int(depth.view(np.uint32)[p]), p))
        s, e = ranges[t]
        np.testing.assert_array_equal(ids[s:e], np.array(members, np.uint32))


@pytest.mark.parametrize("extra,listed", [(0.01, 1), (0.03, 0)])
def test_margin_widens_the_support_by_0_02_plus_1e_5_M(extra, listed):
    # a circle whose support radius (margin excluded) stops short of the
    # next tile: the tile is listed when its distance is within the 0.02
    # margin and not beyond it
    tw = th = 16
    var, o = 4.0, 0.5
    thr0 = 2 * math.log(255 * o)
    bb = (0, 0, 1, 0)
    my = 8.0
    # tile 1's rectangle starts at x = 16.5; solve for the mean's x so that
    # (16.5 - mx)^2 / var = thr0 + extra + 1e-5 M (M depends on mx: iterate)
    mx = 16.5 - math.sqrt(var * (thr0 + extra))
    for _ in range(50):
        X = max(abs(0.5 - mx), abs(31.5 - mx)); Y = max(abs(0.5 - my), abs(15.5 - my))
        M = (X * X + Y * Y) / var
        mx = 16.5 - math.sqrt(var * (thr0 + extra + 1e-5 * M))
    mask, amb = oracle.support_tiles(np.array([[mx], [my]]), np.array([[1 / var], [0.0], [1 / var]]),
                                     np.array([o]), np.array(bb, np.int32).reshape(4, 1),
                                     np.array([1], np.int32), (tw, th))
    assert amb[0] == 0
    assert (int(mask[0]) & 1) == 1 and ((int(mask[0]) >> 1) & 1) == listed
