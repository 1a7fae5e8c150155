"""Pins of the oracle's loss, Adam, binning/sort, k-NN and MLP (no GPU)."""
import math

import numpy as np
import pytest
from scipy import ndimage
from scipy.spatial import cKDTree

import oracle

C1, C2 = 0.01 ** 2, 0.03 ** 2


# ---------------------------------------------------------------- loss

def test_identical_images_give_zero_loss_and_gradient():
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 1, (3, 24, 20))
    mask = (rng.uniform(size=(24, 20)) > 0.3).astype(np.float64)
    r = oracle.loss(x, x, mask)
    assert abs(r["ssim"] - 1.0) < 1e-14 and r["l1"] == 0.0 and abs(r["loss"]) < 1e-14
    assert np.max(np.abs(r["d_image"])) < 1e-14


def test_constant_images_interior_closed_form():
    a, b = 0.7, 0.3
    x = np.full((3, 30, 30), a); y = np.full((3, 30, 30), b)
    r = oracle.loss(x, y, None)
    S = r["ssim_map"]
    expect = (2 * a * b + C1) / (a * a + b * b + C1)
    np.testing.assert_allclose(S[:, 5:-5, 5:-5], expect, rtol=1e-12)
    assert abs(r["l1"] - 0.4) < 1e-13


def test_ssim_map_matches_library_filtering():
    # the same definition evaluated through scipy's separable Gaussian filter
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, (3, 21, 27)); y = np.clip(x + rng.normal(0, 0.1, x.shape), 0, 1)
    mask = (rng.uniform(size=(21, 27)) > 0.2).astype(np.float64)
    xm, ym = x * mask, y * mask
    filt = lambda im: ndimage.gaussian_filter(im, 1.5, mode="constant", cval=0.0, truncate=5 / 1.5)
    S = np.zeros_like(x)
    for c in range(3):
        mx, my = filt(xm[c]), filt(ym[c])
        sxx = filt(xm[c] ** 2) - mx ** 2; syy = filt(ym[c] ** 2) - my ** 2
        sxy = filt(xm[c] * ym[c]) - mx * my
        S[c] = ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx ** 2 + my ** 2 + C1) * (sxx + syy + C2))
    r = oracle.loss(x, y, mask, lam=0.2)
    np.testing.assert_allclose(r["ssim_map"], S, rtol=1e-10, atol=1e-12)
    l1 = np.mean(np.abs(xm - ym))
    assert abs(r["loss"] - (0.8 * l1 + 0.2 * (1 - S.mean()))) < 1e-12


def test_loss_gradient_matches_fd():
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, (3, 14, 17)); y = rng.uniform(0, 1, (3, 14, 17))
    mask = (rng.uniform(size=(14, 17)) > 0.25).astype(np.float64)
    r = oracle.loss(x, y, mask, lam=0.2)
    for idx in [(0, 0, 0), (1, 7, 8), (2, 13, 16), (0, 3, 12), (1, 10, 2)]:
        h = 1e-6
        xp = x.copy(); xp[idx] += h
        xm = x.copy(); xm[idx] -= h
        fd = (oracle.loss(xp, y, mask)["loss"] - oracle.loss(xm, y, mask)["loss"]) / (2 * h)
        assert abs(fd - r["d_image"][idx]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (idx, fd, r["d_image"][idx])
    # masked-out pixels get no gradient
    assert np.all(r["d_image"][:, mask == 0] == 0)


def test_loss_gradient_fd_random_sweep():
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, (3, 12, 12)); y = rng.uniform(0, 1, (3, 12, 12))
    r = oracle.loss(x, y, None, lam=0.35)
    for _ in range(20):
        idx = (int(rng.integers(3)), int(rng.integers(12)), int(rng.integers(12)))
        h = 1e-6
        xp = x.copy(); xp[idx] += h
        xm = x.copy(); xm[idx] -= h
        fd = (oracle.loss(xp, y, None, lam=0.35)["loss"] - oracle.loss(xm, y, None, lam=0.35)["loss"]) / (2 * h)
        assert abs(fd - r["d_image"][idx]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9


# ---------------------------------------------------------------- Adam

def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(4)
    p = rng.normal(size=100); g = rng.normal(size=100)
    p1, m, v = oracle.adam(p, g, np.zeros(100), np.zeros(100), lr=0.01, step=1)
    np.testing.assert_allclose(p1 - p, -0.01 * g / (np.abs(g) + 1e-15), rtol=1e-12)


def test_adam_constant_gradient_constant_step():
    g = np.array([0.3, -2.0, 1e-3])
    p = np.zeros(3); m = np.zeros(3); v = np.zeros(3)
    for step in range(1, 30):
        p_new, m, v = oracle.adam(p, g, m, v, lr=1e-3, step=step)
        np.testing.assert_allclose(p_new - p, -1e-3 * np.sign(g), rtol=1e-9)
        p = p_new


def test_sparse_adam_keeps_hidden_gaussians_and_uses_the_global_step():
    # Gaussian 0 is drawn at every step, Gaussian 1 first at step k, Gaussian
    # 2 never; gradients are constant in time
    b1, b2, lr, k = 0.9, 0.999, 1e-3, 7
    g = np.array([[0.5, -2.0, 0.7], [1e-3, 3.0, -0.2]])
    p = np.array([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0]])
    m = np.zeros_like(p); v = np.zeros_like(p)
    for step in range(1, k + 1):
        vis = np.array([True, step == k, False])
        p_new, m, v = oracle.adam(p, g, m, v, lr=lr, step=step, visible=vis)
        assert np.array_equal(p_new[:, 2], p[:, 2]) and np.all(m[:, 2] == 0) and np.all(v[:, 2] == 0)
        if step < k:
            assert np.array_equal(p_new[:, 1], p[:, 1])
        p_last = p
        p = p_new
    # constant gradient, seen at every step: the step is lr sign(g)
    np.testing.assert_allclose(p[:, 0] - p_last[:, 0], -lr * np.sign(g[:, 0]), rtol=1e-9)
    # first seen at step k: zero moments, bias correction of step k
    ratio = (1 - b1) / (1 - b1 ** k) / np.sqrt((1 - b2) / (1 - b2 ** k))
    np.testing.assert_allclose(p[:, 1] - p_last[:, 1], -lr * ratio * np.sign(g[:, 1]), rtol=1e-9)
    # all visible is the dense step
    d = oracle.adam(p, g, m, v, lr=lr, step=k + 1)
    s_ = oracle.adam(p, g, m, v, lr=lr, step=k + 1, visible=np.ones(3, bool))
    for a, b in zip(d, s_):
        assert np.array_equal(a, b)


# ---------------------------------------------------------------- binning + sort

def brute_tile_lists(tb, nt, depth, slot, tiles_x, tiles_per_slot, n_slots):
    bits = np.asarray(depth, np.float32).view(np.uint32)
    out = []
    for s in range(n_slots):
        for t in range(tiles_per_slot):
            tx, ty = t % tiles_x, t // tiles_x
            members = [p for p in range(len(nt)) if nt[p] > 0 and slot[p] == s and
                       tb[p, 0] <= tx <= tb[p, 2] and tb[p, 1] <= ty <= tb[p, 3]]
            members.sort(key=lambda p: (int(bits[p]), p))
            out.append(members)
    return out


@pytest.mark.parametrize("seed", [0, 1])
def test_bin_sort_matches_per_tile_listing(seed):
    rng = np.random.default_rng(seed)
    m, tiles_x, tiles_y, S = 300, 7, 5, 3
    tx0 = rng.integers(0, tiles_x, m); ty0 = rng.integers(0, tiles_y, m)
    tx1 = np.minimum(tx0 + rng.integers(0, 3, m), tiles_x - 1)
    ty1 = np.minimum(ty0 + rng.integers(0, 3, m), tiles_y - 1)
    tb = np.stack([tx0, ty0, tx1, ty1], 1).astype(np.int32)
    nt = ((tx1 - tx0 + 1) * (ty1 - ty0 + 1)).astype(np.int32)
    nt[rng.uniform(size=m) < 0.2] = 0                       # culled pairs
    depth = rng.uniform(0.5, 4.0, m).astype(np.float32)
    depth[:40] = depth[40:80]                               # exact depth ties
    slot = np.sort(rng.integers(0, S, m)).astype(np.int32)
    keys, ids, ranges = oracle.bin_sort(tb, nt, depth, slot, tiles_x, tiles_x * tiles_y, S)
    lists = brute_tile_lists(tb, nt, depth, slot, tiles_x, tiles_x * tiles_y, S)
    assert len(ids) == int(nt.sum())
    np.testing.assert_array_equal(ids, np.concatenate([np.array(l, np.int64) for l in lists]).astype(np.uint32))
    for t, l in enumerate(lists):
        a, b = ranges[t]
        if len(l) == 0:
            assert a == 0 and b == 0
        else:
            assert b - a == len(l)
            np.testing.assert_array_equal(ids[a:b], l)
    assert np.all(np.diff(keys.astype(np.float64)) >= 0)


# ---------------------------------------------------------------- k-NN

def test_knn_matches_kdtree():
    rng = np.random.default_rng(5)
    pts = rng.uniform(-1, 1, (3, 700))
    idx, dist = oracle.knn(pts, 16)
    d, i = cKDTree(pts.T).query(pts.T, k=17)
    np.testing.assert_allclose(dist, d[:, 1:], rtol=1e-12)
    np.testing.assert_array_equal(idx, i[:, 1:])


def test_knn_ties_break_by_index():
    pts = np.array([[0.0, 1.0, -1.0, 0.0, 0.0], [0.0, 0.0, 0.0, 1.0, 5.0], [0.0] * 5])
    idx, dist = oracle.knn(pts, 3)
    np.testing.assert_array_equal(idx[0], [1, 2, 3])
    np.testing.assert_allclose(dist[0], [1, 1, 1])


# ---------------------------------------------------------------- MLP

def test_bf16_rounding_ties_to_even():
    # bf16 keeps 7 fraction bits: near 1 the spacing is 2^-7 and halfway
    # cases go to the neighbour with an even last bit
    v = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -9, 1 + 2 ** -7 + 2 ** -9,
                  -2.5, 0.0])
    np.testing.assert_array_equal(oracle.bf16_round(v),
                                  [1.0, 1.0, 1 + 2 ** -6, 1.0, 1 + 2 ** -7, -2.5, 0.0])
    # every output is representable with 8 significand bits
    r = oracle.bf16_round(np.random.default_rng(0).normal(size=1000))
    assert np.all(r.astype(np.float32).view(np.uint32) & 0xFFFF == 0)


def _mlp_params(rng, scale=0.3):
    return (rng.normal(0, scale, (96, 64)), rng.normal(0, 0.1, 64), rng.normal(0, scale, (64, 64)),
            rng.normal(0, 0.1, 64), rng.normal(0, scale, (64, 8)), rng.normal(0, 0.1, 8))


def test_mlp_zero_weights_give_bias():
    rng = np.random.default_rng(6)
    x = rng.normal(size=(10, 96))
    W1, b1, W2, b2, W3, b3 = _mlp_params(rng)
    y, _ = oracle.mlp_forward(x, 0 * W1, b1, 0 * W2, b2, 0 * W3, b3, quantize=False)
    np.testing.assert_array_equal(y, np.broadcast_to(b3, (10, 8)))


def test_mlp_backward_matches_fd():
    rng = np.random.default_rng(7)
    x = rng.normal(size=(6, 96))
    P = list(_mlp_params(rng))
    dy = rng.normal(size=(6, 8))
    y, cache = oracle.mlp_forward(x, *P, quantize=False)
    g = oracle.mlp_backward(cache, dy)
    names = ["W1", "b1", "W2", "b2", "W3", "b3"]
    for k, name in enumerate(names):
        flat = P[k].reshape(-1)
        for j in rng.choice(flat.size, size=min(15, flat.size), replace=False):
            h = 1e-6
            old = flat[j]
            flat[j] = old + h; yp, _ = oracle.mlp_forward(x, *P, quantize=False)
            flat[j] = old - h; ym, _ = oracle.mlp_forward(x, *P, quantize=False)
            flat[j] = old
            fd = np.sum(dy * (yp - ym)) / (2 * h)
            assert abs(fd - g[name].reshape(-1)[j]) <= 1e-6 * max(1, abs(fd)), (name, j)
    for j in range(0, 96, 7):
        h = 1e-6
        xp = x.copy(); xp[2, j] += h
        xm = x.copy(); xm[2, j] -= h
        fd = np.sum(dy * (oracle.mlp_forward(xp, *P, quantize=False)[0] -
                          oracle.mlp_forward(xm, *P, quantize=False)[0])) / (2 * h)
        assert abs(fd - g["x"][2, j]) <= 1e-6 * max(1, abs(fd))
