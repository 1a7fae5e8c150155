"""Pins of the oracle's masked PSNR (no GPU): closed forms for constant and
single-pixel errors, the background and clamping invariances, the 20 log10 2
scale law, and the exact-match / empty-mask special cases."""
import math

import numpy as np

import oracle


def _scene(seed=0, H=23, W=31, frac=0.6):
    rng = np.random.default_rng(seed)
    target = rng.uniform(0.2, 0.8, (3, H, W))
    mask = (rng.uniform(size=(H, W)) < frac).astype(np.uint8)
    return rng, target, mask


def test_constant_error_gives_closed_form():
    # every masked channel off by delta: MSE = delta^2, PSNR = -20 log10 delta
    rng, t, m = _scene(1)
    for delta in (0.1, 0.01, 0.137):
        img = t + delta
        assert abs(oracle.masked_psnr(img, t, m) - (-20.0 * math.log10(delta))) < 1e-9


def test_single_pixel_error_counts_masked_pixels_and_channels():
    # one channel of one masked pixel off by e among N masked pixels:
    # MSE = e^2 / (3 N)
    rng, t, m = _scene(2)
    N = int(m.sum())
    ys, xs = np.nonzero(m)
    img = t.copy()
    e = 0.05
    img[1, ys[7], xs[7]] += e
    expect = 10.0 * math.log10(3 * N / e ** 2)
    assert abs(oracle.masked_psnr(img, t, m) - expect) < 1e-9


def test_background_pixels_do_not_count():
    rng, t, m = _scene(3)
    img = np.clip(t + rng.normal(0, 0.05, t.shape), 0, 1)
    a = oracle.masked_psnr(img, t, m)
    img2 = img.copy()
    bg = m == 0
    img2[:, bg] = rng.uniform(0, 1, (3, int(bg.sum())))
    assert a == oracle.masked_psnr(img2, t, m)
    # a full mask is the plain PSNR over all pixels
    full = np.ones_like(m)
    assert oracle.masked_psnr(img, t, full) == oracle.masked_psnr(img, t, None)


def test_rendered_values_are_clamped_to_the_display_range():
    rng, t, m = _scene(4)
    t = t.copy()
    t[:, :5] = 1.0
    t[:, -5:] = 0.0
    img = t.copy()
    img[:, :5] = 1.7          # over-bright where the target is white
    img[:, -5:] = -0.4        # negative where the target is black
    assert oracle.masked_psnr(img, t, m) == math.inf
    img[0, 10, 10] = t[0, 10, 10] + 0.2
    N = int(m.sum())
    expect = 10.0 * math.log10(3 * N / 0.2 ** 2) if m[10, 10] else math.inf
    assert abs(oracle.masked_psnr(img, t, m) - expect) < 1e-9


def test_halving_the_error_adds_20_log10_2():
    rng, t, m = _scene(5)
    err = rng.normal(0, 0.03, t.shape)
    a = oracle.masked_psnr(t + err, t, m)
    b = oracle.masked_psnr(t + 0.5 * err, t, m)
    assert abs((b - a) - 20.0 * math.log10(2.0)) < 1e-9


def test_exact_match_and_empty_mask():
    rng, t, m = _scene(6)
    assert oracle.masked_psnr(t, t, m) == math.inf
    assert math.isnan(oracle.masked_psnr(t + 0.1, t, np.zeros_like(m)))
