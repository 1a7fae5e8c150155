"""Finite-difference pins of the oracle's analytic backward (no GPU).

The backward is the exact derivative of the forward with every discrete
decision (skip below 1/255, the 0.99 clamp, the transmittance stop, culling,
bboxes) held fixed.  Central differences of the FP64 forward check it; a
perturbation that flips any decision is rejected and counted.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2509_12138_amd import scene

W, H = 40, 32


def cam_at(f=36.0, R=np.eye(3), t=(0.0, 0.0, 0.0), W=W, H=H):
    return dict(R=np.asarray(R, np.float64).ravel(), t=np.asarray(t, np.float64), fx=f, fy=f,
                cx=W / 2.0, cy=H / 2.0, znear=0.2, width=W, height=H)


def make_params(seed, n=40):
    g = scene.random_gaussians(n, seed, center=(0, 0, 2.2), extent=0.45, log_scale=(-3.0, -1.9),
                               opacity=(0.2, 0.9))
    g = {k: v.astype(np.float64) for k, v in g.items()}
    # one nearly opaque Gaussian so the 0.99 clamp is exercised
    g["opacity_logit"][0] = 6.0
    return g


def surrogate(params, cam, w, tile=(8, 8), bg=(0.2, 0.1, 0.3)):
    p = oracle.project(params, cam, tile=tile)
    r = oracle.render(p, W, H, tile=tile, bg=bg)
    return float(np.sum(w * r["image"])), r, p


def decisions(r):
    return r["n_contrib"].copy(), r["n_blended"].copy()


@pytest.mark.parametrize("seed", [3, 4])
def test_render_bwd_matches_fd_on_2d_inputs(seed):
    params = make_params(seed)
    cam = cam_at()
    tile = (8, 8)
    bg = (0.2, 0.1, 0.3)
    p = oracle.project(params, cam, tile=tile)
    rng = np.random.default_rng(seed)
    w = rng.normal(size=(3, H, W))
    base = oracle.render(p, W, H, tile=tile, bg=bg)
    an = oracle.render_bwd(p, W, H, w, tile=tile, bg=bg)
    assert (base["n_blended"] > 0).sum() > 200
    checked = rejected = 0
    for key, dkey, rows in (("mean2d", "d_mean2d", 2), ("conic", "d_conic", 3),
                            ("opacity", "d_opacity", 1), ("rgb", "d_rgb", 3)):
        for i in np.nonzero(p["valid"])[0][:25]:
            for r_ in range(rows):
                q = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in p.items()}
                arr = q[key] if rows > 1 else q[key][None, :]
                x0 = arr[r_, i]
                h = 1e-6 * max(1.0, abs(x0))
                arr[r_, i] = x0 + h
                rp = oracle.render(q, W, H, tile=tile, bg=bg)
                arr[r_, i] = x0 - h
                rm = oracle.render(q, W, H, tile=tile, bg=bg)
                if any(not np.array_equal(a, b) for a, b in zip(decisions(rp) + decisions(rm),
                                                                 decisions(base) * 2)):
                    rejected += 1
                    continue
                fd = (np.sum(w * rp["image"]) - np.sum(w * rm["image"])) / (2 * h)
                g = an[dkey][r_, i] if rows > 1 else an[dkey][i]
                scale = an["abs_mass"][{"mean2d": 0, "conic": 2, "opacity": 5, "rgb": 6}[key] + r_, i]
                assert abs(fd - g) <= 1e-6 * max(abs(g), 1e-3 * scale) + 1e-8, (key, r_, i, fd, g)
                checked += 1
    assert checked > 150 and rejected <= checked // 10


@pytest.mark.parametrize("seed", [7, 8])
def test_full_chain_matches_fd_on_parameters(seed):
    params = make_params(seed, n=32)
    R, t = scene.look_at((0.4, -0.3, -0.2), target=(0.0, 0.0, 2.2), up=(0, 1, 0))
    cam = cam_at(R=R, t=t)
    rng = np.random.default_rng(seed)
    w = rng.normal(size=(3, H, W))
    L0, r0, p0 = surrogate(params, cam, w)
    assert p0["valid"].sum() >= 20
    g2d = oracle.render_bwd(p0, W, H, w, tile=(8, 8), bg=(0.2, 0.1, 0.3))
    an = oracle.project_bwd(params, cam, g2d, tile=(8, 8))
    checked = rejected = 0
    for key in ("mean", "log_scale", "quat", "opacity_logit", "color"):
        arr = params[key]
        rows = arr.shape[0] if arr.ndim == 2 else 1
        for i in np.nonzero(p0["valid"])[0][:12]:
            for r_ in range(rows):
                ref = arr if arr.ndim == 2 else arr[None, :]
                x0 = ref[r_, i]
                h = 1e-6 * max(1.0, abs(x0))
                ref[r_, i] = x0 + h
                Lp, rp, _ = surrogate(params, cam, w)
                ref[r_, i] = x0 - h
                Lm, rm, _ = surrogate(params, cam, w)
                ref[r_, i] = x0
                if any(not np.array_equal(a, b) for a, b in zip(decisions(rp) + decisions(rm),
                                                                 decisions(r0) * 2)):
                    rejected += 1
                    continue
                fd = (Lp - Lm) / (2 * h)
                g = an[key][r_, i] if arr.ndim == 2 else an[key][i]
                assert abs(fd - g) <= 2e-6 * abs(g) + 2e-7, (key, r_, i, fd, g)
                checked += 1
    assert checked >= 150 and rejected <= checked // 10


def test_clamped_alpha_has_no_geometry_gradient():
    # a Gaussian whose alpha is clamped at 0.99 at every covered pixel: its
    # mean/conic/opacity gradients vanish, its colour gradient does not
    params = dict(mean=np.array([[0.0], [0.0], [2.0]]), log_scale=np.log(np.full((3, 1), 0.02)),
                  quat=np.array([[1.0], [0.0], [0.0], [0.0]]), opacity_logit=np.array([12.0]),
                  color=np.array([[1.0], [1.0], [1.0]]))
    # cov so small that only the nearest pixels see it, with o e^power > 0.99
    cam = cam_at(f=8.0)
    p = oracle.project(params, cam, tile=(8, 8))
    r = oracle.render(p, W, H, tile=(8, 8))
    g = oracle.render_bwd(p, W, H, np.ones((3, H, W)), tile=(8, 8))
    covered = r["n_blended"] > 0
    # every blended pixel is clamped only if 0.99 <= o exp(power) there
    dx = np.arange(W) + 0.5 - p["mean2d"][0, 0]
    dy = np.arange(H) + 0.5 - p["mean2d"][1, 0]
    Q = p["conic"][:, 0]
    a = p["opacity"][0] * np.exp(-0.5 * (Q[0] * dx[None, :] ** 2 + 2 * Q[1] * dx[None, :] * dy[:, None]
                                         + Q[2] * dy[:, None] ** 2))
    if np.all(a[covered] >= 0.99):
        assert np.all(g["d_mean2d"] == 0) and np.all(g["d_conic"] == 0) and g["d_opacity"][0] == 0
    assert np.all(g["d_rgb"][:, 0] > 0)


def test_project_bwd_frustum_clamp_branch():
    # a Gaussian far to the side (t_x/t_z beyond 1.3 tan(fov/2)) still has a
    # visible footprint; the clamped branch must match FD as well
    params = dict(mean=np.array([[1.05], [0.0], [1.0]]), log_scale=np.log(np.array([[0.6], [0.2], [0.3]])),
                  quat=np.array([[0.9], [0.2], [-0.1], [0.3]]), opacity_logit=np.array([2.0]),
                  color=np.array([[0.3], [0.1], [-0.2]]))
    cam = cam_at(f=30.0)
    p = oracle.project(params, cam, tile=(8, 8))
    assert p["valid"][0] == 1 and p["mean2d"][0, 0] > W * 1.1
    rng = np.random.default_rng(0)
    g2d = dict(d_mean2d=rng.normal(size=(2, 1)), d_conic=rng.normal(size=(3, 1)),
               d_opacity=rng.normal(size=1), d_rgb=rng.normal(size=(3, 1)))

    def lin(pr):
        q = oracle.project(pr, cam, tile=(8, 8))
        return (np.sum(g2d["d_mean2d"] * q["mean2d"]) + np.sum(g2d["d_conic"] * q["conic"])
                + np.sum(g2d["d_opacity"] * q["opacity"]) + np.sum(g2d["d_rgb"] * q["rgb"]))

    an = oracle.project_bwd(params, cam, g2d, tile=(8, 8))
    for key in params:
        for r_ in range(params[key].shape[0] if params[key].ndim == 2 else 1):
            ref = params[key] if params[key].ndim == 2 else params[key][None, :]
            x0 = ref[r_, 0]; h = 1e-6 * max(1.0, abs(x0))
            ref[r_, 0] = x0 + h; Lp = lin(params)
            ref[r_, 0] = x0 - h; Lm = lin(params)
            ref[r_, 0] = x0
            g = an[key][r_, 0] if params[key].ndim == 2 else an[key][0]
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - g) <= 1e-6 * abs(g) + 1e-7, (key, r_, fd, g)


def test_term_mass_bounds_contributions():
    # the pre-cancellation term mass is never below the post-cancellation mass
    params = make_params(11)
    cam = cam_at()
    p = oracle.project(params, cam, tile=(8, 8))
    w = np.random.default_rng(1).normal(size=(3, H, W))
    g = oracle.render_bwd(p, W, H, w, tile=(8, 8))
    assert np.all(g["term_mass"] >= g["abs_mass"] * (1 - 1e-12))
    np.testing.assert_allclose(g["term_mass"][6:], g["abs_mass"][6:], rtol=1e-12)
    assert np.all(g["abs_mass"] >= np.abs(np.concatenate([g["d_mean2d"], g["d_conic"],
                                                          g["d_opacity"][None], g["d_rgb"]])) * (1 - 1e-12))
