"""Pins of the oracle's view-dependent colour (no GPU).

The colour of a Gaussian is max(0, sum_k Y_k(d) c_k + 1/2) with Y_k the real
spherical harmonics of degree <= 3 and d the unit vector from the camera
centre to the mean (the 3D-GS colour model behind the paper's
view-dependent images, Sec. I).  The oracle evaluates Y_k from the textbook
definition (Legendre-polynomial derivatives); these tests tie that to
quadrature, to scipy's complex harmonics, to finite differences and to
closed-form views, and the analytic backward to central differences of the
FP64 forward.
"""
import math

import numpy as np
import pytest
import scipy.special

import oracle
from paper_2509_12138_amd import scene

W, H = 40, 32


def cam_at(f=36.0, R=np.eye(3), t=(0.0, 0.0, 0.0)):
    return dict(R=np.asarray(R, np.float64).ravel(), t=np.asarray(t, np.float64), fx=f, fy=f,
                cx=W / 2.0, cy=H / 2.0, znear=0.2, width=W, height=H)


def sphere_dirs(n, seed):
    v = np.random.default_rng(seed).normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def with_sh(params, D, seed, scale=0.3):
    """Copy of params whose colour has degree D: the plain coefficients in
    rows 0..2, seeded normal higher-order coefficients after them."""
    p = {k: np.array(v, np.float64, copy=True) for k, v in params.items()}
    n = p["opacity_logit"].shape[0]
    K = (D + 1) ** 2
    rng = np.random.default_rng(seed)
    col = np.zeros((3 * K, n))
    col[:3] = p["color"][:3]
    col[3:] = scale * rng.normal(size=(3 * K - 3, n))
    p["color"] = col
    return p


def test_sh_orthonormal_on_the_sphere():
    # Gauss-Legendre in z (8 nodes) x 16 uniform azimuths integrates every
    # product of two degree-3 harmonics exactly
    z, wz = np.polynomial.legendre.leggauss(8)
    phi = 2 * np.pi * np.arange(16) / 16
    Z, P = np.meshgrid(z, phi, indexing="ij")
    r = np.sqrt(1 - Z ** 2)
    d = np.stack([r * np.cos(P), r * np.sin(P), Z], -1).reshape(-1, 3)
    w = np.repeat(wz, 16) * (2 * np.pi / 16)
    Y, _ = oracle.sh_basis(3, d)
    gram = (Y * w[:, None]).T @ Y
    assert np.abs(gram - np.eye(16)).max() < 1e-12


def test_sh_matches_scipy_complex_harmonics():
    # real form with the Condon-Shortley phase: m > 0 -> sqrt2 Re Y_l^m,
    # m < 0 -> sqrt2 Im Y_l^|m|, m = 0 -> Y_l^0 (scipy's Y_l^m carries the
    # phase in its associated Legendre function)
    d = sphere_dirs(200, 1)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    Y, _ = oracle.sh_basis(3, d)
    for l in range(4):
        for m in range(-l, l + 1):
            c = scipy.special.sph_harm_y(l, abs(m), theta, phi)
            ref = c.real if m == 0 else math.sqrt(2) * (c.real if m > 0 else c.imag)
            assert np.abs(Y[:, l * l + l + m] - ref).max() < 1e-12, (l, m)


def test_sh_known_values():
    # a few values fixed by hand: Y_00 = 1/(2 sqrt(pi)); Y_1,1 at +x is
    # -sqrt(3/(4 pi)) (Condon-Shortley sign); Y_20 at +z is sqrt(5/(4 pi))
    Y, _ = oracle.sh_basis(3, np.array([[1.0, 0, 0], [0, 0, 1.0]]))
    assert Y[0, 0] == pytest.approx(0.5 / math.sqrt(math.pi), abs=1e-15)
    assert Y[0, 3] == pytest.approx(-math.sqrt(3 / (4 * math.pi)), abs=1e-14)
    assert Y[1, 6] == pytest.approx(math.sqrt(5 / (4 * math.pi)), abs=1e-14)
    assert Y[1, 12] == pytest.approx(math.sqrt(7 / (4 * math.pi)), abs=1e-14)


def test_sh_gradient_matches_fd_along_the_sphere():
    d = sphere_dirs(20, 2)
    _, G = oracle.sh_basis(3, d)
    rng = np.random.default_rng(3)
    h = 1e-6
    for i in range(len(d)):
        t = rng.normal(size=3)
        t -= d[i] * (t @ d[i])
        t /= np.linalg.norm(t)
        dp = d[i] + h * t; dp /= np.linalg.norm(dp)
        dm = d[i] - h * t; dm /= np.linalg.norm(dm)
        Yp, _ = oracle.sh_basis(3, dp[None])
        Ym, _ = oracle.sh_basis(3, dm[None])
        fd = (Yp[0] - Ym[0]) / (2 * h)
        assert np.abs(fd - G[i] @ t).max() < 1e-8


def one_gaussian(mean, color):
    return dict(mean=np.asarray(mean, np.float64).reshape(3, 1),
                log_scale=np.log(np.full((3, 1), 0.05)),
                quat=np.array([[1.0], [0.0], [0.0], [0.0]]), opacity_logit=np.array([1.0]),
                color=np.asarray(color, np.float64).reshape(-1, 1))


def test_colour_depends_on_the_view_direction():
    # camera at the origin looking down +z (R = I, t = 0)
    C1 = math.sqrt(3 / (4 * math.pi))
    cam = cam_at()
    col = np.zeros(12)
    col[3 * 2 + 0] = 0.4            # Y_10 = C1 z, red
    col[3 * 3 + 1] = 0.5            # Y_11 = -C1 x, green
    p = oracle.project(one_gaussian((0.0, 0.0, 2.0), col), cam)
    assert p["rgb"][:, 0] == pytest.approx([C1 * 0.4 + 0.5, 0.5, 0.5], abs=1e-14)
    x = 0.6
    v = np.array([x, 0.0, 2.0]); d = v / np.linalg.norm(v)
    p = oracle.project(one_gaussian(v, col), cam)
    assert p["rgb"][:, 0] == pytest.approx(
        [C1 * d[2] * 0.4 + 0.5, -C1 * d[0] * 0.5 + 0.5, 0.5], abs=1e-14)
    # the same Gaussian seen from a camera moved to (0, 0, 4) looking back
    # down -z: the direction to the mean flips
    R = np.diag([-1.0, 1.0, -1.0])
    cam2 = cam_at(R=R, t=-R @ np.array([0.0, 0.0, 4.0]))
    p = oracle.project(one_gaussian((0.0, 0.0, 2.0), col), cam2)
    assert p["valid"][0] == 1
    assert p["rgb"][:, 0] == pytest.approx([-C1 * 0.4 + 0.5, 0.5, 0.5], abs=1e-14)


def test_degree_zero_is_the_plain_colour_and_zero_bands_change_nothing():
    params = scene.random_gaussians(50, 11, center=(0, 0, 2.2), extent=0.45,
                                    log_scale=(-3.0, -1.9), opacity=(0.2, 0.9))
    params = {k: v.astype(np.float64) for k, v in params.items()}
    cam = cam_at()
    p0 = oracle.project(params, cam)
    C0 = 0.5 / math.sqrt(math.pi)
    ref = np.maximum(C0 * params["color"] + 0.5, 0.0)
    v = p0["valid"] == 1
    assert np.abs(p0["rgb"][:, v] - ref[:, v]).max() < 1e-14
    p3 = oracle.project(with_sh(params, 3, 0, scale=0.0), cam)
    for k in p0:
        assert np.array_equal(p0[k], p3[k]) or np.abs(p0[k] - p3[k]).max() < 1e-14, k


@pytest.mark.parametrize("D", [1, 2, 3])
def test_project_bwd_matches_fd_with_sh(D):
    # a linear functional of every projected output, so no discrete decision
    # can flip; Gaussians spread across the view so the direction varies
    base = scene.random_gaussians(6, 20 + D, center=(0.1, -0.1, 2.0), extent=0.8,
                                  log_scale=(-2.5, -1.5), opacity=(0.3, 0.9))
    params = with_sh({k: v.astype(np.float64) for k, v in base.items()}, D, 5 + D)
    R, t = scene.look_at((0.3, -0.2, -0.4), target=(0.0, 0.0, 2.0), up=(0, 1, 0))
    cam = cam_at(R=R, t=t)
    p = oracle.project(params, cam, tile=(8, 8))
    valid = np.nonzero(p["valid"])[0]
    assert len(valid) >= 4
    rng = np.random.default_rng(D)
    n = params["opacity_logit"].shape[0]
    g2d = dict(d_mean2d=rng.normal(size=(2, n)), d_conic=rng.normal(size=(3, n)),
               d_opacity=rng.normal(size=n), d_rgb=rng.normal(size=(3, n)))
    # some channels clamp at 0 (their gradient is masked); most do not
    assert (p["rgb"][:, valid] > 0).mean() > 0.7

    def lin(pr):
        q = oracle.project(pr, cam, tile=(8, 8))
        s = 0.0
        for key, dkey in (("mean2d", "d_mean2d"), ("conic", "d_conic"), ("opacity", "d_opacity"),
                          ("rgb", "d_rgb")):
            s += np.sum((g2d[dkey] * q[key])[..., valid])
        return s

    an = oracle.project_bwd(params, cam, g2d, tile=(8, 8))
    for key in ("mean", "color"):
        arr = params[key]
        for i in valid:
            for r_ in range(arr.shape[0]):
                x0 = arr[r_, i]
                h = 1e-6 * max(1.0, abs(x0))
                arr[r_, i] = x0 + h; Lp = lin(params)
                arr[r_, i] = x0 - h; Lm = lin(params)
                arr[r_, i] = x0
                fd = (Lp - Lm) / (2 * h)
                g = an[key][r_, i]
                assert abs(fd - g) <= 1e-6 * abs(g) + 1e-7, (key, r_, i, fd, g)
    # the colour gradient of coefficient k, channel c is Y_k(d) dL/drgb_c
    campos = -R.T @ np.asarray(t)
    for i in valid:
        v = params["mean"][:, i] - campos
        Y, _ = oracle.sh_basis(D, (v / np.linalg.norm(v))[None])
        exp = np.outer(Y[0], g2d["d_rgb"][:, i] * (p["rgb"][:, i] > 0)).ravel()
        assert np.abs(an["color"][:, i] - exp).max() < 1e-12
