"""Pins of the oracle's projection and compositing (no GPU).

The paper prints no worked example (its Sec. II delegates the step to the
cited 3D-GS method), so every expected value here is a closed form of a
special case derived by hand, a brute-force evaluation, or an invariant.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2509_12138_amd import scene

F = 32.0
W = H = 32
EYE = np.eye(3)


def cam_axis(W=W, H=H, f=F, R=EYE, t=(0.0, 0.0, 0.0)):
    """Camera record kept in FP64 (the oracle reads whatever precision it is given)."""
    return dict(R=np.asarray(R, np.float64).ravel(), t=np.asarray(t, np.float64), fx=f, fy=f,
                cx=W / 2.0, cy=H / 2.0, znear=0.2, width=W, height=H)


def one(mean, scale, quat=(1, 0, 0, 0), opacity=0.5, color=(0, 0, 0)):
    mean = np.asarray(mean, np.float64).reshape(3, 1)
    s = np.asarray(scale, np.float64).reshape(-1)
    if s.size == 1:
        s = np.repeat(s, 3)
    return dict(mean=mean, log_scale=np.log(s).reshape(3, 1),
                quat=np.asarray(quat, np.float64).reshape(4, 1),
                opacity_logit=np.array([math.log(opacity / (1 - opacity))]),
                color=np.asarray(color, np.float64).reshape(3, 1))


def rgb_to_sh(c):
    return (np.asarray(c, np.float64) - 0.5) / oracle.C0


def cat(*ps):
    return {k: np.concatenate([p[k] for p in ps], axis=-1) for k in ps[0]}


# ---------------------------------------------------------------- projection

def test_on_axis_isotropic_closed_form():
    # camera at the origin looking down +z, mu = (0,0,2), s = 0.1: the
    # Jacobian is diag(f/z, f/z) so Sigma2 = (f s / z)^2 I + 0.3 I
    p = oracle.project(one((0, 0, 2), 0.1), cam_axis())
    var = (F * 0.1 / 2.0) ** 2 + 0.3
    assert p["valid"][0] == 1
    np.testing.assert_allclose(p["mean2d"][:, 0], [16.0, 16.0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(p["cov2d"][:, 0], [var, 0.0, var], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(p["conic"][:, 0], [1 / var, 0.0, 1 / var], rtol=1e-12, atol=1e-15)
    kappa = 2 * math.log(255 * 0.5)
    h = math.sqrt(kappa * var)
    assert abs(h - 5.26604459) < 1e-6
    lo, hi = math.floor(16 - h) - 1, math.floor(16 + h) + 1
    assert (lo, hi) == (9, 22)
    np.testing.assert_array_equal(p["pix_bbox"][:, 0], [9, 9, 22, 22])
    np.testing.assert_array_equal(p["tile_bbox"][:, 0], [0, 0, 1, 1])
    assert p["n_tiles"][0] == 4
    assert p["depth"][0] == 2.0
    np.testing.assert_allclose(p["opacity"][0], 0.5, rtol=1e-15)


def test_axis_aligned_anisotropic_and_quarter_turn():
    sx, sy, sz = 0.05, 0.12, 0.3
    k = (F / 2.0) ** 2
    p = oracle.project(one((0, 0, 2), (sx, sy, sz)), cam_axis())
    np.testing.assert_allclose(p["cov2d"][:, 0], [k * sx * sx + 0.3, 0, k * sy * sy + 0.3],
                               rtol=1e-12, atol=1e-14)
    # a 90-degree turn about z swaps the x and y extents
    c, s = math.cos(math.pi / 4), math.sin(math.pi / 4)
    p = oracle.project(one((0, 0, 2), (sx, sy, sz), quat=(c, 0, 0, s)), cam_axis())
    np.testing.assert_allclose(p["cov2d"][:, 0], [k * sy * sy + 0.3, 0, k * sx * sx + 0.3],
                               rtol=1e-12, atol=1e-12)
    # quaternion norm does not matter
    p2 = oracle.project(one((0, 0, 2), (sx, sy, sz), quat=(3 * c, 0, 0, 3 * s)), cam_axis())
    np.testing.assert_allclose(p2["cov2d"], p["cov2d"], rtol=1e-13)
    # a Gaussian stretched along the view axis looks the same as an isotropic
    # one of the two transverse scales (J's third column vanishes on axis)
    p3 = oracle.project(one((0, 0, 2), (sx, sy, 5.0)), cam_axis())
    np.testing.assert_allclose(p3["cov2d"][:, 0], [k * sx * sx + 0.3, 0, k * sy * sy + 0.3],
                               rtol=1e-12, atol=1e-14)


def test_off_axis_mean_and_depth_jacobian():
    # point off-axis: mean2d = f x/z + c; the 2D covariance of a tiny
    # isotropic Gaussian tends to sigma^2 J J^T + 0.3 I with J from the
    # pinhole derivative
    mu = np.array([0.3, -0.2, 2.5])
    s = 1e-3
    p = oracle.project(one(mu, s), cam_axis(W=64, H=64))
    np.testing.assert_allclose(p["mean2d"][:, 0], [F * 0.3 / 2.5 + 32, F * -0.2 / 2.5 + 32],
                               rtol=1e-14)
    z = mu[2]
    J = np.array([[F / z, 0, -F * mu[0] / z ** 2], [0, F / z, -F * mu[1] / z ** 2]])
    V = s * s * J @ J.T
    np.testing.assert_allclose(p["cov2d"][:, 0], [V[0, 0] + 0.3, V[0, 1], V[1, 1] + 0.3],
                               rtol=1e-12)


def test_rotated_camera_equals_moved_gaussian():
    # rotating the camera by R is the same as rotating the scene by R^T
    rng = np.random.default_rng(0)
    A = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    if np.linalg.det(A) < 0:
        A[:, 0] *= -1
    g = one((0.1, 0.05, 0.0), (0.1, 0.05, 0.02), quat=(0.9, 0.1, 0.3, -0.2))
    t = np.array([0.0, 0.0, 3.0])
    p1 = oracle.project(g, cam_axis(W=64, H=64, R=A, t=t))
    # move the Gaussian instead: mean -> A mean, rotation -> A R
    w, x, y, z = g["quat"][:, 0] / np.linalg.norm(g["quat"][:, 0])
    Rq = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                   [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                   [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    R2 = A @ Rq
    # quaternion of R2 (Shepperd)
    tr = np.trace(R2)
    qw = math.sqrt(max(0.0, 1 + tr)) / 2
    q2 = np.array([qw, (R2[2, 1] - R2[1, 2]) / (4 * qw), (R2[0, 2] - R2[2, 0]) / (4 * qw),
                   (R2[1, 0] - R2[0, 1]) / (4 * qw)])
    g2 = dict(g); g2["mean"] = (A @ g["mean"][:, 0]).reshape(3, 1); g2["quat"] = q2.reshape(4, 1)
    p2 = oracle.project(g2, cam_axis(W=64, H=64, t=t))
    for k in ("mean2d", "cov2d", "conic", "depth"):
        np.testing.assert_allclose(p1[k], p2[k], rtol=1e-10, atol=1e-12)


def test_culling_rules():
    cam = cam_axis()
    assert oracle.project(one((0, 0, 0.1), 0.1), cam)["valid"][0] == 0      # behind near
    assert oracle.project(one((0, 0, -2), 0.1), cam)["valid"][0] == 0       # behind camera
    assert oracle.project(one((0, 0, 2), 0.1, opacity=1 / 255.0 * 0.999), cam)["valid"][0] == 0
    assert oracle.project(one((0, 0, 2), 0.1, opacity=1 / 255.0 * 1.01), cam)["valid"][0] == 1
    far = oracle.project(one((5.0, 0, 2), 0.01), cam)                         # off screen
    assert far["valid"][0] == 0 and far["n_tiles"][0] == 0


def test_colour_activation():
    p = oracle.project(one((0, 0, 2), 0.1, color=rgb_to_sh([1.0, 0.5, -0.2])), cam_axis())
    np.testing.assert_allclose(p["rgb"][:, 0], [1.0, 0.5, 0.0], atol=1e-15)


# ---------------------------------------------------------------- compositing

def render_scene(g, W=W, H=H, cam=None, **kw):
    cam = cam or cam_axis(W=W, H=H)
    p = oracle.project(g, cam)
    return p, oracle.render(p, W, H, **kw)


def test_single_gaussian_pixels():
    var = (F * 0.1 / 2.0) ** 2 + 0.3
    _, r = render_scene(one((0, 0, 2), 0.1, color=rgb_to_sh([1.0, 0.5, 0.0])))
    img = r["image"]
    for (px, py) in [(16, 16), (18, 16), (15, 14), (20, 19)]:
        d2 = (px + 0.5 - 16) ** 2 + (py + 0.5 - 16) ** 2
        a = 0.5 * math.exp(-0.5 * d2 / var)
        exp_val = [a, 0.5 * a, 0.0] if a >= 1 / 255 else [0, 0, 0]
        np.testing.assert_allclose(img[:, py, px], exp_val, rtol=1e-13, atol=1e-15)
        assert abs(r["T_final"][py, px] - (1 - a if a >= 1 / 255 else 1.0)) < 1e-13
    assert abs(img[0, 16, 16] - 0.458149482) < 1e-9
    # pixel (21, 16): alpha = 0.00241679 < 1/255 -> skipped
    assert img[0, 16, 21] == 0.0 and r["n_contrib"][16, 21] == 0
    assert r["n_contrib"][16, 16] == 1 and r["n_blended"][16, 16] == 1
    # outside the tile bbox nothing is evaluated
    assert np.all(img[:, :, 23:] == 0)


def test_two_gaussian_ordering():
    c1, c2 = rgb_to_sh([1.0, 0.5, 0.0]), rgb_to_sh([0.0, 0.0, 1.0])
    g1 = one((0, 0, 2), 0.1, color=c1)
    g2 = one((0, 0, 3), 0.15, color=c2)             # same 2D footprint, behind
    _, r = render_scene(cat(g1, g2))
    var = (F * 0.1 / 2.0) ** 2 + 0.3
    a = 0.5 * math.exp(-0.5 * 0.5 / var)
    np.testing.assert_allclose(r["image"][:, 16, 16], [a, 0.5 * a, a * (1 - a)], rtol=1e-12)
    assert abs(r["T_final"][16, 16] - (1 - a) ** 2) < 1e-13
    # swapped depths swap the layering; listing order does not matter
    _, r2 = render_scene(cat(one((0, 0, 3), 0.15, color=c1), one((0, 0, 2), 0.1, color=c2)))
    np.testing.assert_allclose(r2["image"][:, 16, 16], [a * (1 - a), 0.5 * a * (1 - a), a],
                               rtol=1e-12)
    _, r3 = render_scene(cat(g2, g1))
    np.testing.assert_array_equal(r3["image"], r["image"])


def test_transmittance_cutoff_stack():
    # alpha = 0.5 exactly (mean on the pixel centre, o = 0.5): blending k
    # Gaussians leaves T = 2^-k; the 14th would drop T below 1e-4
    mu_x = (16.5 - 16) * 2.0 / F
    gs = [one((mu_x * (2 + 0.1 * i) / 2.0, mu_x * (2 + 0.1 * i) / 2.0, 2 + 0.1 * i), 0.01,
              color=rgb_to_sh([1, 1, 1])) for i in range(20)]
    p, r = render_scene(cat(*gs))
    np.testing.assert_allclose(p["mean2d"][:, :], 16.5, rtol=0, atol=1e-12)
    k = math.ceil(math.log(1e-4) / math.log(0.5)) - 1
    assert k == 13
    assert r["n_blended"][16, 16] == 13
    assert r["n_contrib"][16, 16] == 13
    assert abs(r["T_final"][16, 16] - 0.5 ** 13) < 1e-15
    assert abs(r["image"][0, 16, 16] - (1 - 0.5 ** 13)) < 1e-13


def test_alpha_clamp_099():
    # o close to 1 at the centre: alpha clamps to 0.99
    g = one((0.5 * 2 / F, 0.5 * 2 / F, 2), 0.1, opacity=0.999, color=rgb_to_sh([1, 1, 1]))
    _, r = render_scene(g)
    assert abs(r["image"][0, 16, 16] - 0.99) < 1e-14
    assert abs(r["T_final"][16, 16] - 0.01) < 1e-14


def brute_force_image(p, W, H, bg=(0, 0, 0)):
    """Independent per-pixel evaluation over ALL Gaussians (no bboxes)."""
    n = p["depth"].shape[0]
    order = sorted([i for i in range(n) if p["valid"][i]], key=lambda i: (p["depth"][i], i))
    img = np.zeros((3, H, W))
    for y in range(H):
        for x in range(W):
            T, C = 1.0, np.zeros(3)
            for i in order:
                d = np.array([x + 0.5, y + 0.5]) - p["mean2d"][:, i]
                Q = np.array([[p["conic"][0, i], p["conic"][1, i]],
                              [p["conic"][1, i], p["conic"][2, i]]])
                power = -0.5 * d @ Q @ d
                if power > 0:
                    continue
                alpha = min(0.99, p["opacity"][i] * math.exp(power))
                if alpha < 1 / 255:
                    continue
                if T * (1 - alpha) < 1e-4:
                    break
                C += p["rgb"][:, i] * alpha * T
                T *= 1 - alpha
            img[:, y, x] = C + T * np.asarray(bg)
    return img


@pytest.mark.parametrize("seed", [0, 1])
def test_brute_force_agrees(seed):
    g = scene.random_gaussians(48, seed, center=(0, 0, 2.2), extent=0.5, log_scale=(-3.2, -1.8))
    cam = cam_axis()
    p = oracle.project({k: v.astype(np.float64) for k, v in g.items()}, cam, tile=(8, 8))
    assert p["valid"].sum() > 20
    r = oracle.render(p, W, H, tile=(8, 8), bg=(0.1, 0.2, 0.3))
    ref = brute_force_image(p, W, H, bg=(0.1, 0.2, 0.3))
    np.testing.assert_allclose(r["image"], ref, rtol=0, atol=1e-12)
    # a different bin tile gives the same image (bboxes are conservative)
    r2 = oracle.render(oracle.project({k: v.astype(np.float64) for k, v in g.items()}, cam,
                                      tile=(16, 4)), W, H, tile=(16, 4), bg=(0.1, 0.2, 0.3))
    np.testing.assert_allclose(r2["image"], ref, rtol=0, atol=1e-12)


def test_permutation_invariance():
    g = scene.random_gaussians(300, 5, center=(0, 0, 2.0), extent=0.6)
    perm = np.random.default_rng(1).permutation(300)
    gp = {k: v[..., perm] for k, v in g.items()}
    cam = cam_axis(W=48, H=40)
    r1 = oracle.render(oracle.project(g, cam), 48, 40)
    r2 = oracle.render(oracle.project(gp, cam), 48, 40)
    np.testing.assert_array_equal(r1["image"], r2["image"])
    np.testing.assert_array_equal(r1["T_final"], r2["T_final"])


def test_window_matches_full_render():
    g = scene.random_gaussians(200, 9, center=(0, 0, 2.0), extent=0.6)
    cam = cam_axis(W=48, H=40)
    p = oracle.project(g, cam)
    full = oracle.render(p, 48, 40)
    win = oracle.render(p, 48, 40, window=(5, 7, 30, 33))
    np.testing.assert_array_equal(win["image"][:, 7:33, 5:30], full["image"][:, 7:33, 5:30])


def test_decision_bands_classify_only():
    """The guard-band width marks which pixels sit near a threshold (an
    opacity of 1/255 (1 + 5e-4) at the pixel centre is outside a 1e-5 band
    and inside a 1e-3 one; likewise 0.99 (1 - 5e-4) for the clamp) and
    never changes the composite."""
    cx = 0.5 * 2 / F
    for o, bit in (((1 / 255) * (1 + 5e-4), 2), (0.99 * (1 - 5e-4), 4)):
        g = one((cx, cx, 2), 0.1, opacity=o, color=rgb_to_sh([1, 1, 1]))
        _, narrow = render_scene(g)
        _, wide = render_scene(g, band=1e-3)
        np.testing.assert_array_equal(narrow["image"], wide["image"])
        np.testing.assert_array_equal(narrow["T_final"], wide["T_final"])
        assert not narrow["ambiguity"][16, 16] & bit
        assert wide["ambiguity"][16, 16] & bit
        assert np.all(wide["ambiguous"] >= narrow["ambiguous"])


def test_depth_tie_at_the_stopping_entry_is_ambiguous():
    """The pixel of the transmittance-cut-off stack stops at its 14th
    Gaussian; a further Gaussian that passes the alpha test at a depth
    within 5e-7 (relative) of that stopping one could be sorted before it
    from FP32 depths and then be blended, so the pixel is marked (reason
    16); at a clearly larger depth it is not, and the composite is the same
    either way at that pixel."""
    mu_x = (16.5 - 16) * 2.0 / F

    def g_at(z):
        return one((mu_x * z / 2.0, mu_x * z / 2.0, z), 0.01, color=rgb_to_sh([1, 1, 1]))

    base = [g_at(2 + 0.1 * i) for i in range(14)]
    z_stop = 2 + 0.1 * 13
    _, r0 = render_scene(cat(*base))
    _, r_far = render_scene(cat(*base, g_at(z_stop * (1 + 1e-3))))
    _, r_tie = render_scene(cat(*base, g_at(z_stop * (1 + 1e-7))))
    assert r0["n_blended"][16, 16] == 13 and r_tie["n_blended"][16, 16] == 13
    assert not r0["ambiguity"][16, 16] & 16
    assert not r_far["ambiguity"][16, 16] & 16
    assert r_tie["ambiguity"][16, 16] & 16
    np.testing.assert_array_equal(r_tie["image"][:, 16, 16], r0["image"][:, 16, 16])
