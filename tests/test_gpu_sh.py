"""GPU parity of the view-dependent colour (spherical harmonics of degree 1-3)
through the C ABI: gs_project's colours, gs_project_bwd's colour and mean
gradients, a model stored at degree 3 drawn at a lower degree, and the fused
projection-backward + Adam call, against the FP64 oracle or the unfused
calls.  Tolerances as the degree-0 parity tests: projection 1e-5 relative,
gradients 1e-4 in norm and 1e-3 per element with a floor of 1e-5 x the
largest, fused Adam bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_2509_12138_amd import scene
from _gpu_helpers import perturbed, say, surface_scene, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops(gpu):
    from paper_2509_12138_amd import ops as _ops
    return _ops


def sh_params(n, seed, D, scale=0.25):
    """Perturbed surface Gaussians whose colour has 3 (D+1)^2 rows: the plain
    colour first, seeded normal higher-order coefficients after it."""
    p = perturbed(surface_scene(n, seed), seed)
    K = (D + 1) ** 2
    rng = np.random.default_rng(seed + 100)
    col = np.zeros((3 * K, n), np.float32)
    col[:3] = p["color"]
    col[3:] = scale * rng.normal(size=(3 * K - 3, n))
    p["color"] = col
    return p


def make_bufs(ops, n, cams, W, H, tile=(16, 16)):
    return ops.RasterBuffers(ops.Views.single(n, cams), W, H, tile)


def clear_pairs(params, cams):
    """Per view, the oracle's visible pairs away from FP32 decision
    boundaries (bbox edges, the 1/255 support threshold), and its colours."""
    out = []
    for c in cams:
        o = oracle.project(params, scene.camera_dict(c))
        kappa = 2 * np.log(np.maximum(255 * o["opacity"], 1e-300))
        hx = np.sqrt(np.maximum(kappa, 0) * o["cov2d"][0])
        hy = np.sqrt(np.maximum(kappa, 0) * o["cov2d"][2])
        e = np.stack([o["mean2d"][0] - hx, o["mean2d"][0] + hx, o["mean2d"][1] - hy,
                      o["mean2d"][1] + hy])
        near = np.any(np.abs(e - np.round(e)) < 1e-4, axis=0) | (np.abs(255 * o["opacity"] - 1) < 1e-4)
        out.append(((o["n_tiles"] > 0) & ~near, o))
    return out


@pytest.mark.parametrize("D", [1, 2, 3])
def test_project_colour_matches_oracle(ops, D):
    say("project sh", D)
    W, H, n = 190, 140, 3000
    params = sh_params(n, 70 + D, D)
    cams = scene.orbit_cameras(4, W, H)
    bufs = make_bufs(ops, n, cams, W, H)
    gst = ops.gaussians_struct(to_dev(params, torch))
    assert gst.sh_degree == D
    bufs.project(gst)
    torch.cuda.synchronize()
    rec = bufs.rec.cpu().numpy()
    for v, (ok, o) in enumerate(clear_pairs(params, cams)):
        r = rec[v * n:(v + 1) * n]
        assert ok.sum() > 500
        np.testing.assert_allclose(r[ok, 6:9], o["rgb"].T[ok], rtol=1e-5, atol=2e-6)
        np.testing.assert_allclose(r[ok, 0:2], o["mean2d"].T[ok], rtol=1e-5, atol=1e-4)
    # the colour really varies with the view: the same Gaussian differs
    # between views by far more than the tolerance
    rgb = rec[:, 6:9].reshape(4, n, 3)
    vis = np.all(rec[:, 5].reshape(4, n) > 0, axis=0)
    assert np.median(np.abs(rgb[0, vis] - rgb[2, vis])) > 1e-2


def _oracle_grads(params, cams, drec, n):
    ref = {k: np.zeros(np.shape(v)) for k, v in params.items()}
    for v, c in enumerate(cams):
        d = drec[v * n:(v + 1) * n].astype(np.float64)
        g = oracle.project_bwd(params, scene.camera_dict(c),
                               dict(d_mean2d=d[:, 0:2].T, d_conic=d[:, 2:5].T, d_opacity=d[:, 5],
                                    d_rgb=d[:, 6:9].T))
        for k in ref:
            ref[k] += g[k]
    return ref


def _check(got, ref, keys):
    for k in keys:
        g = got[k].astype(np.float64)
        r = ref[k]
        nr = np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-30)
        assert nr <= 1e-4, (k, nr)
        scale = np.abs(r).max()
        assert np.all(np.abs(g - r) <= 1e-3 * np.abs(r) + 1e-5 * scale), k


def _upstream(params, cams, n, seed):
    """Seeded upstream gradients on clearly visible pairs; colour channels
    the oracle clamps (or nearly) get none, so the clamp decision never
    depends on FP32 rounding."""
    rng = np.random.default_rng(seed)
    parts = []
    for ok, o in clear_pairs(params, cams):
        d = rng.normal(size=(n, 9)) * ok[:, None]
        d[:, 6:9] *= (o["rgb"].T > 1e-4)
        parts.append(d)
    return np.concatenate(parts).astype(np.float32)


@pytest.mark.parametrize("D", [1, 2, 3])
def test_project_bwd_colour_and_mean_gradients_match_oracle(ops, D):
    say("project_bwd sh", D)
    W, H, n = 200, 150, 4000
    params = sh_params(n, 80 + D, D)
    cams = scene.orbit_cameras(3, W, H)
    bufs = make_bufs(ops, n, cams, W, H)
    dp = to_dev(params, torch)
    gst = ops.gaussians_struct(dp)
    bufs.project(gst)
    drec = _upstream(params, cams, n, D)
    bufs.d_rec.copy_(torch.as_tensor(drec))
    grads = {k: torch.zeros_like(v) for k, v in dp.items()}
    bufs.project_bwd(gst, ops.grads_struct(grads, n))
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in grads.items()}
    _check(got, _oracle_grads(params, cams, drec, n), params.keys())


def test_lower_active_degree_draws_the_leading_rows(ops):
    say("sh stored 3, drawn at 1")
    W, H, n = 160, 120, 3000
    params = sh_params(n, 90, 3)
    low = dict(params, color=params["color"][:12].copy())
    cams = scene.orbit_cameras(3, W, H)
    bufs = make_bufs(ops, n, cams, W, H)
    dp = to_dev(params, torch)
    gst = ops.gaussians_struct(dp, sh_degree=1)
    bufs.project(gst)
    torch.cuda.synchronize()
    rec = bufs.rec.cpu().numpy()
    for v, (ok, o) in enumerate(clear_pairs(low, cams)):
        np.testing.assert_allclose(rec[v * n:(v + 1) * n][ok, 6:9], o["rgb"].T[ok], rtol=1e-5,
                                   atol=2e-6)
    drec = _upstream(low, cams, n, 5)
    bufs.d_rec.copy_(torch.as_tensor(drec))
    grads = {k: torch.zeros_like(v) for k, v in dp.items()}
    bufs.project_bwd(gst, ops.grads_struct(grads, n))
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in grads.items()}
    assert np.all(got["color"][12:] == 0)
    got["color"] = got["color"][:12]
    _check(got, _oracle_grads(low, cams, drec, n), low.keys())
    with pytest.raises(ValueError):
        ops.gaussians_struct(dict(dp, color=dp["color"][:12].contiguous()), sh_degree=2)


@pytest.mark.parametrize("D,active,V,rest", [(3, 3, 3, False), (3, 1, 3, False), (1, 1, 3, False),
                                             (3, 3, 1, False), (3, 2, 1, False), (1, 1, 1, False),
                                             (3, 3, 1, True), (3, 3, 3, True), (2, 1, 1, True)])
def test_fused_projection_backward_adam_bitwise_with_sh(ops, D, active, V, rest):
    """Fused against unfused, several slots (LDS sums) and one slot (the
    kernel that keeps only the pair's direction and colour gradient); with
    rest, six Adam groups step the higher bands at their own rate."""
    say("project_bwd + adam fused, sh", D, active, V, rest)
    W, H, n = 200, 150, 4000
    params = sh_params(n, 95, D)
    cams = scene.orbit_cameras(V, W, H)
    lrs = {"mean": 4.4e-4, "log_scale": 5e-3, "quat": 1e-3, "opacity_logit": 5e-2,
           "color": 2.5e-3}
    if rest:
        lrs["color_rest"] = 2.5e-3 / 20
    runs = []
    for fused in (False, True):
        bufs = make_bufs(ops, n, cams, W, H)
        dp = to_dev(params, torch)
        gst = ops.gaussians_struct(dp, sh_degree=active)
        dm = {k: torch.zeros_like(v) for k, v in dp.items()}
        dv = {k: torch.zeros_like(v) for k, v in dp.items()}
        dg = {k: torch.zeros_like(v) for k, v in dp.items()}
        adam = ops.DeviceAdam(ops.adam_groups(dp, dg, dm, dv, lrs),
                              lr_final=[4.4e-6, 0, 0, 0, 0], decay_steps=7)
        rng = np.random.default_rng(6)
        for step in range(3):
            bufs.project(gst)
            drec = rng.normal(size=(V * n, 9)).astype(np.float32)
            drec[rng.uniform(size=V * n) < 0.3] = 0.0
            bufs.d_rec.copy_(torch.as_tensor(drec))
            if fused:
                bufs.project_bwd_adam(gst, adam)
            else:
                bufs.project_bwd(gst, ops.grads_struct(dg, n))
                adam(zero_grad=True)
        torch.cuda.synchronize()
        runs.append([{k: v.cpu().numpy() for k, v in d.items()} for d in (dp, dm, dv)])
    for a, b in zip(runs[0], runs[1]):
        for k in a:
            np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    K = (active + 1) ** 2
    moved = runs[1][0]["color"] != params["color"]
    assert moved[:3 * K].any()
    assert not moved[3 * K:].any()          # rows above the active degree stay put
    if rest:
        # three Adam steps move a parameter by at most about 3 lr
        step = np.abs(runs[1][0]["color"].astype(np.float64) - params["color"])
        assert step[3:3 * K].max() <= 3.05 * lrs["color_rest"]
        assert step[:3].max() > 3.05 * lrs["color_rest"]
