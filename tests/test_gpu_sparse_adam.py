"""GPU parity of the sparse (visible-only) Adam step of gs_project_bwd_adam
through the C ABI: Gaussians drawn by no pair keep parameters and moments
bit for bit, drawn ones get exactly the dense step, and the whole update
matches the FP64 oracle (oracle projection backward + oracle Adam with the
oracle's visibility) within the gradient tolerance of the parity tests."""
import numpy as np
import pytest

import oracle
from paper_2509_12138_amd import scene
from _gpu_helpers import perturbed, say, surface_scene, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LRS = {"mean": 4.4e-4, "log_scale": 5e-3, "quat": 1e-3, "opacity_logit": 5e-2, "color": 2.5e-3}
B1, B2, EPS = 0.9, 0.999, 1e-15


@pytest.fixture(scope="module")
def ops(gpu):
    from paper_2509_12138_amd import ops as _ops
    return _ops


def _state(n, seed, D=0):
    p = perturbed(surface_scene(n, seed), seed)
    if D:
        rng0 = np.random.default_rng(seed + 1)
        col = np.zeros((3 * (D + 1) ** 2, n), np.float32)
        col[:3] = p["color"]
        col[3:] = 0.2 * rng0.normal(size=(col.shape[0] - 3, n))
        p["color"] = col
    rng = np.random.default_rng(seed + 2)
    m = {k: (1e-3 * rng.normal(size=np.shape(v))).astype(np.float32) for k, v in p.items()}
    v = {k: (1e-6 * rng.uniform(0.5, 1.5, size=np.shape(x))).astype(np.float32)
         for k, x in p.items()}
    return p, m, v


def _run(ops, p, m, v, cams, W, H, drec, visible_only, step0):
    n = p["opacity_logit"].shape[0]
    bufs = ops.RasterBuffers(ops.Views.single(n, cams), W, H, (16, 16))
    dp, dm, dv = to_dev(p, torch), to_dev(m, torch), to_dev(v, torch)
    dg = {k: torch.zeros_like(x) for k, x in dp.items()}
    adam = ops.DeviceAdam(ops.adam_groups(dp, dg, dm, dv, LRS), beta1=B1, beta2=B2, eps=EPS)
    adam.step_dev.fill_(step0)
    gst = ops.gaussians_struct(dp)
    bufs.project(gst)
    bufs.d_rec.copy_(torch.as_tensor(drec))
    bufs.project_bwd_adam(gst, adam, visible_only=visible_only)
    torch.cuda.synchronize()
    nt = bufs.n_tiles.cpu().numpy().reshape(len(cams), n)
    return ([{k: x.cpu().numpy() for k, x in d.items()} for d in (dp, dm, dv)],
            (nt > 0).any(0), int(adam.step_dev.item()))


@pytest.mark.parametrize("D", [0, 3])
def test_sparse_step_keeps_hidden_and_equals_dense_on_drawn(ops, D):
    say("sparse adam vs dense", D)
    W, H, n = 200, 150, 5000
    p, m, v = _state(n, 120 + D, D)
    cams = scene.orbit_cameras(2, W, H, fov_x_deg=15.0)  # views that see part of the surface
    rng = np.random.default_rng(7)
    drec = rng.normal(size=(2 * n, 9)).astype(np.float32)
    (sp, sm, sv), drawn, t_s = _run(ops, p, m, v, cams, W, H, drec, True, 5)
    (dp, dm, dv), drawn_d, t_d = _run(ops, p, m, v, cams, W, H, drec, False, 5)
    assert t_s == t_d == 6
    np.testing.assert_array_equal(drawn, drawn_d)
    assert 0.2 < drawn.mean() < 0.95, drawn.mean()
    for k in p:
        for got, dense, orig in ((sp[k], dp[k], p[k]), (sm[k], dm[k], m[k]), (sv[k], dv[k], v[k])):
            got, dense, orig = (np.atleast_2d(a) for a in (got, dense, orig))
            np.testing.assert_array_equal(got[:, drawn], dense[:, drawn], err_msg=k)
            np.testing.assert_array_equal(got[:, ~drawn], orig[:, ~drawn].astype(np.float32),
                                          err_msg=k)
        # the dense step does move hidden Gaussians (momentum)
        assert not np.array_equal(np.atleast_2d(dp[k])[:, ~drawn],
                                  np.atleast_2d(p[k])[:, ~drawn].astype(np.float32))


def test_sparse_step_matches_oracle(ops):
    say("sparse adam vs oracle")
    W, H, n = 200, 150, 4000
    p, m, v = _state(n, 130)
    cams = scene.orbit_cameras(2, W, H, fov_x_deg=15.0)  # views that see part of the surface
    rng = np.random.default_rng(8)
    # upstream gradients on the oracle's clearly visible pairs; Gaussians
    # whose visibility sits at an FP32 decision boundary are left out
    vis_o, amb = np.zeros(n, bool), np.zeros(n, bool)
    parts = []
    orec = []
    for c in cams:
        o = oracle.project(p, scene.camera_dict(c))
        kappa = 2 * np.log(np.maximum(255 * o["opacity"], 1e-300))
        hx = np.sqrt(np.maximum(kappa, 0) * o["cov2d"][0])
        hy = np.sqrt(np.maximum(kappa, 0) * o["cov2d"][2])
        e = np.stack([o["mean2d"][0] - hx, o["mean2d"][0] + hx, o["mean2d"][1] - hy,
                      o["mean2d"][1] + hy])
        near = np.any(np.abs(e - np.round(e)) < 1e-4, axis=0) | (np.abs(255 * o["opacity"] - 1) < 1e-4)
        amb |= near
        ok = (o["n_tiles"] > 0) & ~near
        vis_o |= o["n_tiles"] > 0
        d = rng.normal(size=(n, 9)) * ok[:, None]
        d[:, 6:9] *= (o["rgb"].T > 1e-4)
        parts.append(d)
        orec.append(o)
    drec = np.concatenate(parts).astype(np.float32)
    (gp, gm, gv), drawn, _ = _run(ops, p, m, v, cams, W, H, drec, True, 5)
    clear = ~amb
    np.testing.assert_array_equal(drawn[clear], vis_o[clear])
    grad = {k: np.zeros(np.shape(x)) for k, x in p.items()}
    for i, c in enumerate(cams):
        d = drec[i * n:(i + 1) * n].astype(np.float64)
        g = oracle.project_bwd(p, scene.camera_dict(c),
                               dict(d_mean2d=d[:, 0:2].T, d_conic=d[:, 2:5].T, d_opacity=d[:, 5],
                                    d_rgb=d[:, 6:9].T))
        for k in grad:
            grad[k] += g[k]
    for k in p:
        rp, rm, rv = oracle.adam(p[k], grad[k], m[k], v[k], LRS[k], 6, B1, B2, EPS,
                                 visible=vis_o)
        P2, M2, V2 = (np.atleast_2d(a).astype(np.float64) for a in (gp[k], gm[k], gv[k]))
        rp, rm, rv = (np.atleast_2d(a) for a in (rp, rm, rv))
        p0 = np.atleast_2d(p[k]).astype(np.float64)
        hid = clear & ~vis_o
        np.testing.assert_array_equal(P2[:, hid], p0[:, hid], err_msg=k)
        sel = clear & vis_o
        # m follows the gradient tolerance of the parity tests (scaled by 1 - b1)
        gs = np.abs(np.atleast_2d(grad[k])).max()
        assert np.all(np.abs(M2[:, sel] - rm[:, sel])
                      <= (1 - B1) * (1e-3 * np.abs(np.atleast_2d(grad[k])[:, sel]) + 1e-5 * gs)
                      + 1e-6 * np.abs(rm[:, sel])), k
        step_ref = rp[:, sel] - p0[:, sel]
        step_got = P2[:, sel] - p0[:, sel]
        # the update is a bounded ratio times lr: compare within 1% of lr
        # (FP32 parameters resolve steps to their ulp)
        ulp = np.spacing(np.abs(p0[:, sel]).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(step_got - step_ref) <= 1e-2 * LRS[k] + 2 * ulp), k
