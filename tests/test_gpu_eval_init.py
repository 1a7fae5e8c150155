"""GPU parity of the evaluation metric, the plain initialisation and the
autograd path against the FP64 oracle:

* gs_masked_psnr: per-image masked PSNR (clamped image, peak 1) within
  1e-5 dB of oracle.masked_psnr, with +inf for an exact match and NaN for an
  empty mask;
* gs_knn's mean distance and gs_plain_init against the brute-force oracle
  k-NN (1e-5 relative);
* RenderFn + LossFn (torch.autograd) with an upstream gradient per image
  (gs_scale_rows): parameter gradients against the oracle's projection,
  compositing, loss and backward chain.
"""
import math

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


@pytest.mark.parametrize("S,H,W", [(3, 37, 53), (2, 1080, 1920)])
def test_masked_psnr_matches_oracle(ops, S, H, W):
    say("masked psnr", S, H, W)
    rng = np.random.default_rng(S * 1000 + H)
    tgt = rng.uniform(0, 1, (S, 3, H, W)).astype(np.float32)
    img = (tgt + rng.normal(0, 0.04, tgt.shape)).astype(np.float32)   # some values outside [0, 1]
    img[0, :, : H // 3] = tgt[0, :, : H // 3]
    mask = (rng.uniform(size=(S, H, W)) < 0.55).astype(np.uint8)
    mask[-1, :, : W // 4] = 0
    got = ops.masked_psnr(torch.as_tensor(img).cuda(), torch.as_tensor(tgt).cuda(),
                          torch.as_tensor(mask).cuda()).cpu().numpy()
    for s in range(S):
        ref = oracle.masked_psnr(img[s], tgt[s], mask[s])
        assert abs(float(got[s]) - ref) <= 1e-5 * max(1.0, abs(ref) / 10), (s, got[s], ref)
    # all pixels: the plain PSNR
    full = ops.masked_psnr(torch.as_tensor(img).cuda(), torch.as_tensor(tgt).cuda()).cpu().numpy()
    for s in range(S):
        ref = oracle.masked_psnr(img[s], tgt[s], None)
        assert abs(float(full[s]) - ref) <= 1e-5 * max(1.0, abs(ref) / 10)


def test_masked_psnr_special_cases(ops):
    say("masked psnr special cases")
    H, W = 40, 70
    rng = np.random.default_rng(2)
    tgt = rng.uniform(0, 1, (3, 3, H, W)).astype(np.float32)
    img = tgt.copy()
    img[1] += 0.25
    mask = np.ones((3, H, W), np.uint8)
    mask[2] = 0                                   # empty mask
    got = ops.masked_psnr(torch.as_tensor(img).cuda(), torch.as_tensor(tgt).cuda(),
                          torch.as_tensor(mask).cuda()).cpu().numpy()
    assert got[0] == math.inf                     # exact match
    ref1 = oracle.masked_psnr(img[1], tgt[1], mask[1])
    assert abs(float(got[1]) - ref1) <= 1e-5
    assert math.isnan(float(got[2]))
    from paper_2509_12138_amd.train import mean_over_views
    assert mean_over_views([20.0, float("nan"), 40.0]) == 30.0


def test_knn_mean_distance_and_plain_init_match_oracle(ops):
    say("knn mean + plain init")
    n = 5000
    pts, nrm = scene.sample_surface(scene.field_sphere_sines, n, 64, seed=12)
    P = np.ascontiguousarray(pts.T, np.float32)
    N = np.ascontiguousarray(nrm.T, np.float32)
    _, rdist = oracle.knn(P.astype(np.float64), 3)
    rmean = rdist.mean(axis=1)
    Pd, Nd = torch.as_tensor(P).cuda(), torch.as_tensor(N).cuda()
    mean = ops.knn_mean_distance(Pd, 3).cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(mean, rmean, rtol=1e-5)
    idx, dist, mean2 = ops.knn(Pd, 3, with_mean=True)
    np.testing.assert_array_equal(mean2.cpu().numpy(), mean.astype(np.float32))
    g = ops.plain_init(Pd, Nd, 0.1)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}
    np.testing.assert_array_equal(got["mean"], P.astype(np.float64))
    np.testing.assert_allclose(got["log_scale"], np.tile(np.log(rmean), (3, 1)), atol=2e-5)
    np.testing.assert_array_equal(got["quat"], np.array([[1.0], [0.0], [0.0], [0.0]]) * np.ones((4, n)))
    assert np.all(np.abs(got["opacity_logit"] - math.log(0.1 / 0.9)) <= 1e-6)
    # colour from the normal: C0 f + 1/2 = (n + 1) / 2
    np.testing.assert_allclose(oracle.C0 * got["color"] + 0.5, (N.astype(np.float64) + 1) / 2,
                               atol=1e-6)
    # mean and colour only (the learned initialisation's call)
    g2 = ops.plain_init(Pd, Nd, 0.1, shape=False)
    np.testing.assert_array_equal(g2["color"].cpu().numpy(), got["color"].astype(np.float32))


def test_autograd_render_and_loss_match_oracle(ops):
    """image = RenderFn(params); per-image loss = LossFn(image); the
    upstream gradient w of each image's loss reaches the parameters through
    gs_scale_rows, gs_raster_bwd and gs_project_bwd.  Pixels the oracle
    marks ambiguous (FP32 and FP64 decisions may differ) are masked out of
    the loss, so the comparison covers the rest exactly."""
    say("autograd render + loss")
    W, H = 96, 80
    n = 3000
    params = perturbed(surface_scene(n, 91), 91)
    cams = scene.orbit_cameras(3, W, H)
    cam = cams[1]
    camd = scene.camera_dict(cam)
    p = oracle.project(params, camd)
    r = oracle.render(p, W, H)
    rng = np.random.default_rng(5)
    target = rng.uniform(0, 1, (3, H, W)).astype(np.float32)
    mask = ((rng.uniform(size=(H, W)) < 0.8) & ~r["ambiguous"].astype(bool)).astype(np.uint8)
    w = 2.5
    lo = oracle.loss(r["image"], target, mask)
    g_ref = oracle.project_bwd(params, camd, oracle.render_bwd(p, W, H, w * lo["d_image"]))

    leaves = {k: v.clone().requires_grad_(True) for k, v in to_dev(params, torch).items()}
    bufs = ops.RasterBuffers(ops.Views.single(n, [cam]), W, H)
    img = ops.render(leaves, bufs)
    lb = ops.LossBuffers(1, H, W)
    L = ops.LossFn.apply(img, torch.as_tensor(target[None]).cuda(),
                         torch.as_tensor(mask[None]).cuda(), 0.2, lb)
    (w * L).sum().backward()
    torch.cuda.synchronize()
    assert abs(float(L[0]) - lo["loss"]) <= 1e-5 * abs(lo["loss"])
    for k, ref in g_ref.items():
        got = leaves[k].grad.cpu().numpy().astype(np.float64)
        nr = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-30)
        assert nr <= 1e-3, (k, nr)
