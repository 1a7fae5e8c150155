"""GPU parity of the learned-initialisation calls against the FP64 oracle
with bf16 emulation (features, forward, backward incl. dx, targets, loss,
apply), a short GPU training run of the network, and what the trained
network gains over the plain k-NN initialisation on a tiny scene.

Tolerances: network outputs and gradients normwise relative <= 1e-3 (the
oracle rounds to bf16 exactly where the kernels do; what remains is FP32
accumulation order and rare bf16 rounding flips of hidden values that FP32
and FP64 place on opposite sides of a rounding boundary); features within one
bf16 step (2^-7 relative, where FP32 and FP64 round to neighbouring bf16
values) plus 1e-6; geometry (targets / apply)
1e-5 absolute."""
import math

import numpy as np
import pytest

import oracle
from paper_2509_12138_amd import scene
from _gpu_helpers import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NAMES = ("w1", "w2", "w3", "b1", "b2", "b3")
ORACLE_NAMES = dict(w1="W1", w2="W2", w3="W3", b1="b1", b2="b2", b3="b3")


@pytest.fixture(scope="module")
def li(gpu):
    from paper_2509_12138_amd import learned_init
    return learned_init


def weights(seed):
    rng = np.random.default_rng(seed)
    return dict(w1=rng.normal(0, math.sqrt(2 / 96), (96, 64)), w2=rng.normal(0, math.sqrt(2 / 64), (64, 64)),
                w3=rng.normal(0, 0.2, (64, 8)), b1=rng.normal(0, 0.1, 64), b2=rng.normal(0, 0.1, 64),
                b3=rng.normal(0, 0.1, 8))


def dev32(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float32)).cuda()


def bf16_bits(a):
    """bf16 bit patterns (int16) of the oracle's bf16 rounding of a."""
    r = oracle.bf16_round(a).astype(np.float32)
    return (r.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def oracle_net(w):
    return [w[k].astype(np.float32).astype(np.float64) for k in ("w1", "b1", "w2", "b2", "w3", "b3")]


def normwise(g, r):
    return float(np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-30))


@pytest.mark.parametrize("n", [1, 17, 1000, 50000])
def test_mlp_fwd_matches_oracle(li, n):
    say(f"mlp fwd n={n}")
    rng = np.random.default_rng(100 + n)
    w = weights(505)
    xq = oracle.bf16_round(rng.normal(size=(n, 96)))
    mlp = li.InitMLP({k: dev32(v) for k, v in w.items()})
    y = mlp.forward(torch.as_tensor(bf16_bits(xq)).cuda()).cpu().numpy()
    ref, _ = oracle.mlp_forward(xq, *oracle_net(w), quantize=True)
    assert normwise(y, ref) <= 1e-3, normwise(y, ref)
    assert np.abs(y - ref).max() <= 1e-2 * np.abs(ref).max()


@pytest.mark.parametrize("n,with_dx", [(17, True), (1000, True), (70000, False)])
def test_mlp_bwd_matches_oracle(li, n, with_dx):
    say(f"mlp bwd n={n} dx={with_dx}")
    rng = np.random.default_rng(200 + n)
    w = weights(506)
    xq = oracle.bf16_round(rng.normal(size=(n, 96)))
    dy = rng.normal(size=(n, 8)) / n
    mlp = li.InitMLP({k: dev32(v) for k, v in w.items()})
    grads = {k: torch.zeros_like(v) for k, v in mlp.w.items()}
    dx = torch.empty((n, 96), dtype=torch.float32, device="cuda") if with_dx else None
    x_dev = torch.as_tensor(bf16_bits(xq)).cuda()
    mlp.backward(x_dev, dev32(dy), grads, dx)
    _, cache = oracle.mlp_forward(xq, *oracle_net(w), quantize=True)
    ref = oracle.mlp_backward(cache, dy, quantize=True)
    for k in NAMES:
        g = grads[k].cpu().numpy()
        e = normwise(g, ref[ORACLE_NAMES[k]])
        say(f"  {k}: normwise {e:.2e}")
        assert e <= 1e-3, (k, e)
    if with_dx:
        e = normwise(dx.cpu().numpy(), ref["x"])
        assert e <= 1e-3, ("dx", e)
    # a second call adds the same values again (fixed reduction order)
    first = {k: v.clone() for k, v in grads.items()}
    mlp.backward(x_dev, dev32(dy), grads, None)
    for k in NAMES:
        assert torch.equal(grads[k], 2 * first[k]), k


def _surface(n, seed):
    pts, nrm = scene.sample_surface(scene.field_sphere_sines, n, 64, seed=seed)
    return pts.T.copy(), nrm.T.copy()


def _frame_ambiguous(nrm, rel=1e-5):
    a = np.sort(np.abs(nrm / np.linalg.norm(nrm, axis=0)), axis=0)
    return (a[1] - a[0]) <= rel * np.maximum(a[1], 1e-30)


def test_mlp_features_match_oracle(li):
    say("mlp features")
    pts, nrm = _surface(3000, 31)
    idx, dist = oracle.knn(pts, 16)
    x, dbar = li.features_from_knn(dev32(pts), dev32(nrm), torch.as_tensor(idx).cuda(),
                                   dev32(dist))
    xb = x.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    xg = xb.view(np.float32).astype(np.float64)
    xr, dr = oracle.mlp_features(pts.astype(np.float32), nrm.astype(np.float32), idx,
                                 dist.astype(np.float32), quantize=True)
    np.testing.assert_allclose(dbar.cpu().numpy(), dr, rtol=2e-6)
    ok = ~_frame_ambiguous(nrm.astype(np.float32))
    assert ok.mean() > 0.99
    d = np.abs(xg - xr)[ok]
    assert np.all(d <= 2.0 ** -7 * np.abs(xr[ok]) + 1e-6), float(d.max())
    assert np.mean(d > 1e-6) < 0.01            # flips of one bf16 step are rare
    # the GPU k-NN route gives the same features where its neighbour lists
    # equal the oracle's
    x2, _ = li.features(dev32(pts), dev32(nrm))
    from paper_2509_12138_amd import ops
    gi, _ = ops.knn(dev32(pts), 16)
    same = np.all(gi.cpu().numpy() == idx, axis=1) & ok
    assert same.mean() > 0.95
    x2g = (x2.cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32)
    d2 = np.abs(x2g.astype(np.float64) - xr)[same]
    assert np.all(d2 <= 2.0 ** -7 * np.abs(xr[same]) + 1e-6), float(d2.max())


def _up_to_sign(a, b):
    return np.minimum(np.abs(a - b).max(axis=1), np.abs(a + b).max(axis=1))


def test_mlp_targets_and_apply_match_oracle(li):
    say("mlp targets/apply")
    rng = np.random.default_rng(41)
    n = 2000
    nrm = rng.normal(size=(3, n)).astype(np.float32)
    dbar = rng.uniform(0.005, 0.05, n).astype(np.float32)
    ls = rng.normal(-4, 0.5, (3, n)).astype(np.float32)
    q = rng.normal(size=(4, n)).astype(np.float32)
    lo = rng.normal(0, 2, n).astype(np.float32)
    t = li.targets(dev32(ls), dev32(q), dev32(lo), dev32(nrm), dev32(dbar)).cpu().numpy()
    tr = oracle.mlp_targets(ls, q, lo, nrm, dbar.astype(np.float64))
    ok = ~_frame_ambiguous(nrm)
    np.testing.assert_allclose(t[:, [0, 1, 2, 7]], tr[:, [0, 1, 2, 7]], atol=1e-5)
    assert _up_to_sign(t[ok, 3:7], tr[ok, 3:7]).max() <= 1e-5
    y = rng.normal(size=(n, 8)).astype(np.float32)
    g = li.apply(dev32(y), dev32(nrm), dev32(dbar))
    gr = oracle.mlp_apply(y, nrm, dbar.astype(np.float64))
    np.testing.assert_allclose(g["log_scale"].cpu().numpy(), gr["log_scale"], atol=1e-5)
    np.testing.assert_array_equal(g["opacity_logit"].cpu().numpy(), y[:, 7])
    assert _up_to_sign(g["quat"].cpu().numpy().T[ok], gr["quat"].T[ok]).max() <= 1e-5


@pytest.mark.parametrize("n", [1, 5000])
def test_mlp_loss_matches_oracle(li, n):
    say(f"mlp loss n={n}")
    rng = np.random.default_rng(50 + n)
    t = rng.normal(size=(n, 8))
    t[:, 3:7] /= np.linalg.norm(t[:, 3:7], axis=1, keepdims=True)
    y = (t + rng.normal(0, 0.4, t.shape)).astype(np.float32)
    t = t.astype(np.float32)
    L, dy = li.loss(dev32(y), dev32(t))
    Lr, dr = oracle.mlp_loss(y, t)
    assert abs(float(L.item()) - Lr) <= 1e-5 * abs(Lr) + 1e-7
    np.testing.assert_allclose(dy.cpu().numpy(), dr, atol=1e-6 * np.abs(dr).max(), rtol=1e-4)


def test_mlp_training_fits_a_teacher(li):
    """Adam through the library's kernels fits a random teacher network's
    outputs (computed by the oracle) to a small fraction of the start loss."""
    say("mlp training")
    rng = np.random.default_rng(60)
    n = 16384
    xq = oracle.bf16_round(rng.normal(size=(n, 96)))
    teacher = weights(61)
    t, _ = oracle.mlp_forward(xq, *oracle_net(teacher), quantize=False)
    t[:, 3:7] /= np.linalg.norm(t[:, 3:7], axis=1, keepdims=True)
    mlp = li.InitMLP.random(seed=505)
    tr = li.MLPTrainer(mlp, torch.as_tensor(bf16_bits(xq)).cuda(), dev32(t), lr=2e-3, batch=4096)
    hist = tr.train(600, log_every=100, log=say)
    assert hist[-1][1] < 0.2 * hist[0][1], hist
    assert all(np.isfinite(v.cpu().numpy()).all() for v in mlp.w.values())


def test_learned_init_beats_plain_init(li):
    """Fit a tiny partition with the plain trainer, train the network on the
    fitted Gaussians, then initialise a different partition of the same
    field both ways: the learned start renders closer to the targets."""
    say("learned init vs plain")
    from paper_2509_12138_amd import workloads
    from paper_2509_12138_amd.train import PlainTrainer

    def prepare(seed):
        wl = workloads.tiny_partition(dict(seed=seed))
        tg, mk = workloads.render_targets_gpu(wl["reference"], wl["cams"])
        return wl, tg, mk

    wa, tga, mka = prepare(1)
    fit = PlainTrainer(wa["params"], wa["cams"], tga, mka)
    fit.fit_capacity()
    fit.train(400, order_seed=1001)
    pts_a, nrm_a = dev32(wa["points"].T), dev32(wa["normals"].T)
    xa, dba = li.features(pts_a, nrm_a)
    p = fit.params
    ta = li.targets(p["log_scale"], p["quat"], p["opacity_logit"], nrm_a, dba)
    mean_t = ta.mean(0).cpu().numpy()
    mlp = li.InitMLP.random(seed=505, out_bias=mean_t)
    tr = li.MLPTrainer(mlp, xa, ta, lr=2e-3, batch=4096)
    hist = tr.train(800, log_every=200, log=say)
    assert hist[-1][1] < hist[0][1]
    l_plain = li.plain_outputs_loss(pts_a, nrm_a, dba, ta)
    say(f"network loss {hist[-1][1]:.4f} vs plain init {l_plain:.4f} on the fitted set")
    assert hist[-1][1] < l_plain

    wb, tgb, mkb = prepare(2)
    pts_b, nrm_b = dev32(wb["points"].T), dev32(wb["normals"].T)
    learned, kind = li.choose_init(mlp, pts_b, nrm_b)
    assert kind == "learned"
    plain = li.plain_init(pts_b, nrm_b)
    ps = {}
    for name, params in (("plain", plain), ("learned", learned)):
        t = PlainTrainer(params, wb["cams"], tgb, mkb)
        t.fit_capacity()
        ps[name] = [t.evaluate()]
        t.train(50, order_seed=1002)
        ps[name].append(t.evaluate())
    say(f"masked PSNR start/after 50 steps: plain {ps['plain']}, learned {ps['learned']}")
    assert ps["learned"][0] > ps["plain"][0] + 1.0
    assert ps["learned"][1] > ps["plain"][1]
