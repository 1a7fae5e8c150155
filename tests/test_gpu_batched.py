"""Batched uneven partitions in one launch, graph replay and the device-side
Adam schedule."""
import numpy as np
import pytest

import oracle
from paper_2509_12138_amd import scene
from _gpu_helpers import perturbed, say, surface_scene, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

W, H = 96, 72


@pytest.fixture(scope="module")
def parts(gpu):
    """Three uneven slabs of the bumpy sphere (x-slabs with 0.02 ghost
    overlap), each with its own targets/masks rendered by the oracle."""
    pts, nrm = scene.sample_surface(scene.field_sphere_sines, 9000, 64, seed=5)
    edges = [-1.0, -0.1, 0.25, 1.0]
    cams = scene.orbit_cameras(8, W, H)
    out = []
    for i in range(3):
        sel = (pts[:, 0] >= edges[i] - 0.02) & (pts[:, 0] <= edges[i + 1] + 0.02)
        d = scene.knn_mean_distance(pts[sel], 3)
        prm = scene.gaussians_from_points(pts[sel], nrm[sel], d, opacity=0.3)
        ref = scene.gaussians_from_points(pts[sel], nrm[sel], d, opacity=0.9, thin=0.2)
        tg, mk = [], []
        for cam in cams:
            r = oracle.render(oracle.project(ref, scene.camera_dict(cam)), W, H)
            tg.append(r["image"]); mk.append(r["T_final"] <= 0.5)
        out.append(dict(params=prm, targets=torch.as_tensor(np.stack(tg).astype(np.float32)).cuda(),
                        masks=torch.as_tensor(np.stack(mk).astype(np.uint8)).cuda()))
    assert len({p["params"]["opacity_logit"].shape[0] for p in out}) == 3     # uneven
    return out, cams


def test_batched_images_equal_single_renders(parts):
    say("batched images")
    from paper_2509_12138_amd import ops
    from paper_2509_12138_amd.train import BatchedTrainer
    prts, cams = parts
    bt = BatchedTrainer(prts, cams, views_per_part=2, graphs=False)
    bt.views.use_cameras(bt.cams_g[1])
    bt.bufs.render_checked(bt.gst)
    torch.cuda.synchronize()
    got = bt.bufs.image.cpu().numpy()
    for p in range(3):
        prm = bt.partition_params(p)
        single = ops.RasterBuffers(ops.Views.single(bt.counts[p], cams[bt.group_views[1]]), W, H)
        single.render_checked(ops.gaussians_struct({k: v.contiguous() for k, v in prm.items()}))
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got[2 * p:2 * p + 2], single.image.cpu().numpy())


def test_graph_replay_matches_eager(parts):
    say("graph replay")
    from paper_2509_12138_amd.train import BatchedTrainer
    prts, cams = parts
    runs = {}
    # (graphs, deterministic): the atomic step eager and replayed, and the
    # eager step with fixed-order gradient sums as the measure of the atomic
    # sums' summation-order noise
    for graphs, det in ((False, False), (True, False), ("det", True)):
        bt = BatchedTrainer(prts, cams, views_per_part=2, graphs=graphs is True, order_seed=3,
                            deterministic=det)
        bt.fit_capacity()
        losses, m1 = [], None
        for s in range(10):
            g = s % bt.G
            bt.step(g)
            torch.cuda.synchronize()
            losses.append(bt.loss.loss.cpu().numpy().copy())
            if s == 0:
                m1 = {k: v.cpu().numpy().copy() for k, v in bt.m.items()}
            # eager work between replays
            _ = (bt.params["mean"] * 2).sum().item()
        bt.check()
        runs[graphs] = (np.array(losses), m1, int(bt.adam.step_dev.item()))
    le, lg = runs[False][0], runs[True][0]
    np.testing.assert_allclose(lg, le, rtol=2e-4, atol=1e-7)
    assert runs[True][2] == runs[False][2] == 10
    # first Adam moments after step 1 (0.1 x the gradient): the atomic sums'
    # order differs from run to run, so the replay may differ from the eager
    # run by that noise, which the eager run's distance from the fixed-order
    # run measures (it dominates in the rotation gradients, sums of terms
    # that nearly cancel); a wrong replay would differ at the gradients' own
    # scale
    for k in runs[False][1]:
        a, b, d = runs[False][1][k], runs[True][1][k], runs["det"][1][k]
        noise = np.linalg.norm(a - d)
        assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(a) + 1e-12 + 2.0 * noise, k
        assert noise <= np.linalg.norm(a) + 1e-12, k


def test_device_adam_schedule_matches_oracle(gpu):
    say("device adam")
    from paper_2509_12138_amd import ops
    rng = np.random.default_rng(1)
    p0 = rng.normal(size=(3, 500)).astype(np.float32)
    p = torch.as_tensor(p0).cuda(); g = torch.zeros_like(p)
    m = torch.zeros_like(p); v = torch.zeros_like(p)
    groups = ops.adam_groups(dict(mean=p, log_scale=p[:0], quat=p[:0], opacity_logit=p[0, :0],
                                  color=p[:0]),
                             dict(mean=g, log_scale=g[:0], quat=g[:0], opacity_logit=g[0, :0],
                                  color=g[:0]),
                             dict(mean=m, log_scale=m[:0], quat=m[:0], opacity_logit=m[0, :0],
                                  color=m[:0]),
                             dict(mean=v, log_scale=v[:0], quat=v[:0], opacity_logit=v[0, :0],
                                  color=v[:0]),
                             dict(mean=1e-2, log_scale=1, quat=1, opacity_logit=1, color=1))
    adam = ops.DeviceAdam(groups, lr_final=[1e-4, 0, 0, 0, 0], decay_steps=7)
    ref = (p0.astype(np.float64), np.zeros(p0.shape), np.zeros(p0.shape))
    for t in range(1, 11):
        gr = rng.normal(size=p0.shape).astype(np.float32)
        g.copy_(torch.as_tensor(gr))
        adam()
        lr = 1e-2 * (1e-4 / 1e-2) ** min(t / 7, 1.0)
        ref = oracle.adam(ref[0], gr, ref[1], ref[2], lr, t)
        torch.cuda.synchronize()
        np.testing.assert_allclose(p.cpu().numpy(), ref[0], rtol=2e-6, atol=2e-6)
    assert int(adam.step_dev.item()) == 10


def test_prepare_captures_without_training(parts):
    """prepare() captures every group's step and leaves the state as it was;
    the replayed training then matches an eager run."""
    say("prepare + replay")
    from paper_2509_12138_amd.train import BatchedTrainer
    prts, cams = parts
    bt = BatchedTrainer(prts, cams, views_per_part=2, graphs=True, order_seed=3)
    bt.fit_capacity()
    before = {k: v.cpu().numpy().copy() for k, v in bt.params.items()}
    bt.prepare()
    assert len(bt.graphs) == bt.G
    assert int(bt.adam.step_dev.item()) == 0
    for k, v in bt.params.items():
        np.testing.assert_array_equal(v.cpu().numpy(), before[k])
    ref = BatchedTrainer(prts, cams, views_per_part=2, graphs=False, order_seed=3)
    ref.fit_capacity()
    for s in range(6):
        bt.step(s % bt.G)
        ref.step(s % ref.G)
        torch.cuda.synchronize()
        np.testing.assert_allclose(bt.loss.loss.cpu().numpy(), ref.loss.loss.cpu().numpy(),
                                   rtol=2e-4, atol=1e-7)


def test_graph_replay_with_rising_colour_degree(parts):
    """View-dependent colour in the batched trainer: the active degree rises
    (0 -> 1 -> 2) during training, the captured graphs are re-captured with
    the new degree, and the replayed steps match eager ones."""
    say("graph replay, rising sh degree")
    from paper_2509_12138_amd.train import BatchedTrainer
    prts, cams = parts
    runs = {}
    for graphs in (False, True):
        bt = BatchedTrainer(prts, cams, views_per_part=2, graphs=graphs, order_seed=3,
                            sh_degree=2, sh_up_every=3)
        bt.fit_capacity()
        assert bt.params["color"].shape[0] == 27 and len(bt.groups) == 6
        losses, degrees = [], []
        for s in range(9):
            bt.step(s % bt.G)
            torch.cuda.synchronize()
            losses.append(bt.loss.loss.cpu().numpy().copy())
            degrees.append(bt.active_sh)
            _ = (bt.params["mean"] * 2).sum().item()
        bt.check()
        col = bt.params["color"].cpu().numpy()
        runs[graphs] = (np.array(losses), degrees, col)
        for k, v in bt.params.items():
            assert torch.isfinite(v).all(), k
    assert runs[True][1] == runs[False][1] == [0, 0, 0, 1, 1, 1, 2, 2, 2]
    np.testing.assert_allclose(runs[True][0], runs[False][0], rtol=2e-4, atol=1e-7)
    # bands 1 and 2 moved once active
    col = runs[True][2]
    assert np.abs(col[3:12]).max() > 0 and np.abs(col[12:27]).max() > 0


def test_batched_density_control_keeps_partitions_apart(parts):
    """Density control in the graph-captured batched trainer: the
    densifications change every partition's count, the graphs are
    re-captured on the new arrays, and afterwards each partition's slots of
    a batched render still equal that partition rendered alone (so the
    per-partition ranges followed the new Gaussians)."""
    say("batched density control")
    from paper_2509_12138_amd import ops
    from paper_2509_12138_amd.train import BatchedTrainer, DensityControl
    prts, cams = parts
    dc = DensityControl(start=2, until=12, interval=3, grad_threshold=1e-5, reset_interval=1000,
                        seed=2)
    bt = BatchedTrainer(prts, cams, views_per_part=2, graphs=True, order_seed=4, density=dc)
    bt.fit_capacity()
    counts0 = list(bt.counts)
    for s in range(14):
        bt.step(s % bt.G)
        _ = (bt.params["mean"] * 2).sum().item()
    bt.check()
    assert bt.counts != counts0 and sum(bt.counts) == bt.n
    for k, v in bt.params.items():
        assert torch.isfinite(v).all() and v.shape[-1] == bt.n, k
    assert bt.views.struct.total_pairs == bt.n * bt.vpp
    bt.views.use_cameras(bt.cams_g[1])
    bt.bufs.render_checked(bt.gst)
    torch.cuda.synchronize()
    got = bt.bufs.image.cpu().numpy()
    for p in range(3):
        prm = bt.partition_params(p)
        single = ops.RasterBuffers(ops.Views.single(bt.counts[p], cams[bt.group_views[1]]), W, H)
        single.render_checked(ops.gaussians_struct({k: v.contiguous() for k, v in prm.items()}))
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got[2 * p:2 * p + 2], single.image.cpu().numpy())


def _unambiguous_masks(prts, cams, views):
    """Copies of the partitions made anisotropic, rotated and varied (so that
    no gradient vanishes identically, as the rotation's does for isotropic
    Gaussians) whose masks also cut every pixel where FP32 and FP64
    decisions may differ for the partition's own Gaussians in the given
    views (render ambiguity, or an L1 sign within the image tolerance),
    with the oracle's projections and renders of those views.  The GPU
    projects the Gaussians itself, so the decision bands are those of its
    projection's tolerance (BAND_E2E), not of FP32 rounding alone."""
    from _gpu_helpers import BAND_E2E, decision_safe_mask
    out, orc = [], []
    for i, part in enumerate(prts):
        prm = perturbed(part["params"], 40 + i)
        masks = part["masks"].clone()
        per = {}
        for vi in views:
            cam = scene.camera_dict(cams[vi])
            pr = oracle.project(prm, cam)
            r = oracle.render(pr, W, H, band=BAND_E2E)
            keep = decision_safe_mask(masks[vi].cpu().numpy(), r,
                                      part["targets"][vi].cpu().numpy())
            masks[vi] = torch.as_tensor(keep.astype(np.uint8)).cuda()
            per[vi] = (cam, pr, r)
        out.append(dict(part, params=prm, masks=masks))
        orc.append(per)
    return out, orc


def _batched_step_vs_oracle(parts, lam, per_pair):
    from paper_2509_12138_amd.train import BatchedTrainer
    from _gpu_helpers import BAND_E2E, grad_tolerance_check
    prts, cams = parts
    vpp = 4
    bt0 = BatchedTrainer(prts, cams, views_per_part=vpp, graphs=False, order_seed=11)
    views = [int(v) for v in bt0.group_views[0]]
    mod, orc = _unambiguous_masks(prts, cams, views)
    bt = BatchedTrainer(mod, cams, views_per_part=vpp, graphs=False, order_seed=11, lam=lam)
    assert [int(v) for v in bt.group_views[0]] == views
    bt.fit_capacity()
    bt.step(0)
    bt.check()
    torch.cuda.synchronize()
    assert int(bt.views.gauss_offset[vpp].item()) == bt.counts[0] > 0
    img = bt.bufs.image.cpu().numpy()
    drec = bt.bufs.d_rec.cpu().numpy().astype(np.float64)
    po = bt.views.pair_offset_host
    b1 = np.float32(bt.adam.betas[0])           # 0.9^4 with the batch-size rule
    inv = np.float32(1.0) / (np.float32(1.0) - b1)
    gpu_g = {k: (v.cpu().numpy() * inv).astype(np.float64) for k, v in bt.m.items()}
    off = 0
    for p, part in enumerate(mod):
        n = bt.counts[p]
        g_ref = {k: np.zeros_like(np.asarray(v, np.float64)) for k, v in part["params"].items()}
        for j, vi in enumerate(views):
            s = p * vpp + j
            cam, pr, r = orc[p][vi]
            ok = ~r["ambiguous"].astype(bool)
            err = np.abs(img[s] - r["image"])[:, ok]
            assert err.max() <= 1e-4, (p, j, err.max())
            lo = oracle.loss(r["image"], part["targets"][vi].cpu().numpy(),
                             part["masks"][vi].cpu().numpy(), lam=lam)
            rb = oracle.render_bwd(pr, W, H, lo["d_image"] / vpp, band=BAND_E2E)
            if per_pair:
                ref = np.concatenate([rb["d_mean2d"], rb["d_conic"], rb["d_opacity"][None],
                                      rb["d_rgb"]]).T
                okg, worst = grad_tolerance_check(drec[po[s]:po[s + 1]], ref,
                                                  rb["term_mass"].T, rb["amb_mass"].T)
                assert okg, f"slot {p},{j}: {worst}"
            gp = oracle.project_bwd(part["params"], cam, rb)
            for k in g_ref:
                g_ref[k] += gp[k]
        for k, ref in g_ref.items():
            got = gpu_g[k][..., off:off + n]
            scale = np.abs(ref).max()
            assert np.all(np.abs(got - ref) <= 1e-3 * np.abs(ref) + 1e-4 * scale), (p, k)
            nr = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-30)
            assert nr <= 1e-3, (p, k, nr)
        off += n


def test_batched_step_matches_oracle(parts):
    """One batched step of three uneven partitions stored back to back
    (slots with gauss_offset != 0), four views each, in one launch per stage,
    with the L1 loss alone: every slot's image, every pair's record gradient
    (per element, term-mass bound) and every partition's parameter gradient
    (the mean over its four views, read back from Adam's first moment
    m = (1 - beta1) g after the first step, beta1 = 0.9^4) against the oracle run partition
    by partition and view by view.  With the L1 sign decided the same way on
    both sides the image gradient is identical, so every difference comes
    from the launch itself."""
    say("batched step vs oracle (L1)")
    _batched_step_vs_oracle(parts, lam=0.0, per_pair=True)


def test_batched_step_with_dssim_matches_oracle(parts):
    """The same step with the configured 0.8 L1 + 0.2 D-SSIM loss: images and
    per-partition parameter gradients against the oracle (per element
    1e-3 |r| + 1e-4 max |r|, normwise 1e-3).  The D-SSIM gradient moves by
    about 40x the image's own FP32 error relative to its largest value, so a
    pair whose gradient cancels across pixels of both signs is compared at
    the parameter level only; the loss's own parity is tested by itself."""
    say("batched step vs oracle (L1 + D-SSIM)")
    _batched_step_vs_oracle(parts, lam=0.2, per_pair=False)


def test_captured_step_replays_bit_identically_to_eager(parts):
    """The batched step captured through the C ABI (gs_graph_begin /
    gs_graph_end, replayed by gs_graph_launch) with deterministic gradient
    sums: ten steps over alternating view groups, with the program's own
    eager work and synchronisations between replays, give bit-identical
    losses, parameters and Adam moments to the same steps run eagerly."""
    say("graph replay bit-identical")
    from paper_2509_12138_amd.train import BatchedTrainer
    prts, cams = parts
    runs = {}
    for graphs in (False, True):
        bt = BatchedTrainer(prts, cams, views_per_part=2, graphs=graphs, order_seed=3,
                            deterministic=True)
        bt.fit_capacity()
        if graphs:
            bt.prepare()
            assert len(bt.graphs) == bt.G
        losses = []
        for s in range(10):
            bt.step(s % bt.G)
            torch.cuda.synchronize()
            losses.append(bt.loss.loss.cpu().numpy().copy())
            _ = (bt.params["mean"] * 2).sum().item()          # eager work between replays
        bt.check()
        runs[graphs] = (np.array(losses), {k: v.cpu().numpy() for k, v in bt.params.items()},
                        {k: v.cpu().numpy() for k, v in bt.m.items()},
                        int(bt.adam.step_dev.item()))
    assert runs[True][3] == runs[False][3] == 10
    np.testing.assert_array_equal(runs[True][0], runs[False][0])
    for k in runs[False][1]:
        np.testing.assert_array_equal(runs[True][1][k], runs[False][1][k])
        np.testing.assert_array_equal(runs[True][2][k], runs[False][2][k])


def test_graph_handles_through_the_c_abi(gpu):
    """gs_graph_* directly: capture two library fills on a created stream,
    replay the graph three times with eager writes in between (each replay
    restores the captured effect), and refuse capture on the null stream."""
    import ctypes as C
    lib = gpu.load()
    say("graph handles")
    buf = torch.full((1 << 16,), 7.0, device="cuda")
    s = torch.cuda.Stream()
    h = C.c_void_p(s.cuda_stream)
    torch.cuda.synchronize()
    assert lib.gs_graph_begin(h) == 0, lib.gs_last_error()
    assert lib.gs_zero(C.c_void_p(buf.data_ptr()), 4 * 4096, h) == 0
    assert lib.gs_zero(C.c_void_p(buf.data_ptr() + 4 * 8192), 4 * 4096, h) == 0
    g = C.c_void_p()
    assert lib.gs_graph_end(h, C.byref(g)) == 0, lib.gs_last_error()
    torch.cuda.synchronize()
    assert float(buf[0]) == 7.0                # capturing ran nothing
    for r in range(3):
        buf.fill_(float(r + 1))
        assert lib.gs_graph_launch(g, C.c_void_p(torch.cuda.current_stream().cuda_stream)) == 0
        torch.cuda.synchronize()
        host = buf.cpu().numpy()
        assert np.all(host[:4096] == 0) and np.all(host[8192:12288] == 0)
        assert np.all(host[4096:8192] == r + 1) and np.all(host[12288:] == r + 1)
    lib.gs_graph_destroy(g)
    assert lib.gs_graph_begin(None) == -1
