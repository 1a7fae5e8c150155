"""Global reconstruction helpers (Sec. II "Global Reconstruction"): merging,
the position colour code and the seam band.  CPU tests use torch CPU
tensors; the GPU test renders a plane of discs through the library."""
import numpy as np
import pytest
import torch

from paper_2509_12138_amd import reconstruct, scene, ttt

C0 = 0.28209479177387814


def test_merge_concatenates_partitions_in_order():
    a = {"mean": torch.arange(6.0).reshape(3, 2), "opacity_logit": torch.tensor([1.0, 2.0])}
    b = {"mean": torch.arange(6.0, 15.0).reshape(3, 3), "opacity_logit": torch.tensor([3.0, 4.0, 5.0])}
    m = reconstruct.merge([a, b])
    assert m["mean"].shape == (3, 5)
    assert torch.equal(m["mean"][:, :2], a["mean"]) and torch.equal(m["mean"][:, 2:], b["mean"])
    assert torch.equal(m["opacity_logit"], torch.tensor([1.0, 2.0, 3.0, 4.0, 5.0]))


def test_position_colour_renders_as_normalised_x():
    E = ttt.SURFACE_EXTENT
    x = np.array([-E, -0.3, 0.0, 0.25, E, 2 * E])
    pts = np.stack([x, np.zeros_like(x), np.zeros_like(x)], 1)
    f = reconstruct.position_colour(pts)
    assert f.shape == (3, len(x))
    grey = C0 * f.astype(np.float64) + 0.5               # the projection's colour rule
    np.testing.assert_allclose(grey[0], np.clip((x + E) / (2 * E), 0, 1), atol=1e-6)
    np.testing.assert_array_equal(f[0], f[2])


def test_seam_band_marks_pixels_near_faces_only():
    faces = ttt.slab_faces(8)
    assert len(faces) == 7 and np.allclose(np.diff(faces), 2 * ttt.SURFACE_EXTENT / 8)
    xmap = torch.tensor([[faces[0] + 0.005, faces[0] + 0.02, faces[3] - 0.01, 0.5]])
    cover = torch.tensor([[True, True, True, False]])
    band = reconstruct.seam_band(xmap, cover, faces, 0.01)
    assert band.tolist() == [[True, False, True, False]]


def test_slab_ghost_margin_widens_the_sampled_box():
    with_g = ttt.slab_part(-0.1, 0.1, 400, seed=3, ref_factor=1.0, grid=64, ghost_voxels=2)
    no_g = ttt.slab_part(-0.1, 0.1, 400, seed=3, ref_factor=1.0, grid=64, ghost_voxels=0)
    g = 2 * 2.0 / 64
    assert with_g["points"][:, 0].min() >= -0.1 - g - 1e-12
    assert with_g["points"][:, 0].max() <= 0.1 + g + 1e-12
    assert no_g["points"][:, 0].min() >= -0.1 - 1e-12 and no_g["points"][:, 0].max() <= 0.1 + 1e-12
    assert (np.abs(with_g["points"][:, 0]) > 0.1).any()


@pytest.mark.gpu
def test_position_render_recovers_the_x_of_a_plane():
    """Discs on the plane x = 0.1 facing +x, rendered with the position
    colour from a camera on the +x axis: every covered pixel reads x = 0.1."""
    rng = np.random.default_rng(4)
    n = 4000
    pts = np.stack([np.full(n, 0.1), rng.uniform(-0.3, 0.3, n), rng.uniform(-0.3, 0.3, n)], 1)
    nrm = np.tile([1.0, 0.0, 0.0], (n, 1))
    discs = scene.gaussians_from_points(pts, nrm, np.full(n, 0.02), opacity=0.9, thin=0.1)
    discs["color"] = reconstruct.position_colour(pts)
    R, t = scene.look_at(np.array([2.5, 0.0, 0.0]))
    cam = scene.single_camera(R, t, 300.0, 160, 120)
    E = ttt.SURFACE_EXTENT
    for _, img, T in reconstruct.render_views(discs, cam, (0.0, 0.0, 0.0)):
        cover = 1.0 - T
        xmap = img[0] / cover.clamp_min(1e-6) * (2 * E) - E
        sel = cover > 0.5
        assert float(sel.float().mean()) > 0.2
        assert float((xmap[sel] - 0.1).abs().max()) < 1e-4
