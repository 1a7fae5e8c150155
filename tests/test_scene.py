"""Input generators: surface samples lie on f = 0, cameras look at the origin."""
import numpy as np

from paper_2509_12138_amd import scene


def test_sphere_sines_samples_on_surface():
    pts, nrm = scene.sample_surface(scene.field_sphere_sines, 4096, 64, seed=1)
    assert pts.shape == (4096, 3)
    f, _ = scene.field_sphere_sines(pts)
    assert np.max(np.abs(f)) <= 1e-6
    np.testing.assert_allclose(np.linalg.norm(nrm, axis=1), 1.0, rtol=1e-12)
    # outward normals on a sphere-like surface
    assert np.mean(np.sum(nrm * pts, 1) > 0) > 0.99
    # seeded: same seed, same points
    pts2, _ = scene.sample_surface(scene.field_sphere_sines, 4096, 64, seed=1)
    np.testing.assert_array_equal(pts, pts2)


def test_box_restricted_sampling():
    box = (np.array([0.0, 0.0, 0.0]), np.array([1.0, 1.0, 1.0]))
    pts, _ = scene.sample_surface(scene.field_sphere_sines, 2000, 128, seed=3, box=box)
    assert np.all(pts >= 0) and len(pts) == 2000


def test_screened_candidate_cells_equal_the_full_sweep():
    """The Lipschitz block screen keeps exactly the cells the corner sweep
    finds (same cells, same order), whole grid and boxes with ragged blocks."""
    f = scene.field_sphere_sines
    sweep = lambda p: f(p)                         # no lipschitz attribute: full sweep
    assert not hasattr(sweep, "lipschitz") and f.lipschitz > 1
    for grid, box, block in ((64, None, 16), (200, ((-0.3, 0.1, -1.0), (0.9, 0.7, 0.2)), 16),
                             (150, ((0.0, 0.0, 0.0), (1.0, 1.0, 1.0)), 7)):
        a, h = scene.candidate_cells(f, grid, box=box, block=block)
        b, h2 = scene.candidate_cells(sweep, grid, box=box)
        assert h == h2 and len(a) > 1000
        np.testing.assert_array_equal(a, b)


def test_octant_box_has_two_voxel_ghosts():
    from paper_2509_12138_amd import workloads
    lo, hi = workloads.octant_box(2048, 2)
    np.testing.assert_allclose(lo, -2 * 2 / 2047)
    np.testing.assert_array_equal(hi, 1.0)
    pts, _ = scene.sample_surface(scene.field_sphere_sines, 3000, 256, seed=3,
                                  box=workloads.octant_box(256, 2))
    assert np.all(pts >= -2 * 2 / 255) and (pts < 0).any()


def test_mixing_interface_samples():
    mi = scene.MixingInterface(seed=2)
    assert abs(mi.A.sum() - 0.25) < 1e-12 and len(mi.A) == 32
    pts, nrm = mi.sample(20000, seed=4)
    assert pts.shape == (20000, 3)
    np.testing.assert_allclose(np.linalg.norm(nrm, axis=1), 1.0, rtol=1e-9)
    layer = np.abs(pts[:, 2] - mi.height(pts[:, :2])) < 1e-12
    assert layer.mean() > 0.5


def test_orbit_cameras_look_at_origin():
    cams = scene.orbit_cameras(16, 128, 96)
    for c in cams:
        R = c["R"].reshape(3, 3).astype(np.float64)
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-6)
        assert abs(np.linalg.det(R) - 1) < 1e-6
        o = R @ np.zeros(3) + c["t"]             # origin in camera space
        assert abs(o[0]) < 1e-5 and abs(o[1]) < 1e-5 and abs(o[2] - 2.5) < 1e-5
    assert abs(cams[0]["fx"] - 64 / np.tan(np.radians(25))) < 1e-3


def test_views_table():
    po, go = scene.views_table([5, 3], 2)
    np.testing.assert_array_equal(po, [0, 5, 10, 13, 16])
    np.testing.assert_array_equal(go, [0, 0, 5, 5])


def test_morton_order_is_a_permutation_that_keeps_neighbours_close():
    rng = np.random.default_rng(3)
    p = rng.uniform(-1, 1, (20000, 3))
    o = scene.morton_order(p)
    assert np.array_equal(np.sort(o), np.arange(len(p)))
    step = np.linalg.norm(np.diff(p[o], axis=0), axis=1)
    rand = np.linalg.norm(np.diff(p, axis=0), axis=1)
    assert np.median(step) < 0.1 * np.median(rand)
    # the 8 octant corners: each bit triple is (x, y, z), x the highest
    c = np.array([[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)], float)
    code = 4 * c[:, 0] + 2 * c[:, 1] + c[:, 2]
    assert np.array_equal(scene.morton_order(c), np.argsort(code, kind="stable"))
