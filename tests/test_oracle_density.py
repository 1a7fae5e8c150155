"""Pins of the oracle's adaptive density control (3D-GS clone / split /
prune / opacity reset) against hand-worked cases, closed forms and the
covariance of the Gaussian a split samples from."""
import math

import numpy as np
import pytest

import oracle


def _gauss(n, rng):
    return dict(mean=rng.normal(size=(3, n)), log_scale=rng.normal(-3, 0.3, (3, n)),
                quat=rng.normal(size=(4, n)), opacity_logit=rng.normal(size=n),
                color=rng.normal(size=(3, n)))


def test_stats_add_the_ndc_gradient_norm_of_visible_pairs():
    W, H, n = 200, 100, 3
    d = np.zeros((2 * n, 9), np.float32)
    d[0, :2] = (3.0 / 100, 4.0 / 50)        # norm 5 in NDC units
    d[1, :2] = (1.0, 1.0)                     # invisible in slot 0
    d[n + 0, :2] = (0.0, 2.0 / 50)            # slot 1: norm 2
    d[n + 2, :2] = (-6.0 / 100, 8.0 / 50)     # norm 10
    nt = np.array([1, 0, 2, 3, 0, 1])
    a, c = oracle.densify_stats(d, nt, n, W, H, np.zeros(n, np.float32), np.zeros(n, np.float32))
    np.testing.assert_allclose(a, [7.0, 0.0, 10.0], rtol=1e-6)
    np.testing.assert_array_equal(c, [2.0, 0.0, 2.0])
    a2, c2 = oracle.densify_stats(d, nt, n, W, H, a, c)     # accumulates
    np.testing.assert_allclose(a2, 2 * a, rtol=1e-6)
    np.testing.assert_array_equal(c2, 2 * c)


def test_select_truth_table():
    # columns: faint | grow small | grow large | big | normal | split too big | no stats
    ls = np.array([[-5.0, -5.0, -1.0, 0.5, -4.0, 0.3, -4.0]] * 3)
    logit = np.array([-6.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0])
    acc = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 1.0, 0.0], np.float32)
    den = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 0.0], np.float32)
    act, n_out = oracle.densify_select(ls, logit, acc, den, grad_threshold=0.5,
                                       max_log_scale_clone=-2.0, min_opacity_logit=-5.0,
                                       max_log_scale=0.0, log_split=math.log(1.6))
    # the split of column 5 leaves children at 0.3 - 0.47 < 0: kept as a split
    assert act.tolist() == [0, 2, 3, 0, 1, 3, 1]
    assert n_out == 0 + 2 + 2 + 0 + 1 + 2 + 1
    act2, _ = oracle.densify_select(ls, logit, acc, den, 0.5, -2.0, -5.0, -0.2, math.log(1.6))
    assert act2[5] == oracle.ACT_DROP          # children still above -0.2


def test_clone_and_keep_copy_parameters_and_moments():
    rng = np.random.default_rng(1)
    n = 4
    p = _gauss(n, rng)
    m = {k: rng.normal(size=np.shape(v)) for k, v in p.items()}
    v = {k: rng.uniform(size=np.shape(x)) for k, x in p.items()}
    act = np.array([oracle.ACT_KEEP, oracle.ACT_DROP, oracle.ACT_CLONE, oracle.ACT_KEEP])
    P, M, V = oracle.densify_apply(p, m, v, act, np.zeros((n, 2, 3)), math.log(1.6))
    idx = [0, 2, 2, 3]
    for k in p:
        np.testing.assert_array_equal(np.atleast_2d(P[k]), np.atleast_2d(p[k])[:, idx])
    np.testing.assert_array_equal(M["mean"][:, [0, 1, 3]], m["mean"][:, [0, 2, 3]])
    assert np.all(M["mean"][:, 2] == 0) and np.all(V["quat"][:, 2] == 0)


def test_split_children_follow_the_rotated_axes():
    """Unit-vector draws land on the Gaussian's principal axes: z = e_k gives
    mean + s_k * (column k of R), here for a 90 degree turn about z."""
    h = math.sqrt(0.5)
    p = dict(mean=np.array([[1.0], [2.0], [3.0]]), log_scale=np.log([[0.2], [0.5], [0.1]]),
             quat=np.array([[h], [0.0], [0.0], [h]]), opacity_logit=np.array([0.3]),
             color=np.array([[0.1], [0.2], [0.3]]))
    zero = {k: np.zeros(np.shape(v)) for k, v in p.items()}
    z = np.array([[[1.0, 0.0, 0.0], [0.0, -1.0, 0.0]]])
    P, M, _ = oracle.densify_apply(p, zero, zero, np.array([oracle.ACT_SPLIT]), z, math.log(1.6))
    # R rotates x -> y and y -> -x
    np.testing.assert_allclose(P["mean"][:, 0], [1.0, 2.2, 3.0], atol=1e-12)
    np.testing.assert_allclose(P["mean"][:, 1], [1.5, 2.0, 3.0], atol=1e-12)
    np.testing.assert_allclose(P["log_scale"], np.log([[0.2, 0.2], [0.5, 0.5], [0.1, 0.1]]) - math.log(1.6))
    np.testing.assert_array_equal(P["opacity_logit"], [0.3, 0.3])
    assert np.all(M["mean"] == 0)


def test_split_offsets_have_the_gaussian_covariance():
    rng = np.random.default_rng(2)
    p = _gauss(1, rng)
    p["log_scale"] = np.log([[0.3], [0.1], [0.05]])
    zero = {k: np.zeros(np.shape(v)) for k, v in p.items()}
    N = 20000
    offs = []
    for _ in range(N // 2):
        z = rng.normal(size=(1, 2, 3))
        P, _, _ = oracle.densify_apply(p, zero, zero, np.array([oracle.ACT_SPLIT]), z, 0.0)
        offs.append(P["mean"] - p["mean"])
    offs = np.concatenate(offs, axis=1)
    R = oracle._rot_wxyz(p["quat"])[:, :, 0]
    cov = R @ np.diag(np.exp(2 * p["log_scale"][:, 0])) @ R.T
    emp = offs @ offs.T / offs.shape[1]
    assert np.abs(emp - cov).max() <= 0.04 * np.abs(cov).max()


def test_opacity_reset_clamps_only_large_logits():
    r = oracle.opacity_reset(np.array([-6.0, -4.59, 0.0, 3.0]), math.log(0.01 / 0.99))
    np.testing.assert_allclose(r, [-6.0, -4.59511985, -4.59511985, -4.59511985], rtol=1e-7)
