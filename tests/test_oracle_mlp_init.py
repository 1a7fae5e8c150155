"""Pins of the oracle's learned-initialisation functions: local frames,
neighbour features, targets / apply, the network loss and the bf16-emulated
backward.  Each check comes from a closed form, an invariant or a finite
difference, not from the functions themselves."""
import math

import numpy as np
import pytest

import oracle


def _quat_to_rot(q):
    """Standard rotation matrix of a unit quaternion (w, x, y, z)."""
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _random_rotation(rng):
    q = rng.normal(size=4)
    return _quat_to_rot(q / np.linalg.norm(q))


def test_local_frame_closed_forms():
    # n = +z: least aligned axis is x (tie x/y -> lowest index); x-axis =
    # z cross x = +y, y-axis = z cross (+y) = -x
    F = oracle.local_frames(np.array([[0.0], [0.0], [1.0]]))[0]
    np.testing.assert_allclose(F, [[0, 1, 0], [-1, 0, 0], [0, 0, 1]], atol=1e-15)
    # n = +x: least aligned is y (tie y/z); x-axis = x cross y = +z,
    # y-axis = x cross z = -y
    F = oracle.local_frames(np.array([[2.0], [0.0], [0.0]]))[0]
    np.testing.assert_allclose(F, [[0, 0, 1], [0, -1, 0], [1, 0, 0]], atol=1e-15)


def test_local_frames_orthonormal_right_handed():
    rng = np.random.default_rng(11)
    n = rng.normal(size=(3, 500))
    F = oracle.local_frames(n)
    eye = np.einsum("nij,nkj->nik", F, F)
    np.testing.assert_allclose(eye, np.broadcast_to(np.eye(3), eye.shape), atol=1e-12)
    np.testing.assert_allclose(np.linalg.det(F), 1.0, atol=1e-12)
    np.testing.assert_allclose(F[:, 2, :], (n / np.linalg.norm(n, axis=0)).T, atol=1e-12)


def test_features_of_a_rotated_plane():
    """Points on a plane with the plane's normal: every local offset and
    neighbour normal lies in / along the local z axis, offset lengths are the
    distances over their mean."""
    rng = np.random.default_rng(12)
    Q = _random_rotation(rng)
    flat = np.column_stack([rng.uniform(-1, 1, (300, 2)), np.zeros(300)])
    pts = (Q @ flat.T)
    nrm = np.repeat((Q @ np.array([0.0, 0.0, 1.0]))[:, None], 300, axis=1)
    idx, dist = oracle.knn(pts, 16)
    x, dbar = oracle.mlp_features(pts, nrm, idx, dist, quantize=False)
    f = x.reshape(300, 16, 6)
    np.testing.assert_allclose(f[:, :, 2], 0.0, atol=1e-12)               # local z of offsets
    np.testing.assert_allclose(f[:, :, 3:5], 0.0, atol=1e-12)             # normals along z
    np.testing.assert_allclose(f[:, :, 5], 1.0, atol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(f[:, :, 0:3], axis=2), dist / dbar[:, None],
                               rtol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(f[:, :, 0:3], axis=2).mean(1), 1.0, rtol=1e-12)
    np.testing.assert_allclose(dbar, dist.mean(1), rtol=1e-15)


def test_features_missing_neighbours_and_quantisation():
    rng = np.random.default_rng(13)
    pts = rng.normal(size=(3, 5))
    nrm = rng.normal(size=(3, 5))
    idx, dist = oracle.knn(pts, 16)               # only 4 neighbours exist
    assert np.all(idx[:, 4:] == -1) and np.all(np.isinf(dist[:, 4:]))
    x, dbar = oracle.mlp_features(pts, nrm, idx, dist)
    np.testing.assert_array_equal(x[:, 24:], 0.0)
    np.testing.assert_allclose(dbar, dist[:, :4].mean(1), rtol=1e-15)
    np.testing.assert_array_equal(oracle.bf16_round(x), x)
    # single point: no neighbours, dbar = 1, all zero
    x1, d1 = oracle.mlp_features(pts[:, :1], nrm[:, :1], -np.ones((1, 16), np.int32),
                                 np.full((1, 16), np.inf))
    assert d1[0] == 1.0 and np.all(x1 == 0)


def _fitted(rng, n):
    return dict(log_scale=rng.normal(-4, 0.5, (3, n)), quat=rng.normal(size=(4, n)),
                opacity_logit=rng.normal(0, 2, n))


def test_apply_of_zero_offsets_is_the_frame():
    """y = (0, 0, 0, identity, w): log-scale = log dbar and the Gaussian's
    local z axis (third column of its rotation) is the surface normal."""
    rng = np.random.default_rng(14)
    n = 200
    nrm = rng.normal(size=(3, n))
    dbar = rng.uniform(0.01, 0.1, n)
    y = np.zeros((n, 8)); y[:, 3] = 1.0; y[:, 7] = rng.normal(size=n)
    g = oracle.mlp_apply(y, nrm, dbar)
    np.testing.assert_allclose(g["log_scale"], np.tile(np.log(dbar), (3, 1)), rtol=1e-15)
    np.testing.assert_array_equal(g["opacity_logit"], y[:, 7])
    unit = nrm / np.linalg.norm(nrm, axis=0)
    for i in range(n):
        R = _quat_to_rot(g["quat"][:, i])
        np.testing.assert_allclose(R[:, 2], unit[:, i], atol=1e-12)
    assert np.all(g["quat"][0] >= 0)


def test_targets_then_apply_round_trip():
    rng = np.random.default_rng(15)
    n = 300
    fit = _fitted(rng, n)
    nrm = rng.normal(size=(3, n))
    dbar = rng.uniform(0.01, 0.1, n)
    t = oracle.mlp_targets(fit["log_scale"], fit["quat"], fit["opacity_logit"], nrm, dbar)
    np.testing.assert_allclose(np.linalg.norm(t[:, 3:7], axis=1), 1.0, atol=1e-12)
    g = oracle.mlp_apply(t, nrm, dbar)
    np.testing.assert_allclose(g["log_scale"], fit["log_scale"], atol=1e-12)
    np.testing.assert_array_equal(g["opacity_logit"], fit["opacity_logit"])
    for i in range(n):
        np.testing.assert_allclose(_quat_to_rot(g["quat"][:, i]), _quat_to_rot(fit["quat"][:, i]),
                                   atol=1e-12)


def test_target_of_a_frame_aligned_gaussian_is_identity():
    rng = np.random.default_rng(16)
    n = 50
    nrm = rng.normal(size=(3, n))
    F = oracle.local_frames(nrm)
    # quaternion of F^T built from the closed-form rotation matrix via trace formula
    qs = []
    for i in range(n):
        R = F[i].T
        w = math.sqrt(max(0.0, 1 + np.trace(R))) / 2
        if w > 1e-3:
            qs.append([w, (R[2, 1] - R[1, 2]) / (4 * w), (R[0, 2] - R[2, 0]) / (4 * w),
                       (R[1, 0] - R[0, 1]) / (4 * w)])
        else:
            qs.append(None)
    keep = [i for i, q in enumerate(qs) if q is not None]
    quat = np.array([qs[i] for i in keep]).T
    t = oracle.mlp_targets(np.zeros((3, len(keep))), quat, np.zeros(len(keep)),
                           nrm[:, keep], np.ones(len(keep)))
    np.testing.assert_allclose(t[:, 3:7], np.tile([1.0, 0, 0, 0], (len(keep), 1)), atol=1e-12)


def test_mlp_loss_values_and_gradient():
    rng = np.random.default_rng(17)
    n = 40
    t = np.zeros((n, 8))
    t[:, [0, 1, 2, 7]] = rng.normal(size=(n, 4))
    q = rng.normal(size=(n, 4)); t[:, 3:7] = q / np.linalg.norm(q, axis=1, keepdims=True)
    # zero at the target, and blind to the sign and length of the quaternion
    y = t.copy(); y[:, 3:7] *= -2.5
    L, d = oracle.mlp_loss(y, t)
    assert abs(L) < 1e-15
    # closed form for a pure log-scale / opacity offset: mean of squared offsets
    y2 = t.copy(); y2[:, 0] += 0.5; y2[:, 7] -= 0.25
    assert abs(oracle.mlp_loss(y2, t)[0] - (0.25 + 0.0625)) < 1e-14
    # finite differences at a generic point
    y3 = t + rng.normal(0, 0.3, t.shape)
    L3, d3 = oracle.mlp_loss(y3, t)
    for i, j in [(0, 0), (3, 2), (5, 3), (7, 4), (11, 5), (13, 6), (17, 7), (19, 1)]:
        h = 1e-6
        yp = y3.copy(); yp[i, j] += h
        ym = y3.copy(); ym[i, j] -= h
        fd = (oracle.mlp_loss(yp, t)[0] - oracle.mlp_loss(ym, t)[0]) / (2 * h)
        assert abs(fd - d3[i, j]) <= 1e-7 * max(1.0, abs(fd)), (i, j, fd, d3[i, j])


def _dyadic_net(rng):
    """Weights in {-1, 0, 1} with at most two non-zeros per output column and
    half-integer biases: every forward / backward value is a small dyadic
    rational, exact in bf16."""
    def sparse(rows, cols):
        W = np.zeros((rows, cols))
        for c in range(cols):
            r = rng.choice(rows, size=2, replace=False)
            W[r, c] = rng.choice([-1.0, 1.0], size=2)
        return W
    return (sparse(96, 64), rng.choice([0.0, 0.5], 64), sparse(64, 64), rng.choice([0.0, 0.5], 64),
            sparse(64, 8), rng.choice([0.0, 0.5], 8))


def test_quantised_backward_equals_exact_on_bf16_exact_values():
    rng = np.random.default_rng(18)
    P = _dyadic_net(rng)
    x = rng.choice([-1.0, 0.0, 1.0], size=(50, 96))
    dy = rng.choice([-1.0, 0.0, 1.0], size=(50, 8))
    yq, cq = oracle.mlp_forward(x, *P, quantize=True)
    ye, ce = oracle.mlp_forward(x, *P, quantize=False)
    np.testing.assert_array_equal(yq, ye)
    gq = oracle.mlp_backward(cq, dy, quantize=True)
    ge = oracle.mlp_backward(ce, dy, quantize=False)
    for k in ge:
        np.testing.assert_array_equal(gq[k], ge[k])
    assert np.abs(ge["W1"]).max() > 0


def test_quantised_backward_close_to_exact():
    """Generic inputs: bf16 rounding of dy, dZ2, dZ1 moves the gradients by
    no more than a few bf16 half-ulps normwise (2^-9 each)."""
    rng = np.random.default_rng(19)
    W1 = rng.normal(0, math.sqrt(2 / 96), (96, 64)); W2 = rng.normal(0, math.sqrt(2 / 64), (64, 64))
    W3 = rng.normal(0, 0.1, (64, 8))
    b1 = rng.normal(0, 0.1, 64); b2 = rng.normal(0, 0.1, 64); b3 = rng.normal(0, 0.1, 8)
    x = oracle.bf16_round(rng.normal(size=(400, 96)))
    dy = rng.normal(size=(400, 8))
    _, cq = oracle.mlp_forward(x, W1, b1, W2, b2, W3, b3, quantize=True)
    gq = oracle.mlp_backward(cq, dy, quantize=True)
    ge = oracle.mlp_backward(cq, dy, quantize=False)
    for k in ("W1", "W2", "W3", "b1", "b2", "b3"):
        rel = np.linalg.norm(gq[k] - ge[k]) / np.linalg.norm(ge[k])
        assert 0 < rel < 3 * 2.0 ** -9, (k, rel)
