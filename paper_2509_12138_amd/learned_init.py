"""Learned initialisation of the Gaussians of one partition.

The paper places one Gaussian at every isosurface point (Sec. II,
"Isosurface Extraction") and starts it from the 3D-GS default: isotropic
scale from the 3 nearest neighbours, identity rotation, opacity 0.1.  This
module adds a 96 -> 64 -> 64 -> 8 network (bf16 MFMA kernels of libgsmi)
that predicts the starting log-scale, rotation and opacity from the point's
16 nearest neighbours, trained on Gaussians the training step has fitted.

Inference:  gs_knn(16) -> gs_mlp_features -> gs_mlp_fwd -> gs_mlp_apply
Training:   gs_mlp_targets, then gs_mlp_fwd -> gs_mlp_loss -> gs_mlp_bwd ->
            gs_adam per step.
Fallback:   the plain k-NN initialisation when an output is not finite or
            when the network's held-out loss is not below the plain
            initialisation's loss against the same targets.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _lib, ops
from ._lib import call
from .ops import _ptr, stream_handle

MLP_SHAPES = dict(w1=(96, 64), w2=(64, 64), w3=(64, 8), b1=(64,), b2=(64,), b3=(8,))
MLP_NAMES = ("w1", "w2", "w3", "b1", "b2", "b3")
SQRT_PI = math.sqrt(math.pi)
PLAIN_OPACITY = 0.1


def _f32(t, name):
    ops._check_f32(t, name)
    return t


class InitMLP:
    """FP32 master weights on the device plus the libgsmi calls that use them."""

    def __init__(self, weights):
        self.w = {k: _f32(weights[k].contiguous(), k) for k in MLP_NAMES}
        for k in MLP_NAMES:
            if tuple(self.w[k].shape) != MLP_SHAPES[k]:
                raise ValueError(f"{k} has shape {tuple(self.w[k].shape)}, want {MLP_SHAPES[k]}")
        self._ws = None

    @classmethod
    def random(cls, seed=505, device="cuda", out_bias=None):
        """He-normal hidden layers, a small output layer, zero hidden biases."""
        rng = np.random.default_rng(seed)
        w = dict(w1=rng.normal(0, math.sqrt(2 / 96), (96, 64)),
                 w2=rng.normal(0, math.sqrt(2 / 64), (64, 64)),
                 w3=rng.normal(0, 0.1 * math.sqrt(1 / 64), (64, 8)),
                 b1=np.zeros(64), b2=np.zeros(64),
                 b3=np.zeros(8) if out_bias is None else np.asarray(out_bias, np.float64))
        return cls({k: torch.as_tensor(v.astype(np.float32)).to(device) for k, v in w.items()})

    def struct(self):
        return _lib.gs_mlp(*[self.w[k].data_ptr() for k in MLP_NAMES])

    def state(self):
        return {k: v.detach().cpu().numpy().copy() for k, v in self.w.items()}

    def forward(self, x, y=None):
        n = x.shape[0]
        y = torch.empty((n, 8), dtype=torch.float32, device=x.device) if y is None else y
        st = self.struct()
        call("gs_mlp_fwd", _ptr(x), n, ctypes.byref(st), _ptr(y), stream_handle())
        return y

    def backward(self, x, dy, grads, dx=None):
        """Adds parameter gradients into grads (dict like the weights)."""
        n = x.shape[0]
        nbytes = _lib.load().gs_mlp_bwd_workspace_bytes(n)
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
        g = _lib.gs_mlp_grads(*[grads[k].data_ptr() for k in MLP_NAMES],
                              dx.data_ptr() if dx is not None else 0)
        st = self.struct()
        call("gs_mlp_bwd", _ptr(x), n, ctypes.byref(st), _ptr(dy), ctypes.byref(g), _ptr(self._ws), nbytes,
             stream_handle())


def features(points, normals, k=16):
    """Device features x [n,96] (bf16 bits in an int16 tensor) and the mean
    16-NN distance dbar [n] of device points / normals [3,n]."""
    _f32(points, "points"); _f32(normals, "normals")
    n = points.shape[1]
    idx, dist = ops.knn(points, k)
    return features_from_knn(points, normals, idx, dist)


def features_from_knn(points, normals, idx, dist):
    n = points.shape[1]
    if idx.shape != (n, 16) or dist.shape != (n, 16):
        raise ValueError("features need 16 neighbours per point")
    x = torch.empty((n, 96), dtype=torch.int16, device=points.device)
    dbar = torch.empty(n, dtype=torch.float32, device=points.device)
    call("gs_mlp_features", _ptr(points), _ptr(normals), n, _ptr(idx.contiguous()),
         _ptr(dist.contiguous()), _ptr(x), _ptr(dbar), stream_handle())
    return x, dbar


def targets(log_scale, quat, opacity_logit, normals, dbar):
    n = dbar.shape[0]
    t = torch.empty((n, 8), dtype=torch.float32, device=dbar.device)
    for name, a in (("log_scale", log_scale), ("quat", quat), ("opacity_logit", opacity_logit)):
        _f32(a, name)
    call("gs_mlp_targets", _ptr(log_scale), _ptr(quat), _ptr(opacity_logit), _ptr(normals),
         _ptr(dbar), n, _ptr(t), stream_handle())
    return t


class LossBuf:
    def __init__(self, n, device):
        self.n = n
        nbytes = _lib.load().gs_mlp_loss_workspace_bytes(n)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.nbytes = nbytes
        self.dy = torch.empty((n, 8), dtype=torch.float32, device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)


def loss(y, t, buf=None):
    """(loss [1] device, dy [n,8] device) of outputs y against targets t."""
    n = y.shape[0]
    buf = LossBuf(n, y.device) if buf is None or buf.n != n else buf
    call("gs_mlp_loss", _ptr(y), _ptr(t), n, _ptr(buf.dy), _ptr(buf.ws), buf.nbytes,
         _ptr(buf.loss), stream_handle())
    return buf.loss, buf.dy


def apply(y, normals, dbar):
    n = y.shape[0]
    dev = y.device
    out = dict(log_scale=torch.empty((3, n), dtype=torch.float32, device=dev),
               quat=torch.empty((4, n), dtype=torch.float32, device=dev),
               opacity_logit=torch.empty(n, dtype=torch.float32, device=dev))
    call("gs_mlp_apply", _ptr(y), _ptr(normals), _ptr(dbar), n, _ptr(out["log_scale"]),
         _ptr(out["quat"]), _ptr(out["opacity_logit"]), stream_handle())
    return out


def plain_init(points, normals, opacity=PLAIN_OPACITY):
    """The plain k-NN initialisation on the device: isotropic scale = mean
    distance to the 3 nearest neighbours, identity rotation, fixed opacity,
    colour from the normal."""
    return ops.plain_init(points.contiguous(), normals.contiguous(), opacity)


def learned_params(mlp, points, normals, x=None, dbar=None):
    """Gaussians initialised by the network; None if an output is not finite."""
    if x is None:
        x, dbar = features(points, normals)
    y = mlp.forward(x)
    if not bool(torch.isfinite(y).all()):
        return None
    g = apply(y, normals, dbar)
    mc = ops.plain_init(points.contiguous(), normals.contiguous(), PLAIN_OPACITY, shape=False)
    g.update(mean=mc["mean"], color=mc["color"])
    return {k: g[k].contiguous() for k in ops.PARAM_NAMES}


class MLPTrainer:
    """Adam on the network over (features, targets) held on the device, in
    mini-batches of contiguous rows of a once-shuffled copy."""

    def __init__(self, mlp: InitMLP, x, t, lr=1e-3, batch=65536, seed=0):
        self.mlp = mlp
        n = x.shape[0]
        g = torch.Generator(device="cpu").manual_seed(seed)
        perm = torch.randperm(n, generator=g).to(x.device)
        self.x = x[perm].contiguous()
        self.t = t[perm].contiguous()
        self.n = n
        self.batch = min(batch, n)
        self.grads = {k: torch.zeros_like(v) for k, v in mlp.w.items()}
        self.m = {k: torch.zeros_like(v) for k, v in mlp.w.items()}
        self.v = {k: torch.zeros_like(v) for k, v in mlp.w.items()}
        self.lr = lr
        self.groups = (_lib.gs_adam_group * len(MLP_NAMES))()
        for i, k in enumerate(MLP_NAMES):
            self.groups[i] = _lib.gs_adam_group(mlp.w[k].data_ptr(), self.grads[k].data_ptr(),
                                                self.m[k].data_ptr(), self.v[k].data_ptr(),
                                                mlp.w[k].numel(), float(lr))
        self.y = torch.empty((self.batch, 8), dtype=torch.float32, device=x.device)
        self.lbuf = LossBuf(self.batch, x.device)
        self.steps = 0
        self.cursor = 0

    def step(self):
        b = self.batch
        if self.cursor + b > self.n:
            self.cursor = 0
        xs = self.x[self.cursor:self.cursor + b]
        ts = self.t[self.cursor:self.cursor + b]
        self.cursor += b
        self.mlp.forward(xs, self.y)
        L, dy = loss(self.y, ts, self.lbuf)
        self.mlp.backward(xs, dy, self.grads)
        self.steps += 1
        call("gs_adam", self.groups, len(MLP_NAMES), 0.9, 0.999, 1e-8, self.steps, 1,
             stream_handle())
        return L

    def train(self, steps, log_every=0, log=None):
        hist = []
        for s in range(steps):
            L = self.step()
            if log_every and (s % log_every == 0 or s == steps - 1):
                hist.append((s, float(L.item())))
                if log:
                    log(f"mlp step {s}: loss {hist[-1][1]:.5f}")
        return hist


def evaluate_loss(mlp, x, t):
    y = mlp.forward(x)
    L, _ = loss(y, t)
    return float(L.item())


def plain_outputs_loss(points, normals, dbar, t):
    """Loss of the plain initialisation expressed in network-output space."""
    p = plain_init(points, normals)
    yp = targets(p["log_scale"], p["quat"], p["opacity_logit"], normals, dbar)
    L, _ = loss(yp, t)
    return float(L.item())


def choose_init(mlp, points, normals, held_x=None, held_dbar=None, held_t=None,
                held_points=None, held_normals=None):
    """Learned Gaussians unless the fallback rule picks the plain ones.

    Returns (params, "learned" | "plain")."""
    if held_x is not None:
        l_mlp = evaluate_loss(mlp, held_x, held_t)
        l_plain = plain_outputs_loss(held_points, held_normals, held_dbar, held_t)
        if not (math.isfinite(l_mlp) and l_mlp < l_plain):
            return plain_init(points, normals), "plain"
    p = learned_params(mlp, points, normals)
    if p is None:
        return plain_init(points, normals), "plain"
    return p, "learned"


def mlp_bench(n=4_000_000, reps=10, seed=0):
    """Time the network's forward and backward kernels on n seeded bf16
    feature rows (the size of the learned partition): mean ms per call of
    gs_mlp_fwd and gs_mlp_bwd (no dx), HIP events on the launch stream."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    x = (torch.randn((n, 96), generator=g, device="cuda") * 0.5).to(torch.bfloat16)
    x = x.view(torch.int16).contiguous()
    mlp = InitMLP.random(seed=seed)
    dy = torch.randn((n, 8), generator=g, device="cuda") * 1e-3
    grads = {k: torch.zeros_like(v) for k, v in mlp.w.items()}
    y = mlp.forward(x)
    mlp.backward(x, dy, grads)
    torch.cuda.synchronize()
    out = {}
    for name, fn in (("fwd", lambda: mlp.forward(x, y)), ("bwd", lambda: mlp.backward(x, dy, grads))):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name + "_ms"] = e0.elapsed_time(e1) / reps
    out["n"] = n
    return out


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser(description="time the initialisation network's kernels")
    ap.add_argument("--n", type=int, default=4_000_000)
    ap.add_argument("--reps", type=int, default=10)
    a = ap.parse_args()
    print(json.dumps(mlp_bench(a.n, a.reps)), flush=True)
