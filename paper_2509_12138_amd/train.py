"""Plain per-partition trainer: one view per step through the library calls.

One step (the training step the paper's Sec. II "Parallel Training" runs on
each partition):
    gs_project -> gs_bin_sort -> gs_raster_fwd -> gs_loss -> gs_raster_bwd
    -> gs_project_bwd -> gs_adam (clears the gradients)
Everything stays on the device; the duplicate-capacity status is read back
only every ``check_every`` steps (the one host synchronisation).
"""
from __future__ import annotations

import ctypes as C
import math
import time

import numpy as np
import torch

from . import _lib
from . import ops

DEFAULT_LR = dict(mean=1.6e-4, log_scale=5e-3, quat=1e-3, opacity_logit=5e-2, color=2.5e-3)


def mean_lr(step, extent, lr0=1.6e-4, lr1=1.6e-6, total=30000):
    """Log-linear decay of the position learning rate, scaled by the scene extent."""
    t = min(max(step / float(total), 0.0), 1.0)
    return extent * math.exp(math.log(lr0) * (1 - t) + math.log(lr1) * t)


def masked_psnr(image, target, mask):
    """10 log10(1/MSE) over masked pixels of clamped images (evaluation only)."""
    m = mask.to(image.dtype).unsqueeze(-3)
    se = ((image.clamp(0, 1) - target) ** 2 * m).sum(dim=(-3, -2, -1))
    cnt = 3.0 * m.sum(dim=(-3, -2, -1)).clamp_min(1.0)
    return 10.0 * torch.log10(1.0 / (se / cnt).clamp_min(1e-20))


class PlainTrainer:
    """Trains one partition's Gaussians against per-view targets and masks."""

    def __init__(self, params, cams_np, targets, masks, tile=(16, 16), lam=0.2,
                 bg=(0.0, 0.0, 0.0), stored=True, extent=2.75, lrs=None, dup_capacity=None,
                 schedule="default", chunk=0, device="cuda"):
        self.device = device
        self.params = {k: torch.as_tensor(np.ascontiguousarray(v, np.float32)).to(device)
                       if not torch.is_tensor(v) else v.contiguous().to(device)
                       for k, v in params.items()}
        self.n = self.params["opacity_logit"].shape[-1]
        self.grads = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.m = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.v = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.V = len(cams_np)
        self.W, self.H = int(cams_np[0]["width"]), int(cams_np[0]["height"])
        self.cams = ops.Views.cams_to_device(cams_np, device)
        self.targets = targets
        self.masks = masks
        self.bg = tuple(bg)
        self.lam = lam
        self.extent = extent
        self.lrs = dict(DEFAULT_LR if lrs is None else lrs)
        self.views = ops.Views.single(self.n, cams_np[:1], device)
        self.views.use_cameras(self.cams[0:1])
        self.bufs = ops.RasterBuffers(self.views, self.W, self.H, tile, dup_capacity=dup_capacity,
                                      store_state=stored)
        self.bufs.set_schedule(schedule, chunk=chunk)
        self.loss = ops.LossBuffers(1, self.H, self.W, device)
        self.mode = _lib.GS_BWD_STORED if stored else _lib.GS_BWD_RECOMPUTE
        self.gst = ops.gaussians_struct(self.params)
        self.grst = ops.grads_struct(self.grads, self.n)
        self.groups = ops.adam_groups(self.params, self.grads, self.m, self.v, self.lrs)
        self.step_count = 0
        self.timing = None            # optional dict of lists of (start, end) events

    def fit_capacity(self, margin=1.5, views=None):
        """Size the duplicate buffers from the largest view's true count."""
        need = 0
        for vi in (range(self.V) if views is None else views):
            self.views.use_cameras(self.cams[vi:vi + 1])
            need = max(need, self.bufs.render_checked(self.gst, self.bg))
        self.bufs.ensure_capacity(int(need * margin) + 4096)
        return need

    def _ev(self, name):
        if self.timing is None:
            return None
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        self.timing.setdefault(name, []).append(e)
        return e

    def step(self, vi):
        """One training step on view vi (asynchronous; no host sync)."""
        b = self.bufs
        self.views.use_cameras(self.cams[vi:vi + 1])
        self._ev("project")
        b.project(self.gst)
        self._ev("bin_sort")
        b.bin_sort()
        self._ev("raster_fwd")
        b.order_tiles()
        b.raster_fwd(self.bg)
        self._ev("loss")
        self.loss(b.image, self.targets[vi:vi + 1], self.masks[vi:vi + 1] if self.masks is not None
                  else None, self.lam, 1.0, b.status)
        self._ev("zero")
        b.zero_d_rec()
        self._ev("raster_bwd")
        b.raster_bwd(self.loss.d_image, self.bg, self.mode)
        self._ev("project_bwd")
        b.project_bwd(self.gst, self.grst)
        self._ev("adam")
        self.step_count += 1
        self.groups[0].lr = mean_lr(self.step_count, self.extent, self.lrs["mean"])
        ops.adam_step(self.groups, self.step_count, zero_grad=True)
        self._ev("end")

    def check(self):
        """Synchronise and raise on duplicate overflow / non-finite loss."""
        st, req = self.bufs.check()
        if st != _lib.GS_OK:
            raise _lib.GSError("training step", st, _lib.last_error())
        return req

    def evaluate(self, views=None):
        """Mean masked PSNR over views (renders each; evaluation only)."""
        views = range(self.V) if views is None else views
        ps = []
        for vi in views:
            self.views.use_cameras(self.cams[vi:vi + 1])
            self.bufs.render_checked(self.gst, self.bg)
            ps.append(masked_psnr(self.bufs.image[0], self.targets[vi], self.masks[vi]))
        return float(torch.stack(ps).mean())

    def train(self, steps, order_seed=0, eval_every=0, target_psnr=None, check_every=50,
              log=None):
        """Run `steps` steps over a seeded view order.  Returns a history of
        (step, wall seconds excluding evaluation, psnr)."""
        rng = np.random.default_rng(order_seed)
        order = []
        hist = []
        train_time = 0.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            if not order:
                order = list(rng.permutation(self.V))
            self.step(order.pop())
            if check_every and (s + 1) % check_every == 0:
                self.check()
            if eval_every and (s + 1) % eval_every == 0:
                torch.cuda.synchronize()
                train_time += time.perf_counter() - t0
                p = self.evaluate()
                hist.append((s + 1, train_time, p))
                if log:
                    log(s + 1, train_time, p)
                if target_psnr is not None and p >= target_psnr:
                    return hist
                torch.cuda.synchronize()
                t0 = time.perf_counter()
        torch.cuda.synchronize()
        train_time += time.perf_counter() - t0
        self.check()
        hist.append((steps, train_time, None))
        return hist
