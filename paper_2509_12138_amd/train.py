"""Plain per-partition trainer: one view per step through the library calls.

One step (the training step the paper's Sec. II "Parallel Training" runs on
each partition):
    gs_project -> gs_bin_sort -> gs_raster_fwd -> gs_loss -> gs_raster_bwd
    -> gs_project_bwd -> gs_adam (clears the gradients)
Everything stays on the device; the duplicate-capacity status is read back
only every ``check_every`` steps (the one host synchronisation).  With a
DensityControl, the 3D-GS adaptive density control runs between steps
(statistics every step, clone / split / prune every ``interval`` steps,
opacity reset every ``reset_interval`` steps).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
import time

import numpy as np
import torch

from . import _lib
from . import ops

# color_rest: the colour rows above degree 0 (spherical-harmonic bands 1-3)
DEFAULT_LR = dict(mean=1.6e-4, log_scale=5e-3, quat=1e-3, opacity_logit=5e-2, color=2.5e-3,
                  color_rest=2.5e-3 / 20)


@dataclasses.dataclass
class DensityControl:
    """Adaptive density control schedule and thresholds (the 3D-GS defaults):
    statistics from `start` until `until`, densification every `interval`
    steps after `start`, opacity reset every `reset_interval` steps; clone
    when the largest scale is at most percent_dense x extent, else split
    into two children with scales / split_divisor; prune opacity below
    min_opacity and, after the first opacity reset, scales above
    max_world_scale x extent."""
    start: int = 500
    until: int = 15000
    interval: int = 100
    grad_threshold: float = 2e-4
    percent_dense: float = 0.01
    reset_interval: int = 3000
    min_opacity: float = 0.005
    max_world_scale: float = 0.1
    split_divisor: float = 1.6
    seed: int = 0


def mean_lr(step, extent, lr0=1.6e-4, lr1=1.6e-6, total=30000):
    """Log-linear decay of the position learning rate, scaled by the scene extent."""
    t = min(max(step / float(total), 0.0), 1.0)
    return extent * math.exp(math.log(lr0) * (1 - t) + math.log(lr1) * t)


def mean_over_views(psnr):
    """Mean of per-view masked PSNRs (host array); views with an empty mask
    (NaN) are left out."""
    v = np.asarray(psnr, np.float64)
    v = v[~np.isnan(v)]
    return float(v.mean()) if v.size else float("nan")


class PlainTrainer:
    """Trains one partition's Gaussians against per-view targets and masks."""

    def __init__(self, params, cams_np, targets, masks, tile=(16, 16), lam=0.2,
                 bg=(0.0, 0.0, 0.0), stored=True, extent=2.75, lrs=None, dup_capacity=None,
                 schedule="default", chunk=0, fwd_waves=1, deterministic=False, fused_adam=True,
                 density=None, sh_degree=0, sh_up_every=1000, sparse_adam=False,
                 device="cuda"):
        self.device = device
        if sparse_adam and not fused_adam:
            raise ValueError("sparse_adam needs fused_adam (the fused call makes the step)")
        self.sparse_adam = bool(sparse_adam)
        self.V = len(cams_np)
        self.W, self.H = int(cams_np[0]["width"]), int(cams_np[0]["height"])
        self.cams_np = cams_np
        self.cams = ops.Views.cams_to_device(cams_np, device)
        self.targets = targets
        self.masks = masks
        self.bg = tuple(bg)
        self.lam = lam
        self.extent = extent
        self.lrs = dict(DEFAULT_LR if lrs is None else lrs)
        self.tile, self.stored = tuple(tile), stored
        self.plan = dict(mode=schedule, chunk=chunk, fwd_waves=fwd_waves,
                         deterministic=deterministic)
        self.loss = ops.LossBuffers(1, self.H, self.W, device)
        self.mode = _lib.GS_BWD_STORED if stored else _lib.GS_BWD_RECOMPUTE
        # fused projection backward + Adam: the step count and the position
        # lr decay live on the device
        self.fused_adam = fused_adam
        self.density = density
        self.dev_adam = None
        self.densifier = None
        p = {k: torch.as_tensor(np.ascontiguousarray(v, np.float32)).to(device)
             if not torch.is_tensor(v) else v.contiguous().to(device) for k, v in params.items()}
        # view-dependent colour: coefficients up to sh_degree (the higher
        # ones start at zero); the active degree starts at 0 and rises by
        # one every sh_up_every steps (the 3D-GS schedule), or is sh_degree
        # from the start when sh_up_every <= 0
        self.sh_degree, self.sh_up_every = int(sh_degree), int(sh_up_every)
        rows = 3 * (self.sh_degree + 1) ** 2
        if p["color"].shape[0] < rows:
            pad = torch.zeros((rows - p["color"].shape[0], p["color"].shape[1]),
                              dtype=p["color"].dtype, device=device)
            p["color"] = torch.cat([p["color"], pad]).contiguous()
        self.active_sh = 0 if self.sh_up_every > 0 else self.sh_degree
        self._bind(p, {k: torch.zeros_like(v) for k, v in p.items()},
                   {k: torch.zeros_like(v) for k, v in p.items()}, dup_capacity)
        if density is not None:
            self.gen = torch.Generator(device=device).manual_seed(int(density.seed))
        self.step_count = 0
        self.timing = None            # optional dict of lists of (start, end) events

    def _bind(self, params, m, v, dup_capacity=None):
        """Point every buffer and call structure at a (new) set of Gaussians
        with their Adam moments; the device step count carries over."""
        self.params, self.m, self.v = params, m, v
        self.n = self.params["opacity_logit"].shape[-1]
        self.grads = {k: torch.zeros_like(t) for k, t in self.params.items()}
        self.views = ops.Views.single(self.n, self.cams_np[:1], self.device)
        self.views.use_cameras(self.cams[0:1])
        self.bufs = ops.RasterBuffers(self.views, self.W, self.H, self.tile,
                                      dup_capacity=dup_capacity, store_state=self.stored)
        self.bufs.set_schedule(self.plan["mode"], chunk=self.plan["chunk"],
                               fwd_waves=self.plan["fwd_waves"],
                               deterministic=self.plan["deterministic"])
        self.gst = ops.gaussians_struct(self.params, sh_degree=self.active_sh)
        self.grst = ops.grads_struct(self.grads, self.n)
        self.groups = ops.adam_groups(self.params, self.grads, self.m, self.v, self.lrs)
        if self.fused_adam:
            step_dev = self.dev_adam.step_dev if self.dev_adam is not None else None
            lrs_dev = dict(self.lrs, mean=self.lrs["mean"] * self.extent)
            self.dev_adam = ops.DeviceAdam(
                ops.adam_groups(self.params, self.grads, self.m, self.v, lrs_dev),
                lr_final=[1.6e-6 * self.extent, 0, 0, 0, 0], decay_steps=30000,
                device=self.device)
            if step_dev is not None:
                self.dev_adam.step_dev = step_dev
        if self.density is not None:
            if self.densifier is None:
                self.densifier = ops.Densifier(self.n, self.device)
            else:
                self.densifier.resize(self.n)

    def densify(self):
        """Clone / split / prune from the statistics gathered since the last
        call (one host synchronisation for the new count); returns it."""
        c = self.density
        big = (math.log(c.max_world_scale * self.extent) if self.step_count > c.reset_interval
               else float("inf"))
        log_split = math.log(c.split_divisor)
        n_out = self.densifier.select(self.params, self.m, self.v, c.grad_threshold,
                                      math.log(c.percent_dense * self.extent),
                                      math.log(c.min_opacity / (1.0 - c.min_opacity)), big,
                                      log_split)
        z = torch.randn((self.n, 2, 3), generator=self.gen, device=self.device)
        P, M, V = self.densifier.apply(self.params, self.m, self.v, n_out, z, log_split)
        per_gauss = self.bufs.dup_capacity / max(self.n, 1)
        self._bind(P, M, V, dup_capacity=int(per_gauss * max(n_out, 1) * 1.2) + 4096)
        self.densifier.reset_stats()
        return n_out

    def opacity_reset(self):
        """Clamp every opacity to 0.01 and clear its Adam moments."""
        ops.Densifier.opacity_reset(self.params, self.m, self.v, math.log(0.01 / 0.99))

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
        if (self.active_sh < self.sh_degree and self.step_count > 0
                and self.sh_up_every > 0 and self.step_count % self.sh_up_every == 0):
            self.active_sh += 1
            self.gst = ops.gaussians_struct(self.params, sh_degree=self.active_sh)
        self.views.use_cameras(self.cams[vi:vi + 1])
        self._ev("project")
        b.project(self.gst)
        self._ev("bin_sort")
        b.bin_sort()
        b.order_tiles()
        self._ev("raster_fwd")
        b.raster_fwd(self.bg)
        self._ev("loss")
        self.loss(b.image, self.targets[vi:vi + 1], self.masks[vi:vi + 1] if self.masks is not None
                  else None, self.lam, 1.0, b.status)
        self._ev("zero")
        b.zero_d_rec()
        self._ev("raster_bwd")
        b.raster_bwd(self.loss.d_image, self.bg, self.mode)
        c = self.density
        if c is not None and self.step_count < c.until:
            self.densifier.stats(b)
        self._ev("project_bwd")
        self.step_count += 1
        if self.fused_adam:
            b.project_bwd_adam(self.gst, self.dev_adam, visible_only=self.sparse_adam)
            self._ev("adam")
        else:
            b.project_bwd(self.gst, self.grst)
            self._ev("adam")
            self.groups[0].lr = mean_lr(self.step_count, self.extent, self.lrs["mean"])
            ops.adam_step(self.groups, self.step_count, zero_grad=True)
        self._ev("end")
        if c is not None and self.step_count < c.until:
            t = self.step_count
            if t > c.start and t % c.interval == 0:
                self.densify()
            if t % c.reset_interval == 0:
                self.opacity_reset()

    def check(self, grow=False):
        """Synchronise and raise on duplicate overflow / non-finite loss.
        With grow, an overflow instead enlarges the duplicate buffers to
        1.25 x the count needed and training goes on (the steps since the
        last check rasterised truncated lists); returns the count."""
        st, req = self.bufs.check()
        if st == _lib.GS_ERR_CAPACITY and grow:
            self.bufs.ensure_capacity(int(req * 1.25) + 4096)
            self.bufs.clear_status()
            self.capacity_grown = getattr(self, "capacity_grown", 0) + 1
            return req
        if st != _lib.GS_OK:
            raise _lib.GSError("training step", st, _lib.last_error())
        return req

    def evaluate(self, views=None):
        """Mean masked PSNR over views (gs_masked_psnr of each rendered view;
        evaluation only, views with an empty mask left out)."""
        views = list(range(self.V) if views is None else views)
        if getattr(self, "_psnr", None) is None:
            self._psnr = ops.PsnrBuffers(1, self.H, self.W, self.device)
            self._psnr_views = torch.empty(self.V, dtype=torch.float32, device=self.device)
        for i, vi in enumerate(views):
            self.views.use_cameras(self.cams[vi:vi + 1])
            self.bufs.render_checked(self.gst, self.bg)
            self._psnr(self.bufs.image, self.targets[vi:vi + 1],
                       self.masks[vi:vi + 1] if self.masks is not None else None,
                       out=self._psnr_views[i:i + 1])
        return mean_over_views(self._psnr_views[:len(views)].cpu().numpy())

    def train(self, steps, order_seed=0, eval_every=0, target_psnr=None, check_every=50,
              log=None, grow=False):
        """Run `steps` steps over a seeded view order.  Returns a history of
        (step, wall seconds excluding evaluation, psnr).  grow: see check()."""
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
                self.check(grow=grow)
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


class BatchedTrainer:
    """Uneven, ghost-padded partitions trained together: every step renders
    ``views_per_part`` views of every partition (S = partitions x views slots)
    through ONE launch per stage, and each stage's work is balanced by the
    longest-first tile order (and the chunked backward).  The views are cut
    into fixed groups (a seeded permutation of the orbit); each group's step
    is captured once in a HIP graph (gs_graph_begin / gs_graph_end through
    ops.StepGraph) and then replayed with gs_graph_launch: the step count
    and the position-lr decay live on the device.

    parts: list of dicts with params (planar SoA arrays), targets [V,3,H,W]
    float32 and masks [V,H,W] uint8 on the device, all seen from cams_np.
    The loss of a slot is scaled by 1/views_per_part, so each partition's
    gradient is the mean over its views; one Adam step per batch.
    """

    def __init__(self, parts, cams_np, views_per_part=4, tile=(16, 16), schedule="lpt",
                 chunk=64, stored=True, lam=0.2, bg=(0.0, 0.0, 0.0), extent=2.75, lrs=None,
                 order_seed=0, graphs=True, dup_capacity=None, fwd_waves=1, deterministic=False,
                 fused_adam=True, sparse_adam=False, sh_degree=0, sh_up_every=1000,
                 density=None, batch_scaling=True, device="cuda"):
        from .scene import concat_params
        self.device = device
        if sparse_adam and not fused_adam:
            raise ValueError("sparse_adam needs fused_adam (the fused call makes the step)")
        self.sparse_adam = bool(sparse_adam)
        self.P = len(parts)
        self.vpp = views_per_part
        self.counts = [int(p["params"]["opacity_logit"].shape[-1]) for p in parts]
        cat = concat_params([{k: np.asarray(v, np.float32) for k, v in p["params"].items()}
                             for p in parts])
        self.params = {k: torch.as_tensor(v).to(device) for k, v in cat.items()}
        self.n = sum(self.counts)
        # view-dependent colour as in the plain trainer (higher bands start
        # at zero; the active degree rises every sh_up_every steps, or is
        # sh_degree from the start when sh_up_every <= 0)
        self.sh_degree, self.sh_up_every = int(sh_degree), int(sh_up_every)
        rows = 3 * (self.sh_degree + 1) ** 2
        c = self.params["color"]
        if c.shape[0] < rows:
            self.params["color"] = torch.cat(
                [c, torch.zeros((rows - c.shape[0], c.shape[1]), dtype=c.dtype, device=device)]
            ).contiguous()
        self.active_sh = 0 if self.sh_up_every > 0 else self.sh_degree
        self.V = len(cams_np)
        assert self.V % views_per_part == 0, "the orbit must split into whole view groups"
        self.G = self.V // views_per_part
        self.S = self.P * views_per_part
        self.W, self.H = int(cams_np[0]["width"]), int(cams_np[0]["height"])
        rng = np.random.default_rng(order_seed)
        perm = rng.permutation(self.V)
        self.group_views = [perm[g * views_per_part:(g + 1) * views_per_part] for g in range(self.G)]
        cams_all = ops.Views.cams_to_device(cams_np, device)
        # per group: slot s = p * vpp + j sees view group_views[g][j]
        self.cams_g = torch.stack([torch.cat([cams_all[self.group_views[g]]] * self.P)
                                   for g in range(self.G)]).contiguous()
        self.targets_g = torch.empty((self.G, self.S, 3, self.H, self.W), dtype=torch.float32,
                                     device=device)
        self.masks_g = torch.empty((self.G, self.S, self.H, self.W), dtype=torch.uint8, device=device)
        for g in range(self.G):
            for p, part in enumerate(parts):
                idx = torch.as_tensor(self.group_views[g], device=part["targets"].device)
                self.targets_g[g, p * self.vpp:(p + 1) * self.vpp] = part["targets"][idx]
                self.masks_g[g, p * self.vpp:(p + 1) * self.vpp] = part["masks"][idx]
        self.bg, self.lam, self.extent = tuple(bg), lam, extent
        self.lrs = dict(DEFAULT_LR if lrs is None else lrs)
        self.lrs["mean"] = self.lrs["mean"] * extent
        # a step averages views_per_part views: with batch_scaling the Adam
        # rates grow by sqrt(B) and the moment decays become beta^B (B the
        # views per partition), so B views move the parameters about as far
        # as B one-view steps would
        B = views_per_part if batch_scaling else 1
        self.lr_scale = math.sqrt(B)
        self.betas = (0.9 ** B, 0.999 ** B)
        self.lrs = {k: v * self.lr_scale for k, v in self.lrs.items()}
        self.device = device
        self.plan = dict(tile=tuple(tile), stored=stored, schedule=schedule, chunk=chunk,
                         fwd_waves=fwd_waves, deterministic=deterministic)
        self.mode = _lib.GS_BWD_STORED if stored else _lib.GS_BWD_RECOMPUTE
        self.loss = ops.LossBuffers(self.S, self.H, self.W, device)
        # adaptive density control over all partitions at once (the outputs
        # keep input order, so every partition stays one contiguous range)
        self.density = density
        self.densifier = None
        if density is not None:
            self.gen = torch.Generator(device=device).manual_seed(int(density.seed))
        self.adam = None
        self._bind(self.params, {k: torch.zeros_like(v) for k, v in self.params.items()},
                   {k: torch.zeros_like(v) for k, v in self.params.items()}, dup_capacity)
        self.fused_adam = fused_adam
        self.use_graphs = graphs
        self.graphs = {}
        self._graph_gen = self.bufs.generation
        self._warm = set()
        self.steps_done = 0
        self._graph_stats = self._stats_on()    # whether the step body gathers statistics

    def _bind(self, params, m, v, dup_capacity=None):
        """Point every buffer, call structure and the optimiser at a (new) set
        of Gaussians in self.counts partitions; the device step count carries
        over and captured graphs are dropped (they hold the old pointers)."""
        self.params, self.m, self.v = params, m, v
        self.n = sum(self.counts)
        self.grads = {k: torch.zeros_like(t) for k, t in self.params.items()}
        pl = self.plan
        self.views = ops.Views.batch(self.counts, self.vpp, self.cams_g[0], self.device)
        self.bufs = ops.RasterBuffers(self.views, self.W, self.H, pl["tile"],
                                      dup_capacity=dup_capacity, store_state=pl["stored"])
        self.bufs.set_schedule(pl["schedule"], chunk=pl["chunk"], fwd_waves=pl["fwd_waves"],
                               deterministic=pl["deterministic"])
        self.gst = ops.gaussians_struct(self.params, sh_degree=self.active_sh)
        self.grst = ops.grads_struct(self.grads, self.n)
        self.groups = ops.adam_groups(self.params, self.grads, self.m, self.v, self.lrs)
        step_dev = self.adam.step_dev if self.adam is not None else None
        self.adam = ops.DeviceAdam(self.groups,
                                   lr_final=[1.6e-6 * self.extent * self.lr_scale, 0, 0, 0, 0],
                                   beta1=self.betas[0], beta2=self.betas[1],
                                   decay_steps=30000, device=self.device)
        if step_dev is not None:
            self.adam.step_dev = step_dev
        if self.density is not None:
            if self.densifier is None:
                self.densifier = ops.Densifier(self.n, self.device)
            else:
                self.densifier.resize(self.n)
        self.graphs = {}
        self._graph_gen = self.bufs.generation

    def set_plan(self, tile, schedule, chunk, fwd_waves=1, deterministic=False):
        """Rebind the raster buffers to another plan (tile shape, schedule,
        backward chunk, forward waves, deterministic sums); parameters,
        moments and the step count are kept, captured graphs dropped."""
        self.plan.update(tile=tuple(tile), schedule=schedule, chunk=int(chunk),
                         fwd_waves=int(fwd_waves), deterministic=bool(deterministic))
        self._bind(self.params, self.m, self.v)
        self.fit_capacity()

    def _stats_on(self):
        c = self.density
        return c is not None and self.steps_done < c.until

    def densify(self):
        """Clone / split / prune every partition from the statistics gathered
        since the last call; the partitions' new counts come from the
        actions (one host synchronisation).  Returns the new total."""
        c = self.density
        big = (math.log(c.max_world_scale * self.extent) if self.steps_done > c.reset_interval
               else float("inf"))
        log_split = math.log(c.split_divisor)
        n_out = self.densifier.select(self.params, self.m, self.v, c.grad_threshold,
                                      math.log(c.percent_dense * self.extent),
                                      math.log(c.min_opacity / (1.0 - c.min_opacity)), big,
                                      log_split)
        act = self.densifier.action[:self.n].cpu().numpy()
        outs = np.select([act == 1, act == 2, act == 3], [1, 2, 2], 0)
        bounds = np.cumsum([0] + list(self.counts))
        counts = [int(outs[bounds[p]:bounds[p + 1]].sum()) for p in range(self.P)]
        assert sum(counts) == n_out
        z = torch.randn((self.n, 2, 3), generator=self.gen, device=self.device)
        P, M, V = self.densifier.apply(self.params, self.m, self.v, n_out, z, log_split)
        per_gauss = self.bufs.dup_capacity / max(self.n, 1)
        self.counts = counts
        self._bind(P, M, V, dup_capacity=int(per_gauss * max(n_out, 1) * 1.2) + 4096)
        self.densifier.reset_stats()
        return n_out

    def fit_capacity(self, margin=1.3):
        need = 0
        for g in range(self.G):
            self.views.use_cameras(self.cams_g[g])
            need = max(need, self.bufs.render_checked(self.gst, self.bg))
        self.bufs.ensure_capacity(int(need * margin) + 4096)
        self.graphs = {}
        self._graph_gen = self.bufs.generation
        return need

    def _ev(self, name, timing):
        if timing is None:
            return
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        timing.setdefault(name, []).append(e)

    def _step_body(self, g, timing=None):
        b = self.bufs
        self.views.use_cameras(self.cams_g[g])
        self._ev("project", timing)
        b.project(self.gst)
        self._ev("bin_sort", timing)
        b.bin_sort()
        b.order_tiles()
        self._ev("raster_fwd", timing)
        b.raster_fwd(self.bg)
        self._ev("loss", timing)
        self.loss(b.image, self.targets_g[g], self.masks_g[g], self.lam, 1.0 / self.vpp, b.status)
        self._ev("zero", timing)
        b.zero_d_rec()
        self._ev("raster_bwd", timing)
        b.raster_bwd(self.loss.d_image, self.bg, self.mode)
        if self._graph_stats:
            self.densifier.stats(b)
        self._ev("project_bwd", timing)
        if self.fused_adam:
            b.project_bwd_adam(self.gst, self.adam, visible_only=self.sparse_adam)
        else:
            b.project_bwd(self.gst, self.grst)
            self.adam(zero_grad=True)
        self._ev("end", timing)

    def _drop_stale_graphs(self):
        """Captured graphs hold the buffers' pointers: drop them when a
        buffer was reallocated (capacity growth, e.g. inside evaluate)."""
        if self.bufs.generation != self._graph_gen:
            self.graphs = {}
            self._graph_gen = self.bufs.generation

    def step(self, g, timing=None):
        """One batched step on view group g (graph replay after the first).
        With a timing dict the step runs eagerly with HIP events around its
        stages (on the launch stream), appended to timing[stage]."""
        self._drop_stale_graphs()
        if (self.active_sh < self.sh_degree and self.steps_done > 0 and self.sh_up_every > 0
                and self.steps_done % self.sh_up_every == 0):
            # the degree is a kernel argument baked into the captured graphs
            self.active_sh += 1
            self.gst = ops.gaussians_struct(self.params, sh_degree=self.active_sh)
            self.graphs = {}
        if self._stats_on() != self._graph_stats:
            # the density statistics leave (or join) the captured step
            self._graph_stats = self._stats_on()
            self.graphs = {}
        if timing is not None or not self.use_graphs or g not in self._warm:
            # eager (also the first time, so every kernel is loaded before capture)
            self._step_body(g, timing)
            self._warm.add(g)
        else:
            graph = self.graphs.get(g)
            if graph is None:
                # capture; the capture itself does not execute the work
                torch.cuda.synchronize()
                graph = ops.StepGraph(lambda: self._step_body(g), self.device)
                self.graphs[g] = graph
            graph.replay()
        self.steps_done += 1
        c = self.density
        if c is not None and self.steps_done < c.until:
            t = self.steps_done
            if t > c.start and t % c.interval == 0:
                self.densify()
            if t % c.reset_interval == 0:
                ops.Densifier.opacity_reset(self.params, self.m, self.v, math.log(0.01 / 0.99))

    def check(self):
        st, req = self.bufs.check()
        if st != _lib.GS_OK:
            raise _lib.GSError("batched step", st, _lib.last_error())
        return req

    def prepare(self):
        """Capture every view group's step before training (set-up, not
        training): one eager step loads the kernels, its effect on the
        parameters and optimiser state is undone, then each group's step is
        captured (capturing does not run it)."""
        if not self.use_graphs:
            return
        self._drop_stale_graphs()
        saved = [t.clone() for d in (self.params, self.m, self.v) for t in d.values()]
        step0 = self.adam.step_dev.clone()
        self._step_body(0)
        torch.cuda.synchronize()
        i = 0
        for d in (self.params, self.m, self.v):
            for t in d.values():
                t.copy_(saved[i])
                i += 1
        self.adam.step_dev.copy_(step0)
        if self.densifier is not None:
            self.densifier.reset_stats()      # the undone step's statistics too
        for g in range(self.G):
            if g not in self.graphs:
                torch.cuda.synchronize()
                self.graphs[g] = ops.StepGraph(lambda: self._step_body(g), self.device)
            self._warm.add(g)
        torch.cuda.synchronize()

    def evaluate(self):
        """Masked PSNR per partition (gs_masked_psnr of every slot, mean over
        the partition's views); evaluation only."""
        if getattr(self, "_psnr", None) is None:
            self._psnr = ops.PsnrBuffers(self.S, self.H, self.W, self.device)
        ps = np.zeros((self.P, self.V))
        for g in range(self.G):
            self.views.use_cameras(self.cams_g[g])
            self.bufs.render_checked(self.gst, self.bg)
            pv = self._psnr(self.bufs.image, self.targets_g[g], self.masks_g[g]).cpu().numpy()
            for p in range(self.P):
                for j in range(self.vpp):
                    ps[p, self.group_views[g][j]] = pv[p * self.vpp + j]
        return np.array([mean_over_views(ps[p]) for p in range(self.P)])

    def partition_params(self, p):
        o = sum(self.counts[:p])
        return {k: v[..., o:o + self.counts[p]] for k, v in self.params.items()}
