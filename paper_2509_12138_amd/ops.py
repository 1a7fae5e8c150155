"""PyTorch-facing wrappers of libgsmi: buffers, calls and autograd Functions.

PyTorch supplies device memory and the stream only; every computation runs
in the library's HIP kernels through the C ABI (include/gs.h).
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from . import _lib
from ._lib import call

PARAM_NAMES = ("mean", "log_scale", "quat", "opacity_logit", "color")
PARAM_ROWS = {"mean": 3, "log_scale": 3, "quat": 4, "opacity_logit": 1, "color": 3}


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def stream_handle(device=None):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_f32(t, name):
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")


# --------------------------------------------------------------------------
# Structures
# --------------------------------------------------------------------------

SH_MAX_DEGREE = 3


def sh_degree_of(color):
    """Highest spherical-harmonic degree D whose 3 (D+1)^2 coefficient rows
    a planar colour array [rows, n] holds."""
    rows = color.shape[0]
    D = int(round(math.sqrt(rows / 3.0))) - 1
    if rows % 3 or D < 0 or D > SH_MAX_DEGREE or 3 * (D + 1) ** 2 != rows:
        raise ValueError(f"colour has {rows} rows; expected 3 (D+1)^2 with D <= {SH_MAX_DEGREE}")
    return D


def gaussians_struct(params, n=None, sh_degree=None):
    """gs_gaussians over planar tensors; sh_degree defaults to the degree the
    colour rows hold (a lower one draws the leading coefficients only)."""
    for k in PARAM_NAMES:
        _check_f32(params[k], k)
    n = params["opacity_logit"].shape[-1] if n is None else n
    stored = sh_degree_of(params["color"])
    D = stored if sh_degree is None else int(sh_degree)
    if not 0 <= D <= stored:
        raise ValueError(f"sh_degree {D} outside 0..{stored} (the degree the colour rows hold)")
    return _lib.gs_gaussians(*[params[k].data_ptr() for k in PARAM_NAMES], n, D, 0)


def grads_struct(grads, n):
    for k in PARAM_NAMES:
        _check_f32(grads[k], "grad " + k)
    return _lib.gs_grads(*[grads[k].data_ptr() for k in PARAM_NAMES], n)


class Views:
    """Device-side slot table: which Gaussians each image draws and with
    which camera.  Camera records are the 80-byte gs_camera layout."""

    def __init__(self, pair_offset, gauss_offset, cams_u8, device):
        self.device = device
        self.pair_offset_host = np.asarray(pair_offset, np.int64)
        self.n_slots = len(self.pair_offset_host) - 1
        self.total_pairs = int(self.pair_offset_host[-1])
        self.pair_offset = torch.as_tensor(self.pair_offset_host, device=device)
        self.gauss_offset = torch.as_tensor(np.asarray(gauss_offset, np.int64), device=device)
        self.cams = cams_u8
        self.struct = _lib.gs_views(self.n_slots, self.total_pairs, self.pair_offset.data_ptr(),
                                    self.gauss_offset.data_ptr(), self.cams.data_ptr())

    @staticmethod
    def cams_to_device(cams_np, device):
        raw = np.ascontiguousarray(cams_np).view(np.uint8).reshape(len(cams_np), 80)
        return torch.as_tensor(raw, device=device)

    @classmethod
    def single(cls, n, cams_np, device="cuda"):
        """One partition of n Gaussians seen through every camera in cams_np."""
        V = len(cams_np)
        po = np.arange(V + 1, dtype=np.int64) * n
        return cls(po, np.zeros(V, np.int64), cls.cams_to_device(cams_np, device), device)

    @classmethod
    def batch(cls, counts, views_per_part, cams_dev_u8, device="cuda"):
        """Partitions stored back to back (counts[p] Gaussians each), each
        seen from views_per_part slots; cams_dev_u8 holds one record per slot."""
        from .scene import views_table
        po, go = views_table(counts, views_per_part)
        return cls(po, go, cams_dev_u8, device)

    def use_cameras(self, cams_u8):
        """Point the slots at other camera records (device uint8 [S, 80])."""
        assert cams_u8.shape[0] >= self.n_slots and cams_u8.dtype == torch.uint8
        self.cams = cams_u8
        self.struct.cams = cams_u8.data_ptr()


def tiling_struct(width, height, tile=(16, 16)):
    return _lib.gs_tiling(width, height, tile[0], tile[1])


# --------------------------------------------------------------------------
# Buffers of one rasterisation configuration
# --------------------------------------------------------------------------

class RasterBuffers:
    """All device buffers one (views, tiling) configuration needs.

    dup_capacity grows on overflow (see ``ensure_capacity``).  keep_keys: also
    keep the sorted 64-bit (tile, depth) keys in ``keys`` (the rasterisers
    need only ids and ranges; without it the sort carries 32-bit tile keys)."""

    def __init__(self, views: Views, width, height, tile=(16, 16), dup_capacity=None,
                 store_state=True, keep_keys=False):
        dev = views.device
        self.views = views
        self.W, self.H, self.tile = width, height, tuple(tile)
        self.tiling = tiling_struct(width, height, tile)
        self.tiles_x = math.ceil(width / tile[0])
        self.tiles_y = math.ceil(height / tile[1])
        self.tiles_per_slot = self.tiles_x * self.tiles_y
        S, m = views.n_slots, views.total_pairs
        self.S, self.m = S, m
        self.rec = torch.empty((max(m, 1), 12), dtype=torch.float32, device=dev)
        self.tile_bbox = torch.empty((max(m, 1), 4), dtype=torch.int16, device=dev)
        self.n_tiles = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
        self.proj = _lib.gs_projected(self.rec.data_ptr(), self.tile_bbox.data_ptr(),
                                      self.n_tiles.data_ptr(), m)
        self.ranges = torch.empty((S * self.tiles_per_slot, 2), dtype=torch.int32, device=dev)
        self.image = torch.empty((S, 3, height, width), dtype=torch.float32, device=dev)
        self.store_state = store_state
        if store_state:
            self.T_final = torch.empty((S, height, width), dtype=torch.float32, device=dev)
            self.n_contrib = torch.empty((S, height, width), dtype=torch.int32, device=dev)
        else:
            self.T_final = self.n_contrib = None
        self.d_rec = torch.zeros((max(m, 1), 9), dtype=torch.float32, device=dev)
        self.pair_first = torch.empty(2 * max(m, 1), dtype=torch.int32, device=dev)   # (first, count)
        self.status = torch.zeros(4, dtype=torch.int64, device=dev)
        self.keys = self.ids = self.ws = None
        self.keep_keys = bool(keep_keys)
        self.dup_grads = None
        self.deterministic = False
        self.plan = None
        self.schedule = "default"
        self.chunk = 0
        self.fwd_waves = 1
        self.dup_capacity = 0
        # bumped whenever a buffer that launches point at is reallocated, so
        # that holders of captured graphs know to re-capture them
        self.generation = 0
        # a failure status read (and cleared) by render_checked before a
        # trainer's own check saw it
        self._pending = None
        self.ensure_capacity(dup_capacity or max(4 * m, 1024))

    def ensure_capacity(self, cap):
        """Grow the duplicate buffers to at least cap entries; returns True
        if they were reallocated (graphs holding the old pointers are then
        stale: ``generation`` changes)."""
        cap = int(min(max(cap, 1024), 0xFFFFFFFF))
        if cap <= self.dup_capacity:
            return False
        self.generation += 1
        dev = self.views.device
        self.dup_capacity = cap
        self.keys = torch.empty(cap, dtype=torch.int64, device=dev) if self.keep_keys else None
        self.ids = torch.empty(cap, dtype=torch.int32, device=dev)
        self.emit = torch.empty(cap, dtype=torch.int32, device=dev)
        nbytes = _lib.load().gs_bin_sort_workspace_bytes(self.m, cap, C.byref(self.tiling),
                                                         self.S)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        if self.chunk:
            self._alloc_chunks()
        if self.deterministic:
            self._alloc_dup_grads()
        return True

    # ---------------------------------------------------------- the calls

    def project(self, gstruct, stream=None):
        s = stream or stream_handle()
        call("gs_project", C.byref(gstruct), C.byref(self.views.struct), C.byref(self.tiling),
             C.byref(self.proj), s)

    def bin_sort(self, stream=None):
        s = stream or stream_handle()
        call("gs_bin_sort", C.byref(self.proj), C.byref(self.views.struct), C.byref(self.tiling),
             self.dup_capacity, _ptr(self.ws), self.ws.numel(),
             _ptr(self.keys) if self.keep_keys else None, _ptr(self.ids),
             _ptr(self.ranges), _ptr(self.pair_first) if self.deterministic else None,
             _ptr(self.emit) if self.deterministic else None, _ptr(self.status), s)

    # ---------------------------------------------------------- tile schedule

    def set_schedule(self, mode="default", persistent_waves=0, chunk=0, fwd_waves=1,
                     deterministic=False, split=False):
        """How the rasterisers walk the tiles: "default" (XCD-aware order, one
        work-group per tile), "lpt" (longest tile lists first) or "persistent"
        (longest first, pulled from an atomic queue by a persistent grid).
        chunk > 0 (a multiple of 64) cuts the backward's tile lists into
        chunk-entry work items (stored mode), using forward checkpoints.
        fwd_waves (1, 2, 4) splits each tile's pixels over that many waves in
        the forward.  deterministic: per-entry gradient slots summed per pair
        instead of atomics (bitwise reproducible gradients).  split (chunked
        plans; also a "+split" suffix of the mode, e.g. "lpt+split"): the
        forward composites the chunk items in parallel and joins them per
        tile."""
        dev = self.views.device
        if mode.endswith("+split"):
            mode, split = mode[:-len("+split")], True
        self.schedule = mode
        self.chunk = int(chunk) if self.store_state else 0
        self.fwd_waves = int(fwd_waves)
        self.deterministic = bool(deterministic)
        self.split = bool(split) and self.chunk > 0
        n = self.S * self.tiles_per_slot
        self.plan = _lib.gs_raster_plan()
        self.plan.fwd_waves = self.fwd_waves
        if mode != "default":
            self.tile_order = torch.empty(n, dtype=torch.int32, device=dev)
            nb = _lib.load().gs_tile_order_workspace_bytes(n)
            self.order_ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
            self.queue = torch.zeros(1, dtype=torch.int32, device=dev) if mode == "persistent" else None
            self.plan.tile_order = self.tile_order.data_ptr()
            self.plan.queue = self.queue.data_ptr() if self.queue is not None else None
            self.plan.persistent_waves = int(persistent_waves)
        if self.chunk:
            self.chunk_offset = torch.empty(n + 1, dtype=torch.int32, device=dev)
            self._alloc_chunks()
        if self.deterministic:
            self._alloc_dup_grads()
        else:
            self.dup_grads = None
        if mode == "default" and not self.chunk and self.fwd_waves <= 1 and not self.deterministic:
            self.plan = None

    def _alloc_dup_grads(self):
        self.dup_grads = torch.empty((self.dup_capacity, 9), dtype=torch.float32,
                                     device=self.views.device)
        self.plan.dup_grads = self.dup_grads.data_ptr()
        self.plan.pair_first = self.pair_first.data_ptr()
        self.plan.dup_capacity = self.dup_capacity
        self.plan.emit_idx = self.emit.data_ptr()

    def _alloc_chunks(self):
        dev = self.views.device
        n = self.S * self.tiles_per_slot
        self.max_items = int(_lib.load().gs_chunk_max_items(n, self.dup_capacity, self.chunk))
        self.chunk_items = torch.empty(self.max_items, dtype=torch.int32, device=dev)
        self.checkpoints = torch.empty((self.max_items, self.tile[0] * self.tile[1], 4),
                                       dtype=torch.float32, device=dev)
        self.plan.chunk = self.chunk
        self.plan.chunk_offset = self.chunk_offset.data_ptr()
        self.plan.chunk_items = self.chunk_items.data_ptr()
        self.plan.checkpoints = self.checkpoints.data_ptr()
        self.plan.max_items = self.max_items
        if getattr(self, "split", False):
            self.chunk_last = torch.empty((self.max_items, self.tile[0] * self.tile[1]),
                                          dtype=torch.int16, device=dev)
            self.plan.fwd_split = 1
            self.plan.chunk_last = self.chunk_last.data_ptr()

    def order_tiles(self, stream=None):
        """Per-step plan inputs that depend on the sorted lists."""
        if self.plan is None:
            return
        s = stream or stream_handle()
        n = self.S * self.tiles_per_slot
        if self.schedule != "default":
            call("gs_tile_order", _ptr(self.ranges), n, _ptr(self.order_ws), self.order_ws.numel(),
                 _ptr(self.tile_order), s)
        if self.chunk:
            call("gs_chunk_items", _ptr(self.ranges), n, self.chunk, self.max_items,
                 _ptr(self.chunk_offset), _ptr(self.chunk_items), s)

    def _plan_ref(self):
        return C.byref(self.plan) if self.plan is not None else None

    def raster_fwd(self, bg=(0.0, 0.0, 0.0), stream=None):
        s = stream or stream_handle()
        call("gs_raster_fwd", C.byref(self.proj), C.byref(self.views.struct),
             C.byref(self.tiling), _ptr(self.ids), _ptr(self.ranges), _lib.F3(*bg),
             _ptr(self.image), _ptr(self.T_final), _ptr(self.n_contrib), self._plan_ref(), s)

    def count_blended(self, stream=None):
        """Per-pixel number of blended list entries (gs_raster_count) of the
        current lists, as a new [S, H, W] int32 tensor."""
        out = torch.empty((self.S, self.H, self.W), dtype=torch.int32, device=self.views.device)
        call("gs_raster_count", C.byref(self.proj), C.byref(self.views.struct),
             C.byref(self.tiling), _ptr(self.ids), _ptr(self.ranges), _ptr(out),
             stream or stream_handle())
        return out

    def raster_bwd(self, d_image, bg=(0.0, 0.0, 0.0), mode=None, stream=None):
        s = stream or stream_handle()
        if mode is None:
            mode = _lib.GS_BWD_STORED if self.store_state else _lib.GS_BWD_RECOMPUTE
        _check_f32(d_image, "d_image")
        call("gs_raster_bwd", C.byref(self.proj), C.byref(self.views.struct),
             C.byref(self.tiling), _ptr(self.ids), _ptr(self.ranges), _lib.F3(*bg),
             _ptr(self.T_final), _ptr(self.n_contrib), _ptr(d_image), int(mode),
             _ptr(self.d_rec), self._plan_ref(), s)

    def project_bwd(self, gstruct, grads_struct_, stream=None):
        s = stream or stream_handle()
        call("gs_project_bwd", C.byref(gstruct), C.byref(self.views.struct),
             C.byref(self.tiling), C.byref(self.proj), _ptr(self.d_rec),
             C.byref(grads_struct_), s)

    def project_bwd_adam(self, gstruct, adam, visible_only=False, stream=None):
        """gs_project_bwd_adam: projection backward and the DeviceAdam step
        `adam` in one pass (gradient arrays untouched); visible_only selects
        the sparse step (Gaussians the views do not draw stay as they are)."""
        s = stream or stream_handle()
        call("gs_project_bwd_adam", C.byref(gstruct), C.byref(self.views.struct),
             C.byref(self.tiling), C.byref(self.proj), _ptr(self.d_rec), adam.groups,
             len(adam.groups), adam.lr_final, adam.decay_steps, adam.betas[0], adam.betas[1], adam.betas[2],
             int(bool(visible_only)), _ptr(adam.step_dev), s)

    def zero_d_rec(self, stream=None):
        s = stream or stream_handle()
        call("gs_zero", _ptr(self.d_rec), self.d_rec.numel() * 4, s)

    def _read_status(self, stream=None):
        s = stream or stream_handle()
        req = C.c_int64(0)
        st = _lib.load().gs_check_status(_ptr(self.status), s, C.byref(req))
        return st, int(req.value)

    def check(self, stream=None):
        """Synchronise and report (status, required duplicates), including a
        failure that render_checked read before this call."""
        st, req = self._read_status(stream)
        if self._pending is not None:
            pst, preq = self._pending
            self._pending = None
            if st == _lib.GS_OK or st == pst:
                st, req = pst, max(req, preq)
        return st, req

    def clear_status(self, stream=None):
        call("gs_zero", _ptr(self.status), self.status.numel() * 8, stream or stream_handle())

    def render_checked(self, gstruct, bg=(0.0, 0.0, 0.0), max_retry=3):
        """project + bin_sort (+ capacity growth on overflow) + raster_fwd.
        A failure flagged by earlier asynchronous steps is kept for the next
        check() before the status is cleared."""
        st, req = self._read_status()
        if st != _lib.GS_OK:
            if self._pending is not None and self._pending[0] == st:
                req = max(req, self._pending[1])
            self._pending = (st, req)
        for _ in range(max_retry + 1):
            self.clear_status()
            self.project(gstruct)
            self.bin_sort()
            st, req = self.check()
            if st == _lib.GS_ERR_CAPACITY:
                self.ensure_capacity(int(req * 1.25) + 1024)
                continue
            if st not in (_lib.GS_OK,):
                raise _lib.GSError("gs_bin_sort", st, _lib.last_error())
            self.order_tiles()
            self.raster_fwd(bg)
            return req
        raise RuntimeError("duplicate capacity could not be satisfied")


# --------------------------------------------------------------------------
# Loss and optimiser
# --------------------------------------------------------------------------

class StepGraph:
    """A sequence of library calls captured into a HIP graph through the C
    ABI (gs_graph_begin / gs_graph_end on a stream of its own, default
    priority) and replayed with gs_graph_launch.  body() must enqueue only
    library calls on the current stream and allocate nothing; the buffers it
    names must outlive the graph."""

    def __init__(self, body, device=None):
        self._h = None
        lib = _lib.load()
        self._stream = torch.cuda.Stream(device=device)
        self._stream.wait_stream(torch.cuda.current_stream(device))
        h = C.c_void_p(self._stream.cuda_stream)
        out = C.c_void_p()
        with torch.cuda.stream(self._stream):
            call("gs_graph_begin", h)
            try:
                body()
            except BaseException:
                if lib.gs_graph_end(h, C.byref(out)) == _lib.GS_OK:
                    lib.gs_graph_destroy(out)
                raise
            call("gs_graph_end", h, C.byref(out))
        self._h = out

    def replay(self, stream=None):
        call("gs_graph_launch", self._h, stream or stream_handle())

    def __del__(self):
        if self._h:
            _lib.load().gs_graph_destroy(self._h)
            self._h = None


class LossBuffers:
    def __init__(self, S, H, W, device="cuda"):
        self.S, self.H, self.W = S, H, W
        nbytes = _lib.load().gs_loss_workspace_bytes(S, H, W)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.loss = torch.zeros(S, dtype=torch.float32, device=device)
        self.d_image = torch.empty((S, 3, H, W), dtype=torch.float32, device=device)

    def __call__(self, image, target, mask=None, lam=0.2, grad_scale=1.0, status=None,
                 stream=None):
        _check_f32(image, "image"); _check_f32(target, "target")
        if mask is not None and (mask.dtype != torch.uint8 or not mask.is_contiguous()):
            raise ValueError("mask must be a contiguous uint8 tensor")
        call("gs_loss", _ptr(image), _ptr(target), _ptr(mask), self.S, self.H, self.W,
             float(lam), float(grad_scale), _ptr(self.ws), self.ws.numel(), _ptr(self.loss),
             _ptr(self.d_image), _ptr(status), stream or stream_handle())
        return self.loss, self.d_image


def adam_groups(params, grads, m, v, lrs):
    """gs_adam_group array over the five parameter arrays.  With an lrs
    entry "color_rest" and more than 3 colour rows, a sixth group takes the
    colour rows from 3 on (the higher spherical-harmonic bands) at that
    rate and group 4 keeps rows 0-2."""
    rest = "color_rest" in lrs and params["color"].shape[0] > 3
    arr = (_lib.gs_adam_group * (len(PARAM_NAMES) + int(rest)))()
    for i, k in enumerate(PARAM_NAMES):
        cnt = params[k].numel()
        if rest and k == "color":
            cnt = 3 * params[k].shape[-1]
        arr[i] = _lib.gs_adam_group(params[k].data_ptr(), grads[k].data_ptr(), m[k].data_ptr(),
                                    v[k].data_ptr(), cnt, float(lrs[k]))
    if rest:
        off = 3 * params["color"].shape[-1] * 4           # bytes
        c = params["color"]
        arr[5] = _lib.gs_adam_group(c.data_ptr() + off, grads["color"].data_ptr() + off,
                                    m["color"].data_ptr() + off, v["color"].data_ptr() + off,
                                    c.numel() - 3 * c.shape[-1], float(lrs["color_rest"]))
    return arr


def adam_step(groups, step, beta1=0.9, beta2=0.999, eps=1e-15, zero_grad=True, stream=None):
    call("gs_adam", groups, len(groups), beta1, beta2, eps, int(step), int(bool(zero_grad)),
         stream or stream_handle())


class DeviceAdam:
    """Adam whose step count and position-lr decay live on the device
    (gs_adam_dev), so that captured graphs replay whole training steps."""

    def __init__(self, groups, lr_final=None, decay_steps=30000, beta1=0.9, beta2=0.999,
                 eps=1e-15, device="cuda"):
        self.groups = groups
        n = len(groups)
        lf = [0.0] * n if lr_final is None else list(lr_final)[:n]
        self.lr_final = (_lib.f32 * n)(*(lf + [0.0] * (n - len(lf))))
        self.decay_steps = int(decay_steps)
        self.betas = (beta1, beta2, eps)
        self.step_dev = torch.zeros(1, dtype=torch.int32, device=device)

    def __call__(self, zero_grad=True, stream=None):
        call("gs_adam_dev", self.groups, len(self.groups), self.lr_final, self.decay_steps,
             self.betas[0], self.betas[1], self.betas[2], _ptr(self.step_dev),
             int(bool(zero_grad)), stream or stream_handle())


# --------------------------------------------------------------------------
# autograd
# --------------------------------------------------------------------------

class RenderFn(torch.autograd.Function):
    """image = render(Gaussians) through the library's projection, binning,
    sort and compositing; backward runs the hand-written reverse replay and
    the projection backward."""

    @staticmethod
    def forward(ctx, mean, log_scale, quat, opacity_logit, color, bufs: RasterBuffers, bg,
                mode):
        params = dict(mean=mean, log_scale=log_scale, quat=quat, opacity_logit=opacity_logit,
                      color=color)
        gst = gaussians_struct(params)
        bufs.render_checked(gst, bg)
        ctx.bufs, ctx.bg, ctx.mode = bufs, bg, mode
        ctx.save_for_backward(mean, log_scale, quat, opacity_logit, color)
        return bufs.image.clone()

    @staticmethod
    def backward(ctx, d_image):
        mean, log_scale, quat, opacity_logit, color = ctx.saved_tensors
        params = dict(mean=mean, log_scale=log_scale, quat=quat, opacity_logit=opacity_logit,
                      color=color)
        bufs = ctx.bufs
        grads = {k: torch.zeros_like(v) for k, v in params.items()}
        bufs.zero_d_rec()
        bufs.raster_bwd(d_image.contiguous(), ctx.bg, ctx.mode)
        n = opacity_logit.shape[-1]
        bufs.project_bwd(gaussians_struct(params), grads_struct(grads, n))
        return (grads["mean"], grads["log_scale"], grads["quat"], grads["opacity_logit"],
                grads["color"], None, None, None)


def render(params, bufs: RasterBuffers, bg=(0.0, 0.0, 0.0), mode=None):
    if mode is None:
        mode = _lib.GS_BWD_STORED if bufs.store_state else _lib.GS_BWD_RECOMPUTE
    return RenderFn.apply(params["mean"], params["log_scale"], params["quat"],
                          params["opacity_logit"], params["color"], bufs, tuple(bg), mode)


class LossFn(torch.autograd.Function):
    """Masked (1 - lam) L1 + lam D-SSIM per image (gs_loss); returns [S]."""

    @staticmethod
    def forward(ctx, image, target, mask, lam, lbufs: LossBuffers):
        loss, d_image = lbufs(image.contiguous(), target, mask, lam, 1.0)
        ctx.save_for_backward(d_image.clone())
        return loss.clone()

    @staticmethod
    def backward(ctx, d_loss):
        (d_image,) = ctx.saved_tensors
        out = d_image.clone()
        S = out.shape[0]
        call("gs_scale_rows", _ptr(out), _ptr(d_loss.contiguous().float()), S,
             out.numel() // max(S, 1), stream_handle())
        return out, None, None, None, None


class PsnrBuffers:
    """Workspace and output of gs_masked_psnr for S images of H x W."""

    def __init__(self, S, H, W, device="cuda"):
        self.S, self.H, self.W = S, H, W
        nbytes = _lib.load().gs_psnr_workspace_bytes(S, H, W)
        self.ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        self.psnr = torch.empty(S, dtype=torch.float32, device=device)

    def __call__(self, image, target, mask=None, out=None, stream=None):
        """Masked PSNR of each image (device [S] tensor; `out` may be a
        slice of a longer device array to write into)."""
        _check_f32(image, "image"); _check_f32(target, "target")
        if mask is not None and (mask.dtype != torch.uint8 or not mask.is_contiguous()):
            raise ValueError("mask must be a contiguous uint8 tensor")
        dst = self.psnr if out is None else out
        if dst.dtype != torch.float32 or dst.numel() < self.S or not dst.is_contiguous():
            raise ValueError("psnr output must be a contiguous float32 tensor of S entries")
        call("gs_masked_psnr", _ptr(image), _ptr(target), _ptr(mask), self.S, self.H, self.W,
             _ptr(self.ws), self.ws.numel(), _ptr(dst), stream or stream_handle())
        return dst


def masked_psnr(image, target, mask=None):
    """Masked PSNR of a stack of images [S, 3, H, W] (gs_masked_psnr):
    device tensor [S]; NaN for an empty mask, +inf for an exact match."""
    if image.dim() == 3:
        image, target = image.unsqueeze(0), target.unsqueeze(0)
        mask = mask.unsqueeze(0) if mask is not None else None
    S, _, H, W = image.shape
    return PsnrBuffers(S, H, W, image.device)(image.contiguous(), target.contiguous(),
                                              mask.contiguous() if mask is not None else None)


# --------------------------------------------------------------------------
# k nearest neighbours
# --------------------------------------------------------------------------

def knn(points, k, with_mean=False):
    """Exact k-NN of device points [3, n] (gs_knn); returns (idx [n,k] int32,
    dist [n,k] float32) sorted by (distance, index), and with_mean also the
    mean distance [n]."""
    _check_f32(points, "points")
    n = points.shape[1]
    idx = torch.empty((n, k), dtype=torch.int32, device=points.device)
    dist = torch.empty((n, k), dtype=torch.float32, device=points.device)
    mean = torch.empty(n, dtype=torch.float32, device=points.device) if with_mean else None
    if n > 0:
        nbytes = _lib.load().gs_knn_workspace_bytes(n, k)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=points.device)
        call("gs_knn", _ptr(points), n, int(k), _ptr(ws), nbytes, _ptr(idx), _ptr(dist),
             _ptr(mean), stream_handle())
    return (idx, dist, mean) if with_mean else (idx, dist)


def knn_mean_distance(points, k=3):
    """Mean distance to the k nearest neighbours of each device point
    (computed by gs_knn; the neighbour lists are not written)."""
    _check_f32(points, "points")
    n = points.shape[1]
    mean = torch.empty(n, dtype=torch.float32, device=points.device)
    if n > 0:
        nbytes = _lib.load().gs_knn_workspace_bytes(n, k)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=points.device)
        call("gs_knn", _ptr(points), n, int(k), _ptr(ws), nbytes, None, None, _ptr(mean),
             stream_handle())
    return mean


def plain_init(points, normals, opacity, shape=True):
    """gs_plain_init: Gaussians of device surface points [3, n] with unit
    normals [3, n]; shape=False writes only mean and colour (the other
    arrays are returned uninitialised)."""
    _check_f32(points, "points"); _check_f32(normals, "normals")
    n = points.shape[1]
    dev = points.device
    out = dict(mean=torch.empty((3, n), dtype=torch.float32, device=dev),
               log_scale=torch.empty((3, n), dtype=torch.float32, device=dev),
               quat=torch.empty((4, n), dtype=torch.float32, device=dev),
               opacity_logit=torch.empty(n, dtype=torch.float32, device=dev),
               color=torch.empty((3, n), dtype=torch.float32, device=dev))
    if n == 0:
        return out
    nbytes = _lib.load().gs_plain_init_workspace_bytes(n) if shape else 0
    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
    call("gs_plain_init", _ptr(points), _ptr(normals), n, float(opacity), _ptr(ws), nbytes,
         _ptr(out["mean"]), _ptr(out["log_scale"]) if shape else None,
         _ptr(out["quat"]) if shape else None, _ptr(out["opacity_logit"]) if shape else None,
         _ptr(out["color"]), stream_handle())
    return out


# --------------------------------------------------------------------------
# adaptive density control
# --------------------------------------------------------------------------

def gaussian_state(params, m=None, v=None):
    """gs_gaussian_state over planar parameter tensors (and Adam moments)."""
    st = _lib.gs_gaussian_state()
    for i, k in enumerate(PARAM_NAMES):
        st.param[i] = params[k].data_ptr()
        st.m[i] = m[k].data_ptr() if m is not None else None
        st.v[i] = v[k].data_ptr() if v is not None else None
    st.n = params["opacity_logit"].shape[-1]
    st.color_rows = params["color"].shape[0]
    return st


class Densifier:
    """Statistics and the clone / split / prune / opacity-reset calls of
    the 3D-GS density control for n Gaussians."""

    def __init__(self, n, device="cuda"):
        self.device = device
        self.resize(n)

    def resize(self, n):
        self.n = int(n)
        self.accum = torch.zeros(max(self.n, 1), dtype=torch.float32, device=self.device)
        self.denom = torch.zeros(max(self.n, 1), dtype=torch.float32, device=self.device)
        self.action = torch.empty(max(self.n, 1), dtype=torch.int32, device=self.device)
        nb = _lib.load().gs_densify_workspace_bytes(self.n)
        self.ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=self.device)
        self.n_out = torch.zeros(1, dtype=torch.int64, device=self.device)

    def reset_stats(self, stream=None):
        s = stream or stream_handle()
        call("gs_zero", _ptr(self.accum), self.accum.numel() * 4, s)
        call("gs_zero", _ptr(self.denom), self.denom.numel() * 4, s)

    def stats(self, bufs: RasterBuffers, stream=None):
        call("gs_densify_stats", C.byref(bufs.views.struct), C.byref(bufs.tiling),
             C.byref(bufs.proj), _ptr(bufs.d_rec), self.n, _ptr(self.accum), _ptr(self.denom),
             stream or stream_handle())

    def select(self, params, m, v, grad_threshold, max_log_scale_clone, min_opacity_logit,
               max_log_scale, log_split, stream=None):
        """Actions on the device; returns the output count (synchronises)."""
        st = gaussian_state(params, m, v)
        call("gs_densify_select", C.byref(st), _ptr(self.accum), _ptr(self.denom),
             float(grad_threshold), float(max_log_scale_clone), float(min_opacity_logit),
             float(max_log_scale), float(log_split), _ptr(self.ws), self.ws.numel(),
             _ptr(self.action), _ptr(self.n_out), stream or stream_handle())
        return int(self.n_out.item())

    def apply(self, params, m, v, n_out, z, log_split, stream=None):
        """New (params, m, v) dicts of n_out Gaussians (after select)."""
        P = {k: torch.empty(t.shape[:-1] + (n_out,), dtype=torch.float32, device=self.device)
             for k, t in params.items()}
        M = {k: torch.empty_like(t) for k, t in P.items()} if m is not None else None
        V = {k: torch.empty_like(t) for k, t in P.items()} if v is not None else None
        sin = gaussian_state(params, m, v)
        sout = gaussian_state(P, M, V)
        call("gs_densify_apply", C.byref(sin), _ptr(self.action), _ptr(self.ws), _ptr(z),
             float(log_split), C.byref(sout), stream or stream_handle())
        return P, M, V

    @staticmethod
    def opacity_reset(params, m, v, max_opacity_logit, stream=None):
        st = gaussian_state(params, m, v)
        call("gs_opacity_reset", C.byref(st), float(max_opacity_logit), stream or stream_handle())
