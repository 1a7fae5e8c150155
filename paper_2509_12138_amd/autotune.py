"""Autotuner for the rasteriser plan: bin-tile shape, tile schedule and
backward chunk size, picked by timing real training steps on the workload.

The choice cannot change results: images do not depend on the tile shape
(the support bbox is a strict superset of the alpha >= 1/255 ellipse) and the
schedule, chunking and waves per tile only reorder or split work.  Results are cached in a JSON file
keyed by device, image size, slot count, Gaussian-count bucket and backward
mode.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np
import torch

# (tile, schedule, backward chunk, forward waves per tile, deterministic
# gradients); every tile shape here has a compiled rasteriser.  A fixed set
# of plans (the full-size parity tests run each); the tuner itself searches
# the plan space in stages (staged_search)
CANDIDATES = [
    ((16, 16), "lpt", 64, 4, True), ((16, 16), "lpt", 64, 4, False),
    ((16, 16), "lpt", 128, 4, True), ((16, 16), "lpt", 64, 2, True),
    ((16, 16), "lpt", 64, 1, False), ((16, 16), "persistent", 64, 1, True),
    ((16, 8), "lpt", 64, 2, True), ((8, 16), "lpt", 64, 2, True), ((8, 16), "lpt", 64, 1, False),
    ((8, 8), "lpt", 0, 1, True), ((16, 16), "lpt", 0, 4, True), ((32, 8), "lpt", 128, 4, True),
    ((8, 8), "lpt", 64, 1, False), ((8, 8), "lpt", 0, 1, False), ((16, 16), "lpt", 0, 4, False),
    # split forward (chunk items composited in parallel, joined per tile)
    ((8, 8), "lpt+split", 64, 1, False), ((8, 8), "lpt+split", 128, 1, False),
    ((16, 16), "lpt+split", 64, 1, False),
]


def normalize(plan):
    """Plans of older caches lack the trailing fields: fill the defaults."""
    tile, sched, chunk = plan[0], plan[1], plan[2]
    nw = plan[3] if len(plan) > 3 else 1
    det = bool(plan[4]) if len(plan) > 4 else False
    return (tuple(tile), sched, int(chunk), int(nw), det)

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "gsmi", "autotune.json")


def cache_key(width, height, n_slots, n_gauss, stored):
    dev = torch.cuda.get_device_properties(0)
    arch = getattr(dev, "gcnArchName", dev.name)
    return f"{arch}|{width}x{height}|S{n_slots}|N2^{int(math.log2(max(n_gauss, 1)))}|{'stored' if stored else 'recompute'}"


def load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(path, cache):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_plan(make_trainer, plan, views, steps=8, warmup=2):
    """Mean ms per training step of a trainer built with `plan`."""
    tile, sched, chunk, nw, det = normalize(plan)
    tr = make_trainer(tile)
    tr.bufs.set_schedule(sched, chunk=chunk, fwd_waves=nw, deterministic=det)
    tr.fit_capacity(views=views)
    for s in range(warmup):
        tr.step(views[s % len(views)])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        tr.step(views[(warmup + s) % len(views)])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    tr.check()
    del tr
    torch.cuda.empty_cache()
    return ms


TILES = [(16, 16), (8, 8), (16, 8), (8, 16), (32, 8), (32, 16), (16, 32)]
SCHEDULES = ["lpt", "default", "persistent", "lpt+split"]


def valid_waves(tile):
    """Forward waves per tile that divide the tile's pixels per lane."""
    px = tile[0] * tile[1] // 64
    return [w for w in (1, 2, 4) if px % w == 0]


def valid(plan):
    tile, sched, chunk, nw, det = plan
    if sched == "persistent" and nw > 1:
        return False                                   # the queue takes one wave per tile
    if sched.endswith("+split") and (chunk == 0 or nw != 1):
        return False                                   # split: chunked, joined by one wave
    return nw in valid_waves(tile)


def staged_search(measure, stored):
    """Coordinate search over the plan space: every tile shape with a
    representative plan (LPT order, 64-entry chunks, the most forward waves
    the shape allows, atomic sums), then, for the two fastest shapes, one
    parameter at a time from the best plan so far: schedule (LPT, XCD-aware,
    persistent, split forward), backward chunk (64, 128, whole tiles),
    forward waves, deterministic sums."""
    first = {}
    for tile in TILES:
        plan = (tile, "lpt", 64 if stored else 0, max(valid_waves(tile)), False)
        ms = measure(plan)
        if ms is not None:
            first[tile] = (ms, plan)
    for tile in sorted(first, key=lambda t: first[t][0])[:2]:
        best_ms, best = first[tile]
        axes = [lambda p, v: (p[0], v, p[2], 1 if v.endswith("+split") or v == "persistent"
                               else p[3], p[4]),
                lambda p, v: (p[0], p[1], v, p[3], p[4]),
                lambda p, v: (p[0], p[1], p[2], v, p[4]),
                lambda p, v: (p[0], p[1], p[2], p[3], v)]
        values = [SCHEDULES, [64, 128, 0] if stored else [0], valid_waves(tile), [False, True]]
        for axis, vals in zip(axes, values):
            for v in vals:
                plan = axis(best, v)
                if not valid(plan):
                    continue
                ms = measure(plan)
                if ms is not None and ms < best_ms:
                    best_ms, best = ms, plan


def tune(make_trainer, width, height, n_slots, n_gauss, stored=True, views=None,
         candidates=None, cache_path=DEFAULT_CACHE, force=False, log=None):
    """Return the fastest (tile, schedule, chunk, fwd_waves, deterministic)
    for this workload: the given candidate plans, or the staged search over
    the plan space (staged_search).

    make_trainer(tile) builds a fresh trainer (with .bufs, .step(view),
    .fit_capacity(views=...), .check()).  The choice is cached unless force.
    """
    key = cache_key(width, height, n_slots, n_gauss, stored)
    cache = load_cache(cache_path) if cache_path else {}
    if not force and key in cache:
        e = cache[key]
        return normalize((e["tile"], e["schedule"], e["chunk"], e.get("fwd_waves", 1),
                          e.get("deterministic", False))), e
    views = list(views if views is not None else range(8))
    results = []
    timed = {}

    def measure(plan):
        plan = normalize(plan)
        if not stored and plan[2]:
            return None                                # chunking needs stored state
        if plan not in timed:
            timed[plan] = time_plan(make_trainer, plan, views)
            results.append((timed[plan], plan))
            if log:
                log(f"autotune {plan}: {timed[plan]:.3f} ms/step")
        return timed[plan]

    if candidates is not None:
        for plan in candidates:
            measure(plan)
    else:
        staged_search(measure, stored)
    ms, best = min(results, key=lambda r: r[0])
    entry = dict(tile=list(best[0]), schedule=best[1], chunk=best[2], fwd_waves=best[3],
                 deterministic=best[4], ms_per_step=ms,
                 tried=[dict(tile=list(p[0]), schedule=p[1], chunk=p[2], fwd_waves=p[3],
                             deterministic=p[4], ms=m) for m, p in results])
    if cache_path:
        cache[key] = entry
        save_cache(cache_path, cache)
    return best, entry
