"""Measured peaks of the MI355X units the rooflines price.

Runs the library's microbenchmarks (gs_peak_*) on the current device and
stream, times each launch with events (median of several, after a warm-up)
and prints one JSON object: HBM copy bandwidth, FP32 FMA and exponential
issue rates (plain, not packed), LDS read bandwidth, FP32 global atomics
into an L2-sized and a 36 MB array, and BF16 matrix-core flops.

    python -m paper_2509_12138_amd.peaks
"""
from __future__ import annotations

import ctypes as C
import json
import sys

import torch

from . import _lib
from ._lib import call

CUS = 256
CLOCK_HZ = 2.4e9


def _timed(fn, reps=5):
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    fn(s)                                   # warm-up (loads the kernel)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn(s)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    times.sort()
    return times[len(times) // 2]


def measure(copy_bytes=1 << 30, blocks=CUS * 16, iters=4096):
    _lib.load()
    dev = "cuda"
    out = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    res = {}
    a = torch.empty(copy_bytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    t = _timed(lambda s: call("gs_peak_copy", C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()),
                              copy_bytes, s))
    res["hbm_copy_TBps"] = 2 * copy_bytes / t / 1e12
    # the same copy by the runtime's own device copy, for comparison
    t = _timed(lambda s: b.copy_(a))
    res["hbm_runtime_copy_TBps"] = 2 * copy_bytes / t / 1e12
    del a, b
    lanes = blocks * 256
    t = _timed(lambda s: call("gs_peak_fma", C.c_void_p(out.data_ptr()), blocks, iters, s))
    res["fp32_fma_T_lane_ops"] = lanes * iters * 16 / t / 1e12
    t = _timed(lambda s: call("gs_peak_exp", C.c_void_p(out.data_ptr()), blocks, iters // 4, s))
    res["exp_T_per_s"] = lanes * (iters // 4) * 16 / t / 1e12
    t = _timed(lambda s: call("gs_peak_lds", C.c_void_p(out.data_ptr()), blocks, iters // 4, s))
    lds = lanes * (iters // 4) * 4 * 16 / t
    res["lds_TBps"] = lds / 1e12
    res["lds_B_per_clk_per_CU"] = lds / (CUS * CLOCK_HZ)
    for name, n_addr, contiguous in (("atomic_scattered_4MB_G_per_s", 1 << 20, 0),
                                     ("atomic_scattered_36MB_G_per_s", 9 << 20, 0),
                                     ("atomic_contiguous_36MB_G_per_s", 9 << 20, 1)):
        dst = torch.zeros(n_addr, dtype=torch.float32, device=dev)
        it = 64
        t = _timed(lambda s: call("gs_peak_atomic", C.c_void_p(dst.data_ptr()), n_addr, blocks,
                                  it, contiguous, s))
        res[name] = lanes * it / t / 1e9
        del dst
    t = _timed(lambda s: call("gs_peak_mfma", C.c_void_p(out.data_ptr()), blocks, iters // 4, s))
    res["bf16_mfma_TFLOPs"] = blocks * 4 * (iters // 4) * 8 * 16384 / t / 1e12
    res["published"] = dict(hbm_TBps=8.0, fp32_fma_T_lane_ops_plain=39.3, bf16_TFLOPs=2500.0)
    return res


def main():
    if not torch.cuda.is_available():
        sys.exit("peaks needs a GPU")
    print(json.dumps(measure()), flush=True)


if __name__ == "__main__":
    main()
