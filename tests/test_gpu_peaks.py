"""The unit microbenchmarks run through the C ABI and give plausible rates
(a short run; the measured peaks themselves come from
``python -m paper_2509_12138_amd.peaks``)."""
import pytest

from _gpu_helpers import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_peaks_short_run(gpu):
    say("peaks, short run")
    from paper_2509_12138_amd import peaks
    r = peaks.measure(copy_bytes=64 << 20, blocks=1024, iters=256)
    say(r)
    assert 0.5 < r["hbm_copy_TBps"] < 12.0
    assert r["fp32_fma_T_lane_ops"] > 2.0 and r["exp_T_per_s"] > 0.5
    assert r["lds_TBps"] > 2.0 and r["bf16_mfma_TFLOPs"] > 50.0
    assert r["atomic_scattered_4MB_G_per_s"] > 1.0 and r["atomic_contiguous_36MB_G_per_s"] > 1.0
