"""The allocation-free loss entry point (gs_loss_noalloc) against gs_loss
with a caller workspace, through the C ABI: two calls in a row, the second
on a smaller input (the shared scratch keeps the first call's partials),
and a request above the scratch's maximum rejected on the host."""
import ctypes as C

import numpy as np
import pytest

from _gpu_helpers import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _inputs(rng, S, H, W):
    tgt = rng.uniform(0, 1, (S, 3, H, W)).astype(np.float32)
    img = np.clip(tgt + rng.normal(0, 0.1, tgt.shape), -0.1, 1.1).astype(np.float32)
    mask = (rng.uniform(size=(S, H, W)) < 0.7).astype(np.uint8)
    mask[:, : H // 3, : W // 3] = 0                     # whole background tiles
    dev = lambda a: torch.as_tensor(a).cuda()
    return dev(img), dev(tgt), dev(mask)


def _run(lib, name, img, tgt, mask, lam, scale, ws=None):
    S, _, H, W = img.shape
    loss = torch.full((S,), float("nan"), device="cuda")
    dI = torch.full_like(img, float("nan"))
    status = torch.zeros(4, dtype=torch.int64, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda t: C.c_void_p(t.data_ptr())
    if ws is None:
        st = getattr(lib, name)(p(img), p(tgt), p(mask), S, H, W, lam, scale, p(loss), p(dI),
                                p(status), stream)
    else:
        st = getattr(lib, name)(p(img), p(tgt), p(mask), S, H, W, lam, scale, p(ws), ws.numel(),
                                p(loss), p(dI), p(status), stream)
    assert st == 0, lib.gs_last_error().decode()
    torch.cuda.synchronize()
    return loss.cpu().numpy(), dI.cpu().numpy(), status.cpu().numpy()


def test_noalloc_loss_equals_workspace_loss(gpu):
    lib = gpu.load()
    rng = np.random.default_rng(77)
    for (S, H, W, lam, scale) in [(3, 200, 333, 0.2, 0.25), (1, 72, 96, 0.5, 1.0)]:
        say("noalloc loss", S, H, W)
        img, tgt, mask = _inputs(rng, S, H, W)
        nbytes = lib.gs_loss_workspace_bytes(S, H, W)
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        ref_l, ref_d, ref_s = _run(lib, "gs_loss", img, tgt, mask, lam, scale, ws)
        got_l, got_d, got_s = _run(lib, "gs_loss_noalloc", img, tgt, mask, lam, scale)
        assert np.all(np.isfinite(ref_l)) and np.all(np.isfinite(ref_d))
        np.testing.assert_array_equal(got_l, ref_l)
        np.testing.assert_array_equal(got_d, ref_d)
        np.testing.assert_array_equal(got_s, ref_s)


def test_noalloc_loss_rejects_oversized_requests(gpu):
    lib = gpu.load()
    say("noalloc loss size limit")
    dummy = C.c_void_p(16)              # never dereferenced: the host check fails first
    st = lib.gs_loss_noalloc(dummy, dummy, None, 100, 1080, 1920, 0.2, 1.0, dummy, dummy, None,
                             None)
    assert st == -1
    assert "maximum" in lib.gs_last_error().decode()
