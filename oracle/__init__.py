"""FP64 CPU oracle of one 3D Gaussian Splatting training step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library ``paper_2509_12138_amd`` and never imports it.

The heavy definitions (projection, per-pixel compositing and its analytic
backward, projection backward, tile binning + sort, masked L1 + D-SSIM, brute
force k-NN) are plain C in ``gs_oracle.c``; Adam, the initialisation MLP and
the adaptive density control are plain numpy below.  Everything is FP64,
except the density statistics and decisions, which are FP32 integers-by-
comparison (see that section).  Which passage each function
follows is stated in its docstring; the paper itself (Sec. II) delegates the
training step to the 3D-GS method it cites, so the oracle restates that
method's standard definitions.

Parity pins: every function here is pinned by a CPU test against closed
forms, finite differences, brute force or library routines; the MLP
(``mlp_*``) is pinned by finite differences and the zero-weight special case.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

C0 = 0.28209479177387814  # degree-0 SH basis constant 1/(2 sqrt(pi))


def build(force: bool = False) -> str:
    """Compile gs_oracle.c with gcc (FP64, OpenMP) into liboracle.so."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-Wall", "-Wno-misleading-indentation", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            lib.or_bin_sort.restype = ctypes.c_int64
            lib.or_max_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def max_threads() -> int:
    return int(_load().or_max_threads())


def camera_vector(cam):
    """(16 doubles R, t, fx, fy, cx, cy; znear; W; H) from a camera record."""
    v = np.concatenate([np.asarray(cam["R"], np.float64).ravel(),
                        np.asarray(cam["t"], np.float64).ravel(),
                        np.array([cam["fx"], cam["fy"], cam["cx"], cam["cy"]],
                                 np.float64)])
    return v, float(cam["znear"]), int(cam["width"]), int(cam["height"])


# --------------------------------------------------------------------------
# Projection (EWA splatting step of the 3D-GS method)
# --------------------------------------------------------------------------

def sh_degree_of(color):
    """Spherical-harmonic degree D of a colour array with 3 (D+1)^2 rows."""
    rows = np.shape(color)[0]
    D = int(round(np.sqrt(rows / 3.0))) - 1
    if D < 0 or D > SH_MAX or 3 * (D + 1) ** 2 != rows:
        raise ValueError(f"colour array has {rows} rows; expected 3 (D+1)^2, D <= {SH_MAX}")
    return D


SH_MAX = 3


def sh_basis(D, dirs):
    """Real spherical harmonics (Condon-Shortley phase, index l*l + l + m) of
    degree <= D at unit vectors dirs [p, 3]: returns Y [p, K] and the
    gradient of their Cartesian polynomials [p, K, 3], K = (D+1)^2."""
    lib = _load()
    d = np.ascontiguousarray(np.asarray(dirs, np.float64).reshape(-1, 3))
    K = (D + 1) ** 2
    Y = np.zeros((len(d), K)); G = np.zeros((len(d), K, 3))
    lib.or_sh_basis(ctypes.c_int(D), ctypes.c_int64(len(d)), _p(d), _p(Y), _p(G))
    return Y, G


def project(params, cam, tile=(16, 16)):
    """Project every Gaussian through one camera (3D-GS projection step).

    params: dict of planar SoA arrays mean [3,n], log_scale [3,n], quat [4,n],
    opacity_logit [n], color [3(D+1)^2, n] (spherical-harmonic coefficient k
    of channel c in row 3k + c; D = 0 is the plain colour).  Returns a dict
    of FP64 SoA outputs plus integer pixel/tile bboxes [4,n] (tx0, ty0, tx1,
    ty1), n_tiles and valid.
    """
    lib = _load()
    mean = _f64(params["mean"]); n = mean.shape[1]
    ls = _f64(params["log_scale"]); q = _f64(params["quat"])
    ol = _f64(params["opacity_logit"]); col = _f64(params["color"])
    D = sh_degree_of(col)
    cv, znear, W, H = camera_vector(cam)
    out = dict(mean2d=np.zeros((2, n)), conic=np.zeros((3, n)), depth=np.zeros(n),
               opacity=np.zeros(n), rgb=np.zeros((3, n)), cov2d=np.zeros((3, n)),
               pix_bbox=np.zeros((4, n), np.int32), tile_bbox=np.zeros((4, n), np.int32),
               n_tiles=np.zeros(n, np.int32), valid=np.zeros(n, np.int32))
    lib.or_project(ctypes.c_int64(n), _p(mean), _p(ls), _p(q), _p(ol), _p(col), ctypes.c_int(D),
                   _p(cv),
                   ctypes.c_double(znear), ctypes.c_int(W), ctypes.c_int(H),
                   ctypes.c_int(tile[0]), ctypes.c_int(tile[1]),
                   _p(out["mean2d"]), _p(out["conic"]), _p(out["depth"]), _p(out["opacity"]),
                   _p(out["rgb"]), _p(out["cov2d"]), _p(out["pix_bbox"]), _p(out["tile_bbox"]),
                   _p(out["n_tiles"]), _p(out["valid"]))
    return out


def _proj_arrays(proj):
    n = proj["depth"].shape[0]
    valid = proj["valid"] if "valid" in proj else (np.asarray(proj["n_tiles"]) > 0)
    valid = np.ascontiguousarray(valid, dtype=np.int32)
    tb = np.ascontiguousarray(proj["tile_bbox"], dtype=np.int32)
    if tb.shape == (n, 4) and n != 4:
        tb = np.ascontiguousarray(tb.T)
    return (n, _f64(proj["mean2d"]), _f64(proj["conic"]), _f64(proj["depth"]),
            _f64(proj["opacity"]), _f64(proj["rgb"]), tb, valid)


def render(proj, W, H, tile=(16, 16), bg=(0.0, 0.0, 0.0), window=None, band=1e-5,
           support=True):
    """Composite every pixel front to back (3D-GS rasteriser definition).

    proj holds SoA mean2d [2,n], conic [3,n], depth, opacity, rgb [3,n],
    tile_bbox [4,n] and valid (or n_tiles).  window = (x0, y0, x1, y1).
    Returns image [3,H,W], T_final, n_contrib, n_blended, ambiguous ([H,W],
    reasons 1-16); pixels outside the window are left zero.  ``ambiguity`` holds the reason
    bits of an ambiguous pixel: 1 power near 0, 2 alpha near 1/255, 4 alpha
    near 0.99, 8 transmittance near the cut-off, 16 near-equal depths, 32 a
    pair listed on the pixel's tile by an ambiguous decision before its last
    blended entry (only n_contrib, a list position, can differ there).
    ``band`` is the relative half-width of the alpha and cut-off guard bands
    (1e-5 for records given to both sides in the same FP32 values; wider
    where the other side computes its records itself, to the projection's
    own tolerance).  It only classifies pixels.  ``support`` lists a pair on
    the tiles that meet its widened support (``support_tiles``, the binning
    the method uses); False lists it on every tile of its bbox.  Images,
    T_final and n_blended do not depend on it.
    """
    lib = _load()
    n, m2, cn, dp, op, rgb, tb, valid = _proj_arrays(proj)
    x0, y0, x1, y1 = window if window is not None else (0, 0, W, H)
    img = np.zeros((3, H, W)); T = np.zeros((H, W)); nc = np.zeros((H, W), np.int32)
    nb = np.zeros((H, W), np.int32); amb = np.zeros((H, W), np.uint8)
    bgv = _f64(bg)
    lib.or_render(ctypes.c_int64(n), _p(m2), _p(cn), _p(dp), _p(op), _p(rgb), _p(tb), _p(valid),
                  W, H, tile[0], tile[1], _p(bgv), x0, y0, x1, y1, _p(img), _p(T), _p(nc),
                  _p(nb), _p(amb), ctypes.c_double(band), ctypes.c_int(1 if support else 0))
    # ``ambiguous`` covers what images, T_final and n_blended depend on
    return dict(image=img, T_final=T, n_contrib=nc, n_blended=nb,
                ambiguous=(amb & 31).astype(bool), ambiguity=amb)


def render_bwd(proj, W, H, d_image, tile=(16, 16), bg=(0.0, 0.0, 0.0), window=None,
               amb_bits=31, band=1e-5):
    """Analytic backward of ``render`` with all decisions held fixed.

    Returns per-Gaussian SoA gradients d_mean2d [2,n], d_conic [3,n],
    d_opacity [n], d_rgb [3,n] and abs_mass / amb_mass [9,n] (sum of absolute
    per-pixel contributions, all pixels / ambiguous pixels only; amb_bits
    selects which ambiguity reasons of ``render`` count) and term_mass [9,n]
    (the same sums over the magnitudes of the terms before they cancel inside
    dL/dalpha, a condition measure for FP32 comparisons).  ``band`` as in
    ``render``.
    """
    lib = _load()
    n, m2, cn, dp, op, rgb, tb, valid = _proj_arrays(proj)
    x0, y0, x1, y1 = window if window is not None else (0, 0, W, H)
    dI = _f64(d_image)
    out = dict(d_mean2d=np.zeros((2, n)), d_conic=np.zeros((3, n)), d_opacity=np.zeros(n),
               d_rgb=np.zeros((3, n)), abs_mass=np.zeros((9, n)), amb_mass=np.zeros((9, n)),
               term_mass=np.zeros((9, n)))
    bgv = _f64(bg)
    lib.or_render_bwd(ctypes.c_int64(n), _p(m2), _p(cn), _p(dp), _p(op), _p(rgb), _p(tb),
                      _p(valid), W, H, tile[0], tile[1], _p(bgv), x0, y0, x1, y1, _p(dI),
                      _p(out["d_mean2d"]), _p(out["d_conic"]), _p(out["d_opacity"]),
                      _p(out["d_rgb"]), _p(out["abs_mass"]), _p(out["amb_mass"]),
                      ctypes.c_int(amb_bits), _p(out["term_mass"]), ctypes.c_double(band))
    return out


def project_bwd(params, cam, grads2d, tile=(16, 16)):
    """Chain rule from the projected outputs back to the parameters."""
    lib = _load()
    mean = _f64(params["mean"]); n = mean.shape[1]
    ls = _f64(params["log_scale"]); q = _f64(params["quat"])
    ol = _f64(params["opacity_logit"]); col = _f64(params["color"])
    D = sh_degree_of(col)
    cv, znear, W, H = camera_vector(cam)
    g = dict(mean=np.zeros((3, n)), log_scale=np.zeros((3, n)), quat=np.zeros((4, n)),
             opacity_logit=np.zeros(n), color=np.zeros(col.shape))
    lib.or_project_bwd(ctypes.c_int64(n), _p(mean), _p(ls), _p(q), _p(ol), _p(col),
                       ctypes.c_int(D), _p(cv),
                       ctypes.c_double(znear), W, H, tile[0], tile[1],
                       _p(_f64(grads2d["d_mean2d"])), _p(_f64(grads2d["d_conic"])),
                       _p(_f64(grads2d["d_opacity"])), _p(_f64(grads2d["d_rgb"])),
                       _p(g["mean"]), _p(g["log_scale"]), _p(g["quat"]), _p(g["opacity_logit"]),
                       _p(g["color"]))
    return g


# --------------------------------------------------------------------------
# Binning + sort
# --------------------------------------------------------------------------

LIST_BAND = 2e-4   # relative band of the single-precision listing decisions


def support_tiles(mean2d, conic, opacity, tile_bbox, valid, tile=(16, 16), band=LIST_BAND):
    """Tiles of each pair's tile bbox that meet its widened support.

    SoA inputs mean2d [2,n], conic [3,n], opacity [n], tile_bbox [4,n] and
    valid [n].  A tile is listed when its pixel-centre rectangle meets
    {d : d^T conic d <= 2 ln(255 o) + 0.02 + 1e-5 M} (M bounds the terms of
    the quadratic form over the bbox): outside it no pixel centre passes the
    alpha >= 1/255 test.  Returns (mask, amb) uint64 [n]: bit (ty - ty0) *
    span + (tx - tx0) of mask is set for a listed tile (mask 0 for a bbox of
    more than 64 tiles, all listed), of amb for a decision within ``band``
    of the threshold.
    """
    lib = _load()
    n = np.asarray(opacity).shape[0]
    m2 = _f64(mean2d); cn = _f64(conic); op = _f64(opacity)
    tb = np.ascontiguousarray(tile_bbox, dtype=np.int32)
    va = np.ascontiguousarray(valid, dtype=np.int32)
    mask = np.zeros(n, np.uint64); amb = np.zeros(n, np.uint64)
    lib.or_support_tiles(ctypes.c_int64(n), _p(m2), _p(cn), _p(op), _p(tb), _p(va),
                         tile[0], tile[1], ctypes.c_double(band), _p(mask), _p(amb))
    return mask, amb


def sup_from_records(rec):
    """The listing inputs of pair-major FP32 records [m,12]: mean x, y, conic
    a, b, c and opacity, as FP64 [m,6]."""
    return np.ascontiguousarray(np.asarray(rec, np.float32)[:, 0:6], dtype=np.float64)


def bin_sort(tile_bbox, n_tiles, depth_f32, slot, tiles_x, tiles_per_slot, n_slots, sup=None,
             tile=(16, 16), band=LIST_BAND, details=False):
    """Emit (tile, depth) keys per pair and sort them stably (plain definition).

    tile_bbox [m,4] pair-major (tx0, ty0, tx1, ty1); depth_f32 float32 [m]
    (its raw bits form the low key word).  sup [m,6] (mean x, y, conic a, b,
    c, opacity; see ``sup_from_records``) lists each pair on the tiles of
    ``support_tiles``; None lists it on every bbox tile.  Returns keys u64,
    ids u32 and ranges u32 [n_slots*tiles_per_slot, 2]; with details=True
    also the entry count of every pair and whether any of its listing
    decisions is ambiguous (within ``band``).
    """
    lib = _load()
    tb = np.ascontiguousarray(tile_bbox, dtype=np.int32).reshape(-1, 4)
    m = tb.shape[0]
    nt = np.ascontiguousarray(n_tiles, dtype=np.int32)
    db = np.ascontiguousarray(np.asarray(depth_f32, dtype=np.float32).view(np.uint32))
    sl = np.ascontiguousarray(slot, dtype=np.int32)
    sp = None if sup is None else np.ascontiguousarray(sup, dtype=np.float64).reshape(-1, 6)
    count = np.zeros(max(m, 1), np.int32); amb = np.zeros(max(m, 1), np.uint8)
    args = (ctypes.c_int64(m), _p(tb), _p(nt), None if sp is None else _p(sp), tile[0], tile[1],
            ctypes.c_double(band), _p(db), _p(sl), tiles_x, tiles_per_slot, n_slots)
    total = int(lib.or_bin_sort(*args, ctypes.c_int64(-1), None, None, None, _p(count), _p(amb)))
    keys = np.zeros(max(total, 1), np.uint64); ids = np.zeros(max(total, 1), np.uint32)
    ranges = np.zeros((n_slots * tiles_per_slot, 2), np.uint32)
    got = lib.or_bin_sort(*args, ctypes.c_int64(total), _p(keys), _p(ids), _p(ranges), None, None)
    assert got == total
    if details:
        return keys[:total], ids[:total], ranges, count[:m], amb[:m].astype(bool)
    return keys[:total], ids[:total], ranges


# --------------------------------------------------------------------------
# Loss
# --------------------------------------------------------------------------

def loss(image, target, mask=None, lam=0.2):
    """Masked (1-lam) L1 + lam (1 - SSIM) of one [3,H,W] image and its gradient."""
    lib = _load()
    img = _f64(image); tgt = _f64(target)
    H, W = img.shape[1], img.shape[2]
    mk = _f64(mask) if mask is not None else None
    L = ctypes.c_double(); l1 = ctypes.c_double(); ss = ctypes.c_double()
    dI = np.zeros_like(img); smap = np.zeros_like(img)
    lib.or_loss(_p(img), _p(tgt), _p(mk), H, W, ctypes.c_double(lam), ctypes.byref(L),
                ctypes.byref(l1), ctypes.byref(ss), _p(dI), _p(smap))
    return dict(loss=L.value, l1=l1.value, ssim=ss.value, d_image=dI, ssim_map=smap)


def masked_psnr(image, target, mask=None):
    """Masked PSNR of one image [3,H,W] against its target, in dB (FP64).

    The paper reports reconstruction quality as PSNR (Sec. III, Tables II,
    V, VI) of images whose background is removed by a mask (Sec. II "Image
    Rendering and Masking").  Reading taken here: the rendered image is
    clamped to [0, 1] (the displayable range, peak value 1), the squared
    error is averaged over the three channels of the masked pixels only,
    and PSNR = 10 log10(1 / MSE).  An exact match gives +inf; an empty
    mask leaves the value undefined (NaN) and such a view is left out of a
    mean over views."""
    img = np.clip(np.asarray(image, np.float64), 0.0, 1.0)
    tgt = np.asarray(target, np.float64)
    m = np.ones(img.shape[1:], bool) if mask is None else np.asarray(mask) != 0
    count = 3 * int(m.sum())
    if count == 0:
        return float("nan")
    se = float(((img - tgt) ** 2)[:, m].sum())
    if se == 0.0:
        return float("inf")
    return 10.0 * np.log10(count / se)


# --------------------------------------------------------------------------
# Adam (dense, bias-corrected)
# --------------------------------------------------------------------------

def adam(param, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-15, visible=None):
    """One Adam step (Kingma & Ba, Alg. 1) in FP64; returns new (param, m, v).

    visible: optional boolean mask over the last axis (the Gaussians).  The
    sparse (visible-only) form of the 3D-GS optimiser updates only the
    Gaussians the step's views draw; the others keep parameter and both
    moments unchanged, while the step count (and so the bias correction)
    stays global."""
    p0 = np.asarray(param, np.float64); grad = np.asarray(grad, np.float64)
    m0 = np.asarray(m, np.float64); v0 = np.asarray(v, np.float64)
    m1 = beta1 * m0 + (1.0 - beta1) * grad
    v1 = beta2 * v0 + (1.0 - beta2) * grad * grad
    mhat = m1 / (1.0 - beta1 ** step)
    vhat = v1 / (1.0 - beta2 ** step)
    p1 = p0 - lr * mhat / (np.sqrt(vhat) + eps)
    if visible is None:
        return p1, m1, v1
    keep = ~np.asarray(visible, bool)
    return (np.where(keep, p0, p1), np.where(keep, m0, m1), np.where(keep, v0, v1))


# --------------------------------------------------------------------------
# k nearest neighbours
# --------------------------------------------------------------------------

def knn(points, k):
    """Brute-force k nearest other points of each point, sorted by (distance, index).

    points [3,n]; returns idx [n,k] int32 and dist [n,k] float64.
    """
    if not 1 <= k <= 64:
        raise ValueError("k must be in [1, 64]")
    lib = _load()
    pts = _f64(points); n = pts.shape[1]
    idx = np.zeros((n, k), np.int32); dist = np.zeros((n, k))
    lib.or_knn(ctypes.c_int64(n), _p(pts), k, _p(idx), _p(dist))
    return idx, dist


# --------------------------------------------------------------------------
# Initialisation MLP (plain numpy, FP64, optional bf16 rounding)
# --------------------------------------------------------------------------

def bf16_round(x):
    """Round FP64 values to the nearest bfloat16 (ties to even), returned as FP64."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def mlp_forward(x, W1, b1, W2, b2, W3, b3, quantize=True):
    """y = W3^T relu(W2^T relu(W1^T x + b1) + b2) + b3, row-major batches.

    x [n,96]; W1 [96,64], W2 [64,64], W3 [64,8]; biases FP32-valued.  With
    quantize, x, the weights and both hidden activations are rounded to bf16
    exactly where the GPU stores them in bf16.  Returns y and the cache.
    """
    q = bf16_round if quantize else (lambda a: np.asarray(a, np.float64))
    xq = q(x); W1q = q(W1); W2q = q(W2); W3q = q(W3)
    z1 = xq @ W1q + b1
    h1 = q(np.maximum(z1, 0.0))
    z2 = h1 @ W2q + b2
    h2 = q(np.maximum(z2, 0.0))
    y = h2 @ W3q + b3
    return y, dict(x=xq, W1=W1q, W2=W2q, W3=W3q, z1=z1, h1=h1, z2=z2, h2=h2)


def mlp_backward(cache, dy, quantize=False):
    """Gradients of the MLP for upstream dy [n,8] (ReLU derivative 0 at 0).

    With quantize, dy and the masked hidden gradients dZ2, dZ1 are rounded to
    bf16 where the GPU keeps them in bf16 (the products use the bf16 weights
    and activations of a quantised forward's cache)."""
    q = bf16_round if quantize else (lambda a: np.asarray(a, np.float64))
    dy = q(dy)
    dW3 = cache["h2"].T @ dy
    db3 = dy.sum(0)
    dh2 = dy @ cache["W3"].T
    dz2 = q(dh2 * (cache["z2"] > 0))
    dW2 = cache["h1"].T @ dz2
    db2 = dz2.sum(0)
    dh1 = dz2 @ cache["W2"].T
    dz1 = q(dh1 * (cache["z1"] > 0))
    dW1 = cache["x"].T @ dz1
    db1 = dz1.sum(0)
    dx = dz1 @ cache["W1"].T
    return dict(W1=dW1, b1=db1, W2=dW2, b2=db2, W3=dW3, b3=db3, x=dx)


# --------------------------------------------------------------------------
# Learned initialisation: features, targets, loss, apply (plain numpy, FP64)
#
# One Gaussian per isosurface point (Sec. II, "Isosurface Extraction"); the
# network reads the point's 16 nearest neighbours in its local frame and
# predicts the starting log-scale, rotation and opacity.  Rotations are
# converted with scipy.spatial.transform (a library routine).
# --------------------------------------------------------------------------

def local_frames(normals):
    """[n,3,3] world->local frames: rows x, y, z with z = unit normal,
    x = normalise(z x e), e the world axis least aligned with z (lowest
    index on ties), y = z x x."""
    nz = _f64(normals).T
    nz = nz / np.linalg.norm(nz, axis=1, keepdims=True)
    e = np.zeros_like(nz)
    e[np.arange(len(nz)), np.argmin(np.abs(nz), axis=1)] = 1.0   # argmin: first minimum
    xa = np.cross(nz, e)
    xa /= np.linalg.norm(xa, axis=1, keepdims=True)
    ya = np.cross(nz, xa)
    return np.stack([xa, ya, nz], axis=1)


def mlp_features(points, normals, idx, dist, quantize=True):
    """Features [n,96] and mean neighbour distance dbar [n].

    For neighbour k of point p (idx/dist [n,16] sorted, -1 = missing):
    x[6k:6k+3] = F (p_j - p) / dbar, x[6k+3:6k+6] = F n_j (zero if missing);
    dbar = mean distance over the present neighbours (1 if none)."""
    P = _f64(points).T
    N = _f64(normals).T
    idx = np.asarray(idx)
    dist = np.asarray(dist, np.float64)
    n, k = idx.shape
    F = local_frames(normals)
    present = idx >= 0
    cnt = present.sum(1)
    dbar = np.where(cnt > 0, np.where(present, dist, 0.0).sum(1) / np.maximum(cnt, 1), 1.0)
    x = np.zeros((n, 6 * k))
    for kk in range(k):
        j = idx[:, kk]
        ok = j >= 0
        js = np.where(ok, j, 0)
        off = (P[js] - P) / dbar[:, None]
        x[:, 6 * kk:6 * kk + 3] = np.where(ok[:, None], np.einsum("nab,nb->na", F, off), 0.0)
        x[:, 6 * kk + 3:6 * kk + 6] = np.where(ok[:, None], np.einsum("nab,nb->na", F, N[js]), 0.0)
    return (bf16_round(x) if quantize else x), dbar


def _rot_from_wxyz(q):
    from scipy.spatial.transform import Rotation
    q = np.asarray(q, np.float64)
    return Rotation.from_quat(np.column_stack([q[:, 1], q[:, 2], q[:, 3], q[:, 0]])).as_matrix()


def _wxyz_from_rot(R):
    from scipy.spatial.transform import Rotation
    xyzw = Rotation.from_matrix(R).as_quat()
    q = np.column_stack([xyzw[:, 3], xyzw[:, 0], xyzw[:, 1], xyzw[:, 2]])
    return q * np.where(q[:, :1] < 0, -1.0, 1.0)


def mlp_targets(log_scale, quat, opacity_logit, normals, dbar):
    """Targets [n,8] of fitted Gaussians: log-scale minus log dbar, the unit
    quaternion (w >= 0) of F R(quat), and the opacity logit."""
    F = local_frames(normals)
    Rg = _rot_from_wxyz(_f64(quat).T)
    t = np.zeros((len(dbar), 8))
    t[:, 0:3] = _f64(log_scale).T - np.log(dbar)[:, None]
    t[:, 3:7] = _wxyz_from_rot(F @ Rg)
    t[:, 7] = _f64(opacity_logit)
    return t


def mlp_apply(y, normals, dbar):
    """Initial Gaussians from outputs y [n,8]: log_scale [3,n] = log dbar +
    y[:,0:3], quat [4,n] = unit quaternion (w >= 0) of F^T R(y[:,3:7]),
    opacity_logit [n] = y[:,7]; the inverse of mlp_targets."""
    y = _f64(y)
    F = local_frames(normals)
    R = np.transpose(F, (0, 2, 1)) @ _rot_from_wxyz(y[:, 3:7])
    return dict(log_scale=(np.log(dbar)[:, None] + y[:, 0:3]).T.copy(),
                quat=_wxyz_from_rot(R).T.copy(), opacity_logit=y[:, 7].copy())


def mlp_loss(y, t):
    """Mean over points of the squared error of log-scale (3) and opacity
    logit plus 1 - |<q/|q|, q*>| for the rotation; returns (loss, dL/dy)."""
    y = _f64(y); t = _f64(t)
    n = len(y)
    d = np.zeros_like(y)
    r = y[:, [0, 1, 2, 7]] - t[:, [0, 1, 2, 7]]
    d[:, [0, 1, 2, 7]] = 2.0 * r / n
    q = y[:, 3:7]
    qn = np.linalg.norm(q, axis=1)
    qh = q / np.maximum(qn, 1e-300)[:, None]
    c = np.sum(qh * t[:, 3:7], axis=1)
    L = np.sum(r * r) + np.sum(1.0 - np.abs(c))
    # derivative of |c| through the normalisation q -> q/|q|
    d[:, 3:7] = -np.sign(c)[:, None] * (t[:, 3:7] - qh * c[:, None]) / qn[:, None] / n
    return L / n, d


# --------------------------------------------------------------------------
# Adaptive density control (clone / split / prune / opacity reset) of the
# 3D-GS method the partitions are trained with.  The statistics and the
# decisions are integers decided by FP32 values, so they are computed in
# FP32 with the device's operation order (one IEEE operation at a time);
# the new parameters are FP64.
# --------------------------------------------------------------------------

ACT_DROP, ACT_KEEP, ACT_CLONE, ACT_SPLIT = 0, 1, 2, 3


def densify_stats(d_rec, n_tiles, n, W, H, accum, denom):
    """Add one step's statistics: for every slot s (pairs s*n .. s*n+n-1 of
    a single-partition view set) and visible pair (n_tiles > 0), the norm of
    (dL/dx W/2, dL/dy H/2) (the gradient of the projected mean in normalised
    device coordinates) to accum and 1 to denom.  FP32 throughout."""
    f = np.float32
    d_rec = np.asarray(d_rec, f).reshape(-1, 9)
    n_tiles = np.asarray(n_tiles).reshape(-1)
    a = np.array(accum, f, copy=True)
    d = np.array(denom, f, copy=True)
    hw, hh = f(0.5 * W), f(0.5 * H)
    for s in range(len(n_tiles) // n):
        vis = n_tiles[s * n:(s + 1) * n] > 0
        gx = d_rec[s * n:(s + 1) * n, 0] * hw
        gy = d_rec[s * n:(s + 1) * n, 1] * hh
        norm = np.sqrt(gx * gx + gy * gy)
        a = np.where(vis, a + norm, a).astype(f)
        d = np.where(vis, d + f(1.0), d).astype(f)
    return a, d


def densify_select(log_scale, opacity_logit, accum, denom, grad_threshold, max_log_scale_clone,
                   min_opacity_logit, max_log_scale, log_split):
    """Action per Gaussian: dropped when faint (opacity logit below the
    threshold); cloned when its mean gradient norm accum / denom reaches the
    threshold (decided exactly, as accum >= threshold x denom)
    and its largest log-scale is at most max_log_scale_clone; split when
    the gradient reaches it and the Gaussian is larger; kept otherwise; an
    output whose largest log-scale exceeds max_log_scale is dropped (split
    children are log_split smaller).  Returns (action [n], n_out)."""
    f = np.float32
    ls = np.asarray(log_scale, f).max(axis=0)
    acc = np.asarray(accum, f)
    den = np.asarray(denom, f)
    # mean >= threshold decided exactly (FP64 products of FP32 values are exact)
    grow = (den > 0) & (acc.astype(np.float64) >= np.float64(f(grad_threshold)) * den.astype(np.float64))
    faint = np.asarray(opacity_logit, f) < f(min_opacity_logit)
    small = ls <= f(max_log_scale_clone)
    act = np.full(len(ls), ACT_KEEP, np.int32)
    act[grow & small] = ACT_CLONE
    act[grow & ~small] = ACT_SPLIT
    too_big = np.where(act == ACT_SPLIT, (ls - f(log_split)).astype(f), ls) > f(max_log_scale)
    act[too_big | faint] = ACT_DROP
    counts = np.select([act == ACT_KEEP, act == ACT_CLONE, act == ACT_SPLIT], [1, 2, 2], 0)
    return act, int(counts.sum())


def _rot_wxyz(q):
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q, axis=0, keepdims=True)
    w, x, y, z = q
    return np.stack([np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)]),
                     np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)]),
                     np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)])])


def densify_apply(params, m, v, action, z, log_split):
    """The new Gaussians in input order: kept ones with their moments; a
    clone as the original then a copy with zero moments; a split Gaussian
    as two children c = 0, 1 at mean + R(q) (exp(log_scale) * z[g, c]) with
    log-scale - log_split and zero moments.  params / m / v: dicts of planar
    [rows][n] arrays; z [n, 2, 3].  Returns (params, m, v) dicts, FP64."""
    names = ("mean", "log_scale", "quat", "opacity_logit", "color")
    P = {k: np.atleast_2d(np.asarray(params[k], np.float64)) for k in names}
    M = {k: np.atleast_2d(np.asarray(m[k], np.float64)) for k in names}
    Vv = {k: np.atleast_2d(np.asarray(v[k], np.float64)) for k in names}
    z = np.asarray(z, np.float64)
    outs = {k: [] for k in names}
    om = {k: [] for k in names}
    ov = {k: [] for k in names}
    R = _rot_wxyz(P["quat"])                      # [3, 3, n]
    s = np.exp(P["log_scale"])
    for g, a in enumerate(np.asarray(action)):
        if a == ACT_DROP:
            continue
        if a in (ACT_KEEP, ACT_CLONE):
            for c in range(1 if a == ACT_KEEP else 2):
                for k in names:
                    outs[k].append(P[k][:, g])
                    om[k].append(M[k][:, g] if c == 0 else np.zeros(len(M[k])))
                    ov[k].append(Vv[k][:, g] if c == 0 else np.zeros(len(Vv[k])))
            continue
        for c in range(2):
            child = {k: P[k][:, g].copy() for k in names}
            child["mean"] = P["mean"][:, g] + R[:, :, g] @ (s[:, g] * z[g, c])
            child["log_scale"] = P["log_scale"][:, g] - log_split
            for k in names:
                outs[k].append(child[k])
                om[k].append(np.zeros(len(M[k])))
                ov[k].append(np.zeros(len(Vv[k])))

    def stack(lst, rows):
        return np.stack(lst, axis=1) if lst else np.zeros((rows, 0))
    res = []
    for d in (outs, om, ov):
        r = {k: stack(d[k], len(P[k])) for k in names}
        r["opacity_logit"] = r["opacity_logit"][0]
        res.append(r)
    return tuple(res)


def opacity_reset(opacity_logit, max_opacity_logit):
    """Opacity clamp of the periodic reset: min(logit, threshold)."""
    return np.minimum(np.asarray(opacity_logit, np.float64), max_opacity_logit)
