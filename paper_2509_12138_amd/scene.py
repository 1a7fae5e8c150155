"""Seeded synthetic inputs: isosurface fields, surface samples, orbital cameras.

This module only builds inputs.  It holds none of the training step's
arithmetic (projection, compositing, loss, optimiser); both the GPU library
and the CPU oracle consume what it produces.

Stand-ins for the paper's data (Sec. III: Kingsnake, Rayleigh-Taylor and
Richtmyer-Meshkov isosurface point clouds extracted with ParaView, Sec. II
"Isosurface Extraction"; orbital training views, Sec. II "Camera Setup"):

* ``field_sphere_sines``   f(x) = |x| - 0.5 + 0.05 sin6x sin6y sin6z, a
  bumpy sphere; surface points are jittered cell samples projected onto
  f = 0 by Newton steps.
* ``MixingInterface``      a Richtmyer-Meshkov-like mixing layer
  z = sum_k A_k sin(pi (m_k x + n_k y) + phi_k) (32 seeded modes,
  A_k ~ |k|^-1.5, sum A_k = 0.25) plus gradient-noise-perturbed droplets
  above and bubbles below the layer.
* ``orbit_cameras``        a Fibonacci-sphere orbit of V views at radius 2.5
  looking at the origin, horizontal field of view 50 degrees.
"""
from __future__ import annotations

import math

import numpy as np

# Same byte layout as gs_camera in include/gs.h (80 bytes).
CAMERA_DTYPE = np.dtype([
    ("R", np.float32, (9,)), ("t", np.float32, (3,)),
    ("fx", np.float32), ("fy", np.float32), ("cx", np.float32), ("cy", np.float32),
    ("znear", np.float32), ("width", np.int32), ("height", np.int32),
    ("reserved", np.int32),
])
assert CAMERA_DTYPE.itemsize == 80

SQRT_PI = math.sqrt(math.pi)


# --------------------------------------------------------------------------
# Cameras
# --------------------------------------------------------------------------

def look_at(center, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)):
    """World-to-camera (R, t) in OpenCV axes (x right, y down, z forward)."""
    c = np.asarray(center, np.float64)
    f = np.asarray(target, np.float64) - c
    f /= np.linalg.norm(f)
    u = np.asarray(up, np.float64)
    if abs(np.dot(f, u)) > 0.99:
        u = np.array([0.0, 1.0, 0.0])
    r = np.cross(f, u); r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    return R, -R @ c


def morton_order(points, bits=10):
    """Permutation that sorts points along a Z-order (Morton) curve of their
    positions quantised to 2^bits cells per axis over their bounding box
    (stable on equal codes).  Stored in this order, Gaussians that are close
    in space are close in memory: a view's visible set then covers whole
    wavefronts and cache lines, and a tile's list gathers neighbouring
    records."""
    p = np.asarray(points, np.float64)
    lo, hi = p.min(0), p.max(0)
    q = np.floor((p - lo) / np.maximum(hi - lo, 1e-30) * ((1 << bits) - 1) + 0.5)
    q = np.clip(q, 0, (1 << bits) - 1).astype(np.uint64)
    code = np.zeros(len(p), np.uint64)
    for b in range(bits):
        for a in range(3):
            code |= ((q[:, a] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + (2 - a))
    return np.argsort(code, kind="stable")


def orbit_cameras(n_views, width, height, fov_x_deg=50.0, radius=2.5, znear=0.2):
    """Fibonacci-sphere orbit: z_i = 1 - (2i+1)/V, golden-angle azimuth."""
    cams = np.zeros(n_views, CAMERA_DTYPE)
    golden = math.pi * (3.0 - math.sqrt(5.0))
    fx = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    for i in range(n_views):
        z = 1.0 - (2.0 * i + 1.0) / n_views
        rxy = math.sqrt(max(0.0, 1.0 - z * z))
        phi = golden * i
        c = radius * np.array([rxy * math.cos(phi), rxy * math.sin(phi), z])
        R, t = look_at(c)
        cams[i]["R"] = R.ravel(); cams[i]["t"] = t
        cams[i]["fx"] = fx; cams[i]["fy"] = fx
        cams[i]["cx"] = width / 2.0; cams[i]["cy"] = height / 2.0
        cams[i]["znear"] = znear
        cams[i]["width"] = width; cams[i]["height"] = height
    return cams


def camera_dict(cam):
    """Plain dict view of one camera record (for the oracle)."""
    return {k: cam[k] for k in CAMERA_DTYPE.names}


def single_camera(R, t, f, width, height, znear=0.2):
    cam = np.zeros(1, CAMERA_DTYPE)
    cam[0]["R"] = np.asarray(R, np.float32).ravel(); cam[0]["t"] = t
    cam[0]["fx"] = f; cam[0]["fy"] = f
    cam[0]["cx"] = width / 2.0; cam[0]["cy"] = height / 2.0
    cam[0]["znear"] = znear; cam[0]["width"] = width; cam[0]["height"] = height
    return cam


# --------------------------------------------------------------------------
# Fields
# --------------------------------------------------------------------------

def field_sphere_sines(p):
    """f(x) = |x| - 0.5 + 0.05 sin(6x) sin(6y) sin(6z) and its gradient; p [...,3]."""
    x, y, z = p[..., 0], p[..., 1], p[..., 2]
    r = np.sqrt(x * x + y * y + z * z)
    sx, sy, sz = np.sin(6 * x), np.sin(6 * y), np.sin(6 * z)
    cx, cy, cz = np.cos(6 * x), np.cos(6 * y), np.cos(6 * z)
    f = r - 0.5 + 0.05 * sx * sy * sz
    rs = np.maximum(r, 1e-12)
    g = np.stack([x / rs + 0.3 * cx * sy * sz,
                  y / rs + 0.3 * sx * cy * sz,
                  z / rs + 0.3 * sx * sy * cz], axis=-1)
    return f, g


# |grad f| <= 1 + 0.3 |(cos sin sin, sin cos sin, sin sin cos)| <= 1 + 0.3 sqrt(3)
field_sphere_sines.lipschitz = 1.0 + 0.3 * np.sqrt(3.0)


class GradientNoise3D:
    """Perlin-style gradient noise with a seeded permutation and seeded unit
    gradients (written from Perlin's description: lattice gradients, quintic
    fade, trilinear blend)."""

    def __init__(self, seed, size=256):
        rng = np.random.default_rng(seed)
        self.perm = np.concatenate([rng.permutation(size)] * 2)
        g = rng.normal(size=(size, 3))
        self.grads = g / np.linalg.norm(g, axis=1, keepdims=True)
        self.size = size

    def __call__(self, p):
        p = np.asarray(p, np.float64)
        i0 = np.floor(p).astype(np.int64)
        fr = p - i0
        i0 %= self.size
        u = fr * fr * fr * (fr * (fr * 6 - 15) + 10)
        out = 0.0
        for dx in (0, 1):
            for dy in (0, 1):
                for dz in (0, 1):
                    ix = (i0[..., 0] + dx) % self.size
                    iy = (i0[..., 1] + dy) % self.size
                    iz = (i0[..., 2] + dz) % self.size
                    h = self.perm[self.perm[self.perm[ix] + iy] + iz]
                    d = fr - np.array([dx, dy, dz], np.float64)
                    dot = np.sum(self.grads[h] * d, axis=-1)
                    wx = u[..., 0] if dx else 1 - u[..., 0]
                    wy = u[..., 1] if dy else 1 - u[..., 1]
                    wz = u[..., 2] if dz else 1 - u[..., 2]
                    out = out + wx * wy * wz * dot
        return out


class MixingInterface:
    """Richtmyer-Meshkov-like mixing layer plus perturbed droplets/bubbles.

    Height field h(x, y) = sum_k A_k sin(pi (m_k x + n_k y) + phi_k) over 32
    integer wave vectors (m, n) in [-8, 8]^2 \\ {0} drawn without replacement,
    A_k proportional to |(m, n)|^-1.5 scaled so sum A_k = 0.25.  24 spheres of
    radius U[0.04, 0.12] whose radius is modulated by gradient noise: half sit
    above the layer (droplets), half below (bubbles).  Points are sampled
    directly on each piece, so no grid search is needed; ``grid`` only sets
    the quoted resolution of the stand-in volume.
    """

    def __init__(self, seed=2, n_modes=32, n_drops=24, grid=512):
        rng = np.random.default_rng(seed)
        ks = np.array([(m, n) for m in range(-8, 9) for n in range(-8, 9) if (m, n) != (0, 0)])
        pick = rng.choice(len(ks), size=n_modes, replace=False)
        self.k = ks[pick].astype(np.float64)
        a = np.linalg.norm(self.k, axis=1) ** -1.5
        self.A = 0.25 * a / a.sum()
        self.phi = rng.uniform(0, 2 * math.pi, n_modes)
        self.noise = GradientNoise3D(seed + 17)
        self.drops = []
        for i in range(n_drops):
            r = rng.uniform(0.04, 0.12)
            xy = rng.uniform(-0.8, 0.8, 2)
            above = i % 2 == 0
            z0 = self.height(xy[None, :])[0] + (1 if above else -1) * (r + rng.uniform(0.05, 0.3))
            self.drops.append((np.array([xy[0], xy[1], z0]), r))
        self.grid = grid

    def height(self, xy):
        ph = math.pi * (xy @ self.k.T) + self.phi
        return np.sin(ph) @ self.A

    def height_grad(self, xy):
        ph = math.pi * (xy @ self.k.T) + self.phi
        c = np.cos(ph) * self.A
        return math.pi * (c @ self.k)

    def _radius(self, center, r, dirs):
        return r * (1.0 + 0.3 * self.noise(dirs * 2.0 + center * 7.0))

    def sample(self, n, seed):
        """n surface points and unit normals, area-weighted across the pieces."""
        rng = np.random.default_rng(seed)
        area_layer = 4.0 * 1.3
        areas = np.array([area_layer] + [4 * math.pi * r * r for _, r in self.drops])
        counts = rng.multinomial(n, areas / areas.sum())
        pts, nrm = [], []
        xy = rng.uniform(-1, 1, (counts[0], 2))
        z = self.height(xy)
        g = self.height_grad(xy)
        nl = np.stack([-g[:, 0], -g[:, 1], np.ones(len(xy))], axis=1)
        nl /= np.linalg.norm(nl, axis=1, keepdims=True)
        pts.append(np.column_stack([xy, z])); nrm.append(nl)
        for (c, r), cnt in zip(self.drops, counts[1:]):
            if cnt == 0:
                continue
            d = rng.normal(size=(cnt, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
            rad = self._radius(c, r, d)
            p = c + d * rad[:, None]
            # normal of the radially perturbed sphere by central differences
            eps = 1e-4
            t1 = np.cross(d, np.where(np.abs(d[:, :1]) < 0.9, [[1.0, 0, 0]], [[0, 1.0, 0]]))
            t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
            t2 = np.cross(d, t1)
            def at(dd):
                dd = dd / np.linalg.norm(dd, axis=1, keepdims=True)
                return c + dd * self._radius(c, r, dd)[:, None]
            e1 = at(d + eps * t1) - at(d - eps * t1)
            e2 = at(d + eps * t2) - at(d - eps * t2)
            nn = np.cross(e1, e2); nn /= np.linalg.norm(nn, axis=1, keepdims=True)
            nn *= np.sign(np.sum(nn * d, axis=1, keepdims=True))
            pts.append(p); nrm.append(nn)
        return np.concatenate(pts).astype(np.float64), np.concatenate(nrm).astype(np.float64)


# --------------------------------------------------------------------------
# Surface sampling of an implicit field
# --------------------------------------------------------------------------

def candidate_cells(field, grid, lo=-1.0, hi=1.0, box=None, block=16):
    """Integer (i, j, k) of grid cells whose 8 corner values straddle zero,
    sorted by (k, i, j).

    box = (lo3, hi3) restricts the search to cells inside an axis-aligned box.
    A field with a ``lipschitz`` attribute (a bound on |grad f|) is screened
    block by block first: a block of block^3 cells whose centre value exceeds
    the bound times its half-diagonal has one sign throughout and holds no
    straddling cell, so only blocks near the surface have their corners
    evaluated (same corner coordinates, same cells as the full sweep).
    Otherwise the volume is swept in z slabs so large grids fit in memory.
    """
    h = (hi - lo) / grid
    if box is None:
        kmin = np.zeros(3, np.int64); kmax = np.full(3, grid, np.int64)
    else:
        kmin = np.clip(np.floor((np.asarray(box[0]) - lo) / h).astype(np.int64), 0, grid)
        kmax = np.clip(np.ceil((np.asarray(box[1]) - lo) / h).astype(np.int64), 0, grid)
    lip = getattr(field, "lipschitz", None)
    if lip is not None and block > 1:
        return _candidate_cells_screened(field, lip, lo, h, kmin, kmax, block), h
    xs = lo + h * np.arange(kmin[0], kmax[0] + 1)
    ys = lo + h * np.arange(kmin[1], kmax[1] + 1)
    out = []
    prev = None
    for kz in range(kmin[2], kmax[2] + 1):
        z = lo + h * kz
        X, Y = np.meshgrid(xs, ys, indexing="ij")
        P = np.stack([X, Y, np.full_like(X, z)], axis=-1)
        f, _ = field(P)
        s = f > 0
        if prev is not None:
            c8 = np.stack([prev[:-1, :-1], prev[1:, :-1], prev[:-1, 1:], prev[1:, 1:],
                           s[:-1, :-1], s[1:, :-1], s[:-1, 1:], s[1:, 1:]])
            mixed = c8.any(0) & ~c8.all(0)
            ii, jj = np.nonzero(mixed)
            if len(ii):
                out.append(np.column_stack([ii + kmin[0], jj + kmin[1],
                                            np.full(len(ii), kz - 1)]))
        prev = s
    return np.concatenate(out) if out else np.zeros((0, 3), np.int64), h


def _candidate_cells_screened(field, lip, lo, h, kmin, kmax, block):
    edges = [np.append(np.arange(kmin[a], kmax[a], block), kmax[a]) for a in range(3)]
    b0 = np.meshgrid(*[e[:-1] for e in edges], indexing="ij")
    b1 = np.meshgrid(*[e[1:] for e in edges], indexing="ij")
    b0 = np.stack([b.ravel() for b in b0], -1)
    b1 = np.stack([b.ravel() for b in b1], -1)
    centre = lo + h * 0.5 * (b0 + b1)
    half_diag = 0.5 * h * np.sqrt(np.sum((b1 - b0).astype(np.float64) ** 2, axis=1))
    fc, _ = field(centre)
    near = np.abs(fc) <= lip * half_diag * (1 + 1e-6) + 1e-12
    out = []
    for k0, k1 in zip(b0[near], b1[near]):
        ax = [lo + h * np.arange(k0[a], k1[a] + 1) for a in range(3)]
        P = np.stack(np.meshgrid(*ax, indexing="ij"), axis=-1)
        s = field(P)[0] > 0
        c8 = np.stack([s[:-1, :-1, :-1], s[1:, :-1, :-1], s[:-1, 1:, :-1], s[1:, 1:, :-1],
                       s[:-1, :-1, 1:], s[1:, :-1, 1:], s[:-1, 1:, 1:], s[1:, 1:, 1:]])
        ii, jj, kk = np.nonzero(c8.any(0) & ~c8.all(0))
        if len(ii):
            out.append(np.column_stack([ii + k0[0], jj + k0[1], kk + k0[2]]))
    if not out:
        return np.zeros((0, 3), np.int64)
    cells = np.concatenate(out).astype(np.int64)
    return cells[np.lexsort((cells[:, 1], cells[:, 0], cells[:, 2]))]


def sample_surface(field, n, grid, seed, lo=-1.0, hi=1.0, box=None, newton=3, tol=1e-6):
    """n jittered points on f = 0: uniform cell choice among straddling cells,
    uniform point in the cell, ``newton`` steps x <- x - f grad/|grad|^2;
    points with |f| > tol afterwards (or leaving the box) are redrawn."""
    rng = np.random.default_rng(seed)
    cells, h = candidate_cells(field, grid, lo, hi, box)
    pts = np.zeros((0, 3))
    while len(pts) < n:
        need = n - len(pts)
        pick = cells[rng.integers(0, len(cells), size=int(need * 1.1) + 16)]
        p = lo + h * (pick + rng.uniform(0, 1, (len(pick), 3)))
        for _ in range(newton):
            f, g = field(p)
            p = p - (f / np.maximum(np.sum(g * g, -1), 1e-20))[:, None] * g
        f, _ = field(p)
        ok = np.abs(f) <= tol
        if box is not None:
            ok &= np.all((p >= np.asarray(box[0])) & (p <= np.asarray(box[1])), axis=1)
        pts = np.concatenate([pts, p[ok]])
    pts = pts[:n]
    _, g = field(pts)
    nrm = g / np.linalg.norm(g, axis=1, keepdims=True)
    return pts, nrm


# --------------------------------------------------------------------------
# Gaussians built from surface samples
# --------------------------------------------------------------------------

def quat_z_to(normals):
    """Unit quaternions (w, x, y, z) rotating +z onto each unit normal."""
    nz = np.asarray(normals, np.float64)
    z = np.array([0.0, 0.0, 1.0])
    axis = np.cross(np.broadcast_to(z, nz.shape), nz)
    s = np.linalg.norm(axis, axis=1)
    c = nz[:, 2]
    ang = np.arctan2(s, c)
    axis = np.where(s[:, None] > 1e-12, axis / np.maximum(s, 1e-12)[:, None], [[1.0, 0, 0]])
    return np.column_stack([np.cos(ang / 2), axis * np.sin(ang / 2)[:, None]])


def knn_mean_distance(points, k=3):
    """Mean distance of each point to its k nearest other points (SciPy kd-tree;
    input preparation only)."""
    from scipy.spatial import cKDTree
    tree = cKDTree(points)
    d, _ = tree.query(points, k=k + 1, workers=-1)
    return d[:, 1:].mean(1)


def gaussians_from_points(points, normals, scale, opacity=0.1, thin=None):
    """Planar SoA float32 Gaussian parameters centred at surface points.

    scale: per-point isotropic scale (thin: optional factor for the axis along
    the normal, which then becomes a disc aligned with the surface).  Colour
    is the SH degree-0 coefficient whose rendered colour is (n + 1)/2.
    """
    n = len(points)
    sc = np.asarray(scale, np.float64).reshape(-1)
    ls = np.tile(np.log(sc), (3, 1))
    if thin is not None:
        ls[2] += math.log(thin)
        quat = quat_z_to(normals).T
    else:
        quat = np.tile(np.array([[1.0], [0.0], [0.0], [0.0]]), (1, n))
    logit = math.log(opacity / (1.0 - opacity))
    return dict(
        mean=np.ascontiguousarray(points.T, np.float32),
        log_scale=np.ascontiguousarray(ls, np.float32),
        quat=np.ascontiguousarray(quat, np.float32),
        opacity_logit=np.full(n, logit, np.float32),
        color=np.ascontiguousarray((normals * SQRT_PI).T, np.float32),
    )


def random_gaussians(n, seed, center=(0.0, 0.0, 0.0), extent=0.6, log_scale=(-4.0, -2.5),
                     opacity=(0.05, 0.95)):
    """Seeded random anisotropic Gaussians in a cube (parity-test inputs)."""
    rng = np.random.default_rng(seed)
    mean = (np.asarray(center)[:, None] + rng.uniform(-extent, extent, (3, n)))
    ls = rng.uniform(log_scale[0], log_scale[1], (3, n))
    q = rng.normal(size=(4, n))
    op = rng.uniform(opacity[0], opacity[1], n)
    return dict(
        mean=mean.astype(np.float32), log_scale=ls.astype(np.float32),
        quat=q.astype(np.float32),
        opacity_logit=np.log(op / (1 - op)).astype(np.float32),
        color=rng.normal(0, 1.2, (3, n)).astype(np.float32),
    )


def concat_params(parts):
    """Concatenate several planar SoA parameter dicts along the Gaussian axis."""
    return {k: np.ascontiguousarray(np.concatenate([p[k] for p in parts], axis=-1))
            for k in parts[0]}


def take_params(params, idx):
    return {k: np.ascontiguousarray(v[..., idx]) for k, v in params.items()}


def views_table(counts, views_per_part):
    """Slot table of a batch: partition p (counts[p] Gaussians, stored
    contiguously) seen from views_per_part views.  Returns (pair_offset
    [S+1], gauss_offset [S]) int64 with slot s = p * views_per_part + j."""
    counts = list(counts)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int64)
    sizes, goff = [], []
    for p, c in enumerate(counts):
        for _ in range(views_per_part):
            sizes.append(c); goff.append(starts[p])
    po = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return po, np.asarray(goff, np.int64)
