"""Seeded synthetic inputs: Gaussian scenes, pinhole cameras and target images.

This module only draws random numbers and builds camera poses.  It holds none of
the rasterizer's arithmetic, so both the HIP path and the CPU reference can take
their inputs from it.

Scene layout (structure of arrays, float32, component-major):
    mean          [3][N]   world position
    log_scale     [3][N]   log of the per-axis scale
    quat          [4][N]   rotation quaternion (w, x, y, z), not normalised
    opacity_logit [N]      opacity before the sigmoid
    sh            [16][3][N]  degree-3 SH colour coefficients (coefficient, channel)
    lod           [N] uint8   level-of-detail label (finest-level index)

The paper trains on aerial captures of cities (Mill-19, UrbanScene3D,
MatrixCity).  Those datasets are not available here; the "city" generator below
stands in for their scale and structure: a 1 km x 1 km ground plane with
box-shaped buildings whose facades and roofs carry half of the Gaussians.

Camera convention: world-to-camera rotation R (row-major 3x3, rows = camera
right, down and forward axes) and translation t, so x_cam = R x_world + t.
Pixel (u, v) samples the image plane at (u + 0.5, v + 0.5).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SH_COEFFS = 16  # degree 3


@dataclasses.dataclass
class Scene:
    mean: np.ndarray
    log_scale: np.ndarray
    quat: np.ndarray
    opacity_logit: np.ndarray
    sh: np.ndarray
    lod: np.ndarray

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    def arrays(self):
        return dict(mean=self.mean, log_scale=self.log_scale, quat=self.quat,
                    opacity_logit=self.opacity_logit, sh=self.sh, lod=self.lod)

    def subset(self, idx: np.ndarray) -> "Scene":
        idx = np.asarray(idx)
        return Scene(mean=np.ascontiguousarray(self.mean[:, idx]),
                     log_scale=np.ascontiguousarray(self.log_scale[:, idx]),
                     quat=np.ascontiguousarray(self.quat[:, idx]),
                     opacity_logit=np.ascontiguousarray(self.opacity_logit[idx]),
                     sh=np.ascontiguousarray(self.sh[:, :, idx]),
                     lod=np.ascontiguousarray(self.lod[idx]))


    def spatially_ordered(self) -> "Scene":
        """The same Gaussians in Morton order of their means (see
        morton_order): Gaussians close in space are close in memory, so a
        view's visible set covers few, long index ranges."""
        return self.subset(morton_order(self.mean))


def _spread_bits3(v: np.ndarray) -> np.ndarray:
    """Moves bit k of a 21-bit integer to bit 3k."""
    v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
    return v


def morton_order(mean: np.ndarray, bits: int = 21) -> np.ndarray:
    """Permutation sorting points [3][N] by the Morton (Z-order) code of their
    coordinates quantised to 2^bits cells per axis over the bounding box;
    equal codes keep their index order."""
    mean = np.asarray(mean, dtype=np.float64)
    if mean.shape[1] == 0:
        return np.zeros(0, dtype=np.int64)
    lo = mean.min(axis=1, keepdims=True)
    span = np.maximum(mean.max(axis=1, keepdims=True) - lo, 1e-12)
    top = (1 << bits) - 1
    q = np.clip(np.floor((mean - lo) / span * top), 0, top).astype(np.uint64)
    code = _spread_bits3(q[0]) | (_spread_bits3(q[1]) << np.uint64(1)) | (_spread_bits3(q[2]) << np.uint64(2))
    return np.argsort(code, kind="stable")


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray          # (3, 3) float64, world -> camera
    t: np.ndarray          # (3,) float64
    znear: float = 0.2

    @property
    def position(self) -> np.ndarray:
        return -self.R.T @ self.t

    @property
    def n_pixels(self) -> int:
        return self.width * self.height


def _finish(mean, log_scale, quat, opacity_logit, sh, lod_levels=8) -> Scene:
    mean = np.ascontiguousarray(mean, dtype=np.float32)
    log_scale = np.ascontiguousarray(log_scale, dtype=np.float32)
    # Level-of-detail labels for synthetic scenes: octaves of the largest scale
    # below a reference scale (the 90th percentile), finer levels for smaller
    # Gaussians.  This is an input of the LOD gate, not part of its arithmetic.
    smax = np.exp(log_scale.astype(np.float64).max(axis=0))
    s_ref = np.percentile(smax, 90.0) if smax.size else 1.0
    lvl = np.floor(np.log2(s_ref / smax) + 0.5)
    lod = np.clip(lvl, 0, lod_levels - 1).astype(np.uint8)
    return Scene(mean=mean, log_scale=log_scale,
                 quat=np.ascontiguousarray(quat, dtype=np.float32),
                 opacity_logit=np.ascontiguousarray(opacity_logit, dtype=np.float32),
                 sh=np.ascontiguousarray(sh, dtype=np.float32), lod=lod)


def _quats(rng, n):
    return rng.standard_normal((4, n))


def cube_scene(n: int = 4096, seed: int = 0, log_scale_mu: float = -3.0,
               log_scale_sigma: float = 0.5) -> Scene:
    """Means uniform in [-1,1]^3, log-scales ~N(-3, 0.5), random quaternions,
    opacity logits ~N(0,1), SH coefficients ~N(0, 0.2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mean = rng.uniform(-1.0, 1.0, (3, n))
    log_scale = rng.normal(log_scale_mu, log_scale_sigma, (3, n))
    quat = _quats(rng, n)
    opacity_logit = rng.normal(0.0, 1.0, n)
    sh = rng.normal(0.0, 0.2, (SH_COEFFS, 3, n))
    return _finish(mean, log_scale, quat, opacity_logit, sh)


def city_scene(n: int, seed: int = 2, extent: float = 500.0, grid: float = 40.0,
               p_building: float = 0.6, chunk: int = 1 << 21) -> Scene:
    """Synthetic aerial city of n Gaussians on a (2*extent)^2 m ground plane.

    Buildings sit on a `grid` m lattice, each cell occupied with probability
    p_building, footprint U(10,30) m per side, height U(5,80) m.  Half of the
    Gaussians lie area-uniformly on the ground outside the footprints, half
    area-uniformly on the facades and roofs.  Log-scales ~N(ln 0.3, 0.7),
    uniform rotations, opacity logits ~N(0, 1.5), SH ~N(0, 0.2).  Up is +z.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    cells = int(round(2 * extent / grid))
    occ = rng.random((cells, cells)) < p_building
    gx, gy = np.nonzero(occ)
    nb = gx.size
    w = rng.uniform(10.0, 30.0, nb)
    d = rng.uniform(10.0, 30.0, nb)
    h = rng.uniform(5.0, 80.0, nb)
    x0 = -extent + gx * grid + rng.uniform(0.0, 1.0, nb) * (grid - w)
    y0 = -extent + gy * grid + rng.uniform(0.0, 1.0, nb) * (grid - d)

    n_ground = n // 2
    n_bld = n - n_ground
    mean = np.empty((3, n), dtype=np.float64)

    # Ground: rejection sampling against the footprints via the cell lattice.
    filled = 0
    while filled < n_ground:
        m = min(chunk, 2 * (n_ground - filled) + 1024)
        px = rng.uniform(-extent, extent, m)
        py = rng.uniform(-extent, extent, m)
        cx = np.clip(((px + extent) // grid).astype(np.int64), 0, cells - 1)
        cy = np.clip(((py + extent) // grid).astype(np.int64), 0, cells - 1)
        bid = np.full((cells, cells), -1, dtype=np.int64)
        bid[gx, gy] = np.arange(nb)
        b = bid[cx, cy]
        inside = np.zeros(m, dtype=bool)
        has = b >= 0
        bb = b[has]
        inside[has] = ((px[has] >= x0[bb]) & (px[has] <= x0[bb] + w[bb]) &
                       (py[has] >= y0[bb]) & (py[has] <= y0[bb] + d[bb]))
        keep = np.nonzero(~inside)[0][: n_ground - filled]
        mean[0, filled:filled + keep.size] = px[keep]
        mean[1, filled:filled + keep.size] = py[keep]
        mean[2, filled:filled + keep.size] = 0.0
        filled += keep.size

    # Facades (4 per building) and roofs, chosen with probability ∝ area.
    areas = np.stack([w * h, w * h, d * h, d * h, w * d], axis=1).reshape(-1)
    cdf = np.cumsum(areas)
    cdf /= cdf[-1]
    face = np.searchsorted(cdf, rng.random(n_bld), side="right")
    face = np.minimum(face, areas.size - 1)
    b = face // 5
    kind = face % 5
    u = rng.random(n_bld)
    v = rng.random(n_bld)
    bx = np.empty(n_bld)
    by = np.empty(n_bld)
    bz = np.empty(n_bld)
    k0 = kind == 0  # south facade, y = y0
    k1 = kind == 1  # north facade, y = y0 + d
    k2 = kind == 2  # west facade, x = x0
    k3 = kind == 3  # east facade, x = x0 + w
    k4 = kind == 4  # roof, z = h
    bx[k0 | k1] = x0[b[k0 | k1]] + u[k0 | k1] * w[b[k0 | k1]]
    by[k0] = y0[b[k0]]
    by[k1] = y0[b[k1]] + d[b[k1]]
    bx[k2] = x0[b[k2]]
    bx[k3] = x0[b[k3]] + w[b[k3]]
    by[k2 | k3] = y0[b[k2 | k3]] + u[k2 | k3] * d[b[k2 | k3]]
    bz[~k4] = v[~k4] * h[b[~k4]]
    bx[k4] = x0[b[k4]] + u[k4] * w[b[k4]]
    by[k4] = y0[b[k4]] + v[k4] * d[b[k4]]
    bz[k4] = h[b[k4]]
    mean[0, n_ground:] = bx
    mean[1, n_ground:] = by
    mean[2, n_ground:] = bz

    # Shuffle so ground and building Gaussians interleave in index order.
    perm = rng.permutation(n)
    mean = mean[:, perm]
    log_scale = rng.normal(math.log(0.3), 0.7, (3, n))
    quat = _quats(rng, n)
    opacity_logit = rng.normal(0.0, 1.5, n)
    sh = rng.normal(0.0, 0.2, (SH_COEFFS, 3, n)).astype(np.float32)
    return _finish(mean, log_scale, quat, opacity_logit, sh)


def camera_from_rt(width, height, fx, fy, R, t, cx=None, cy=None, znear=0.2) -> Camera:
    return Camera(width=int(width), height=int(height), fx=float(fx), fy=float(fy),
                  cx=float(width) / 2 if cx is None else float(cx),
                  cy=float(height) / 2 if cy is None else float(cy),
                  R=np.asarray(R, dtype=np.float64).reshape(3, 3),
                  t=np.asarray(t, dtype=np.float64).reshape(3), znear=float(znear))


def look_at(position, target, width, height, hfov_deg=60.0, up=(0.0, 0.0, 1.0),
            znear=0.2) -> Camera:
    """Camera at `position` looking at `target` (x right, y down, z forward)."""
    pos = np.asarray(position, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - pos
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, dtype=np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    f = (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    return camera_from_rt(width, height, f, f, R, -R @ pos, znear=znear)


def yaw_pitch_camera(position, yaw, pitch, width, height, hfov_deg=60.0, znear=0.2) -> Camera:
    """Camera at `position`, heading `yaw` (0 = +y), pitched `pitch` radians down."""
    pos = np.asarray(position, dtype=np.float64)
    head = np.array([math.sin(yaw), math.cos(yaw), 0.0])
    right = np.array([math.cos(yaw), -math.sin(yaw), 0.0])
    fwd = math.cos(pitch) * head - math.sin(pitch) * np.array([0.0, 0.0, 1.0])
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    f = (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    return camera_from_rt(width, height, f, f, R, -R @ pos, znear=znear)


def cube_camera(width=128, height=128, f=128.0) -> Camera:
    """Pinhole at (0,0,-4) looking along +z (R = I, t = (0,0,4))."""
    return camera_from_rt(width, height, f, f, np.eye(3), np.array([0.0, 0.0, 4.0]))


def aerial_camera(width=1920, height=1080, heading_deg=0.0) -> Camera:
    """150 m above ground, 150 m back from the origin, pitched 45 degrees down
    towards the origin; `heading_deg` rotates the pose about the vertical axis."""
    a = math.radians(heading_deg)
    pos = np.array([150.0 * math.sin(a), -150.0 * math.cos(a), 150.0])
    return look_at(pos, (0.0, 0.0, 0.0), width, height)


def orbit_cameras(n_views=64, radius=500.0, altitude=300.0, width=1920, height=1080):
    cams = []
    for k in range(n_views):
        a = 2.0 * math.pi * k / n_views
        cams.append(look_at((radius * math.cos(a), radius * math.sin(a), altitude),
                            (0.0, 0.0, 0.0), width, height))
    return cams


SERVE_RESOLUTIONS = ((640, 360), (1280, 720), (1920, 1080), (3840, 2160))


def serving_requests(n: int, rate_hz: float = 200.0, seed: int = 6):
    """Poisson arrivals of novel-view requests with mixed resolutions and random
    aerial poses: xy ~ U[-400,400]^2, altitude U(80,400) m, yaw U(0, 2pi),
    pitch U(30, 90) degrees down, 60 degree horizontal field of view."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_hz, n)
    arrivals = np.cumsum(gaps)
    out = []
    for i in range(n):
        w, h = SERVE_RESOLUTIONS[int(rng.integers(0, len(SERVE_RESOLUTIONS)))]
        xy = rng.uniform(-400.0, 400.0, 2)
        alt = rng.uniform(80.0, 400.0)
        yaw = rng.uniform(0.0, 2.0 * math.pi)
        pitch = math.radians(rng.uniform(30.0, 90.0))
        out.append((float(arrivals[i]), yaw_pitch_camera((xy[0], xy[1], alt), yaw, pitch, w, h)))
    return out


def target_image(width: int, height: int, seed: int = 1) -> np.ndarray:
    """Uniform [0,1) target image, layout [3][H][W] float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random((3, height, width), dtype=np.float64).astype(np.float32)


def scene_nbytes(n: int) -> int:
    """Bytes of one scene's float parameters (59 floats per Gaussian) + lod."""
    return n * (59 * 4 + 1)
