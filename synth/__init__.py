"""Seeded synthetic inputs for the splatting hot path.

This module only draws numbers and lays them out: Gaussian parameter arrays,
pinhole cameras, cell boxes, loss targets and request traces.  It contains
none of the rendering arithmetic (projection, blending, composition or their
gradients); both the FP64 oracle and the HIP path consume the FP32 arrays it
returns, so the two sides always see bit-identical inputs.

Every generator uses ``numpy.random.default_rng(PCG64(seed))`` and draws in
FP64 in the fixed order means -> log_scales -> quats -> opacity logits -> SH,
then casts to FP32.  The workloads stand in for the city-scale aerial/street
captures the paper trains on (its experimental setup section): a ground plane
of Gaussians seen from an aerial camera pitched 45 degrees down, at the
resolutions and scene sizes of the paper's per-GPU shares.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# --------------------------------------------------------------------------
# containers
# --------------------------------------------------------------------------


@dataclass
class Scene:
    """Gaussian parameters, SoA, FP32 (the parametrisation of the paper's
    background section: position, rotation, scale, opacity, colour).

    means        [N,3]   world position (z up, metres)
    log_scales   [N,3]   log of the per-axis standard deviation
    quats        [N,4]   rotation quaternion (w, x, y, z), not necessarily unit
    opacity_logits [N]   opacity before the logistic sigmoid
    sh           [N,(D+1)^2,3]  real spherical-harmonic colour coefficients,
                         coefficient index l*l+l+m, channel fastest
    """

    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def sh_degree(self) -> int:
        k = self.sh.shape[1]
        d = int(round(math.sqrt(k))) - 1
        assert (d + 1) ** 2 == k
        return d

    def subset(self, idx: np.ndarray) -> "Scene":
        return Scene(
            np.ascontiguousarray(self.means[idx]),
            np.ascontiguousarray(self.log_scales[idx]),
            np.ascontiguousarray(self.quats[idx]),
            np.ascontiguousarray(self.opacity_logits[idx]),
            np.ascontiguousarray(self.sh[idx]),
        )

    def astype(self, dtype) -> "Scene":
        return Scene(*(np.ascontiguousarray(a.astype(dtype)) for a in
                       (self.means, self.log_scales, self.quats,
                        self.opacity_logits, self.sh)))

    def arrays(self):
        return (self.means, self.log_scales, self.quats, self.opacity_logits,
                self.sh)


@dataclass
class Camera:
    """Pinhole camera, world->camera ``x_cam = R @ x_world + t`` with OpenCV
    axes (x right, y down, z forward).  Pixel (i, j) has its centre at
    (i + 0.5, j + 0.5)."""

    R: np.ndarray  # [3,3] float32
    t: np.ndarray  # [3] float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    znear: float = 0.2

    @property
    def n_pixels(self) -> int:
        return self.width * self.height

    def center(self) -> np.ndarray:
        R = self.R.astype(np.float64)
        return -R.T @ self.t.astype(np.float64)


@dataclass
class Cell:
    """Axis-aligned convex cell (one GPU's partition in the paper); bounds may
    be infinite."""

    lo: Tuple[float, float, float]
    hi: Tuple[float, float, float]


@dataclass
class Partition:
    """A scene split into K cells: ``order`` is the stable permutation that
    groups Gaussians by cell, ``offsets[k]:offsets[k+1]`` the k-th block."""

    cells: List[Cell]
    cell_of: np.ndarray  # [N] int32 cell index per Gaussian (original order)
    order: np.ndarray  # [N] int64
    offsets: np.ndarray  # [K+1] int64

    @property
    def k(self) -> int:
        return len(self.cells)

    def cell_scenes(self, scene: Scene) -> List[Scene]:
        return [scene.subset(self.order[self.offsets[k]:self.offsets[k + 1]])
                for k in range(self.k)]


# --------------------------------------------------------------------------
# primitives
# --------------------------------------------------------------------------


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _unit_quats(rng: np.random.Generator, n: int) -> np.ndarray:
    q = rng.normal(0.0, 1.0, size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


# The DC real spherical harmonic is the constant 1/(2*sqrt(pi)); a scene whose
# colour is specified directly as RGB stores k0 = (rgb - 0.5) * 2*sqrt(pi) so
# that the evaluated colour is exactly that RGB (SH degree 0).
_INV_Y00 = 2.0 * math.sqrt(math.pi)


def make_cube_scene(seed: int, n: int, half: float = 1.0,
                    log_scale: Tuple[float, float] = (-4.0, 0.5),
                    logit_sigma: float = 1.0, sh_degree: int = 0,
                    sh_sigma: float = 0.2) -> Scene:
    """Means uniform in [-half, half]^3 (the small object-scale config)."""
    rng = rng_for(seed)
    means = rng.uniform(-half, half, size=(n, 3))
    log_scales = rng.normal(log_scale[0], log_scale[1], size=(n, 3))
    quats = _unit_quats(rng, n)
    logits = rng.normal(0.0, logit_sigma, size=n)
    if sh_degree == 0:
        rgb = rng.uniform(0.0, 1.0, size=(n, 3))
        sh = ((rgb - 0.5) * _INV_Y00)[:, None, :]
    else:
        sh = rng.normal(0.0, sh_sigma, size=(n, (sh_degree + 1) ** 2, 3))
    return Scene(means, log_scales, quats, logits, sh).astype(np.float32)


def make_ground_scene(seed: int, n: int, half_extent: float = 500.0,
                      z_sigma: float = 20.0,
                      log_scale: Tuple[float, float] = (-1.0, 0.7),
                      logit_sigma: float = 1.5, sh_degree: int = 3,
                      sh_sigma: float = 0.2, chunk: int = 1 << 22) -> Scene:
    """City-scale ground plane: x, y uniform over a square of side
    2*half_extent, z = |N(0, z_sigma)|, SH coefficients N(0, sh_sigma).

    Generated in chunks of ``chunk`` Gaussians (each chunk draws in the fixed
    order) so that tens of millions of Gaussians never need a full FP64 copy.
    """
    rng = rng_for(seed)
    k = (sh_degree + 1) ** 2
    means = np.empty((n, 3), np.float32)
    log_scales = np.empty((n, 3), np.float32)
    quats = np.empty((n, 4), np.float32)
    logits = np.empty((n,), np.float32)
    sh = np.empty((n, k, 3), np.float32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        m = e - s
        xy = rng.uniform(-half_extent, half_extent, size=(m, 2))
        z = np.abs(rng.normal(0.0, z_sigma, size=m))
        means[s:e, :2] = xy
        means[s:e, 2] = z
        log_scales[s:e] = rng.normal(log_scale[0], log_scale[1], size=(m, 3))
        quats[s:e] = _unit_quats(rng, m)
        logits[s:e] = rng.normal(0.0, logit_sigma, size=m)
        sh[s:e] = rng.normal(0.0, sh_sigma, size=(m, k, 3))
    return Scene(means, log_scales, quats, logits, sh)


def focal_from_hfov(width: int, hfov_deg: float) -> float:
    return (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)


def camera_from_rows(rows: np.ndarray, position: Sequence[float], width: int,
                     height: int, fx: float, fy: Optional[float] = None,
                     cx: Optional[float] = None, cy: Optional[float] = None,
                     znear: float = 0.2) -> Camera:
    R = np.asarray(rows, np.float64)
    p = np.asarray(position, np.float64)
    t = -R @ p
    return Camera(R.astype(np.float32), t.astype(np.float32), float(fx),
                  float(fy if fy is not None else fx),
                  float(cx if cx is not None else width / 2.0),
                  float(cy if cy is not None else height / 2.0),
                  int(width), int(height), float(znear))


def aerial_camera(position: Sequence[float], yaw: float, pitch: float,
                  width: int, height: int, hfov_deg: float = 70.0,
                  znear: float = 0.2) -> Camera:
    """Camera at ``position`` heading ``yaw`` (radians, 0 = +y, towards +x
    positive) and looking ``pitch`` radians below the horizon."""
    f = np.array([math.sin(yaw) * math.cos(pitch),
                  math.cos(yaw) * math.cos(pitch), -math.sin(pitch)])
    r = np.array([math.cos(yaw), -math.sin(yaw), 0.0])
    d = np.cross(f, r)
    return camera_from_rows(np.stack([r, d, f]), position, width, height,
                            focal_from_hfov(width, hfov_deg), znear=znear)


def look_at_camera(position: Sequence[float], target: Sequence[float],
                   width: int, height: int, hfov_deg: float = 70.0,
                   znear: float = 0.2) -> Camera:
    p = np.asarray(position, np.float64)
    f = np.asarray(target, np.float64) - p
    f /= np.linalg.norm(f)
    r = np.cross(f, np.array([0.0, 0.0, 1.0]))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    return camera_from_rows(np.stack([r, d, f]), p, width, height,
                            focal_from_hfov(width, hfov_deg), znear=znear)


def grid_partition(scene: Scene, xedges: Sequence[float],
                   yedges: Sequence[float]) -> Partition:
    """Assign each Gaussian to the ground-grid cell containing its centre:
    half-open [lo, hi) per axis with the outermost edges closed; cells are
    prisms unbounded in z, numbered k = iy * nx + ix."""
    xe = np.asarray(xedges, np.float64)
    ye = np.asarray(yedges, np.float64)
    nx, ny = len(xe) - 1, len(ye) - 1
    x = scene.means[:, 0].astype(np.float64)
    y = scene.means[:, 1].astype(np.float64)
    ix = np.clip(np.searchsorted(xe, x, side="right") - 1, 0, nx - 1)
    iy = np.clip(np.searchsorted(ye, y, side="right") - 1, 0, ny - 1)
    cell_of = (iy * nx + ix).astype(np.int32)
    cells = [Cell((float(xe[i]), float(ye[j]), -math.inf),
                  (float(xe[i + 1]), float(ye[j + 1]), math.inf))
             for j in range(ny) for i in range(nx)]
    return _finish_partition(cells, cell_of)


def axis_slab_partition(scene: Scene, axis: int,
                        edges: Sequence[float]) -> Partition:
    """Slabs along one world axis: cell k holds centres in
    [edges[k], edges[k+1]) (outer edges closed); other axes unbounded."""
    e = np.asarray(edges, np.float64)
    v = scene.means[:, axis].astype(np.float64)
    k = len(e) - 1
    cell_of = np.clip(np.searchsorted(e, v, side="right") - 1, 0,
                      k - 1).astype(np.int32)
    cells = []
    for i in range(k):
        lo = [-math.inf] * 3
        hi = [math.inf] * 3
        lo[axis], hi[axis] = float(e[i]), float(e[i + 1])
        cells.append(Cell(tuple(lo), tuple(hi)))
    return _finish_partition(cells, cell_of)


def quantile_edges(values: np.ndarray, k: int) -> np.ndarray:
    """k slab edges at the midpoints between consecutive order statistics
    nearest the k-quantiles, so no value sits on an inner edge."""
    v = np.sort(values.astype(np.float64))
    n = len(v)
    edges = [v[0] - 1.0]
    for i in range(1, k):
        j = (i * n) // k
        edges.append(0.5 * (v[j - 1] + v[j]))
    edges.append(v[-1] + 1.0)
    return np.asarray(edges)


def _finish_partition(cells: List[Cell], cell_of: np.ndarray) -> Partition:
    order = np.argsort(cell_of, kind="stable").astype(np.int64)
    counts = np.bincount(cell_of, minlength=len(cells))
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return Partition(cells, cell_of, order, offsets)


def random_image(seed: int, width: int, height: int) -> np.ndarray:
    """Loss target: U[0,1] RGB, [H, W, 3] FP32."""
    return rng_for(seed).uniform(0.0, 1.0,
                                 size=(height, width, 3)).astype(np.float32)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4
EPS2D = 0.3
FOV_GUARD = 1.3  # field-of-view cull by the mean: half-extents widened by 30%


@dataclass
class RenderSettings:
    tile_w: int = 16
    tile_h: int = 16
    alpha_min: float = ALPHA_MIN
    alpha_max: float = ALPHA_MAX
    t_min: float = T_MIN
    eps2d: float = EPS2D
    bg: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    fov_guard: float = FOV_GUARD


def tiny_scene(seed: int = 0, n: int = 5000) -> Scene:
    """5k Gaussians in [-1,1]^3, log-scales N(-4, 0.5), SH degree 0."""
    return make_cube_scene(seed, n)


def tiny_camera(width: int = 128, height: int = 128) -> Camera:
    """Camera at (0,0,-3) looking +z, 60 degree field of view."""
    f = (width / 2.0) / math.tan(math.radians(30.0))
    return camera_from_rows(np.eye(3), (0.0, 0.0, -3.0), width, height, f)


def screen_scene(seed: int = 0, n: int = 5000, n_near: int = 32) -> Scene:
    """The tiny scene plus n_near faint Gaussians just in front of the tiny
    camera (camera depth 0.25..3 m, within 0.1 m of the optical axis,
    log-scales N(-1.5, 0.3), opacity logits N(-2, 0.5)): their footprints
    cover the whole 128x128 view, the way Gaussians near the camera plane
    cover the whole frame in the aerial scenes, and they interleave in depth
    with the cube's Gaussians."""
    base = make_cube_scene(seed, n)
    rng = rng_for(seed + 7001)
    xy = rng.uniform(-0.1, 0.1, size=(n_near, 2))
    d = rng.uniform(0.25, 3.0, size=n_near)
    means = np.concatenate([xy, (d - 3.0)[:, None]], axis=1)
    log_scales = rng.normal(-1.5, 0.3, size=(n_near, 3))
    quats = _unit_quats(rng, n_near)
    logits = rng.normal(-2.0, 0.5, size=n_near)
    rgb = rng.uniform(0.0, 1.0, size=(n_near, 3))
    sh = ((rgb - 0.5) * _INV_Y00)[:, None, :]
    near = Scene(means, log_scales, quats, logits, sh).astype(np.float32)
    cat = [np.concatenate([a, b]) for a, b in zip(base.arrays(), near.arrays())]
    return Scene(*cat)


def fd_scene(seed: int, n: int = 64, sh_degree: int = 3) -> Scene:
    """Finite-difference sub-scene: 64 Gaussians large enough to overlap in a
    64x64 view (log-scales N(-2.5, 0.3), SH3 N(0, 0.2))."""
    return make_cube_scene(seed, n, half=0.6, log_scale=(-2.5, 0.3),
                           sh_degree=sh_degree)


def fd_camera() -> Camera:
    return tiny_camera(64, 64)


def clamp_fd_scene(seed: int) -> Scene:
    """The finite-difference scene (FP64) with Gaussian 0 made nearly opaque
    (logit 8, o = 0.99966), large (log-scales about -1) and in front of the
    others on the optical axis, so that o exp(-q/2) exceeds an alpha clamp of
    0.99 at the pixel centres within about 1.4 of its 10-pixel sigma."""
    s = fd_scene(seed).astype(np.float64)
    s.means[0] = (0.03, -0.02, -1.2)
    s.log_scales[0] = (-0.85, -1.15, -1.0)
    s.opacity_logits[0] = 8.0
    return s


def same_frame_fd_scenes(seed: int):
    """A 32-Gaussian finite-difference scene (FP64) in two depth slabs
    (camera-side slab z < 0) with the front slab's Gaussians made larger
    (log-scale + 0.4) and opaque (logit + 4), so that the transmittance
    through it drops below a threshold of 0.05 on part of the 64x64 view.
    Returns (cell scenes, cells)."""
    s = fd_scene(seed, n=32).astype(np.float64)
    front = s.means[:, 2] < 0
    s.log_scales[front] += 0.4
    s.opacity_logits[front] += 4.0
    part = axis_slab_partition(s, 2, [-10.0, 0.0, 10.0])
    return part.cell_scenes(s), part.cells


def g2_scene(seed: int = 1, n: int = 2_000_000) -> Scene:
    """One GPU's share: 2M Gaussians on a 1 km x 1 km ground plane, SH3."""
    return make_ground_scene(seed, n)


def g2_camera(width: int = 1920, height: int = 1080) -> Camera:
    """Aerial view from (0,0,150) m heading +y, pitched 45 degrees down,
    70 degree horizontal field of view."""
    return aerial_camera((0.0, 0.0, 150.0), 0.0, math.radians(45.0), width,
                         height)


def g2_target(width: int = 1920, height: int = 1080) -> np.ndarray:
    return random_image(101, width, height)


GRID_X = (-500.0, -250.0, 0.0, 250.0, 500.0)
GRID_Y = (-500.0, 0.0, 500.0)


def g8_scene(seed: int = 2, n: int = 8_000_000) -> Scene:
    return make_ground_scene(seed, n)


def g8_cameras(width: int = 1600, height: int = 1200,
               n_views: int = 8) -> List[Camera]:
    """Views from (10,20,150) m, yaw k*45 degrees, pitched 45 degrees down
    (placed off the cell boundaries so no ray starts on one)."""
    return [aerial_camera((10.0, 20.0, 150.0), math.radians(45.0 * k),
                          math.radians(45.0), width, height)
            for k in range(n_views)]


def nadir_camera(position: Sequence[float], width: int, height: int,
                 hfov_deg: float = 70.0) -> Camera:
    """Camera looking straight down (-z); camera depth is monotone in world
    z, so world-z slabs are depth-separated cells for it."""
    return aerial_camera(position, 0.0, math.radians(90.0), width, height,
                         hfov_deg)


def g15_scene(seed: int = 3, n: int = 15_000_000) -> Scene:
    return make_ground_scene(seed, n)


def g15_cameras(seed: int = 3, n_views: int = 16) -> List[Camera]:
    """16 views of uneven resolution (W ~ U{960..2048}, H ~ U{540..1365}) on
    a 200 m orbit at 150 m altitude looking at the origin."""
    rng = rng_for(seed + 1000)
    cams = []
    for _ in range(n_views):
        w = int(rng.integers(960, 2049))
        h = int(rng.integers(540, 1366))
        phi = rng.uniform(0.0, 2.0 * math.pi)
        cams.append(look_at_camera((200.0 * math.cos(phi),
                                    200.0 * math.sin(phi), 150.0),
                                   (0.0, 0.0, 0.0), w, h))
    return cams


def g30_scene(seed: int = 4, n: int = 30_000_000) -> Scene:
    """One quarter of a 120M-Gaussian city: 2 km x 2 km ground plane."""
    return make_ground_scene(seed, n, half_extent=1000.0)


SERVE_RESOLUTIONS = ((640, 360), (1280, 720), (1920, 1080), (3840, 2160))


@dataclass
class Request:
    arrival_s: float
    camera: Camera
    rid: int = 0


def serve_trace(n: int, rate_hz: float = 200.0, seed: int = 40,
                resolutions: Sequence[Tuple[int, int]] = SERVE_RESOLUTIONS,
                extent: float = 800.0) -> List[Request]:
    """Poisson arrivals (exponential gaps), uniform resolution choice, random
    aerial poses over the scene at 150 m, pitched 45 degrees down."""
    rng = rng_for(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate_hz)
        w, h = resolutions[int(rng.integers(0, len(resolutions)))]
        x, y = rng.uniform(-extent, extent, size=2)
        yaw = rng.uniform(0.0, 2.0 * math.pi)
        cam = aerial_camera((float(x), float(y), 150.0), float(yaw),
                            math.radians(45.0), w, h)
        out.append(Request(t, cam, i))
    return out


def sample_tiles(seed: int, cam: Camera, count: int, tile_w: int = 16,
                 tile_h: int = 16) -> np.ndarray:
    """Distinct random tile indices (row-major over the tile grid)."""
    tx = (cam.width + tile_w - 1) // tile_w
    ty = (cam.height + tile_h - 1) // tile_h
    rng = rng_for(seed)
    return np.sort(rng.choice(tx * ty, size=min(count, tx * ty),
                              replace=False)).astype(np.int64)
