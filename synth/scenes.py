"""Procedural box scenes, octree anchors, MLP weights, cameras and Gaussians.

Recipe (all draws from ``numpy.random.default_rng(seed)`` in a fixed order):

* Points are sampled area-uniformly on the visible faces (4 sides + top) of
  random axis-aligned boxes, plus an optional ground rectangle.  They stand in
  for the sparse SfM points the paper starts from (Sec. IV-A, "Anchor
  Initialization").
* Anchors are built per octree level L = 0..K-1 as the distinct lattice points
  round(P / v_L) * v_L with v_L = delta / 2^L (the voxelisation of Eq. 6).  The
  base voxel size delta is bisected so that the total anchor count hits the
  requested size.  This is input preparation, not a step of the render path.
* d_max / d_min are the 99.9 % / 0.1 % quantiles of the camera-to-point
  distances (Sec. IV-A, the r_d quantiles before Eq. 5); the Eq. 5 depth is
  reported next to the configured K.
* Anchor attributes: features ~ N(0, 1); offsets O ~ N(0, sigma_o); the six
  per-anchor log-scales are drawn and exponentiated here (first three: the
  offset scaling l_v of Eq. 3, last three: the base Gaussian scale).
* MLP heads (opacity, colour, covariance) are 2-layer, Xavier-uniform weights
  and zero biases, input width F + 4 (feature, relative distance, direction).
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

# Planar field order of a Gaussian record, shared by every consumer of
# Gaussian buffers: [field][slot].
GAUSS_FIELDS = ("mx", "my", "mz", "sx", "sy", "sz", "qw", "qx", "qy", "qz",
                "opacity", "r", "g", "b")


@dataclasses.dataclass
class Camera:
    """Pinhole camera.  Camera-space point = R @ (p - C); x right, y down, z forward."""

    R: np.ndarray          # (3, 3) float32, rows are the camera axes in world space
    C: np.ndarray          # (3,) float32 camera centre
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    z_near: float = 0.2
    lod_scale: float = 1.0  # focal scale factor s of Eq. 7

    def __post_init__(self):
        self.R = np.ascontiguousarray(self.R, dtype=np.float32)
        self.C = np.ascontiguousarray(self.C, dtype=np.float32)
        # round the scalars to float32 so every consumer sees the same values
        for name in ("fx", "fy", "cx", "cy", "z_near", "lod_scale"):
            setattr(self, name, float(np.float32(getattr(self, name))))


@dataclasses.dataclass
class Scene:
    pos: np.ndarray            # (N, 3) float32 anchor positions
    level: np.ndarray          # (N,) uint8 octree level
    lod_bias: np.ndarray       # (N,) float32 per-anchor LOD bias (Delta L)
    feat: np.ndarray           # (N, F) float32
    offsets: np.ndarray        # (N, k, 3) float32
    offset_scale: np.ndarray   # (N, 3) float32, l_v of Eq. 3
    base_scale: np.ndarray     # (N, 3) float32
    mlp: Dict[str, np.ndarray]  # w1_{a,c,s} (in, W), b1_* (W,), w2_* (W, out), b2_* (out,)
    d_max: float
    d_min: float
    n_levels: int
    delta: float
    k: int
    feat_dim: int
    width: int
    info: Dict[str, object]

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def level_counts(self) -> List[int]:
        return [int(c) for c in np.bincount(self.level, minlength=self.n_levels)]


# ----------------------------------------------------------------------------
# cameras
# ----------------------------------------------------------------------------

def _intrinsics(width: int, height: int, fov_x_deg: float):
    fx = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return fx, fx, width / 2.0, height / 2.0


def look_at(center, target, width: int, height: int, fov_x_deg: float = 60.0,
            up=(0.0, 0.0, 1.0), z_near: float = 0.2) -> Camera:
    c = np.asarray(center, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - c
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, dtype=np.float64))
    if np.linalg.norm(r) < 1e-9:  # looking along up: pick any right vector
        r = np.cross(f, np.array([0.0, 1.0, 0.0]))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    fx, fy, cx, cy = _intrinsics(width, height, fov_x_deg)
    return Camera(R=R, C=c, fx=fx, fy=fy, cx=cx, cy=cy, width=width,
                  height=height, z_near=z_near)


def camera_from_yaw_pitch(center, yaw: float, pitch: float, width: int,
                          height: int, fov_x_deg: float = 60.0,
                          z_near: float = 0.2) -> Camera:
    """yaw, pitch in radians; pitch < 0 looks down.  Valid down to pitch = -pi/2."""
    f = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw),
                  math.sin(pitch)])
    r = np.array([math.sin(yaw), -math.cos(yaw), 0.0])
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    fx, fy, cx, cy = _intrinsics(width, height, fov_x_deg)
    return Camera(R=R, C=np.asarray(center, dtype=np.float64), fx=fx, fy=fy,
                  cx=cx, cy=cy, width=width, height=height, z_near=z_near)


def zoomout_trajectory(n: int, h0: float, h1: float, width: int, height: int,
                       fov_x_deg: float = 60.0) -> List[Camera]:
    """n cameras at log-spaced altitude h from h0 to h1, placed at (0, -h, h)
    and looking at the origin (45 degree pitch)."""
    cams = []
    for i in range(n):
        h = h0 * (h1 / h0) ** (i / max(n - 1, 1))
        cams.append(look_at((0.0, -h, h), (0.0, 0.0, 0.0), width, height, fov_x_deg))
    return cams


def trajectory_family_views(n: int, seed: int, h_lo: float, h_hi: float, width: int,
                            height: int, fov_x_deg: float = 60.0, jitter: float = 0.1) -> List[Camera]:
    """Views of the zoom-out's family: altitude h log-uniform in [h_lo, h_hi],
    the camera at (0, -h, h) + N(0, (jitter h)^2) per horizontal axis and
    looking at its own ground point (0, 0, 0) + the same offset plus
    N(0, (jitter h)^2) per horizontal axis, so the pitch stays near 45
    degrees and the yaw near the trajectory's."""
    rng = np.random.default_rng(seed)
    cams = []
    for _ in range(n):
        h = math.exp(rng.uniform(math.log(h_lo), math.log(h_hi)))
        ox, oy = rng.normal(0.0, jitter * h, 2)
        tx, ty = rng.normal(0.0, jitter * h, 2)
        cams.append(look_at((ox, oy - h, h), (ox + tx, oy + ty, 0.0), width, height, fov_x_deg))
    return cams


def random_views(n: int, seed: int, extent: float, h_lo: float, h_hi: float,
                 width: int, height: int, fov_x_deg: float = 60.0) -> List[Camera]:
    """Random aerial views: altitude log-uniform in [h_lo, h_hi], position
    uniform over the plane square of half-size `extent`, yaw uniform, pitch
    uniform in [-90, -20] degrees."""
    rng = np.random.default_rng(seed)
    cams = []
    for _ in range(n):
        h = math.exp(rng.uniform(math.log(h_lo), math.log(h_hi)))
        x, y = rng.uniform(-extent, extent, 2)
        yaw = rng.uniform(0, 2 * math.pi)
        pitch = math.radians(rng.uniform(-90.0, -20.0))
        cams.append(camera_from_yaw_pitch((x, y, h), yaw, pitch, width, height, fov_x_deg))
    return cams


# ----------------------------------------------------------------------------
# points on boxes
# ----------------------------------------------------------------------------

def _boxes_in_cube(rng, n_boxes: int, lo: float, hi: float, min_extent: float):
    boxes = []
    while len(boxes) < n_boxes:
        a = rng.uniform(lo, hi, 3)
        b = rng.uniform(lo, hi, 3)
        bmin, bmax = np.minimum(a, b), np.maximum(a, b)
        if np.all(bmax - bmin >= min_extent):
            boxes.append((bmin, bmax))
    return boxes


def _boxes_on_plane(rng, n_boxes: int, extent: float, foot=(5.0, 50.0),
                    height=(3.0, 60.0), clear_halfwidth: float = 30.0):
    """Boxes standing on z = 0 inside [-extent, extent]^2, kept off the street
    x in [-clear_halfwidth, clear_halfwidth], y < clear_halfwidth along which
    the zoom-out trajectory looks."""
    boxes = []
    while len(boxes) < n_boxes:
        sx, sy = rng.uniform(foot[0], foot[1], 2)
        h = rng.uniform(height[0], height[1])
        cx, cy = rng.uniform(-extent + sx / 2, extent - sx / 2), rng.uniform(-extent + sy / 2, extent - sy / 2)
        x0, x1, y0, y1 = cx - sx / 2, cx + sx / 2, cy - sy / 2, cy + sy / 2
        if x1 > -clear_halfwidth and x0 < clear_halfwidth and y0 < clear_halfwidth:
            continue
        boxes.append((np.array([x0, y0, 0.0]), np.array([x1, y1, h])))
    return boxes


def _box_faces(bmin, bmax, with_bottom: bool):
    """Rectangles (origin, u, v) of a box surface."""
    x0, y0, z0 = bmin
    x1, y1, z1 = bmax
    dx, dy, dz = x1 - x0, y1 - y0, z1 - z0
    faces = [
        ((x0, y0, z1), (dx, 0, 0), (0, dy, 0)),  # top
        ((x0, y0, z0), (dx, 0, 0), (0, 0, dz)),  # y = y0
        ((x0, y1, z0), (dx, 0, 0), (0, 0, dz)),  # y = y1
        ((x0, y0, z0), (0, dy, 0), (0, 0, dz)),  # x = x0
        ((x1, y0, z0), (0, dy, 0), (0, 0, dz)),  # x = x1
    ]
    if with_bottom:
        faces.append(((x0, y0, z0), (dx, 0, 0), (0, dy, 0)))
    return faces


def sample_surface_points(rng, faces, n_points: int) -> np.ndarray:
    o = np.array([f[0] for f in faces], dtype=np.float64)
    u = np.array([f[1] for f in faces], dtype=np.float64)
    v = np.array([f[2] for f in faces], dtype=np.float64)
    area = np.linalg.norm(np.cross(u, v), axis=1)
    counts = rng.multinomial(n_points, area / area.sum())
    idx = np.repeat(np.arange(len(faces)), counts)
    pts = np.empty((n_points, 3), dtype=np.float32)
    chunk = 1 << 22
    for s in range(0, n_points, chunk):
        e = min(n_points, s + chunk)
        ab = rng.random((e - s, 2))
        ii = idx[s:e]
        pts[s:e] = (o[ii] + ab[:, :1] * u[ii] + ab[:, 1:] * v[ii]).astype(np.float32)
    return pts


# ----------------------------------------------------------------------------
# octree voxelisation (input preparation; the anchor-initialisation recipe)
# ----------------------------------------------------------------------------

_OFF = 1 << 20


def _lattice_keys(points: np.ndarray, voxel: float) -> np.ndarray:
    q = np.floor(points.astype(np.float64) / voxel + 0.5).astype(np.int64)
    if np.abs(q).max(initial=0) >= _OFF:
        raise ValueError("voxel too small for the 21-bit lattice key")
    return ((q[:, 0] + _OFF) << 42) | ((q[:, 1] + _OFF) << 21) | (q[:, 2] + _OFF)


def _keys_to_pos(keys: np.ndarray, voxel: float) -> np.ndarray:
    qx = (keys >> 42) - _OFF
    qy = ((keys >> 21) & ((1 << 21) - 1)) - _OFF
    qz = (keys & ((1 << 21) - 1)) - _OFF
    return (np.stack([qx, qy, qz], axis=1).astype(np.float64) * voxel)


def _seg_dist(points: np.ndarray, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Distance from each point to the segment [a, b] (float64)."""
    p = points.astype(np.float64)
    ab = b - a
    L2 = float(ab @ ab)
    if L2 == 0.0:  # a single camera position
        return np.linalg.norm(p - a, axis=1)
    t = np.clip(((p - a) @ ab) / L2, 0.0, 1.0)
    return np.linalg.norm(p - (a + t[:, None] * ab), axis=1)


def _near_dist(points: np.ndarray, near) -> np.ndarray:
    """Distance to the nearest camera path element: `near` is a list of
    segments (a, b); a single camera is a zero-length segment."""
    d = None
    for a, b in near:
        di = _seg_dist(points, np.asarray(a, np.float64), np.asarray(b, np.float64))
        d = di if d is None else np.minimum(d, di)
    return d


def _level_anchors(points, delta, L, near=None, r0=None, dist=None):
    """Distinct lattice points of level L; with `near`, only those within
    r0 / 2^L of the camera path (dist: precomputed point distances)."""
    v = delta / 2 ** L
    if near is None:
        return np.unique(_lattice_keys(points, v)), v
    r = r0 / 2 ** L
    pre = points[dist <= r + v]
    keys = np.unique(_lattice_keys(pre, v))
    if len(keys) == 0:
        return keys, v
    pos = _keys_to_pos(keys, v)
    return keys[_near_dist(pos, near) <= r], v


def _count_levels(points, delta, n_levels, near=None, r0=None, dist=None):
    return [len(_level_anchors(points, delta, L, near, r0, dist)[0]) for L in range(n_levels)]


def fit_delta(points: np.ndarray, n_levels: int, target: int, rel_tol: float = 0.005,
              subsample: Optional[int] = None, rng=None, near=None, r0=None) -> float:
    """Bisect the coarsest voxel size so that the total anchor count over all
    levels is within rel_tol of target.  A subsample narrows the bracket
    before the full point set is used."""
    ext = float(np.max(points.max(0) - points.min(0)))
    lo, hi = ext * 1e-5, ext * 4.0

    def total(pts, d, dist):
        return sum(_count_levels(pts, d, n_levels, near, r0, dist))

    dist_all = _near_dist(points, near) if near is not None else None
    if subsample is not None and len(points) > subsample:
        pick = rng.choice(len(points), subsample, replace=False)
        sub = points[pick]
        dsub = dist_all[pick] if dist_all is not None else None
        for _ in range(30):
            mid = math.sqrt(lo * hi)
            if total(sub, mid, dsub) > target:
                lo = mid
            else:
                hi = mid
            if hi / lo < 1.05:
                break
        lo, hi = lo / 1.6, hi * 1.6
    best = None
    for _ in range(40):
        mid = math.sqrt(lo * hi)
        t = total(points, mid, dist_all)
        if best is None or abs(t - target) < abs(best[1] - target):
            best = (mid, t)
        if abs(t - target) <= rel_tol * target:
            return mid
        if t > target:
            lo = mid
        else:
            hi = mid
    return best[0]


def voxelize(points: np.ndarray, delta: float, n_levels: int, near=None, r0=None):
    """Distinct lattice points per level, ordered by level then lattice key."""
    dist = _near_dist(points, near) if near is not None else None
    pos, lev = [], []
    for L in range(n_levels):
        keys, v = _level_anchors(points, delta, L, near, r0, dist)
        pos.append(_keys_to_pos(keys, v).astype(np.float32))
        lev.append(np.full(len(keys), L, dtype=np.uint8))
    return np.concatenate(pos), np.concatenate(lev)


def distance_quantiles(points: np.ndarray, centers: np.ndarray, rng, q: float = 0.999,
                       max_pairs: int = 20_000_000):
    """(d_max, d_min): the q and 1-q quantiles of all camera-point distances,
    from a random point subsample when the pair count is large."""
    centers = np.asarray(centers, dtype=np.float64).reshape(-1, 3)
    n_pts = max(1, min(len(points), max_pairs // len(centers)))
    sub = points if n_pts >= len(points) else points[rng.choice(len(points), n_pts, replace=False)]
    d = np.sqrt(((sub[None, :, :].astype(np.float64) - centers[:, None, :]) ** 2).sum(-1)).ravel()
    return float(np.quantile(d, q)), float(np.quantile(d, 1.0 - q))


# ----------------------------------------------------------------------------
# attributes and MLPs
# ----------------------------------------------------------------------------

def xavier_mlp(rng, in_dim: int, width: int, k: int) -> Dict[str, np.ndarray]:
    mlp = {}
    for head, out in (("a", k), ("c", 3 * k), ("s", 7 * k)):
        a1 = math.sqrt(6.0 / (in_dim + width))
        a2 = math.sqrt(6.0 / (width + out))
        mlp["w1_" + head] = rng.uniform(-a1, a1, (in_dim, width)).astype(np.float32)
        mlp["b1_" + head] = np.zeros(width, dtype=np.float32)
        mlp["w2_" + head] = rng.uniform(-a2, a2, (width, out)).astype(np.float32)
        mlp["b2_" + head] = np.zeros(out, dtype=np.float32)
    return mlp


def make_scene(points: np.ndarray, n_levels: int, target_anchors: int, cams_for_dist,
               k: int, feat_dim: int, width: int, seed: int, scale_mode: str,
               offset_sigma: float, logscale_range=(-4.0, -1.0), subsample=None,
               near=None, delta: Optional[float] = None, info=None) -> Scene:
    """Anchors from points.  With `near` (camera path segments), level-L
    anchors are kept only within d_max / 2^L of the path: the anchor set a
    trained model keeps after its view-frequency pruning (Sec. IV-B), where
    fine levels survive only where training cameras come close.  `delta`
    skips the bisection when the fitted base voxel size is already known."""
    rng = np.random.default_rng(seed + 1000)
    centers = np.array([c.C for c in cams_for_dist], dtype=np.float64)
    d_max, d_min = distance_quantiles(points, centers, rng)
    d_max = float(np.float32(d_max))
    r0 = d_max if near is not None else None
    if delta is None:
        delta = fit_delta(points, n_levels, target_anchors, subsample=subsample, rng=rng,
                          near=near, r0=r0)
    pos, level = voxelize(points, delta, n_levels, near=near, r0=r0)
    n = len(pos)
    feat = rng.standard_normal((n, feat_dim)).astype(np.float32)
    offsets = (offset_sigma * rng.standard_normal((n, k, 3))).astype(np.float32)
    if scale_mode == "literal":
        ls = rng.uniform(logscale_range[0], logscale_range[1], (n, 6))
    elif scale_mode == "voxel":
        # log-scales around the log voxel size of the anchor's level
        lv = np.log(delta / 2.0 ** level.astype(np.float64))[:, None]
        ls = np.concatenate([lv + rng.uniform(-0.5, 0.0, (n, 3)),
                             lv + rng.uniform(-1.5, -0.5, (n, 3))], axis=1)
    else:
        raise ValueError(scale_mode)
    scales = np.exp(ls).astype(np.float32)
    mlp = xavier_mlp(rng, feat_dim + 4, width, k)
    k_eq5 = int(math.floor(math.log2(d_max / max(d_min, 1e-12)) + 0.5)) + 1
    meta = dict(info or {})
    meta.update(n_points=int(len(points)), k_eq5=k_eq5)
    return Scene(pos=pos, level=level, lod_bias=np.zeros(n, dtype=np.float32), feat=feat,
                 offsets=offsets, offset_scale=np.ascontiguousarray(scales[:, :3]),
                 base_scale=np.ascontiguousarray(scales[:, 3:]), mlp=mlp, d_max=d_max,
                 d_min=d_min, n_levels=n_levels, delta=delta, k=k, feat_dim=feat_dim,
                 width=width, info=meta)


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------

def config1_camera() -> Camera:
    d = np.array([1.0, -2.0, 1.5])
    d /= np.linalg.norm(d)
    return look_at(30.0 * d, (0.0, 0.0, 0.0), 128, 128, 60.0)


def make_config1(seed: int = 0) -> Scene:
    """~2,000 anchors over 3 levels from 20k points on 8 boxes in [-10, 10]^3."""
    rng = np.random.default_rng(seed)
    boxes = _boxes_in_cube(rng, 8, -10.0, 10.0, 1.0)
    faces = [f for b in boxes for f in _box_faces(b[0], b[1], with_bottom=True)]
    pts = sample_surface_points(rng, faces, 20_000)
    return make_scene(pts, 3, 2000, [config1_camera()], k=10, feat_dim=32, width=32,
                      seed=seed, scale_mode="literal", offset_sigma=0.1,
                      info=dict(name="c1"))


def _street_points(rng, n_points: int, n_boxes: int, extent: float):
    boxes = _boxes_on_plane(rng, n_boxes, extent)
    faces = [f for b in boxes for f in _box_faces(b[0], b[1], with_bottom=False)]
    faces.append(((-extent, -extent, 0.0), (2 * extent, 0, 0), (0, 2 * extent, 0)))
    return sample_surface_points(rng, faces, n_points)


# base voxel size bisected once for the default config-2 arguments
# (1,002,919 anchors; per level 21056, 117569, 304029, 325449, 205544, 26392, 2671, 209)
C2_DELTA = 13.890095477461857


def config2_cameras(n: int = 200, width: int = 1920, height: int = 1080):
    return zoomout_trajectory(n, 10.0, 800.0, width, height, 60.0)


def make_config2(seed: int = 1, n_anchors: int = 1_000_000, n_points: int = 20_000_000,
                 n_boxes: int = 2000, extent: float = 500.0, n_levels: int = 8,
                 delta: Optional[float] = C2_DELTA) -> Scene:
    """1M anchors over 8 levels from 20M points on 2,000 boxes over [-500, 500]^2.
    The default delta is the value `fit_delta` returns for the default
    arguments (pass delta=None to bisect again; about a minute)."""
    rng = np.random.default_rng(seed)
    pts = _street_points(rng, n_points, n_boxes, extent)
    near = [((0.0, -10.0, 10.0), (0.0, -800.0, 800.0))]
    return make_scene(pts, n_levels, n_anchors, config2_cameras(), k=10, feat_dim=32,
                      width=64, seed=seed, scale_mode="voxel", offset_sigma=0.25,
                      subsample=max(1, n_points // 8), near=near, delta=delta,
                      info=dict(name="c2", n_boxes=n_boxes, extent=extent))


def config3_views(seed: int = 3):
    return random_views(4, seed, 500.0, 10.0, 800.0, 1600, 1066)


# base voxel size bisected once for the default config-3 arguments
# (498,520 anchors; per level 8000, 43649, 126737, 165092, 107526, 47516)
C3_DELTA = 20.50295138003223


def perturbed_copy(sc: Scene, sigma: float, seed: int) -> Scene:
    """The scene with N(0, sigma^2) noise added to every anchor feature (the
    source of the training targets of config 3)."""
    rng = np.random.default_rng(seed)
    out = dataclasses.replace(sc)
    out.feat = (sc.feat + sigma * rng.standard_normal(sc.feat.shape)).astype(np.float32)
    return out


def make_config3(seed: int = 3, delta: Optional[float] = C3_DELTA) -> Scene:
    """500k anchors over 6 levels on the c2 procedural box scene, kept near
    the 4 training views (the same pruning model as config 2)."""
    rng = np.random.default_rng(1)
    pts = _street_points(rng, 20_000_000, 2000, 500.0)
    views = config3_views(seed)
    near = [(tuple(c.C.astype(np.float64)), tuple(c.C.astype(np.float64))) for c in views]
    return make_scene(pts, 6, 500_000, views, k=10, feat_dim=32, width=64,
                      seed=seed, scale_mode="voxel", offset_sigma=0.25,
                      subsample=2_500_000, near=near, delta=delta, info=dict(name="c3"))


def config5_cameras(n: int = 200, width: int = 3840, height: int = 2160):
    return zoomout_trajectory(n, 20.0, 3000.0, width, height, 60.0)


def config5_train_views():
    """The training step's 8 views at 2048x1024: evenly spaced along the
    zoom-out, where the pruned scene keeps its fine levels."""
    return zoomout_trajectory(8, 20.0, 3000.0, 2048, 1024, 60.0)


# base voxel size bisected once for the default config-5 arguments
# (4,000,407 anchors; per level 109592, 496537, 1012137, 1015771, 890174,
# 380807, 84299, 10671, 419, 0: no camera of the zoom-out comes within
# d_max / 2^9 of a surface, so the pruning leaves the finest level empty)
C5_DELTA = 18.174696515286612


def make_config5(seed: int = 5, delta: Optional[float] = C5_DELTA) -> Scene:
    """4M anchors over 10 levels from 80M points on 8,000 boxes over
    [-2000, 2000]^2, with the same path pruning as config 2 along the
    20 -> 3000 m zoom-out."""
    rng = np.random.default_rng(seed)
    pts = _street_points(rng, 80_000_000, 8000, 2000.0)
    near = [((0.0, -20.0, 20.0), (0.0, -3000.0, 3000.0))]
    return make_scene(pts, 10, 4_000_000, config5_cameras(), k=10, feat_dim=32, width=64,
                      seed=seed, scale_mode="voxel", offset_sigma=0.25, subsample=10_000_000,
                      near=near, delta=delta, info=dict(name="c5"))


def make_gradcheck_scene(seed: int = 7, n: int = 50, k: int = 10, feat_dim: int = 32,
                         width: int = 16) -> (Scene, Camera):
    """50 anchors in front of a 64x64 camera, sized so their Gaussians cover a
    few pixels each; all at level 0 so every anchor is selected."""
    rng = np.random.default_rng(seed)
    cam = look_at((0.0, -6.0, 0.0), (0.0, 0.0, 0.0), 64, 64, 60.0)
    pos = np.stack([rng.uniform(-2.2, 2.2, n), rng.uniform(-1.5, 1.5, n),
                    rng.uniform(-2.2, 2.2, n)], axis=1).astype(np.float32)
    feat = rng.standard_normal((n, feat_dim)).astype(np.float32)
    offsets = (0.5 * rng.standard_normal((n, k, 3))).astype(np.float32)
    ls = rng.uniform(-2.0, -1.2, (n, 6))
    scales = np.exp(ls).astype(np.float32)
    mlp = xavier_mlp(rng, feat_dim + 4, width, k)
    sc = Scene(pos=pos, level=np.zeros(n, dtype=np.uint8), lod_bias=np.zeros(n, np.float32),
               feat=feat, offsets=offsets, offset_scale=np.ascontiguousarray(scales[:, :3]),
               base_scale=np.ascontiguousarray(scales[:, 3:]), mlp=mlp,
               d_max=float(np.float32(12.0)), d_min=3.0, n_levels=1, delta=1.0, k=k,
               feat_dim=feat_dim, width=width, info=dict(name="gradcheck"))
    return sc, cam


# ----------------------------------------------------------------------------
# raw Gaussians for rasterizer-stage tests
# ----------------------------------------------------------------------------

def _random_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def random_gaussians(n: int, cam: Camera, seed: int, depth=(2.0, 40.0), scale=(0.02, 0.6),
                     opacity=(0.05, 0.95), margin: float = 0.15,
                     neg_opacity_frac: float = 0.0, behind_frac: float = 0.0) -> np.ndarray:
    """n Gaussians spread over (and slightly beyond) the view frustum of cam,
    returned planar as float32 [14][n] in GAUSS_FIELDS order."""
    rng = np.random.default_rng(seed)
    z = np.exp(rng.uniform(math.log(depth[0]), math.log(depth[1]), n))
    u = rng.uniform(-margin * cam.width, (1 + margin) * cam.width, n)
    v = rng.uniform(-margin * cam.height, (1 + margin) * cam.height, n)
    xc = (u - cam.cx) / cam.fx * z
    yc = (v - cam.cy) / cam.fy * z
    if behind_frac > 0:
        m = rng.random(n) < behind_frac
        z = np.where(m, -z * 0.1, z)
    pc = np.stack([xc, yc, z], axis=1)
    R = cam.R.astype(np.float64)
    pw = pc @ R + cam.C.astype(np.float64)[None, :]
    s = np.exp(rng.uniform(math.log(scale[0]), math.log(scale[1]), (n, 3)))
    q = _random_quats(rng, n)
    op = rng.uniform(opacity[0], opacity[1], n)
    if neg_opacity_frac > 0:
        m = rng.random(n) < neg_opacity_frac
        op = np.where(m, -op, op)
    rgb = rng.random((n, 3))
    g = np.concatenate([pw, s, q, op[:, None], rgb], axis=1).T
    return np.ascontiguousarray(g.astype(np.float32))


def tile_aligned_gaussians(cam: Camera, depths: Sequence[float], seed: int) -> np.ndarray:
    """Axis-aligned Gaussians on pixel centres, several sharing one depth, for
    exercising the equal-depth tie-break."""
    rng = np.random.default_rng(seed)
    n = len(depths)
    u = rng.integers(0, cam.width, n) + 0.5
    v = rng.integers(0, cam.height, n) + 0.5
    z = np.asarray(depths, dtype=np.float64)
    xc = (u - cam.cx) / cam.fx * z
    yc = (v - cam.cy) / cam.fy * z
    pc = np.stack([xc, yc, z], axis=1)
    pw = pc @ cam.R.astype(np.float64) + cam.C.astype(np.float64)[None, :]
    s = np.full((n, 3), 0.05) * z[:, None] / 10.0
    q = np.tile([1.0, 0.0, 0.0, 0.0], (n, 1))
    op = rng.uniform(0.2, 0.9, n)
    rgb = rng.random((n, 3))
    g = np.concatenate([pw, s, q, op[:, None], rgb], axis=1).T
    return np.ascontiguousarray(g.astype(np.float32))


# ----------------------------------------------------------------------------
# explicit Gaussians per anchor (the 3D-GS instance of the anchor framework)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class ExplicitScene:
    """Anchors that each carry k explicit 3D Gaussians (Sec. V, "Our-3D-GS":
    the octree anchors and Eq. 7 selection of the framework with 3D-GS
    primitives).  Per Gaussian: world mean, log-scales, an unnormalised
    rotation quaternion (w, x, y, z), an opacity logit and spherical-harmonic
    colour coefficients [(D+1)^2][3]."""

    pos: np.ndarray        # (N, 3) float32 anchor positions
    level: np.ndarray      # (N,) uint8
    lod_bias: np.ndarray   # (N,) float32
    mean: np.ndarray       # (N, k, 3) float32
    log_scale: np.ndarray  # (N, k, 3) float32
    rot: np.ndarray        # (N, k, 4) float32
    opacity: np.ndarray    # (N, k) float32 logits
    sh: np.ndarray         # (N, k, (D+1)^2, 3) float32
    sh_degree: int
    d_max: float
    n_levels: int
    k: int
    info: Dict[str, object]

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def make_explicit(sc: Scene, sh_degree: int = 3, seed: int = 11,
                  opacity_logit=(-4.0, 2.0), dc_sigma: float = 0.6,
                  rest_sigma: float = 0.15) -> ExplicitScene:
    """Explicit Gaussians on the anchors of a neural scene, drawn with
    statistics close to what the neural decode of that scene emits: means at
    x_v + O_i * l_v, scales base_scale * U(0.2, 0.8) (the sigmoid-bounded
    neural scale), random unnormalised rotations, opacity logits
    U(opacity_logit), DC colour coefficients N(0, dc_sigma^2) and degree-l
    coefficients N(0, (rest_sigma / l)^2)."""
    rng = np.random.default_rng(seed)
    n, k = sc.n, sc.k
    nc = (sh_degree + 1) ** 2
    mean = (sc.pos[:, None, :].astype(np.float64)
            + sc.offsets.astype(np.float64) * sc.offset_scale[:, None, :]).astype(np.float32)
    u = rng.uniform(0.2, 0.8, (n, k, 3))
    log_scale = (np.log(sc.base_scale.astype(np.float64))[:, None, :] + np.log(u)).astype(np.float32)
    rot = rng.standard_normal((n, k, 4), dtype=np.float32)
    opacity = rng.uniform(opacity_logit[0], opacity_logit[1], (n, k)).astype(np.float32)
    sh = np.empty((n, k, nc, 3), np.float32)
    sh[:, :, 0, :] = dc_sigma * rng.standard_normal((n, k, 3), dtype=np.float32)
    for l in range(1, sh_degree + 1):
        sh[:, :, l * l:(l + 1) * (l + 1), :] = np.float32(rest_sigma / l) * rng.standard_normal(
            (n, k, 2 * l + 1, 3), dtype=np.float32)
    return ExplicitScene(pos=sc.pos, level=sc.level, lod_bias=sc.lod_bias, mean=mean,
                         log_scale=log_scale, rot=rot, opacity=opacity, sh=sh,
                         sh_degree=sh_degree, d_max=sc.d_max, n_levels=sc.n_levels, k=k,
                         info=dict(sc.info, explicit_seed=seed))
