"""Python shim over the plain C oracle (``octgs_oracle.c``).  TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module.  It never imports the HIP package, and the HIP package never
imports it.

Conventions shared with the callers (not with the HIP code):
  * a camera is passed as 18 float32 values: R (9, row-major world->camera),
    C (3), fx, fy, cx, cy, z_near, s^2, plus the integer image size;
  * raster parameters are 8 float32 values: alpha_max, alpha_min, t_min,
    dilation (px^2), jac_clamp, background rgb;
  * Gaussians are planar [14][n]: mean(3), scale(3), quat(w,x,y,z), opacity, rgb(3).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "octgs_oracle.c")
_LIB = os.path.join(_HERE, "liboctgs_oracle.so")
_lib = None

DEFAULT_PARAMS = dict(alpha_max=0.99, alpha_min=0.0, t_min=1e-4, dilation=0.3,
                      jac_clamp=1.3, bg=(0.0, 0.0, 0.0))


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, no FP contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
        _declare(_lib)
    return _lib


def source() -> str:
    """The oracle's C source text."""
    with open(_SRC) as f:
        return f.read()


class variant:
    """Context manager for tests that plant a mistake in the oracle: compiles
    the given C source text (normally source() with one edit) into `dirname`
    and routes this module's calls to it until the block ends."""

    def __init__(self, src_text: str, dirname: str, tag: str = "variant"):
        self.src = os.path.join(dirname, f"octgs_oracle_{tag}.c")
        self.so = os.path.join(dirname, f"liboctgs_oracle_{tag}.so")
        with open(self.src, "w") as f:
            f.write(src_text)
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-fPIC", "-shared", "-o", self.so, self.src,
                               "-lm"])

    def __enter__(self):
        global _lib
        self._saved = lib()
        v = ctypes.CDLL(self.so)
        _declare(v)
        _lib = v
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self._saved
        return False


_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int


def _declare(L):
    L.orc_lod_thr2.argtypes = [_i64, _p, _p, ctypes.c_float, _p]
    L.orc_bound_radius.argtypes = [_i64, _i32, _p, _p, _p, _p]
    L.orc_bound_radius_explicit.argtypes = [_i64, _i32, _p, _p, _p, _p]
    L.orc_select_fp32.argtypes = [_i64, _p, _p, _p, _i32, _p, _i32, _i32, _p, _p]
    L.orc_select_fp32.restype = _i64
    L.orc_select_eq7.argtypes = [_i64, _p, _p, _p, ctypes.c_float, _i32, _p, _i32, _p, _i32, _i32,
                                 _p, _p]
    L.orc_select_eq7.restype = _i64
    L.orc_decode.argtypes = [_i64, _p, _p, _p, _p, _p, _p, _i32, _i32, _i32, _p, _p,
                             ctypes.c_float, _i32, _p, _p, _i32, ctypes.c_float, _p]
    L.orc_lod_blend_factor.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_float,
                                       ctypes.c_float, _i32, _i32]
    L.orc_lod_blend_factor.restype = ctypes.c_double
    L.orc_project.argtypes = [_i64, _i64, _p, _p, _p, _i32, _i32, _p, _p, _p, _p, _p, _p]
    L.orc_project.restype = _i64
    L.orc_count_pairs.argtypes = [_i64, _p, _p, _p, _i32, _i32]
    L.orc_fragile.argtypes = [_i64, _i64, _p, _p, _p, _i32, _i32, _p, _p, _p, ctypes.c_double,
                              _p, _p, _p, _p]
    L.orc_fragile.restype = _i64
    L.orc_count_pairs.restype = _i64
    L.orc_count_rect_pairs.argtypes = [_i64, _p, _p]
    L.orc_count_rect_pairs.restype = _i64
    L.orc_tile_test.argtypes = [_p, _i32, _i32, _i32, _i32]
    L.orc_tile_test.restype = _i32
    L.orc_bin_sort.argtypes = [_i64, _p, _p, _p, _p, _i32, _i32, _p, _p, _p]
    L.orc_bin_sort.restype = _i64
    L.orc_composite.argtypes = [_p, _p, _p, _i32, _i32, _p, _p, _p, _p, _p]
    L.orc_render_bruteforce.argtypes = [_i64, _p, _p, _p, _p, _p, _i32, _i32, _p, _p, _p]
    L.orc_num_threads.restype = _i32
    L.orc_set_num_threads.argtypes = [_i32]
    L.orc_set_num_threads.restype = None
    L.orc_composite_backward.argtypes = [_p, _p, _p, _i32, _i32, _p, _p, _p]
    L.orc_project_backward.argtypes = [_i64, _i64, _p, _p, _p, _i32, _i32, _p, _p, _p]
    L.orc_skip_features.argtypes = [_i64, _p, _p, _p, _p, _p, _p, ctypes.c_float, _p]
    L.orc_skip_mlp.argtypes = [_i64, _p, _p, ctypes.c_float, _p, _p, _p, _p]
    L.orc_decode_backward.argtypes = [_i64, _p, _p, _p, _p, _p, _p, _i32, _i32, _i32, _p, _p,
                                      ctypes.c_float, _p, _p, _p, _p, _p, _p, _p]


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads the oracle's parallel loops use from now on (for timing)."""
    lib().orc_set_num_threads(int(n))


def cam_array(cam) -> np.ndarray:
    return np.concatenate([cam.R.reshape(-1), cam.C.reshape(-1),
                           [cam.fx, cam.fy, cam.cx, cam.cy, cam.z_near,
                            cam.lod_scale * cam.lod_scale]]).astype(np.float32)


def params_array(**kw) -> np.ndarray:
    p = dict(DEFAULT_PARAMS)
    p.update(kw)
    return np.array([p["alpha_max"], p["alpha_min"], p["t_min"], p["dilation"],
                     p["jac_clamp"], *p["bg"]], dtype=np.float32)


# ----------------------------------------------------------------------------
# selection
# ----------------------------------------------------------------------------

def lod_thr2(level, lod_bias, d_max) -> np.ndarray:
    level = _c(level, np.uint8)
    lod_bias = _c(lod_bias, np.float32)
    out = np.empty(len(level), np.float32)
    lib().orc_lod_thr2(len(level), _ptr(level), _ptr(lod_bias), float(d_max), _ptr(out))
    return out


def bound_radius(offsets, offset_scale, base_scale) -> np.ndarray:
    offsets = _c(offsets, np.float32)
    n, k = offsets.shape[0], offsets.shape[1]
    out = np.empty(n, np.float32)
    lib().orc_bound_radius(n, k, _ptr(offsets), _ptr(_c(offset_scale, np.float32)),
                           _ptr(_c(base_scale, np.float32)), _ptr(out))
    return out


def bound_radius_explicit(pos, mean, log_scale) -> np.ndarray:
    """Canonical FP32 bound radius of anchors carrying explicit Gaussians."""
    mean = _c(mean, np.float32)
    n, k = mean.shape[0], mean.shape[1]
    out = np.empty(n, np.float32)
    lib().orc_bound_radius_explicit(n, k, _ptr(_c(pos, np.float32)), _ptr(mean),
                                    _ptr(_c(log_scale, np.float32)), _ptr(out))
    return out


def select_mask(pos, thr2, rho, cam, blend=False, prm=None) -> np.ndarray:
    """Canonical FP32 selection mask; blend also takes level L_hat + 1
    (LOD transition blending).  The visibility test is conservative for a
    render with raster parameters prm (default params_array())."""
    pos = _c(pos, np.float32)
    mask = np.empty(len(pos), np.uint8)
    prm = params_array() if prm is None else prm
    lib().orc_select_fp32(len(pos), _ptr(pos), _ptr(_c(thr2, np.float32)),
                          _ptr(_c(rho, np.float32)), int(blend), _ptr(cam_array(cam)),
                          cam.width, cam.height, _ptr(_c(prm, np.float32)), _ptr(mask))
    return mask


def select_eq7_mask(pos, level, lod_bias, d_max, n_levels, rho, cam, blend=False,
                    prm=None) -> np.ndarray:
    pos = _c(pos, np.float32)
    mask = np.empty(len(pos), np.uint8)
    prm = params_array() if prm is None else prm
    lib().orc_select_eq7(len(pos), _ptr(pos), _ptr(_c(level, np.uint8)),
                         _ptr(_c(lod_bias, np.float32)), float(d_max), int(n_levels),
                         _ptr(_c(rho, np.float32)), int(blend), _ptr(cam_array(cam)), cam.width,
                         cam.height, _ptr(_c(prm, np.float32)), _ptr(mask))
    return mask


def lod_blend_factor(dist, s, d_max, bias, level, n_levels) -> float:
    return float(lib().orc_lod_blend_factor(float(dist), float(s), float(d_max), float(bias),
                                            int(level), int(n_levels)))


def scene_thresholds(scene):
    """(thr2, rho) of a synth.Scene."""
    return (lod_thr2(scene.level, scene.lod_bias, scene.d_max),
            bound_radius(scene.offsets, scene.offset_scale, scene.base_scale))


def select(scene, cam, thr2=None, rho=None, blend=False, prm=None) -> np.ndarray:
    """Ascending indices of the anchors selected for cam (canonical FP32 rule)."""
    if thr2 is None or rho is None:
        thr2, rho = scene_thresholds(scene)
    return np.flatnonzero(select_mask(scene.pos, thr2, rho, cam, blend, prm)).astype(np.int64)


# ----------------------------------------------------------------------------
# decode
# ----------------------------------------------------------------------------

MLP_ORDER = ("w1_a", "b1_a", "w2_a", "b2_a", "w1_c", "b1_c", "w2_c", "b2_c",
             "w1_s", "b1_s", "w2_s", "b2_s")


def decode(scene, idx, cam, blend=False) -> np.ndarray:
    """Double-precision decode of anchors idx: planar [14][len(idx) * k].
    blend scales opacities by the LOD transition factor."""
    idx = _c(idx, np.int64)
    m, k = len(idx), scene.k
    keep = [_c(scene.mlp[name], np.float32) for name in MLP_ORDER]
    arr = (ctypes.c_void_p * 12)(*[a.ctypes.data for a in keep])
    out = np.empty((14, m * k), np.float64)
    lv, lb = _c(scene.level, np.uint8), _c(scene.lod_bias, np.float32)
    lib().orc_decode(m, _ptr(idx), _ptr(_c(scene.pos, np.float32)),
                     _ptr(_c(scene.feat, np.float32)), _ptr(_c(scene.offsets, np.float32)),
                     _ptr(_c(scene.offset_scale, np.float32)),
                     _ptr(_c(scene.base_scale, np.float32)), k, scene.feat_dim,
                     scene.width, arr, _ptr(_c(cam.C, np.float32)), float(scene.d_max), int(blend),
                     _ptr(lv), _ptr(lb), int(scene.n_levels), float(cam.lod_scale) ** 2,
                     _ptr(out))
    return out


# ----------------------------------------------------------------------------
# rasterizer
# ----------------------------------------------------------------------------

def project(gf: np.ndarray, cam, prm: np.ndarray, gd: Optional[np.ndarray] = None) -> Dict[str, np.ndarray]:
    gf = _c(gf, np.float32)
    n = gf.shape[1]
    gd = None if gd is None else _c(gd, np.float64)
    vis = np.empty(n, np.uint8)
    rect = np.empty((n, 4), np.int32)
    depth = np.empty(n, np.float32)
    proj = np.empty((n, 9), np.float64)
    cf = np.zeros((n, 5), np.float32)
    cnt = lib().orc_project(n, n, _ptr(gf), _ptr(gd), _ptr(cam_array(cam)), cam.width,
                            cam.height, _ptr(_c(prm, np.float32)), _ptr(vis), _ptr(rect),
                            _ptr(depth), _ptr(proj), _ptr(cf))
    return dict(vis=vis, rect=rect, depth=depth, proj=proj, cf=cf, n_visible=int(cnt))


def tile_test(cf_row, tx, ty, W, H) -> bool:
    """Canonical FP32 tile test of one Gaussian (cf_row = mx, my, qa, qb, qc)
    against tile (tx, ty) of a W x H image."""
    return bool(lib().orc_tile_test(_ptr(_c(cf_row, np.float32)), int(tx), int(ty), int(W),
                                    int(H)))


def count_rect_pairs(pj) -> int:
    return int(lib().orc_count_rect_pairs(len(pj["vis"]), _ptr(pj["vis"]), _ptr(pj["rect"])))


def bin_sort(pj: Dict[str, np.ndarray], cam) -> Dict[str, np.ndarray]:
    n = len(pj["vis"])
    P = int(lib().orc_count_pairs(n, _ptr(pj["vis"]), _ptr(pj["rect"]), _ptr(pj["cf"]),
                                  cam.width, cam.height))
    tiles = ((cam.width + 15) // 16) * ((cam.height + 15) // 16)
    tile_of = np.empty(max(P, 1), np.uint32)
    gid_of = np.empty(max(P, 1), np.uint32)
    ranges = np.empty((tiles, 2), np.uint32)
    lib().orc_bin_sort(n, _ptr(pj["vis"]), _ptr(pj["rect"]), _ptr(pj["cf"]), _ptr(pj["depth"]),
                       cam.width, cam.height, _ptr(tile_of), _ptr(gid_of), _ptr(ranges))
    return dict(tile_of=tile_of[:P], gid_of=gid_of[:P], ranges=ranges, n_pairs=P,
                n_rect_pairs=count_rect_pairs(pj))


def composite(pj, bs, cam, prm, weights: bool = False):
    W, H = cam.width, cam.height
    img = np.empty((3, H, W), np.float64)
    Tf = np.empty((H, W), np.float64)
    last = np.empty((H, W), np.int32)
    w = np.zeros(len(pj["vis"]), np.float64) if weights else None
    gid = bs["gid_of"] if bs["n_pairs"] > 0 else np.zeros(1, np.uint32)
    lib().orc_composite(_ptr(gid), _ptr(bs["ranges"]), _ptr(pj["proj"]), W, H,
                        _ptr(_c(prm, np.float32)), _ptr(img), _ptr(Tf), _ptr(last), _ptr(w))
    return dict(img=img, T=Tf, last=last, weights=w)


def render_bruteforce(pj, cam, prm):
    W, H = cam.width, cam.height
    img = np.empty((3, H, W), np.float64)
    Tf = np.empty((H, W), np.float64)
    n = len(pj["vis"])
    lib().orc_render_bruteforce(n, _ptr(pj["vis"]), _ptr(pj["rect"]), _ptr(pj["cf"]),
                                _ptr(pj["depth"]), _ptr(pj["proj"]), W, H,
                                _ptr(_c(prm, np.float32)), _ptr(img), _ptr(Tf))
    return dict(img=img, T=Tf)


def rasterize(gf, cam, prm, gd=None, weights=False):
    """Project, bin, sort and composite planar Gaussians (float decisions,
    double continuous values)."""
    pj = project(gf, cam, prm, gd)
    bs = bin_sort(pj, cam)
    out = composite(pj, bs, cam, prm, weights=weights)
    out.update(pj=pj, bs=bs)
    return out


def fragile(out, cam, prm, eb, slack=2e-6) -> Dict[str, np.ndarray]:
    """Tiles of a render (`out` from rasterize or render, its double
    Gaussians in out["gauss"] or out["gd"]) whose lists or pixels a decision
    near its threshold can change, when the Gaussians are decoded in FP32
    within eb[14][n] of the oracle's values (orc_fragile in the C source
    explains the margins).  Also a depth-order check: visible Gaussians
    whose depth intervals (depth -+ margin) overlap a neighbour's mark every
    tile they are listed in.  Returns flags per Gaussian (bits: 1 cull,
    2 tile test, 4 depth order, 8 rectangle), `tiles` [tiles_y][tiles_x]
    bool, the pixel mask `near_flagged` of those tiles, and `near_t_min`:
    pixels whose transmittance after the last entry, or before it where the
    pixel stopped, is within 1e-3 relative of t_min, where the stop decision
    can flip."""
    gd = _c(out["gauss"] if "gauss" in out else out["gd"], np.float64)
    n = gd.shape[1]
    pj, bs = out["pj"], out["bs"]
    W, H = cam.width, cam.height
    tx, ty = (W + 15) // 16, (H + 15) // 16
    flags = np.zeros(n, np.uint8)
    z = np.zeros(n)
    zm = np.zeros(n)
    tmask = np.zeros((ty, tx), np.uint8)
    lib().orc_fragile(n, n, _ptr(gd), _ptr(_c(eb, np.float64)), _ptr(cam_array(cam)), W, H,
                      _ptr(_c(prm, np.float32)), _ptr(pj["vis"]), _ptr(pj["rect"]), float(slack),
                      _ptr(flags), _ptr(z), _ptr(zm), _ptr(tmask))
    tiles = tmask.astype(bool)
    # depth order: visible Gaussians whose depth intervals overlap a neighbour's
    vis = np.flatnonzero(pj["vis"])
    order = vis[np.argsort(z[vis], kind="stable")]
    if len(order) > 1:
        zs, ms = z[order], zm[order]
        close = (zs[1:] - zs[:-1]) <= (ms[1:] + ms[:-1])
        hit = np.zeros(len(order), bool)
        hit[1:] |= close
        hit[:-1] |= close
        flags[order[hit]] |= 4
        if hit.any():
            dep = np.zeros(n, bool)
            dep[order[hit]] = True
            listed = bs["tile_of"][dep[bs["gid_of"]]]
            tiles.reshape(-1)[listed] = True
    near_flagged = np.repeat(np.repeat(tiles, 16, 0), 16, 1)[:H, :W]
    # the stop decision: T after the last entry, and before it for pixels
    # that stopped, within 1e-3 relative of t_min
    t_min = float(np.float32(prm[2]))
    T = out["T"]
    near_t = np.abs(T - t_min) <= 1e-3 * t_min
    ys, xs = np.nonzero((T < t_min) & (out["last"] > 0))
    if len(ys):
        e = bs["ranges"][(ys // 16) * tx + xs // 16, 0].astype(np.int64) + out["last"][ys, xs] - 1
        q = pj["proj"][bs["gid_of"][e]]
        dx, dy = xs + 0.5 - q[:, 0], ys + 0.5 - q[:, 1]
        a = np.minimum(float(np.float32(prm[0])),
                       q[:, 5] * np.exp(-0.5 * (q[:, 2] * dx * dx + q[:, 4] * dy * dy) - q[:, 3] * dx * dy))
        T_prev = T[ys, xs] / np.maximum(1.0 - a, 1e-300)
        near_t[ys, xs] |= np.abs(T_prev - t_min) <= 1e-3 * t_min
    return dict(flags=flags, tiles=tiles, near_flagged=near_flagged, near_t_min=near_t,
                n_flagged=int(np.count_nonzero(flags)))


def render(scene, cam, prm, thr2=None, rho=None, weights=False, blend=False):
    """Full path for one view: select, decode, rasterize (blend: LOD
    transition blending)."""
    idx = select(scene, cam, thr2, rho, blend, prm)
    gd = decode(scene, idx, cam, blend)
    out = rasterize(gd.astype(np.float32), cam, prm, gd=gd, weights=weights)
    out.update(idx=idx, gauss=gd)
    return out


# ----------------------------------------------------------------------------
# backward passes
# ----------------------------------------------------------------------------

def composite_backward(pj, bs, cam, prm, dimg) -> np.ndarray:
    """dL/dproj [n][9] (mx, my, ca, cb, cc, op, r, g, b) for L = sum(dimg * img)."""
    n = len(pj["vis"])
    dproj = np.zeros((n, 9), np.float64)
    gid = bs["gid_of"] if bs["n_pairs"] > 0 else np.zeros(1, np.uint32)
    lib().orc_composite_backward(_ptr(gid), _ptr(bs["ranges"]), _ptr(pj["proj"]), cam.width,
                                 cam.height, _ptr(_c(prm, np.float32)),
                                 _ptr(_c(dimg, np.float64)), _ptr(dproj))
    return dproj


def project_backward(gd, pj, cam, prm, dproj) -> np.ndarray:
    """dL/dGaussian [14][n] from dL/dproj, at double attributes gd [14][n]."""
    gd = _c(gd, np.float64)
    n = gd.shape[1]
    out = np.zeros((14, n), np.float64)
    lib().orc_project_backward(n, n, _ptr(gd), _ptr(pj["vis"]), _ptr(cam_array(cam)), cam.width,
                               cam.height, _ptr(_c(prm, np.float32)),
                               _ptr(_c(dproj, np.float64)), _ptr(out))
    return out


def decode_backward(scene, idx, cam, dgauss):
    """Gradients of the anchor arrays and MLP weights for L = sum(dgauss * decode)."""
    idx = _c(idx, np.int64)
    m, k = len(idx), scene.k
    keep = [_c(scene.mlp[name], np.float32) for name in MLP_ORDER]
    arr = (ctypes.c_void_p * 12)(*[a.ctypes.data for a in keep])
    d = dict(pos=np.zeros((scene.n, 3)), feat=np.zeros((scene.n, scene.feat_dim)),
             offsets=np.zeros((scene.n, k, 3)), offset_scale=np.zeros((scene.n, 3)),
             base_scale=np.zeros((scene.n, 3)))
    dm = {name: np.zeros(scene.mlp[name].shape) for name in MLP_ORDER}
    darr = (ctypes.c_void_p * 12)(*[dm[name].ctypes.data for name in MLP_ORDER])
    lib().orc_decode_backward(m, _ptr(idx), _ptr(_c(scene.pos, np.float32)),
                              _ptr(_c(scene.feat, np.float32)), _ptr(_c(scene.offsets, np.float32)),
                              _ptr(_c(scene.offset_scale, np.float32)),
                              _ptr(_c(scene.base_scale, np.float32)), k, scene.feat_dim,
                              scene.width, arr, _ptr(cam.C), float(scene.d_max),
                              _ptr(_c(dgauss, np.float64)), _ptr(d["pos"]), _ptr(d["feat"]),
                              _ptr(d["offsets"]), _ptr(d["offset_scale"]), _ptr(d["base_scale"]),
                              darr)
    d.update(dm)
    return d


def render_backward(scene, cam, prm, dimg, fwd=None):
    """Full-chain gradients of L = sum(dimg * render(scene, cam)) with the
    forward's discrete decisions held fixed."""
    if fwd is None:
        fwd = render(scene, cam, prm)
    dproj = composite_backward(fwd["pj"], fwd["bs"], cam, prm, dimg)
    dg = project_backward(fwd["gauss"], fwd["pj"], cam, prm, dproj)
    return decode_backward(scene, fwd["idx"], cam, dg)


# ----------------------------------------------------------------------------
# anchor-skip predictor
# ----------------------------------------------------------------------------

SKIP_ORDER = ("w1", "b1", "w2", "b2", "w3", "b3")


def skip_features(scene, idx, cam) -> np.ndarray:
    idx = _c(idx, np.int64)
    z = np.empty((len(idx), 37), np.float64)
    lib().orc_skip_features(len(idx), _ptr(idx), _ptr(_c(scene.pos, np.float32)),
                            _ptr(_c(scene.feat, np.float32)), _ptr(_c(scene.level, np.uint8)),
                            _ptr(cam.R), _ptr(cam.C), float(scene.d_max), _ptr(z))
    return z


def skip_mlp(z, net, y=None, pos_weight=1.0, grads=False):
    """(logits, loss, grads dict or None) of the predictor on rows z [B][37]."""
    z = _c(z, np.float64)
    B = z.shape[0]
    keep = [_c(net[k], np.float32) for k in SKIP_ORDER]
    arr = (ctypes.c_void_p * 6)(*[a.ctypes.data for a in keep])
    logit = np.empty(B, np.float64)
    loss = np.zeros(1, np.float64)
    g = {k: np.zeros(np.asarray(net[k]).shape, np.float64) for k in SKIP_ORDER} if grads else None
    garr = (ctypes.c_void_p * 6)(*[g[k].ctypes.data for k in SKIP_ORDER]) if grads else None
    yy = None if y is None else _c(y, np.float32)
    lib().orc_skip_mlp(B, _ptr(z), _ptr(yy), float(pos_weight), arr, _ptr(logit),
                       _ptr(loss) if y is not None else None, garr)
    return logit, (float(loss[0]) if y is not None else None), g
