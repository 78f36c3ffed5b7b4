"""Device-side scene and per-view render driver over the C ABI.

PyTorch allocates device memory and supplies the stream; every computation
of the path runs in liboctgs kernels.  There is no CPU fallback: without a
GPU or without the built library these classes raise.
"""

from __future__ import annotations

import ctypes
from typing import Dict, Optional

import numpy as np
import torch

from . import _lib as L

MLP_HEADS = ("a", "c", "s")  # opacity, colour, covariance
GAUSS_FIELDS = 14


def _dev() -> torch.device:
    if not torch.cuda.is_available():
        raise L.OctgsError("liboctgs needs a HIP device; none is visible")
    return torch.device("cuda", torch.cuda.current_device())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def stream_handle(stream: Optional[torch.cuda.Stream] = None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _events(events):
    """ctypes array of hipEvent_t handles from torch.cuda.Event objects."""
    if events is None:
        return None
    arr = (ctypes.c_void_p * len(events))()
    for i, e in enumerate(events):
        arr[i] = e.cuda_event if e is not None else None
    return arr


def make_camera(cam, lod_blend: bool = False) -> L.Camera:
    """octgs_camera from any object with R (3x3), C (3), fx, fy, cx, cy,
    width, height, z_near and lod_scale (s of Eq. 7); lod_blend turns on LOD
    transition blending."""
    c = L.Camera()
    R = np.asarray(cam.R, np.float32).reshape(9)
    C = np.asarray(cam.C, np.float32).reshape(3)
    for i in range(9):
        c.R[i] = float(R[i])
    for i in range(3):
        c.C[i] = float(C[i])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    c.z_near = float(cam.z_near)
    s = float(np.float32(getattr(cam, "lod_scale", 1.0)))
    c.lod_scale2 = float(np.float32(s) * np.float32(s))
    c.lod_blend = 1 if lod_blend else 0
    return c


def raster_params(alpha_max=0.99, alpha_min=0.0, t_min=1e-4, dilation=0.3, jac_clamp=1.3,
                  bg=(0.0, 0.0, 0.0), train: bool = False,
                  tile_order=None) -> L.RasterParams:
    """Rasterizer constants; train=True makes the forward keep what the
    backward pass needs (required before rasterize_bwd).  tile_order orders
    each XCD's tiles longest-first before compositing (faster for a frame
    that runs alone on the GPU, slower with several frames in flight); it
    defaults to train."""
    p = L.RasterParams()
    p.alpha_max, p.alpha_min, p.t_min = alpha_max, alpha_min, t_min
    p.dilation, p.jac_clamp = dilation, jac_clamp
    for i in range(3):
        p.bg[i] = bg[i]
    if tile_order is None:
        tile_order = train
    p.flags = (L.OCTGS_RASTER_TRAIN if train else 0) | (L.OCTGS_RASTER_TILE_ORDER if tile_order else 0)
    return p


def raise_on_status(bits: int, what: str = "frames"):
    """Raise OctgsError naming the OCTGS_STATUS_* bits set in `bits`."""
    if bits:
        names = [n for b, n in ((L.OCTGS_STATUS_PAIR_OVERFLOW, "pair list overflow"),
                                (L.OCTGS_STATUS_SYNC_ERROR, "look-back wait bound"),
                                (L.OCTGS_STATUS_TRUNCATED, "decode truncated at the Gaussian "
                                                           "capacity")) if bits & b]
        raise L.OctgsError(f"{what}: " + ", ".join(names))


class _nullctx:
    def __enter__(self):
        return self

    def __exit__(self, *exc):
        return False


class DeviceScene:
    """An anchor set resident in HBM, with its per-scene Eq. 7 thresholds."""

    def __init__(self, pos, level, lod_bias, feat, offsets, offset_scale, base_scale, mlp: Dict,
                 d_max: float, n_levels: int, k: int, width: int, stream=None):
        dev = _dev()
        f32 = dict(dtype=torch.float32, device=dev)
        self.n = int(np.asarray(pos).shape[0])
        self.k, self.width, self.n_levels = int(k), int(width), int(n_levels)
        self.feat_dim = int(np.asarray(feat).shape[1])
        self.d_max = float(np.float32(d_max))
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(**f32)
        self.pos = t(pos)
        self.level = torch.as_tensor(np.ascontiguousarray(level, np.uint8)).to(dev)
        self.lod_bias = t(lod_bias)
        self.feat = t(feat)
        # BF16 copy for the fast path, written by octgs_prepare_anchors
        self.feat_bf16 = torch.empty(self.feat.shape, dtype=torch.int16, device=dev)
        self.offsets = t(offsets)
        self.offset_scale = t(offset_scale)
        self.base_scale = t(base_scale)
        self.mlp = {kk: t(v) for kk, v in mlp.items()}
        self.thr2 = torch.empty(self.n, **f32)
        self.bound_r = torch.empty(self.n, **f32)
        self._anchors = self._make_anchors()
        self.refresh(stream)
        self._mlp = L.Mlp()
        self._mlp.width = self.width
        for h, name in enumerate(MLP_HEADS):
            self._mlp.w1[h] = self.mlp["w1_" + name].data_ptr()
            self._mlp.b1[h] = self.mlp["b1_" + name].data_ptr()
            self._mlp.w2[h] = self.mlp["w2_" + name].data_ptr()
            self._mlp.b2[h] = self.mlp["b2_" + name].data_ptr()

    def refresh(self, stream=None, bf16: bool = True):
        """Recompute what the library derives from the trained arrays: the
        Eq. 7 thresholds (lod_bias), the bound radii (offsets, offset_scale,
        base_scale) and, unless bf16 is False, the BF16 feature copy.  Needed
        after every update of those arrays (an optimiser step, a LOD-bias
        update) before the next selection or decode.  A BF16 decode after a
        refresh without the copy raises until the copy is refreshed."""
        L.check(L.lib().octgs_prepare_anchors(ctypes.byref(self._anchors), _ptr(self.thr2),
                                             _ptr(self.bound_r),
                                             _ptr(self.feat_bf16) if bf16 else None,
                                             stream_handle(stream)), "octgs_prepare_anchors")
        self.bf16_valid = bool(bf16)

    @classmethod
    def from_scene(cls, sc, stream=None) -> "DeviceScene":
        return cls(sc.pos, sc.level, sc.lod_bias, sc.feat, sc.offsets, sc.offset_scale,
                   sc.base_scale, sc.mlp, sc.d_max, sc.n_levels, sc.k, sc.width, stream)

    def _make_anchors(self) -> L.Anchors:
        a = L.Anchors()
        a.n, a.k, a.feat_dim, a.n_levels, a.d_max = self.n, self.k, self.feat_dim, self.n_levels, self.d_max
        a.pos = self.pos.data_ptr() if self.n else None
        a.level = self.level.data_ptr() if self.n else None
        a.lod_bias = self.lod_bias.data_ptr() if self.n else None
        a.feat = self.feat.data_ptr() if self.n else None
        a.feat_bf16 = self.feat_bf16.data_ptr() if self.n else None
        a.offsets = self.offsets.data_ptr() if self.n else None
        a.offset_scale = self.offset_scale.data_ptr() if self.n else None
        a.base_scale = self.base_scale.data_ptr() if self.n else None
        a.thr2 = getattr(self, "thr2", None).data_ptr() if hasattr(self, "thr2") and self.n else None
        a.bound_r = self.bound_r.data_ptr() if hasattr(self, "bound_r") and self.n else None
        return a

    @property
    def anchors(self) -> L.Anchors:
        return self._anchors


EXPLICIT_FIELDS = ("mean", "log_scale", "rot", "opacity", "sh")


class DeviceExplicit:
    """Anchors carrying k explicit 3D Gaussians each (the 3D-GS instance of
    the framework), resident in HBM with their Eq. 7 thresholds and bound
    radii.  The SH coefficients are also kept as BF16 for OCTGS_BF16."""

    def __init__(self, pos, level, lod_bias, mean, log_scale, rot, opacity, sh, sh_degree: int,
                 d_max: float, n_levels: int, stream=None):
        dev = _dev()
        f32 = dict(dtype=torch.float32, device=dev)
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(**f32)
        self.n = int(np.asarray(pos).shape[0])
        self.k = int(np.asarray(mean).shape[1])
        self.sh_degree, self.n_levels = int(sh_degree), int(n_levels)
        self.d_max = float(np.float32(d_max))
        self.pos = t(pos)
        self.level = torch.as_tensor(np.ascontiguousarray(level, np.uint8)).to(dev)
        self.lod_bias = t(lod_bias)
        self.mean, self.log_scale, self.rot = t(mean), t(log_scale), t(rot)
        self.opacity, self.sh = t(opacity), t(sh)
        # BF16 copy of the coefficients, written by octgs_prepare_explicit
        self.sh_bf16 = torch.empty(self.sh.shape, dtype=torch.int16, device=dev)
        self.thr2 = torch.empty(max(1, self.n), **f32)
        self.bound_r = torch.empty(max(1, self.n), **f32)
        self._ex = L.Explicit()
        self._ex.sh_degree = self.sh_degree
        for name in EXPLICIT_FIELDS:
            setattr(self._ex, name, getattr(self, name).data_ptr() if self.n else None)
        self._ex.sh_bf16 = self.sh_bf16.data_ptr() if self.n else None
        a = L.Anchors()
        a.n, a.k, a.feat_dim, a.n_levels, a.d_max = self.n, self.k, 0, self.n_levels, self.d_max
        if self.n:
            a.pos, a.level, a.lod_bias = (self.pos.data_ptr(), self.level.data_ptr(),
                                          self.lod_bias.data_ptr())
            a.thr2, a.bound_r = self.thr2.data_ptr(), self.bound_r.data_ptr()
        self._anchors = a
        self.refresh(stream)

    def refresh(self, stream=None):
        """Recompute the Eq. 7 thresholds, bound radii and the BF16 SH copy
        from the current arrays (after any update of them)."""
        L.check(L.lib().octgs_prepare_explicit(ctypes.byref(self._anchors), ctypes.byref(self._ex),
                                              _ptr(self.thr2), _ptr(self.bound_r),
                                              _ptr(self.sh_bf16) if self.n else None,
                                              stream_handle(stream)), "octgs_prepare_explicit")

    @classmethod
    def from_scene(cls, ex, stream=None) -> "DeviceExplicit":
        return cls(ex.pos, ex.level, ex.lod_bias, ex.mean, ex.log_scale, ex.rot, ex.opacity,
                   ex.sh, ex.sh_degree, ex.d_max, ex.n_levels, stream)

    @property
    def anchors(self) -> L.Anchors:
        return self._anchors


class ExplicitGrads:
    """Device gradient buffers shaped like a DeviceExplicit's arrays."""

    def __init__(self, ex: DeviceExplicit):
        self.arrays = {n: torch.zeros_like(getattr(ex, n)) for n in EXPLICIT_FIELDS}
        self._g = L.ExplicitGrads(*[self.arrays[n].data_ptr() for n in EXPLICIT_FIELDS])

    def zero_(self):
        for t in self.arrays.values():
            t.zero_()


class DensifyStats:
    """Device statistics of one densification interval (Sec. IV-B) for n
    anchors of k Gaussians, and the decision outputs."""

    def __init__(self, n: int, k: int):
        dev = _dev()
        self.n, self.k = int(n), int(k)
        self.grad_sum = torch.zeros(max(1, n * k), dtype=torch.float32, device=dev)
        self.grad_count = torch.zeros(max(1, n * k), dtype=torch.int32, device=dev)
        self.opacity_sum = torch.zeros(max(1, n), dtype=torch.float32, device=dev)
        self.view_count = torch.zeros(max(1, n), dtype=torch.int32, device=dev)
        self.grow_level = torch.empty(max(1, n * k), dtype=torch.int8, device=dev)
        self.prune = torch.empty(max(1, n), dtype=torch.uint8, device=dev)
        self.counts = torch.zeros(4, dtype=torch.int32, device=dev)
        self._st = L.DensifyStats(self.grad_sum.data_ptr(), self.grad_count.data_ptr(),
                                  self.opacity_sum.data_ptr(), self.view_count.data_ptr())

    def zero_(self):
        for t in (self.grad_sum, self.grad_count, self.opacity_sum, self.view_count):
            t.zero_()

    def accumulate(self, vb: "ViewBuffers", cam: L.Camera, idx: Optional[torch.Tensor] = None,
                   count: Optional[torch.Tensor] = None, stream=None):
        """Add the view last rendered and back-propagated with vb."""
        idx = vb.sel_idx if idx is None else idx
        count = vb.sel_count if count is None else count
        L.check(L.lib().octgs_densify_accumulate(ctypes.byref(vb._g), ctypes.byref(cam), vb.pcap,
                                                 _ptr(vb.ras_ws), vb.ras_ws.numel(), _ptr(idx),
                                                 _ptr(count), self.k, ctypes.byref(self._st),
                                                 stream_handle(stream)),
                "octgs_densify_accumulate")

    def decide(self, scene, n_views: int, tau_g=2e-4, beta=0.2, epsilon=0.01,
               tau_opacity=0.005, tau_v=0.01, stream=None):
        """Growth levels, pruning mask and counts; updates scene.lod_bias in
        place (rerun the scene's threshold preparation afterwards)."""
        p = L.DensifyParams(tau_g, beta, epsilon, tau_opacity, tau_v, int(n_views))
        L.check(L.lib().octgs_densify_decide(ctypes.byref(scene.anchors), ctypes.byref(self._st),
                                             ctypes.byref(p), _ptr(scene.lod_bias),
                                             _ptr(self.grow_level), _ptr(self.prune),
                                             _ptr(self.counts), stream_handle(stream)),
                "octgs_densify_decide")


PARAM_NAMES = ("pos", "feat", "offsets", "offset_scale", "base_scale")


class SceneGrads:
    """Device gradient buffers shaped like a DeviceScene's trainable arrays."""

    def __init__(self, scene: "DeviceScene"):
        # one flat buffer (each array 256-byte aligned), so zeroing is one launch
        shapes = [(n, getattr(scene, n).shape) for n in PARAM_NAMES]
        shapes += [(k, v.shape) for k, v in scene.mlp.items()]
        sizes = [int(np.prod(sh)) for _, sh in shapes]
        offs, o = [], 0
        for n_ in sizes:
            offs.append(o)
            o += (n_ + 63) // 64 * 64
        self.flat = torch.zeros(max(o, 1), dtype=torch.float32, device=scene.pos.device)
        views = {name: self.flat[off:off + n_].view(sh)
                 for (name, sh), off, n_ in zip(shapes, offs, sizes)}
        self.arrays = {n: views[n] for n in PARAM_NAMES}
        self.mlp = {k: views[k] for k in scene.mlp}
        self._ag = L.AnchorGrads(*[self.arrays[n].data_ptr() for n in PARAM_NAMES])
        self._mg = L.MlpGrads()
        for h, name in enumerate(MLP_HEADS):
            self._mg.w1[h] = self.mlp["w1_" + name].data_ptr()
            self._mg.b1[h] = self.mlp["b1_" + name].data_ptr()
            self._mg.w2[h] = self.mlp["w2_" + name].data_ptr()
            self._mg.b2[h] = self.mlp["b2_" + name].data_ptr()

    def zero_(self):
        self.flat.zero_()

    def all(self) -> Dict[str, torch.Tensor]:
        d = dict(self.arrays)
        d.update(self.mlp)
        return d


def l1_loss_grad(img: torch.Tensor, target: torch.Tensor, scale: float, dimg: torch.Tensor,
                 loss: torch.Tensor, stream=None):
    L.check(L.lib().octgs_l1_loss_grad(_ptr(img), _ptr(target), img.numel(), float(scale),
                                       _ptr(dimg), _ptr(loss), stream_handle(stream)),
            "octgs_l1_loss_grad")


def photometric_loss_grad(img: torch.Tensor, target: torch.Tensor, dimg: torch.Tensor,
                          loss: torch.Tensor, w_l1: float = 0.8, w_ssim: float = 0.2,
                          ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """w_l1 L1 + w_ssim (1 - SSIM) over images [..., H, W] (each leading
    index one plane); dimg receives the gradient, loss (device scalar) is
    incremented.  Returns the workspace used (pass it back to reuse it)."""
    H, W = int(img.shape[-2]), int(img.shape[-1])
    planes = img.numel() // max(1, H * W)
    need = L.lib().octgs_photometric_workspace_bytes(planes, H, W)
    if w_ssim != 0.0 and (ws is None or ws.numel() < need):
        ws = torch.empty(need, dtype=torch.uint8, device=img.device)
    L.check(L.lib().octgs_photometric_loss_grad(_ptr(img), _ptr(target), planes, H, W,
                                                float(w_l1), float(w_ssim), _ptr(dimg),
                                                _ptr(loss), _ptr(ws),
                                                0 if ws is None else ws.numel(),
                                                stream_handle(stream)),
            "octgs_photometric_loss_grad")
    return ws


def adam_step(param: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
              lr: float, step: int, beta1=0.9, beta2=0.999, eps=1e-15, stream=None):
    L.check(L.lib().octgs_adam_step(_ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.numel(),
                                    float(lr), float(beta1), float(beta2), float(eps), int(step),
                                    stream_handle(stream)), "octgs_adam_step")


class AdamMany:
    """One Adam update of several device arrays per launch; the pointer
    tables are built once for a fixed list of (param, grad, m, v)."""

    def __init__(self, params, grads, moments):
        cnt = len(params)
        arr = lambda ts: (ctypes.c_void_p * max(1, cnt))(*[t.data_ptr() for t in ts])
        self.count = cnt
        self._p = arr(params)
        self._g = arr(grads)
        self._m = arr([m for m, _ in moments])
        self._v = arr([v for _, v in moments])
        self._n = (ctypes.c_int64 * max(1, cnt))(*[p.numel() for p in params])
        self._keep = (params, grads, moments)

    def step(self, lr: float, step: int, beta1=0.9, beta2=0.999, eps=1e-15, stream=None):
        L.check(L.lib().octgs_adam_step_many(self.count, self._p, self._g, self._m, self._v,
                                             self._n, float(lr), float(beta1), float(beta2),
                                             float(eps), int(step), stream_handle(stream)),
                "octgs_adam_step_many")


class ViewBuffers:
    """Per-view device buffers: selection, decoded Gaussians, rasterizer
    workspace and outputs, sized for a scene, an image and a pair capacity."""

    def __init__(self, n_anchors: int, k: int, width: int, height: int, pair_capacity: int,
                 gauss_capacity: Optional[int] = None, log_weights: bool = False):
        dev = _dev()
        lib = L.lib()
        self.n, self.k, self.W, self.H = int(n_anchors), int(k), int(width), int(height)
        self.gcap = int(gauss_capacity if gauss_capacity is not None else max(1, self.n) * k)
        self.pcap = int(pair_capacity)
        self.sel_idx = torch.empty(max(1, self.n), dtype=torch.int32, device=dev)
        self.sel_count = torch.zeros(1, dtype=torch.int32, device=dev)
        sw = lib.octgs_select_workspace_bytes(self.n)
        self.sel_ws = torch.empty(max(256, sw), dtype=torch.uint8, device=dev)
        self.gauss = torch.empty((GAUSS_FIELDS, self.gcap), dtype=torch.float32, device=dev)
        self.gauss_count = torch.zeros(1, dtype=torch.int32, device=dev)
        rw = lib.octgs_raster_workspace_bytes(self.gcap, self.pcap, self.W, self.H)
        if rw == 0:
            raise L.OctgsError("bad rasterizer sizes")
        self.ras_ws = torch.empty(rw, dtype=torch.uint8, device=dev)
        self.rgb = torch.empty((3, self.H, self.W), dtype=torch.float32, device=dev)
        self.T = torch.empty((self.H, self.W), dtype=torch.float32, device=dev)
        self.last = torch.empty((self.H, self.W), dtype=torch.int32, device=dev)
        self.gauss_w = torch.empty(self.gcap, dtype=torch.float32, device=dev) if log_weights else None
        # OCTGS_STATUS_* bits of every frame decoded and rasterized with these
        # buffers since the last clear_status (the library ORs them in)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self._g = L.Gaussians()
        self._g.capacity = self.gcap
        self._g.data = self.gauss.data_ptr()
        self._g.count = self.gauss_count.data_ptr()
        self._g.status = self.status.data_ptr()

    # ---- frame status ----
    def clear_status(self, stream=None):
        """Zero the status word (enqueued on `stream`)."""
        with torch.cuda.stream(stream) if stream is not None else _nullctx():
            self.status.zero_()

    def check_status(self, what: str = "frames"):
        """Raise if any frame since the last clear flagged a pair-list
        overflow, a look-back wait bound or a truncated decode (syncs), then
        clear the word."""
        bits = int(self.status.item())
        self.status.zero_()
        raise_on_status(bits, what)

    # ---- stages ----
    def select(self, scene, cam: L.Camera, params: Optional[L.RasterParams] = None, stream=None):
        """Eq. 7 selection over a DeviceScene or a DeviceExplicit; the
        visibility test is conservative for a render with `params` (default
        raster_params())."""
        params = raster_params() if params is None else params
        L.check(L.lib().octgs_select_lod(ctypes.byref(scene.anchors), ctypes.byref(cam),
                                         ctypes.byref(params), _ptr(self.sel_idx),
                                         _ptr(self.sel_count), _ptr(self.sel_ws),
                                         self.sel_ws.numel(), stream_handle(stream)),
                "octgs_select_lod")

    def decode(self, scene: DeviceScene, cam: L.Camera, precision: int = L.OCTGS_FP32,
               idx: Optional[torch.Tensor] = None, count: Optional[torch.Tensor] = None,
               stream=None):
        idx = self.sel_idx if idx is None else idx
        count = self.sel_count if count is None else count
        if int(precision) == L.OCTGS_BF16 and not getattr(scene, "bf16_valid", True):
            raise L.OctgsError("the BF16 feature copy is stale: call scene.refresh() first")
        lib = L.lib()
        need = lib.octgs_decode_workspace_bytes(int(precision))
        if getattr(self, "dec_fwd_ws", None) is None or self.dec_fwd_ws.numel() < need:
            self.dec_fwd_ws = torch.empty(max(need, 16), dtype=torch.uint8,
                                          device=self.gauss.device)
        L.check(lib.octgs_decode(ctypes.byref(scene.anchors), ctypes.byref(scene._mlp),
                                 ctypes.byref(cam), _ptr(idx), _ptr(count), int(precision),
                                 ctypes.byref(self._g), _ptr(self.dec_fwd_ws),
                                 self.dec_fwd_ws.numel(), stream_handle(stream)), "octgs_decode")

    def decode_explicit(self, ex: "DeviceExplicit", cam: L.Camera, precision: int = L.OCTGS_FP32,
                        idx: Optional[torch.Tensor] = None, count: Optional[torch.Tensor] = None,
                        stream=None):
        idx = self.sel_idx if idx is None else idx
        count = self.sel_count if count is None else count
        L.check(L.lib().octgs_decode_explicit(ctypes.byref(ex.anchors), ctypes.byref(ex._ex),
                                              ctypes.byref(cam), _ptr(idx), _ptr(count),
                                              int(precision), ctypes.byref(self._g),
                                              stream_handle(stream)), "octgs_decode_explicit")

    def render_explicit(self, ex: "DeviceExplicit", cam: L.Camera, params: L.RasterParams,
                        precision: int = L.OCTGS_FP32, stream=None, stage_events=None,
                        keep_last: bool = True):
        self.select(ex, cam, params, stream=stream)
        self.decode_explicit(ex, cam, precision, stream=stream)
        self.rasterize(cam, params, stream=stream, stage_events=stage_events,
                       keep_last=keep_last)

    def decode_explicit_bwd(self, ex: "DeviceExplicit", cam: L.Camera, grads: "ExplicitGrads",
                            dgauss: Optional[torch.Tensor] = None,
                            idx: Optional[torch.Tensor] = None,
                            count: Optional[torch.Tensor] = None, stream=None):
        dg = self.dgauss if dgauss is None else dgauss
        idx = self.sel_idx if idx is None else idx
        count = self.sel_count if count is None else count
        L.check(L.lib().octgs_decode_explicit_bwd(ctypes.byref(ex.anchors), ctypes.byref(ex._ex),
                                                  ctypes.byref(cam), _ptr(idx), _ptr(count),
                                                  _ptr(dg), dg.shape[1], ctypes.byref(grads._g),
                                                  stream_handle(stream)),
                "octgs_decode_explicit_bwd")

    def rasterize(self, cam: L.Camera, params: L.RasterParams, gauss: Optional[torch.Tensor] = None,
                  count: Optional[torch.Tensor] = None, stream=None, stage_events=None,
                  keep_last: bool = True):
        """Forward rasterization into self.rgb and self.T; self.last (the
        per-pixel list entry count the backward replays from) only with
        keep_last, which a render that no backward follows may leave off."""
        g = self._g
        if gauss is not None:
            g = L.Gaussians()
            g.capacity = gauss.shape[1]
            g.data = gauss.data_ptr()
            g.count = count.data_ptr()
            g.status = self.status.data_ptr()
            if gauss.shape[1] != self.gcap:
                raise L.OctgsError("Gaussian buffer capacity must equal the workspace capacity")
        L.check(L.lib().octgs_rasterize_fwd(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(params),
                                            self.pcap, _ptr(self.rgb), _ptr(self.T),
                                            _ptr(self.last) if keep_last else None,
                                            _ptr(self.gauss_w), _ptr(self.ras_ws), self.ras_ws.numel(),
                                            _events(stage_events), stream_handle(stream)),
                "octgs_rasterize_fwd")
        self.last_valid = bool(keep_last)

    def render(self, scene: DeviceScene, cam: L.Camera, params: L.RasterParams,
               precision: int = L.OCTGS_FP32, stream=None, stage_events=None,
               keep_last: bool = True):
        self.select(scene, cam, params, stream=stream)
        self.decode(scene, cam, precision, stream=stream)
        self.rasterize(cam, params, stream=stream, stage_events=stage_events,
                       keep_last=keep_last)

    def volume_loss_grad(self, weight: float, loss: torch.Tensor, stream=None):
        """Adds weight * sum Prod(s) over the decoded, rendered slots to loss and
        its gradient to self.dgauss (after rasterize_bwd)."""
        L.check(L.lib().octgs_volume_loss_grad(ctypes.byref(self._g), float(weight),
                                               _ptr(self.dgauss), _ptr(loss),
                                               stream_handle(stream)), "octgs_volume_loss_grad")

    def rasterize_bwd(self, cam: L.Camera, params: L.RasterParams, dimg: torch.Tensor,
                      stream=None, stage_events=None):
        """dL/dGaussian planar [14][gcap] into self.dgauss, for the image of
        the last rasterize() with these buffers."""
        if not getattr(self, "last_valid", False):
            raise L.OctgsError("rasterize_bwd needs a forward rasterize() with keep_last=True")
        if getattr(self, "dgauss", None) is None:
            self.dgauss = torch.empty_like(self.gauss)
        L.check(L.lib().octgs_rasterize_bwd(ctypes.byref(self._g), ctypes.byref(cam),
                                            ctypes.byref(params), self.pcap, _ptr(self.T),
                                            _ptr(self.last), _ptr(dimg.contiguous()),
                                            _ptr(self.dgauss), _ptr(self.ras_ws),
                                            self.ras_ws.numel(), _events(stage_events),
                                            stream_handle(stream)),
                "octgs_rasterize_bwd")

    def _dec_ws(self, scene: "DeviceScene", cap: int):
        need = L.lib().octgs_decode_bwd_workspace_bytes(cap // self.k, self.k, scene.width)
        if getattr(self, "dec_ws", None) is None or self.dec_ws.numel() < need:
            self.dec_ws = torch.empty(need, dtype=torch.uint8, device=self.gauss.device)
        return self.dec_ws

    def decode_bwd(self, scene: "DeviceScene", cam: L.Camera, grads: SceneGrads,
                   dgauss: Optional[torch.Tensor] = None, idx: Optional[torch.Tensor] = None,
                   count: Optional[torch.Tensor] = None, stream=None):
        """Decode backward of the listed anchors (default: the last
        selection), added into grads."""
        dg = self.dgauss if dgauss is None else dgauss
        idx = self.sel_idx if idx is None else idx
        count = self.sel_count if count is None else count
        ws = self._dec_ws(scene, dg.shape[1])
        L.check(L.lib().octgs_decode_bwd(ctypes.byref(scene.anchors), ctypes.byref(scene._mlp),
                                         ctypes.byref(cam), _ptr(idx), _ptr(count), _ptr(dg),
                                         dg.shape[1], ctypes.byref(grads._ag),
                                         ctypes.byref(grads._mg), _ptr(ws), ws.numel(),
                                         stream_handle(stream)), "octgs_decode_bwd")

    def decode_bwd_rows(self, scene: "DeviceScene", cam: L.Camera, stream=None):
        """The first half of decode_bwd for the last selection: gradient rows
        and weight partial sums into this buffer set's workspace, no gradient
        array touched (views in flight run theirs at the same time)."""
        ws = self._dec_ws(scene, self.dgauss.shape[1])
        L.check(L.lib().octgs_decode_bwd_rows(ctypes.byref(scene.anchors), ctypes.byref(scene._mlp),
                                              ctypes.byref(cam), _ptr(self.sel_idx),
                                              _ptr(self.sel_count), _ptr(self.dgauss),
                                              self.dgauss.shape[1], _ptr(ws), ws.numel(),
                                              stream_handle(stream)), "octgs_decode_bwd_rows")

    def decode_bwd_apply(self, scene: "DeviceScene", grads: SceneGrads, stream=None):
        """The second half: add the rows of the last decode_bwd_rows into
        grads (order the applies of views that share grads)."""
        ws = self._dec_ws(scene, self.dgauss.shape[1])
        L.check(L.lib().octgs_decode_bwd_apply(ctypes.byref(scene.anchors), ctypes.byref(scene._mlp),
                                               _ptr(self.sel_idx), _ptr(self.sel_count),
                                               self.dgauss.shape[1], ctypes.byref(grads._ag),
                                               ctypes.byref(grads._mg), _ptr(ws), ws.numel(),
                                               stream_handle(stream)), "octgs_decode_bwd_apply")

    # ---- readback helpers (synchronise) ----
    def stats(self) -> Dict[str, int]:
        torch.cuda.synchronize()
        h = self.ras_ws[:64].cpu().numpy().view(np.uint32)
        return dict(n_slots=int(h[0]), n_visible=int(h[1]), n_pairs=int(h[2]),
                    pair_overflow=int(h[3]), sync_error=int(h[4]), n_candidates=int(h[5]),
                    n_selected=int(self.sel_count.item()))

    def sorted_lists(self):
        """(pair_tile, pair_slot, ranges) as CPU numpy arrays, after a forward."""
        lib = L.lib()
        st, pt, ps, rg = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        L.check(lib.octgs_raster_views(_ptr(self.ras_ws), self.gcap, self.pcap, self.W, self.H,
                                       ctypes.byref(st), ctypes.byref(pt), ctypes.byref(ps),
                                       ctypes.byref(rg)), "octgs_raster_views")
        s = self.stats()
        P = s["n_pairs"]
        base = self.ras_ws.data_ptr()
        ws32 = self.ras_ws.view(torch.int32)

        def view(ptr, n):
            off = (ptr.value - base) // 4
            return ws32[off:off + n].cpu().numpy().view(np.uint32).copy()

        ntiles = ((self.W + 15) // 16) * ((self.H + 15) // 16)
        return view(pt, P), view(ps, P), view(rg, 2 * ntiles).reshape(ntiles, 2)


class RenderFn(torch.autograd.Function):
    """Differentiable view render: decode + rasterize forward through the
    library, backward through octgs_rasterize_bwd and octgs_decode_bwd
    (params made with raster_params(train=True)).
    The inputs after the first four are the scene's trainable tensors (the
    ones the DeviceScene points to), in PARAM_NAMES then sorted MLP-key order;
    their gradients are returned."""

    @staticmethod
    def forward(ctx, vb, scene, cam, params, *tensors):
        # the trained tensors may have changed in place since the last call
        scene.refresh(bf16=False)  # this render decodes in FP32
        vb.status.zero_()
        vb.render(scene, cam, params, precision=L.OCTGS_FP32)
        vb.check_status("RenderFn forward")
        ctx.vb, ctx.scene, ctx.cam, ctx.params = vb, scene, cam, params
        return vb.rgb.clone()

    @staticmethod
    def backward(ctx, dimg):
        vb, scene, cam, params = ctx.vb, ctx.scene, ctx.cam, ctx.params
        vb.rasterize_bwd(cam, params, dimg.contiguous())
        grads = SceneGrads(scene)
        vb.decode_bwd(scene, cam, grads)
        g = grads.all()
        out = [g[n] for n in PARAM_NAMES] + [g[k] for k in sorted(scene.mlp)]
        return (None, None, None, None, *out)


def trainable(scene: "DeviceScene"):
    """The tensors RenderFn differentiates, in its argument order."""
    return [getattr(scene, n) for n in PARAM_NAMES] + [scene.mlp[k] for k in sorted(scene.mlp)]


def render_diff(vb: "ViewBuffers", scene: "DeviceScene", cam: L.Camera, params: L.RasterParams):
    return RenderFn.apply(vb, scene, cam, params, *trainable(scene))
