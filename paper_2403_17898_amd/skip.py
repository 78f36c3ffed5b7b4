"""Learned anchor skip: predictor weights, training and the skip render path.

The predictor decides, per view and per selected anchor, whether the anchor's
Gaussians would contribute to the image; anchors predicted not to are left
out before decoding.  Training data are the per-anchor blend weights the
rasterizer logs (sum over pixels of a_i T_i of the anchor's Gaussians) on
training views; the label is weight > tau.  All arithmetic runs in liboctgs
kernels; this module allocates buffers, samples rows and drives the loop.
"""

from __future__ import annotations

import ctypes
import math
from typing import Dict, List, Optional

import numpy as np
import torch

from . import _lib as L
from .render import DeviceScene, ViewBuffers, _ptr, adam_step, stream_handle

SKIP_ORDER = ("w1", "b1", "w2", "b2", "w3", "b3")
Z_DIM, HID = 37, 64


# columns of the predictor input z: the anchor feature, the camera-frame
# viewing direction, log2 of the distance over d_max, the octree level
Z_FEATURE, Z_DIRECTION, Z_LOG_DISTANCE, Z_LEVEL = range(0, 32), range(32, 35), 35, 36


class SkipNet:
    """FP32 master weights of the 37 -> 64 -> 64 -> 1 predictor, with their
    gradient buffers and Adam moments, on the current device.  `inputs`
    restricts the network to some columns of z (the first layer's other
    rows are held at zero): the same network and kernels then implement a
    rule on, say, the distance alone."""

    def __init__(self, seed: int = 0, inputs=None):
        dev = torch.device("cuda", torch.cuda.current_device())
        g = torch.Generator().manual_seed(seed)
        used = list(range(Z_DIM)) if inputs is None else sorted(set(inputs))
        # bit i set: input i is read (the training kernel zeroes the others)
        self.input_mask = sum(1 << i for i in used)

        def xavier(i, o, rows=None):
            a = math.sqrt(6.0 / (i + o))
            w = (torch.rand(i, o, generator=g) * 2 - 1) * a
            if rows is not None:
                keep = torch.zeros(i, 1)
                keep[rows] = 1.0
                w = w * keep  # host-side initialisation
            return w.to(dev)

        self.w = {"w1": xavier(Z_DIM, HID, used), "b1": torch.zeros(HID, device=dev),
                  "w2": xavier(HID, HID), "b2": torch.zeros(HID, device=dev),
                  "w3": xavier(HID, 1), "b3": torch.zeros(1, device=dev)}
        self.g = {k: torch.zeros_like(v) for k, v in self.w.items()}
        self.m = {k: torch.zeros_like(v) for k, v in self.w.items()}
        self.v = {k: torch.zeros_like(v) for k, v in self.w.items()}
        self.step = 0
        self._ws = None

    def struct(self) -> L.SkipNet:
        return L.SkipNet(*[self.w[k].data_ptr() for k in SKIP_ORDER])

    def grad_struct(self) -> L.SkipNet:
        return L.SkipNet(*[self.g[k].data_ptr() for k in SKIP_ORDER])

    def numpy(self) -> Dict[str, np.ndarray]:
        return {k: v.detach().cpu().numpy() for k, v in self.w.items()}

    def train_grad(self, z: torch.Tensor, y: torch.Tensor, pos_weight: float, loss: torch.Tensor,
                   rows: Optional[torch.Tensor] = None, batch: Optional[int] = None):
        """Gradients of the batch rows `rows` (int32 row indices of z and y;
        None: all rows of z) into self.g; adds the batch loss to `loss`."""
        B = int(batch if batch is not None else (rows.numel() if rows is not None else z.shape[0]))
        if rows is not None:
            assert rows.dtype == torch.int32 and rows.numel() >= B
        need = L.lib().octgs_skip_train_workspace_bytes(B)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=z.device)
        net, gr = self.struct(), self.grad_struct()
        L.check(L.lib().octgs_skip_train_grad(ctypes.byref(net), _ptr(z), _ptr(y),
                                              _ptr(rows), B,
                                              self.input_mask, float(pos_weight),
                                              ctypes.byref(gr), _ptr(loss), _ptr(self._ws),
                                              self._ws.numel(), stream_handle()),
                "octgs_skip_train_grad")

    def adam(self, lr: float):
        self.step += 1
        for k in SKIP_ORDER:
            adam_step(self.w[k], self.g[k], self.m[k], self.v[k], lr, self.step, eps=1e-8)


class SkipBuffers:
    """Per-view skip buffers sized for a ViewBuffers."""

    def __init__(self, vb: ViewBuffers):
        dev = vb.gauss.device
        cap = max(1, vb.n)
        self.cap = cap
        self.keep_idx = torch.empty(cap, dtype=torch.int32, device=dev)
        self.keep_count = torch.zeros(1, dtype=torch.int32, device=dev)
        self.logits = torch.empty(cap, dtype=torch.float32, device=dev)
        self.ws = torch.empty(max(256, L.lib().octgs_skip_predict_workspace_bytes(cap)),
                              dtype=torch.uint8, device=dev)


def predict(vb: ViewBuffers, sb: SkipBuffers, scene: DeviceScene, cam: L.Camera, net: SkipNet,
            logit_threshold: float, keep_logits: bool = False, stream=None):
    n = net.struct()
    L.check(L.lib().octgs_skip_predict(ctypes.byref(scene.anchors), ctypes.byref(cam),
                                       ctypes.byref(n), float(logit_threshold), _ptr(vb.sel_idx),
                                       _ptr(vb.sel_count), sb.cap, _ptr(sb.keep_idx),
                                       _ptr(sb.keep_count), _ptr(sb.logits) if keep_logits else None,
                                       _ptr(sb.ws), sb.ws.numel(), stream_handle(stream)),
            "octgs_skip_predict")


def render_skip(vb: ViewBuffers, sb: SkipBuffers, scene: DeviceScene, cam: L.Camera,
                params: L.RasterParams, net: SkipNet, logit_threshold: float,
                precision: int = L.OCTGS_BF16, stream=None, stage_events=None,
                keep_last: bool = True):
    """select -> skip prediction -> decode of the kept anchors -> rasterize."""
    vb.select(scene, cam, params, stream=stream)
    predict(vb, sb, scene, cam, net, logit_threshold, stream=stream)
    vb.decode(scene, cam, precision, idx=sb.keep_idx, count=sb.keep_count, stream=stream)
    vb.rasterize(cam, params, stream=stream, stage_events=stage_events, keep_last=keep_last)


def anchor_weights(vb: ViewBuffers, out: torch.Tensor, stream=None):
    """Per selected anchor, the sum of its Gaussians' logged blend weights."""
    L.check(L.lib().octgs_anchor_weights(_ptr(vb.gauss_w), _ptr(vb.sel_count), vb.k,
                                         out.numel(), _ptr(out), stream_handle(stream)),
            "octgs_anchor_weights")


def features(vb: ViewBuffers, scene: DeviceScene, cam: L.Camera, z: torch.Tensor, stream=None):
    L.check(L.lib().octgs_skip_features(ctypes.byref(scene.anchors), ctypes.byref(cam),
                                        _ptr(vb.sel_idx), _ptr(vb.sel_count), z.shape[0], _ptr(z),
                                        stream_handle(stream)), "octgs_skip_features")


def collect(vb: ViewBuffers, scene: DeviceScene, cams: List[L.Camera], params: L.RasterParams,
            tau: float, rows_per_view: int, seed: int = 0):
    """Training rows (z, y) from the renderer's blend-weight log: every view
    is rendered with the plain path, per-anchor weights are reduced, labels
    are weight > tau; up to rows_per_view random rows are kept per view."""
    assert vb.gauss_w is not None, "ViewBuffers needs log_weights=True"
    dev = vb.gauss.device
    cap = max(1, vb.n)
    w = torch.empty(cap, device=dev)
    zbuf = torch.empty(cap, Z_DIM, device=dev)
    zs, ys = [], []
    gen = torch.Generator(device=dev).manual_seed(seed)
    for c in cams:
        vb.render(scene, c, params, precision=L.OCTGS_FP32)  # status checked by the caller
        anchor_weights(vb, w)
        features(vb, scene, c, zbuf)
        m = int(vb.sel_count.item())
        if m == 0:
            continue
        take = torch.randperm(m, generator=gen, device=dev)[:rows_per_view]
        zs.append(zbuf[:m][take].clone())
        ys.append((w[:m][take] > tau).float())
    return torch.cat(zs), torch.cat(ys)


def train(net: SkipNet, z: torch.Tensor, y: torch.Tensor, epochs: int = 4, batch: int = 16384,
          lr: float = 2e-3, pos_weight: float = 1.0, seed: int = 0) -> List[float]:
    """Mini-batch Adam on weighted binary cross-entropy; returns the mean
    loss of each epoch."""
    R = z.shape[0]
    gen = torch.Generator(device=z.device).manual_seed(seed)
    loss = torch.zeros(1, device=z.device)
    hist = []
    for _ in range(epochs):
        perm = torch.randperm(R, generator=gen, device=z.device, dtype=torch.int32)
        loss.zero_()
        nb = 0
        for s in range(0, R - batch + 1, batch):
            net.train_grad(z, y, pos_weight, loss, rows=perm[s:s + batch])
            net.adam(lr)
            nb += 1
        hist.append(loss.item() / max(nb, 1))
    return hist


def psnr(a: torch.Tensor, b: torch.Tensor) -> float:
    mse = torch.mean((a - b) ** 2).item()
    return float("inf") if mse == 0 else 10.0 * math.log10(1.0 / mse)


def choose_threshold(vb: ViewBuffers, sb: SkipBuffers, scene: DeviceScene, cams, params, net,
                     candidates, min_psnr: float):
    """Most aggressive logit threshold whose worst-view PSNR against the full
    decode (the arbiter of quality) on the given views is >= min_psnr; None if none is."""
    refs = []
    for c in cams:
        vb.render(scene, c, params, precision=L.OCTGS_FP32)
        refs.append(vb.rgb.clone())
    best = None
    for thr in sorted(candidates):
        worst = float("inf")
        for c, r in zip(cams, refs):
            render_skip(vb, sb, scene, c, params, net, thr, precision=L.OCTGS_FP32)
            worst = min(worst, psnr(vb.rgb, r))
        if worst >= min_psnr:
            best = (thr, worst)
    return best


def weight_keep_lists(vb: ViewBuffers, scene: DeviceScene, cams: List[L.Camera],
                      params: L.RasterParams, tau: float):
    """Per view, the selected anchors whose logged blend weight exceeds tau
    (what a perfect predictor of the label would keep), as (idx, count)
    device tensors ready for the decode; vb needs log_weights=True."""
    dev = vb.gauss.device
    w = torch.empty(max(1, vb.n), device=dev)
    out = []
    for c in cams:
        vb.render(scene, c, params, precision=L.OCTGS_FP32)
        anchor_weights(vb, w)
        m = int(vb.sel_count.item())
        keep = vb.sel_idx[:m][w[:m] > tau].contiguous()
        out.append((keep, torch.tensor([keep.numel()], dtype=torch.int32, device=dev)))
    return out
