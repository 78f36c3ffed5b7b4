"""Gradient of a photometric loss summed over several training views, with
the views in flight on separate streams (the multi-view loss of Sec. V).

Each view renders, computes its loss and runs the rasterizer backward and
the decode backward's compute half on its own stream and buffer set, so the
views' latency-bound kernels (scans, sorts, emission, the MLP backward)
overlap.  The steps that read-modify-write arrays shared by all views, the
decode backward's apply half into the scene gradients and the
densification statistics, run in view order, chained by events, so the
gradients are those of the views taken one after another."""

from __future__ import annotations

from typing import List, Optional

import torch

from . import _lib as L
from .render import (DensifyStats, DeviceScene, SceneGrads, ViewBuffers, l1_loss_grad,
                     photometric_loss_grad, raise_on_status)


class MultiViewBackward:
    """Buffers for `n_views` views of width x height, `inflight` of them at a
    time (view i uses stream and buffer set i % inflight; the first stream
    is the caller's current stream when run() is called)."""

    def __init__(self, scene: DeviceScene, width: int, height: int, n_views: int,
                 pair_capacity: int, gauss_capacity: Optional[int] = None, inflight: int = 4):
        self.n_views = int(n_views)
        self.nbuf = max(1, min(int(inflight), self.n_views))
        self.vbs = [ViewBuffers(scene.n, scene.k, width, height, pair_capacity,
                                gauss_capacity=gauss_capacity) for _ in range(self.nbuf)]
        self.side = [torch.cuda.Stream() for _ in range(self.nbuf - 1)]
        dev = self.vbs[0].gauss.device
        self.dimgs = [torch.empty(3, height, width, device=dev) for _ in range(self.nbuf)]
        self.losses = torch.zeros(self.n_views, device=dev)  # one slot per view
        self._ssim_ws: List[Optional[torch.Tensor]] = [None] * self.nbuf

    def check(self):
        """Raise if any view rendered since the last check overflowed its pair
        list, hit a look-back wait bound or selected more anchors than the
        Gaussian capacity decodes (syncs), then clear the status words (each
        buffer set's, which the library ORs every frame's conditions into)."""
        bits = 0
        for vb in self.vbs:
            bits |= int(vb.status.item())
            vb.status.zero_()
        raise_on_status(bits, "training views")

    def run(self, scene: DeviceScene, cams: List[L.Camera], targets: List[torch.Tensor],
            params: L.RasterParams, grads: SceneGrads, l1_scale: float = 1.0,
            full: bool = False, w_l1: float = 0.8, w_ssim: float = 0.2, w_vol: float = 0.01,
            dstats: Optional[DensifyStats] = None) -> torch.Tensor:
        """Zero `grads` and `self.losses`, then add each view's loss gradient.
        Loss per view: l1_scale * sum |img - target| (mean L1 when l1_scale
        is 1 / (views * pixels * 3)); with full, (w_l1 L1 + w_ssim (1 - SSIM))
        / views + w_vol sum Prod(s) over the view's rendered Gaussians.
        dstats (optional) accumulates the densification statistics.  params
        must include OCTGS_RASTER_TRAIN.  Returns the per-view losses
        (device); the caller's current stream has waited for all of it.
        The scene's derived arrays (thresholds, bound radii) are recomputed
        first, since an optimiser step may have changed the trained arrays
        (the BF16 feature copy is left stale: refresh the scene before a BF16
        render); each view's device-detected conditions are kept in
        its buffer set's status word (see check())."""
        assert len(cams) == len(targets) == self.n_views
        main = torch.cuda.current_stream()
        streams = [main] + self.side
        scene.refresh(stream=main, bf16=False)  # the train step decodes in FP32
        grads.zero_()
        self.losses.zero_()
        go = torch.cuda.Event()
        go.record(main)
        for st in self.side:
            st.wait_event(go)
        nv = self.n_views
        chain = None
        for i, (c, tg) in enumerate(zip(cams, targets)):
            k = i % self.nbuf
            st, vb, dimg, li = streams[k], self.vbs[k], self.dimgs[k], self.losses[i:i + 1]
            vb.render(scene, c, params, stream=st)
            if full:
                self._ssim_ws[k] = photometric_loss_grad(vb.rgb, tg, dimg, li, w_l1 / nv,
                                                         w_ssim / nv, self._ssim_ws[k], stream=st)
            else:
                l1_loss_grad(vb.rgb, tg, l1_scale, dimg, li, stream=st)
            vb.rasterize_bwd(c, params, dimg, stream=st)
            if full:
                vb.volume_loss_grad(w_vol, li, stream=st)
            # the decode backward's own work, then what touches the shared
            # arrays: one view after another
            vb.decode_bwd_rows(scene, c, stream=st)
            if chain is not None:
                st.wait_event(chain)
            if dstats is not None:
                dstats.accumulate(vb, c, stream=st)
            vb.decode_bwd_apply(scene, grads, stream=st)
            chain = torch.cuda.Event()
            chain.record(st)
        # the last link follows every view's work
        main.wait_event(chain)
        return self.losses
