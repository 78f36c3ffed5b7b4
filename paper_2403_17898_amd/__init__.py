"""Octree-GS render path on AMD MI355X: HIP kernels behind a C ABI
(include/octgs.h), with a thin ctypes binding.

    from paper_2403_17898_amd import DeviceScene, ViewBuffers, make_camera, raster_params
"""

from ._lib import (OCTGS_BF16, OCTGS_FP32, OCTGS_STATUS_PAIR_OVERFLOW,  # noqa: F401
                   OCTGS_STATUS_SYNC_ERROR, OCTGS_STATUS_TRUNCATED, OctgsError, lib)
from .render import (AdamMany, DensifyStats, DeviceExplicit, DeviceScene, ExplicitGrads, RenderFn,  # noqa: F401
                     SceneGrads, ViewBuffers, adam_step, l1_loss_grad, make_camera,
                     photometric_loss_grad, raise_on_status, raster_params, render_diff,
                     stream_handle, trainable)
from .train import MultiViewBackward  # noqa: F401
