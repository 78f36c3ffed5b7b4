"""Densification statistics and decisions of the adaptive anchor control
(Sec. IV-B): the accumulated view-space positional gradient of every
Gaussian, the anchors' average opacity and view frequency, and the
decisions taken from them every T iterations.  TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module.  It never imports the HIP package, and the HIP package never
imports it.

Statistics (per training view, after its backward pass):
  * every Gaussian that the view rasterizes (survives the projection culls)
    adds |dL/dmu'| to its gradient sum and 1 to its count, mu' its projected
    centre in normalised device coordinates (x in [-1, 1] across the width),
    i.e. the pixel-space gradient scaled by (W/2, H/2) - the convention of
    the 3D-GS criterion whose threshold 2e-4 the paper adopts;
  * every anchor the view selects adds 1 to its view count and the sum of
    its Gaussians' opacities, negative ones taken as 0, to its opacity sum.
Decisions (canonical FP32; the level thresholds are rounded once from
double, so both sides compare the same float values):
  * grad_g = sum / count (0 if never visible);
  * tau_L = tau_g 2^(beta L); a Gaussian of a level-L anchor grows if
    grad_g > tau_L, at level L + 1 if also grad_g > tau_(L+1) and L + 1 < K,
    else at level L ("next-level growing"); -1 means no growth;
  * grad_v = mean of grad_g over the anchor's Gaussians that were visible at
    least once (0 if none); Delta L += epsilon if grad_v > tau_L / 4;
  * prune if view_count / n_views < tau_v (view frequency), or if the anchor
    was selected and its average opacity opacity_sum / (k view_count) is
    below tau_opacity.
"""

from __future__ import annotations

import numpy as np

F32 = np.float32


def level_thresholds(tau_g: float, beta: float, n_levels: int) -> np.ndarray:
    """tau_g 2^(beta L) for L = 0..K from the FP32 values of tau_g and beta,
    evaluated in double and rounded once to FP32."""
    t, b = float(F32(tau_g)), float(F32(beta))
    return np.array([t * np.exp2(b * L) for L in range(n_levels + 1)], np.float64).astype(F32)


def accumulate(stats, gidx, visible, dmean2d_px, width, height, anchor_idx, opacity, k):
    """Add one view's contributions to stats (dict of float64 / int arrays):
    gidx [slots] global Gaussian ids of the view's slots, visible [slots]
    bool, dmean2d_px [slots][2] pixel-space gradients, anchor_idx [m] the
    selected anchors, opacity [m*k] their decoded opacities."""
    g = np.asarray(dmean2d_px, np.float64)
    norm = np.hypot(g[:, 0] * (width / 2.0), g[:, 1] * (height / 2.0))
    vis = np.asarray(visible, bool)
    np.add.at(stats["grad_sum"], gidx[vis], norm[vis])
    np.add.at(stats["grad_count"], gidx[vis], 1)
    stats["view_count"][anchor_idx] += 1
    op = np.maximum(np.asarray(opacity, np.float64).reshape(len(anchor_idx), k), 0.0)
    stats["opacity_sum"][anchor_idx] += op.sum(axis=1)
    return stats


def new_stats(n, k):
    return dict(grad_sum=np.zeros(n * k), grad_count=np.zeros(n * k, np.int64),
                view_count=np.zeros(n, np.int64), opacity_sum=np.zeros(n))


def decide(level, lod_bias, grad_sum, grad_count, opacity_sum, view_count, k, n_levels,
           n_views, tau_g=2e-4, beta=0.2, epsilon=0.01, tau_opacity=0.005, tau_v=0.01):
    """(grow_level int8 [n*k], new lod_bias float32 [n], prune uint8 [n]) from
    FP32 statistics, every operation in FP32 as listed in the module doc."""
    level = np.asarray(level, np.int64)
    n = len(level)
    thr = level_thresholds(tau_g, beta, n_levels)
    gs = np.asarray(grad_sum, F32).reshape(n, k)
    gc = np.asarray(grad_count, np.int64).reshape(n, k)
    grad = np.where(gc > 0, gs / np.maximum(gc, 1).astype(F32), F32(0)).astype(F32)
    tl = thr[level][:, None]
    tn = thr[np.minimum(level + 1, n_levels)][:, None]
    can_promote = (level + 1 < n_levels)[:, None]
    grow = np.where(grad > tl, np.where(can_promote & (grad > tn), level[:, None] + 1,
                                        level[:, None]), -1).astype(np.int8)
    # grad_v: FP32 sum over the visible Gaussians in index order, then divide
    s = np.zeros(n, F32)
    cnt = np.zeros(n, np.int64)
    for i in range(k):
        m = gc[:, i] > 0
        s = np.where(m, (s + grad[:, i]).astype(F32), s)
        cnt += m
    gv = np.where(cnt > 0, s / np.maximum(cnt, 1).astype(F32), F32(0)).astype(F32)
    bias = np.asarray(lod_bias, F32).copy()
    up = gv > (thr[level] * F32(0.25)).astype(F32)
    bias[up] = (bias[up] + F32(epsilon)).astype(F32)
    vc = np.asarray(view_count, np.int64)
    freq = (vc.astype(F32) / F32(n_views)).astype(F32)
    avg = np.where(vc > 0, np.asarray(opacity_sum, F32) / (F32(k) * np.maximum(vc, 1).astype(F32)),
                   F32(0))
    prune = (freq < F32(tau_v)) | ((vc > 0) & (avg.astype(F32) < F32(tau_opacity)))
    return grow.reshape(-1), bias, prune.astype(np.uint8)
