"""Training losses of the framework (Sec. V, implementation details): the
photometric loss w_l1 * L1 + w_ssim * (1 - SSIM) (weights 0.8 and 0.2 for
the 3D-GS model) and the volume regularisation L_vol = sum_i Prod(s_i)
(weight 0.01 for the Scaffold-GS model).  FP64.  TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module.  It never imports the HIP package, and the HIP package never
imports it.

SSIM is the structural similarity of Wang et al. (2004), which the paper
names but does not restate; the constants here are that standard form:
an 11 x 11 Gaussian window with sigma 1.5 (normalised to sum 1), C1 =
(0.01)^2, C2 = (0.03)^2 for a data range of 1, the windowed statistics taken
as a same-size correlation with zero padding outside the image, evaluated
per colour channel, and the map averaged over views, channels and pixels:
  mu_x = w * x, s_xx = w * x^2 - mu_x^2, s_xy = w * (x y) - mu_x mu_y,
  S = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_xx + s_yy + C2)).
L1 is the mean absolute difference over the same elements.  L_vol sums
s_0 s_1 s_2 over the decoded Gaussians that are rendered (opacity > 0).
"""

from __future__ import annotations

import math

import numpy as np
from scipy.ndimage import correlate1d

SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2
SSIM_SIGMA = 1.5
SSIM_TAPS = 11


def gaussian_window() -> np.ndarray:
    i = np.arange(SSIM_TAPS) - SSIM_TAPS // 2
    g = np.exp(-(i * i) / (2.0 * SSIM_SIGMA ** 2))
    return g / g.sum()


def _blur(a: np.ndarray) -> np.ndarray:
    """Same-size 2D correlation with the separable window over the last two
    axes, zero outside the image."""
    g = gaussian_window()
    a = correlate1d(a, g, axis=-1, mode="constant", cval=0.0)
    return correlate1d(a, g, axis=-2, mode="constant", cval=0.0)


def ssim_map(x, y) -> np.ndarray:
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my = _blur(x), _blur(y)
    sxx = _blur(x * x) - mx * mx
    syy = _blur(y * y) - my * my
    sxy = _blur(x * y) - mx * my
    return ((2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)
            / ((mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2)))


def photometric_loss_grad(img, target, w_l1: float = 0.8, w_ssim: float = 0.2):
    """(loss, dloss/dimg) for loss = w_l1 mean|img - target| + w_ssim (1 - mean SSIM)
    over images [..., H, W] (every leading index is a separate channel image).

    The SSIM gradient is the chain rule through the windowed statistics:
    with A1 = 2 mx my + C1, A2 = 2 sxy + C2, B1 = mx^2 + my^2 + C1,
    B2 = sxx + syy + C2 and S = A1 A2 / (B1 B2), the derivatives of S with
    respect to mx, E[x^2] and E[x y] (the window averages) are
      S (2 my / A1 - 2 my / A2 - 2 mx / B1 + 2 mx / B2),  -S / B2,  2 S / A2,
    and dS/dx(p) sums them over the windows that contain p: the same
    correlation (the window is symmetric) applied to the three maps, the
    second times 2 x(p), the third times y(p)."""
    x = np.asarray(img, np.float64)
    y = np.asarray(target, np.float64)
    n = x.size
    mx, my = _blur(x), _blur(y)
    sxx = _blur(x * x) - mx * mx
    syy = _blur(y * y) - my * my
    sxy = _blur(x * y) - mx * my
    A1 = 2 * mx * my + SSIM_C1
    A2 = 2 * sxy + SSIM_C2
    B1 = mx * mx + my * my + SSIM_C1
    B2 = sxx + syy + SSIM_C2
    S = A1 * A2 / (B1 * B2)
    d_m = S * (2 * my / A1 - 2 * my / A2 - 2 * mx / B1 + 2 * mx / B2)
    d_xx = -S / B2
    d_xy = 2 * S / A2
    dS = _blur(d_m) + 2 * x * _blur(d_xx) + y * _blur(d_xy)
    loss = w_l1 * np.abs(x - y).mean() + w_ssim * (1.0 - S.mean())
    grad = w_l1 * np.sign(x - y) / n - w_ssim * dS / n
    return float(loss), grad


def volume_loss_grad(gauss, count: int, weight: float = 0.01):
    """(loss, d_gauss [14][n]) of weight * sum over slots s < count with
    opacity > 0 of scale_x scale_y scale_z; gauss planar [14][n]."""
    g = np.asarray(gauss, np.float64)
    d = np.zeros_like(g)
    s = g[3:6, :count]
    keep = g[10, :count] > 0.0
    prod = s[0] * s[1] * s[2]
    loss = weight * float(prod[keep].sum())
    d[3, :count] = np.where(keep, weight * s[1] * s[2], 0.0)
    d[4, :count] = np.where(keep, weight * s[0] * s[2], 0.0)
    d[5, :count] = np.where(keep, weight * s[0] * s[1], 0.0)
    return loss, d
