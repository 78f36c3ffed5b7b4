"""Explicit-Gaussian anchors (the 3D-GS instance of the anchor framework,
Sec. V "Our-3D-GS"): FP64 decode, its backward and a full-view render.
TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module.  It never imports the HIP package, and the HIP package never
imports it.

What is computed (the 3D-GS primitive of Sec. III-A, attached to the anchors
that Eq. 7 selects):
  * mean       = the stored world position;
  * scale      = exp(log-scale);
  * quaternion = the stored rotation normalised (identity when its norm is 0);
  * opacity    = sigmoid(logit), times the LOD transition factor when
                 blending (Sec. IV-A, last paragraph of "Anchor Selection");
  * colour     = max(0, sum_lm sh_lm Y_lm(d) + 0.5), with d the unit vector
                 from the camera centre to the Gaussian mean and Y_lm the real
                 spherical harmonics below (view-dependent colour from SH
                 coefficients, Sec. III-A).

Real spherical harmonics: built here from the associated Legendre functions
P_l^m (Condon-Shortley phase included) by their three-term recurrence, with
K_lm = sqrt((2l + 1) / (4 pi) (l - m)! / (l + m)!):
  m = 0: K_l0 P_l^0(cos t);  m > 0: sqrt(2) K_lm P_l^m(cos t) cos(m p);
  m < 0: sqrt(2) K_l|m| P_l^|m|(cos t) sin(|m| p),
for polar angle t and azimuth p of d, ordered by l then m = -l..l (column
l^2 + l + m).  That is sqrt(2) Re / Im of the complex harmonics with the
phase kept, the sign convention of the 3D-GS colour model.  Pins: the
complex harmonics of scipy, orthonormality on the sphere by exact
quadrature, and finite differences of the derivative.
"""

from __future__ import annotations

import math
from typing import Dict

import numpy as np


def _legendre(l_max: int, ct: np.ndarray, st: np.ndarray) -> Dict:
    """P[(l, m)] for 0 <= m <= l <= l_max with the Condon-Shortley phase:
    P_m^m = (-1)^m (2m - 1)!! st^m, P_{m+1}^m = (2m + 1) ct P_m^m,
    (l - m) P_l^m = (2l - 1) ct P_{l-1}^m - (l + m - 1) P_{l-2}^m."""
    P = {}
    pmm = np.ones_like(ct)
    for m in range(l_max + 1):
        if m > 0:
            pmm = -(2 * m - 1) * st * pmm
        P[(m, m)] = pmm
        if m + 1 <= l_max:
            P[(m + 1, m)] = (2 * m + 1) * ct * pmm
        for l in range(m + 2, l_max + 1):
            P[(l, m)] = ((2 * l - 1) * ct * P[(l - 1, m)] - (l + m - 1) * P[(l - 2, m)]) / (l - m)
    return P


def _norm(l: int, m: int) -> float:
    return math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))


def _angles(dirs):
    d = np.asarray(dirs, np.float64)
    d = d / np.linalg.norm(d, axis=-1, keepdims=True)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    st = np.hypot(x, y)
    return z, st, np.arctan2(y, x)


def sh_basis(dirs, degree: int) -> np.ndarray:
    """Real SH Y [..., (degree+1)^2] at the directions dirs [..., 3]."""
    ct, st, ph = _angles(dirs)
    P = _legendre(degree, ct, st)
    out = np.empty(ct.shape + ((degree + 1) ** 2,), np.float64)
    r2 = math.sqrt(2.0)
    for l in range(degree + 1):
        out[..., l * l + l] = _norm(l, 0) * P[(l, 0)]
        for m in range(1, l + 1):
            out[..., l * l + l + m] = r2 * _norm(l, m) * P[(l, m)] * np.cos(m * ph)
            out[..., l * l + l - m] = r2 * _norm(l, m) * P[(l, m)] * np.sin(m * ph)
    return out


def sh_basis_grad(dirs, degree: int) -> np.ndarray:
    """Gradient of each Y_lm on the unit sphere at dirs: [..., (degree+1)^2, 3],
    dY/dt e_t + (1 / sin t) dY/dp e_p with e_t = (ct cp, ct sp, -st) and
    e_p = (-sp, cp, 0).  dP_l^m/dt = P_l^1 for m = 0 and
    (P_l^{m+1} - (l + m)(l - m + 1) P_l^{m-1}) / 2 for m >= 1 (P_l^{l+1} = 0).
    The gradient with respect to an unnormalised v is this divided by |v|."""
    ct, st, ph = _angles(dirs)
    P = _legendre(degree, ct, st)
    get = lambda l, m: P.get((l, m), np.zeros_like(ct))
    cp, sp = np.cos(ph), np.sin(ph)
    e_t = np.stack([ct * cp, ct * sp, -st], axis=-1)
    e_p = np.stack([-sp, cp, np.zeros_like(ct)], axis=-1)
    out = np.zeros(ct.shape + ((degree + 1) ** 2, 3), np.float64)
    r2 = math.sqrt(2.0)
    for l in range(degree + 1):
        dP0 = get(l, 1)
        out[..., l * l + l, :] = (_norm(l, 0) * dP0)[..., None] * e_t
        for m in range(1, l + 1):
            dPm = 0.5 * (get(l, m + 1) - (l + m) * (l - m + 1) * get(l, m - 1))
            k = r2 * _norm(l, m)
            Pm_over_st = P[(l, m)] / st
            # cos(m p) term, then sin(m p) term
            out[..., l * l + l + m, :] = ((k * dPm * np.cos(m * ph))[..., None] * e_t
                                          + (-m * k * Pm_over_st * np.sin(m * ph))[..., None] * e_p)
            out[..., l * l + l - m, :] = ((k * dPm * np.sin(m * ph))[..., None] * e_t
                                          + (m * k * Pm_over_st * np.cos(m * ph))[..., None] * e_p)
    return out


def _blend_factor(ex, idx, cam) -> np.ndarray:
    """Opacity factor min(1, max(0, L* - L + 1)) per listed anchor, L* the
    clamped fractional level log2(d_max / (d s)) + Delta L."""
    d = ex.pos[idx].astype(np.float64) - cam.C.astype(np.float64)
    dist = np.linalg.norm(d, axis=1)
    ls = np.clip(np.log2(ex.d_max / (dist * cam.lod_scale)) + ex.lod_bias[idx], 0.0,
                 ex.n_levels - 1)
    return np.clip(ls - ex.level[idx].astype(np.float64) + 1.0, 0.0, 1.0)


def _gather(ex, idx):
    idx = np.asarray(idx, np.int64)
    m, k = len(idx), ex.k
    f = lambda a: a[idx].astype(np.float64).reshape((m * k,) + a.shape[2:])
    return (f(ex.mean), f(ex.log_scale), f(ex.rot), f(ex.opacity), f(ex.sh))


def decode_explicit(ex, idx, cam, blend: bool = False) -> np.ndarray:
    """Planar [14][len(idx) * k] Gaussians of the listed anchors, slot p*k + i
    for Gaussian i of the p-th listed anchor."""
    idx = np.asarray(idx, np.int64)
    mean, ls, rot, logit, sh = _gather(ex, idx)
    out = np.empty((14, len(mean)), np.float64)
    out[0:3] = mean.T
    out[3:6] = np.exp(ls).T
    n = np.linalg.norm(rot, axis=1)
    q = np.where(n[:, None] > 0, rot / np.where(n > 0, n, 1.0)[:, None],
                 np.array([1.0, 0.0, 0.0, 0.0]))
    out[6:10] = q.T
    op = 1.0 / (1.0 + np.exp(-logit))
    if blend:
        op = op * np.repeat(_blend_factor(ex, idx, cam), ex.k)
    out[10] = op
    v = mean - cam.C.astype(np.float64)[None, :]
    Y = sh_basis(v, ex.sh_degree)
    raw = np.einsum("sl,slc->sc", Y, sh) + 0.5
    out[11:14] = np.maximum(raw, 0.0).T
    return out


def decode_explicit_backward(ex, idx, cam, dgauss) -> Dict[str, np.ndarray]:
    """Gradients of mean, log_scale, rot, opacity (logit) and sh for
    L = sum(dgauss * decode_explicit(ex, idx, cam)); full-size arrays, zero
    for anchors not listed."""
    idx = np.asarray(idx, np.int64)
    m, k = len(idx), ex.k
    dg = np.asarray(dgauss, np.float64)[:, :m * k]
    mean, ls, rot, logit, sh = _gather(ex, idx)
    v = mean - cam.C.astype(np.float64)[None, :]
    vn = np.linalg.norm(v, axis=1)
    Y = sh_basis(v, ex.sh_degree)
    raw = np.einsum("sl,slc->sc", Y, sh) + 0.5
    g = dg[11:14].T * (raw > 0.0)                      # d colour, through the clamp
    d_sh = Y[:, :, None] * g[:, None, :]
    dY = sh_basis_grad(v, ex.sh_degree)                # [s, lm, 3] on the sphere
    d_dir = np.einsum("slc,sc,slx->sx", sh, g, dY)
    d_mean = dg[0:3].T + d_dir / vn[:, None]
    d_ls = dg[3:6].T * np.exp(ls)
    n = np.linalg.norm(rot, axis=1)
    safe = np.where(n > 0, n, 1.0)
    qn = rot / safe[:, None]
    dq = dg[6:10].T
    d_rot = np.where(n[:, None] > 0,
                     (dq - qn * np.sum(qn * dq, axis=1, keepdims=True)) / safe[:, None], 0.0)
    sig = 1.0 / (1.0 + np.exp(-logit))
    d_logit = dg[10] * sig * (1.0 - sig)
    out = dict(mean=np.zeros(ex.mean.shape), log_scale=np.zeros(ex.log_scale.shape),
               rot=np.zeros(ex.rot.shape), opacity=np.zeros(ex.opacity.shape),
               sh=np.zeros(ex.sh.shape))
    out["mean"][idx] = d_mean.reshape(m, k, 3)
    out["log_scale"][idx] = d_ls.reshape(m, k, 3)
    out["rot"][idx] = d_rot.reshape(m, k, 4)
    out["opacity"][idx] = d_logit.reshape(m, k)
    out["sh"][idx] = d_sh.reshape(ex.sh[idx].shape)
    return out


def thresholds(ex):
    """(thr2, rho) of an ExplicitScene: the Eq. 7 thresholds and the canonical
    FP32 bound radius of each anchor's explicit Gaussians."""
    from . import oracle as O
    return (O.lod_thr2(ex.level, ex.lod_bias, ex.d_max),
            O.bound_radius_explicit(ex.pos, ex.mean, ex.log_scale))


def render_explicit(ex, cam, prm, blend: bool = False, weights: bool = False):
    """Select (Eq. 7), decode the explicit Gaussians, rasterize."""
    from . import oracle as O
    thr2, rho = thresholds(ex)
    idx = np.flatnonzero(O.select_mask(ex.pos, thr2, rho, cam, blend)).astype(np.int64)
    gd = decode_explicit(ex, idx, cam, blend)
    out = O.rasterize(gd.astype(np.float32), cam, prm, gd=gd, weights=weights)
    out.update(idx=idx, gauss=gd)
    return out


def render_explicit_backward(ex, cam, prm, dimg, fwd=None):
    """Full-chain gradients of L = sum(dimg * render_explicit(ex, cam)) with
    the forward's discrete decisions held fixed."""
    from . import oracle as O
    if fwd is None:
        fwd = render_explicit(ex, cam, prm)
    dproj = O.composite_backward(fwd["pj"], fwd["bs"], cam, prm, dimg)
    dg = O.project_backward(fwd["gauss"], fwd["pj"], cam, prm, dproj)
    return decode_explicit_backward(ex, fwd["idx"], cam, dg)
