"""Pins of the explicit-Gaussian oracle (3D-GS primitives on the anchors).

The real spherical-harmonic basis is checked against scipy's complex
harmonics (a separate implementation), against orthonormality on the sphere
by a quadrature that is exact for these polynomial degrees, and against the
low-order closed forms that fix its sign convention.  Its derivative and the
decode backward are checked by central differences of the FP64 forward.
"""

import math

import numpy as np
import pytest

from synth import scenes as S


@pytest.fixture(scope="module")
def EX():
    from oracle import explicit as E
    return E


def _dirs(n, seed):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def test_sh_basis_matches_scipy(EX):
    from scipy.special import sph_harm_y
    d = _dirs(200, 1)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    Y = EX.sh_basis(d, 3)
    for l in range(4):
        for m in range(-l, l + 1):
            c = sph_harm_y(l, abs(m), theta, phi)
            if m == 0:
                ref = c.real
            elif m > 0:
                ref = math.sqrt(2.0) * c.real
            else:
                ref = math.sqrt(2.0) * c.imag
            np.testing.assert_allclose(Y[:, l * l + l + m], ref, atol=1e-13, rtol=0)


def test_sh_basis_orthonormal(EX):
    # Gauss-Legendre in cos(t) is exact for polynomials of degree <= 2*8-1 in
    # cos(t); 16 equispaced azimuths integrate trigonometric terms up to
    # order 15 exactly.  Products of two degree-3 harmonics stay below both.
    x, w = np.polynomial.legendre.leggauss(8)
    ph = 2 * np.pi * np.arange(16) / 16
    ct, pp = np.meshgrid(x, ph, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(pp), st * np.sin(pp), ct], axis=-1).reshape(-1, 3)
    wt = (w[:, None] * np.full(16, 2 * np.pi / 16)[None, :]).reshape(-1)
    Y = EX.sh_basis(d, 3)
    G = (Y * wt[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-13)


def test_sh_low_order_closed_forms(EX):
    d = _dirs(50, 2)
    Y = EX.sh_basis(d, 1)
    c0 = 0.5 / math.sqrt(math.pi)
    c1 = math.sqrt(3.0 / (4.0 * math.pi))
    np.testing.assert_allclose(Y[:, 0], c0, rtol=1e-14)
    np.testing.assert_allclose(Y[:, 1], -c1 * d[:, 1], atol=1e-14)
    np.testing.assert_allclose(Y[:, 2], c1 * d[:, 2], atol=1e-14)
    np.testing.assert_allclose(Y[:, 3], -c1 * d[:, 0], atol=1e-14)
    # unnormalised input directions give the same values
    np.testing.assert_allclose(EX.sh_basis(7.5 * d, 1), Y, atol=1e-14)


def test_sh_gradient_fd(EX):
    v = 3.0 * _dirs(40, 3)
    ana = EX.sh_basis_grad(v, 3) / np.linalg.norm(v, axis=1)[:, None, None]
    h = 1e-6
    fd = np.zeros_like(ana)
    for c in range(3):
        dv = np.zeros(3)
        dv[c] = h
        fd[:, :, c] = (EX.sh_basis(v + dv, 3) - EX.sh_basis(v - dv, 3)) / (2 * h)
    np.testing.assert_allclose(ana, fd, atol=1e-8)
    # the gradient lies in the tangent plane
    radial = np.einsum("slx,sx->sl", ana, v)
    assert np.abs(radial).max() < 1e-12


def _tiny_explicit(degree=3, n=6, k=3, seed=5):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-1, 1, (n, 3)).astype(np.float32)
    ex = S.ExplicitScene(
        pos=pos, level=np.zeros(n, np.uint8), lod_bias=np.zeros(n, np.float32),
        mean=(pos[:, None, :] + 0.3 * rng.standard_normal((n, k, 3))).astype(np.float32),
        log_scale=rng.uniform(-3, -1, (n, k, 3)).astype(np.float32),
        rot=rng.standard_normal((n, k, 4)).astype(np.float32),
        opacity=rng.uniform(-3, 3, (n, k)).astype(np.float32),
        sh=(0.4 * rng.standard_normal((n, k, (degree + 1) ** 2, 3))).astype(np.float32),
        sh_degree=degree, d_max=10.0, n_levels=1, k=k, info={})
    cam = S.look_at((0.5, -6.0, 1.0), (0.0, 0.0, 0.0), 32, 32, 60.0)
    return ex, cam


def test_decode_explicit_closed_forms(EX):
    ex, cam = _tiny_explicit(degree=0, n=2, k=2)
    ex.log_scale[0, 0] = (0.0, math.log(2.0), -1.0)
    ex.rot[0, 0] = (2.0, 0.0, 0.0, 0.0)
    ex.rot[0, 1] = (0.0, 0.0, 0.0, 0.0)
    ex.opacity[0, 0] = 0.0
    ex.sh[0, 0, 0] = (0.0, 1.0, -10.0)
    g = EX.decode_explicit(ex, [0, 1], cam)
    np.testing.assert_allclose(g[0:3, 0], ex.mean[0, 0], rtol=0)
    np.testing.assert_allclose(g[3:6, 0], (1.0, 2.0, math.exp(-1.0)), rtol=1e-7)
    np.testing.assert_allclose(g[6:10, 0], (1, 0, 0, 0))
    np.testing.assert_allclose(g[6:10, 1], (1, 0, 0, 0))           # zero norm: identity
    assert g[10, 0] == 0.5
    c0 = 0.5 / math.sqrt(math.pi)
    np.testing.assert_allclose(g[11:14, 0], (0.5, 0.5 + c0, 0.0), rtol=1e-7)  # clamp at 0
    # degree 0: colour does not depend on the viewpoint
    cam2 = S.look_at((4.0, 3.0, -2.0), (0.0, 0.0, 0.0), 32, 32, 60.0)
    np.testing.assert_allclose(EX.decode_explicit(ex, [0, 1], cam2)[11:14], g[11:14], rtol=0)


def test_decode_explicit_unit_quaternions(EX):
    ex, cam = _tiny_explicit()
    g = EX.decode_explicit(ex, np.arange(ex.n), cam)
    np.testing.assert_allclose(np.linalg.norm(g[6:10], axis=0), 1.0, rtol=1e-14)
    assert (g[10] > 0).all() and (g[10] < 1).all()
    assert (g[11:14] >= 0).all()


def _perturbed(ex, name, flat_i, h):
    arr = getattr(ex, name).copy()
    f = arr.reshape(-1)
    old = f[flat_i]
    f[flat_i] = np.float32(old + h)
    step = float(f[flat_i]) - float(old)
    import dataclasses
    return dataclasses.replace(ex, **{name: arr}), step


def test_decode_explicit_backward_fd(EX):
    ex, cam = _tiny_explicit()
    idx = np.array([0, 2, 3, 5])
    rng = np.random.default_rng(9)
    dg = rng.standard_normal((14, len(idx) * ex.k))
    ana = EX.decode_explicit_backward(ex, idx, cam, dg)
    base = EX.decode_explicit(ex, idx, cam)
    for name in ("mean", "log_scale", "rot", "opacity", "sh"):
        a = ana[name].reshape(-1)
        fd = np.zeros_like(a)
        for i in range(a.size):
            vals = []
            for sgn in (1, -1):
                ex2, step = _perturbed(ex, name, i, sgn * 2e-3)
                out = EX.decode_explicit(ex2, idx, cam)
                # a colour crossing the clamp at 0 is a kink: skip it
                if not np.array_equal(out[11:14] > 0, base[11:14] > 0):
                    vals = None
                    break
                vals.append(((dg * out).sum(), step))
            if vals is None:
                fd[i] = a[i]
                continue
            fd[i] = (vals[0][0] - vals[1][0]) / (vals[0][1] - vals[1][1])
        err = np.linalg.norm(fd - a) / max(np.linalg.norm(a), 1e-300)
        assert err < 2e-5, (name, err)
    # anchors not listed get no gradient
    assert np.abs(ana["sh"][[1, 4]]).max() == 0.0


def test_bound_radius_explicit_holds_every_gaussian(orc):
    ex, _ = _tiny_explicit(n=40, k=7)
    rho = orc.bound_radius_explicit(ex.pos, ex.mean, ex.log_scale).astype(np.float64)
    d = np.linalg.norm(ex.mean.astype(np.float64) - ex.pos[:, None, :].astype(np.float64), axis=2)
    s = np.exp(ex.log_scale.astype(np.float64)).max(axis=2)
    need = (d + 3.0 * s).max(axis=1)
    assert (rho >= need * (1 - 1e-6)).all()
    # the radius is the largest distance plus three times the largest scale
    np.testing.assert_allclose(rho, d.max(axis=1) + 3.0 * s.max(axis=1), rtol=1e-6)


def test_render_explicit_blend_removes_lod_popping(EX, orc):
    """Moving the focal scale s across the value where a level-1 anchor's L*
    crosses 1: without blending its explicit Gaussians pop in, with blending
    the image changes by O(eps)."""
    sc = S.make_config1()
    ex = S.make_explicit(sc, sh_degree=1)
    cam = S.config1_camera()
    thr, rho = EX.thresholds(ex)
    d = np.linalg.norm(ex.pos.astype(np.float64) - cam.C.astype(np.float64), axis=1)
    vis = orc.select_mask(ex.pos, np.full_like(thr, np.inf), rho, cam).astype(bool)
    cand = np.flatnonzero(vis & (ex.level == 1))
    j = cand[np.argmin(np.abs(d[cand] - np.median(d[cand])))]
    s_star = float(np.float32(ex.d_max)) / (2.0 * d[j])
    prm = orc.params_array()
    eps = 1e-5

    def img(scale, blend):
        c = S.Camera(R=cam.R, C=cam.C, fx=cam.fx, fy=cam.fy, cx=cam.cx, cy=cam.cy,
                     width=cam.width, height=cam.height, z_near=cam.z_near, lod_scale=scale)
        return EX.render_explicit(ex, c, prm, blend=blend)["img"]

    jump = np.abs(img(s_star * (1 + eps), False) - img(s_star * (1 - eps), False)).max()
    cont = np.abs(img(s_star * (1 + eps), True) - img(s_star * (1 - eps), True)).max()
    assert jump > 1e-3
    assert cont < 10 * eps
