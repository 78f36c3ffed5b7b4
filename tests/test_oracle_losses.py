"""Pins of the loss oracle: SSIM against a brute-force window sum written
with plain loops, its identities and closed forms, and the gradients of the
photometric and volume losses against central differences."""

import math

import numpy as np
import pytest


@pytest.fixture(scope="module")
def LO():
    from oracle import losses as L
    return L


def _brute_ssim_mean(x, y):
    """Mean SSIM by explicit 11 x 11 window sums (zero outside the image)."""
    H, W = x.shape
    r = 5
    g1 = [math.exp(-(i * i) / (2 * 1.5 ** 2)) for i in range(-r, r + 1)]
    s = sum(g1)
    g1 = [v / s for v in g1]
    tot = 0.0
    for i in range(H):
        for j in range(W):
            mx = my = exx = eyy = exy = 0.0
            for a in range(-r, r + 1):
                for b in range(-r, r + 1):
                    ii, jj = i + a, j + b
                    if 0 <= ii < H and 0 <= jj < W:
                        w = g1[a + r] * g1[b + r]
                        xv, yv = x[ii, jj], y[ii, jj]
                        mx += w * xv
                        my += w * yv
                        exx += w * xv * xv
                        eyy += w * yv * yv
                        exy += w * xv * yv
            c1, c2 = 0.01 ** 2, 0.03 ** 2
            num = (2 * mx * my + c1) * (2 * (exy - mx * my) + c2)
            den = (mx * mx + my * my + c1) * ((exx - mx * mx) + (eyy - my * my) + c2)
            tot += num / den
    return tot / (H * W)


def test_ssim_matches_brute_force(LO):
    rng = np.random.default_rng(0)
    x = rng.random((9, 14))
    y = np.clip(x + 0.2 * rng.standard_normal(x.shape), 0, 1)
    assert abs(LO.ssim_map(x, y).mean() - _brute_ssim_mean(x, y)) < 1e-13


def test_ssim_identity_and_window(LO):
    w = LO.gaussian_window()
    assert len(w) == 11 and abs(w.sum() - 1) < 1e-15 and np.allclose(w, w[::-1])
    rng = np.random.default_rng(1)
    x = rng.random((3, 20, 25))
    np.testing.assert_allclose(LO.ssim_map(x, x), 1.0, atol=1e-12)
    loss, g = LO.photometric_loss_grad(x, x)
    assert abs(loss) < 1e-12 and np.abs(g).max() < 1e-12


def test_ssim_constant_images_closed_form(LO):
    """Away from the border (where the zero padding enters the window) two
    constant images a and b give (2ab + C1) / (a^2 + b^2 + C1)."""
    a, b = 0.3, 0.7
    x = np.full((30, 30), a)
    y = np.full((30, 30), b)
    S = LO.ssim_map(x, y)
    want = (2 * a * b + 0.01 ** 2) / (a * a + b * b + 0.01 ** 2)
    np.testing.assert_allclose(S[5:-5, 5:-5], want, rtol=1e-12)


def test_photometric_gradient_fd(LO):
    rng = np.random.default_rng(2)
    x = rng.random((2, 3, 7, 12))
    y = rng.random(x.shape)
    loss, g = LO.photometric_loss_grad(x, y)
    h = 1e-6
    fd = np.zeros_like(x)
    it = np.nditer(x, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        xp = x.copy()
        xp[i] += h
        xm = x.copy()
        xm[i] -= h
        fd[i] = (LO.photometric_loss_grad(xp, y)[0] - LO.photometric_loss_grad(xm, y)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, atol=1e-8)
    # the L1 and SSIM weights enter linearly
    l1 = np.abs(x - y).mean()
    assert abs(LO.photometric_loss_grad(x, y, 1.0, 0.0)[0] - l1) < 1e-15
    assert abs(loss - (0.8 * l1 + 0.2 * (1 - LO.ssim_map(x, y).mean()))) < 1e-14


def test_volume_loss_grad(LO):
    rng = np.random.default_rng(3)
    n, cnt = 50, 41
    g = rng.random((14, n))
    g[10] = rng.uniform(-1, 1, n)
    loss, d = LO.volume_loss_grad(g, cnt, 0.01)
    keep = np.flatnonzero(g[10, :cnt] > 0)
    want = 0.01 * sum(g[3, s] * g[4, s] * g[5, s] for s in keep)
    assert abs(loss - want) < 1e-15
    h = 1e-7
    for s in range(n):
        for c in range(3):
            gp = g.copy()
            gp[3 + c, s] += h
            gm = g.copy()
            gm[3 + c, s] -= h
            fd = (LO.volume_loss_grad(gp, cnt)[0] - LO.volume_loss_grad(gm, cnt)[0]) / (2 * h)
            assert abs(fd - d[3 + c, s]) < 1e-9
    assert np.abs(d[:3]).max() == 0 and np.abs(d[6:]).max() == 0
