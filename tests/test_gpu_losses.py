"""Parity of the training losses (photometric L1 + SSIM, volume
regularisation) with the FP64 oracle, through the C ABI.

Bars: the loss within 2e-6 (FP32 sums of 1024 terms in [0, 1] per block,
the block sums then added in double); the image gradient within 1e-4
normwise and 1e-3 of the largest entry elementwise (the gradient
bar used throughout; the windowed variances lose a few bits to cancellation); the volume
gradient within 1e-6 relative (three FP32 products).
"""

import numpy as np
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_17898_amd as P
    P.lib()
    return P


@pytest.fixture(scope="module")
def LO():
    from oracle import losses as L
    return L


def _images(shape, seed):
    """A smooth image plus detail, and a noisy, shifted copy as the target
    (the statistics of a rendering against its ground truth)."""
    rng = np.random.default_rng(seed)
    H, W = shape[-2:]
    yy, xx = np.mgrid[0:H, 0:W]
    base = 0.5 + 0.3 * np.sin(xx / 7.0 + rng.uniform(0, 6, shape[:-2] + (1, 1))) * np.cos(yy / 11.0)
    img = np.clip(base + 0.1 * rng.standard_normal(shape), 0, 1).astype(np.float32)
    tgt = np.clip(img + 0.05 * rng.standard_normal(shape) + 0.02, 0, 1).astype(np.float32)
    return img, tgt


def _run(P, img, tgt, w_l1, w_ssim):
    x = torch.as_tensor(img).cuda()
    y = torch.as_tensor(tgt).cuda()
    d = torch.full_like(x, 7.0)   # overwritten
    loss = torch.full((1,), 0.5, dtype=torch.float32, device="cuda")  # accumulated
    P.photometric_loss_grad(x, y, d, loss, w_l1, w_ssim)
    torch.cuda.synchronize()
    return float(loss.item()) - 0.5, d.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("shape", [(2, 3, 97, 131), (1, 3, 5, 7), (1, 1, 16, 64), (4, 3, 1066, 1600)])
def test_photometric_parity(P, LO, shape):
    img, tgt = _images(shape, sum(shape))
    say("photometric", shape)
    loss, g = _run(P, img, tgt, 0.8, 0.2)
    rl, rg = LO.photometric_loss_grad(img, tgt, 0.8, 0.2)
    e = np.linalg.norm(g - rg) / np.linalg.norm(rg)
    say(f"  loss {loss:.7f} vs {rl:.7f}; grad rel err {e:.2e}, "
        f"max abs err / max {np.abs(g - rg).max() / np.abs(rg).max():.2e}")
    assert abs(loss - rl) <= 2e-6
    assert e <= 1e-4
    assert np.abs(g - rg).max() <= 1e-3 * np.abs(rg).max()


def test_l1_only_and_identity(P, LO):
    img, tgt = _images((2, 3, 40, 70), 5)
    loss, g = _run(P, img, tgt, 1.0, 0.0)
    rl, rg = LO.photometric_loss_grad(img, tgt, 1.0, 0.0)
    assert abs(loss - rl) <= 1e-6
    assert np.array_equal(np.sign(g), np.sign(rg))
    np.testing.assert_allclose(g, rg, rtol=1e-6)
    # identical images: SSIM 1, loss 0
    loss, g = _run(P, img, img, 0.8, 0.2)
    assert abs(loss) <= 1e-6
    # gradient entries are O(w_ssim / n) in general; here FP32 leaves ~1e-6 of that
    assert np.abs(g).max() <= 1e-4 * 0.2 / img.size


def test_volume_loss_parity(P, LO):
    from paper_2403_17898_amd import _lib as L
    import ctypes
    rng = np.random.default_rng(8)
    cap, cnt = 5000, 4321
    gd = rng.random((14, cap)).astype(np.float32)
    gd[10] = rng.uniform(-1, 1, cap).astype(np.float32)
    g = torch.as_tensor(gd).cuda()
    c = torch.tensor([cnt], dtype=torch.int32).cuda()
    dg0 = np.full((14, cap), 0.25, np.float32)   # accumulated onto a known value
    dg = torch.as_tensor(dg0).cuda()
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    gs = L.Gaussians()
    gs.capacity, gs.data, gs.count = cap, g.data_ptr(), c.data_ptr()
    L.check(L.lib().octgs_volume_loss_grad(ctypes.byref(gs), 0.01, ctypes.c_void_p(dg.data_ptr()),
                                           ctypes.c_void_p(loss.data_ptr()), None),
            "octgs_volume_loss_grad")
    torch.cuda.synchronize()
    rl, rd = LO.volume_loss_grad(gd, cnt, 0.01)
    assert abs(float(loss.item()) - rl) <= 1e-6 * rl
    got = dg.cpu().numpy().astype(np.float64) - dg0
    np.testing.assert_allclose(got, rd, rtol=1e-6, atol=3e-8)
