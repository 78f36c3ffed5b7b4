"""Tile order of the compositing kernels (OCTGS_RASTER_TILE_ORDER).

The per-view longest-first order only changes which block composites which
tile.  So against the fixed group mapping:
* the image, transmittance and consumed-entry counts are the same bit for bit;
* the backward's gradients are the same bit for bit: the per-pair stores do
  not depend on the order, and the per-Gaussian reduction adds the partials
  of a Gaussian whose pairs span several 64-pair chunks in chunk order;
* the blend-weight log (float atomics across tiles) agrees to rounding.
With the oracle parity of the unordered forward and the ordered backward
(the training default), this carries both bars to the other mode.  Cases:
a single tile, ragged tile grids (partial 4x4 groups, group counts that are
not a multiple of 8), long lists, and the street-view and training sizes.
"""

import numpy as np
import pytest

from synth import scenes as S
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


def _np(t):
    return t.detach().cpu().numpy()


def _same_grads(a, b):
    """Every gradient the same bit for bit (a Gaussian listed in thousands of
    tiles included: its chunk partials are added in a fixed order)."""
    nz = int(np.count_nonzero(a))
    say(f"  gradients: {nz} nonzero, bit-identical {np.array_equal(a.view(np.uint32), b.view(np.uint32))}")
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def _run(P, gf, cam, order, train, pcap, seed):
    n = gf.shape[1]
    gt = torch.as_tensor(gf).cuda()
    cnt = torch.tensor([n], dtype=torch.int32).cuda()
    c = P.make_camera(cam)
    prm = P.raster_params(train=train, tile_order=order)
    for _ in range(2):
        vb = P.ViewBuffers(n, 1, cam.width, cam.height, pcap, gauss_capacity=n,
                           log_weights=True)
        vb.rasterize(c, prm, gauss=gt, count=cnt)
        torch.cuda.synchronize()
        st = vb.stats()
        if not st["pair_overflow"]:
            break
        # the candidate count is reported on overflow: retry with exactly that
        pcap = st["n_candidates"] + 16
        del vb
    out = dict(rgb=_np(vb.rgb), T=_np(vb.T), last=_np(vb.last), w=_np(vb.gauss_w),
               stats=vb.stats())
    if train:
        vb.gauss.copy_(gt)  # the backward reads the Gaussians of the forward call
        vb.gauss_count.copy_(cnt)
        rng = np.random.default_rng(seed)
        dimg = rng.standard_normal((3, cam.height, cam.width)).astype(np.float32)
        vb.rasterize_bwd(c, prm, torch.as_tensor(dimg).cuda())
        torch.cuda.synchronize()
        out["dg"] = _np(vb.dgauss)
    return out


CASES = [(16, 16, 50, 1), (97, 61, 1500, 2), (333, 200, 20000, 3), (1600, 1066, 60000, 4),
         (1920, 1080, 150000, 5)]


@pytest.mark.parametrize("train", [False, True])
@pytest.mark.parametrize("W,H,n,seed", CASES)
def test_tile_order_same_result(P, W, H, n, seed, train):
    cam = S.look_at((3.0, -20.0, 4.0), (0.0, 0.0, 0.0), W, H, 60.0)
    gf = S.random_gaussians(n, cam, seed, scale=(0.01, 0.4), neg_opacity_frac=0.1,
                            behind_frac=0.05)
    pcap = 32 * n + 4096
    say("tile order", W, H, n, seed, "train" if train else "render")
    a = _run(P, gf, cam, False, train, pcap, seed)
    b = _run(P, gf, cam, True, train, pcap, seed)
    for r in (a, b):
        assert r["stats"]["pair_overflow"] == 0 and r["stats"]["sync_error"] == 0
    assert a["stats"]["n_pairs"] == b["stats"]["n_pairs"]
    say(f"  pairs {a['stats']['n_pairs']}")
    assert np.array_equal(a["rgb"].view(np.uint32), b["rgb"].view(np.uint32))
    assert np.array_equal(a["T"].view(np.uint32), b["T"].view(np.uint32))
    assert np.array_equal(a["last"], b["last"])
    np.testing.assert_allclose(b["w"], a["w"], rtol=1e-5, atol=1e-6)
    if train:
        _same_grads(a["dg"], b["dg"])


def test_tile_order_long_lists(P):
    """A few dense tiles with thousands of entries among sparse ones: the
    ordering puts them first; results are unchanged."""
    W, H = 256, 160
    cam = S.look_at((3.0, -20.0, 4.0), (0.0, 0.0, 0.0), W, H, 60.0)
    dense = S.random_gaussians(6000, cam, 11, scale=(0.005, 0.02), neg_opacity_frac=0.0,
                               behind_frac=0.0)
    # squeeze the dense set into a small screen region around the centre
    dense[0:3] *= np.float32(0.05)
    sparse = S.random_gaussians(3000, cam, 12, scale=(0.01, 0.3), neg_opacity_frac=0.1,
                                behind_frac=0.05)
    gf = np.ascontiguousarray(np.concatenate([dense, sparse], axis=1))
    pcap = 32 * gf.shape[1]
    say("tile order, long lists")
    a = _run(P, gf, cam, False, True, pcap, 13)
    b = _run(P, gf, cam, True, True, pcap, 13)
    assert a["stats"]["pair_overflow"] == 0 and b["stats"]["pair_overflow"] == 0
    assert np.array_equal(a["rgb"].view(np.uint32), b["rgb"].view(np.uint32))
    assert np.array_equal(a["last"], b["last"])
    _same_grads(a["dg"], b["dg"])
    say(f"  max entries consumed by a pixel {int(a['last'].max())}")


def test_backward_deterministic(P):
    """The backward run twice on the same view gives the same gradients bit
    for bit, with Gaussians listed in thousands of tiles (their pairs span
    up to ~110 64-pair chunks of the per-Gaussian reduction)."""
    W, H, n = 1920, 1080, 150000
    cam = S.look_at((3.0, -20.0, 4.0), (0.0, 0.0, 0.0), W, H, 60.0)
    gf = S.random_gaussians(n, cam, 5, scale=(0.01, 0.4), neg_opacity_frac=0.1, behind_frac=0.05)
    pcap = 32 * n + 4096
    say("backward determinism", W, H, n)
    a = _run(P, gf, cam, True, True, pcap, 5)
    b = _run(P, gf, cam, True, True, pcap, 5)
    per = np.bincount(_pairs_per_slot(P, gf, cam, pcap), minlength=n)
    say(f"  most tiles of one Gaussian: {per.max()}")
    assert per.max() > 8 * 64  # the chunk walk takes several rounds of eight
    _same_grads(a["dg"], b["dg"])


def _pairs_per_slot(P, gf, cam, pcap):
    n = gf.shape[1]
    for _ in range(2):
        vb = P.ViewBuffers(n, 1, cam.width, cam.height, pcap, gauss_capacity=n)
        vb.rasterize(P.make_camera(cam), P.raster_params(), gauss=torch.as_tensor(gf).cuda(),
                     count=torch.tensor([n], dtype=torch.int32).cuda())
        torch.cuda.synchronize()
        st = vb.stats()
        if not st["pair_overflow"]:
            break
        pcap = st["n_candidates"] + 16  # retry with exactly the reported count
    assert st["pair_overflow"] == 0
    _, slot, _ = vb.sorted_lists()
    return slot.astype(np.int64)
