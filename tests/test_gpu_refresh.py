"""The library's derived per-scene arrays follow in-place updates of the
trained arrays, and per-frame device conditions reach the caller.

  * The BF16 copies the library writes (anchor features, SH coefficients)
    are the round-to-nearest-even bits of the FP32 values (checked against
    PyTorch's CPU conversion, including exact ties).
  * After offsets, scales and features change in place (as an optimiser
    step changes them), DeviceScene.refresh / MultiViewBackward.run bring
    the bound radii, thresholds and BF16 copy up to date: the selection is
    then bit-exact against the oracle run on the updated arrays, and the
    BF16 image equals that of a scene built fresh from them.
  * the status word the Gaussians carry reports a pair-list overflow and a
    decode truncated at the Gaussian capacity, and MultiViewBackward.check
    raises on them.
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


def _rne_bits(a):
    """BF16 bit patterns of float32 values by PyTorch's CPU conversion."""
    t = torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).numpy().view(np.uint16)


def _with_ties(rng, shape):
    """Random values, a quarter of them exact halfway cases between two BF16
    values (low 16 bits 0x8000), with even and odd upper halves."""
    x = rng.standard_normal(shape).astype(np.float32)
    u = x.view(np.uint32)
    tie = rng.random(shape) < 0.25
    u[tie] = (u[tie] & np.uint32(0xFFFF0000)) | np.uint32(0x8000)
    return u.view(np.float32)


def test_bf16_copies_round_to_nearest_even(P):
    rng = np.random.default_rng(3)
    sc = S.make_config1()
    sc.feat = _with_ties(rng, sc.feat.shape)
    say("BF16 feature copy", sc.feat.shape)
    ds = P.DeviceScene.from_scene(sc)
    torch.cuda.synchronize()
    got = _np(ds.feat_bf16).view(np.uint16)
    want = _rne_bits(sc.feat)
    assert np.count_nonzero((sc.feat.view(np.uint32) & 0xFFFF) == 0x8000) > 1000
    assert np.array_equal(got, want)
    ex = S.make_explicit(sc, sh_degree=3)
    ex.sh = _with_ties(rng, ex.sh.shape)
    say("BF16 SH copy", ex.sh.shape)
    de = P.DeviceExplicit.from_scene(ex)
    torch.cuda.synchronize()
    assert np.array_equal(_np(de.sh_bf16).view(np.uint16).reshape(-1), _rne_bits(ex.sh).reshape(-1))


def _perturb_in_place(ds, seed):
    """What an optimiser step does to the trained arrays: in-place updates on
    the device (offsets and scales grow, features move)."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    ds.offsets.mul_(1.8).add_(0.05 * torch.randn(ds.offsets.shape, generator=g, device="cuda"))
    ds.offset_scale.mul_(1.3)
    ds.base_scale.mul_(1.6)
    ds.feat.add_(0.3 * torch.randn(ds.feat.shape, generator=g, device="cuda"))


def _scene_now(sc, ds):
    """A synth.Scene carrying the device arrays' current values."""
    import copy
    s2 = copy.copy(sc)
    s2.offsets = _np(ds.offsets).copy()
    s2.offset_scale = _np(ds.offset_scale).copy()
    s2.base_scale = _np(ds.base_scale).copy()
    s2.feat = _np(ds.feat).copy()
    return s2


def _cams():
    from tests.test_oracle_visibility import generic_camera
    d = np.array([1.0, -2.0, 1.5]) / np.linalg.norm([1.0, -2.0, 1.5])
    return [S.look_at(9.0 * d, (0, 0, 0), 128, 128, 60.0),
            generic_camera(C=(5.0, -9.0, 4.0), target=(0.5, 0.0, 0.0))]


def test_refresh_follows_in_place_updates(P, orc):
    sc = S.make_config1()
    ds = P.DeviceScene.from_scene(sc)
    prm = P.raster_params()
    _perturb_in_place(ds, 1)
    torch.cuda.synchronize()
    now = _scene_now(sc, ds)
    thr, rho = orc.scene_thresholds(now)
    stale_differs = False
    for i, cam in enumerate(_cams()):
        vb = P.ViewBuffers(sc.n, sc.k, cam.width, cam.height, 1 << 18)
        c = P.make_camera(cam)
        vb.select(ds, c, prm)  # before refresh: the old bound radii
        torch.cuda.synchronize()
        m = int(vb.sel_count.item())
        stale = _np(vb.sel_idx[:m]).astype(np.int64)
        ref = orc.select(now, cam, thr, rho)
        stale_differs |= not np.array_equal(stale, ref)
    assert stale_differs, "the update does not change the selection: the test would prove nothing"
    ds.refresh()
    torch.cuda.synchronize()
    assert np.array_equal(_np(ds.bound_r).view(np.uint32), rho.view(np.uint32))
    fresh = P.DeviceScene.from_scene(now)
    for i, cam in enumerate(_cams()):
        say("refreshed scene, view", i)
        c = P.make_camera(cam)
        vb = P.ViewBuffers(sc.n, sc.k, cam.width, cam.height, 1 << 18)
        vb.select(ds, c, prm)
        torch.cuda.synchronize()
        m = int(vb.sel_count.item())
        assert np.array_equal(_np(vb.sel_idx[:m]).astype(np.int64), orc.select(now, cam, thr, rho))
        vb.render(ds, c, prm, precision=P.OCTGS_BF16)
        img = _np(vb.rgb).copy()
        vf = P.ViewBuffers(sc.n, sc.k, cam.width, cam.height, 1 << 18)
        vf.render(fresh, c, prm, precision=P.OCTGS_BF16)
        torch.cuda.synchronize()
        assert np.array_equal(img, _np(vf.rgb))


def test_training_run_refreshes_the_scene(P, orc):
    """A training run recomputes the bound radii from the updated arrays
    (the selection depends on them); the BF16 copy waits for a refresh."""
    sc = S.make_config1()
    ds = P.DeviceScene.from_scene(sc)
    cams = [P.make_camera(c) for c in _cams()[:1]] * 2
    prm = P.raster_params(train=True)
    targets = [torch.zeros(3, 128, 128, device="cuda") for _ in cams]
    mv = P.MultiViewBackward(ds, 128, 128, len(cams), 1 << 18, inflight=2)
    grads = P.SceneGrads(ds)
    mv.run(ds, cams, targets, prm, grads, l1_scale=1e-3)
    mv.check()
    _perturb_in_place(ds, 2)
    say("training run after an in-place update")
    mv.run(ds, cams, targets, prm, grads, l1_scale=1e-3)
    mv.check()
    torch.cuda.synchronize()
    now = _scene_now(sc, ds)
    _, rho = orc.scene_thresholds(now)
    assert np.array_equal(_np(ds.bound_r).view(np.uint32), rho.view(np.uint32))
    # the train step decodes in FP32 and leaves the BF16 copy stale: a BF16
    # render refuses until the scene is refreshed, and then reads the update
    assert not ds.bf16_valid
    vb = P.ViewBuffers(sc.n, sc.k, 128, 128, 1 << 18)
    with pytest.raises(P.OctgsError):
        vb.render(ds, cams[0], P.raster_params(), precision=P.OCTGS_BF16)
    ds.refresh()
    torch.cuda.synchronize()
    assert ds.bf16_valid
    assert np.array_equal(_np(ds.feat_bf16).view(np.uint16), _rne_bits(now.feat))


def test_frame_status_reports_overflow_and_truncation(P):
    sc = S.make_config1()
    ds = P.DeviceScene.from_scene(sc)
    cam = P.make_camera(S.config1_camera())
    prm = P.raster_params()
    say("frame status: clean frame")
    vb = P.ViewBuffers(sc.n, sc.k, 128, 128, 1 << 18)
    vb.render(ds, cam, prm)
    vb.check_status()
    say("frame status: pair overflow")
    vb = P.ViewBuffers(sc.n, sc.k, 128, 128, 64)
    vb.render(ds, cam, prm)
    torch.cuda.synchronize()
    assert int(vb.status.item()) == P.OCTGS_STATUS_PAIR_OVERFLOW
    with pytest.raises(P.OctgsError, match="overflow"):
        vb.check_status()
    say("frame status: truncated decode")
    vb = P.ViewBuffers(sc.n, sc.k, 128, 128, 1 << 18, gauss_capacity=5 * sc.k)
    vb.render(ds, cam, prm)
    torch.cuda.synchronize()
    assert int(vb.status.item()) & P.OCTGS_STATUS_TRUNCATED
    say("frame status: a training step with too small a pair capacity")
    mv = P.MultiViewBackward(ds, 128, 128, 2, 64, inflight=2)
    targets = [torch.zeros(3, 128, 128, device="cuda") for _ in range(2)]
    mv.run(ds, [cam, cam], targets, P.raster_params(train=True), P.SceneGrads(ds), l1_scale=1e-3)
    with pytest.raises(P.OctgsError, match="overflow"):
        mv.check()
