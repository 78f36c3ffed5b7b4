"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars: selections, tile lists and ranges bit-exact; FP32 images within 1e-4
max-abs; decoded attributes within the FP32 / BF16 dot-product error bounds
derived in gpu_util.decode_bounds.  Every input comes from the seeded
generators (synth) or from the oracle; nothing the oracle reads comes from
the GPU.
"""

import ctypes

import numpy as np
import pytest

from synth import scenes as S
from tests.gpu_util import decision_bounds, decoded_field_bounds, e2e_compare, psnr, say

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
def c1():
    return S.make_config1()


def _cams_c1():
    base = S.config1_camera()
    d = np.array([1.0, -2.0, 1.5]) / np.linalg.norm([1.0, -2.0, 1.5])
    cams = [base]
    for dist in (18.0, 9.0, 4.0):  # closer cameras reach levels 1 and 2
        cams.append(S.look_at(dist * d, (0, 0, 0), 128, 128, 60.0))
    cams.append(S.look_at((0.0, 0.0, 40.0), (0.0, 0.0, 80.0), 128, 128, 60.0))  # looks away
    cams.append(S.look_at((2.0, -3.0, 1.0), (0.0, 0.0, 0.0), 97, 61, 70.0))    # ragged size
    return cams


def _np(t):
    return t.detach().cpu().numpy()


def test_prepare_bit_exact(P, orc, c1):
    rng = np.random.default_rng(5)
    sc = c1
    bias = rng.uniform(-0.5, 0.5, sc.n).astype(np.float32)
    for b in (sc.lod_bias, bias):
        say("prepare", "bias" if b is bias else "zero-bias", sc.n)
        ds = P.DeviceScene(sc.pos, sc.level, b, sc.feat, sc.offsets, sc.offset_scale,
                           sc.base_scale, sc.mlp, sc.d_max, sc.n_levels, sc.k, sc.width)
        torch.cuda.synchronize()
        thr = orc.lod_thr2(sc.level, b, sc.d_max)
        rho = orc.bound_radius(sc.offsets, sc.offset_scale, sc.base_scale)
        assert np.array_equal(_np(ds.thr2).view(np.uint32), thr.view(np.uint32))
        assert np.array_equal(_np(ds.bound_r).view(np.uint32), rho.view(np.uint32))


def test_select_bit_exact_c1(P, orc, c1):
    sc = c1
    ds = P.DeviceScene.from_scene(sc)
    thr, rho = orc.scene_thresholds(sc)
    for i, cam in enumerate(_cams_c1()):
        say("select c1 camera", i)
        vb = P.ViewBuffers(sc.n, sc.k, cam.width, cam.height, 1 << 16)
        vb.select(ds, P.make_camera(cam))
        torch.cuda.synchronize()
        m = int(vb.sel_count.item())
        got = _np(vb.sel_idx[:m]).astype(np.int64)
        ref = orc.select(sc, cam, thr, rho)
        assert np.array_equal(got, ref), (i, m, len(ref))
    assert True


def test_select_hand_placed_spheres(P, orc):
    """Spheres just inside and just outside each frustum plane of a rotated,
    non-square, off-centre camera (the oracle's pin cases): the GPU takes
    the oracle's decisions, which are the geometric ones."""
    from tests.test_oracle_visibility import generic_camera, hand_placed_cases, world
    import math as _m
    cam = generic_camera()
    prm = P.raster_params()
    pad = 3.0 * _m.sqrt(float(np.float32(0.3)))
    rows = hand_placed_cases(cam, pad, 1.3)
    n = len(rows)
    pos = world(cam, np.array([r[0] for r in rows])).astype(np.float32)
    rho = np.array([r[1] for r in rows], np.float32)
    want = np.array([r[2] for r in rows])
    k = 1
    rng = np.random.default_rng(0)
    ds = P.DeviceScene(pos, np.zeros(n, np.uint8), np.zeros(n, np.float32),
                       rng.standard_normal((n, 32)).astype(np.float32),
                       np.zeros((n, k, 3), np.float32), np.ones((n, 3), np.float32),
                       np.full((n, 3), 1e-3, np.float32), S.xavier_mlp(rng, 36, 16, k), 100.0, 1,
                       k, 16)
    ds.bound_r.copy_(torch.as_tensor(rho))
    vb = P.ViewBuffers(n, k, cam.width, cam.height, 1 << 12)
    say("select hand-placed spheres", n)
    vb.select(ds, P.make_camera(cam), prm)
    torch.cuda.synchronize()
    m = int(vb.sel_count.item())
    got = np.zeros(n, bool)
    got[_np(vb.sel_idx[:m]).astype(np.int64)] = True
    ref = orc.select_mask(pos, np.full(n, np.inf, np.float32), rho, cam).astype(bool)
    assert np.array_equal(ref, want)
    assert np.array_equal(got, ref)


def test_culling_never_changes_the_image(P, orc):
    """On the GPU too: rendering with the real bound radii equals, bit for
    bit, rendering with every LOD-passing anchor kept (bound radius inf)."""
    from tests.test_oracle_visibility import generic_camera
    sc = S.make_config1()
    cam = generic_camera(C=(5.0, -9.0, 4.0), target=(0.5, 0.0, 0.0))
    prm = P.raster_params()
    ds = P.DeviceScene.from_scene(sc)
    vb = P.ViewBuffers(sc.n, sc.k, cam.width, cam.height, 1 << 18)
    say("culling vs no culling, config 1, rotated off-centre camera")
    vb.render(ds, P.make_camera(cam), prm)
    torch.cuda.synchronize()
    m_cut = int(vb.sel_count.item())
    img_cut, T_cut, last_cut = _np(vb.rgb).copy(), _np(vb.T).copy(), _np(vb.last).copy()
    ds.bound_r.fill_(float("inf"))
    vb.render(ds, P.make_camera(cam), prm)
    torch.cuda.synchronize()
    assert int(vb.sel_count.item()) > m_cut + 100
    assert np.array_equal(_np(vb.rgb), img_cut)
    assert np.array_equal(_np(vb.T), T_cut)
    assert np.array_equal(_np(vb.last), last_cut)


def test_select_bit_exact_random_bias(P, orc):
    rng = np.random.default_rng(2)
    n, K = 300_001, 7
    pos = rng.uniform(-100, 100, (n, 3)).astype(np.float32)
    level = rng.integers(0, K, n).astype(np.uint8)
    bias = rng.uniform(-0.5, 0.5, n).astype(np.float32)
    k = 4
    offsets = rng.normal(0, 0.5, (n, k, 3)).astype(np.float32)
    osc = np.exp(rng.uniform(-2, 0, (n, 3))).astype(np.float32)
    bsc = np.exp(rng.uniform(-3, -1, (n, 3))).astype(np.float32)
    mlp = S.xavier_mlp(rng, 36, 16, k)
    feat = rng.standard_normal((n, 32)).astype(np.float32)
    say("select random-bias", n)
    ds = P.DeviceScene(pos, level, bias, feat, offsets, osc, bsc, mlp, 180.0, K, k, 16)
    thr = orc.lod_thr2(level, bias, 180.0)
    rho = orc.bound_radius(offsets, osc, bsc)
    for seed in range(4):
        cam = S.random_views(1, seed, 80.0, 5.0, 120.0, 640, 480)[0]
        vb = P.ViewBuffers(n, k, 640, 480, 1 << 16, gauss_capacity=1024)
        vb.select(ds, P.make_camera(cam))
        torch.cuda.synchronize()
        m = int(vb.sel_count.item())
        ref = np.flatnonzero(orc.select_mask(pos, thr, rho, cam))
        assert np.array_equal(_np(vb.sel_idx[:m]).astype(np.int64), ref)
        assert m > 0


@pytest.mark.parametrize("bf16", [False, True])
def test_decode_within_bounds(P, orc, c1, bf16):
    sc = c1
    cam = S.config1_camera()
    idx = np.arange(3, sc.n, 5, dtype=np.int64)  # generator-chosen anchor list
    say("decode", "bf16" if bf16 else "fp32", len(idx))
    ds = P.DeviceScene.from_scene(sc)
    vb = P.ViewBuffers(sc.n, sc.k, 128, 128, 1 << 16)
    idx_t = torch.as_tensor(idx.astype(np.int32)).cuda()
    cnt_t = torch.tensor([len(idx)], dtype=torch.int32).cuda()
    vb.decode(ds, P.make_camera(cam), P.OCTGS_BF16 if bf16 else P.OCTGS_FP32, idx=idx_t, count=cnt_t)
    torch.cuda.synchronize()
    G = len(idx) * sc.k
    assert int(vb.gauss_count.item()) == G
    got = _np(vb.gauss[:, :G]).astype(np.float64)
    ref = orc.decode(sc, idx, cam)
    bound = decoded_field_bounds(sc, idx, cam, ref, bf16)
    err = np.abs(got - ref)
    for f in range(14):
        ratio = (err[f] / np.maximum(bound[f], 1e-30)).max()
        say(f"  field {f}: max err {err[f].max():.2e}  max err/bound {ratio:.3f}")
    assert np.all(err <= bound), np.argwhere(err > bound)[:5]


def _gpu_raster(P, vb, gf, cam, prm):
    gt = torch.as_tensor(gf).cuda()
    cnt = torch.tensor([gf.shape[1]], dtype=torch.int32).cuda()
    vb.rasterize(P.make_camera(cam), prm, gauss=gt, count=cnt)
    torch.cuda.synchronize()


CASES = [(64, 64, 300, 1), (128, 128, 3000, 2), (97, 61, 1500, 3), (333, 200, 20000, 4),
         (1600, 1066, 60000, 5)]


@pytest.mark.parametrize("W,H,n,seed", CASES)
def test_raster_stage_parity(P, orc, W, H, n, seed):
    _stage_parity(P, orc, W, H, n, seed, (0.01, 0.4))


def test_raster_three_tile_sort_passes(P, orc):
    """An image of more than 2^16 tiles (8192 x 2112: 512 x 132 = 67,584),
    so tile ids take 17 bits and the tile sort runs three 8-bit passes; the
    bottom four tile rows (ids from 65,536) hold ~57k of the 1.76M pairs."""
    assert (8192 // 16) * (2112 // 16) > 1 << 16
    _stage_parity(P, orc, 8192, 2112, 30000, 6, (0.005, 0.05), min_high_tile=1 << 16)


def _stage_parity(P, orc, W, H, n, seed, scale, min_high_tile=None):
    cam = S.look_at((3.0, -20.0, 4.0), (0.0, 0.0, 0.0), W, H, 60.0)
    gf = S.random_gaussians(n, cam, seed, scale=scale, neg_opacity_frac=0.1,
                            behind_frac=0.05)
    prm_o = orc.params_array()
    say("raster stage", W, H, n, seed)
    ref = orc.rasterize(gf, cam, prm_o, weights=True)
    P_ref = ref["bs"]["n_pairs"]
    C_ref = ref["bs"]["n_rect_pairs"]
    # capacity exactly the candidate count: the tightest that must not overflow
    vb = P.ViewBuffers(n, 1, W, H, max(C_ref, 1), gauss_capacity=n, log_weights=True)
    _gpu_raster(P, vb, gf, cam, P.raster_params())
    st = vb.stats()
    assert st["sync_error"] == 0 and st["pair_overflow"] == 0
    assert st["n_visible"] == ref["pj"]["n_visible"]
    assert st["n_candidates"] == C_ref
    assert st["n_pairs"] == P_ref
    tile, slot, ranges = vb.sorted_lists()
    if min_high_tile is not None:
        say(f"  pairs with tile id >= {min_high_tile}: {int((tile >= min_high_tile).sum())}")
        assert (tile >= min_high_tile).sum() > 1000
    assert np.array_equal(tile, ref["bs"]["tile_of"])
    assert np.array_equal(slot, ref["bs"]["gid_of"])
    assert np.array_equal(ranges, ref["bs"]["ranges"])
    img = _np(vb.rgb).astype(np.float64)
    T = _np(vb.T).astype(np.float64)
    e_img = np.abs(img - ref["img"]).max()
    e_T = np.abs(T - ref["T"]).max()
    same_last = np.mean(_np(vb.last) == ref["last"])
    say(f"  img max abs {e_img:.2e}  PSNR {psnr(img, ref['img']):.1f} dB  T max abs {e_T:.2e}"
        f"  last equal {same_last:.6f}")
    assert e_img <= 1e-4 and e_T <= 1e-4
    assert same_last >= 0.999
    w = _np(vb.gauss_w).astype(np.float64)
    np.testing.assert_allclose(w, ref["weights"], rtol=2e-4, atol=2e-4)


@pytest.mark.parametrize("alpha_min,log", [(0.0, False), (1.0 / 255.0, False), (0.0, True),
                                             (1.0 / 255.0, True)])
def test_forward_without_entry_count(P, alpha_min, log):
    """A forward with a null `last` (a render that no backward follows)
    writes the same image, transmittance and blend-weight log bit for bit,
    leaves the `last` buffer alone, and the backward then refuses to run."""
    W, H, n = 333, 200, 20000
    cam = S.look_at((3.0, -20.0, 4.0), (0.0, 0.0, 0.0), W, H, 60.0)
    gf = S.random_gaussians(n, cam, 9, scale=(0.01, 0.4), neg_opacity_frac=0.1,
                            behind_frac=0.05)
    say("forward without last", alpha_min, log)
    prm = P.raster_params(alpha_min=alpha_min)
    vb = P.ViewBuffers(n, 1, W, H, 1 << 22, gauss_capacity=n, log_weights=log)
    gt = torch.as_tensor(gf).cuda()
    cnt = torch.tensor([n], dtype=torch.int32).cuda()
    c = P.make_camera(cam)
    out = []
    for keep in (True, False):
        vb.last.fill_(-7)
        if log:
            vb.gauss_w.zero_()
        vb.rasterize(c, prm, gauss=gt, count=cnt, keep_last=keep)
        torch.cuda.synchronize()
        out.append((_np(vb.rgb).copy(), _np(vb.T).copy(), _np(vb.last).copy(),
                    _np(vb.gauss_w).copy() if log else None))
    (i1, t1, l1, w1), (i2, t2, l2, w2) = out
    assert np.array_equal(i1.view(np.uint32), i2.view(np.uint32))
    assert np.array_equal(t1.view(np.uint32), t2.view(np.uint32))
    assert (l1 >= 0).all() and (l2 == -7).all()
    if log:
        # per-slot sums gathered with float atomics: the order can differ
        np.testing.assert_allclose(w1, w2, rtol=1e-5, atol=1e-7)
    with pytest.raises(P.OctgsError):
        vb.rasterize_bwd(c, prm, torch.zeros(3, H, W, device="cuda"))


def test_raster_equal_depths(P, orc):
    cam = S.look_at((0.0, 0.0, -10.0), (0.0, 0.0, 0.0), 64, 64, 60.0)
    gf = S.tile_aligned_gaussians(cam, [5.0] * 40 + [7.0] * 40, seed=3)
    say("raster equal depths")
    ref = orc.rasterize(gf, cam, orc.params_array())
    vb = P.ViewBuffers(80, 1, 64, 64, 4096, gauss_capacity=80)
    _gpu_raster(P, vb, gf, cam, P.raster_params())
    tile, slot, ranges = vb.sorted_lists()
    assert np.array_equal(slot, ref["bs"]["gid_of"])
    assert np.abs(_np(vb.rgb) - ref["img"]).max() <= 1e-4


def test_end_to_end_c1(P, orc, c1):
    sc = c1
    ds = P.DeviceScene.from_scene(sc)
    prm = P.raster_params()
    thr, rho = orc.scene_thresholds(sc)
    for prec in (P.OCTGS_FP32, P.OCTGS_BF16):
        for i, cam in enumerate(_cams_c1()[:4]):
            say("end-to-end c1", "bf16" if prec else "fp32", i)
            vb = P.ViewBuffers(sc.n, sc.k, cam.width, cam.height, 1 << 18)
            vb.render(ds, P.make_camera(cam), prm, precision=prec)
            torch.cuda.synchronize()
            ref = orc.render(sc, cam, orc.params_array(), thr, rho)
            m = int(vb.sel_count.item())
            assert np.array_equal(_np(vb.sel_idx[:m]).astype(np.int64), ref["idx"])
            if prec == P.OCTGS_FP32:
                eb = decision_bounds(sc, ref["idx"], cam, ref["gauss"])
                fr = orc.fragile(ref, cam, orc.params_array(), eb)
                e2e_compare(vb, ref, fr, 1e-4, min_checked=0.3, what=f"c1 view {i}")
            else:
                img = _np(vb.rgb).astype(np.float64)
                err = np.abs(img - ref["img"])
                p = psnr(img, ref["img"])
                say(f"  BF16: max abs {err.max():.2e} PSNR {p:.1f} dB")
                assert p >= 40.0


def test_zero_anchors_and_zero_selected(P, orc):
    say("zero anchors")
    k = 2
    rng = np.random.default_rng(0)
    mlp = S.xavier_mlp(rng, 36, 16, k)
    e = np.zeros((0, 3), np.float32)
    ds = P.DeviceScene(e, np.zeros(0, np.uint8), np.zeros(0, np.float32), np.zeros((0, 32), np.float32),
                       np.zeros((0, k, 3), np.float32), e, e, mlp, 10.0, 1, k, 16)
    cam = S.look_at((0, -5, 0), (0, 0, 0), 48, 40, 60.0)
    vb = P.ViewBuffers(0, k, 48, 40, 1024, gauss_capacity=16)
    vb.render(ds, P.make_camera(cam), P.raster_params(bg=(0.25, 0.5, 0.75)))
    torch.cuda.synchronize()
    assert int(vb.sel_count.item()) == 0
    img = _np(vb.rgb)
    for c, v in enumerate((0.25, 0.5, 0.75)):
        assert np.all(img[c] == np.float32(v))
    assert np.all(_np(vb.T) == 1.0) and np.all(_np(vb.last) == 0)


def test_all_behind_near_plane(P, orc):
    cam = S.look_at((0, 0, 0), (0, 0, 10), 64, 64, 60.0)
    gf = S.random_gaussians(500, cam, 1, behind_frac=1.0)
    say("all behind")
    vb = P.ViewBuffers(500, 1, 64, 64, 1024, gauss_capacity=500)
    _gpu_raster(P, vb, gf, cam, P.raster_params())
    st = vb.stats()
    assert st["n_visible"] == 0 and st["n_pairs"] == 0
    assert np.all(_np(vb.rgb) == 0.0)


def test_pair_overflow_flag(P, orc):
    cam = S.look_at((3.0, -20.0, 4.0), (0.0, 0.0, 0.0), 128, 128, 60.0)
    gf = S.random_gaussians(2000, cam, 7)
    ref = orc.rasterize(gf, cam, orc.params_array())
    say("pair overflow")
    # a capacity between the kept pairs and the candidates still overflows:
    # candidates are written before the ellipse test
    cap = (ref["bs"]["n_pairs"] + ref["bs"]["n_rect_pairs"]) // 2
    assert ref["bs"]["n_pairs"] < cap < ref["bs"]["n_rect_pairs"]
    vb = P.ViewBuffers(2000, 1, 128, 128, cap, gauss_capacity=2000)
    _gpu_raster(P, vb, gf, cam, P.raster_params())
    st = vb.stats()
    assert st["pair_overflow"] == 1 and st["n_candidates"] == ref["bs"]["n_rect_pairs"]
    assert st["n_pairs"] == 0
    assert np.all(_np(vb.rgb) == 0.0)


def test_degenerate_quaternion_decodes_to_identity(P, orc, c1):
    sc = S.make_config1()
    for key in ("w1_s", "b1_s", "w2_s", "b2_s"):
        sc.mlp[key][:] = 0.0
    cam = S.config1_camera()
    ds = P.DeviceScene.from_scene(sc)
    vb = P.ViewBuffers(sc.n, sc.k, 128, 128, 1 << 16)
    idx = torch.arange(0, 64, dtype=torch.int32).cuda()
    cnt = torch.tensor([64], dtype=torch.int32).cuda()
    say("degenerate quaternion")
    vb.decode(ds, P.make_camera(cam), P.OCTGS_FP32, idx=idx, count=cnt)
    torch.cuda.synchronize()
    q = _np(vb.gauss[6:10, :64 * sc.k])
    assert np.all(q[0] == 1.0) and np.all(q[1:] == 0.0)
    np.testing.assert_allclose(_np(vb.gauss[3:6, :64 * sc.k]),
                               0.5 * np.repeat(sc.base_scale[:64], sc.k, axis=0).T, rtol=1e-6)


def test_invalid_arguments_rejected(P):
    import ctypes
    from paper_2403_17898_amd import _lib as L
    lib = L.lib()
    assert lib.octgs_select_lod(None, None, None, None, None, None, 0, None) == L.OCTGS_EINVAL
    assert lib.octgs_raster_workspace_bytes(-1, 0, 10, 10) == 0
    g = L.Gaussians()
    assert lib.octgs_rasterize_fwd(ctypes.byref(g), None, None, 0, None, None, None, None, None, 0,
                                   None, None) == L.OCTGS_EINVAL
    # the decode backward's halves check their pointers before any launch
    assert lib.octgs_decode_bwd_rows(None, None, None, None, None, None, 0, None, 0,
                                     None) == L.OCTGS_EINVAL
    assert lib.octgs_decode_bwd_apply(None, None, None, None, 0, None, None, None, 0,
                                      None) == L.OCTGS_EINVAL
    assert lib.octgs_decode_bwd_workspace_bytes(-1, 10, 64) == 0
    assert lib.octgs_decode_bwd_workspace_bytes(100, 17, 64) == 0  # k above 16


# --------------------------------------------------------------------------
# LOD transition blending (Sec. IV-A)
# --------------------------------------------------------------------------

def _blend_scene(c1):
    """Config 1 with a random LOD bias, so transition anchors span levels."""
    rng = np.random.default_rng(21)
    sc = S.make_config1()
    sc.lod_bias = rng.uniform(-0.6, 0.6, sc.n).astype(np.float32)
    return sc


def test_select_blend_bit_exact(P, orc, c1):
    sc = _blend_scene(c1)
    ds = P.DeviceScene.from_scene(sc)
    thr, rho = orc.scene_thresholds(sc)
    for i, cam in enumerate(_cams_c1()):
        say("select blend camera", i)
        vb = P.ViewBuffers(sc.n, sc.k, cam.width, cam.height, 1 << 16)
        vb.select(ds, P.make_camera(cam, lod_blend=True))
        torch.cuda.synchronize()
        m = int(vb.sel_count.item())
        got = _np(vb.sel_idx[:m]).astype(np.int64)
        ref = orc.select(sc, cam, thr, rho, blend=True)
        assert np.array_equal(got, ref), (i, m, len(ref))
        assert len(ref) >= len(orc.select(sc, cam, thr, rho))


def test_decode_blend_factor(P, orc, c1):
    """Blended decode equals the plain decode except the opacity, which is
    scaled by the transition factor (FP32 log2 of the distance ratio: a few
    ulp of L* on top of the opacity's own bound)."""
    sc = _blend_scene(c1)
    cam = S.look_at(9.0 * np.array([1.0, -2.0, 1.5]) / np.linalg.norm([1.0, -2.0, 1.5]),
                    (0, 0, 0), 128, 128, 60.0)
    thr, rho = orc.scene_thresholds(sc)
    idx = orc.select(sc, cam, thr, rho, blend=True)
    say("decode blend", len(idx))
    ds = P.DeviceScene.from_scene(sc)
    vb = P.ViewBuffers(sc.n, sc.k, 128, 128, 1 << 16)
    idx_t = torch.as_tensor(idx.astype(np.int32)).cuda()
    cnt_t = torch.tensor([len(idx)], dtype=torch.int32).cuda()
    vb.decode(ds, P.make_camera(cam, lod_blend=True), P.OCTGS_FP32, idx=idx_t, count=cnt_t)
    torch.cuda.synchronize()
    G = len(idx) * sc.k
    got = _np(vb.gauss[:, :G]).astype(np.float64)
    ref = orc.decode(sc, idx, cam, blend=True)
    plain = orc.decode(sc, idx, cam)
    bound = decoded_field_bounds(sc, idx, cam, plain, False)
    err = np.abs(got - ref)
    for f in range(14):
        if f != 10:
            assert np.all(err[f] <= bound[f]), f
    fac = np.divide(ref[10], plain[10], out=np.ones_like(ref[10]), where=plain[10] != 0)
    assert np.all(err[10] <= bound[10] * np.abs(fac) + 8e-6 * np.abs(plain[10]) + 1e-7)
    # some anchors are in transition (0 < factor < 1) and none above L_hat + 1
    assert np.any((fac > 0.01) & (fac < 0.99)) and np.all((fac >= 0) & (fac <= 1 + 1e-12))


def test_end_to_end_blend_c1(P, orc, c1):
    sc = _blend_scene(c1)
    ds = P.DeviceScene.from_scene(sc)
    prm = P.raster_params()
    thr, rho = orc.scene_thresholds(sc)
    for i, cam in enumerate(_cams_c1()[:4]):
        say("end-to-end blend c1", i)
        vb = P.ViewBuffers(sc.n, sc.k, cam.width, cam.height, 1 << 18)
        vb.render(ds, P.make_camera(cam, lod_blend=True), prm, precision=P.OCTGS_FP32)
        torch.cuda.synchronize()
        ref = orc.render(sc, cam, orc.params_array(), thr, rho, blend=True)
        m = int(vb.sel_count.item())
        assert np.array_equal(_np(vb.sel_idx[:m]).astype(np.int64), ref["idx"])
        # the opacity also carries the FP32 transition factor's error
        eb = decision_bounds(sc, ref["idx"], cam, ref["gauss"])
        plain = orc.decode(sc, ref["idx"], cam)
        eb[10] = eb[10] + 8e-6 * np.abs(plain[10]) + 1e-7
        fr = orc.fragile(ref, cam, orc.params_array(), eb)
        e2e_compare(vb, ref, fr, 1e-4, min_checked=0.3, what=f"c1 blended view {i}")


def test_decode_bwd_rejects_blend(P, c1):
    sc = c1
    ds = P.DeviceScene.from_scene(sc)
    cam = S.config1_camera()
    vb = P.ViewBuffers(sc.n, sc.k, 128, 128, 1 << 16)
    vb.render(ds, P.make_camera(cam), P.raster_params(train=True))
    vb.rasterize_bwd(P.make_camera(cam), P.raster_params(train=True), torch.ones_like(vb.rgb))
    grads = P.SceneGrads(ds)
    with pytest.raises(P.OctgsError):
        vb.decode_bwd(ds, P.make_camera(cam, lod_blend=True), grads)


@pytest.mark.parametrize("bf16", [False, True])
def test_decode_follows_weight_updates(P, orc, c1, bf16):
    """Each decode call rewrites its weight fragments from the MLP as it is
    at that moment: after the weights change in place, the next decode with
    the same workspace matches the oracle's decode of the new weights (and
    differs from the old result); a workspace below the stated size is
    rejected."""
    import copy
    sc = copy.copy(c1)
    sc.mlp = {k: v.copy() for k, v in c1.mlp.items()}
    cam = S.config1_camera()
    idx = np.arange(0, sc.n, 3, dtype=np.int64)
    prec = P.OCTGS_BF16 if bf16 else P.OCTGS_FP32
    ds = P.DeviceScene.from_scene(sc)
    vb = P.ViewBuffers(sc.n, sc.k, 128, 128, 1 << 16)
    idx_t = torch.as_tensor(idx.astype(np.int32)).cuda()
    cnt_t = torch.tensor([len(idx)], dtype=torch.int32).cuda()
    c = P.make_camera(cam)
    G = len(idx) * sc.k
    vb.decode(ds, c, prec, idx=idx_t, count=cnt_t)
    torch.cuda.synchronize()
    first = _np(vb.gauss[:, :G]).copy()
    rng = np.random.default_rng(5)
    for name in sorted(sc.mlp):
        sc.mlp[name] = (sc.mlp[name] * np.float32(0.5)
                        + np.float32(0.1) * rng.standard_normal(sc.mlp[name].shape)
                        ).astype(np.float32)
        ds.mlp[name].copy_(torch.as_tensor(sc.mlp[name]))
    say("decode after a weight update", "bf16" if bf16 else "fp32", len(idx))
    vb.decode(ds, c, prec, idx=idx_t, count=cnt_t)
    torch.cuda.synchronize()
    got = _np(vb.gauss[:, :G]).astype(np.float64)
    ref = orc.decode(sc, idx, cam)
    bound = decoded_field_bounds(sc, idx, cam, ref, bf16)
    assert np.all(np.abs(got - ref) <= bound)
    assert np.abs(got[10:] - first[10:]).max() > 1e-3
    from paper_2403_17898_amd import _lib as L
    need = L.lib().octgs_decode_workspace_bytes(int(prec))
    assert need > 0 and L.lib().octgs_decode_workspace_bytes(7) == 0
    r = L.lib().octgs_decode(ctypes.byref(ds.anchors), ctypes.byref(ds._mlp), ctypes.byref(c),
                             idx_t.data_ptr(), cnt_t.data_ptr(), int(prec), ctypes.byref(vb._g),
                             vb.dec_fwd_ws.data_ptr(), need - 16, None)
    assert r == L.OCTGS_EINVAL


@pytest.mark.parametrize("k,W", [(1, 16), (16, 64), (7, 48), (13, 32)])
def test_decode_shapes(P, orc, k, W):
    """Decode forward (FP32 and BF16, within the per-element bounds) and the
    fused decode backward (against the oracle's FP64 gradients) at the
    extremes of the supported shapes: k = 1..16 Gaussians per anchor, MLP
    width 16..64, with a ragged anchor count (not a multiple of the tile)."""
    sc, cam = S.make_gradcheck_scene(seed=11 + k, n=77, k=k, width=W)
    idx = np.arange(0, sc.n, dtype=np.int64)[::-1][:71].copy()
    ds = P.DeviceScene.from_scene(sc)
    G = len(idx) * k
    vb = P.ViewBuffers(sc.n, k, 64, 64, 1 << 14, gauss_capacity=G + 5 * k)
    idx_t = torch.as_tensor(idx.astype(np.int32)).cuda()
    cnt_t = torch.tensor([len(idx)], dtype=torch.int32).cuda()
    c = P.make_camera(cam)
    ref = orc.decode(sc, idx, cam)
    for bf16 in (False, True):
        say(f"decode k={k} W={W}", "bf16" if bf16 else "fp32")
        vb.decode(ds, c, P.OCTGS_BF16 if bf16 else P.OCTGS_FP32, idx=idx_t, count=cnt_t)
        torch.cuda.synchronize()
        assert int(vb.gauss_count.item()) == G
        got = _np(vb.gauss[:, :G]).astype(np.float64)
        bound = decoded_field_bounds(sc, idx, cam, ref, bf16)
        assert np.all(np.abs(got - ref) <= bound), np.argwhere(np.abs(got - ref) > bound)[:5]
    rng = np.random.default_rng(k * 100 + W)
    dg = rng.standard_normal((14, G)).astype(np.float32)
    want = orc.decode_backward(sc, idx, cam, dg.astype(np.float64))
    grads = P.SceneGrads(ds)
    dgt = torch.zeros(14, vb.gcap, device="cuda")
    dgt[:, :G] = torch.as_tensor(dg).cuda()
    vb.decode_bwd(ds, c, grads, dgauss=dgt, idx=idx_t, count=cnt_t)
    torch.cuda.synchronize()
    got = {n: _np(v) for n, v in grads.all().items()}
    for name, r in want.items():
        a, b = np.asarray(got[name], np.float64), np.asarray(r, np.float64)
        e = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
        say(f"  d{name}: rel err {e:.2e}")
        assert e <= 1e-4, name


@pytest.mark.parametrize("n,seed", [(300, 21), (1800, 22), (6000, 23)])
def test_raster_long_tile_lists(P, orc, n, seed):
    """Every Gaussian covers every tile of a 48x32 image, so each tile's list
    holds exactly n entries (up to 6000, longer than any benchmark view's).
    Sorted lists and tile ranges bit-exact, image within 1e-4, blend-weight
    log within its bar."""
    cam = S.look_at((0.0, -8.0, 0.0), (0.0, 0.0, 0.0), 48, 32, 60.0)
    gf = S.random_gaussians(n, cam, seed, depth=(3.0, 6.0), scale=(1.5, 3.0), margin=0.0,
                            opacity=(0.002, 0.02))
    prm_o = orc.params_array()
    say("raster long lists", n, seed)
    ref = orc.rasterize(gf, cam, prm_o, weights=True)
    lens = ref["bs"]["ranges"][:, 1].astype(np.int64) - ref["bs"]["ranges"][:, 0]
    say(f"  list lengths {lens.min()}..{lens.max()}")
    vb = P.ViewBuffers(n, 1, 48, 32, max(ref["bs"]["n_rect_pairs"], 1), gauss_capacity=n,
                       log_weights=True)
    _gpu_raster(P, vb, gf, cam, P.raster_params())
    st = vb.stats()
    assert st["sync_error"] == 0 and st["pair_overflow"] == 0
    assert st["n_pairs"] == ref["bs"]["n_pairs"]
    tile, slot, ranges = vb.sorted_lists()
    assert np.array_equal(tile, ref["bs"]["tile_of"])
    assert np.array_equal(slot, ref["bs"]["gid_of"])
    assert np.array_equal(ranges, ref["bs"]["ranges"])
    img = _np(vb.rgb).astype(np.float64)
    e = np.abs(img - ref["img"]).max()
    say(f"  img max abs {e:.2e}")
    assert e <= 1e-4
    np.testing.assert_allclose(_np(vb.gauss_w).astype(np.float64), ref["weights"], rtol=2e-4,
                               atol=2e-4)
