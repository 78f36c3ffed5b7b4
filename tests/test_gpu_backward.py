"""Parity of the HIP backward passes with the oracle's FP64 analytic
gradients (themselves pinned by finite differences), through the C ABI.

Bar: per-array normwise relative error <= 1e-3 (the gradient-check bar),
element-wise within 1e-3 relative on every entry above 1e-6 of its array's
largest (on the end-to-end chain: of anchors that no near-threshold decision
touches), and the FP32 GPU gradient against central differences of the FP64
oracle forward on the 50-anchor 64x64 scene.
"""

import numpy as np
import pytest

from synth import scenes as S
from tests.gpu_util import decision_bounds, elementwise, grad_compare, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_17898_amd as P
    P.lib()
    return P


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("W,H,n,seed", [(64, 48, 400, 1), (97, 61, 1500, 2), (320, 200, 8000, 3)])
def test_raster_backward_parity(P, orc, W, H, n, seed):
    cam = S.look_at((3.0, -20.0, 4.0), (0.0, 0.0, 0.0), W, H, 60.0)
    gf = S.random_gaussians(n, cam, seed, scale=(0.05, 0.6), neg_opacity_frac=0.1,
                            behind_frac=0.05)
    _raster_backward_parity(P, orc, cam, gf, seed)


def test_raster_backward_parity_huge_gaussians(P, orc):
    """40 Gaussians that cover most or all of a 640x400 image's 1,000 tiles
    among 3,000 smaller ones: their pairs span up to 16 chunks of the
    per-Gaussian reduction (several rounds of its chunk walk)."""
    W, H = 640, 400
    cam = S.look_at((3.0, -20.0, 4.0), (0.0, 0.0, 0.0), W, H, 60.0)
    small = S.random_gaussians(3000, cam, 7, scale=(0.05, 0.6), neg_opacity_frac=0.1,
                               behind_frac=0.05)
    huge = S.random_gaussians(40, cam, 8, scale=(1.5, 3.0), opacity=(0.02, 0.2))
    gf = np.concatenate([small, huge], axis=1)
    ref = orc.rasterize(gf, cam, orc.params_array())
    per = np.bincount(ref["bs"]["gid_of"].astype(np.int64), minlength=gf.shape[1])
    say(f"  Gaussians listed in more than 512 tiles: {(per > 512).sum()}, most {per.max()}")
    assert (per > 8 * 64).sum() >= 20
    _raster_backward_parity(P, orc, cam, gf, 4)


def _raster_backward_parity(P, orc, cam, gf, seed):
    W, H, n = cam.width, cam.height, gf.shape[1]
    prm = orc.params_array()
    rng = np.random.default_rng(seed)
    dimg = rng.standard_normal((3, H, W)).astype(np.float32)
    say("raster backward", W, H, n)
    ref = orc.rasterize(gf, cam, prm)
    dproj = orc.composite_backward(ref["pj"], ref["bs"], cam, prm, dimg.astype(np.float64))
    dref = orc.project_backward(gf.astype(np.float64), ref["pj"], cam, prm, dproj)
    vb = P.ViewBuffers(n, 1, W, H, ref["bs"]["n_rect_pairs"] + 16, gauss_capacity=n)
    gt = torch.as_tensor(gf).cuda()
    cnt = torch.tensor([n], dtype=torch.int32).cuda()
    c = P.make_camera(cam)
    vb.rasterize(c, P.raster_params(train=True), gauss=gt, count=cnt)
    vb.gauss.copy_(gt)  # the backward reads the Gaussians of the forward call
    vb.gauss_count.copy_(cnt)
    vb.rasterize_bwd(c, P.raster_params(train=True), torch.as_tensor(dimg).cuda())
    torch.cuda.synchronize()
    got = _np(vb.dgauss).astype(np.float64)
    names = ("mean", "scale", "quat", "opacity", "rgb")
    spans = ((0, 3), (3, 6), (6, 10), (10, 11), (11, 14))
    for nm, (a, b) in zip(names, spans):
        e = rel(got[a:b], dref[a:b])
        say(f"  d{nm}: rel err {e:.2e}")
        assert e <= 1e-3, nm
        # identical FP32 Gaussians: every decision is the same on both sides
        _, nbad, _ = elementwise(got[a:b].T, dref[a:b].T, what="d" + nm)
        assert nbad == 0, nm


@pytest.mark.parametrize("count", [25, 1, 16, 17, 33, 49])
def test_decode_backward_parity(P, orc, count):
    """Anchor lists of 1 to 49 rows: tiles of 16 go to the block's two wave
    groups in pairs, so these cover a lone partial tile, a full pair, a pair
    whose second tile holds one row, and a last pair with no second tile."""
    sc, cam = S.make_gradcheck_scene()
    if count == 25:
        idx = np.arange(1, sc.n, 2, dtype=np.int64)
    else:
        idx = np.random.default_rng(count).permutation(sc.n)[:count].astype(np.int64)
    assert len(idx) == count
    rng = np.random.default_rng(3)
    G = len(idx) * sc.k
    dgauss = rng.standard_normal((14, G)).astype(np.float32)
    say("decode backward", len(idx))
    ref = orc.decode_backward(sc, idx, cam, dgauss.astype(np.float64))
    ds = P.DeviceScene.from_scene(sc)
    grads = P.SceneGrads(ds)
    vb = P.ViewBuffers(sc.n, sc.k, 64, 64, 1 << 12, gauss_capacity=G)
    idx_t = torch.as_tensor(idx.astype(np.int32)).cuda()
    cnt = torch.tensor([len(idx)], dtype=torch.int32).cuda()
    vb.decode_bwd(ds, P.make_camera(cam), grads, dgauss=torch.as_tensor(dgauss).cuda(), idx=idx_t,
                  count=cnt)
    torch.cuda.synchronize()
    got = {k: _np(v) for k, v in grads.all().items()}
    for name, r in ref.items():
        e = rel(got[name], r)
        say(f"  {name}: rel err {e:.2e}")
        assert e <= 1e-4, name
        _, nbad, _ = elementwise(got[name], r, what=name)
        assert nbad == 0, name


def test_decode_bwd_halves_match_whole(P):
    """Two views' decode backwards into one set of gradients: the rows of
    both computed first (separate workspaces) and then applied in view order
    give the same gradients bit for bit as the whole call per view."""
    sc, cam = S.make_gradcheck_scene()
    ds = P.DeviceScene.from_scene(sc)
    c = P.make_camera(cam)
    rng = np.random.default_rng(12)
    views = []
    for m in (37, 45):
        idx = rng.permutation(sc.n)[:m].astype(np.int32)
        dg = rng.standard_normal((14, m * sc.k)).astype(np.float32)
        views.append((torch.as_tensor(idx).cuda(), torch.tensor([m], dtype=torch.int32).cuda(),
                      torch.as_tensor(dg).cuda()))
    whole = P.SceneGrads(ds)
    vbw = P.ViewBuffers(sc.n, sc.k, 64, 64, 1 << 12, gauss_capacity=45 * sc.k)
    for idx, cnt, dg in views:
        vbw.decode_bwd(ds, c, whole, dgauss=dg, idx=idx, count=cnt)
    halves = P.SceneGrads(ds)
    vbs = []
    for idx, cnt, dg in views:
        vb = P.ViewBuffers(sc.n, sc.k, 64, 64, 1 << 12, gauss_capacity=dg.shape[1])
        vb.sel_idx, vb.sel_count, vb.dgauss = idx, cnt, dg
        vb.decode_bwd_rows(ds, c)
        vbs.append(vb)
    for vb in vbs:
        vb.decode_bwd_apply(ds, halves)
    torch.cuda.synchronize()
    a, b = whole.all(), halves.all()
    for name in a:
        x, y = _np(a[name]), _np(b[name])
        assert np.count_nonzero(x) > 0, name
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), name
    # an empty list adds nothing
    before = {k: _np(v).copy() for k, v in halves.all().items()}
    vb = vbs[0]
    vb.sel_count = torch.zeros(1, dtype=torch.int32).cuda()
    vb.decode_bwd_rows(ds, c)
    vb.decode_bwd_apply(ds, halves)
    torch.cuda.synchronize()
    for name, v in halves.all().items():
        # value equality: the weight sums add +0.0, which turns a -0.0 into +0.0
        assert np.array_equal(_np(v), before[name]), name


def test_full_chain_gradient(P, orc):
    """50 anchors, 64x64: GPU FP32 gradient of sum(w * image) against the
    oracle's FP64 analytic gradient and against central differences of the
    oracle forward on sampled coordinates."""
    sc, cam = S.make_gradcheck_scene()
    prm = orc.params_array()
    thr, rho = orc.scene_thresholds(sc)
    rng = np.random.default_rng(7)
    dimg = rng.standard_normal((3, cam.height, cam.width)).astype(np.float32)
    fwd = orc.render(sc, cam, prm, thr, rho)
    ref = orc.render_backward(sc, cam, prm, dimg.astype(np.float64), fwd)
    say("full chain gradient", sc.n)
    ds = P.DeviceScene.from_scene(sc)
    vb = P.ViewBuffers(sc.n, sc.k, cam.width, cam.height, 1 << 16)
    c = P.make_camera(cam)
    pr = P.raster_params(train=True)
    vb.render(ds, c, pr)
    vb.rasterize_bwd(c, pr, torch.as_tensor(dimg).cuda())
    grads = P.SceneGrads(ds)
    vb.decode_bwd(ds, c, grads)
    torch.cuda.synchronize()
    got = {k: _np(v) for k, v in grads.all().items()}
    fr = orc.fragile(fwd, cam, prm, decision_bounds(sc, fwd["idx"], cam, fwd["gauss"]))
    grad_compare(got, ref, fwd, fr, sc.k, what="50 anchors, 64x64")
    # central differences of the FP64 oracle forward, float32-exact steps
    fd_err = []
    for name in ("feat", "offsets", "w1_a", "w2_c", "w2_s"):
        arr = getattr(sc, name) if name in ("feat", "offsets") else sc.mlp[name]
        pick = rng.choice(arr.size, 12, replace=False)
        a_vals, f_vals = [], []
        for fi in pick:
            x = float(arr.flat[fi])
            h = np.float32(2.0 ** -14 * max(1.0, abs(x)))
            vals = []
            for sgn in (1, -1):
                a2 = arr.copy()
                a2.flat[fi] = np.float32(x + sgn * h)
                import copy
                s2 = copy.copy(sc)
                if name in sc.mlp:
                    s2.mlp = dict(sc.mlp)
                    s2.mlp[name] = a2
                else:
                    setattr(s2, name, a2)
                o = orc.render(s2, cam, prm, thr, rho)
                vals.append((float((dimg.astype(np.float64) * o["img"]).sum()), float(a2.flat[fi])))
            f_vals.append((vals[0][0] - vals[1][0]) / (vals[0][1] - vals[1][1]))
            a_vals.append(float(got[name].flat[fi]))
        fd_err.append(rel(a_vals, f_vals))
        say(f"  {name}: GPU vs FD rel err {fd_err[-1]:.2e}")
    assert max(fd_err) <= 1e-3


def test_l1_and_adam(P):
    rng = np.random.default_rng(0)
    a = rng.standard_normal(10007).astype(np.float32)
    b = rng.standard_normal(10007).astype(np.float32)
    at, bt = torch.as_tensor(a).cuda(), torch.as_tensor(b).cuda()
    d = torch.empty_like(at)
    loss = torch.zeros(1, device="cuda")
    say("l1 and adam")
    P.l1_loss_grad(at, bt, 1.0 / a.size, d, loss)
    torch.cuda.synchronize()
    np.testing.assert_allclose(loss.item(), np.abs(a - b).mean(), rtol=1e-5)
    np.testing.assert_array_equal(_np(d), np.sign(a - b).astype(np.float32) / np.float32(a.size))
    p = rng.standard_normal(5000).astype(np.float32)
    g = rng.standard_normal(5000).astype(np.float32)
    pt, gt = torch.as_tensor(p).cuda(), torch.as_tensor(g).cuda()
    m, v = torch.zeros_like(pt), torch.zeros_like(pt)
    pe, me, ve = p.astype(np.float64), np.zeros(5000), np.zeros(5000)
    for step in (1, 2, 3):
        P.adam_step(pt, gt, m, v, 1e-2, step, eps=1e-8)
        me = 0.9 * me + 0.1 * g
        ve = 0.999 * ve + 0.001 * g.astype(np.float64) ** 2
        pe = pe - 1e-2 * (me / (1 - 0.9 ** step)) / (np.sqrt(ve / (1 - 0.999 ** step)) + 1e-8)
    torch.cuda.synchronize()
    np.testing.assert_allclose(_np(pt), pe, rtol=1e-5, atol=1e-6)


def test_autograd_function_matches_direct(P):
    sc, cam = S.make_gradcheck_scene()
    ds = P.DeviceScene.from_scene(sc)
    c = P.make_camera(cam)
    pr = P.raster_params(train=True)
    vb = P.ViewBuffers(sc.n, sc.k, cam.width, cam.height, 1 << 16)
    ts = P.trainable(ds)
    for t in ts:
        t.requires_grad_(True)
    say("autograd function")
    img = P.render_diff(vb, ds, c, pr)
    w = torch.linspace(-1, 1, img.numel(), device="cuda").reshape(img.shape)
    (img * w).sum().backward()
    grads = P.SceneGrads(ds)
    vb2 = P.ViewBuffers(sc.n, sc.k, cam.width, cam.height, 1 << 16)
    with torch.no_grad():
        vb2.render(ds, c, pr)
        vb2.rasterize_bwd(c, pr, w)
        vb2.decode_bwd(ds, c, grads)
    torch.cuda.synchronize()
    names = list(P.render.PARAM_NAMES) + sorted(ds.mlp)
    direct = grads.all()
    for t, nm in zip(ts, names):
        assert t.grad is not None, nm
        assert rel(_np(t.grad), _np(direct[nm])) <= 1e-5, nm


def test_backward_needs_training_forward(P):
    """The forward keeps the pair indices the backward needs only in
    training mode; the backward refuses parameters without that flag."""
    cam = S.look_at((0.0, -8.0, 0.0), (0.0, 0.0, 0.0), 32, 32, 60.0)
    gf = S.random_gaussians(50, cam, 3)
    vb = P.ViewBuffers(50, 1, 32, 32, 1 << 12, gauss_capacity=50)
    gt = torch.as_tensor(gf).cuda()
    cnt = torch.tensor([50], dtype=torch.int32).cuda()
    c = P.make_camera(cam)
    vb.rasterize(c, P.raster_params(), gauss=gt, count=cnt)
    with pytest.raises(P.OctgsError):
        vb.rasterize_bwd(c, P.raster_params(), torch.zeros(3, 32, 32, device="cuda"))


def test_adam_many_matches_single(P):
    """One launch over several arrays (sizes across chunk boundaries, an
    empty one) updates each exactly as the single-array update does."""
    rng = np.random.default_rng(11)
    sizes = [1, 4095, 4096, 4097, 0, 100_003, 37]
    mk = lambda n: torch.as_tensor(rng.standard_normal(n).astype(np.float32)).cuda()
    ps = [mk(n) for n in sizes]
    gs = [mk(n) for n in sizes]
    ms = [(torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")) for n in sizes]
    ref_p = [p.clone() for p in ps]
    ref_m = [(m.clone(), v.clone()) for m, v in ms]
    opt = P.AdamMany(ps, gs, ms)
    for step in (1, 2, 3):
        opt.step(1e-2, step, eps=1e-8)
        for p, g, (m, v) in zip(ref_p, gs, ref_m):
            if p.numel():
                P.adam_step(p, g, m, v, 1e-2, step, eps=1e-8)
    torch.cuda.synchronize()
    for a, b in zip(ps, ref_p):
        assert torch.equal(a, b)
    for (m1, v1), (m2, v2) in zip(ms, ref_m):
        assert torch.equal(m1, m2) and torch.equal(v1, v2)


@pytest.mark.parametrize("n,seed", [(1800, 31), (6000, 32)])
def test_raster_backward_long_tile_lists(P, orc, n, seed):
    """The backward over tiles whose lists hold thousands of entries (each
    pair's emission index travels through the tile sort with it)."""
    cam = S.look_at((0.0, -8.0, 0.0), (0.0, 0.0, 0.0), 48, 32, 60.0)
    gf = S.random_gaussians(n, cam, seed, depth=(3.0, 6.0), scale=(1.5, 3.0), margin=0.0,
                            opacity=(0.002, 0.02))
    prm = orc.params_array()
    rng = np.random.default_rng(seed)
    dimg = rng.standard_normal((3, 32, 48)).astype(np.float32)
    say("raster backward, long lists", n)
    ref = orc.rasterize(gf, cam, prm)
    dproj = orc.composite_backward(ref["pj"], ref["bs"], cam, prm, dimg.astype(np.float64))
    dref = orc.project_backward(gf.astype(np.float64), ref["pj"], cam, prm, dproj)
    vb = P.ViewBuffers(n, 1, 48, 32, ref["bs"]["n_rect_pairs"] + 16, gauss_capacity=n)
    gt = torch.as_tensor(gf).cuda()
    cnt = torch.tensor([n], dtype=torch.int32).cuda()
    c = P.make_camera(cam)
    vb.rasterize(c, P.raster_params(train=True), gauss=gt, count=cnt)
    vb.gauss.copy_(gt)
    vb.gauss_count.copy_(cnt)
    vb.rasterize_bwd(c, P.raster_params(train=True), torch.as_tensor(dimg).cuda())
    torch.cuda.synchronize()
    got = _np(vb.dgauss).astype(np.float64)
    for nm, (a, b) in zip(("mean", "scale", "quat", "opacity", "rgb"),
                          ((0, 3), (3, 6), (6, 10), (10, 11), (11, 14))):
        e = rel(got[a:b], dref[a:b])
        say(f"  d{nm}: rel err {e:.2e}")
        assert e <= 1e-3, nm
