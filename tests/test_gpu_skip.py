"""Learned anchor skip on the GPU: inputs, training gradients, BF16
prediction and ordered compaction against the oracle; blend-weight logging;
and what the trained predictor gains over the path without it."""

import math

import numpy as np
import pytest

from synth import scenes as S
from tests.gpu_util import U32, UBF, say

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
def SK(P):
    from paper_2403_17898_amd import skip as SK
    return SK


def _np(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _listed(P, sc, cam, idx):
    ds = P.DeviceScene.from_scene(sc)
    vb = P.ViewBuffers(sc.n, sc.k, cam.width, cam.height, 1 << 16)
    vb.sel_idx[:len(idx)].copy_(torch.as_tensor(idx.astype(np.int32)))
    vb.sel_count.fill_(len(idx))
    return ds, vb


def test_features_parity(P, SK, orc):
    sc = S.make_config1()
    sc.level = np.random.default_rng(0).integers(0, 3, sc.n).astype(np.uint8)
    cam = S.config1_camera()
    idx = np.arange(2, sc.n, 3, dtype=np.int64)
    say("skip features", len(idx))
    ds, vb = _listed(P, sc, cam, idx)
    z = torch.empty(sc.n, 37, device="cuda")
    SK.features(vb, ds, P.make_camera(cam), z)
    torch.cuda.synchronize()
    got = _np(z[:len(idx)]).astype(np.float64)
    ref = orc.skip_features(sc, idx, cam)
    assert np.abs(got - ref).max() <= 1e-5


def bf16_round(x):
    """FP32 -> nearest BF16 (ties to even), returned as float64."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _grad_bounds(z, y, net, pw, depth, lam=8.0):
    """Bounds on |GPU - exact| for the fused BF16 training pass, per gradient
    entry and for the loss.  z and the weights are taken already rounded as
    the kernel rounds them (BF16 copies of z, w1, w2), so the exact values
    are the gradient of that network; what remains is the rounding of
    ReLU(layer 1), dH2 and dH1 to BF16 (u = 2^-8) and FP32 arithmetic.
    Per row, first-order worst-case error terms are propagated through the
    forward and backward; a ReLU mask counts as uncertain wherever its
    pre-activation lies within its error bound.  Rows round independently,
    so their contributions to a batch sum are combined as lam times the root
    sum of squares (Hoeffding: each entry exceeds it with probability below
    2 exp(-lam^2 / 2)), plus the worst-case FP32 summation error gamma_depth
    sum |term| of a sum evaluated `depth` additions deep."""
    w1, b1, w2, b2, w3, b3 = (np.asarray(net[k], np.float64)
                              for k in ("w1", "b1", "w2", "b2", "w3", "b3"))
    w3 = w3[:, 0]
    B = z.shape[0]
    u, g, gd = UBF, 70 * U32, depth * U32
    az, A1, A2, A3 = np.abs(z), np.abs(w1), np.abs(w2), np.abs(w3)
    a1 = z @ w1 + b1
    h1 = np.maximum(a1, 0)
    e_a1 = g * (az @ A1 + np.abs(b1))
    e_h1 = e_a1 + u * (h1 + e_a1)
    H1 = h1 + e_h1
    a2 = h1 @ w2 + b2
    h2 = np.maximum(a2, 0)
    e_a2 = e_h1 @ A2 + g * (H1 @ A2 + np.abs(b2))
    H2 = h2 + e_a2
    x = h2 @ w3 + b3[0]
    e_x = e_a2 @ A3 + g * (H2 @ A3 + abs(b3[0]))
    wgt = np.where(y > 0.5, pw, 1.0)
    sg = 1.0 / (1.0 + np.exp(-x))
    dx = wgt * (sg - y) / B
    e_dx = wgt / B * (e_x / 4 + 8 * U32)
    adx = np.abs(dx)
    D2 = np.outer(adx + e_dx, A3)                           # >= |dH2|
    e_d2 = (np.abs(a2) <= e_a2) * D2 + np.outer(e_dx, A3) + U32 * D2
    e_d2b = e_d2 + u * D2
    pre = D2 @ A2.T
    e_pre = e_d2b @ A2.T + g * pre
    D1 = pre + e_pre                                        # >= |dH1|
    e_d1 = (np.abs(a1) <= e_a1) * D1 + e_pre
    e_d1b = e_d1 + u * D1
    rss = lambda sq: lam * np.sqrt(sq)
    e = {}
    e["b3"] = np.array([rss(np.sum(e_dx ** 2)) + gd * adx.sum()])
    e["w3"] = (rss(2 * (e_a2 ** 2).T @ (adx ** 2) + 2 * (H2 ** 2).T @ (e_dx ** 2))
               + gd * (H2.T @ adx))[:, None]
    e["b2"] = rss((e_d2 ** 2).sum(0)) + gd * D2.sum(0)
    e["w2"] = (rss(2 * (e_h1 ** 2).T @ (D2 ** 2) + 2 * (H1 ** 2).T @ (e_d2b ** 2))
               + gd * (H1.T @ D2))
    e["b1"] = rss((e_d1 ** 2).sum(0)) + gd * D1.sum(0)
    e["w1"] = rss((az ** 2).T @ (e_d1b ** 2)) + gd * (az.T @ D1)
    sp = np.maximum(x, 0) + np.log1p(np.exp(-np.abs(x)))
    t_loss = wgt / B * (sp + np.abs(y * x))
    e_row = wgt / B * (np.abs(sg - y) * e_x) + 8 * U32 * t_loss
    e_loss = float(rss(np.sum(e_row ** 2)) + gd * t_loss.sum())
    return e, e_loss


def _check_train(SK, orc, z, y, rows, mask_cols, pw, seed):
    """One fused training pass against the oracle's FP64 gradient of the
    network the kernel evaluates (BF16-rounded z, w1, w2), entry by entry
    within the derived bound."""
    net = SK.SkipNet(seed=seed, inputs=mask_cols)
    zt, yt = torch.as_tensor(z).cuda(), torch.as_tensor(y).cuda()
    rt = None if rows is None else torch.as_tensor(rows.astype(np.int32)).cuda()
    loss = torch.full((1,), 0.25, device="cuda")
    net.train_grad(zt, yt, pw, loss, rows=rt)
    torch.cuda.synchronize()
    zb = (z[rows] if rows is not None else z).astype(np.float64)
    yb = (y[rows] if rows is not None else y).astype(np.float64)
    if mask_cols is not None:
        off = np.setdiff1d(np.arange(37), np.asarray(list(mask_cols)))
        zb[:, off] = 0.0
    B = zb.shape[0]
    w = net.numpy()
    wr = dict(w, w1=bf16_round(w["w1"]), w2=bf16_round(w["w2"]))
    zr = bf16_round(zb)
    _, lref, gref = orc.skip_mlp(zr, wr, yb.astype(np.float32), pos_weight=pw, grads=True)
    # the kernel sums each block's rows, then the block sums in order
    nblk = min((B + 63) // 64, 256)
    depth = 64 * ((B + 64 * nblk - 1) // (64 * nblk)) + nblk
    eb, eloss = _grad_bounds(zr, yb, wr, pw, depth)
    got_loss = loss.item() - 0.25
    say(f"  loss {got_loss:.6f} ref {lref:.6f} err/bound {abs(got_loss - lref) / eloss:.3f}")
    assert abs(got_loss - lref) <= eloss + 2 * U32
    for k in SK.SKIP_ORDER:
        got = _np(net.g[k]).astype(np.float64).reshape(gref[k].shape)
        bound = eb[k].reshape(gref[k].shape) + 1e-30
        err = np.abs(got - gref[k])
        say(f"  d{k}: max err {err.max():.2e}, max err/bound {(err / bound).max():.3f}, "
            f"rel {rel(got, gref[k]):.2e}")
        assert np.all(err <= bound), k
    if mask_cols is not None:
        assert np.all(_np(net.g["w1"])[off] == 0.0)


def test_train_gradient_parity(P, SK, orc):
    """BF16 MFMA training pass: a ragged batch (not a multiple of the 64-row
    tile), several tiles per block, gathered rows, restricted inputs, a
    single row, a batch below one tile and a network that reads no input."""
    rng = np.random.default_rng(1)
    for B, gather, cols in ((4133, False, None), (20011, False, None), (3000, True, None),
                            (2500, True, [35, 36]), (1, False, None), (63, True, None),
                            (65, False, [])):
        R = B + 1500 if gather else B
        z = rng.standard_normal((R, 37)).astype(np.float32)
        y = (rng.random(R) < 0.3).astype(np.float32)
        rows = rng.permutation(R)[:B] if gather else None
        say("skip train grad", B, "gathered" if gather else "", cols)
        _check_train(SK, orc, z, y, rows, cols, 2.5, seed=3 + B % 7)


def _logit_bound(z, net):
    """Bound on |BF16-MFMA logit - exact logit|: inputs, weights and the
    first hidden layer rounded to BF16 (unit roundoff 2^-8), FP32 sums."""
    w1, b1, w2, b2, w3 = (net[k].astype(np.float64) for k in ("w1", "b1", "w2", "b2", "w3"))
    az = np.abs(z)
    h1 = np.maximum(z @ w1 + b1, 0)
    g = 70 * U32
    e1 = (2 * UBF + g) * (az @ np.abs(w1)) + g * np.abs(b1)
    e1 = e1 + UBF * (np.abs(h1) + e1)
    h2 = np.maximum(h1 @ w2 + b2, 0)
    e2 = (UBF + g) * ((np.abs(h1) + e1) @ np.abs(w2)) + e1 @ np.abs(w2) + g * np.abs(b2)
    e3 = (UBF + g) * ((np.abs(h2) + e2) @ np.abs(w3)) + e2 @ np.abs(w3)
    return e3[:, 0]


def test_predict_parity_and_order(P, SK, orc):
    sc = S.make_config1()
    cam = S.config1_camera()
    idx = np.arange(0, sc.n, 2, dtype=np.int64)
    net = SK.SkipNet(seed=5)
    with torch.no_grad():
        net.w["b3"].fill_(0.1)
    say("skip predict", len(idx))
    ds, vb = _listed(P, sc, cam, idx)
    sb = SK.SkipBuffers(vb)
    thr = 0.05
    SK.predict(vb, sb, ds, P.make_camera(cam), net, thr, keep_logits=True)
    torch.cuda.synchronize()
    got = _np(sb.logits[:len(idx)]).astype(np.float64)
    z = orc.skip_features(sc, idx, cam)
    ref, _, _ = orc.skip_mlp(z, net.numpy())
    bound = _logit_bound(z, net.numpy())
    err = np.abs(got - ref)
    say(f"  logit max err {err.max():.2e}, max err/bound {(err / bound).max():.3f}")
    assert np.all(err <= bound)
    kc = int(sb.keep_count.item())
    keep = _np(sb.keep_idx[:kc]).astype(np.int64)
    # the kept list is the listed anchors whose GPU logit passes, in order
    assert np.array_equal(keep, idx[got >= thr])
    # and agrees with the exact logits wherever they are farther than the bound
    sure = np.abs(ref - thr) > bound
    assert np.array_equal(np.isin(idx[sure], keep), (ref >= thr)[sure])
    assert 0 < kc < len(idx)


def test_anchor_weights_parity(P, SK, orc):
    sc = S.make_config1()
    cam = S.config1_camera()
    ds = P.DeviceScene.from_scene(sc)
    vb = P.ViewBuffers(sc.n, sc.k, cam.width, cam.height, 1 << 16, log_weights=True)
    say("anchor weights")
    vb.render(ds, P.make_camera(cam), P.raster_params())
    w = torch.empty(sc.n, device="cuda")
    SK.anchor_weights(vb, w)
    torch.cuda.synchronize()
    ref = orc.render(sc, cam, orc.params_array(), weights=True)
    m = len(ref["idx"])
    wref = ref["weights"].reshape(m, sc.k).sum(1)
    np.testing.assert_allclose(_np(w[:m]), wref, rtol=1e-4, atol=1e-5)


def test_trained_predictor_gains(P, SK):
    """On the 1M-anchor street scene at 640x360: the predictor trained on
    logged blend weights of views of the zoom-out's family skips a larger
    share of selected anchors on held-out zoom-out views, at the same bound
    on the worst view's PSNR against full decode (45 dB), than the same
    network trained on one input alone (the log distance, or the level),
    by at least 3 percentage points; and more than the untrained network."""
    sc = S.make_config2()
    ds = P.DeviceScene.from_scene(sc)
    W, H = 640, 360
    train_cams = [P.make_camera(c) for c in S.trajectory_family_views(200, 4, 10.0, 800.0, W, H)]
    eval_cams = [P.make_camera(c) for c in S.zoomout_trajectory(12, 10.0, 800.0, W, H)]
    prm = P.raster_params()
    vb = P.ViewBuffers(sc.n, sc.k, W, H, 8 << 20, gauss_capacity=1 << 20, log_weights=True)
    sb = SK.SkipBuffers(vb)
    say("skip gain: collect")
    z, y = SK.collect(vb, ds, train_cams, prm, tau=1e-2, rows_per_view=20000)
    vb.check_status("skip training views")
    say(f"  rows {z.shape[0]}, positive fraction {y.mean().item():.3f}")

    def skip_at(netx):
        cands = [-4.0, -3.0, -2.0, -1.0, -0.5, 0.0, 0.5, 1.0, 2.0]
        best = SK.choose_threshold(vb, sb, ds, eval_cams, prm, netx, cands, 45.0)
        if best is None:
            return 0.0, None
        thr = best[0]
        sel = kept = 0
        for c in eval_cams:
            vb.select(ds, c, prm)
            SK.predict(vb, sb, ds, c, netx, thr)
            sel += int(vb.sel_count.item())
            kept += int(sb.keep_count.item())
        return 1.0 - kept / max(sel, 1), best

    res = {}
    for name, inputs in (("learned", None), ("distance only", [SK.Z_LOG_DISTANCE]),
                         ("level only", [SK.Z_LEVEL])):
        net = SK.SkipNet(seed=1, inputs=inputs)
        hist = SK.train(net, z, y, epochs=6, batch=8192, lr=2e-3, pos_weight=4.0)
        assert hist[-1] < hist[0], name
        res[name] = skip_at(net)
        say(f"  {name}: loss {[round(h, 4) for h in hist]}, skipped at >=45 dB {res[name]}")
    res["untrained"] = skip_at(SK.SkipNet(seed=1))
    say(f"  untrained: {res['untrained']}")
    best_single = max(res["distance only"][0], res["level only"][0])
    assert res["learned"][0] >= best_single + 0.03, res
    assert res["learned"][0] > res["untrained"][0], res
