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


def test_train_gradient_parity(P, SK, orc):
    rng = np.random.default_rng(1)
    B = 4096
    z = rng.standard_normal((B, 37)).astype(np.float32)
    y = (rng.random(B) < 0.3).astype(np.float32)
    net = SK.SkipNet(seed=3)
    say("skip train grad", B)
    loss = torch.zeros(1, device="cuda")
    net.train_grad(torch.as_tensor(z).cuda(), torch.as_tensor(y).cuda(), 2.5, loss)
    torch.cuda.synchronize()
    _, lref, gref = orc.skip_mlp(z.astype(np.float64), net.numpy(), y, pos_weight=2.5, grads=True)
    assert abs(loss.item() - lref) <= 1e-5 * abs(lref)
    for k in SK.SKIP_ORDER:
        e = rel(_np(net.g[k]), gref[k])
        say(f"  d{k}: rel err {e:.2e}")
        assert e <= 1e-4, k


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
