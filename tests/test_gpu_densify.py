"""Parity of the densification statistics and decisions with the oracle,
through the C ABI.

Bars: decisions (growth level, pruning, the updated LOD bias, the counts)
bit-exact on the same FP32 statistics; accumulated counts bit-exact;
accumulated gradient norms within the gradient bar (1e-3 normwise and of
the largest entry); opacity sums within 1e-5 relative (FP32 sums of at most
k x views terms in [0, 1])."""

import numpy as np
import pytest

from synth import scenes as S
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

F32 = np.float32


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_17898_amd as P
    P.lib()
    return P


@pytest.fixture(scope="module")
def DO():
    from oracle import densify as D
    return D


class _Anchors:
    """The fields octgs_densify_decide reads, resident on the device."""

    def __init__(self, P, level, lod_bias, k, n_levels):
        from paper_2403_17898_amd import _lib as L
        self.level = torch.as_tensor(level).cuda()
        self.lod_bias = torch.as_tensor(lod_bias).cuda()
        a = L.Anchors()
        a.n, a.k, a.n_levels = len(level), k, n_levels
        a.level = self.level.data_ptr()
        a.lod_bias = self.lod_bias.data_ptr()
        self.anchors = a


def test_decide_bit_exact(P, DO):
    rng = np.random.default_rng(0)
    n, k, K, views = 100_003, 10, 8, 37
    level = rng.integers(0, K, n).astype(np.uint8)
    thr = DO.level_thresholds(2e-4, 0.2, K)
    cnt = rng.integers(0, 6, n * k)
    cnt[rng.random(n * k) < 0.2] = 0
    # mean gradients spread over the thresholds, some exactly on them
    g = np.exp(rng.uniform(np.log(2e-5), np.log(2e-3), n * k)).astype(F32)
    lv = np.repeat(level, k)
    on = rng.random(n * k) < 0.05
    g[on] = thr[np.minimum(lv[on] + rng.integers(0, 2, on.sum()), K)]
    gs = (g * cnt.astype(F32)).astype(F32)
    gs[cnt == 0] = 0
    vc = rng.integers(0, views + 1, n)
    op = (rng.uniform(0, 0.02, n) * k * vc).astype(F32)
    bias = rng.uniform(-0.5, 0.5, n).astype(F32)
    say("densify decide", n)
    A = _Anchors(P, level, bias, k, K)
    st = P.DensifyStats(n, k)
    st.grad_sum.copy_(torch.as_tensor(gs))
    st.grad_count.copy_(torch.as_tensor(cnt.astype(np.int32)))
    st.opacity_sum.copy_(torch.as_tensor(op))
    st.view_count.copy_(torch.as_tensor(vc.astype(np.int32)))
    st.decide(A, views, tau_opacity=0.005, tau_v=0.1)
    torch.cuda.synchronize()
    rg, rb, rp = DO.decide(level, bias, gs, cnt, op, vc, k, K, views, tau_opacity=0.005, tau_v=0.1)
    gg = st.grow_level.cpu().numpy()
    assert np.array_equal(gg, rg)
    assert np.array_equal(st.prune.cpu().numpy(), rp)
    assert np.array_equal(A.lod_bias.cpu().numpy().view(np.uint32), rb.view(np.uint32))
    want = [int((rg >= 0).sum()), int((rg == np.repeat(level, k).astype(np.int8) + 1).sum()),
            int((rb != bias).sum()), int(rp.sum())]
    say("  counts", st.counts.cpu().numpy().tolist(), "want", want)
    assert st.counts.cpu().numpy().tolist() == want
    assert min(want) > 0 and want[0] < n * k


def test_decide_empty(P):
    A = _Anchors(P, np.zeros(0, np.uint8), np.zeros(0, F32), 4, 3)
    st = P.DensifyStats(0, 4)
    st.counts.fill_(9)
    st.decide(A, 5)
    torch.cuda.synchronize()
    assert st.counts.cpu().numpy().tolist() == [0, 0, 0, 0]


def test_accumulate_parity(P, orc, DO):
    sc = S.make_config1()
    ds = P.DeviceScene.from_scene(sc)
    prm = P.raster_params(train=True)
    d = np.array([1.0, -2.0, 1.5]) / np.linalg.norm([1.0, -2.0, 1.5])
    cams = [S.config1_camera(), S.look_at(12.0 * d, (0, 0, 0), 128, 128, 60.0),
            S.look_at((2.0, -3.0, 1.0), (0.0, 0.0, 0.0), 97, 61, 70.0)]
    st = P.DensifyStats(sc.n, sc.k)
    ref = DO.new_stats(sc.n, sc.k)
    thr, rho = orc.scene_thresholds(sc)
    rng = np.random.default_rng(1)
    for i, cam in enumerate(cams):
        say("densify accumulate view", i)
        dimg = rng.standard_normal((3, cam.height, cam.width)).astype(F32)
        vb = P.ViewBuffers(sc.n, sc.k, cam.width, cam.height, 1 << 18)
        c = P.make_camera(cam)
        vb.render(ds, c, prm)
        vb.rasterize_bwd(c, prm, torch.as_tensor(dimg).cuda())
        st.accumulate(vb, c)
        torch.cuda.synchronize()
        fwd = orc.render(sc, cam, orc.params_array(), thr, rho)
        dproj = orc.composite_backward(fwd["pj"], fwd["bs"], cam, orc.params_array(),
                                       dimg.astype(np.float64))
        idx = fwd["idx"]
        gidx = (idx[:, None] * sc.k + np.arange(sc.k)).reshape(-1)
        DO.accumulate(ref, gidx, fwd["pj"]["vis"].astype(bool), dproj[:, :2], cam.width,
                      cam.height, idx, fwd["gauss"][10], sc.k)
    assert np.array_equal(st.grad_count.cpu().numpy(), ref["grad_count"])
    assert np.array_equal(st.view_count.cpu().numpy(), ref["view_count"])
    gs = st.grad_sum.cpu().numpy().astype(np.float64)
    e = np.linalg.norm(gs - ref["grad_sum"]) / np.linalg.norm(ref["grad_sum"])
    say(f"  grad_sum rel err {e:.2e}; {int((ref['grad_count'] > 0).sum())} Gaussians seen")
    assert e <= 1e-3
    assert np.abs(gs - ref["grad_sum"]).max() <= 1e-3 * np.abs(ref["grad_sum"]).max()
    np.testing.assert_allclose(st.opacity_sum.cpu().numpy(), ref["opacity_sum"], rtol=1e-5,
                               atol=1e-7)
