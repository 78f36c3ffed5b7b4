"""The multi-view training gradient with views in flight on separate streams
(MultiViewBackward) equals the one-view-at-a-time gradient: the decode
backward and the densification statistics are chained in view order, and
every other step of a view uses its own buffers.

On 128x128 views (64 tiles) no Gaussian is listed in enough tiles for the
per-Gaussian reduction to add three or more partials by atomics, so the
gradient is deterministic and the comparison is bit for bit: scene gradients
and densification statistics, for the mean-L1 loss and for the full loss
(L1 + SSIM + volume); the per-view losses agree to rounding (the L1 kernel
adds its block partials by float atomics).  Five views with three in flight also
reuse a buffer set within the step."""

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


def _views():
    d = np.array([1.0, -2.0, 1.5]) / np.linalg.norm([1.0, -2.0, 1.5])
    cams = [S.config1_camera()]
    for dist in (18.0, 9.0, 4.0):
        cams.append(S.look_at(dist * d, (0, 0, 0), 128, 128, 60.0))
    cams.append(S.look_at((6.0, 5.0, 3.0), (0.0, 0.0, 0.0), 128, 128, 60.0))
    return cams


@pytest.mark.parametrize("full", [False, True])
def test_views_in_flight_match_one_at_a_time(P, full):
    sc = S.make_config1()
    ds = P.DeviceScene.from_scene(sc)
    dt = P.DeviceScene.from_scene(S.perturbed_copy(sc, 0.05, seed=3))
    cams = [P.make_camera(c) for c in _views()]
    prm = P.raster_params(train=True)
    vb = P.ViewBuffers(sc.n, sc.k, 128, 128, 1 << 18)
    targets = []
    for c in cams:
        vb.render(dt, c, prm)
        targets.append(vb.rgb.clone())
    del vb
    scale = 1.0 / (len(cams) * 3 * 128 * 128)
    out = {}
    for inflight in (1, 3):
        mv = P.MultiViewBackward(ds, 128, 128, len(cams), 1 << 18, inflight=inflight)
        grads = P.SceneGrads(ds)
        dstats = P.DensifyStats(sc.n, sc.k) if full else None
        losses = mv.run(ds, cams, targets, prm, grads, l1_scale=scale, full=full, dstats=dstats)
        torch.cuda.synchronize()
        for v in mv.vbs:
            st = v.stats()
            assert st["sync_error"] == 0 and st["pair_overflow"] == 0
        res = {"loss": losses.cpu().numpy().copy()}
        res.update({k: t.cpu().numpy().copy() for k, t in grads.all().items()})
        if full:
            for name in ("grad_sum", "grad_count", "opacity_sum", "view_count"):
                res["densify_" + name] = getattr(dstats, name).cpu().numpy().copy()
        out[inflight] = res
    say(f"{'full' if full else 'L1'} loss per view: {out[1]['loss']}")
    for name, a in out[1].items():
        b = out[3][name]
        assert a.shape == b.shape, name
        if name == "loss":
            # the L1 kernel adds its block partials by float atomics
            np.testing.assert_allclose(b, a, rtol=1e-6)
        else:
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), name
    # the comparison is not of zeros
    assert any(np.abs(v.astype(np.float64)).sum() > 0 for k, v in out[1].items()
               if not k.startswith(("loss", "densify")))
    assert out[1]["loss"].sum() > 0
