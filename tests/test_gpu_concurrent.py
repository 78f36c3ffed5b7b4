"""Frames in flight on several streams at once, as the benchmark renders
them: every view's image, transmittance and consumed-entry counts are the
same bit for bit as when the view is rendered alone, and no look-back wait
(candidate scan, emission, sort passes) reports an error.  The forward has
no float atomics outside the optional weight log, so concurrency may change
timing only.  Look-back partitions are taken by ticket in the order blocks
start, so a block never waits on a block that other kernels keep from
being dispatched."""

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


@pytest.fixture(scope="module")
def c2_scene(P):
    say("generating the 1M-anchor street scene")
    sc = S.make_config2()
    return sc, P.DeviceScene.from_scene(sc)


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("depth", [4, 6])
def test_frames_in_flight_match_sequential(P, c2_scene, depth):
    sc, ds = c2_scene
    cams = [P.make_camera(c) for c in S.config2_cameras(200)[::25]]  # 8 views of the zoom-out
    prm = P.raster_params()
    W, H = 1920, 1080
    mk = lambda: P.ViewBuffers(sc.n, sc.k, W, H, pair_capacity=6 << 20, gauss_capacity=700_000)
    # each view alone
    ref = []
    vb = mk()
    for c in cams:
        vb.render(ds, c, prm, precision=P.OCTGS_BF16)
        torch.cuda.synchronize()
        st = vb.stats()
        assert st["sync_error"] == 0 and st["pair_overflow"] == 0
        ref.append((_np(vb.rgb).copy(), _np(vb.T).copy(), _np(vb.last).copy(), st["n_pairs"]))
    del vb
    # the same views, `depth` at a time on separate streams, three rounds
    bufs = [mk() for _ in range(depth)]
    streams = [torch.cuda.Stream() for _ in range(depth)]
    say(f"{len(cams)} views, {depth} in flight")
    for rnd in range(3):
        order = list(range(len(cams)))
        for i0 in range(0, len(order), depth):
            group = order[i0:i0 + depth]
            for k, v in enumerate(group):
                bufs[k].render(ds, cams[v], prm, precision=P.OCTGS_BF16, stream=streams[k])
            torch.cuda.synchronize()
            for k, v in enumerate(group):
                st = bufs[k].stats()
                assert st["sync_error"] == 0 and st["pair_overflow"] == 0, (rnd, v)
                assert st["n_pairs"] == ref[v][3], (rnd, v)
                assert np.array_equal(_np(bufs[k].rgb).view(np.uint32), ref[v][0].view(np.uint32))
                assert np.array_equal(_np(bufs[k].T).view(np.uint32), ref[v][1].view(np.uint32))
                assert np.array_equal(_np(bufs[k].last), ref[v][2])
