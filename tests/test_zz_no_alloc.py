"""octgs_select_lod_noalloc (selection with the library's static device
buffer instead of a workspace argument) returns what octgs_select_lod
returns, call after call, including a second, smaller input on the same
buffer; and refuses anchor counts above its stated maximum."""

import ctypes

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


def _random_scene(P, n, seed):
    rng = np.random.default_rng(seed)
    K, k = 7, 4
    pos = rng.uniform(-100, 100, (n, 3)).astype(np.float32)
    level = rng.integers(0, K, n).astype(np.uint8)
    bias = rng.uniform(-0.5, 0.5, n).astype(np.float32)
    offsets = rng.normal(0, 0.5, (n, k, 3)).astype(np.float32)
    osc = np.exp(rng.uniform(-2, 0, (n, 3))).astype(np.float32)
    bsc = np.exp(rng.uniform(-3, -1, (n, 3))).astype(np.float32)
    mlp = S.xavier_mlp(rng, 36, 16, k)
    feat = rng.standard_normal((n, 32)).astype(np.float32)
    return P.DeviceScene(pos, level, bias, feat, offsets, osc, bsc, mlp, 180.0, K, k, 16)


def _both(P, ds, cam, prm=None):
    """(indices, count) from the workspace entry point and from the
    allocation-free one, outputs pre-filled with a sentinel."""
    from paper_2403_17898_amd import _lib as L
    lib = L.lib()
    n = ds.n
    dev = torch.device("cuda", 0)
    prm = P.raster_params() if prm is None else prm
    out = []
    for noalloc in (False, True):
        idx = torch.full((max(1, n),), -1, dtype=torch.int32, device=dev)
        cnt = torch.full((1,), -1, dtype=torch.int32, device=dev)
        if noalloc:
            st = lib.octgs_select_lod_noalloc(ctypes.byref(ds.anchors), ctypes.byref(cam),
                                              ctypes.byref(prm), idx.data_ptr(), cnt.data_ptr(),
                                              None)
        else:
            ws = torch.empty(max(256, lib.octgs_select_workspace_bytes(n)), dtype=torch.uint8,
                             device=dev)
            st = lib.octgs_select_lod(ctypes.byref(ds.anchors), ctypes.byref(cam),
                                      ctypes.byref(prm), idx.data_ptr(), cnt.data_ptr(),
                                      ws.data_ptr(), ws.numel(), None)
        assert st == L.OCTGS_OK, st
        torch.cuda.synchronize()
        m = int(cnt.item())
        out.append((idx[:max(m, 0)].cpu().numpy().copy(), m))
    return out


def test_noalloc_matches_workspace_selection(P):
    big = _random_scene(P, 300_001, 2)
    c1 = S.make_config1()
    small = P.DeviceScene.from_scene(c1)
    cams = S.random_views(2, 7, 80.0, 5.0, 120.0, 640, 480)
    # large input first, then a smaller one on the same static buffer
    cases = [("random 300001", big, P.make_camera(cams[0])),
             ("config 1 (1999 anchors)", small, P.make_camera(S.config1_camera())),
             ("random 300001, second view", big, P.make_camera(cams[1])),
             ("config 1, blended", small, P.make_camera(S.config1_camera(), lod_blend=True))]
    for name, ds, cam in cases:
        say("noalloc select", name)
        (ref_idx, ref_m), (got_idx, got_m) = _both(P, ds, cam)
        assert ref_m > 0
        assert got_m == ref_m, (name, got_m, ref_m)
        assert np.array_equal(got_idx, ref_idx), name


def test_noalloc_empty_and_limit(P):
    from paper_2403_17898_amd import _lib as L
    lib = L.lib()
    ds = P.DeviceScene.from_scene(S.make_config1())
    cam = P.make_camera(S.config1_camera())
    dev = torch.device("cuda", 0)
    idx = torch.zeros(4, dtype=torch.int32, device=dev)
    cnt = torch.full((1,), 7, dtype=torch.int32, device=dev)
    prm = P.raster_params()
    a = L.Anchors.from_buffer_copy(ds.anchors)
    a.n = 0
    say("noalloc select: empty input")
    assert lib.octgs_select_lod_noalloc(ctypes.byref(a), ctypes.byref(cam), ctypes.byref(prm),
                                        idx.data_ptr(), cnt.data_ptr(), None) == L.OCTGS_OK
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0
    # above the stated maximum: refused before any device work
    a.n = L.OCTGS_SELECT_NOALLOC_MAX_ANCHORS + 1
    say("noalloc select: above the maximum")
    assert lib.octgs_select_lod_noalloc(ctypes.byref(a), ctypes.byref(cam), ctypes.byref(prm),
                                        idx.data_ptr(), cnt.data_ptr(), None) == L.OCTGS_ENOSPC
