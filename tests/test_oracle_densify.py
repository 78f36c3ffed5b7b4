"""Pins of the densification oracle: the level thresholds against their
closed form, the growth / promotion / LOD-bias / pruning rules of Sec. IV-B
on hand-built statistics at and around each threshold, and the statistics
accumulation against a plain loop."""

import numpy as np
import pytest

F32 = np.float32


@pytest.fixture(scope="module")
def DO():
    from oracle import densify as D
    return D


def test_level_thresholds(DO):
    thr = DO.level_thresholds(2e-4, 0.2, 8)
    assert len(thr) == 9 and thr.dtype == F32
    assert thr[0] == F32(2e-4)
    assert thr[5] == F32(4e-4)          # 2^(0.2 * 5) = 2
    assert np.all(np.diff(thr) > 0)     # growing to finer levels gets harder
    np.testing.assert_allclose(thr, 2e-4 * 2.0 ** (0.2 * np.arange(9)), rtol=2e-7)


def _one(DO, level, grads, counts=None, K=4, bias=0.0, vc=5, opsum=None, n_views=10, **kw):
    k = len(grads)
    counts = np.ones(k, np.int64) if counts is None else np.asarray(counts)
    gs = (np.asarray(grads, F32) * counts.astype(F32)).astype(F32)
    opsum = F32(0.5 * k * vc) if opsum is None else opsum
    return DO.decide([level], [bias], gs, counts, [opsum], [vc], k, K, n_views, **kw)


def test_growth_and_next_level_promotion(DO):
    thr = DO.level_thresholds(2e-4, 0.2, 4)
    up = lambda v: np.nextafter(F32(v), F32(1))
    dn = lambda v: np.nextafter(F32(v), F32(0))
    g, _, _ = _one(DO, 2, [dn(thr[2]), thr[2], up(thr[2]), thr[3], up(thr[3]), 1.0], K=4)
    # at or below tau_2: no growth; above: level 2; above tau_3: level 3
    assert list(g) == [-1, -1, 2, 2, 3, 3]
    # the finest level has no next level: it grows in place
    g, _, _ = _one(DO, 3, [up(thr[3]), 1.0], K=4)
    assert list(g) == [3, 3]
    # never visible: no statistics, no growth
    g, _, _ = _one(DO, 0, [1.0, 1.0], counts=[0, 3], K=4)
    assert list(g) == [-1, 0 + 1]


def test_lod_bias_update(DO):
    thr = DO.level_thresholds(2e-4, 0.2, 4)
    q = F32(thr[1] * F32(0.25))
    _, b, _ = _one(DO, 1, [q, q], K=4, bias=0.125)
    assert b[0] == F32(0.125)                        # not strictly above tau_L / 4
    _, b, _ = _one(DO, 1, [q, np.nextafter(q, F32(1)) * 3], K=4, bias=0.125)
    assert b[0] == F32(F32(0.125) + F32(0.01))       # Delta L += epsilon
    # invisible Gaussians do not dilute the anchor's mean gradient
    _, b, _ = _one(DO, 1, [2 * q, 0.0], counts=[1, 0], K=4)
    assert b[0] == F32(0.01)


def test_pruning_rules(DO):
    # never selected: view frequency 0 < tau_v
    _, _, p = _one(DO, 0, [0.0], vc=0, opsum=F32(0), n_views=10, tau_v=0.01)
    assert p[0] == 1
    # selected often enough and opaque enough: kept
    _, _, p = _one(DO, 0, [0.0, 0.0], vc=5, opsum=F32(0.02 * 2 * 5), n_views=10,
                   tau_v=0.5, tau_opacity=0.005)
    assert p[0] == 0
    # view frequency 4 / 10 below 0.5
    _, _, p = _one(DO, 0, [0.0], vc=4, n_views=10, tau_v=0.5)
    assert p[0] == 1
    # average opacity 0.004 < 0.005
    _, _, p = _one(DO, 0, [0.0, 0.0], vc=5, opsum=F32(0.004 * 2 * 5), n_views=10, tau_v=0.0,
                   tau_opacity=0.005)
    assert p[0] == 1


def test_accumulate_matches_loop(DO):
    rng = np.random.default_rng(0)
    n, k, W, H = 30, 4, 64, 48
    st = DO.new_stats(n, k)
    ref_sum = np.zeros(n * k)
    ref_cnt = np.zeros(n * k, np.int64)
    ref_vc = np.zeros(n, np.int64)
    ref_op = np.zeros(n)
    for view in range(5):
        anchors = np.sort(rng.choice(n, 12, replace=False))
        gidx = (anchors[:, None] * k + np.arange(k)).reshape(-1)
        vis = rng.random(len(gidx)) < 0.7
        dm = rng.standard_normal((len(gidx), 2))
        op = rng.uniform(-1, 1, len(gidx))
        DO.accumulate(st, gidx, vis, dm, W, H, anchors, op, k)
        for s, g in enumerate(gidx):
            if vis[s]:
                ref_sum[g] += ((dm[s, 0] * W / 2) ** 2 + (dm[s, 1] * H / 2) ** 2) ** 0.5
                ref_cnt[g] += 1
        for p, a in enumerate(anchors):
            ref_vc[a] += 1
            ref_op[a] += sum(max(op[p * k + i], 0.0) for i in range(k))
    np.testing.assert_allclose(st["grad_sum"], ref_sum, rtol=1e-14)
    assert np.array_equal(st["grad_count"], ref_cnt)
    assert np.array_equal(st["view_count"], ref_vc)
    np.testing.assert_allclose(st["opacity_sum"], ref_op, rtol=1e-14)
    # closed form: gradient (3, 4) in NDC units in each of three views -> mean 5
    st = DO.new_stats(1, 1)
    for _ in range(3):
        DO.accumulate(st, np.array([0]), np.array([True]), [[3 * 2 / W, 4 * 2 / H]], W, H,
                      np.array([0]), [0.5], 1)
    assert abs(st["grad_sum"][0] / st["grad_count"][0] - 5.0) < 1e-12
