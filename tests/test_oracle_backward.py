"""Finite-difference pins of the oracle's analytic backward passes.

Each stage is checked on its own against central differences of the
oracle's double-precision forward, with the discrete decisions (culls,
rectangles, order, termination) held fixed; coordinates whose perturbation
changes a decision are skipped and counted.  The full chain is checked on the
50-anchor 64x64 scene.  Parameters stored in float32 are perturbed by steps
exactly representable in float32 (the realised step is used in the
quotient).
"""

import numpy as np
import pytest

from synth import scenes as S


def rel_err(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _decisions(pj, out=None):
    """Culls, rectangles, the sorted pair order and where each pixel stopped."""
    key = (pj["vis"].tobytes(), pj["rect"].tobytes())
    if out is not None:
        key = key + (out["bs"]["gid_of"].tobytes(), out["bs"]["tile_of"].tobytes(), out["last"].tobytes())
    return key


def test_composite_backward_fd(orc):
    cam = S.look_at((3.0, -20.0, 4.0), (0.0, 0.0, 0.0), 40, 33, 60.0)
    gf = S.random_gaussians(120, cam, 3, scale=(0.1, 0.8))
    prm = orc.params_array()
    pj = orc.project(gf, cam, prm)
    bs = orc.bin_sort(pj, cam)
    rng = np.random.default_rng(0)
    dimg = rng.standard_normal((3, cam.height, cam.width))
    base = orc.composite(pj, bs, cam, prm)
    ana = orc.composite_backward(pj, bs, cam, prm, dimg)
    vis = np.flatnonzero(pj["vis"])
    h = 1e-6
    fd = np.zeros_like(ana)
    skipped = 0
    for g in vis:
        for q in range(9):
            vals = []
            for sgn in (1, -1):
                pj2 = dict(pj)
                pj2["proj"] = pj["proj"].copy()
                pj2["proj"][g, q] += sgn * h
                o = orc.composite(pj2, bs, cam, prm)
                if not np.array_equal(o["last"], base["last"]):
                    vals = None
                    break
                vals.append(float((dimg * o["img"]).sum()))
            if vals is None:
                skipped += 1
                fd[g, q] = ana[g, q]
                continue
            fd[g, q] = (vals[0] - vals[1]) / (2 * h)
    assert skipped < 0.01 * len(vis) * 9
    for q in range(9):
        assert rel_err(ana[vis, q], fd[vis, q]) < 1e-5, q


def test_project_backward_fd(orc):
    cam = S.look_at((3.0, -20.0, 4.0), (0.0, 0.0, 0.0), 96, 80, 60.0)
    gf = S.random_gaussians(200, cam, 4, scale=(0.05, 0.6), margin=0.4)
    gd = gf.astype(np.float64)
    prm = orc.params_array()
    pj = orc.project(gf, cam, prm, gd)
    rng = np.random.default_rng(1)
    v = rng.standard_normal((len(pj["vis"]), 9))
    ana = orc.project_backward(gd, pj, cam, prm, v)
    vis = np.flatnonzero(pj["vis"])
    h = 1e-6
    fd = np.zeros_like(ana)
    for f in range(14):
        for g in vis:
            vals = []
            for sgn in (1, -1):
                gd2 = gd.copy()
                gd2[f, g] += sgn * h
                p2 = orc.project(gf, cam, prm, gd2)
                vals.append(float((v[g] * p2["proj"][g]).sum()))
            fd[f, g] = (vals[0] - vals[1]) / (2 * h)
    for f in range(14):
        assert rel_err(ana[f, vis], fd[f, vis]) < 1e-5, f


def _perturb(arr, flat_i, rel):
    """Float32 array copies with element flat_i moved by an exactly
    representable step of about rel * max(1, |x|); returns (plus, minus, step)."""
    x = float(arr.flat[flat_i])
    h = np.float32(rel * max(1.0, abs(x)))
    p, m = arr.copy(), arr.copy()
    p.flat[flat_i] = np.float32(x + h)
    m.flat[flat_i] = np.float32(x - h)
    return p, m, float(p.flat[flat_i]) - float(m.flat[flat_i])


def test_decode_backward_fd(orc):
    sc, cam = S.make_gradcheck_scene()
    idx = np.arange(0, sc.n, 2, dtype=np.int64)
    rng = np.random.default_rng(2)
    gd0 = orc.decode(sc, idx, cam)
    v = rng.standard_normal(gd0.shape)
    ana = orc.decode_backward(sc, idx, cam, v)

    def loss(s2):
        return float((v * orc.decode(s2, idx, cam)).sum())

    checks = [("pos", sc.pos), ("feat", sc.feat), ("offsets", sc.offsets),
              ("offset_scale", sc.offset_scale), ("base_scale", sc.base_scale)]
    for name in ("w1_a", "b1_a", "w2_a", "b2_a", "w1_c", "w2_c", "w1_s", "b1_s", "w2_s", "b2_s"):
        checks.append((name, sc.mlp[name]))
    for name, arr in checks:
        n_el = arr.size
        pick = rng.choice(n_el, min(n_el, 40), replace=False)
        a_vals, f_vals = [], []
        for fi in pick:
            p, m, step = _perturb(arr, fi, 2.0 ** -12)
            s_p = _with(sc, name, p)
            s_m = _with(sc, name, m)
            f_vals.append((loss(s_p) - loss(s_m)) / step)
            a_vals.append(ana[name].flat[fi])
        assert rel_err(a_vals, f_vals) < 1e-5, name


def _with(sc, name, arr):
    import copy
    s2 = copy.copy(sc)
    if name in sc.mlp:
        s2.mlp = dict(sc.mlp)
        s2.mlp[name] = arr
    else:
        setattr(s2, name, arr)
    return s2


def test_full_chain_gradcheck_fd(orc):
    """50-anchor scene at 64x64: gradient of sum(w * image) through
    compositing, projection and decode, against central differences of the
    FP64 forward; gradient bar: normwise relative error <= 1e-3."""
    sc, cam = S.make_gradcheck_scene()
    prm = orc.params_array()
    thr, rho = orc.scene_thresholds(sc)
    fwd = orc.render(sc, cam, prm, thr, rho)
    assert len(fwd["idx"]) == sc.n and fwd["pj"]["n_visible"] > 100
    rng = np.random.default_rng(5)
    dimg = rng.standard_normal((3, cam.height, cam.width))
    ana = orc.render_backward(sc, cam, prm, dimg, fwd)
    key0 = _decisions(fwd["pj"], fwd)

    def loss(s2):
        o = orc.render(s2, cam, prm, thr, rho)
        return float((dimg * o["img"]).sum()), _decisions(o["pj"], o)

    report = {}
    skipped = total = 0
    checks = [("pos", sc.pos), ("feat", sc.feat), ("offsets", sc.offsets),
              ("offset_scale", sc.offset_scale), ("base_scale", sc.base_scale)]
    for name in ("w1_a", "w2_a", "b2_a", "w1_c", "w2_c", "w1_s", "w2_s", "b1_s"):
        checks.append((name, sc.mlp[name]))
    for name, arr in checks:
        pick = rng.choice(arr.size, min(arr.size, 25), replace=False)
        a_vals, f_vals = [], []
        for fi in pick:
            total += 1
            p, m, step = _perturb(arr, fi, 2.0 ** -14)
            lp, kp = loss(_with(sc, name, p))
            lm, km = loss(_with(sc, name, m))
            if kp != key0 or km != key0:
                skipped += 1
                continue
            f_vals.append((lp - lm) / step)
            a_vals.append(ana[name].flat[fi])
        report[name] = rel_err(a_vals, f_vals)
    assert skipped <= 0.05 * total, (skipped, total)
    for name, e in report.items():
        assert e <= 1e-3, (name, e, report)
