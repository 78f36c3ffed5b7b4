"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these tests touches the HIP library.  Each one checks the oracle
against something other than its own code: closed-form images, brute force,
invariants of Eq. 2 and Eq. 7, and hand-evaluable special cases of the decode
MLPs.  The paper prints no worked numeric example, so closed forms stand in
for one.
"""

import math

import numpy as np
import pytest

from synth import scenes as S

F32 = np.float32


def ident_cam(W=64, H=64, f=80.0, C=(0.0, 0.0, 0.0)):
    return S.Camera(R=np.eye(3), C=np.asarray(C, np.float64), fx=f, fy=f, cx=W / 2, cy=H / 2,
                    width=W, height=H)


def gauss(mean, scale, quat=(1, 0, 0, 0), op=0.8, rgb=(0.2, 0.5, 0.9)):
    g = np.array([*mean, *scale, *quat, op, *rgb], np.float32).reshape(14, 1)
    return g


def cat(*gs):
    return np.ascontiguousarray(np.concatenate(gs, axis=1))


def pix_grid(W, H):
    x = np.arange(W) + 0.5
    y = np.arange(H) + 0.5
    return np.meshgrid(x, y)


def tile_mask(W, H, x0, y0, x1, y1, keep=None):
    X, Y = np.meshgrid(np.arange(W) // 16, np.arange(H) // 16)
    m = (X >= x0) & (X < x1) & (Y >= y0) & (Y < y1)
    if keep is not None:
        m &= np.vectorize(keep)(X, Y)
    return m


def ellipse_meets_box(mx, my, A, B, C, X0, X1, Y0, Y1):
    """Does {A dx^2 + 2B dx dy + C dy^2 <= 9} (dx = x - mx) meet the box
    [X0, X1] x [Y0, Y1]?  Root form, in double: the mean is inside, or on
    some edge line the chord cut by the ellipse overlaps the edge."""
    if X0 <= mx <= X1 and Y0 <= my <= Y1:
        return True
    # (P, Q, d, lo, hi): q(t) = P d^2 + 2 B d t + Q t^2 along an edge at
    # offset d from the mean, t in [lo, hi]
    edges = [(A, C, X - mx, Y0 - my, Y1 - my) for X in (X0, X1)]
    edges += [(C, A, Y - my, X0 - mx, X1 - mx) for Y in (Y0, Y1)]
    for P, Q, d, lo, hi in edges:
        D = (B * d) ** 2 - Q * (P * d * d - 9.0)
        if D >= 0:
            r0, r1 = (-B * d - math.sqrt(D)) / Q, (-B * d + math.sqrt(D)) / Q
            if r1 >= lo and r0 <= hi:
                return True
    return False


def box_qmin_sampled(mx, my, A, B, C, X0, X1, Y0, Y1, k=2001):
    """Minimum of the quadratic over the box boundary (and 0 inside), by
    dense sampling: used only to leave out near-ties from exact checks."""
    if X0 <= mx <= X1 and Y0 <= my <= Y1:
        return 0.0
    t = np.linspace(0.0, 1.0, k)
    xs = np.concatenate([X0 + (X1 - X0) * t, X0 + (X1 - X0) * t, np.full(k, X0), np.full(k, X1)])
    ys = np.concatenate([np.full(k, Y0), np.full(k, Y1), Y0 + (Y1 - Y0) * t, Y0 + (Y1 - Y0) * t])
    dx, dy = xs - mx, ys - my
    return float((A * dx * dx + 2 * B * dx * dy + C * dy * dy).min())


def tile_keep(mx, my, A, B, C):
    def keep(tx, ty):
        X0, Y0 = 16.0 * tx + 0.5, 16.0 * ty + 0.5
        return ellipse_meets_box(mx, my, A, B, C, X0, X0 + 15, Y0, Y0 + 15)
    return keep


# --------------------------------------------------------------------------
# Eq. 1 / EWA projection / Eq. 2 closed forms
# --------------------------------------------------------------------------

def closed_form_axis_cov(cam, m, s, dil):
    """2D covariance of an axis-aligned Gaussian seen by an identity-rotation
    camera: J diag(s^2) J^T + dil I with J the perspective Jacobian at m."""
    f = float(cam.fx)
    x, y, z = (float(v) for v in m)
    sx, sy, sz = (float(v) ** 2 for v in s)
    a = f * f * sx / z ** 2 + f * f * x * x * sz / z ** 4 + dil
    b = f * f * x * y * sz / z ** 4
    c = f * f * sy / z ** 2 + f * f * y * y * sz / z ** 4 + dil
    return a, b, c


@pytest.mark.parametrize("mean", [(0.0, 0.0, 10.0), (1.3, -0.7, 9.0), (-2.0, 1.5, 14.0)])
def test_single_gaussian_closed_form(orc, mean):
    cam = ident_cam()
    prm = orc.params_array()
    dil = float(F32(0.3))
    s = np.array([0.35, 0.2, 0.5], np.float32)
    g = gauss(mean, s, op=0.7)
    m32 = g[:3, 0].astype(np.float64)
    out = orc.rasterize(g, cam, prm)
    a, b, c = closed_form_axis_cov(cam, m32, g[3:6, 0].astype(np.float64), dil)
    det = a * c - b * b
    mx = cam.fx * m32[0] / m32[2] + cam.cx
    my = cam.fy * m32[1] / m32[2] + cam.cy
    X, Y = pix_grid(cam.width, cam.height)
    dx, dy = X - mx, Y - my
    G = np.exp(-0.5 * (c * dx * dx - 2 * b * dx * dy + a * dy * dy) / det)
    alpha = np.minimum(0.99, float(g[10, 0]) * G)
    lam = 0.5 * (a + c) + math.sqrt(max(0.25 * (a - c) ** 2 + b * b, 0))
    r = math.ceil(3 * math.sqrt(lam))
    tx0, tx1 = max(0, math.floor((mx - r) / 16)), min(4, math.floor((mx + r) / 16) + 1)
    ty0, ty1 = max(0, math.floor((my - r) / 16)), min(4, math.floor((my + r) / 16) + 1)
    inside = tile_mask(cam.width, cam.height, tx0, ty0, tx1, ty1,
                       tile_keep(mx, my, c / det, -b / det, a / det))
    assert tuple(out["pj"]["rect"][0]) == (tx0, ty0, tx1, ty1)
    for ch in range(3):
        exp_img = np.where(inside, alpha * float(g[11 + ch, 0]), 0.0)
        np.testing.assert_allclose(out["img"][ch], exp_img, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(out["T"], np.where(inside, 1 - alpha, 1.0), rtol=1e-9, atol=1e-12)
    # conic is the inverse of the closed-form 2D covariance
    p = out["pj"]["proj"][0]
    np.testing.assert_allclose(p[2:5], [c / det, -b / det, a / det], rtol=1e-9)


def test_rotation_swaps_axes(orc):
    """A 90-degree turn about the viewing axis swaps the x and y scales; a
    90-degree turn about x swaps y and z (checks R(q) and Sigma = R S S^T R^T)."""
    cam = ident_cam()
    prm = orc.params_array()
    h = math.sqrt(0.5)
    m = (0.4, -0.3, 8.0)
    ref = orc.rasterize(gauss(m, (0.2, 0.45, 0.3)), cam, prm)["img"]
    rot = orc.rasterize(gauss(m, (0.45, 0.2, 0.3), quat=(h, 0, 0, h)), cam, prm)["img"]
    np.testing.assert_allclose(rot, ref, atol=1e-6)
    ref2 = orc.rasterize(gauss(m, (0.3, 0.25, 0.4)), cam, prm)["img"]
    rot2 = orc.rasterize(gauss(m, (0.3, 0.4, 0.25), quat=(h, h, 0, 0)), cam, prm)["img"]
    np.testing.assert_allclose(rot2, ref2, atol=1e-6)


def test_two_gaussians_front_to_back(orc):
    """C = a1 c1 + (1 - a1) a2 c2 + (1 - a1)(1 - a2) bg, nearer first,
    whatever their index order."""
    cam = ident_cam()
    bg = (0.1, 0.2, 0.3)
    prm = orc.params_array(bg=bg)
    far = gauss((0.0, 0.0, 12.0), (0.5, 0.5, 0.5), op=0.6, rgb=(1.0, 0.0, 0.0))
    near = gauss((0.1, 0.0, 6.0), (0.2, 0.2, 0.2), op=0.5, rgb=(0.0, 1.0, 0.5))
    out = orc.rasterize(cat(far, near), cam, prm)
    dil = float(F32(0.3))
    X, Y = pix_grid(cam.width, cam.height)

    def alpha(g):
        m = g[:3, 0].astype(np.float64)
        a, b, c = closed_form_axis_cov(cam, m, g[3:6, 0].astype(np.float64), dil)
        det = a * c - b * b
        dx = X - (cam.fx * m[0] / m[2] + cam.cx)
        dy = Y - (cam.fy * m[1] / m[2] + cam.cy)
        G = np.exp(-0.5 * (c * dx * dx - 2 * b * dx * dy + a * dy * dy) / det)
        return np.minimum(0.99, float(g[10, 0]) * G)

    a1, a2 = alpha(near), alpha(far)
    r1 = out["pj"]["rect"][1]
    r2 = out["pj"]["rect"][0]
    in1 = tile_mask(64, 64, *r1)
    in2 = tile_mask(64, 64, *r2)
    a1 = np.where(in1, a1, 0)
    a2 = np.where(in2, a2, 0)
    for ch in range(3):
        c1, c2 = float(near[11 + ch, 0]), float(far[11 + ch, 0])
        exp_img = a1 * c1 + (1 - a1) * a2 * c2 + (1 - a1) * (1 - a2) * float(F32(bg[ch]))
        np.testing.assert_allclose(out["img"][ch], exp_img, rtol=1e-9, atol=1e-12)


# --------------------------------------------------------------------------
# Compositing invariants and brute force
# --------------------------------------------------------------------------

@pytest.mark.parametrize("W,H,n,seed", [(64, 48, 300, 1), (50, 37, 500, 2), (33, 17, 80, 3)])
def test_bruteforce_equals_tiled(orc, W, H, n, seed):
    cam = S.look_at((3.0, -20.0, 4.0), (0.0, 0.0, 0.0), W, H, 60.0)
    g = S.random_gaussians(n, cam, seed, neg_opacity_frac=0.1, behind_frac=0.05)
    prm = orc.params_array()
    out = orc.rasterize(g, cam, prm)
    bf = orc.render_bruteforce(out["pj"], cam, prm)
    assert out["bs"]["n_pairs"] > n // 4
    assert np.array_equal(bf["img"], out["img"])
    assert np.array_equal(bf["T"], out["T"])


def test_partition_of_unity_and_weights(orc):
    cam = S.look_at((3.0, -20.0, 4.0), (0.0, 0.0, 0.0), 64, 64, 60.0)
    g = S.random_gaussians(800, cam, 5)
    g[11:14] = 1.0
    prm = orc.params_array()
    out = orc.rasterize(g, cam, prm, weights=True)
    T = out["T"]
    assert np.all(T > 0) and np.all(T <= 1)
    for ch in range(3):
        np.testing.assert_allclose(out["img"][ch] + T, 1.0, atol=1e-12)
    np.testing.assert_allclose(out["weights"].sum(), (1 - T).sum(), rtol=1e-10)
    # a pixel that stops before the end of its tile list went below t_min
    rng = out["bs"]["ranges"]
    tiles_x = 4
    for y in range(64):
        for x in range(64):
            t = (y // 16) * tiles_x + x // 16
            n_list = int(rng[t, 1] - rng[t, 0])
            if out["last"][y, x] < n_list:
                assert T[y, x] < 1e-4


def test_skip_error_certificate(orc):
    _check_skip_certificate(orc)


def test_skip_certificate_catches_a_planted_mistake(orc):
    """Logging a_i T_(i+1) (the transmittance after the Gaussian) instead of
    a_i T_i, in a copy of the oracle, breaks the certificate."""
    import tempfile
    src = orc.source()
    good = "      w[list[i]] += wt;"
    assert src.count(good) == 1
    with tempfile.TemporaryDirectory() as d:
        with orc.variant(src.replace(good, "      w[list[i]] += wt * (1.0 - a);"), d,
                         tag="weight_after"):
            with pytest.raises(AssertionError):
                _check_skip_certificate(orc)


def _check_skip_certificate(orc):
    """The logged blend weight bounds what leaving an anchor out can change:
    with colours and background in [0, 1] and no early stop (t_min = 0),
    removing anchor j's Gaussians changes each channel by at most
    sum_{i in j} a_i T_i at every pixel, so summed over the image by at
    most the anchor's logged weight w_j.  Groups of k = 10 consecutive
    Gaussians stand for anchors."""
    cam = S.look_at((3.0, -20.0, 4.0), (0.0, 0.0, 0.0), 64, 64, 60.0)
    g = S.random_gaussians(800, cam, 9)
    rng = np.random.default_rng(9)
    g[11:14] = rng.uniform(0.0, 1.0, (3, g.shape[1])).astype(np.float32)
    prm = orc.params_array(t_min=0.0, bg=(0.3, 0.6, 0.9))
    base = orc.rasterize(g, cam, prm, weights=True)
    k = 10
    w = base["weights"].reshape(-1, k).sum(axis=1)
    order = np.argsort(-w)
    tight = []
    for j in list(order[:10]) + list(order[40:50]):
        g2 = g.copy()
        g2[10, j * k:(j + 1) * k] = 0.0  # opacity 0: culled
        out = orc.rasterize(g2, cam, prm)
        d = np.abs(out["img"] - base["img"]).sum(axis=(1, 2))
        assert np.all(d <= w[j] * (1 + 1e-12) + 1e-12), (j, d, w[j])
        tight.append(d.max() / max(w[j], 1e-300))
    # the bound is not vacuous: for the heaviest anchors it is within a few times
    assert max(tight[:10]) > 0.2, tight
    # and it is exact where nothing overlaps: 16 small white Gaussians on a
    # grid, black background, so removing one changes the image by exactly
    # its logged weight (T_i = 1 at each of its pixels)
    cam = S.look_at((0.0, -20.0, 0.0), (0.0, 0.0, 0.0), 128, 128, 60.0)
    xs = (-6.0, -2.0, 2.0, 6.0)
    n = 16
    g = np.zeros((14, n), np.float32)
    g[0] = np.repeat(xs, 4)
    g[2] = np.tile(xs, 4)
    g[3:6] = 0.05
    g[6] = 1.0  # identity rotation (w, x, y, z)
    g[10] = 0.7
    g[11:14] = 1.0
    prm = orc.params_array(t_min=0.0)
    base = orc.rasterize(g, cam, prm, weights=True)
    assert base["bs"]["n_pairs"] >= n
    for j in range(n):
        g2 = g.copy()
        g2[10, j] = 0.0
        out = orc.rasterize(g2, cam, prm)
        d = (base["img"] - out["img"]).sum(axis=(1, 2))
        np.testing.assert_allclose(d, base["weights"][j], rtol=1e-9)


def test_transmittance_monotone(orc):
    """T after each prefix of a pixel's list is non-increasing: rendering the
    first j Gaussians (front-most) of the depth order gives T_j >= T_{j+1}."""
    cam = ident_cam(32, 32, 40.0)
    rng = np.random.default_rng(4)
    gs = []
    for i in range(12):
        gs.append(gauss((rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5), 4.0 + i),
                        rng.uniform(0.3, 1.0, 3), op=rng.uniform(0.1, 0.9)))
    prm = orc.params_array(t_min=0.0)
    prev = np.ones((32, 32))
    for j in range(1, 13):
        T = orc.rasterize(cat(*gs[:j]), cam, prm)["T"]
        assert np.all(T <= prev + 1e-15) and np.all(T >= 0)
        prev = T


def test_bin_sort_against_enumeration(orc):
    cam = S.look_at((3.0, -20.0, 4.0), (0.0, 0.0, 0.0), 80, 70, 60.0)
    g = S.random_gaussians(400, cam, 9)
    prm = orc.params_array()
    pj = orc.project(g, cam, prm)
    bs = orc.bin_sort(pj, cam)
    tx = (80 + 15) // 16
    rows = []
    for i in np.flatnonzero(pj["vis"]):
        x0, y0, x1, y1 = pj["rect"][i]
        for y in range(y0, y1):
            for x in range(x0, x1):
                if orc.tile_test(pj["cf"][i], x, y, 80, 70):
                    rows.append((y * tx + x, pj["depth"][i].view(np.uint32), i))
    rows = np.array(rows, dtype=np.int64)
    order = np.lexsort((rows[:, 2], rows[:, 1], rows[:, 0]))
    rows = rows[order]
    assert bs["n_pairs"] == len(rows)
    assert np.array_equal(bs["tile_of"], rows[:, 0])
    assert np.array_equal(bs["gid_of"], rows[:, 2])
    for t in range(bs["ranges"].shape[0]):
        s, e = bs["ranges"][t]
        assert np.all(rows[s:e, 0] == t)
        assert np.count_nonzero(rows[:, 0] == t) == e - s


def test_tile_test_against_root_form(orc):
    """The FP32 tile test keeps exactly the tiles whose pixel-centre box the
    3-sigma ellipse meets (root form in double), away from near-ties; the
    kept tiles are a subset of the rectangle and include every tile holding
    a pixel centre inside the ellipse."""
    rng = np.random.default_rng(7)
    n_chk = n_tie = 0
    W, H = 117, 121  # the last tile column and row hold 5 and 9 pixel centres
    for _ in range(400):
        mx, my = rng.uniform(-20, 100, 2)
        sx, sy = np.exp(rng.uniform(np.log(0.7), np.log(25), 2))
        th = rng.uniform(0, np.pi)
        c, s_ = math.cos(th), math.sin(th)
        Rm = np.array([[c, -s_], [s_, c]])
        cov = Rm @ np.diag([sx * sx, sy * sy]) @ Rm.T
        con = np.linalg.inv(cov)
        cf = np.array([mx, my, con[0, 0], con[0, 1], con[1, 1]], np.float32)
        A, B, C = (float(v) for v in cf[2:])
        fx, fy = float(cf[0]), float(cf[1])
        for tx in range(-1, 8):
            for ty in range(-1, 8):
                X0, Y0 = 16.0 * tx + 0.5, 16.0 * ty + 0.5
                X1, Y1 = min(X0 + 15, W - 0.5), min(Y0 + 15, H - 0.5)
                got = orc.tile_test(cf, tx, ty, W, H)
                qmin = box_qmin_sampled(fx, fy, A, B, C, X0, X1, Y0, Y1)
                if abs(qmin - 9.0) < 1e-3:
                    n_tie += 1
                    continue
                n_chk += 1
                assert got == ellipse_meets_box(fx, fy, A, B, C, X0, X1, Y0, Y1), \
                    (mx, my, sx, sy, th, tx, ty)
                px = np.arange(16) + 16 * tx + 0.5
                py = np.arange(16) + 16 * ty + 0.5
                X, Y = np.meshgrid(px[px < W], py[py < H])
                q = A * (X - fx) ** 2 + 2 * B * (X - fx) * (Y - fy) + C * (Y - fy) ** 2
                if q.min() <= 9.0:
                    assert got
    assert n_chk > 30000 and n_tie < n_chk // 100


def test_ellipse_binning_keeps_rect_subset(orc):
    cam = ident_cam(200, 120)
    g = S.random_gaussians(3000, cam, seed=4)
    out = orc.rasterize(g, cam, orc.params_array())
    bs = out["bs"]
    assert 0 < bs["n_pairs"] < bs["n_rect_pairs"]
    r = out["pj"]["rect"]
    W16 = (cam.width + 15) // 16
    tx, ty = bs["tile_of"] % W16, bs["tile_of"] // W16
    gi = bs["gid_of"]
    assert np.all((tx >= r[gi, 0]) & (tx < r[gi, 2]) & (ty >= r[gi, 1]) & (ty < r[gi, 3]))


def test_ellipse_cutoff_bounded_on_the_image(orc):
    """The ellipse/tile cut (R16) changes the image by no more than the alpha
    of the entries it drops.  With no early stop and colours and background
    in [0, 1], leaving entries out of a pixel's front-to-back list changes
    each channel by at most the sum of their a_i.  So the render that keeps
    every tile of each Gaussian's rectangle (3D-GS's binning, same depth
    order) and the ellipse-cut render differ per pixel by at most that sum,
    computed here from the dropped entries, each of which lies outside the
    3-sigma ellipse at every pixel of its tile (q > 9, so a < 0.0112 op)."""
    cam = ident_cam(96, 80)
    g = S.random_gaussians(400, cam, seed=9)
    prm = orc.params_array(t_min=0.0)
    out = orc.rasterize(g, cam, prm)
    pj, bs = out["pj"], out["bs"]
    W, H = cam.width, cam.height
    ntx, nty = (W + 15) // 16, (H + 15) // 16
    vis = np.flatnonzero(pj["vis"])
    order = vis[np.lexsort((vis, pj["depth"][vis]))]  # depth, then slot
    lists = [[] for _ in range(ntx * nty)]
    for gid in order:
        x0, y0, x1, y1 = pj["rect"][gid]
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                lists[ty * ntx + tx].append(int(gid))
    gid_of = np.array([q for lst in lists for q in lst], np.uint32)
    ends = np.cumsum([len(lst) for lst in lists])
    ranges = np.stack([ends - [len(lst) for lst in lists], ends], axis=1).astype(np.uint32)
    full = orc.composite(pj, dict(gid_of=gid_of, ranges=ranges, n_pairs=len(gid_of)), cam, prm)
    bound = np.zeros((H, W))
    n_drop = 0
    for t, lst in enumerate(lists):
        s_, e_ = bs["ranges"][t]
        kept = set(int(q) for q in bs["gid_of"][s_:e_])
        tx, ty = t % ntx, t // ntx
        xs = np.arange(16 * tx, min(16 * tx + 16, W)) + 0.5
        ys = np.arange(16 * ty, min(16 * ty + 16, H)) + 0.5
        X, Y = np.meshgrid(xs, ys)
        for gid in lst:
            if gid in kept:
                continue
            n_drop += 1
            mx, my, ca, cb, cc, op = pj["proj"][gid][:6]
            dx, dy = X - mx, Y - my
            q = ca * dx * dx + 2.0 * cb * dx * dy + cc * dy * dy
            assert q.min() > 9.0
            a = np.minimum(prm[0], op * np.exp(-0.5 * q))
            assert a.max() < 0.0112 * op
            bound[16 * ty:16 * ty + len(ys), 16 * tx:16 * tx + len(xs)] += a
    assert n_drop > 500
    diff = np.abs(full["img"] - out["img"]).max(axis=0)
    assert diff.max() > 0.0
    assert np.all(diff <= bound + 1e-12)


def test_equal_depth_tie_break(orc):
    cam = ident_cam(64, 64, 60.0)
    g = S.tile_aligned_gaussians(cam, [5.0] * 6 + [7.0] * 6, seed=3)
    pj = orc.project(g, cam, orc.params_array())
    bs = orc.bin_sort(pj, cam)
    for t in range(bs["ranges"].shape[0]):
        s, e = bs["ranges"][t]
        ids = bs["gid_of"][s:e]
        d = pj["depth"][ids]
        for i in range(len(ids) - 1):
            assert d[i] < d[i + 1] or (d[i] == d[i + 1] and ids[i] < ids[i + 1])


# --------------------------------------------------------------------------
# Eq. 7 selection
# --------------------------------------------------------------------------

def test_thr2_closed_form(orc):
    """With Delta L = 0: thr2 = fl(d_max^2) / 4^L exactly, +inf at level 0."""
    level = np.arange(10, dtype=np.uint8)
    d_max = 1463.6878662109375
    thr = orc.lod_thr2(level, np.zeros(10, np.float32), d_max)
    assert np.isinf(thr[0])
    sq = F32(d_max) * F32(d_max)
    for L in range(1, 10):
        assert thr[L] == F32(sq * F32(2.0 ** (-2 * L)))


def _random_anchor_set(rng, n, K):
    pos = rng.uniform(-60, 60, (n, 3)).astype(np.float32)
    level = rng.integers(0, K, n).astype(np.uint8)
    bias = rng.uniform(-0.5, 0.5, n).astype(np.float32)
    rho = np.full(n, 1e6, np.float32)  # visibility always true
    return pos, level, bias, rho


def test_threshold_form_matches_literal_eq7(orc):
    """The transcendental-free FP32 rule equals the literal
    floor(clamp(log2(d_max / (d s)) + Delta L)) rule except within rounding
    distance of a threshold."""
    rng = np.random.default_rng(11)
    K, d_max = 6, 150.0
    pos, level, bias, rho = _random_anchor_set(rng, 200_000, K)
    cam = S.look_at((5.0, -7.0, 3.0), (0.0, 0.0, 0.0), 256, 256, 60.0)
    thr = orc.lod_thr2(level, bias, d_max)
    a = orc.select_mask(pos, thr, rho, cam)
    b = orc.select_eq7_mask(pos, level, bias, d_max, K, rho, cam)
    diff = np.flatnonzero(a != b)
    d = np.linalg.norm(pos.astype(np.float64) - cam.C.astype(np.float64), axis=1)
    lim = float(F32(d_max)) * 2.0 ** (bias.astype(np.float64) - level)
    for j in diff:
        assert level[j] > 0 and abs(d[j] / lim[j] - 1) < 1e-5
    assert len(diff) <= 3
    # both readings of the clamp agree when Delta L = 0
    z = np.zeros_like(bias)
    a0 = orc.select_mask(pos, orc.lod_thr2(level, z, d_max), rho, cam)
    b0 = orc.select_eq7_mask(pos, level, z, d_max, K, rho, cam)
    assert np.count_nonzero(a0 != b0) <= 3


# --------------------------------------------------------------------------
# LOD transition blending (Sec. IV-A): level L_hat + 1 with opacity scaled by
# the fractional level
# --------------------------------------------------------------------------

def test_blend_selection_matches_literal_rule(orc):
    """The FP32 threshold rule with blending (4 thr2) equals the literal
    rule (L <= L_hat, or L = L_hat + 1 with a nonzero factor L* - L_hat)
    except within rounding distance of a threshold; the added anchors are
    exactly level L_hat + 1."""
    rng = np.random.default_rng(12)
    K, d_max = 6, 150.0
    pos, level, bias, rho = _random_anchor_set(rng, 200_000, K)
    cam = S.look_at((5.0, -7.0, 3.0), (0.0, 0.0, 0.0), 256, 256, 60.0)
    thr = orc.lod_thr2(level, bias, d_max)
    a = orc.select_mask(pos, thr, rho, cam, blend=True)
    b = orc.select_eq7_mask(pos, level, bias, d_max, K, rho, cam, blend=True)
    d = np.linalg.norm(pos.astype(np.float64) - cam.C.astype(np.float64), axis=1)
    lim = float(F32(d_max)) * 2.0 ** (bias.astype(np.float64) - level + 1)
    diff = np.flatnonzero(a != b)
    for j in diff:
        assert level[j] > 0 and abs(d[j] / lim[j] - 1) < 1e-5
    assert len(diff) <= 3
    plain = orc.select_mask(pos, thr, rho, cam)
    assert np.all(a[plain == 1] == 1)
    lstar = np.clip(np.log2(float(F32(d_max)) / d) + bias, 0, K - 1)
    extra = np.flatnonzero((a == 1) & (plain == 0))
    near = np.abs(lstar - np.round(lstar)) < 1e-5
    ok = (level[extra] == np.floor(lstar[extra]) + 1) | near[extra]
    assert ok.all() and len(extra) > 1000


def test_blend_factor_closed_form(orc):
    """Factor 1 at and below L_hat, L* - L_hat at L_hat + 1, 0 above; L* is
    clamped to [0, K - 1]."""
    f = orc.lod_blend_factor
    d_max, K = 100.0, 4
    # d = 100 / 2^1.25 -> L* = 1.25, L_hat = 1
    d = 100.0 / 2 ** 1.25
    assert f(d, 1.0, d_max, 0.0, 0, K) == 1.0
    assert f(d, 1.0, d_max, 0.0, 1, K) == 1.0
    assert abs(f(d, 1.0, d_max, 0.0, 2, K) - 0.25) < 1e-12
    assert f(d, 1.0, d_max, 0.0, 3, K) == 0.0
    # bias shifts L*; s scales the distance
    assert abs(f(d, 1.0, d_max, 0.5, 2, K) - 0.75) < 1e-12
    assert abs(f(d / 2 ** 0.5, 2 ** 0.5, d_max, 0.0, 2, K) - 0.25) < 1e-12
    # clamps: far away L* = 0 (level 1 gets 0), very close L* = K - 1
    assert f(1e6, 1.0, d_max, 0.0, 1, K) == 0.0 and f(1e6, 1.0, d_max, 0.0, 0, K) == 1.0
    assert f(1e-3, 1.0, d_max, 0.0, K - 1, K) == 1.0


def test_blend_removes_lod_popping(orc):
    """Moving the focal scale s across the value where a level-1 anchor's
    L* crosses 1: without blending the image jumps (the anchor appears),
    with blending it changes by O(eps)."""
    sc = S.make_config1()
    cam = S.config1_camera()
    thr, rho = orc.scene_thresholds(sc)
    d = np.linalg.norm(sc.pos.astype(np.float64) - cam.C.astype(np.float64), axis=1)
    vis = orc.select_mask(sc.pos, np.full_like(thr, np.inf), rho, cam).astype(bool)
    cand = np.flatnonzero(vis & (sc.level == 1) & (sc.lod_bias == 0))
    j = cand[np.argmin(np.abs(d[cand] - np.median(d[cand])))]
    s_star = float(F32(sc.d_max)) / (2.0 * d[j])   # log2(d_max / (d_j s*)) = 1
    prm = orc.params_array()
    eps = 1e-5

    def img(scale, blend):
        c = S.Camera(R=cam.R, C=cam.C, fx=cam.fx, fy=cam.fy, cx=cam.cx, cy=cam.cy,
                     width=cam.width, height=cam.height, z_near=cam.z_near, lod_scale=scale)
        return orc.render(sc, c, prm, blend=blend)["img"]

    jump = np.abs(img(s_star * (1 + eps), False) - img(s_star * (1 - eps), False)).max()
    cont = np.abs(img(s_star * (1 + eps), True) - img(s_star * (1 - eps), True)).max()
    assert jump > 1e-3
    assert cont < 10 * eps


def test_level_monotone_in_distance(orc):
    """Along a ray from the camera, the anchors of each level that pass Eq. 7
    form a prefix (near ones pass, far ones do not)."""
    cam = S.look_at((0.0, 0.0, 0.0), (1.0, 0.3, 0.2), 64, 64, 60.0)
    dirv = cam.R[2].astype(np.float64)
    t = np.linspace(0.5, 400, 2000)
    K, d_max = 8, 300.0
    for L in range(K):
        pos = (t[:, None] * dirv[None, :]).astype(np.float32)
        level = np.full(len(t), L, np.uint8)
        thr = orc.lod_thr2(level, np.zeros(len(t), np.float32), d_max)
        m = orc.select_mask(pos, thr, np.full(len(t), 1e6, np.float32), cam).astype(bool)
        k = np.argmin(m) if not m.all() else len(m)
        assert m[:k].all() and not m[k:].any()
        if L > 0:
            assert abs(t[k - 1] - d_max / 2 ** L) < 0.25 or abs(t[k] - d_max / 2 ** L) < 0.25


def test_cumulative_levels_nested(orc):
    """Cumulative LOD: wherever a level-L anchor is selected, anchors of every
    coarser level at the same place are selected too."""
    rng = np.random.default_rng(3)
    K = 7
    base = rng.uniform(-80, 80, (3000, 3)).astype(np.float32)
    pos = np.repeat(base, K, axis=0)
    level = np.tile(np.arange(K, dtype=np.uint8), 3000)
    cam = S.look_at((1.0, -2.0, 3.0), (0.0, 0.0, 0.0), 64, 64, 60.0)
    thr = orc.lod_thr2(level, np.zeros(len(level), np.float32), 200.0)
    m = orc.select_mask(pos, thr, np.full(len(level), 1e6, np.float32), cam).reshape(3000, K)
    assert m[:, 0].all()
    assert np.all(np.diff(m.astype(np.int8), axis=1) <= 0)
    assert m[:, 1:].any() and not m.all()


def test_all_levels_render_equals_flat_render(orc):
    sc = S.make_config1()
    cam = S.config1_camera()
    prm = orc.params_array()
    rho = orc.bound_radius(sc.offsets, sc.offset_scale, sc.base_scale)
    thr_all = orc.lod_thr2(sc.level, sc.lod_bias, 1e30)
    a = orc.render(sc, cam, prm, thr2=thr_all, rho=rho)
    flat = np.full(sc.n, np.inf, np.float32)
    b = orc.render(sc, cam, prm, thr2=flat, rho=rho)
    assert np.array_equal(a["idx"], b["idx"])
    assert np.array_equal(a["img"], b["img"])
    assert len(a["idx"]) > len(orc.select(sc, cam))


def test_bound_radius_covers_decoded_gaussians(orc):
    sc = S.make_config1()
    cam = S.config1_camera()
    rho = orc.bound_radius(sc.offsets, sc.offset_scale, sc.base_scale)
    idx = np.arange(0, sc.n, 7)
    gd = orc.decode(sc, idx, cam)
    mean = gd[0:3].T.reshape(len(idx), sc.k, 3)
    smax = gd[3:6].max(axis=0).reshape(len(idx), sc.k)
    reach = np.linalg.norm(mean - sc.pos[idx][:, None, :].astype(np.float64), axis=2) + 3 * smax
    assert np.all(reach <= rho[idx][:, None].astype(np.float64) * (1 + 1e-6))


# --------------------------------------------------------------------------
# Eq. 3 / Eq. 4 decode special cases
# --------------------------------------------------------------------------

def tiny_scene(F=32, W=8, k=2, n=3, seed=0):
    rng = np.random.default_rng(seed)
    pos = np.array([[3.0, 4.0, 0.0], [0.0, 0.0, 2.0], [-1.0, 2.0, 2.0]], np.float32)[:n]
    mlp = S.xavier_mlp(rng, F + 4, W, k)
    for key in mlp:
        mlp[key][:] = 0
    sc = S.Scene(pos=pos, level=np.zeros(n, np.uint8), lod_bias=np.zeros(n, np.float32),
                 feat=rng.standard_normal((n, F)).astype(np.float32),
                 offsets=rng.standard_normal((n, k, 3)).astype(np.float32),
                 offset_scale=rng.uniform(0.5, 2, (n, 3)).astype(np.float32),
                 base_scale=rng.uniform(0.1, 1, (n, 3)).astype(np.float32), mlp=mlp,
                 d_max=10.0, d_min=1.0, n_levels=1, delta=1.0, k=k, feat_dim=F, width=W,
                 info={})
    cam = ident_cam()
    return sc, cam


def sig(x):
    return 1 / (1 + math.exp(-x))


def test_decode_biases_only(orc):
    """All weights zero: every output is its bias through its activation."""
    sc, cam = tiny_scene()
    k = sc.k
    sc.mlp["b2_a"][:] = [0.3, -0.2]
    sc.mlp["b2_c"][:] = np.arange(3 * k) * 0.1 - 0.2
    b2s = np.zeros(7 * k, np.float32)
    b2s[0:3] = [0.5, -1.0, 2.0]
    b2s[3:7] = [0.0, 3.0, 0.0, 4.0]        # quaternion (0, .6, 0, .8)
    b2s[7:10] = [0.0, 0.0, 0.0]
    b2s[10:14] = [0.0, 0.0, 0.0, 0.0]      # zero quaternion -> identity
    sc.mlp["b2_s"][:] = b2s
    gd = orc.decode(sc, np.arange(3), cam)
    G = 3 * k
    for s in range(3):
        for i in range(k):
            g = s * k + i
            np.testing.assert_allclose(gd[10, g], math.tanh(sc.mlp["b2_a"][i]), rtol=1e-15)
            for c in range(3):
                np.testing.assert_allclose(gd[11 + c, g], sig(sc.mlp["b2_c"][3 * i + c]), rtol=1e-15)
                np.testing.assert_allclose(gd[3 + c, g], float(sc.base_scale[s, c]) * sig(b2s[7 * i + c]),
                                           rtol=1e-15)
                exp_mean = float(sc.pos[s, c]) + float(sc.offsets[s, i, c]) * float(sc.offset_scale[s, c])
                np.testing.assert_allclose(gd[c, g], exp_mean, rtol=1e-15)
        np.testing.assert_allclose(gd[6:10, s * k], [0, 0.6, 0, 0.8], atol=1e-15)
        np.testing.assert_allclose(gd[6:10, s * k + 1], [1, 0, 0, 0], atol=0)
    assert gd.shape == (14, G)


def test_decode_input_distance_and_direction(orc):
    """Route inputs F..F+3 (relative distance, direction) straight to the
    opacity of Gaussian 0 and 1 through identity-like weights: the anchor
    at (3, 4, 0) seen from the origin with d_max = 10 has relative distance
    0.5 and direction (0.6, 0.8, 0)."""
    sc, cam = tiny_scene()
    F = sc.feat_dim
    w1 = sc.mlp["w1_a"]
    w1[F + 0, 0] = 1.0   # hidden 0 = relu(dist / d_max)
    w1[F + 2, 1] = 1.0   # hidden 1 = relu(dir_y)
    w1[F + 1, 2] = -1.0  # hidden 2 = relu(-dir_x) -> 0 for this anchor
    w2 = sc.mlp["w2_a"]
    w2[0, 0] = 1.0
    w2[1, 1] = 1.0
    w2[2, 1] = 5.0
    gd = orc.decode(sc, np.array([0]), cam)
    np.testing.assert_allclose(gd[10, 0], math.tanh(0.5), rtol=1e-15)
    np.testing.assert_allclose(gd[10, 1], math.tanh(0.8), rtol=1e-14)


def test_decode_relu_and_feature_path(orc):
    """A hidden unit fed feature 0 with weight 1 and bias -b: the output is
    relu(f0 - b) times the second-layer weight."""
    sc, cam = tiny_scene()
    sc.mlp["w1_c"][0, 3] = 1.0
    sc.mlp["b1_c"][3] = 0.25
    sc.mlp["w2_c"][3, 4] = 2.0
    gd = orc.decode(sc, np.arange(3), cam)
    for s in range(3):
        h = max(float(sc.feat[s, 0]) + 0.25, 0.0)
        # output 4 = Gaussian 1, green channel
        np.testing.assert_allclose(gd[12, s * sc.k + 1], sig(2.0 * h), rtol=1e-14)


# --------------------------------------------------------------------------
# anchor-skip predictor (oracle)
# --------------------------------------------------------------------------

def _skip_net(rng):
    a1, a2, a3 = (math.sqrt(6 / (37 + 64)), math.sqrt(6 / 128), math.sqrt(6 / 65))
    return {"w1": rng.uniform(-a1, a1, (37, 64)).astype(np.float32),
            "b1": rng.uniform(-0.1, 0.1, 64).astype(np.float32),
            "w2": rng.uniform(-a2, a2, (64, 64)).astype(np.float32),
            "b2": rng.uniform(-0.1, 0.1, 64).astype(np.float32),
            "w3": rng.uniform(-a3, a3, (64, 1)).astype(np.float32),
            "b3": np.array([0.05], np.float32)}


def test_skip_features_closed_form(orc):
    sc, cam = tiny_scene()
    sc.level = np.array([0, 3, 7], np.uint8)
    z = orc.skip_features(sc, np.arange(3), cam)
    # anchor 0 at (3, 4, 0) from the origin: direction (0.6, 0.8, 0), distance 5
    np.testing.assert_allclose(z[0, 32:35], [0.6, 0.8, 0.0], atol=1e-15)
    # a camera turned 90 degrees about z sees that direction as (0.8, -0.6, 0)
    cam2 = S.Camera(R=np.array([[0, 1, 0], [-1, 0, 0], [0, 0, 1]]), C=np.zeros(3), fx=80, fy=80,
                    cx=32, cy=32, width=64, height=64)
    z2 = orc.skip_features(sc, np.arange(1), cam2)
    np.testing.assert_allclose(z2[0, 32:35], [0.8, -0.6, 0.0], atol=1e-15)
    np.testing.assert_allclose(z[0, 35], math.log2(5.0 / 10.0), rtol=1e-15)
    np.testing.assert_array_equal(z[:, 36], [0, 3, 7])
    np.testing.assert_array_equal(z[:, :32], sc.feat.astype(np.float64))


def test_skip_mlp_gradient_fd(orc):
    rng = np.random.default_rng(0)
    net = _skip_net(rng)
    z = rng.standard_normal((64, 37))
    y = (rng.random(64) < 0.4).astype(np.float32)
    _, loss0, g = orc.skip_mlp(z, net, y, pos_weight=2.0, grads=True)
    assert loss0 > 0
    for name in ("w1", "b1", "w2", "b2", "w3", "b3"):
        arr = net[name]
        pick = rng.choice(arr.size, min(arr.size, 30), replace=False)
        a_vals, f_vals = [], []
        for fi in pick:
            x = float(arr.flat[fi])
            # small enough that no ReLU kink of the 64 rows is crossed
            h = np.float32(2.0 ** -20 * max(1.0, abs(x)))
            vals = []
            for sgn in (1, -1):
                n2 = dict(net)
                n2[name] = arr.copy()
                n2[name].flat[fi] = np.float32(x + sgn * h)
                vals.append((orc.skip_mlp(z, n2, y, pos_weight=2.0)[1], float(n2[name].flat[fi])))
            f_vals.append((vals[0][0] - vals[1][0]) / (vals[0][1] - vals[1][1]))
            a_vals.append(g[name].flat[fi])
        a_vals, f_vals = np.array(a_vals), np.array(f_vals)
        assert np.linalg.norm(a_vals - f_vals) <= 1e-5 * np.linalg.norm(f_vals) + 1e-12, name


def test_skip_mlp_bce_closed_form(orc):
    """A network that outputs its bias only: loss = softplus(b) - y b."""
    rng = np.random.default_rng(1)
    net = _skip_net(rng)
    for k in ("w1", "w2", "w3", "b1", "b2"):
        net[k] = np.zeros_like(net[k])
    net["b3"] = np.array([0.7], np.float32)
    z = rng.standard_normal((10, 37))
    y = np.array([1, 0] * 5, np.float32)
    logit, loss, _ = orc.skip_mlp(z, net, y, pos_weight=3.0)
    b = float(np.float32(0.7))
    sp = math.log1p(math.exp(b))
    np.testing.assert_allclose(logit, b, rtol=1e-15)
    np.testing.assert_allclose(loss, (5 * 3.0 * (sp - b) + 5 * sp) / 10, rtol=1e-14)
