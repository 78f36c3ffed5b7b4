"""Pins of the oracle's anchor visibility (the "visible anchors" of Sec. IV-A)
and of its EWA projection (Sec. III-A, Eq. 1 with Sigma = R S S^T R^T) under
a rotated camera.  None of them reuses the oracle's own formulas:

  * hand-placed points just inside and just outside each of the five frustum
    planes, the planes built here from back-projected edge rays and cross
    products (a camera with a generic rotation, a non-square image, an
    off-centre principal point and fx != fy);
  * conservativeness: the render with the real bound radii equals, bit for
    bit, the render that keeps every anchor passing the LOD rule;
  * invariance of the render under a rotation of scene and camera together
    (a cyclic permutation of the world axes);
  * the closed-form 2D covariance J Sigma_c J^T + dilation I of one Gaussian
    given in camera space, seen through a rotated camera.

The last test plants mistakes in a copy of the oracle (a side-plane tangent
built from the wrong image dimension, the dilation margin dropped, the
camera rotation transposed in the projection Jacobian) and checks that these
pins catch each of them.
"""

import math
import tempfile

import numpy as np
import pytest

from synth import scenes as S

F32 = np.float32


def generic_camera(C=(6.0, -11.0, 7.5), target=(0.3, 0.2, -0.4), roll_deg=23.0, W=160, H=96,
                   fx=130.0, fy=110.0, cx=70.0, cy=55.0):
    """Rotated camera (look-at plus a roll about the viewing axis) with a
    non-square image, off-centre principal point and fx != fy."""
    base = S.look_at(C, target, W, H, 60.0)
    g = math.radians(roll_deg)
    Rz = np.array([[math.cos(g), -math.sin(g), 0.0], [math.sin(g), math.cos(g), 0.0],
                   [0.0, 0.0, 1.0]])
    R = Rz @ base.R.astype(np.float64)
    return S.Camera(R=R, C=np.asarray(C, np.float64), fx=fx, fy=fy, cx=cx, cy=cy, width=W,
                    height=H)


def world(cam, pc):
    """World coordinates of camera-space points pc [n][3] (float64)."""
    return pc @ cam.R.astype(np.float64) + cam.C.astype(np.float64)[None, :]


def ray(cam, u, v):
    return np.array([(u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy, 1.0])


def side_planes(cam, pad):
    """Per side: (outward unit normal in camera space, slope t of the plane,
    its Jacobian-clamp slope l).  The plane holds the camera centre and the
    image edge moved out by pad pixels; its normal is the cross product of
    the rays through the ends of that edge, turned away from the image."""
    W, H = cam.width, cam.height
    ends = {"right": ((W + pad, 0.0), (W + pad, H)), "left": ((-pad, 0.0), (-pad, H)),
            "bottom": ((0.0, H + pad), (W, H + pad)), "top": ((0.0, -pad), (W, -pad))}
    inside = ray(cam, cam.cx, cam.cy)
    out = {}
    for side, (a, b) in ends.items():
        n = np.cross(ray(cam, *a), ray(cam, *b))
        n /= np.linalg.norm(n)
        if n @ inside > 0:
            n = -n
        out[side] = n
    return out


def weight(cam, side, pad, jac_clamp):
    """Multiple of the radius by which a sphere must lie beyond a side plane
    to be culled, in the reading that the cull is conservative for the EWA
    footprint with a clamped Jacobian: 1 (touching) plus |l - t| / sec(t),
    t the plane's slope and l the clamp slope of its axis."""
    if side in ("right", "left"):
        t = ((cam.width - cam.cx) if side == "right" else cam.cx) + pad
        t /= cam.fx
        lim = jac_clamp * 0.5 * cam.width / cam.fx
    else:
        t = ((cam.height - cam.cy) if side == "bottom" else cam.cy) + pad
        t /= cam.fy
        lim = jac_clamp * 0.5 * cam.height / cam.fy
    return 1.0 + abs(lim - t) / math.sqrt(1.0 + t * t)


# --------------------------------------------------------------------------
# (c) hand-placed spheres at each plane
# --------------------------------------------------------------------------

def hand_placed_cases(cam, pad, jac_clamp):
    """(camera-space centre, radius, expected visibility) just inside and
    just outside each of the five planes."""
    planes = side_planes(cam, pad)
    W, H = cam.width, cam.height
    rows = []
    # a point on each side plane, in the middle of its edge, at two depths
    on_edge = {"right": (W + pad, 0.45 * H), "left": (-pad, 0.6 * H),
               "bottom": (0.4 * W, H + pad), "top": (0.55 * W, -pad)}
    for side, (u, v) in on_edge.items():
        n = planes[side]
        for depth in (3.0, 17.0):
            base = depth * ray(cam, u, v)
            for rho in (0.0, 0.05 * depth):
                reach = rho * weight(cam, side, pad, jac_clamp)
                for sgn, vis in ((-1.0, True), (1.0, False)):
                    # beyond the plane by reach (1 -+ 1e-3), plus 1e-4 depth for rho = 0
                    d = reach * (1.0 + sgn * 1e-3) + sgn * 1e-4 * depth
                    rows.append((base + d * n, rho, vis, f"{side} z={depth} rho={rho:.2f}"))
    # near plane: the sphere reaches z_near or stops short of it
    zn = cam.z_near
    for rho in (0.0, 0.3):
        for sgn, vis in ((1.0, True), (-1.0, False)):
            z = zn - rho + sgn * 1e-3
            rows.append((np.array([0.01 * z, -0.02 * z, z]), rho, vis, f"near rho={rho}"))
    return rows


def check_hand_placed(orc):
    cam = generic_camera()
    prm = orc.params_array()
    pad = 3.0 * math.sqrt(float(prm[3]))
    rows = hand_placed_cases(cam, pad, float(prm[4]))
    pc = np.array([r[0] for r in rows])
    pos = world(cam, pc).astype(np.float32)
    rho = np.array([r[1] for r in rows], np.float32)
    thr = np.full(len(rows), np.inf, np.float32)
    got = orc.select_mask(pos, thr, rho, cam, prm=prm).astype(bool)
    want = np.array([r[2] for r in rows])
    bad = [rows[i][3] + (" kept" if got[i] else " culled") for i in np.flatnonzero(got != want)]
    assert not bad, bad
    return len(rows)


def test_visibility_hand_placed_spheres(orc):
    assert check_hand_placed(orc) == 4 * 2 * 2 * 2 + 4


def test_hand_placed_cases_are_geometric():
    """The placed centres sit where intended: signed distance to their plane
    is the stated multiple of the radius (independent of the oracle)."""
    cam = generic_camera()
    pad = 3.0 * math.sqrt(0.3)
    planes = side_planes(cam, pad)
    # each plane holds the camera centre and both corner rays of its edge
    for side, n in planes.items():
        assert abs(np.linalg.norm(n) - 1) < 1e-12
    assert planes["right"] @ ray(cam, cam.width + pad, 0.3 * cam.height) == pytest.approx(0, abs=1e-12)
    assert planes["top"] @ ray(cam, 0.7 * cam.width, -pad) == pytest.approx(0, abs=1e-12)
    # the image centre ray is inside every plane
    for n in planes.values():
        assert n @ ray(cam, cam.width / 2, cam.height / 2) < 0


# --------------------------------------------------------------------------
# (b) conservativeness: culling never changes the image
# --------------------------------------------------------------------------

def check_conservative(orc):
    sc = S.make_config1()
    cams = [generic_camera(C=(5.0, -9.0, 4.0), target=(0.5, 0.0, 0.0)),
            generic_camera(C=(-7.0, 3.0, 9.0), target=(-1.0, 1.5, -1.0), roll_deg=-31.0, W=97,
                           H=143, fx=95.0, fy=120.0, cx=55.0, cy=64.0)]
    prm = orc.params_array()
    thr, rho = orc.scene_thresholds(sc)
    inf = np.full(sc.n, np.inf, np.float32)
    near_misses = 0
    for cam in cams:
        cut = orc.render(sc, cam, prm, thr, rho)
        full = orc.render(sc, cam, prm, thr, inf)
        dropped = np.setdiff1d(full["idx"], cut["idx"])
        assert len(dropped) > 100
        # Gaussians of dropped anchors that pass the projection culls (their
        # rectangles touch the image) but list no tile: the cases a too-tight
        # cull would get wrong
        slot_anchor = np.repeat(full["idx"], sc.k)
        vis = full["pj"]["vis"].astype(bool)
        near_misses += int(np.count_nonzero(vis & np.isin(slot_anchor, dropped)))
        assert np.array_equal(cut["img"], full["img"])
        assert np.array_equal(cut["T"], full["T"])
        assert np.array_equal(cut["last"], full["last"])
    assert near_misses > 20, near_misses


def test_visibility_is_conservative(orc):
    check_conservative(orc)


# --------------------------------------------------------------------------
# (a) rotating scene and camera together leaves the render unchanged
# --------------------------------------------------------------------------

def cyclic(v):
    """World axes permuted cyclically: (x, y, z) -> (z, x, y), a rotation."""
    return np.stack([v[2], v[0], v[1]])


def check_rotation_invariance(orc):
    cam = generic_camera()
    g = S.random_gaussians(600, cam, 21, scale=(0.02, 0.9))
    # strongly anisotropic scales so that a wrong rotation shows
    g[3] *= 3.0
    g[5] *= 0.2
    gr = g.copy()
    gr[0:3] = cyclic(g[0:3])          # means
    gr[3:6] = cyclic(g[3:6])          # scales follow the axes
    gr[7:10] = cyclic(g[7:10])        # quaternion axis (conjugation by the permutation)
    P = cyclic(np.eye(3))
    camr = S.Camera(R=cam.R.astype(np.float64) @ P.T, C=P @ cam.C.astype(np.float64),
                    fx=cam.fx, fy=cam.fy, cx=cam.cx, cy=cam.cy, width=cam.width,
                    height=cam.height)
    prm = orc.params_array()
    a = orc.rasterize(g, cam, prm)
    b = orc.rasterize(gr, camr, prm)
    assert a["bs"]["n_pairs"] > 2000
    assert np.array_equal(a["pj"]["vis"], b["pj"]["vis"])
    assert np.array_equal(a["pj"]["rect"], b["pj"]["rect"])
    assert np.array_equal(a["bs"]["gid_of"], b["bs"]["gid_of"])
    assert np.array_equal(a["bs"]["ranges"], b["bs"]["ranges"])
    np.testing.assert_allclose(b["img"], a["img"], rtol=0, atol=1e-9)


def test_render_invariant_under_rotation(orc):
    check_rotation_invariance(orc)


# --------------------------------------------------------------------------
# closed-form EWA projection through a rotated camera
# --------------------------------------------------------------------------

def rot_from_axis(axis, ang):
    a = np.asarray(axis, np.float64)
    a /= np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def quat_wxyz(Rm):
    """Unit quaternion (w, x, y, z) of a rotation matrix (Shepperd's method)."""
    from scipy.spatial.transform import Rotation
    x, y, z, w = Rotation.from_matrix(Rm).as_quat()
    return np.array([w, x, y, z])


def check_rotated_closed_form(orc):
    cam = generic_camera()
    prm = orc.params_array()
    dil = float(F32(0.3))
    Rw = cam.R.astype(np.float64)
    cases = [((0.4, -0.3, 6.0), (0.35, 0.1, 0.6), (1.0, 2.0, -0.5), 0.7),
             ((-0.9, 0.5, 9.0), (0.5, 0.25, 0.08), (-0.3, 0.2, 1.0), 1.9),
             ((0.2, 0.6, 4.5), (0.06, 0.3, 0.45), (0.0, 1.0, 0.3), -0.8)]
    for xc, s, axis, ang in cases:
        Rc = rot_from_axis(axis, ang)              # the Gaussian's rotation in camera axes
        Sig_c = Rc @ np.diag(np.square(s)) @ Rc.T  # camera-space covariance
        q = quat_wxyz(Rw.T @ Rc)                   # world rotation: R_w^T R_c
        mean = world(cam, np.array([xc]))[0]
        g = np.array([*mean, *s, *q, 0.6, 0.3, 0.5, 0.7], np.float32).reshape(14, 1)
        out = orc.rasterize(g, cam, prm)
        assert out["pj"]["vis"][0] == 1
        # closed form from camera-space quantities only (|x/z|, |y/z| under the clamp)
        x, y, z = (float(v) for v in (Rw @ (g[:3, 0].astype(np.float64) - cam.C.astype(np.float64))))
        J = np.array([[cam.fx / z, 0.0, -cam.fx * x / z ** 2], [0.0, cam.fy / z, -cam.fy * y / z ** 2]])
        cov = J @ Sig_c @ J.T + dil * np.eye(2)
        con = np.linalg.inv(cov)
        p = out["pj"]["proj"][0]
        np.testing.assert_allclose(p[0:2], [cam.fx * x / z + cam.cx, cam.fy * y / z + cam.cy],
                                   rtol=1e-9)
        np.testing.assert_allclose(p[2:5], [con[0, 0], con[0, 1], con[1, 1]], rtol=2e-5)
        # the image: opacity * exp(-q / 2) on every listed pixel, listed wherever q <= 9
        X, Y = np.meshgrid(np.arange(cam.width) + 0.5, np.arange(cam.height) + 0.5)
        dx, dy = X - p[0], Y - p[1]
        qq = con[0, 0] * dx * dx + 2 * con[0, 1] * dx * dy + con[1, 1] * dy * dy
        alpha = np.minimum(0.99, 0.6 * np.exp(-0.5 * qq))
        drawn = out["img"][0] > 0
        assert np.all(drawn[qq <= 9.0 * (1 - 1e-4)])
        np.testing.assert_allclose(out["img"][0][drawn], 0.3 * alpha[drawn], rtol=1e-4)


def test_projection_closed_form_rotated_camera(orc):
    check_rotated_closed_form(orc)


# --------------------------------------------------------------------------
# the pins catch planted mistakes (oracle copies, CPU only)
# --------------------------------------------------------------------------

def _plant(src, edits):
    for old, new in edits:
        assert src.count(old) >= 1, old
        src = src.replace(old, new)
    return src


MISTAKES = {
    # right-hand side plane built from the image height
    "right tangent from H": ([("float tl = (k->cx + pad) / k->fx, tr = (((float)k->W - k->cx) + pad) / k->fx;",
                               "float tl = (k->cx + pad) / k->fx, tr = (((float)k->H - k->cx) + pad) / k->fx;")],
                             ("hand", "conservative")),
    # bottom side plane built from the image width (a wider plane)
    "bottom tangent from W": ([("tb = (((float)k->H - k->cy) + pad) / k->fy;",
                                "tb = (((float)k->W - k->cy) + pad) / k->fy;")], ("hand",)),
    # no dilation margin
    "no dilation pad": ([("float pad = 3.0f * sqrtf(pp->dilation);", "float pad = 0.0f;")],
                        ("hand",)),
    # R^T in place of R in the projection Jacobian T = J R (float decisions and double values)
    "R transposed in T": ([("T0[c] = fmaf(J00, Rc[c], J02 * Rc[6 + c]);",
                            "T0[c] = fmaf(J00, Rc[3 * c], J02 * Rc[3 * c + 2]);"),
                           ("T1[c] = fmaf(J11, Rc[3 + c], J12 * Rc[6 + c]);",
                            "T1[c] = fmaf(J11, Rc[3 * c + 1], J12 * Rc[3 * c + 2]);"),
                           ("T0[c] = J00 * k->R[c] + J02 * k->R[6 + c];",
                            "T0[c] = J00 * k->R[3 * c] + J02 * k->R[3 * c + 2];"),
                           ("T1[c] = J11 * k->R[3 + c] + J12 * k->R[6 + c];",
                            "T1[c] = J11 * k->R[3 * c + 1] + J12 * k->R[3 * c + 2];")],
                          ("rotation", "closed form")),
}

CHECKS = {"hand": check_hand_placed, "conservative": check_conservative,
          "rotation": check_rotation_invariance, "closed form": check_rotated_closed_form}


@pytest.mark.parametrize("name", sorted(MISTAKES))
def test_pins_catch_planted_mistakes(orc, name):
    edits, must_fail = MISTAKES[name]
    src = _plant(orc.source(), edits)
    with tempfile.TemporaryDirectory() as d:
        with orc.variant(src, d, tag=name.replace(" ", "_")):
            for check in must_fail:
                with pytest.raises(AssertionError):
                    CHECKS[check](orc)
