"""Helpers for the GPU parity tests: device uploads, error bounds, reporting."""

import math
import sys

import numpy as np

U32 = 2.0 ** -24   # unit roundoff, FP32
UBF = 2.0 ** -8    # unit roundoff, BF16 (8-bit significand)


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def psnr(a, b):
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10 * math.log10(1.0 / mse)


def decode_bounds(scene, idx, cam, bf16: bool):
    """Element-wise bound on |decode_gpu - decode_exact| for the pre-activation
    outputs of each head, from the standard dot-product error bound
    |fl(w.x) - w.x| <= gamma_K sum |w||x| (gamma_K = K u / (1 - K u)), applied
    to both layers, plus the input and weight rounding to BF16 on that path.
    Returns (bound_a [m, k], bound_c [m, 3k], bound_s [m, 7k]) in float64."""
    F = scene.feat_dim
    pos = scene.pos[idx].astype(np.float64)
    d = pos - cam.C.astype(np.float64)[None]
    dist = np.linalg.norm(d, axis=1)
    x = np.concatenate([scene.feat[idx].astype(np.float64), (dist / scene.d_max)[:, None],
                        d / dist[:, None]], axis=1)
    ax = np.abs(x)
    # the FP32 path forms dist and dir in FP32: a few ulps each
    ex_in = np.zeros_like(x)
    ex_in[:, F:] = 4 * U32 * ax[:, F:] + 4 * U32
    if bf16:
        ex_in = ex_in + UBF * ax
    out = []
    raw = {}
    for h in ("a", "c", "s"):
        w1 = scene.mlp["w1_" + h].astype(np.float64)
        b1 = scene.mlp["b1_" + h].astype(np.float64)
        w2 = scene.mlp["w2_" + h].astype(np.float64)
        b2 = scene.mlp["b2_" + h].astype(np.float64)
        K1, W = w1.shape
        aw1 = np.abs(w1)
        hpre = x @ w1 + b1
        hid = np.maximum(hpre, 0)
        s1 = ax @ aw1 + np.abs(b1)
        g1 = (K1 + 2) * U32 / (1 - (K1 + 2) * U32)
        eh = g1 * s1 + ex_in @ aw1
        if bf16:
            eh = eh + UBF * (ax @ aw1)          # weight rounding
            eh = eh + UBF * (np.abs(hid) + eh)  # hidden rounded to BF16
        aw2 = np.abs(w2)
        s2 = (np.abs(hid) + eh) @ aw2 + np.abs(b2)
        g2 = (W + 2) * U32 / (1 - (W + 2) * U32)
        ey = g2 * s2 + eh @ aw2
        if bf16:
            ey = ey + UBF * ((np.abs(hid) + eh) @ aw2)
        out.append(ey)
        raw[h] = hid @ w2 + b2
    out.append(raw)
    return out


def decoded_field_bounds(scene, idx, cam, gd, bf16: bool):
    """Per-element bound [14][m*k] on the decoded Gaussian fields: tanh and
    sigmoid are 1- and 1/4-Lipschitz; scale = base_scale * sigmoid; the
    normalised quaternion moves by at most 2 |dq| / |q|; the mean is one fused
    multiply-add (half an ulp); 16 ulps cover each FP32 activation."""
    k = scene.k
    m = len(idx)
    G = m * k
    ba, bc, bs, raw = decode_bounds(scene, idx, cam, bf16)
    act = 16 * U32
    out = np.zeros((14, G))
    out[10] = ba.reshape(G) + act
    out[11:14] = (0.25 * bc.reshape(m, k, 3) + act).reshape(G, 3).T
    bsx = bs.reshape(m, k, 7)
    base = np.repeat(scene.base_scale[idx].astype(np.float64), k, axis=0)  # [G, 3]
    out[3:6] = (base * (0.25 * bsx[:, :, 0:3].reshape(G, 3) + act)).T
    qerr = np.linalg.norm(bsx[:, :, 3:7].reshape(G, 4), axis=1)
    qraw = np.linalg.norm(raw["s"].reshape(m, k, 7)[:, :, 3:7].reshape(G, 4), axis=1)
    out[6:10] = np.broadcast_to(2 * qerr / np.maximum(qraw - qerr, 1e-30) + act, (4, G))
    out[0:3] = np.abs(gd[0:3]) * U32 * 1.01
    return out


def report(name, gpu, ref, tol):
    diff = np.abs(np.asarray(gpu, np.float64) - np.asarray(ref, np.float64))
    say(f"{name}: max abs err {diff.max() if diff.size else 0:.3e} (tol {tol:.1e})")
    return diff


def decision_bounds(scene, idx, cam, gd):
    """Bounds [14][m*k] on how far the FP32 decode of the HIP path can lie
    from the oracle's decode rounded to FP32, for the near-threshold check of
    the rasterizer's decisions (oracle.fragile).  As decoded_field_bounds,
    except the mean: both sides form x_v + O l with one rounding to FP32 (a
    fused multiply-add there, the double sum rounded here), which agree
    unless the double sum lies within one double ulp of a float midpoint;
    only such coordinates keep their half-ulp bound."""
    eb = decoded_field_bounds(scene, idx, cam, gd, False)
    m = gd[0:3]
    f = m.astype(np.float32).astype(np.float64)
    ulp_f = np.spacing(np.abs(m.astype(np.float32))).astype(np.float64)
    mid_lo, mid_hi = f - ulp_f / 2, f + ulp_f / 2
    ulp_d = np.spacing(np.abs(m))
    near_mid = (np.abs(m - mid_lo) <= ulp_d) | (np.abs(m - mid_hi) <= ulp_d)
    eb[0:3] = np.where(near_mid, eb[0:3], 0.0)
    return eb


def e2e_compare(vb, ref, fr, tol=1e-4, min_checked=0.0, what=""):
    """End-to-end FP32 parity of a HIP render (ViewBuffers after render)
    with the oracle's render `ref`, given the near-threshold marks `fr` of
    oracle.fragile: in every tile no near-threshold decision touches, the
    sorted (tile, slot) list is bit-exact; on every pixel of those tiles
    whose stop decision is not near t_min, the image is within tol (the
    final transmittance within 2 tol).  Prints the counts; returns them."""
    tile, slot, ranges = vb.sorted_lists()
    ok_tile = ~fr["tiles"].reshape(-1)
    mg, mr = ok_tile[tile], ok_tile[ref["bs"]["tile_of"]]
    lists_equal = (np.array_equal(tile[mg], ref["bs"]["tile_of"][mr]) and
                   np.array_equal(slot[mg], ref["bs"]["gid_of"][mr]))
    checked = ~fr["near_flagged"] & ~fr["near_t_min"]
    img = vb.rgb.detach().cpu().numpy().astype(np.float64)
    T = vb.T.detach().cpu().numpy().astype(np.float64)
    err = np.abs(img - ref["img"]).max(axis=0)
    e_chk = float(err[checked].max()) if checked.any() else 0.0
    e_T = float(np.abs(T - ref["T"])[checked].max()) if checked.any() else 0.0
    res = dict(pairs=int(len(tile)), pairs_ref=int(ref["bs"]["n_pairs"]),
               flagged_gaussians=fr["n_flagged"], flagged_tiles=int(fr["tiles"].sum()),
               checked_frac=float(checked.mean()), max_abs_checked=e_chk, max_abs_T_checked=e_T,
               max_abs_all=float(err.max()), pixels_over_tol_all=int((err > tol).sum()),
               psnr_all=psnr(img, ref["img"]), lists_equal_unflagged=lists_equal,
               list_pairs_checked=int(mg.sum()))
    say(f"{what} e2e: pairs {res['pairs']} (oracle {res['pairs_ref']}), flagged "
        f"{res['flagged_gaussians']} Gaussians / {res['flagged_tiles']} tiles, checked "
        f"{100 * res['checked_frac']:.1f}% of pixels: max abs {e_chk:.2e} (T {e_T:.2e}); "
        f"all pixels: max abs {res['max_abs_all']:.2e}, {res['pixels_over_tol_all']} over "
        f"{tol:.0e}, PSNR {res['psnr_all']:.1f} dB; unflagged lists equal: {lists_equal}")
    assert lists_equal, what
    # the image bar; the final transmittance, a product over up to thousands
    # of FP32 factors on long lists, gets twice that
    assert e_chk <= tol and e_T <= 2 * tol, what
    assert res["checked_frac"] >= min_checked, (what, res["checked_frac"])
    return res


def grad_compare(got, ref, fwd, fr, k, norm_tol=1e-3, rtol=1e-3, rms_tol=1e-2, what=""):
    """Gradients of the HIP path (`got`, name -> array) against the oracle's
    FP64 analytic gradients (`ref`): every tensor within norm_tol normwise,
    and element-wise |got - ref| <= rtol |ref| + rms_tol rms(ref) on every
    entry of each per-anchor array whose anchor no near-threshold decision
    touches (none of its Gaussians flagged by oracle.fragile, listed in a
    flagged tile or in a tile with a pixel whose stop decision is near
    t_min), and on every MLP weight when no decision is flagged at all (a
    flipped decision moves every weight's gradient).  The absolute part
    covers FP32 sums whose terms cancel: such an entry is small against its
    terms, and its rounding error is not.  Also printed: entries above 1e-6
    of the tensor's largest that miss rtol alone."""
    tiles = fr["tiles"].copy()
    H, W = fr["near_t_min"].shape
    ty, tx = np.nonzero(fr["near_t_min"])
    tiles[ty // 16, tx // 16] = True
    slots = np.flatnonzero(fr["flags"])
    in_flagged = np.isin(fwd["bs"]["tile_of"], np.flatnonzero(tiles.reshape(-1)))
    slots = np.union1d(slots, fwd["bs"]["gid_of"][in_flagged])
    n_anchor = len(ref["pos"])
    bad_anchor = np.zeros(n_anchor, bool)
    bad_anchor[fwd["idx"][slots // k]] = True
    any_flag = bool(fr["n_flagged"]) or bool(tiles.any())
    out = {}
    for name, r in ref.items():
        g = np.asarray(got[name], np.float64)
        r = np.asarray(r, np.float64)
        rel = np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-300)
        per_anchor = r.shape[:1] == (n_anchor,)
        if per_anchor:
            rows = ~bad_anchor
        else:
            rows = np.full(r.shape[0], not any_flag)
        m = rows.reshape((-1,) + (1,) * (r.ndim - 1)) & np.ones(r.shape, bool)
        d, a = np.abs(g - r)[m], np.abs(r)[m]
        rms = float(np.sqrt(np.mean(r * r))) if r.size else 0.0
        lim = rtol * a + rms_tol * rms
        nbad = int((d > lim).sum())
        worst = float((d / np.maximum(lim, 1e-300)).max()) if d.size else 0.0
        big = a > 1e-6 * np.abs(r).max() if r.size else a
        n_strict = int((d[big] > rtol * a[big]).sum())
        out[name] = (rel, worst, int(m.sum()), nbad)
        say(f"  {what} {name}: normwise {rel:.2e}; element-wise on {int(m.sum())} entries: worst "
            f"|err| / ({rtol:.0e} |ref| + {rms_tol:.0e} rms) = {worst:.3f}, {nbad} over; "
            f"{n_strict} of {int(big.sum())} entries above 1e-6 max miss {rtol:.0e} relative alone")
    for name, (rel, worst, n, nbad) in out.items():
        assert rel <= norm_tol, (what, name, rel)
        assert nbad == 0, (what, name, worst, nbad, n)
    return out


def elementwise(got, ref, rtol=1e-3, rms_tol=1e-2, what=""):
    """|got - ref| <= rtol |ref| + rms_tol rms(ref) per entry (the absolute
    part covers FP32 sums whose terms cancel); returns (worst ratio to that
    limit, entries over, entries) and prints them."""
    g = np.asarray(got, np.float64)
    r = np.asarray(ref, np.float64)
    d, a = np.abs(g - r), np.abs(r)
    rms = float(np.sqrt(np.mean(r * r))) if r.size else 0.0
    lim = rtol * a + rms_tol * rms
    worst = float((d / np.maximum(lim, 1e-300)).max()) if r.size else 0.0
    nbad = int((d > lim).sum())
    big = a > 1e-6 * a.max() if r.size else a
    n_strict = int((d[big] > rtol * a[big]).sum())
    say(f"  {what}: element-wise on {r.size} entries: worst |err| / ({rtol:.0e} |ref| + "
        f"{rms_tol:.0e} rms) = {worst:.3f}, {nbad} over; {n_strict} of {int(big.sum())} entries "
        f"above 1e-6 max miss {rtol:.0e} relative alone")
    return worst, nbad, int(r.size)
