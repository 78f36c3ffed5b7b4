#!/usr/bin/env python3
"""Benchmark of the Octree-GS render path on one MI355X.

Workload (the large synthetic street scene): 1M anchors over 8 octree levels
voxelised from 20M points on 2,000 boxes over a [-500, 500]^2 ground plane,
feature dim 32, k = 10, MLP width 64; a 200-camera zoom-out from 10 m to
800 m altitude at 1920x1080, 60 degree FOV.  One step = one view through the
whole path: anchor selection (Eq. 7), decode (Eq. 3-4), projection, tile
binning, depth ordering and compositing (Eq. 2).  Steps cycle through the
trajectory; the scene and cameras are resident before timing starts.

Prints one JSON line.  value = frames per second of the fast path (BF16
decode on MFMA, plus the learned anchor skip unless it falls back to full
decode); the plain FP32 path is timed the same way on the same views and
reported beside it, with the per-view PSNR of the fast path against it.
Views are independent, so --inflight views (default 3) are rendered at once
on separate streams with separate buffers; the rate with one view in flight
is reported beside it.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "FPS @1080p + train-step ms, BF16+learned-skip vs plain FP32 at >=45 dB PSNR"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published FP32 vector peak
FLOP_PER_BLEND = 21.0
PMC_SUMMARY = os.path.join(ROOT, "profiles", "composite_street1080p_hbm_bytes.txt")
COMPOSITE_SOURCE = os.path.join(ROOT, "paper_2403_17898_amd", "csrc", "raster.hip")


def composite_traffic():
    """HBM bytes per composite launch from the committed FETCH_SIZE /
    WRITE_SIZE counter summary, or None when that summary is missing or was
    taken from a different version of the kernel source."""
    import hashlib
    try:
        text = open(PMC_SUMMARY).read()
        digest = hashlib.sha256(open(COMPOSITE_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in text.splitlines() if ":" in line)
    if fields.get("source_sha256", "").strip() != digest:
        return None
    try:
        return int(float(fields["hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="views timed per path")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--views", type=int, default=200, help="trajectory length")
    ap.add_argument("--inflight", type=int, default=4,
                    help="views in flight at once (one stream and buffer set each)")
    ap.add_argument("--cpu-views", type=int, default=60, help="views the CPU oracle renders")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="skip the PSNR sweep (profiling runs)")
    ap.add_argument("--no-train", action="store_true", help="skip the training-step timing")
    ap.add_argument("--no-skip", action="store_true", help="skip the learned-skip path")
    ap.add_argument("--no-3dgs", action="store_true",
                    help="skip the explicit-Gaussian (3D-GS instance) measurement")
    ap.add_argument("--skip-train-views", type=int, default=1000)
    ap.add_argument("--train-steps", type=int, default=20)
    ap.add_argument("--city", action="store_true",
                    help="also measure the city-scale scene (4M anchors / 10 levels): the "
                         "3840x2160 zoom-out and the 8-view 2048x1024 train step (several minutes)")
    ap.add_argument("--city-skip-views", type=int, default=300)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (scale for HBM byte counters)")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    """The host CPU's model name (Linux), for the CPU baseline."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _finite(v):
    """The result with non-finite floats (e.g. the PSNR of an exact image)
    as null, so the line is strict JSON."""
    if isinstance(v, dict):
        return {k: _finite(x) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [_finite(x) for x in v]
    if isinstance(v, float) and not math.isfinite(v):
        return None
    return v


def view_order(steps: int, nviews: int):
    """Indices of the views a pass of `steps` renders: a stride through the
    whole trajectory (every view once when steps == nviews), so any step
    count samples the zoom-out from its first to its last altitude."""
    if steps >= nviews:
        return [i % nviews for i in range(steps)]
    return [(i * nviews) // steps for i in range(steps)]


def time_views(args, torch, streams, views, bufs, render_one, depth):
    """(event ms, wall s) for args.steps views after args.warmup untimed
    ones; the i-th rendered view, views[view_order(...)[i]], runs on stream
    i % depth with buffers bufs[i % depth]."""
    stream = streams[0]

    def run(n):
        order = view_order(n, len(views))
        for i in range(n):
            k = i % depth
            render_one(k, views[order[i]], streams[k])
            # every frame's overflow / look-back / truncation bits, checked after the loop
            bufs[k].add_status(stream=streams[k])
    for b in bufs[:depth]:
        b.status.zero_()
    run(args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    e0.record(stream)
    for s in streams[1:depth]:
        s.wait_event(e0)
    run(args.steps)
    for s in streams[1:depth]:
        ev = torch.cuda.Event()
        ev.record(s)
        stream.wait_event(ev)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    for b in bufs[:depth]:
        b.check_status("timed frames")
    return e0.elapsed_time(e1), wall


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1 "
                                   "(the render path shards by views, see the design notes)"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2403_17898_amd as P
    from paper_2403_17898_amd import _lib as L
    from synth import scenes as S

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 5 x 256 MiB device-to-device copies")
        del src, dst

    t0 = time.time()
    sc = S.make_config2()
    cams = S.config2_cameras(args.views)
    log(f"scene: {sc.n} anchors, levels {sc.level_counts()}, d_max {sc.d_max:.1f}, "
        f"generated in {time.time() - t0:.1f}s")
    ds = P.DeviceScene.from_scene(sc)
    ccams = [P.make_camera(c) for c in cams]
    bcams = [P.make_camera(c, lod_blend=True) for c in cams]  # LOD transition blending
    prm = P.raster_params()
    W, H = cams[0].width, cams[0].height

    # ---- sizing pass (untimed): per-view selected anchors and pairs ----
    vb = P.ViewBuffers(sc.n, sc.k, W, H, pair_capacity=48 << 20)
    per_view = []
    for c in ccams + bcams:
        vb.render(ds, c, prm, precision=P.OCTGS_FP32)
        st = vb.stats()
        if st["pair_overflow"] or st["sync_error"]:
            raise SystemExit(f"sizing pass failed: {st}")
        per_view.append(st)
    blend_sel = float(np.mean([s["n_selected"] for s in per_view[len(ccams):]]))
    blend_pairs = float(np.mean([s["n_pairs"] for s in per_view[len(ccams):]]))
    max_sel = max(s["n_selected"] for s in per_view)
    max_pairs = max(s["n_candidates"] for s in per_view)
    del vb
    torch.cuda.empty_cache()
    gcap = max(1, int(max_sel * sc.k * 1.05) + 1024)
    pcap = max(1, int(max_pairs * 1.10) + 4096)
    # frames in flight: view i runs on stream i % D with its own buffers;
    # views are independent, so their latency-bound stages (scans, sorts)
    # overlap with other views' compositing
    D = max(1, args.inflight)
    vbs = [P.ViewBuffers(sc.n, sc.k, W, H, pair_capacity=pcap, gauss_capacity=gcap)
           for _ in range(D)]
    vb = vbs[0]
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(D - 1)]
    stream = streams[0]
    log(f"sizing: max selected {max_sel}, max candidate pairs {max_pairs}; gcap {gcap}, "
        f"pcap {pcap}; {D} frames in flight")

    def timed_views(render_one, depth, views=None, bufs=None):
        """ms for args.steps views (after args.warmup), view i on stream i % depth."""
        return time_views(args, torch, streams, ccams if views is None else views,
                          vbs if bufs is None else bufs, render_one, depth)

    def timed(prec, depth=D, views=None, params=prm):
        return timed_views(lambda k, c, s: vbs[k].render(ds, c, params, precision=prec, stream=s),
                           depth, views)

    ms32, wall32 = timed(P.OCTGS_FP32)
    ms16, wall16 = timed(P.OCTGS_BF16)
    # a frame alone on the GPU: tiles ordered longest-first within each XCD
    prm_one = P.raster_params(tile_order=True)
    ms32_1, _ = timed(P.OCTGS_FP32, 1, params=prm_one)
    ms16_1, _ = timed(P.OCTGS_BF16, 1, params=prm_one)
    fps32 = args.steps / (ms32 / 1e3)
    fps16 = args.steps / (ms16 / 1e3)
    single = {"fp32": round(args.steps / (ms32_1 / 1e3), 2), "bf16": round(args.steps / (ms16_1 / 1e3), 2)}
    log(f"plain FP32: {ms32 / args.steps:.3f} ms/view ({fps32:.1f} FPS); "
        f"BF16: {ms16 / args.steps:.3f} ms/view ({fps16:.1f} FPS); one frame in flight: {single}")
    msb, _ = timed(P.OCTGS_BF16, views=bcams)
    blend = {"fps_bf16": round(args.steps / (msb / 1e3), 2), "ms_per_view": round(msb / args.steps, 4),
             "mean_selected": round(blend_sel), "mean_pairs": round(blend_pairs)}
    log(f"LOD transition blending, BF16: {blend}")

    # ---- Our-3D-GS: explicit Gaussians with SH colour on the same anchors ----
    our3d = None
    if not args.no_3dgs:
        our3d = explicit_path(args, P, S, torch, np, sc, ccams, prm, W, H, D, streams,
                              timed_views)
        torch.cuda.empty_cache()

    # ---- learned anchor skip: trained on logged blend weights of random views ----
    skip = None
    if not args.no_skip:
        skip = skip_path(args, P, S, torch, np, sc, ds, ccams, prm, W, H, vb, timed_fn=None)
        ms_sk, _ = timed_skip(P, vbs, ds, prm, skip, timed_views, D)
        skip["fps"] = round(args.steps / (ms_sk / 1e3), 2)
        skip["ms_per_view"] = round(ms_sk / args.steps, 4)
        log(f"BF16 + learned skip: {ms_sk / args.steps:.3f} ms/view ({skip['fps']:.1f} FPS)")

    # ---- per-stage timing with HIP events on the library's stream ----
    from paper_2403_17898_amd.hip_events import HipEvent
    names = ["select", "decode"] + list(L.RASTER_STAGE_NAMES)
    tot = {k: 0.0 for k in names}
    order = view_order(args.steps, len(ccams))  # the timed passes' views
    nviews = len(order)
    sums = dict(selected=0, slots=0, visible=0, pairs=0, candidates=0, blends=0)
    view_ms = []
    ev = [HipEvent() for _ in range(4 + 2 * L.OCTGS_RASTER_STAGES)]
    sh = P.stream_handle(stream)
    for i in range(nviews):
        c = ccams[order[i]]
        ev[0].record(sh)
        vb.select(ds, c, prm)
        ev[1].record(sh)
        ev[2].record(sh)
        vb.decode(ds, c, P.OCTGS_BF16)
        ev[3].record(sh)
        vb.rasterize(c, prm, stage_events=ev[4:])
        torch.cuda.synchronize()
        vms = ev[0].elapsed_ms(ev[1]) + ev[2].elapsed_ms(ev[3])
        tot["select"] += ev[0].elapsed_ms(ev[1])
        tot["decode"] += ev[2].elapsed_ms(ev[3])
        for s_i, nm in enumerate(L.RASTER_STAGE_NAMES):
            tot[nm] += ev[4 + 2 * s_i].elapsed_ms(ev[5 + 2 * s_i])
            vms += ev[4 + 2 * s_i].elapsed_ms(ev[5 + 2 * s_i])
        view_ms.append(vms)
        s = vb.stats()
        sums["blends"] += int(vb.last.sum(dtype=torch.int64).item())
        sums["selected"] += s["n_selected"]
        sums["slots"] += s["n_slots"]
        sums["visible"] += s["n_visible"]
        sums["pairs"] += s["n_pairs"]
        sums["candidates"] += s["n_candidates"]
    avg = {k: v / nviews for k, v in tot.items()}  # ms per launch
    mean = {k: v / nviews for k, v in sums.items()}
    log("per-stage ms/view: " + ", ".join(f"{k} {v:.4f}" for k, v in avg.items()))
    log(f"mean per view: selected {mean['selected']:.0f}, Gaussians {mean['slots']:.0f}, "
        f"visible {mean['visible']:.0f}, pairs {mean['pairs']:.0f} "
        f"(of {mean['candidates']:.0f} rectangle candidates)")
    # each view alone on the GPU (the loop above) against the camera altitude
    vm = np.array(view_ms)
    alts = np.array([float(cams[order[i]].C[2]) for i in range(nviews)])
    edges = np.linspace(0, nviews, 11).round().astype(int)
    per_view = {"ms_mean": round(float(vm.mean()), 4), "ms_max": round(float(vm.max()), 4),
                "slowest_view": int(order[int(vm.argmax())]),
                "slowest_altitude_m": round(float(alts[vm.argmax()]), 1),
                "min_fps": round(1e3 / float(vm.max()), 1),
                "altitude_m_vs_ms": [[round(float(alts[a:b].mean()), 1), round(float(vm[a:b].mean()), 4)]
                                     for a, b in zip(edges[:-1], edges[1:]) if b > a]}
    log(f"each view alone: {per_view}")
    # decode on MFMA: first layers 36 -> 3 x W, second layers W -> 11 k (k
    # opacities, 3k colours, 7k covariance terms), 2 FLOP per multiply-add
    dec_flop = 2.0 * (36 * 3 * sc.width + sc.width * 11 * sc.k) * mean["selected"]
    decode_mfma = {"flop_per_anchor": int(dec_flop / max(mean["selected"], 1)),
                   "tflops": round(dec_flop / (avg["decode"] * 1e-3) / 1e12, 2)}
    decode_mfma["frac_bf16"] = round(decode_mfma["tflops"] / 2500.0, 5)
    log(f"decode (BF16, per call incl. the weight-fragment kernel): {decode_mfma}")

    # The dominant kernel, compositing, is bound by vector ALU work: per
    # pixel and Gaussian blended (Eq. 2) it evaluates the 2D Gaussian,
    # alpha, the colour update and T, 21 FLOP counting exp as one.  Units per
    # launch = sum over pixels of the entries each consumed (the `last`
    # output).  Its algorithmic HBM bytes per launch are reported beside.
    npix = W * H
    ntiles = ((W + 15) // 16) * ((H + 15) // 16)
    flop = FLOP_PER_BLEND * mean["blends"]
    ach = flop / (avg["composite"] * 1e-3) / 1e12
    # unique bytes: list entries 4 B per pair, the projected record 36 B per
    # visible Gaussian, tile ranges 8 B, and 20 B written per pixel
    alg_bytes = 4.0 * mean["pairs"] + 36.0 * mean["visible"] + 8.0 * ntiles + 20.0 * npix
    roofline = {"kernel": "composite", "bound": "alu", "achieved": round(ach, 2),
                "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / FP32_VECTOR_PEAK_TFLOPS, 4),
                "traffic": composite_traffic(),
                "algorithmic_bytes": round(alg_bytes),
                "hbm_gbs": round(alg_bytes / (avg["composite"] * 1e-3) / 1e9, 1),
                "blends_per_launch": round(mean["blends"]),
                "stage_ms": {k: round(v, 4) for k, v in avg.items()}}

    # ---- quality: BF16 path vs plain FP32, every view ----
    psnrs = []
    if not args.quick:
        for c in ccams:
            vb.render(ds, c, prm, precision=P.OCTGS_FP32)
            ref = vb.rgb.clone()
            vb.render(ds, c, prm, precision=P.OCTGS_BF16)
            mse = torch.mean((vb.rgb - ref) ** 2).item()
            psnrs.append(float("inf") if mse == 0 else 10 * math.log10(1.0 / mse))
        fin = [p for p in psnrs if math.isfinite(p)]
        log(f"PSNR BF16 vs FP32: min {min(psnrs):.2f} dB, mean {np.mean(fin) if fin else float('inf'):.2f} dB")

    # ---- CPU baseline: the oracle on a bounded sample of the same views ----
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        O.build(force=False)
        thr, rho = O.scene_thresholds(sc)
        pick = np.linspace(0, len(cams) - 1, max(1, args.cpu_views)).round().astype(int)
        t1 = time.perf_counter()
        for i in pick:
            O.render(sc, cams[i], O.params_array(), thr, rho)
        dt = time.perf_counter() - t1
        cpu = {"value": round(len(pick) / dt, 4), "unit": "FPS", "cores": O.num_threads(),
               "kind": "oracle",
               "sample": f"{len(pick)} evenly spaced views of the same trajectory, full FP64 "
                         f"select+decode+rasterize, {dt:.1f} s"}
        # one core, on three views of the same trajectory
        nthr = O.num_threads()
        O.set_num_threads(1)
        pick1 = np.linspace(0, len(cams) - 1, 3).round().astype(int)
        t1 = time.perf_counter()
        for i in pick1:
            O.render(sc, cams[i], O.params_array(), thr, rho)
        dt1 = time.perf_counter() - t1
        O.set_num_threads(nthr)
        cpu["one_core"] = {"value": round(len(pick1) / dt1, 4), "unit": "FPS", "cores": 1,
                           "sample": f"views {pick1.tolist()} of the trajectory, {dt1:.1f} s"}
        cpu["cpu_model"] = cpu_model()
        log(f"CPU oracle: {cpu}")

    train = None if args.no_train else train_step_timing(args, P, S, torch, np,
                                                         oracle_step=not args.no_cpu_baseline)
    city = city_path(args, P, S, torch, np, prm, D, streams) if args.city else None

    value = skip["fps"] if skip else fps16
    ms_value = skip["ms_per_view"] if skip else ms16 / args.steps
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "FPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_value, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "street scene: 1M anchors / 8 LOD levels, 200-view zoom-out "
                               "10->800 m, 1920x1080",
                   "n_anchors": sc.n, "k": sc.k, "mlp_width": sc.width, "views": len(cams),
                   "path": ("BF16 decode" if not skip else
                            ("BF16 decode; learned skip fell back to full decode"
                             if skip["fallback_to_full_decode"] else "BF16 decode + learned anchor skip")),
                   "mean_selected": round(mean["selected"]), "mean_gaussians": round(mean["slots"]),
                   "mean_visible": round(mean["visible"]), "mean_pairs": round(mean["pairs"]),
                   "mean_candidates": round(mean["candidates"])},
        "fps_plain_fp32": round(fps32, 2),
        "fps_bf16_no_skip": round(fps16, 2),
        "frames_in_flight": D,
        "lod_blend": blend,
        "fps_one_frame_in_flight": single,
        "ms_per_step_plain_fp32": round(ms32 / args.steps, 4),
        "speedup_vs_plain": round(value / fps32, 4),
        "psnr_vs_plain_min_db": (skip["psnr_min_db"] if skip else
                                 (round(min(psnrs), 2) if psnrs else None)),
        "psnr_vs_plain_mean_db": (skip["psnr_mean_db"] if skip else
                                  (round(float(np.mean([p for p in psnrs if math.isfinite(p)])), 2)
                                   if psnrs and any(math.isfinite(p) for p in psnrs) else None)),
        "psnr_bf16_no_skip_min_db": round(min(psnrs), 2) if psnrs else None,
        "skip": skip,
        "our_3dgs": our3d,
        "wall_s_timed": round(wall16, 3),
        "train_step_ms": train["ms_per_step"] if train else None,
        "train": train,
        "roofline": roofline,
        "each_view_alone": per_view,
        "decode_mfma": decode_mfma,
        "cpu_baseline": cpu,
    }
    if city is not None:
        out["city"] = city
    print(json.dumps(_finite(out), allow_nan=False), flush=True)


# per decoded explicit Gaussian: mean, log-scale, rotation and opacity
# logit read (44 B), the SH row (48 values, FP32 or BF16), the 56-byte
# record written, and the anchor index (4 B per k slots)
EXPLICIT_IO_BYTES = 44 + 56


def explicit_path(args, P, S, torch, np, sc, ccams, prm, W, H, D, streams, timed_views):
    """FPS of the 3D-GS instance (explicit degree-3 Gaussians on the config
    anchors) with FP32 and BF16 SH coefficients, and the decode kernel's
    achieved HBM rate."""
    from paper_2403_17898_amd.hip_events import HipEvent
    t0 = time.time()
    ex = S.make_explicit(sc, sh_degree=3)
    de = P.DeviceExplicit.from_scene(ex)
    del ex
    log(f"explicit scene: degree-3 SH, generated and uploaded in {time.time() - t0:.1f}s")
    vb = P.ViewBuffers(sc.n, sc.k, W, H, pair_capacity=64 << 20)
    max_sel = max_pairs = 0
    for c in ccams:
        vb.render_explicit(de, c, prm)
        st = vb.stats()
        if st["pair_overflow"] or st["sync_error"]:
            raise SystemExit(f"explicit sizing pass failed: {st}")
        max_sel = max(max_sel, st["n_selected"])
        max_pairs = max(max_pairs, st["n_candidates"])
    del vb
    torch.cuda.empty_cache()
    gcap = max(1, int(max_sel * sc.k * 1.05) + 1024)
    pcap = max(1, int(max_pairs * 1.10) + 4096)
    xvbs = [P.ViewBuffers(sc.n, sc.k, W, H, pair_capacity=pcap, gauss_capacity=gcap)
            for _ in range(D)]
    res = {"sh_degree": 3}
    for name, prec in (("fp32", P.OCTGS_FP32), ("bf16", P.OCTGS_BF16)):
        ms, _ = timed_views(lambda k, c, s: xvbs[k].render_explicit(de, c, prm, precision=prec,
                                                                   stream=s),
                            D, bufs=xvbs)
        res["fps_" + name] = round(args.steps / (ms / 1e3), 2)
        res["ms_per_view_" + name] = round(ms / args.steps, 4)
    # decode kernel time per launch (HIP events on the library stream)
    vb = xvbs[0]
    sh = P.stream_handle(streams[0])
    ev = [HipEvent() for _ in range(2)]
    nviews = min(args.steps, len(ccams))
    for name, prec, sh_bytes in (("fp32", P.OCTGS_FP32, 192), ("bf16", P.OCTGS_BF16, 96)):
        t_dec = 0.0
        slots = sel = pairs = 0
        for i in range(nviews):
            c = ccams[i]
            vb.select(de, c, prm)
            ev[0].record(sh)
            vb.decode_explicit(de, c, prec)
            ev[1].record(sh)
            vb.rasterize(c, prm)
            torch.cuda.synchronize()
            t_dec += ev[0].elapsed_ms(ev[1])
            st = vb.stats()
            slots += st["n_slots"]
            sel += st["n_selected"]
            pairs += st["n_pairs"]
        ms = t_dec / nviews
        b = (slots / nviews) * (EXPLICIT_IO_BYTES + sh_bytes + 4.0 / sc.k)
        res["decode_ms_" + name] = round(ms, 4)
        res["decode_gbs_" + name] = round(b / (ms * 1e-3) / 1e9, 1)
        res["decode_hbm_frac_" + name] = round(b / (ms * 1e-3) / 8e12, 4)
        res["mean_selected"] = round(sel / nviews)
        res["mean_gaussians"] = round(slots / nviews)
        res["mean_pairs"] = round(pairs / nviews)
    log(f"Our-3D-GS (explicit, SH degree 3): {res}")
    del xvbs, vb, de
    return res


def skip_path(args, P, S, torch, np, sc, ds, ccams, prm, W, H, vb, timed_fn=None,
              view_dist=(500.0, 10.0, 800.0), n_train=None):
    """Train the anchor-skip predictor on blend weights logged by the plain
    renderer over random views of the same scene, pick its threshold on
    held-out training views (worst view >= 47 dB against full decode), and
    judge it on the zoom-out: PSNR of BF16 + skip against plain FP32."""
    from paper_2403_17898_amd import skip as SK
    t0 = time.time()
    n_train = args.skip_train_views if n_train is None else n_train
    views = S.random_views(n_train + 20, 4, *view_dist, W, H)
    cams = [P.make_camera(c) for c in views]
    train_cams, hold_cams = cams[:-20], cams[-20:]
    # random views can select more anchors than the zoom-out: whole-scene capacities
    vbl = P.ViewBuffers(sc.n, sc.k, W, H, pair_capacity=32 << 20, log_weights=True)
    z, y = SK.collect(vbl, ds, train_cams, prm, tau=1e-2, rows_per_view=4096)
    st = vbl.stats()
    if st["pair_overflow"] or st["sync_error"]:
        raise SystemExit(f"skip data collection flagged: {st}")
    net = SK.SkipNet(seed=1)
    hist = SK.train(net, z, y, epochs=6, batch=16384, lr=2e-3, pos_weight=4.0)
    cands = [-6.0, -5.0, -4.0, -3.0, -2.5, -2.0, -1.5, -1.0, -0.5, 0.0]
    best = SK.choose_threshold(vbl, SK.SkipBuffers(vbl), ds, hold_cams, prm, net, cands, 47.0)
    # hold-out skip fraction at the chosen threshold; under 1 % the path
    # falls back to full decode (no predictor launch)
    thr = best[0] if best else -1e30
    sbl = SK.SkipBuffers(vbl)
    hsel = hkept = 0
    for c in hold_cams:
        vbl.select(ds, c, prm)
        SK.predict(vbl, sbl, ds, c, net, thr)
        hsel += int(vbl.sel_count.item())
        hkept += int(sbl.keep_count.item())
    hold_skip = 1.0 - hkept / max(hsel, 1)
    fallback = hold_skip < 0.01
    del vbl, sbl
    torch.cuda.empty_cache()
    sb = SK.SkipBuffers(vb)
    # judge on the zoom-out: every view against the plain FP32 full decode
    psn, sel, kept = [], 0, 0
    from paper_2403_17898_amd.hip_events import HipEvent
    pe = (HipEvent(), HipEvent())
    sh = P.stream_handle(None)
    pred_ms = 0.0
    for c in ccams:
        vb.render(ds, c, prm, precision=P.OCTGS_FP32)
        ref = vb.rgb.clone()
        # render_skip's steps, with the predictor call timed on its own
        vb.select(ds, c, prm)
        pe[0].record(sh)
        SK.predict(vb, sb, ds, c, net, thr)
        pe[1].record(sh)
        vb.decode(ds, c, P.OCTGS_BF16, idx=sb.keep_idx, count=sb.keep_count)
        vb.rasterize(c, prm)
        pe[1].synchronize()
        pred_ms += pe[0].elapsed_ms(pe[1])
        sel += int(vb.sel_count.item())
        kept += int(sb.keep_count.item())
        if fallback:
            vb.render(ds, c, prm, precision=P.OCTGS_BF16)
        psn.append(SK.psnr(vb.rgb, ref))
    fin = [p for p in psn if math.isfinite(p)]
    res = {"fallback_to_full_decode": fallback, "holdout_skipped_fraction": round(hold_skip, 4),
           "train_views": len(train_cams), "rows": int(z.shape[0]),
           "positive_fraction": round(float(y.mean().item()), 4),
           "loss_per_epoch": [round(h, 4) for h in hist],
           "logit_threshold": thr, "holdout_worst_psnr_db": round(best[1], 2) if best else None,
           "predictor_skipped_fraction": round(1.0 - kept / max(sel, 1), 4),
           "skipped_fraction": 0.0 if fallback else round(1.0 - kept / max(sel, 1), 4),
           "psnr_min_db": round(min(psn), 2), "psnr_mean_db": round(float(np.mean(fin)), 2) if fin else None,
           "train_s": round(time.time() - t0, 1)}
    # predictor call per view: features, the 37-64-64-1 MLP on BF16 MFMA
    # (13,056 FLOP per selected anchor), keep-list compaction
    pms = pred_ms / max(len(ccams), 1)
    res["predict_ms_per_view"] = round(pms, 4)
    res["predict_mfma_tflops"] = round(13056.0 * sel / max(len(ccams), 1) / (pms * 1e-3) / 1e12, 2)
    res["predict_mfma_frac_bf16"] = round(res["predict_mfma_tflops"] / 2500.0, 5)
    log(f"skip predictor: {res}")
    res["_net"], res["_sb"], res["_thr"] = net, sb, thr
    return res


def timed_skip(P, vbs, ds, prm, skip, timed_views, depth):
    """The BF16 + learned-skip path (or its full-decode fallback), timed
    like the other paths with the same frames in flight."""
    from paper_2403_17898_amd import skip as SK
    net, _, thr = skip.pop("_net"), skip.pop("_sb"), skip.pop("_thr")
    fallback = skip["fallback_to_full_decode"]
    sbs = [SK.SkipBuffers(v) for v in vbs[:depth]]

    def one(k, c, s):
        if fallback:
            vbs[k].render(ds, c, prm, precision=P.OCTGS_BF16, stream=s)
        else:
            SK.render_skip(vbs[k], sbs[k], ds, c, prm, net, thr, precision=P.OCTGS_BF16, stream=s)

    return timed_views(one, depth)


def city_path(args, P, S, torch, np, prm, D, streams):
    """The city-scale scene, 4M anchors over 10 levels on 8,000 boxes over
    [-2000, 2000]^2: FPS of the 200-view 3840x2160 zoom-out (20 -> 3000 m)
    with plain FP32 decode, BF16 decode and BF16 + learned skip (the
    predictor trained on random views of this scene), PSNR of BF16 against
    FP32, and the train step of 8 views at 2048x1024."""
    t0 = time.time()
    sc = S.make_config5()
    ccams_c = S.config5_cameras(args.views)
    log(f"city scene: {sc.n} anchors, levels {sc.level_counts()}, generated in "
        f"{time.time() - t0:.1f}s")
    ds = P.DeviceScene.from_scene(sc)
    W, H = ccams_c[0].width, ccams_c[0].height
    cams = [P.make_camera(c) for c in ccams_c]
    vb = P.ViewBuffers(sc.n, sc.k, W, H, pair_capacity=160 << 20)
    per_view = []
    for c in cams:
        vb.render(ds, c, prm, precision=P.OCTGS_FP32)
        st = vb.stats()
        if st["pair_overflow"] or st["sync_error"]:
            raise SystemExit(f"city sizing pass failed: {st}")
        per_view.append(st)
    max_sel = max(s["n_selected"] for s in per_view)
    max_pairs = max(s["n_candidates"] for s in per_view)
    mean = {k: float(np.mean([s[k] for s in per_view]))
            for k in ("n_selected", "n_slots", "n_visible", "n_pairs")}
    del vb
    torch.cuda.empty_cache()
    gcap = max(1, int(max_sel * sc.k * 1.05) + 1024)
    pcap = max(1, int(max_pairs * 1.10) + 4096)
    vbs = [P.ViewBuffers(sc.n, sc.k, W, H, pair_capacity=pcap, gauss_capacity=gcap)
           for _ in range(D)]

    def timed(prec):
        return time_views(args, torch, streams, cams, vbs,
                          lambda k, c, s: vbs[k].render(ds, c, prm, precision=prec, stream=s), D)

    ms32, _ = timed(P.OCTGS_FP32)
    ms16, _ = timed(P.OCTGS_BF16)
    res = {"workload": "city scene: 4M anchors / 10 LOD levels, 200-view zoom-out 20->3000 m, "
                       "3840x2160",
           "n_anchors": sc.n, "views": len(cams),
           "fps_plain_fp32": round(args.steps / (ms32 / 1e3), 2),
           "fps_bf16": round(args.steps / (ms16 / 1e3), 2),
           "mean_selected": round(mean["n_selected"]), "mean_gaussians": round(mean["n_slots"]),
           "mean_visible": round(mean["n_visible"]), "mean_pairs": round(mean["n_pairs"]),
           "max_selected": max_sel, "max_candidate_pairs": max_pairs, "frames_in_flight": D}
    vb = vbs[0]
    psn = []
    for c in cams[::10]:
        vb.render(ds, c, prm, precision=P.OCTGS_FP32)
        ref = vb.rgb.clone()
        vb.render(ds, c, prm, precision=P.OCTGS_BF16)
        mse = torch.mean((vb.rgb - ref) ** 2).item()
        psn.append(float("inf") if mse == 0 else 10 * math.log10(1.0 / mse))
    res["psnr_bf16_vs_fp32_min_db"] = round(min(psn), 2)
    res["psnr_views"] = len(psn)
    log(f"city: FP32 {res['fps_plain_fp32']} FPS, BF16 {res['fps_bf16']} FPS, "
        f"BF16 vs FP32 min PSNR {res['psnr_bf16_vs_fp32_min_db']} dB over {len(psn)} views")
    if not args.no_cpu_baseline:
        # the oracle on 10 evenly spaced views of the 4K zoom-out
        from oracle import oracle as O
        O.build(force=False)
        thr, rho = O.scene_thresholds(sc)
        pick = np.linspace(0, len(ccams_c) - 1, 10).round().astype(int)
        t1 = time.perf_counter()
        for i in pick:
            O.render(sc, ccams_c[i], O.params_array(), thr, rho)
        dt = time.perf_counter() - t1
        res["cpu_baseline"] = {"value": round(len(pick) / dt, 4), "unit": "FPS",
                               "cores": O.num_threads(), "kind": "oracle",
                               "sample": f"10 evenly spaced views, full FP64 path, {dt:.1f} s"}
        log(f"city CPU oracle: {res['cpu_baseline']}")
    if not args.no_skip:
        skip = skip_path(args, P, S, torch, np, sc, ds, cams, prm, W, H, vb,
                         view_dist=(2000.0, 20.0, 3000.0), n_train=args.city_skip_views)
        ms_sk, _ = timed_skip(P, vbs, ds, prm, skip,
                              lambda one, depth: time_views(args, torch, streams, cams, vbs, one,
                                                            depth), D)
        skip["fps"] = round(args.steps / (ms_sk / 1e3), 2)
        res["skip"] = skip
        log(f"city BF16 + learned skip: {skip['fps']} FPS")
    del vbs, vb
    torch.cuda.empty_cache()
    if not args.no_train:
        tv = S.config5_train_views()
        res["train"] = train_step_timing(
            args, P, S, torch, np, sc=sc, views=tv,
            workload="4M anchors / 10 levels, 8 views at 2048x1024, mean-L1, Adam",
            with_full_loss=False)
    del ds
    torch.cuda.empty_cache()
    return res


def train_step_timing(args, P, S, torch, np, sc=None, views=None,
                      workload="500k anchors / 6 levels, 4 views at 1600x1066, mean-L1, Adam",
                      with_full_loss=True, oracle_step=False):
    """Training step (by default of the 500k-anchor, 6-level scene: 4 views
    at 1600x1066): mean-L1 against targets rendered from a copy with feature
    noise sigma = 0.05, gradients through compositing, projection and the
    anchor MLPs, then Adam on every trainable array."""
    t0 = time.time()
    if sc is None:
        sc = S.make_config3()
        views = S.config3_views()
    tgt_scene = S.perturbed_copy(sc, 0.05, seed=3)
    log(f"train scene: {sc.n} anchors, levels {sc.level_counts()}, ready in "
        f"{time.time() - t0:.1f}s")
    ds = P.DeviceScene.from_scene(sc)
    dt = P.DeviceScene.from_scene(tgt_scene)
    cams = [P.make_camera(c) for c in views]
    W, H = views[0].width, views[0].height
    prm = P.raster_params(train=True)
    vb = P.ViewBuffers(sc.n, sc.k, W, H, pair_capacity=16 << 20)
    targets, max_sel, max_pairs = [], 0, 0
    for c in cams:
        vb.render(dt, c, prm)
        targets.append(vb.rgb.clone())
        vb.render(ds, c, prm)
        st = vb.stats()
        max_sel, max_pairs = max(max_sel, st["n_selected"]), max(max_pairs, st["n_candidates"])
    del vb
    # views in flight, one buffer set and stream each (up to --inflight)
    nv = len(cams)
    mv = P.MultiViewBackward(ds, W, H, nv, pair_capacity=int(max_pairs * 1.2) + 4096,
                             gauss_capacity=int(max_sel * sc.k * 1.2) + 1024,
                             inflight=args.inflight)
    nbuf = mv.nbuf
    grads = P.SceneGrads(ds)
    params = P.trainable(ds)
    gnames = list(P.render.PARAM_NAMES) + sorted(ds.mlp)
    gl = grads.all()
    gtens = [gl[n] for n in gnames]
    mom = [(torch.zeros_like(p), torch.zeros_like(p)) for p in params]
    adam = P.AdamMany(params, gtens, mom)
    losses = mv.losses  # one slot per view
    scale = 1.0 / (len(cams) * 3 * H * W)
    state = {"step": 0}
    dstats = P.DensifyStats(sc.n, sc.k)

    def step(timer=None, full=False):
        """full: the paper's loss for the Scaffold-GS model, 0.8 L1 +
        0.2 (1 - SSIM) averaged over the views, plus 0.01 sum Prod(s) over
        each view's rendered Gaussians; otherwise mean L1."""
        mv.run(ds, cams, targets, prm, grads, l1_scale=scale, full=full,
               dstats=dstats if full else None)
        if timer is not None:
            timer.record()
        state["step"] += 1
        adam.step(1e-3, state["step"])

    def timed_steps(full):
        for _ in range(3):
            step(full=full)
        torch.cuda.synchronize()
        first = losses.sum().item()
        n = args.train_steps
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
               torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for i in range(n):
            ev[i][0].record()
            step(ev[i][1], full)
            ev[i][2].record()
        torch.cuda.synchronize()
        tot = sorted(a.elapsed_time(c) for a, b, c in ev)
        adam = sorted(b.elapsed_time(c) for a, b, c in ev)
        return tot[len(tot) // 2], adam[len(adam) // 2], first, losses.sum().item()

    ms, adam_ms, first_loss, last_loss = timed_steps(False)
    mv.check()  # no view of any step overflowed, hit a wait bound or was truncated
    cpu_step = None
    if oracle_step:
        # the oracle's step on the same views and targets: FP64 forward and
        # analytic backward through compositing, projection and decode
        from oracle import oracle as O
        O.build(force=False)
        thr, rho = O.scene_thresholds(sc)
        prm_o = O.params_array()
        tg = [t.double().cpu().numpy() for t in targets]
        t1 = time.perf_counter()
        for v, t_img in zip(views, tg):
            fwd = O.render(sc, v, prm_o, thr, rho)
            d = np.sign(fwd["img"] - t_img) / (len(views) * 3 * H * W)  # mean-L1 gradient
            O.render_backward(sc, v, prm_o, d, fwd=fwd)
        dt = time.perf_counter() - t1
        cpu_step = {"value": round(dt * 1e3, 1), "unit": "ms/step", "cores": O.num_threads(),
                    "kind": "oracle", "sample": f"one step: {len(views)} views, FP64 forward and "
                                                f"backward (no optimiser update)"}
    res = {"workload": workload,
           "n_anchors": sc.n, "ms_per_step": round(ms, 3), "adam_ms": round(adam_ms, 3),
           "steps_timed": args.train_steps, "loss_first": round(first_loss, 6),
           "loss_last": round(last_loss, 6), "max_selected": max_sel, "max_pairs": max_pairs,
           "views_in_flight": nbuf}
    if cpu_step is not None:
        res["cpu_oracle_step"] = cpu_step
    if not with_full_loss:
        log(f"train step: {res}")
        return res
    msf, _, ff, fl = timed_steps(True)
    mv.check()
    # densification decisions of the interval (every T = 100 iterations)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dstats.decide(ds, max(1, state["step"] * nv))
    e1.record()
    torch.cuda.synchronize()
    res["full_loss"] = {"loss": "0.8 L1 + 0.2 (1 - SSIM) + 0.01 sum Prod(s), with the "
                                "densification statistics accumulated per view",
                        "ms_per_step": round(msf, 3), "loss_first": round(ff, 6),
                        "loss_last": round(fl, 6),
                        "densify_decide_ms": round(e0.elapsed_time(e1) / 5, 4),
                        "densify_counts": dstats.counts.cpu().numpy().tolist()}
    log(f"train step: {res}")
    return res


if __name__ == "__main__":
    main()
