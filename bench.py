#!/usr/bin/env python3
"""Benchmark of the Octree-GS render path on one MI355X.

Workload (the large synthetic street scene): 1M anchors over 8 octree levels
voxelised from 20M points on 2,000 boxes over a [-500, 500]^2 ground plane,
feature dim 32, k = 10, MLP width 64; a 200-camera zoom-out from 10 m to
800 m altitude at 1920x1080, 60 degree FOV.  One step = one view through the
whole path: anchor selection (Eq. 7), decode (Eq. 3-4), projection, tile
binning, depth ordering and compositing (Eq. 2).  A step is one pass over the
whole 200-view trajectory; --steps passes are timed after --warmup untimed
ones, so value = views / s over steps x 200 views, and every per-view figure
of the output is taken over the same 200 views.  The scene and cameras are
resident before timing starts.

Prints one JSON line.  value = frames per second of the fast path (BF16
decode on MFMA, plus the learned anchor skip unless it falls back to full
decode); the plain FP32 path is timed the same way on the same views and
reported beside it, with the PSNR of the fast path against it.  Views are
independent, so --inflight views are rendered at once on separate streams
with separate buffers; the rate with one view in flight is reported beside
it.  The city-scale scene (4M anchors, 3840x2160, and its 8-view training
step) is measured under the "city" key unless --no-city.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "FPS @1080p + train-step ms, BF16+learned-skip vs plain FP32 at >=45 dB PSNR"
CLOCK_HZ = 2.4e9  # MI355X peak engine clock
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published FP32 vector peak
BF16_MFMA_PEAK_TFLOPS = 2500.0    # MI355X dense BF16 matrix peak
FLOP_PER_BLEND = 21.0
COMPOSITE_PMC = os.path.join(ROOT, "profiles", "composite_street1080p_hbm_bytes.txt")
RASTER_PMC = os.path.join(ROOT, "profiles", "raster_street1080p_hbm_bytes.txt")
RASTER_SOURCES = ("paper_2403_17898_amd/csrc/raster.hip", "paper_2403_17898_amd/csrc/sort.hip")
COMPOSITE_BWD_PMC = os.path.join(ROOT, "profiles", "composite_bwd_train_c3_hbm_bytes.txt")
BWD_SOURCES = ("paper_2403_17898_amd/csrc/raster_bwd.hip",)

# The paper's own rendering rates, for context only: another scene, another
# resolution and another GPU (Tab. matrix_traj, Sec. V-B: MatrixCity
# trajectories T1-T3 at "2k", one NVIDIA A100 80G).
PAPER_CONTEXT = {
    "source": "Octree-GS, Tab. matrix_traj (Sec. V-B)",
    "hardware": "NVIDIA A100 80G",
    "workload": "MatrixCity novel-view trajectories T1, T2, T3 at 2k resolution (trained models)",
    "fps_our_scaffold_gs": [40.91, 35.17, 40.31],
    "fps_our_3d_gs": [57.08, 56.85, 56.07],
    "fps_scaffold_gs_t1": 6.69,
    "fps_3d_gs_t1": 13.81,
    "note": "not comparable: different scene, resolution and hardware",
}


def sha256_of(rel: str) -> str:
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def read_summary(path: str):
    """`key: value` lines of a committed profile summary, or None."""
    try:
        with open(path) as f:
            text = f.read()
    except OSError:
        return None
    return dict((a.strip(), b.strip()) for a, b in
                (line.split(":", 1) for line in text.splitlines() if ":" in line))


def summary_valid(fields, sources, views: int) -> bool:
    """The summary was taken on the current source of every listed file and
    on the same views (one pass over the trajectory)."""
    if not fields:
        return False
    for rel in sources:
        if fields.get("source_sha256 " + os.path.basename(rel)) != sha256_of(rel):
            return False
    return fields.get("views") == str(views)


def composite_traffic(views: int):
    """HBM bytes per composite launch from the committed FETCH_SIZE /
    WRITE_SIZE counter summary, or None when that summary is missing, was
    taken from a different version of the kernel source or on another view
    set."""
    f = read_summary(COMPOSITE_PMC)
    if not summary_valid(f, RASTER_SOURCES, views):
        return None
    try:
        return int(float(f["hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def raster_traffic(views: int):
    """HBM bytes per view of the whole rasterizer forward (every kernel of
    octgs_rasterize_fwd) from the committed counter summary, or None (as
    composite_traffic)."""
    f = read_summary(RASTER_PMC)
    if not summary_valid(f, RASTER_SOURCES, views):
        return None
    try:
        return int(float(f["hbm_bytes_per_view"]))
    except (KeyError, ValueError):
        return None


def composite_bwd_traffic():
    """HBM bytes per launch of the compositing backward on the training
    views from the committed FETCH_SIZE / WRITE_SIZE summary, or None when
    it is missing or was taken from another version of the kernel source."""
    f = read_summary(COMPOSITE_BWD_PMC)
    if not f:
        return None
    for rel in BWD_SOURCES:
        if f.get("source_sha256 " + os.path.basename(rel)) != sha256_of(rel):
            return None
    try:
        return int(float(f["hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="views timed per path: a stride through the trajectory")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--views", type=int, default=200, help="trajectory length")
    ap.add_argument("--inflight", type=int, default=4,
                    help="views in flight at once (one stream and buffer set each)")
    ap.add_argument("--cpu-views", type=int, default=40,
                    help="timed views the CPU oracle renders (evenly spaced among them)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="skip the PSNR sweep (profiling runs)")
    ap.add_argument("--stages-only", action="store_true",
                    help="profiling runs: only the sizing pass and the per-stage timing loop "
                         "(one view at a time); no throughput passes, no line printed")
    ap.add_argument("--predict-stages", action="store_true",
                    help="with --stages-only: also run the skip predictor (untrained weights) "
                         "on each view after its render, for kernel profiles")
    ap.add_argument("--train-only", action="store_true",
                    help="profiling runs: only the training-step timing (use --inflight 1 "
                         "for uncontended launches); no line printed")
    ap.add_argument("--no-train", action="store_true", help="skip the training-step timing")
    ap.add_argument("--no-skip", action="store_true", help="skip the learned-skip study")
    ap.add_argument("--no-3dgs", action="store_true",
                    help="skip the explicit-Gaussian (3D-GS instance) measurement")
    ap.add_argument("--skip-train-views", type=int, default=1000)
    ap.add_argument("--train-steps", type=int, default=20)
    ap.add_argument("--no-city", action="store_true",
                    help="skip the city-scale scene (4M anchors / 10 levels): the 3840x2160 "
                         "zoom-out and the 8-view 2048x1024 train step")
    ap.add_argument("--city-skip", action="store_true",
                    help="also train and time the learned skip on the city scene")
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


def rate(args, ms: float, nviews: int) -> float:
    """Views per second of args.steps timed passes over nviews views."""
    return args.steps * nviews / (ms / 1e3)


def time_views(args, torch, streams, views, bufs, render_one, depth):
    """(event ms, wall s) of args.steps passes over the whole trajectory
    `views` after args.warmup untimed passes (a step is one pass over every
    view); the i-th render of a pass runs on stream i % depth with buffers
    bufs[i % depth].  Every frame's device-detected conditions are checked
    after the timed passes."""
    stream = streams[0]

    def run(passes):
        i = 0
        for _ in range(passes):
            for v in views:
                k = i % depth
                # every frame's overflow / look-back / truncation bits land in
                # its buffer set's status word, checked after the loop
                render_one(k, v, streams[k])
                i += 1
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

    if args.train_only:
        res = train_step_timing(args, P, S, torch, np, with_full_loss=False)
        log(f"train step only: {res}")
        return

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
    # a timed pass renders every view of the trajectory in order; every
    # per-view figure below is taken over the same views
    order = list(range(len(cams)))
    tset = order
    nv = len(order)

    # ---- sizing pass (untimed) over the timed views: selected anchors and pairs ----
    vb = P.ViewBuffers(sc.n, sc.k, W, H, pair_capacity=48 << 20)
    plain_st, blend_st = {}, {}
    for i in tset:
        for c, store in ((ccams[i], plain_st), (bcams[i], blend_st)):
            vb.render(ds, c, prm, precision=P.OCTGS_FP32)
            st = vb.stats()
            if st["pair_overflow"] or st["sync_error"]:
                raise SystemExit(f"sizing pass failed: {st}")
            store[i] = st
    allst = list(plain_st.values()) + list(blend_st.values())
    max_sel = max(s_["n_selected"] for s_ in allst)
    max_pairs = max(s_["n_candidates"] for s_ in allst)
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
    log(f"timed: {args.steps} passes over the {nv} views; max selected {max_sel}, max "
        f"candidate pairs {max_pairs}; gcap {gcap}, pcap {pcap}; {D} frames in flight")

    if args.stages_only:
        stage_loop(args, P, L, torch, np, sc, cams, ccams, ds, prm, vb, stream, order)
        return

    def timed_views(render_one, depth, views=None, bufs=None):
        """ms for args.steps views (after args.warmup), view i on stream i % depth."""
        return time_views(args, torch, streams, ccams if views is None else views,
                          vbs if bufs is None else bufs, render_one, depth)

    def timed(prec, depth=D, views=None, params=prm):
        return timed_views(lambda k, c, s_: vbs[k].render(ds, c, params, precision=prec, stream=s_,
                                                          keep_last=False),
                           depth, views)

    ms32, wall32 = timed(P.OCTGS_FP32)
    ms16, wall16 = timed(P.OCTGS_BF16)
    # a frame alone on the GPU: tiles ordered longest-first within each XCD
    prm_one = P.raster_params(tile_order=True)
    ms32_1, _ = timed(P.OCTGS_FP32, 1, params=prm_one)
    ms16_1, _ = timed(P.OCTGS_BF16, 1, params=prm_one)
    fps32 = rate(args, ms32, nv)
    fps16 = rate(args, ms16, nv)
    single = {"fp32": round(rate(args, ms32_1, nv), 2), "bf16": round(rate(args, ms16_1, nv), 2)}
    log(f"plain FP32: {1e3 / fps32:.4f} ms/view ({fps32:.1f} FPS); "
        f"BF16: {1e3 / fps16:.4f} ms/view ({fps16:.1f} FPS); one frame in flight: {single}")
    msb, _ = timed(P.OCTGS_BF16, views=bcams)
    blend = {"fps_bf16": round(rate(args, msb, nv), 2), "ms_per_view": round(1e3 / rate(args, msb, nv), 4),
             "mean_selected": round(float(np.mean([blend_st[i]["n_selected"] for i in order]))),
             "mean_pairs": round(float(np.mean([blend_st[i]["n_pairs"] for i in order])))}
    log(f"LOD transition blending, BF16: {blend}")

    # ---- Our-3D-GS: explicit Gaussians with SH colour on the same anchors ----
    our3d = None
    if not args.no_3dgs:
        our3d = explicit_path(args, P, S, torch, np, sc, ccams, prm, W, H, D, streams,
                              timed_views, order)
        torch.cuda.empty_cache()

    # ---- learned anchor skip: trained on logged blend weights of views of the
    # zoom-out's family, against rules on one input and a perfect predictor ----
    skip = None
    if not args.no_skip:
        skip = skip_study(args, P, S, torch, np, sc, ds, ccams, prm, W, H, vbs, D, streams,
                          order, fps32)

    # ---- per-stage timing with HIP events on the library's stream ----
    avg, mean, view_ms = stage_loop(args, P, L, torch, np, sc, cams, ccams, ds, prm, vb, stream,
                                    order)
    nviews = len(order)
    log("per-stage ms/view: " + ", ".join(f"{k} {v:.4f}" for k, v in avg.items()))
    log(f"mean per view: selected {mean['selected']:.0f}, Gaussians {mean['slots']:.0f}, "
        f"visible {mean['visible']:.0f}, pairs {mean['pairs']:.0f} "
        f"(of {mean['candidates']:.0f} rectangle candidates)")
    # each view alone on the GPU (the loop above) against the camera altitude
    vm = np.array(view_ms)
    alts = np.array([float(cams[order[i]].C[2]) for i in range(nviews)])
    srt = np.argsort(alts, kind="stable")
    edges = np.linspace(0, nviews, min(10, nviews) + 1).round().astype(int)
    per_view = {"ms_mean": round(float(vm.mean()), 4), "ms_max": round(float(vm.max()), 4),
                "slowest_view": int(order[int(vm.argmax())]),
                "slowest_altitude_m": round(float(alts[vm.argmax()]), 1),
                "min_fps": round(1e3 / float(vm.max()), 1),
                "altitude_m_vs_ms": [[round(float(alts[srt[a:b]].mean()), 1),
                                      round(float(vm[srt[a:b]].mean()), 4)]
                                     for a, b in zip(edges[:-1], edges[1:]) if b > a]}
    log(f"each view alone: {per_view}")
    # decode on MFMA: first layers 36 -> 3 x W, second layers W -> 11 k (k
    # opacities, 3k colours, 7k covariance terms), 2 FLOP per multiply-add
    dec_flop = 2.0 * (36 * 3 * sc.width + sc.width * 11 * sc.k) * mean["selected"]
    decode_mfma = {"flop_per_anchor": int(dec_flop / max(mean["selected"], 1)),
                   "tflops": round(dec_flop / (avg["decode"] * 1e-3) / 1e12, 2)}
    decode_mfma["frac_bf16"] = round(decode_mfma["tflops"] / BF16_MFMA_PEAK_TFLOPS, 5)
    log(f"decode (BF16, per call incl. the weight-fragment kernel): {decode_mfma}")

    # The dominant kernel, compositing, is bound by vector ALU work: per
    # pixel and Gaussian blended (Eq. 2) it evaluates the 2D Gaussian,
    # alpha, the colour update and T, 21 FLOP counting exp as one.  Units per
    # launch = sum over pixels of the entries each consumed (the `last`
    # output of a counting pass; the timed launches leave it out).  Its
    # algorithmic HBM bytes per launch are reported beside.
    npix = W * H
    ntiles = ((W + 15) // 16) * ((H + 15) // 16)
    flop = FLOP_PER_BLEND * mean["blends"]
    ach = flop / (avg["composite"] * 1e-3) / 1e12
    # unique bytes: list entries 4 B per pair, the projected record 36 B per
    # visible Gaussian, tile ranges 8 B, and 16 B written per pixel (colour
    # and T_final)
    alg_bytes = 4.0 * mean["pairs"] + 36.0 * mean["visible"] + 8.0 * ntiles + 16.0 * npix
    roofline = {"kernel": "composite", "bound": "alu", "achieved": round(ach, 2),
                "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / FP32_VECTOR_PEAK_TFLOPS, 4),
                "traffic": composite_traffic(nv),
                "algorithmic_bytes": round(alg_bytes),
                "hbm_gbs": round(alg_bytes / (avg["composite"] * 1e-3) / 1e9, 1),
                "blends_per_launch": round(mean["blends"]),
                "launch_ms": round(avg["composite"], 5),
                "stage_ms": {k: round(v, 4) for k, v in avg.items()}}
    # the whole rasterizer forward: HBM bytes per view by counter (the
    # committed summary of this view set) over its measured stage time
    raster_ms = sum(avg[k] for k in L.RASTER_STAGE_NAMES)
    rbytes = raster_traffic(nv)
    raster_hbm = {"ms_per_view": round(raster_ms, 4), "hbm_bytes_per_view": rbytes,
                  "gbs": None if rbytes is None else round(rbytes / (raster_ms * 1e-3) / 1e9, 1),
                  "peak_gbs": HBM_PEAK_GBS,
                  "frac": None if rbytes is None else round(rbytes / (raster_ms * 1e-3) / 1e9 /
                                                            HBM_PEAK_GBS, 4)}
    log(f"rasterizer HBM: {raster_hbm}")

    # ---- quality: BF16 path vs plain FP32, every view of the trajectory ----
    psnrs = []
    if not args.quick:
        for c in ccams:
            vb.render(ds, c, prm, precision=P.OCTGS_FP32)
            ref = vb.rgb.clone()
            vb.render(ds, c, prm, precision=P.OCTGS_BF16)
            mse = torch.mean((vb.rgb - ref) ** 2).item()
            psnrs.append(float("inf") if mse == 0 else 10 * math.log10(1.0 / mse))
        fin = [p_ for p_ in psnrs if math.isfinite(p_)]
        log(f"PSNR BF16 vs FP32: min {min(psnrs):.2f} dB, mean {np.mean(fin) if fin else float('inf'):.2f} dB")

    # ---- CPU baseline: the oracle on the timed views, and the GPU paths
    # against it (max-abs and PSNR of FP32 and BF16 images) ----
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, P, S, torch, np, sc, cams, ccams, ds, prm, vb, tset)

    train = None if args.no_train else train_step_timing(args, P, S, torch, np,
                                                         oracle_step=not args.no_cpu_baseline)
    del vbs, vb
    torch.cuda.empty_cache()
    city = None if args.no_city else city_path(args, P, S, torch, np, prm, D, streams)

    use_skip = skip is not None and not skip["fallback_to_full_decode"]
    value = skip["fps"] if use_skip else fps16
    ms_value = nv * 1e3 / value  # one step = one pass over the trajectory
    copy_gbs = measured_copy_gbs(torch)
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
                   "step": f"one pass over the {nv} views of the trajectory",
                   "path": ("BF16 decode" if skip is None else
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
        "ms_per_view": round(1e3 / value, 4),
        "ms_per_view_plain_fp32": round(1e3 / fps32, 4),
        "speedup_vs_plain": round(value / fps32, 4),
        "psnr_vs_plain_min_db": (skip["psnr_min_db"] if use_skip else
                                 (round(min(psnrs), 2) if psnrs else None)),
        "psnr_vs_plain_mean_db": (skip["psnr_mean_db"] if use_skip else
                                  (round(float(np.mean([p_ for p_ in psnrs if math.isfinite(p_)])), 2)
                                   if psnrs and any(math.isfinite(p_) for p_ in psnrs) else None)),
        "psnr_bf16_no_skip_min_db": round(min(psnrs), 2) if psnrs else None,
        "psnr_views": len(psnrs),
        "skip": skip,
        "our_3dgs": our3d,
        "wall_s_timed": round(wall16, 3),
        "train_step_ms": train["ms_per_step"] if train else None,
        "train": train,
        "roofline": roofline,
        "raster_hbm": raster_hbm,
        "measured_copy_gbs": copy_gbs,
        "each_view_alone": per_view,
        "decode_mfma": decode_mfma,
        "cpu_baseline": cpu,
        "paper_context": PAPER_CONTEXT,
    }
    if city is not None:
        out["city"] = city
    print(json.dumps(_finite(out), allow_nan=False), flush=True)


def measured_copy_gbs(torch) -> float:
    """Attainable HBM rate for context: a plain 256 MiB device-to-device copy
    (read + write bytes over the HIP-event time, best of 5)."""
    src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    best = float("inf")
    for _ in range(6):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    del src, dst
    torch.cuda.empty_cache()
    return round(2 * (256 << 20) / (best * 1e-3) / 1e9, 1)


def stage_loop(args, P, L, torch, np, sc, cams, ccams, ds, prm, vb, stream, order):
    """Each view alone on the GPU, BF16 decode, with HIP events around every
    stage on the library's stream: (ms per stage per view, mean per-view
    counts, per-view ms)."""
    from paper_2403_17898_amd.hip_events import HipEvent
    names = ["select", "decode"] + list(L.RASTER_STAGE_NAMES)
    tot = {k: 0.0 for k in names}
    nviews = len(order)
    sums = dict(selected=0, slots=0, visible=0, pairs=0, candidates=0, blends=0)
    view_ms = []
    ev = [HipEvent() for _ in range(4 + 2 * L.OCTGS_RASTER_STAGES)]
    sh = P.stream_handle(stream)
    if args.predict_stages:
        from paper_2403_17898_amd import skip as SK
        net, sb = SK.SkipNet(seed=1), SK.SkipBuffers(vb)
    # the timed composites leave out the per-pixel entry count (no backward
    # follows them); a pass before the timed loop, so that the loop's
    # dispatches are the last of each kernel, renders the same views with
    # it to count the blends
    for i in range(nviews):
        vb.render(ds, ccams[order[i]], prm, precision=P.OCTGS_BF16, keep_last=True)
        sums["blends"] += int(vb.last.sum(dtype=torch.int64).item())
    for i in range(nviews):
        c = ccams[order[i]]
        ev[0].record(sh)
        vb.select(ds, c, prm)
        ev[1].record(sh)
        ev[2].record(sh)
        vb.decode(ds, c, P.OCTGS_BF16)
        ev[3].record(sh)
        vb.rasterize(c, prm, stage_events=ev[4:], keep_last=False)
        torch.cuda.synchronize()
        vms = ev[0].elapsed_ms(ev[1]) + ev[2].elapsed_ms(ev[3])
        tot["select"] += ev[0].elapsed_ms(ev[1])
        tot["decode"] += ev[2].elapsed_ms(ev[3])
        for s_i, nm in enumerate(L.RASTER_STAGE_NAMES):
            tot[nm] += ev[4 + 2 * s_i].elapsed_ms(ev[5 + 2 * s_i])
            vms += ev[4 + 2 * s_i].elapsed_ms(ev[5 + 2 * s_i])
        view_ms.append(vms)
        if args.predict_stages:
            SK.predict(vb, sb, ds, c, net, 0.0, stream=stream)
            torch.cuda.synchronize()
        st = vb.stats()
        sums["selected"] += st["n_selected"]
        sums["slots"] += st["n_slots"]
        sums["visible"] += st["n_visible"]
        sums["pairs"] += st["n_pairs"]
        sums["candidates"] += st["n_candidates"]
    avg = {k: v / nviews for k, v in tot.items()}  # ms per launch
    mean = {k: v / nviews for k, v in sums.items()}
    return avg, mean, view_ms


def cpu_baseline(args, P, S, torch, np, sc, cams, ccams, ds, prm, vb, tset):
    """The oracle (full FP64 select, decode, rasterize) on up to --cpu-views
    of the timed views, all host threads; the oracle on one core on three of
    them; and each GPU path (plain FP32, BF16) against the oracle's images on
    those views: max abs difference and PSNR."""
    from oracle import oracle as O
    O.build(force=False)
    thr, rho = O.scene_thresholds(sc)
    pick = [tset[j] for j in np.linspace(0, len(tset) - 1, min(args.cpu_views, len(tset)))
            .round().astype(int)]
    dt = 0.0
    acc = {"fp32": [], "bf16": []}
    for i in pick:
        t1 = time.perf_counter()
        ref = O.render(sc, cams[i], O.params_array(), thr, rho)
        dt += time.perf_counter() - t1
        for name, prec in (("fp32", P.OCTGS_FP32), ("bf16", P.OCTGS_BF16)):
            vb.render(ds, ccams[i], prm, precision=prec)
            img = vb.rgb.double().cpu().numpy()
            err = float(np.abs(img - ref["img"]).max())
            mse = float(np.mean((img - ref["img"]) ** 2))
            acc[name].append((err, float("inf") if mse == 0 else 10 * math.log10(1.0 / mse)))
    cpu = {"value": round(len(pick) / dt, 4), "unit": "FPS", "cores": O.num_threads(),
           "kind": "oracle",
           "sample": f"{len(pick)} of the timed views (trajectory views {pick[0]}..{pick[-1]}), "
                     f"full FP64 select+decode+rasterize, {dt:.1f} s"}
    nthr = O.num_threads()
    O.set_num_threads(1)
    pick1 = [pick[0], pick[len(pick) // 2], pick[-1]]
    t1 = time.perf_counter()
    for i in pick1:
        O.render(sc, cams[i], O.params_array(), thr, rho)
    dt1 = time.perf_counter() - t1
    O.set_num_threads(nthr)
    cpu["one_core"] = {"value": round(len(pick1) / dt1, 4), "unit": "FPS", "cores": 1,
                       "sample": f"trajectory views {pick1}, {dt1:.1f} s"}
    cpu["cpu_model"] = cpu_model()
    cpu["gpu_vs_oracle"] = {
        name: {"views": len(v), "max_abs": max(e for e, _ in v),
               "psnr_min_db": round(min(p_ for _, p_ in v), 2),
               "psnr_mean_db": round(float(np.mean([p_ for _, p_ in v if math.isfinite(p_)])), 2)}
        for name, v in acc.items()}
    log(f"CPU oracle: {cpu}")
    return cpu


# per decoded explicit Gaussian: mean, log-scale, rotation and opacity
# logit read (44 B), the SH row (48 values, FP32 or BF16), the 56-byte
# record written, and the anchor index (4 B per k slots)
EXPLICIT_IO_BYTES = 44 + 56


def explicit_path(args, P, S, torch, np, sc, ccams, prm, W, H, D, streams, timed_views, order):
    """FPS of the 3D-GS instance (explicit degree-3 Gaussians on the config
    anchors) with FP32 and BF16 SH coefficients, and the decode kernel's
    achieved HBM rate, over the timed views."""
    from paper_2403_17898_amd.hip_events import HipEvent
    t0 = time.time()
    ex = S.make_explicit(sc, sh_degree=3)
    de = P.DeviceExplicit.from_scene(ex)
    del ex
    log(f"explicit scene: degree-3 SH, generated and uploaded in {time.time() - t0:.1f}s")
    vb = P.ViewBuffers(sc.n, sc.k, W, H, pair_capacity=64 << 20)
    max_sel = max_pairs = 0
    for i in sorted(set(order)):
        c = ccams[i]
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
                                                                   stream=s, keep_last=False),
                            D, bufs=xvbs)
        res["fps_" + name] = round(rate(args, ms, len(ccams)), 2)
        res["ms_per_view_" + name] = round(1e3 / rate(args, ms, len(ccams)), 4)
    # decode kernel time per launch (HIP events on the library stream)
    vb = xvbs[0]
    sh = P.stream_handle(streams[0])
    ev = [HipEvent() for _ in range(2)]
    nviews = len(order)
    for name, prec, sh_bytes in (("fp32", P.OCTGS_FP32, 192), ("bf16", P.OCTGS_BF16, 96)):
        t_dec = 0.0
        slots = sel = pairs = 0
        for i in range(nviews):
            c = ccams[order[i]]
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


SKIP_TAU_W = 1e-2          # label: the anchor's logged blend weight exceeds this
SKIP_MIN_HOLDOUT_DB = 47.0  # threshold choice: worst held-out view at or above this
SKIP_CANDIDATES = [-6.0, -5.0, -4.0, -3.0, -2.5, -2.0, -1.5, -1.0, -0.5, 0.0, 0.5, 1.0]


def skip_study(args, P, S, torch, np, sc, ds, ccams, prm, W, H, vbs, D, streams, order, fps32,
               h_range=(10.0, 800.0), n_train=None):
    """The learned anchor skip against what it can be compared with, on the
    timed views of the zoom-out:
      - the predictor on all its inputs, trained on the blend weights the
        plain renderer logs over views of the zoom-out's family (random
        altitude, jittered position and aim), its logit threshold the most
        aggressive one whose worst held-out family view stays >= 47 dB
        against full decode;
      - the same network and training restricted to one input, the log
        distance or the level (rules on distance alone, level alone);
      - a perfect predictor of the label: keep exactly the anchors whose
        logged weight on that very view exceeds tau (the ceiling of any
        predictor of this label).
    For each: skipped share of selected anchors, pairs removed, PSNR of the
    BF16 + skip render against plain FP32 full decode, and FPS.  The learned
    path falls back to full decode when it skips under 1 % of the held-out
    family views' anchors, or when it is not faster than full decode."""
    from paper_2403_17898_amd import skip as SK
    t0 = time.time()
    n_train = args.skip_train_views if n_train is None else n_train
    fam = [P.make_camera(c) for c in S.trajectory_family_views(n_train + 20, 4, h_range[0],
                                                                 h_range[1], W, H)]
    train_cams, hold_cams = fam[:-20], fam[-20:]
    # family views can select more anchors than the zoom-out: whole-scene capacities
    vbl = P.ViewBuffers(sc.n, sc.k, W, H, pair_capacity=64 << 20, log_weights=True)
    z, y = SK.collect(vbl, ds, train_cams, prm, tau=SKIP_TAU_W, rows_per_view=4096)
    vbl.check_status("skip training views")
    sbl = SK.SkipBuffers(vbl)
    tset = sorted(set(order))
    vb0 = vbs[0]
    sb0 = SK.SkipBuffers(vb0)
    refs, full_pairs = {}, {}
    for i in tset:
        vb0.render(ds, ccams[i], prm, precision=P.OCTGS_FP32)
        refs[i] = vb0.rgb.clone()
        full_pairs[i] = vb0.stats()["n_pairs"]
    sbs = [SK.SkipBuffers(v) for v in vbs[:D]]

    def evaluate(render_view, timed_one):
        """PSNR / skipped / pairs on the timed views, then the timed pass."""
        psn, sel, kept, pairs = [], 0, 0, 0
        for i in tset:
            render_view(i)
            psn.append(SK.psnr(vb0.rgb, refs[i]))
            sel += int(vb0.sel_count.item())
            kept += int(vb0.gauss_count.item()) // sc.k
            pairs += vb0.stats()["n_pairs"]
        ms, _ = time_views(args, torch, streams, ccams, vbs, timed_one, D)
        fin = [p_ for p_ in psn if math.isfinite(p_)]
        return {"skipped_fraction": round(1.0 - kept / max(sel, 1), 4),
                "pairs_removed_fraction": round(1.0 - pairs / max(sum(full_pairs.values()), 1), 4),
                "psnr_min_db": round(min(psn), 2),
                "psnr_mean_db": round(float(np.mean(fin)), 2) if fin else None,
                "fps": round(rate(args, ms, len(ccams)), 2),
                "ms_per_view": round(1e3 / rate(args, ms, len(ccams)), 4),
                "fps_ratio_vs_plain_fp32": round(rate(args, ms, len(ccams)) / fps32, 4)}

    rules = {}
    nets = {}
    for name, inputs in (("learned", None), ("distance_only", [SK.Z_LOG_DISTANCE]),
                         ("level_only", [SK.Z_LEVEL])):
        net = SK.SkipNet(seed=1, inputs=inputs)
        hist = SK.train(net, z, y, epochs=6, batch=16384, lr=2e-3, pos_weight=4.0)
        best = SK.choose_threshold(vbl, sbl, ds, hold_cams, prm, net, SKIP_CANDIDATES,
                                   SKIP_MIN_HOLDOUT_DB)
        thr = best[0] if best else -1e30
        hsel = hkept = 0
        for c in hold_cams:
            vbl.select(ds, c, prm)
            SK.predict(vbl, sbl, ds, c, net, thr)
            hsel += int(vbl.sel_count.item())
            hkept += int(sbl.keep_count.item())

        def view(i, net=net, thr=thr):
            SK.render_skip(vb0, sb0, ds, ccams[i], prm, net, thr, precision=P.OCTGS_BF16)

        def one(k, c, s_, net=net, thr=thr):
            SK.render_skip(vbs[k], sbs[k], ds, c, prm, net, thr, precision=P.OCTGS_BF16,
                           stream=s_, keep_last=False)

        r = {"logit_threshold": thr, "holdout_worst_psnr_db": round(best[1], 2) if best else None,
             "holdout_skipped_fraction": round(1.0 - hkept / max(hsel, 1), 4),
             "loss_per_epoch": [round(h, 4) for h in hist]}
        r.update(evaluate(view, one))
        rules[name] = r
        nets[name] = (net, thr)
        log(f"skip rule {name}: {r}")

    # the ceiling: a perfect predictor of the label on each timed view
    keep = {}
    for i, kc in zip(tset, SK.weight_keep_lists(vbl, ds, [ccams[i] for i in tset], prm,
                                                 SKIP_TAU_W)):
        keep[i] = kc
    del vbl, sbl
    torch.cuda.empty_cache()
    kv = [None] * len(ccams)
    for i in tset:
        kv[i] = (ccams[i], i)

    def ceil_view(i):
        vb0.select(ds, ccams[i], prm)
        vb0.decode(ds, ccams[i], P.OCTGS_BF16, idx=keep[i][0], count=keep[i][1])
        vb0.rasterize(ccams[i], prm)

    def ceil_one(k, v, s_):
        c, i = v
        vbs[k].select(ds, c, prm, stream=s_)
        vbs[k].decode(ds, c, P.OCTGS_BF16, idx=keep[i][0], count=keep[i][1], stream=s_)
        vbs[k].rasterize(c, prm, stream=s_, keep_last=False)

    psn, sel, kept, pairs = [], 0, 0, 0
    for i in tset:
        ceil_view(i)
        psn.append(SK.psnr(vb0.rgb, refs[i]))
        sel += int(vb0.sel_count.item())
        kept += int(keep[i][1].item())
        pairs += vb0.stats()["n_pairs"]
    ms, _ = time_views(args, torch, streams, kv, vbs, ceil_one, D)
    fin = [p_ for p_ in psn if math.isfinite(p_)]
    ceiling = {"what": "keep exactly the anchors whose logged blend weight on the view exceeds "
                       "tau_w (no predictor cost)",
               "skipped_fraction": round(1.0 - kept / max(sel, 1), 4),
               "pairs_removed_fraction": round(1.0 - pairs / max(sum(full_pairs.values()), 1), 4),
               "psnr_min_db": round(min(psn), 2),
               "psnr_mean_db": round(float(np.mean(fin)), 2) if fin else None,
               "fps": round(rate(args, ms, len(ccams)), 2),
               "fps_ratio_vs_plain_fp32": round(rate(args, ms, len(ccams)) / fps32, 4)}
    log(f"skip ceiling: {ceiling}")
    del keep, refs
    torch.cuda.empty_cache()

    lr_ = rules["learned"]
    # the fast path without the predictor, full BF16 decode, on the same views
    ms16, _ = time_views(args, torch, streams, ccams, vbs,
                         lambda k, c, s_: vbs[k].render(ds, c, prm, precision=P.OCTGS_BF16,
                                                       stream=s_, keep_last=False), D)
    fps_full = rate(args, ms16, len(ccams))
    # full decode is the fallback when the predictor skips under 1 % of the
    # held-out anchors or its path is not faster than full decode
    fallback = lr_["holdout_skipped_fraction"] < 0.01 or lr_["fps"] <= fps_full
    best_trivial = max((rules[k]["skipped_fraction"], k) for k in ("distance_only", "level_only"))
    res = {"fallback_to_full_decode": fallback,
           "train_views": len(train_cams),
           "train_family": "views of the zoom-out's family: altitude log-U(%g, %g) m, position "
                           "and aim jittered by N(0, (0.1 h)^2)" % h_range,
           "rows": int(z.shape[0]), "positive_fraction": round(float(y.mean().item()), 4),
           "tau_w": SKIP_TAU_W, "holdout_min_psnr_db": SKIP_MIN_HOLDOUT_DB,
           "rules": rules, "ceiling": ceiling,
           "learned_minus_best_single_input_skipped": round(lr_["skipped_fraction"] -
                                                             best_trivial[0], 4),
           "best_single_input_rule": best_trivial[1],
           "skipped_fraction": 0.0 if fallback else lr_["skipped_fraction"],
           "psnr_min_db": lr_["psnr_min_db"], "psnr_mean_db": lr_["psnr_mean_db"],
           "fps": lr_["fps"], "ms_per_view": lr_["ms_per_view"],
           "study_s": round(time.time() - t0, 1)}
    # predictor call per view: features, the 37-64-64-1 MLP on BF16 MFMA
    # (13,056 FLOP per selected anchor), keep-list compaction
    from paper_2403_17898_amd.hip_events import HipEvent
    net, thr = nets["learned"]
    pe = (HipEvent(), HipEvent())
    sh = P.stream_handle(None)
    pred_ms, sel = 0.0, 0
    for i in order:
        vb0.select(ds, ccams[i], prm)
        pe[0].record(sh)
        SK.predict(vb0, sb0, ds, ccams[i], net, thr)
        pe[1].record(sh)
        pe[1].synchronize()
        pred_ms += pe[0].elapsed_ms(pe[1])
        sel += int(vb0.sel_count.item())
    pms = pred_ms / len(order)
    res["predict_ms_per_view"] = round(pms, 4)
    res["predict_mfma_tflops"] = round(13056.0 * sel / len(order) / (pms * 1e-3) / 1e12, 2)
    res["predict_mfma_frac_bf16"] = round(res["predict_mfma_tflops"] / BF16_MFMA_PEAK_TFLOPS, 5)
    res["fps_full_decode_bf16"] = round(fps_full, 2)
    if fallback:
        res["fps"] = round(fps_full, 2)
        res["ms_per_view"] = round(1e3 / fps_full, 4)
    log(f"skip study: {res}")
    return res


def city_path(args, P, S, torch, np, prm, D, streams):
    """The city-scale scene, 4M anchors over 10 levels on 8,000 boxes over
    [-2000, 2000]^2: FPS of the 3840x2160 zoom-out (20 -> 3000 m; the timed
    views are the same stride through its 200 views) with plain FP32 and BF16
    decode, PSNR of BF16 against FP32 on those views, the oracle on a few of
    them, and the train step of 8 views at 2048x1024; with --city-skip also
    the learned-skip study of this scene."""
    t0 = time.time()
    sc = S.make_config5()
    ccams_c = S.config5_cameras(args.views)
    log(f"city scene: {sc.n} anchors, levels {sc.level_counts()}, generated in "
        f"{time.time() - t0:.1f}s")
    ds = P.DeviceScene.from_scene(sc)
    W, H = ccams_c[0].width, ccams_c[0].height
    cams = [P.make_camera(c) for c in ccams_c]
    order = list(range(len(cams)))
    tset = order
    vb = P.ViewBuffers(sc.n, sc.k, W, H, pair_capacity=160 << 20)
    per_view = {}
    for i in tset:
        vb.render(ds, cams[i], prm, precision=P.OCTGS_FP32)
        st = vb.stats()
        if st["pair_overflow"] or st["sync_error"]:
            raise SystemExit(f"city sizing pass failed: {st}")
        per_view[i] = st
    max_sel = max(s_["n_selected"] for s_ in per_view.values())
    max_pairs = max(s_["n_candidates"] for s_ in per_view.values())
    mean = {k: float(np.mean([per_view[i][k] for i in order]))
            for k in ("n_selected", "n_slots", "n_visible", "n_pairs")}
    del vb
    torch.cuda.empty_cache()
    gcap = max(1, int(max_sel * sc.k * 1.05) + 1024)
    pcap = max(1, int(max_pairs * 1.10) + 4096)
    vbs = [P.ViewBuffers(sc.n, sc.k, W, H, pair_capacity=pcap, gauss_capacity=gcap)
           for _ in range(D)]

    def timed(prec):
        return time_views(args, torch, streams, cams, vbs,
                          lambda k, c, s_: vbs[k].render(ds, c, prm, precision=prec, stream=s_,
                                                         keep_last=False), D)

    ms32, _ = timed(P.OCTGS_FP32)
    ms16, _ = timed(P.OCTGS_BF16)
    fps32 = rate(args, ms32, len(cams))
    res = {"workload": "city scene: 4M anchors / 10 LOD levels, 200-view zoom-out 20->3000 m, "
                       "3840x2160",
           "n_anchors": sc.n, "views": len(cams),
           "step": f"one pass over the {len(cams)} views of the trajectory",
           "fps_plain_fp32": round(fps32, 2),
           "fps_bf16": round(rate(args, ms16, len(cams)), 2),
           "mean_selected": round(mean["n_selected"]), "mean_gaussians": round(mean["n_slots"]),
           "mean_visible": round(mean["n_visible"]), "mean_pairs": round(mean["n_pairs"]),
           "max_selected": max_sel, "max_candidate_pairs": max_pairs, "frames_in_flight": D}
    vb = vbs[0]
    psn = []
    for i in tset:
        vb.render(ds, cams[i], prm, precision=P.OCTGS_FP32)
        ref = vb.rgb.clone()
        vb.render(ds, cams[i], prm, precision=P.OCTGS_BF16)
        mse = torch.mean((vb.rgb - ref) ** 2).item()
        psn.append(float("inf") if mse == 0 else 10 * math.log10(1.0 / mse))
    res["psnr_bf16_vs_fp32_min_db"] = round(min(psn), 2)
    res["psnr_views"] = len(psn)
    log(f"city: FP32 {res['fps_plain_fp32']} FPS, BF16 {res['fps_bf16']} FPS, "
        f"BF16 vs FP32 min PSNR {res['psnr_bf16_vs_fp32_min_db']} dB over {len(psn)} views")
    if not args.no_cpu_baseline:
        # the oracle on 3 of the timed 4K views, and the GPU paths against it
        from oracle import oracle as O
        O.build(force=False)
        thr, rho = O.scene_thresholds(sc)
        pick = [tset[0], tset[len(tset) // 2], tset[-1]]
        dt, acc = 0.0, {"fp32": [], "bf16": []}
        for i in pick:
            t1 = time.perf_counter()
            ref = O.render(sc, ccams_c[i], O.params_array(), thr, rho)
            dt += time.perf_counter() - t1
            for name, prec in (("fp32", P.OCTGS_FP32), ("bf16", P.OCTGS_BF16)):
                vb.render(ds, cams[i], prm, precision=prec)
                img = vb.rgb.double().cpu().numpy()
                mse = float(np.mean((img - ref["img"]) ** 2))
                acc[name].append((float(np.abs(img - ref["img"]).max()),
                                  float("inf") if mse == 0 else 10 * math.log10(1.0 / mse)))
            del ref
        res["cpu_baseline"] = {"value": round(len(pick) / dt, 4), "unit": "FPS",
                               "cores": O.num_threads(), "kind": "oracle",
                               "sample": f"trajectory views {pick} of the timed set, full FP64 "
                                         f"path, {dt:.1f} s",
                               "gpu_vs_oracle": {
                                   name: {"max_abs": max(e for e, _ in v),
                                          "psnr_min_db": round(min(p_ for _, p_ in v), 2)}
                                   for name, v in acc.items()}}
        log(f"city CPU oracle: {res['cpu_baseline']}")
    if args.city_skip and not args.no_skip:
        res["skip"] = skip_study(args, P, S, torch, np, sc, ds, cams, prm, W, H, vbs, D, streams,
                                 order, fps32, h_range=(20.0, 3000.0),
                                 n_train=args.city_skip_views)
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


# Per (pixel, list entry) the backward replay of Eq. 2 recomputes the
# Gaussian, alpha and T (10 FLOP: quadratic, exp counted as one, clamp,
# T = T' / (1 - a)), forms dL/dc (3 FMA), dL/da from the colour behind and
# dL/dC (3 FMA + 2), the running sum of the colour behind (3), dL/dq (2),
# and accumulates the nine per-Gaussian sums (2D mean 2 x 3, conic 3 x 2,
# opacity 2): 50 FLOP.
FLOP_PER_BLEND_BWD = 50.0


def composite_bwd_roofline(P, torch, np, vb, ds, cams, prm, targets, scale, W, H):
    """The train step's dominant kernel, the compositing backward, against
    the FP32 vector peak: each training view alone on the GPU, forward then
    L1 gradient then backward, with HIP events around the compositing
    backward; units = the entries each pixel consumed (Sigma last)."""
    from paper_2403_17898_amd import _lib as L
    from paper_2403_17898_amd.hip_events import HipEvent
    ev = [HipEvent() for _ in range(2 * L.OCTGS_RASTER_BWD_STAGES)]
    sh = P.stream_handle(None)
    dimg = torch.empty(3, H, W, device=vb.gauss.device)
    loss = torch.zeros(1, device=vb.gauss.device)
    t_ms, blends, pairs = 0.0, 0, 0
    for c, tg in zip(cams, targets):
        vb.render(ds, c, prm)
        P.l1_loss_grad(vb.rgb, tg, scale, dimg, loss)
        vb.rasterize_bwd(c, prm, dimg, stage_events=ev)
        torch.cuda.synchronize()
        t_ms += ev[0].elapsed_ms(ev[1])
        blends += int(vb.last.sum(dtype=torch.int64).item())
        pairs += vb.stats()["n_pairs"]
    n = len(cams)
    ms = t_ms / n
    tf = FLOP_PER_BLEND_BWD * blends / n / (ms * 1e-3) / 1e12
    # algorithmic bytes: 40 B read and 36 B written per pair (its record and
    # its nine gradients), 32 B per pixel (T, last, dL/dC, ...)
    alg = (40.0 + 36.0) * pairs / n + 32.0 * W * H
    return {"kernel": "composite_bwd", "bound": "alu", "achieved": round(tf, 2),
            "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tf / FP32_VECTOR_PEAK_TFLOPS, 4), "flop_per_blend": FLOP_PER_BLEND_BWD,
            "blends_per_launch": round(blends / n), "launch_ms": round(ms, 5),
            "algorithmic_bytes": round(alg), "hbm_gbs": round(alg / (ms * 1e-3) / 1e9, 1),
            "traffic": composite_bwd_traffic()}


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
    roof_bwd = composite_bwd_roofline(P, torch, np, mv.vbs[0], ds, cams, prm, targets, scale,
                                      W, H)
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
           "views_in_flight": nbuf, "roofline_bwd": roof_bwd}
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


# ---------------------------------------------------------------------------
# profile summaries (rocprofv3 CSV output -> the text files under profiles/)
# ---------------------------------------------------------------------------

# kernels of one street-scene view in the per-stage timing loop, with their
# launches per view: (label, name substring, launches)
VIEW_KERNELS = [("k_select_mark", "k_select_mark", 1), ("k_select_scatter", "k_select_scatter", 1),
                ("k_decode_prep<BF16>", "k_decode_prep<true>", 1), ("k_decode<BF16>", "k_decode<true>", 1),
                ("k_project_mark", "k_project_mark", 1), ("k_project_compact", "k_project_compact", 1),
                ("depth sort passes", "k_sort_pass<1, 8>", 4), ("k_emit_scan", "k_emit_scan", 1),
                ("k_emit_pairs", "k_emit_pairs", 1), ("tile sort passes", "k_sort_pass<1, 16>", 2),
                ("k_ranges", "k_ranges", 1), ("k_composite", "k_composite<false>", 1)]
RASTER_LABELS = ("k_project_mark", "k_project_compact", "depth sort passes", "k_emit_scan",
                 "k_emit_pairs", "tile sort passes", "k_ranges", "k_composite")


def _csv_rows(d: str, suffix: str):
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)):
        with open(f, newline="") as fh:
            rows += list(csv.DictReader(fh))
    if not rows:
        raise SystemExit(f"no *{suffix} under {d}")
    rows.sort(key=lambda r: int(r.get("Dispatch_Id") or r.get("Correlation_Id") or 0))
    return rows


def _last(rows, sub, n):
    sel = [r for r in rows if sub in r["Kernel_Name"]]
    if len(sel) < n:
        raise SystemExit(f"only {len(sel)} dispatches of {sub}, need {n}")
    return sel[-n:]


def summarize_profiles(trace_dir: str, fetch_dir: str, write_dir: str, views: int, cmds):
    """Writes profiles/raster_street1080p_kernel_trace.txt,
    raster_street1080p_hbm_bytes.txt and composite_street1080p_hbm_bytes.txt
    from the CSV output of the three rocprofv3 runs `cmds` (kernel trace,
    FETCH_SIZE, WRITE_SIZE) of the per-stage timing loop: the last `views`
    views' dispatches of each kernel (one pass over the trajectory).  Counters are KiB per dispatch, scaled
    by what each reads for the 256 MiB copies of --copy-calibration."""
    trace = _csv_rows(trace_dir, "kernel_trace.csv")
    fetch = [r for r in _csv_rows(fetch_dir, "counter_collection.csv") if r["Counter_Name"] == "FETCH_SIZE"]
    write = [r for r in _csv_rows(write_dir, "counter_collection.csv") if r["Counter_Name"] == "WRITE_SIZE"]

    def copy_scale(rows, expect_kib):
        cp = sorted((float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]),
                    reverse=True)[:5]
        return (expect_kib / (sum(cp) / len(cp)), sum(cp) / len(cp)) if cp else (None, None)

    # a 256 MiB device copy reads and writes 256 MiB
    sf, cf = copy_scale(fetch, 262144.0)
    sw, cw = copy_scale(write, 262144.0)
    lines = []
    per = {}
    for label, sub, per_view in VIEW_KERNELS:
        n = per_view * views
        t = _last(trace, sub, n)
        us = sum((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) for r in t) / 1e3 / views
        rd = sum(float(r["Counter_Value"]) for r in _last(fetch, sub, n)) * 1024 * sf / views
        wr = sum(float(r["Counter_Value"]) for r in _last(write, sub, n)) * 1024 * sw / views
        per[label] = (per_view, rd, wr, us)
    hdr = f"{'kernel':<22}{'per view':>9}{'MB read':>10}{'MB written':>12}{'us':>9}{'GB/s':>9}"
    lines.append(hdr)
    for label, (pv, rd, wr, us) in per.items():
        lines.append(f"{label:<22}{pv:>9}{rd / 1e6:>10.2f}{wr / 1e6:>12.2f}{us:>9.1f}"
                     f"{(rd + wr) / (us * 1e-6) / 1e9:>9.1f}")
    rb = sum(per[k][1] + per[k][2] for k in RASTER_LABELS)
    rus = sum(per[k][3] for k in RASTER_LABELS)
    shas = [f"source_sha256 {os.path.basename(f)}: {sha256_of(f)}" for f in RASTER_SOURCES]
    cmd_txt = "\n".join("  " + c for c in cmds)
    raster = (
        "HBM traffic of the whole rasterizer forward (projection, depth sort, pair emission, tile\n"
        f"sort, ranges, compositing) on the street-scene benchmark (1920x1080, the {views} views of\n"
        "the zoom-out, one view in flight), per view:\n"
        "FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by what each counter reads for a plain\n"
        f"256 MiB device copy in the same run (x{sf:.3f} and x{sw:.3f}), over the dispatches of the\n"
        f"per-stage timing loop (the last {views} views), and the kernels' durations from the kernel\n"
        "trace of the same command without counters.\n\n"
        f"commands ($REPO = repository root):\n{cmd_txt}\n\n" + "\n".join(lines) + "\n\n"
        f"rasterizer total per view: {rb / 1e6:.1f} MB in {rus:.1f} us of kernel time -> "
        f"{rb / (rus * 1e-6) / 1e9:.0f} GB/s, {rb / (rus * 1e-6) / 1e9 / HBM_PEAK_GBS:.3f} of the 8 TB/s HBM peak\n"
        f"hbm_bytes_per_view: {int(rb)}\nkernel_us_per_view: {rus:.1f}\nviews: {views}\n"
        + "\n".join(shas) + "\n(bench.py reports these bytes only while both sources are unchanged and\n"
        " for the same --views)\n")
    _, crd, cwr, cus = per["k_composite"]
    comp = (
        "HBM bytes per launch of k_composite on the street-scene benchmark (1920x1080, the\n"
        f"{views} views of the zoom-out), from the FETCH_SIZE and\n"
        "WRITE_SIZE counters (KiB per dispatch), each scaled by what the same counter reads for a plain\n"
        "256 MiB device-to-device copy in the same run.\n\n"
        f"commands ($REPO = repository root):\n{cmd_txt}\n\n"
        f"(the per-stage timing loop's dispatches: the last {views} composites of each run)\n"
        f"FETCH_SIZE 256 MiB copy mean KiB: {cf:.1f} -> scale {sf:.3f}\n"
        f"WRITE_SIZE 256 MiB copy mean KiB: {cw:.1f} -> scale {sw:.3f}\n"
        f"hbm_bytes_per_launch: {int(crd + cwr)}\n"
        f"read bytes per launch (scaled): {int(crd)}\nwrite bytes per launch (scaled): {int(cwr)}\n"
        f"kernel trace average duration of these launches: {cus:.2f} us\nviews: {views}\n"
        + "\n".join(shas) + "\n")
    # whole-run kernel statistics from the trace
    from collections import defaultdict
    agg = defaultdict(list)
    for r in trace:
        agg[r["Kernel_Name"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in agg.values())
    tl = [f"{'kernel':<44}{'calls':>7}{'avg_us':>10}{'min_us':>10}{'max_us':>10}{'share':>8}"]
    for name, v in sorted(agg.items(), key=lambda kv: -sum(kv[1]))[:24]:
        short = name.replace("(anonymous namespace)::", "").replace("octgs::", "")
        short = short.split("(")[0].removeprefix("void ")
        tl.append(f"{short[:43]:<44}{len(v):>7}{sum(v) / len(v):>10.2f}{min(v):>10.2f}"
                  f"{max(v):>10.2f}{100 * sum(v) / total:>7.2f}%")
    trace_txt = (
        "Kernel trace of the street-scene render benchmark (1M anchors, 8 LOD levels, 1920x1080;\n"
        f"the {views} views of the zoom-out), --stages-only run (the sizing pass and the\n"
        "per-stage timing loop, one view at a time).\n\n"
        f"command ($REPO = repository root):\n  {cmds[0]}\n\n" + "\n".join(tl) + "\n\n"
        f"per-stage timing loop (the last {views} views), kernel-trace average per view:\n" +
        "\n".join(f"  {k:<22}{per[k][3]:>9.2f} us" for k in per) + "\n"
        f"k_composite average over the per-stage loop: {cus:.2f} us\nviews: {views}\n")
    out = {"raster_street1080p_hbm_bytes.txt": raster, "composite_street1080p_hbm_bytes.txt": comp,
           "raster_street1080p_kernel_trace.txt": trace_txt}
    for name, txt in out.items():
        with open(os.path.join(ROOT, "profiles", name), "w") as f:
            f.write(txt)
        print(f"wrote profiles/{name}")


def _short(name: str) -> str:
    s_ = name.replace("(anonymous namespace)::", "").replace("octgs::", "")
    return s_.split("(")[0].removeprefix("void ")


def summarize_train_trace(trace_dir: str, steps: int, cmd: str, log_path: str):
    """Writes profiles/train_step_c3_kernel_trace.txt from a kernel trace of
    `bench.py --train-only --inflight 1 --train-steps STEPS`: the dispatches
    of the timed steps (after the third warm-up step's Adam update, through
    the last timed step's), per kernel per step."""
    from collections import defaultdict
    trace = _csv_rows(trace_dir, "kernel_trace.csv")
    trace.sort(key=lambda r: int(r["Start_Timestamp"]))
    adam = [r for r in trace if "k_adam_many" in r["Kernel_Name"]]
    if len(adam) < 3 + steps:
        raise SystemExit(f"{len(adam)} Adam updates in the trace, need {3 + steps}")
    t0, t1 = int(adam[2]["End_Timestamp"]), int(adam[2 + steps]["End_Timestamp"])
    agg = defaultdict(list)
    for r in trace:
        if t0 < int(r["Start_Timestamp"]) <= t1:
            agg[_short(r["Kernel_Name"])].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in agg.values())
    lines = [f"{'kernel':<38}{'per step':>9}{'avg_us':>10}{'ms/step':>10}{'share':>9}"]
    for name, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"{name[:37]:<38}{len(v) / steps:>9.1f}{sum(v) / len(v):>10.2f}"
                     f"{sum(v) / steps / 1e3:>10.3f}{100 * sum(v) / total:>8.2f}%")
    said = ""
    if log_path and os.path.exists(log_path):
        said = [ln.strip() for ln in open(log_path) if "train step only" in ln]
        said = ("\nbench.py in the traced run (HIP events, median step; the profiler adds launch "
                "gaps): " + said[-1].split("] ", 1)[-1] + "\n") if said else ""
    txt = (
        "Kernel trace of the training step (500k anchors / 6 levels, 4 views at 1600x1066; forward,\n"
        "mean-L1 loss, backward through compositing, projection and decode, Adam), run with one view\n"
        "in flight (--inflight 1) so that every launch is uncontended; the benchmark's default step\n"
        f"runs the views on separate streams and overlaps them.  The table covers the {steps} timed\n"
        "steps of the traced run (the dispatches after the third warm-up step's Adam update through\n"
        "the last timed step's).\n\n"
        f"command ($REPO = repository root):\n  {cmd}\n\n" + "\n".join(lines) + "\n\n"
        f"kernel time per step (sum of dispatch durations): {total / steps / 1e3:.3f} ms\n" + said)
    with open(os.path.join(ROOT, "profiles", "train_step_c3_kernel_trace.txt"), "w") as f:
        f.write(txt)
    print("wrote profiles/train_step_c3_kernel_trace.txt")


def summarize_counters(sq_dir: str, trace_dir: str, views: int, cmd: str, out_name: str,
                       kernels=None, title=None):
    """Writes profiles/<out_name> from one rocprofv3 --pmc run of SQ counters
    (and GRBM_GUI_ACTIVE) over the per-stage timing loop: per kernel, VALU
    busy, VALU lane utilisation, MFMA busy and the BF16 MFMA rate the
    counters imply, each over the last `views` views' dispatches.
    GRBM_GUI_ACTIVE reads the sum over the 8 XCDs of the GPU-busy cycles
    (8x a dispatch's duration in cycles), so it is divided by 8; the SIMD
    count is 1024 (256 CUs x 4)."""
    from collections import defaultdict
    if os.path.basename(out_name) != out_name:
        raise SystemExit("the summary name is a file name under profiles/, not a path")
    rows = _csv_rows(sq_dir, "counter_collection.csv")
    trace = _csv_rows(trace_dir, "kernel_trace.csv")
    by = defaultdict(dict)
    name = {}
    for r in rows:
        d = int(r["Dispatch_Id"])
        by[d][r["Counter_Name"]] = float(r["Counter_Value"])
        name[d] = r["Kernel_Name"]
    order = sorted(by)
    simds = 1024
    lines = [f"{'kernel':<22}{'per unit':>9}{'us':>8}{'waves':>8}{'VALU busy':>11}{'lane use':>10}"
             f"{'MFMA busy':>11}{'BF16 TF/s':>11}{'of peak':>9}{'F32 TF/s':>10}{'of peak':>9}"
             f"{'GRBM GHz':>10}"]
    for label, sub, per_view in (kernels or VIEW_KERNELS):
        n = per_view * views
        ds = [d for d in order if sub in name[d]][-n:]
        if len(ds) < n:
            raise SystemExit(f"only {len(ds)} dispatches of {sub} with counters, need {n}")
        c = defaultdict(float)
        for d in ds:
            for k, v in by[d].items():
                c[k] += v
        t = _last(trace, sub, n)
        us = sum((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) for r in t) / 1e3 / n
        cyc = us * 1e-6 * CLOCK_HZ * n  # the dispatches' cycles at the peak engine clock
        grbm_ghz = c["GRBM_GUI_ACTIVE"] / 8.0 / (us * 1e-6 * n) / 1e9
        valu = 4.0 * c["SQ_ACTIVE_INST_VALU"] / (simds * cyc)
        lane = c["SQ_THREAD_CYCLES_VALU"] / max(64.0 * c["SQ_ACTIVE_INST_VALU"], 1.0)
        mfma = c["SQ_VALU_MFMA_BUSY_CYCLES"] / (simds * cyc)
        tf = c["SQ_INSTS_VALU_MFMA_MOPS_BF16"] * 512 / n / (us * 1e-6) / 1e12
        tf32 = c["SQ_INSTS_VALU_MFMA_MOPS_F32"] * 512 / n / (us * 1e-6) / 1e12
        lines.append(f"{label:<22}{per_view:>9}{us:>8.1f}{c['SQ_WAVES'] / n:>8.0f}{100 * valu:>10.1f}%"
                     f"{100 * lane:>9.1f}%{100 * mfma:>10.2f}%{tf:>11.2f}{tf / 2500.0:>9.4f}"
                     f"{tf32:>10.2f}{tf32 / 157.3:>9.4f}{grbm_ghz:>10.2f}")
    head = title.replace("\\n", "\n") + "\n" if title else (
        "SQ counters of the street-scene render benchmark (1M anchors, 8 LOD levels, 1920x1080,\n"
        f"the {views} views of the zoom-out, one view at a time), per kernel over the per-stage\n"
        "timing loop (--stages-only), from one rocprofv3 --pmc run:\n")
    txt = (
        head +
        "  VALU busy  = 4 SQ_ACTIVE_INST_VALU / (1024 SIMDs x cycles)   (the counter is in quad-cycles)\n"
        "  lane use   = SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU)\n"
        "  MFMA busy  = SQ_VALU_MFMA_BUSY_CYCLES / (1024 SIMDs x cycles)\n"
        "  BF16 TF/s  = 512 SQ_INSTS_VALU_MFMA_MOPS_BF16 per dispatch / kernel-trace duration,\n"
        "               'of peak' against the 2.5 PFLOP/s dense BF16 peak\n"
        "  F32 TF/s   = the same for SQ_INSTS_VALU_MFMA_MOPS_F32 (FP32 MFMA), against 157.3 TFLOP/s\n"
        "  us         = kernel-trace average duration of the same dispatches (a separate run\n"
        "               without counters); cycles = us x 2.4 GHz, the peak engine clock, so the\n"
        "               busy fractions are lower bounds if the clock ran lower\n"
        "  GRBM GHz   = GRBM_GUI_ACTIVE / 8 (the counter sums the 8 XCDs) / us: about 2.4 for\n"
        "               long kernels; above it for short ones, whose counter-collection\n"
        "               dispatches carry fixed overhead.\n\n"
        f"command ($REPO = repository root):\n  {cmd}\n\n" + "\n".join(lines) + f"\nunits: {views}\n")
    with open(os.path.join(ROOT, "profiles", out_name), "w") as f:
        f.write(txt)
    print(f"wrote profiles/{out_name}")


def summarize_bwd_traffic(fetch_dir: str, write_dir: str, steps: int, cmds):
    """Writes profiles/composite_bwd_train_c3_hbm_bytes.txt from the
    FETCH_SIZE and WRITE_SIZE runs `cmds` of `bench.py --train-only
    --inflight 1 --train-steps STEPS --copy-calibration`: the last four
    dispatches of k_composite_bwd, which are the launches the backward's
    roofline times (each training view once, alone on the GPU), KiB per
    dispatch scaled by what each counter reads for the 256 MiB copies."""
    fetch = [r for r in _csv_rows(fetch_dir, "counter_collection.csv") if r["Counter_Name"] == "FETCH_SIZE"]
    write = [r for r in _csv_rows(write_dir, "counter_collection.csv") if r["Counter_Name"] == "WRITE_SIZE"]

    def copy_mean(rows):
        cp = sorted((float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]),
                    reverse=True)[:5]
        if not cp:
            raise SystemExit("no calibration copies in the counter run")
        return sum(cp) / len(cp)

    cf, cw = copy_mean(fetch), copy_mean(write)
    sf, sw = 262144.0 / cf, 262144.0 / cw
    n = 4
    rd = sum(float(r["Counter_Value"]) for r in _last(fetch, "k_composite_bwd", n)) / n * 1024 * sf
    wr = sum(float(r["Counter_Value"]) for r in _last(write, "k_composite_bwd", n)) / n * 1024 * sw
    shas = [f"source_sha256 {os.path.basename(f)}: {sha256_of(f)}" for f in BWD_SOURCES]
    cmd_txt = "\n".join("  " + c for c in cmds)
    txt = (
        "HBM bytes per launch of k_composite_bwd in the training step (500k anchors / 6 levels,\n"
        "4 views at 1600x1066, one view in flight), from the FETCH_SIZE and WRITE_SIZE counters (KiB\n"
        "per dispatch), each scaled by what the same counter reads for a plain 256 MiB device copy in\n"
        f"the same run, over the last {n} dispatches: the launches that the backward's roofline in\n"
        f"bench.py times, each training view once, after {steps} timed steps.\n\n"
        f"commands ($REPO = repository root):\n{cmd_txt}\n\n"
        f"FETCH_SIZE 256 MiB copy mean KiB: {cf:.1f} -> scale {sf:.3f}\n"
        f"WRITE_SIZE 256 MiB copy mean KiB: {cw:.1f} -> scale {sw:.3f}\n"
        f"hbm_bytes_per_launch: {int(rd + wr)}\n"
        f"read bytes per launch (scaled): {int(rd)}\nwrite bytes per launch (scaled): {int(wr)}\n"
        + "\n".join(shas) + "\n")
    with open(COMPOSITE_BWD_PMC, "w") as f:
        f.write(txt)
    print(txt)


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-train-trace":
        # python bench.py --summarize-train-trace TRACE_DIR STEPS CMD [LOG]
        a = sys.argv[2:]
        summarize_train_trace(a[0], int(a[1]), a[2], a[3] if len(a) > 3 else "")
    elif len(sys.argv) > 1 and sys.argv[1] == "--summarize-counters":
        # python bench.py --summarize-counters SQ_DIR TRACE_DIR UNITS CMD OUT_NAME [SPEC [TITLE]]
        # SPEC: "label=kernel-name substring:dispatches per unit;..." (default: the
        # per-view render kernels); TITLE: first lines of the summary
        a = sys.argv[2:]
        spec = None
        if len(a) > 5:
            spec = []
            for item in a[5].split(";"):
                lab, rest = item.split("=", 1)
                sub, cnt = rest.rsplit(":", 1)
                spec.append((lab, sub, int(cnt)))
        summarize_counters(a[0], a[1], int(a[2]), a[3], a[4], spec, a[6] if len(a) > 6 else None)
    elif len(sys.argv) > 1 and sys.argv[1] == "--summarize-bwd-traffic":
        # python bench.py --summarize-bwd-traffic FETCH_DIR WRITE_DIR STEPS CMD1 CMD2
        a = sys.argv[2:]
        summarize_bwd_traffic(a[0], a[1], int(a[2]), a[3:5])
    elif len(sys.argv) > 1 and sys.argv[1] == "--summarize-profiles":
        # python bench.py --summarize-profiles TRACE_DIR FETCH_DIR WRITE_DIR VIEWS CMD1 CMD2 CMD3
        a = sys.argv[2:]
        summarize_profiles(a[0], a[1], a[2], int(a[3]), a[4:7])
    else:
        main()
