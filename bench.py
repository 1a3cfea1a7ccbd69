#!/usr/bin/env python3
"""Benchmark of the GES rasterizer on one MI355X.

A step is one pass of the whole hot path over one frame: preprocess (with the key-count readback),
tile binning, per-tile sort, forward raster, the frequency-masked L1 loss and its gradient, the
reverse-order adjoint raster and the preprocess backward.  The default workload is the 3M-splat
1920x1080 training step (64 clusters, SH degree 3, loss 0.5 L1 + 0.5 masked L1 at omega = 0.75,
mask made once outside the timed region); inputs are synthetic and already resident in HBM.

Also measured, and reported under "train_step" (not the headline value): the full optimisation step of
the paper's recipe on a fresh copy of the same scene -- the frequency mask at omega = it / 40000, the loss
0.3 L1 + 0.2 SSIM + 0.5 masked L1, the adjoint, and Adam over the six parameter groups.

Prints ONE JSON line.  Per-kernel times come from HIP events recorded around every launch on the
stream the kernel runs on (library stage timing), over the timed steps.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3       # MI355X published FP32 vector peak (packed FMA)
VALU_PEAK_TOPS = 39.32         # 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz: non-packed lane operations (T/s)

# Raster work per pair in VALU lane-slots (a transcendental counts as 4): the forward examines a pair in
# 8 slots and composites it in 22 (PHI; GEF adds log2 and exp2: 30); the backward walks a pair in 8 and
# differentiates a composited one in 55 (GEF: 67).  Beside them, FLOPs (FMA = 2) for the FP32 peak.
FWD_SLOTS_EXAMINED = 8
FWD_SLOTS_BLENDED = {0: 22, 1: 30}
BWD_SLOTS_WALKED = 8
BWD_SLOTS_BLENDED = {0: 55, 1: 67}
FWD_FLOP_EXAMINED = 9          # dx, dy, quadratic form
FWD_FLOP_BLENDED = {0: 12, 1: 15}   # falloff, alpha, transmittance, colour (PHI, GEF)
BWD_FLOP_EXAMINED = 9
BWD_FLOP_BLENDED = {0: 51, 1: 60}
RASTER_STAGES = ("raster_forward", "raster_backward")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", type=int, default=2, choices=[0, 1, 2, 3])
    ap.add_argument("--tile-cull", choices=["square", "ellipse"], default="ellipse")
    ap.add_argument("--falloff", choices=["phi", "gef"], default="phi")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other-workloads", action="store_true",
                    help="skip the forward+backward measurements of the 1M-splat and 5M-splat workloads")
    ap.add_argument("--no-serving", action="store_true", help="skip the batched-serving measurement")
    ap.add_argument("--no-mixture", action="store_true", help="skip the 1-D mixture-simulation sweep")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the shape-strength sweep and the approximate/exact falloff comparison")
    ap.add_argument("--mixture-epochs", type=int, default=1000)
    ap.add_argument("--no-train-step", action="store_true",
                    help="skip the full optimisation-step measurement (adds SSIM, per-step mask and Adam)")
    ap.add_argument("--no-views-step", action="store_true",
                    help="skip the multi-view optimisation step (views batched vs one after another)")
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests per arrival rate")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for scaling rocprof FETCH/WRITE counters)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(stage, n, sh_coeffs, K, C, L, px, R=0):
    """Minimum HBM bytes of one launch of an HBM-bound stage: n splats, K keys, C candidate slots, L listed
    splats, px pixels, R rows stored by the backward raster (the per-unit figures are the comments below)."""
    splat_in = 12 + 12 + 16 + 4 + 4 + 12 * sh_coeffs
    return {
        # parameters in; record, visibility word, depth key and candidate count out
        "preprocess": n * (splat_in + 64 + 4 + 8),
        # the item keys in, the listed (key, item) pairs out
        "depth_sort": 4 * n + 8 * L,
        # the depth order and the candidate counts in, chunk offsets out
        "key_scan": 8 * L + L // 16,
        # per listed splat its order entry, record and count in, tile count and visibility out; 8 B per slot
        "duplicate": L * (4 + 64 + 4 + 8) + 8 * C,
        # the slots in, the sorted (tile, splat) pairs out
        "tile_sort": 8 * C + 8 * K,
        # the slot marks (1 bit per slot) and every stored row's 10 sums and splat (44 B); the 2-D gradients
        # written (80 B per splat with a row, at most R) are left out, so this is a lower bound
        "row_reduce": C // 8 + 44 * R,
        "preprocess_backward": n * (16 + 12 + 16 + 4 + 12 * sh_coeffs + 48 + 80 + 4 * (3 + 3 + 4 + 1 + 1 + 3 * sh_coeffs)),
        # the row marks cleared before the backward raster
        "zero": C // 8,
        "loss": 37 * px,
        # the preprocess backward with Adam fused in: its inputs as above, no gradient stores, and per
        # parameter the two moments read (8 B) and the parameter and both moments written (12 B)
        "preprocess_backward_adam": n * (16 + 12 + 16 + 4 + 12 * sh_coeffs + 48 + 80
                                         + 20 * (3 + 3 + 4 + 1 + 1 + 3 * sh_coeffs)),
        # per parameter: read p, g, m, v and write p, m, v (binary32)
        "adam": 28 * n * (3 + 3 + 4 + 1 + 1 + 3 * sh_coeffs),
        # per pixel: forward reads img, target (24 B) and writes 9 maps (36 B); backward reads the maps (36 B),
        # img, target and dL (36 B) and writes dL (12 B)
        "ssim": 144 * px,
    }.get(stage)


def raster_work(stage, falloff, pairs_exam, pairs_blend, bwd_walk):
    """(VALU lane-slots, FLOPs) of one launch of a raster stage from its exact pair counts."""
    f = 1 if falloff == 1 else 0
    if stage == "raster_forward":
        slots = FWD_SLOTS_EXAMINED * (pairs_exam - pairs_blend) + FWD_SLOTS_BLENDED[f] * pairs_blend
        flop = FWD_FLOP_EXAMINED * pairs_exam + FWD_FLOP_BLENDED[f] * pairs_blend
    else:
        slots = BWD_SLOTS_WALKED * (bwd_walk - pairs_blend) + BWD_SLOTS_BLENDED[f] * pairs_blend
        flop = BWD_FLOP_EXAMINED * bwd_walk + BWD_FLOP_BLENDED[f] * pairs_blend
    return slots, flop


def stage_rooflines(per_stage, m, falloff, workload):
    """Each stage's fraction of its roofline: VALU lane-slots against 39.3 T/s for the raster (with the FLOP
    figure beside it and, from the committed counters, the issued-over-algorithmic lane-slot ratio), HBM
    bytes against 8 TB/s for the rest (with the counters' measured-over-algorithmic byte ratio)."""
    out = {}
    for stage, ms in per_stage.items():
        if ms <= 0:
            continue
        if stage in RASTER_STAGES:
            slots, flop = raster_work(stage, falloff, m["pairs_exam"], m["pairs_blend"], m["bwd_walk"])
            tops = slots / (ms / 1e3) / 1e12
            row = {"bound": "alu", "achieved": round(tops, 3), "peak": VALU_PEAK_TOPS, "unit": "Tlane-op/s",
                   "frac": round(tops / VALU_PEAK_TOPS, 4), "algorithmic_lane_ops": slots,
                   "flop_tflops": round(flop / (ms / 1e3) / 1e12, 3),
                   "flop_frac_of_157.3": round(flop / (ms / 1e3) / 1e12 / FP32_PEAK_TFLOPS, 4)}
            issued = read_counter(stage, workload, "valu_insts_per_launch")
            if issued is not None:
                row["issued_over_algorithmic"] = round(issued * 64 / slots, 3)
        else:
            nbytes = algorithmic_bytes(stage, m["n"], m["sh_k"], m["K"], m["C"], m["L"], m["px"], m.get("R", 0))
            if nbytes is None:
                continue
            gbs = nbytes / (ms / 1e3) / 1e9
            row = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes": nbytes}
            measured = read_counter(stage, workload, "hbm_bytes_per_launch")
            if measured is not None:
                row["measured_over_algorithmic"] = round(measured / nbytes, 3)
        out[stage] = row
    return out


def kernel_source_hash(stage):
    src = {"raster_forward": "raster.hip", "raster_backward": "raster.hip", "preprocess": "preprocess.hip",
           "preprocess_backward": "preprocess_bwd.hip", "tile_sort": "radix.hip", "depth_sort": "radix.hip",
           "duplicate": "binning.hip", "key_scan": "binning.hip", "row_reduce": "binning.hip", "loss": "loss.hip",
           "zero": "loss.hip"}[stage]
    # the kernel's source file and the shared headers it is built with (layouts and constants live there)
    csrc = os.path.join(HERE, "paper_2402_10128_amd", "csrc")
    h = hashlib.sha256()
    for name in [src] + sorted(f for f in os.listdir(csrc) if f.endswith(".h")):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_counter(stage, workload, field):
    """A per-launch counter figure of a stage from the committed rocprofv3 summary
    profiles/<stage>_counters_workload<k>.md, if that summary was taken from the current source."""
    path = os.path.join(HERE, "profiles", f"{stage}_counters_workload{workload}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("source_sha256_16") != kernel_source_hash(stage):
        return None
    try:
        return float(fields[field])
    except (KeyError, ValueError):
        return None


def _oracle_frame(cfg, falloff, tile_cull, backward=True):
    """One whole frame on the oracle (test infrastructure): preprocess, keys and their sort, the per-pixel
    render and, with backward, the reverse pass and the binary64 chain rule.  Seconds per part."""
    from oracle import oracle as O
    from oracle import preprocess_f64 as PF
    sc, cam = cfg["scene"], cfg["camera"]
    orc = O.Oracle(sc.arrays(), sc.sh_degree, cam, falloff=falloff, tile_cull=tile_cull)
    t = {}
    t0 = time.perf_counter()
    rec = orc.preprocess(O.MODE_F32)
    t["preprocess"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, vals, ranges = orc.build_keys(rec)
    t["keys"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    orc.render(rec, vals, ranges)
    t["render"] = time.perf_counter() - t0
    if backward:
        dL = np.random.default_rng(1).standard_normal((cam.height, cam.width, 3))
        t0 = time.perf_counter()
        g2d, _ = orc.backward2d(rec, dL, vals, ranges)
        t["backward"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        PF.chain_to_params(sc.arrays(), sc.sh_degree, cam, g2d, rec.tiles_touched > 0, rec.clamp_bits, falloff, 0.1)
        t["chain_rule"] = time.perf_counter() - t0
    return t


def _oracle_tiles(cfg, falloff, tile_cull, tiles, backward=True):
    """The oracle on a sample of tiles: full preprocess, those tiles' sorted lists, their per-pixel render
    (and reverse pass).  Seconds per part."""
    from oracle import oracle as O
    sc, cam = cfg["scene"], cfg["camera"]
    orc = O.Oracle(sc.arrays(), sc.sh_degree, cam, falloff=falloff, tile_cull=tile_cull)
    t = {}
    t0 = time.perf_counter()
    rec = orc.preprocess(O.MODE_F32)
    t["preprocess"] = time.perf_counter() - t0
    T = orc.TX * orc.TY
    t0 = time.perf_counter()
    vals, ranges, pos = [], np.zeros((T, 2), np.int64), 0
    for tt in tiles:
        lst = orc.tile_list(rec, int(tt))
        ranges[tt] = (pos, pos + len(lst))
        pos += len(lst)
        vals.append(lst)
    values = np.concatenate(vals) if vals else np.zeros(0, np.uint32)
    t["lists"] = time.perf_counter() - t0
    tl = np.asarray(tiles, np.int32)
    t0 = time.perf_counter()
    orc.render(rec, values, ranges, tiles=tl)
    if backward:
        dL = np.random.default_rng(1).standard_normal((cam.height, cam.width, 3))
        orc.backward2d(rec, dL, values, ranges, tiles=tl)
    t["tiles"] = time.perf_counter() - t0
    return t


def cpu_baseline(cfgs, falloff, tile_cull, log_fn):
    """The oracle as it stands, on this host's cores, on each workload (a baseline, not the target):
    workload 0 whole frame at 1 thread and at all threads, workload 1 whole forward, workload 2 whole
    forward+backward (the headline figure), workload 3 on 80 sampled tiles, workload 4 on 64 whole
    requests."""
    import platform

    import torch
    from oracle import oracle as O
    from paper_2402_10128_amd import synth
    cores = O.num_threads()
    cpu_model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    legs = {}

    def px(cfg):
        return cfg["camera"].width * cfg["camera"].height

    for th in sorted({1, cores}):
        O.set_num_threads(th)
        torch.set_num_threads(th)
        t = _oracle_frame(cfgs[0], falloff, tile_cull)
        legs[f"workload0_fwd_bwd_{th}_threads"] = {"mpix_s": round(px(cfgs[0]) / sum(t.values()) / 1e6, 5),
                                                    "s": round(sum(t.values()), 3), "threads": th}
    O.set_num_threads(cores)
    torch.set_num_threads(cores)
    log_fn(f"cpu: workload 0 {legs}")
    t = _oracle_frame(cfgs[1], falloff, tile_cull, backward=False)
    legs["workload1_forward"] = {"mpix_s": round(px(cfgs[1]) / sum(t.values()) / 1e6, 5), "s": round(sum(t.values()), 2),
                                 "parts_s": {k: round(v, 2) for k, v in t.items()}}
    log_fn(f"cpu: workload 1 forward {legs['workload1_forward']}")
    t = _oracle_frame(cfgs[2], falloff, tile_cull, backward=True)
    head_s = sum(t.values())
    legs["workload2_fwd_bwd"] = {"mpix_s": round(px(cfgs[2]) / head_s / 1e6, 5), "s": round(head_s, 2),
                                 "parts_s": {k: round(v, 2) for k, v in t.items()}}
    log_fn(f"cpu: workload 2 forward+backward {legs['workload2_fwd_bwd']}")
    cam3 = cfgs[3]["camera"]
    TX, TY = (cam3.width + 15) // 16, (cam3.height + 15) // 16
    rng = np.random.default_rng(3)
    block = [ty * TX + tx for ty in range(TY // 2 - 2, TY // 2 + 2) for tx in range(TX // 2 - 2, TX // 2 + 2)]
    tiles = np.unique(np.concatenate([rng.choice(TX * TY, 64, replace=False), block]))
    t = _oracle_tiles(cfgs[3], falloff, tile_cull, tiles)
    legs["workload3_sampled_tiles"] = {"mpix_s": round(256 * len(tiles) / (t["lists"] + t["tiles"]) / 1e6, 5),
                                       "tiles": int(len(tiles)), "parts_s": {k: round(v, 2) for k, v in t.items()},
                                       "note": "forward+backward of 64 random tiles and a central 4x4 block; "
                                               "the rate excludes the whole-scene preprocess"}
    log_fn(f"cpu: workload 3 sampled {legs['workload3_sampled_tiles']}")
    scenes = [synth.scene_clusters(n, 1004 + 10 * i) for i, n in enumerate(synth.SERVING_SIZES)]
    reqs = synth.serving_requests(64, len(scenes), list(synth.SERVING_RESOLUTIONS), seed=2000)
    per_req, tot_px = [], 0
    for k, cam in reqs:
        t = _oracle_frame(dict(scene=scenes[k], camera=cam), falloff, tile_cull, backward=False)
        per_req.append(sum(t.values()))
        tot_px += cam.width * cam.height
    legs["workload4_requests"] = {"mpix_s": round(tot_px / sum(per_req) / 1e6, 5),
                                  "mean_ms_per_request": round(1e3 * float(np.mean(per_req)), 1),
                                  "p99_ms_per_request": round(1e3 * float(np.percentile(per_req, 99)), 1),
                                  "requests": len(reqs),
                                  "note": "64 whole requests of the serving recipe (scenes drawn on the host), "
                                          "rendered one after another"}
    log_fn(f"cpu: workload 4 requests {legs['workload4_requests']}")
    return {"value": legs["workload2_fwd_bwd"]["mpix_s"], "unit": "Mpix/s", "cores": cores, "kind": "oracle",
            "sample": "one whole 3M-splat 1920x1080 forward+backward frame on the oracle (preprocess, keys, "
                      f"per-pixel render and reverse pass, binary64 chain rule): {head_s:.1f} s",
            "cpu_model": cpu_model, "legs": legs}


def serving_bench(dev, n_req, log_fn):
    """Batched vs one-request-at-a-time serving over 8 resident scenes (13.7M splats, SH degree 3) at
    mixed resolutions: closed-loop capacity of each, then Poisson arrivals at 0.5, 0.9 and 1.2 times
    the sequential capacity (0.9 is the headline).  Both servers run the same kernels."""
    import torch
    from paper_2402_10128_amd import synth
    from paper_2402_10128_amd.serve import Server, run_stream
    scenes = [synth.scene_clusters_device(n, 1004 + 10 * i, dev) for i, n in enumerate(synth.SERVING_SIZES)]
    torch.cuda.synchronize()
    res = list(synth.SERVING_RESOLUTIONS)
    reqs = synth.serving_requests(n_req, len(scenes), res, seed=2000)
    sizes = [c.width * c.height * 3 for _, c in reqs]
    flat = torch.zeros(sum(sizes), dtype=torch.float32, device=dev)
    outs, o = [], 0
    for (_, c), sz in zip(reqs, sizes):
        outs.append(flat[o:o + sz].view(c.height, c.width, 3))
        o += sz
    pool_bytes = 8 << 30

    def server(sequential):
        s = Server(pool_bytes, max_slots=16, queue_capacity=max(4096, n_req + 16), sequential=sequential,
                   device=dev)
        ids = [s.add_scene(sc) for sc in scenes]
        return s, [(ids[k], cam) for k, cam in reqs]

    def summary(r):
        return {k: round(r[k], 3) for k in ("p50_ms", "p99_ms", "mean_ms", "mpix_s", "mean_batch")}

    out = {"workload": "8 resident scenes of 0.2/0.5/1/1/2/2/3/4M splats (64 clusters, SH degree 3), "
                       "orbit cameras, resolution uniform over 256x256/512x512/1280x720/1920x1080",
           "requests_per_rate": n_req, "pool_bytes": pool_bytes, "max_slots": 16}
    sat = {}
    n_sat = min(n_req, 400)
    for mode in ("sequential", "batched"):
        s, rq = server(mode == "sequential")
        with s:
            run_stream(s, rq[:32], outs[:32], None)    # warm-up
            r = run_stream(s, rq[:n_sat], outs[:n_sat], None)
        t_s = (max(x["t_done_ns"] for x in r["infos"]) - min(x["t_submit_ns"] for x in r["infos"])) / 1e9
        sat[mode] = dict(summary(r), req_s=round(n_sat / t_s, 2))
        log_fn(f"serving saturation {mode}: {sat[mode]}")
    mu_seq = sat["sequential"]["req_s"]
    out["saturation"] = sat
    out["mu_seq_req_s"] = mu_seq
    rates = []
    for f in (0.5, 0.9, 1.2):
        row = {"load": f, "rate_req_s": round(f * mu_seq, 2)}
        for mode in ("sequential", "batched"):
            s, rq = server(mode == "sequential")
            with s:
                r = run_stream(s, rq, outs, f * mu_seq, seed=int(f * 100))
            assert r["all_done"], f"serving run at load {f} ({mode}) did not complete every request"
            row[mode] = summary(r)
            log_fn(f"serving load {f} {mode}: {row[mode]}")
        rates.append(row)
    out["poisson"] = rates
    head = next(r for r in rates if r["load"] == 0.9)
    out["headline_load_0.9"] = {"batched_p50_ms": head["batched"]["p50_ms"], "batched_p99_ms": head["batched"]["p99_ms"],
                                "batched_mpix_s": head["batched"]["mpix_s"],
                                "sequential_p50_ms": head["sequential"]["p50_ms"],
                                "sequential_p99_ms": head["sequential"]["p99_ms"],
                                "sequential_mpix_s": head["sequential"]["mpix_s"]}
    del flat, outs, scenes
    torch.cuda.empty_cache()
    return out


def train_step_bench(dev, cfg, falloff, tile_cull, nsteps, warmup):
    """The full optimisation step (frequency mask at omega = it / 40000, render, 0.3 L1 + 0.2 SSIM +
    0.5 masked L1, adjoint with Adam fused into the preprocess backward) on a fresh copy of the scene; the key
    count is taken from the device against a frame capacity with headroom (no host sync inside the step)."""
    import torch
    from paper_2402_10128_amd import ges as G
    from paper_2402_10128_amd.train import TrainConfig, TrainStep
    sc, cam = cfg["scene"], cfg["camera"]
    scene = {k: torch.as_tensor(np.ascontiguousarray(v, np.float32)).to(dev) for k, v in sc.arrays().items()}
    target = torch.as_tensor(cfg["target"]).to(dev)
    ts = TrainStep(scene, cam, target, TrainConfig(falloff=falloff, tile_cull=tile_cull))
    it = 1
    for _ in range(max(1, warmup)):
        ts.step(it, read_num_keys=True)
        it += 1
    torch.cuda.synchronize()
    G.ges_profile_enable(True)
    G.ges_profile_read(reset=True)
    for _ in range(min(nsteps, 5)):
        ts.step(it, read_num_keys=False)
        it += 1
    stages = G.ges_profile_read(reset=True)
    G.ges_profile_enable(False)
    per_stage = {name: round(ms / nl, 4) for name, (ms, nl) in stages.items() if nl}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(nsteps):
        ts.step(it, read_num_keys=False)
        it += 1
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / nsteps
    st = G.frame_arrays(ts.frame, sc.n)["stats"]
    if int(st[1]) != 0:
        raise RuntimeError("key capacity overflow during the optimisation-step timing")
    loss = float(ts.loss.cpu())
    W, H = cam.width, cam.height
    sh_k = (sc.sh_degree + 1) ** 2
    out = {"ms_per_step": round(ms, 4), "mpix_per_s": round(W * H / (ms / 1e3) / 1e6, 3), "iterations_run": it - 1,
           "last_loss": round(loss, 6), "stage_ms_per_launch": per_stage}
    for stage in ("adam", "ssim", "preprocess_backward"):
        if stage in per_stage:
            key = "preprocess_backward_adam" if stage == "preprocess_backward" else stage
            nbytes = algorithmic_bytes(key, sc.n, sh_k, 0, 0, 0, W * H)
            gbs = nbytes / (per_stage[stage] / 1e3) / 1e9
            out[key] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_launch": nbytes}
    del ts, scene
    torch.cuda.empty_cache()
    return out


def views_step_bench(dev, cfg, falloff, tile_cull, nsteps, warmup, views=4):
    """The optimisation step over several views of the scene (the workload's camera and views-1 more orbit
    cameras, one resolution): the views batched into one launch sequence against the same views rendered and
    back-propagated one after another (the same bits; checked on the parameters after the timed steps)."""
    import torch
    from paper_2402_10128_amd import synth
    from paper_2402_10128_amd.train import TrainConfig, TrainStep
    sc, cam = cfg["scene"], cfg["camera"]
    rng = np.random.default_rng(77)
    cams = [cam] + [synth.orbit_camera(rng, cam.width, cam.height) for _ in range(views - 1)]
    target = torch.as_tensor(cfg["target"]).to(dev)
    targets = [target] + [torch.flip(target, dims=[1 + (v % 2)]).contiguous() for v in range(views - 1)]
    out, params = {}, {}
    for batched in (True, False):
        scene = {k: torch.as_tensor(np.ascontiguousarray(v, np.float32)).to(dev) for k, v in sc.arrays().items()}
        ts = TrainStep(scene, cams, targets, TrainConfig(falloff=falloff, tile_cull=tile_cull, batch_views=batched))
        it = 1
        for _ in range(max(1, warmup)):
            ts.step(it, read_num_keys=True)
            it += 1
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(nsteps):
            ts.step(it, read_num_keys=False)
            it += 1
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / nsteps
        ts.check_keys()
        out["batched" if batched else "view_by_view"] = {
            "ms_per_step": round(ms, 4), "mpix_per_s": round(views * cam.width * cam.height / (ms / 1e3) / 1e6, 3)}
        params[batched] = scene
        del ts
    out["identical_parameters"] = all(torch.equal(params[True][k], params[False][k]) for k in params[True])
    out["views"] = views
    out["workload"] = f"{sc.n} splats, {views} views of {cam.width}x{cam.height}"
    del params
    torch.cuda.empty_cache()
    return out


def mixture_bench(dev, epochs, log_fn):
    """The paper's 1-D mixture sweep (4 models x 6 signals x 8 N x 20 runs x 2 weight modes on 1,000
    points) in one launch; reports problem-epochs/s, NaN runs and mean final losses per model, and the oracle's
    rate on a bounded sample."""
    import torch
    from paper_2402_10128_amd import ges as G
    from paper_2402_10128_amd import synth
    W = synth.mixture_workload(seed=0)
    P = len(W["problems"])
    probs = torch.from_numpy(W["problems"]).to(dev)
    tg = torch.from_numpy(W["targets"]).to(dev)
    par0 = torch.from_numpy(W["params"]).to(dev)
    par = par0.clone()
    G.ges_mix_fit(probs, tg, W["x0"], W["dx"], par, 10, 0.01)      # warm-up (short)
    par.copy_(par0)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    loss = G.ges_mix_fit(probs, tg, W["x0"], W["dx"], par, epochs, 0.01)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    loss = loss.cpu().numpy()
    pr = W["problems"]
    names = ["gmm", "dog", "log", "gef"]
    per_model = {}
    for k, name in enumerate(names):
        sel = pr[:, 0] == k
        fin = np.isfinite(loss[sel])
        per_model[name] = {"nan_runs": int((~fin).sum()), "runs": int(sel.sum()),
                           "mean_final_mse": float(np.mean(loss[sel][fin])) if fin.any() else None}
    # square signal (target 0), positive weights: mean final MSE per N, the paper's headline comparison
    square = {}
    for k, name in enumerate(names):
        row = {}
        for n in synth.MIX_NS:
            sel = (pr[:, 0] == k) & (pr[:, 1] == n) & (pr[:, 3] == 0) & (pr[:, 2] == 1)
            v = loss[sel]
            v = v[np.isfinite(v)]
            row[str(n)] = float(np.mean(v)) if len(v) else None
        square[name] = row
    # oracle on this host: a sample of problems for a few epochs, scaled to problem-epochs/s
    from oracle import mixture1d as MX
    x = W["x0"] + W["dx"] * np.arange(W["m"], dtype=np.float64)
    rng = np.random.default_rng(0)
    sample = rng.choice(P, 24, replace=False)
    t0 = time.perf_counter()
    pe = 0
    for p in sample:
        model, n, pos, tgt = (int(v) for v in pr[p])
        MX.fit(names[model], x, W["targets"][tgt].astype(np.float64), W["params"][p, :n].astype(np.float64),
               bool(pos), 20, 0.01)
        pe += 20
    cpu_rate = pe / (time.perf_counter() - t0)
    log_fn(f"mixture sweep: {P} problems x {epochs} epochs in {ms:.1f} ms")
    return {"problems": P, "epochs": epochs, "points": W["m"], "ms": round(ms, 3),
            "problem_epochs_per_s": round(P * epochs / (ms / 1e3), 1), "per_model": per_model,
            "square_positive_mean_final_mse_by_n": square,
            "cpu_baseline": {"value": round(cpu_rate, 2), "unit": "problem-epochs/s", "kind": "oracle",
                             "sample": "24 random problems of the sweep, 20 epochs each, binary64 numpy"}}


def variants_bench(dev, cfg, tile_cull, steps, log_fn):
    """The paper's shape-strength sweep (rho in 0.01..0.15, Table 'shape strength') and the approximate
    (PHI) against the exact (GEF) falloff on the same scene: keys, pairs and forward+backward step time."""
    import torch
    from paper_2402_10128_amd import ges as G
    sc, cam = cfg["scene"], cfg["camera"]
    t = {k: torch.as_tensor(v).to(dev) for k, v in sc.arrays().items()}
    s = G.splats_struct(t["means"], t["log_scales"], t["quats"], t["opacity_logits"], t["sh"], t["beta"])
    c = G.camera_struct(cam)
    W, H = cam.width, cam.height
    frame = G.Frame.create(s.n, W, H, dev)
    out = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
    dL = torch.full_like(out, 1e-6)
    grads = {k: torch.empty_like(v) for k, v in t.items()}
    res = []
    beta_orig = t["beta"].clone()
    # the exact modification 2 Gamma(3/b)/Gamma(1/b) is 240 at b = 0.5 (the scene's betas reach 0.5): it is
    # compared with the approximation on a copy whose betas are clipped to [1, 4] (phi_exact <= 4)
    for falloff, rho, clip in [(0, 0.01, False), (0, 0.05, False), (0, 0.1, False), (0, 0.15, False),
                               (1, 0.1, False), (0, 0.1, True), (2, 0.1, True)]:
        t["beta"].copy_(beta_orig.clamp(1.0, 4.0) if clip else beta_orig)
        p = G.params_struct(falloff, tile_cull, rho, (0.0, 0.0, 0.0))

        def step():
            k = G.ges_preprocess(s, c, p, frame.splat_ws, True)
            frame.ensure_keys(k)
            G.ges_render_forward(s, c, p, frame.splat_ws, frame.key_ws, k, frame.pixel_ws, out)
            G.ges_render_backward(s, c, p, frame.splat_ws, frame.key_ws, frame.pixel_ws, dL, grads)
            return k

        for _ in range(2):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            k = step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        st = G.frame_arrays(frame, s.n)["stats"]
        res.append({"falloff": ("phi", "gef", "phi_exact")[falloff], "rho": rho, "beta_clipped_1_4": clip,
                    "num_keys": int(k),
                    "pairs_composited": int(st[3]), "ms_per_step_with_key_readback": round(ms, 4)})
        log_fn(f"variant falloff={res[-1]['falloff']} rho={rho} clip={clip}: {ms:.3f} ms, {k} keys")
    del frame, t, grads, out, dL
    torch.cuda.empty_cache()
    return res


def fwd_bwd(dev, cfg, falloff, tile_cull, steps, warmup, log_fn):
    """Forward + loss + backward steps of one workload: the timed steps (no host synchronisation: the kernels
    take the key count from the device against the frame's capacity, checked afterwards), per-stage device
    times from a separate profiled pass, the dominant kernel's launch time over the timed steps, the pair
    counts and the same step with the key-count read-back."""
    import torch
    from paper_2402_10128_amd import ges as G
    sc, cam = cfg["scene"], cfg["camera"]
    t = {k: torch.as_tensor(v).to(dev) for k, v in sc.arrays().items()}
    target = torch.as_tensor(cfg["target"]).to(dev)
    W, H = cam.width, cam.height
    s = G.splats_struct(t["means"], t["log_scales"], t["quats"], t["opacity_logits"], t["sh"], t["beta"])
    c = G.camera_struct(cam)
    p = G.params_struct(falloff, tile_cull, 0.1, (0.0, 0.0, 0.0))
    frame = G.Frame.create(s.n, W, H, dev)
    masked = cfg.get("loss") == "l1+freq"
    mask = G.ges_freq_mask(target, cfg.get("omega", 0.75)) if masked else None
    lam_l1, lam_w = (0.5, 0.5) if masked else (1.0, 0.0)
    out = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
    dL = torch.empty_like(out)
    loss = torch.empty((), dtype=torch.float32, device=dev)
    loss_scratch = torch.empty(G.lib().ges_loss_scratch_bytes(), dtype=torch.uint8, device=dev)
    grads = {k: torch.empty_like(v) for k, v in t.items()}

    def step(readback):
        """One step.  readback=True reads the slot count back after the preprocess (a host sync in mid-step)
        and renders with exactly that capacity; readback=False renders with the frame's capacity and lets the
        kernels take the count from the device (an overflow would be flagged in the error word)."""
        if readback:
            k = G.ges_preprocess(s, c, p, frame.splat_ws, True)
            frame.ensure_keys(k)
        else:
            G.ges_preprocess(s, c, p, frame.splat_ws, False)
            k = frame.key_capacity
        frame.num_keys = k
        G.ges_render_forward(s, c, p, frame.splat_ws, frame.key_ws, k, frame.pixel_ws, out)
        G.ges_loss(out, target, mask, lam_l1, lam_w, dL, loss, loss_scratch)
        G.ges_render_backward(s, c, p, frame.splat_ws, frame.key_ws, frame.pixel_ws, dL, grads)

    def timed(nsteps, readback):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(nsteps):
            step(readback)
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / nsteps

    for _ in range(max(1, warmup)):
        step(True)
    torch.cuda.synchronize()
    C = int(frame.num_keys)
    G.ges_profile_enable(True)
    G.ges_profile_read(reset=True)
    timed(min(steps, 5), False)
    stages = G.ges_profile_read(reset=True)
    per_stage = {name: round(ms / nl, 4) for name, (ms, nl) in stages.items() if nl}
    dominant = max(per_stage, key=per_stage.get)
    G.ges_profile_select([dominant])
    t_host0 = time.perf_counter()
    ms_step = timed(steps, False)
    t_host = time.perf_counter() - t_host0
    dom = G.ges_profile_read(reset=True)[dominant]
    G.ges_profile_enable(False)
    fa = G.frame_arrays(frame, s.n)
    st = fa["stats"]
    if int(st[1]) != 0:
        raise RuntimeError(f"key capacity overflow during timing: error word {int(st[1])}")
    ms_step_readback = timed(min(steps, 5), True)
    vis = int((fa["records"][:, 15].view(np.uint32) > 0).sum())
    m = dict(ms_step=ms_step, ms_step_readback=ms_step_readback, host_ms=t_host / steps * 1e3, per_stage=per_stage,
             dominant=dominant, dominant_ms=dom[0] / dom[1], n=s.n, sh_k=(sc.sh_degree + 1) ** 2, K=int(st[0]),
             C=C, L=vis, px=W * H, R=fa.get("rows_stored", 0), pairs_exam=int(st[2]), pairs_blend=int(st[3]),
             bwd_walk=int(fa["n_contrib"].astype(np.int64).sum()),
             max_list=int((fa["ranges"][:, 1].astype(np.int64) - fa["ranges"][:, 0]).max(initial=0)))
    log_fn(f"{W}x{H} n={s.n}: {ms_step:.3f} ms/step, {W * H / ms_step / 1e3:.1f} Mpix/s, K={m['K']} slots={C}, "
           f"stages {json.dumps(per_stage)}")
    del frame, t, grads, out, dL
    torch.cuda.empty_cache()
    return m


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1 "
                                   "(sharding across GPUs is not implemented)"}))
        sys.exit(2)
    import torch
    from paper_2402_10128_amd import ges as G
    from paper_2402_10128_amd import synth
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    G.lib()
    dev = torch.device("cuda:0")
    falloff = 0 if args.falloff == "phi" else 1
    tile_cull = 0 if args.tile_cull == "square" else 1
    log(f"generating workload {args.workload}")
    cfg = synth.make_config(args.workload)
    sc, cam = cfg["scene"], cfg["camera"]
    W, H = cam.width, cam.height
    log(f"timing {args.steps} steps")
    m = fwd_bwd(dev, cfg, falloff, tile_cull, args.steps, args.warmup, log)
    ms_step, per_stage, dominant, avg_ms = m["ms_step"], m["per_stage"], m["dominant"], m["dominant_ms"]
    mpix = W * H / (ms_step / 1e3) / 1e6
    rooflines = stage_rooflines(per_stage, m, falloff, args.workload)
    dom = dict(rooflines[dominant])
    if dominant in RASTER_STAGES:
        roof = {"bound": "alu", "achieved": dom["achieved"], "peak": VALU_PEAK_TOPS, "unit": "Tlane-op/s",
                "frac": round(dom["achieved"] / VALU_PEAK_TOPS, 5), "kernel": dominant,
                "algorithmic_lane_ops_per_launch": dom["algorithmic_lane_ops"],
                "flop": {"achieved": dom["flop_tflops"], "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": dom["flop_frac_of_157.3"]}}
        if "issued_over_algorithmic" in dom:
            roof["issued_over_algorithmic"] = dom["issued_over_algorithmic"]
    else:
        roof = {"bound": "hbm", "achieved": dom["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dom["frac"], "kernel": dominant, "algorithmic_bytes_per_launch": dom["algorithmic_bytes"]}
    roof["traffic"] = read_counter(dominant, args.workload, "hbm_bytes_per_launch")
    roof["avg_launch_ms"] = avg_ms

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    others, cfgs = {}, {args.workload: cfg}
    if not args.no_other_workloads:
        for wl in (1, 3):
            if wl == args.workload:
                continue
            log(f"workload {wl} forward+backward")
            cfgs[wl] = synth.make_config(wl)
            mw = fwd_bwd(dev, cfgs[wl], falloff, tile_cull, min(args.steps, 10), min(args.warmup, 2), log)
            cw = cfgs[wl]["camera"]
            others[str(wl)] = {"workload": {1: "1M splats 1600x1040", 3: "5M splats 1920x1080 heavy overlap"}[wl],
                               "ms_per_step": round(mw["ms_step"], 4),
                               "mpix_s": round(cw.width * cw.height / (mw["ms_step"] / 1e3) / 1e6, 3),
                               "num_keys": mw["K"], "candidate_slots": mw["C"], "max_list": mw["max_list"],
                               "stage_ms_per_launch": mw["per_stage"],
                               "stage_roofline": stage_rooflines(mw["per_stage"], mw, falloff, wl)}
    train = None
    if not args.no_train_step:
        log("optimisation step (mask + render + L1/SSIM/frequency loss + adjoint + Adam)")
        train = train_step_bench(dev, cfg, falloff, tile_cull, args.steps, args.warmup)
        log(f"optimisation step {train['ms_per_step']:.3f} ms: " + json.dumps(train["stage_ms_per_launch"]))
    views_step = None
    if not args.no_train_step and not args.no_views_step:
        log("multi-view optimisation step (4 views batched vs one after another)")
        views_step = views_step_bench(dev, cfg, falloff, tile_cull, min(args.steps, 10), args.warmup)
        log(f"views step: {json.dumps(views_step)}")
    variants = None
    if not args.no_variants:
        log("shape-strength sweep and falloff comparison")
        variants = variants_bench(dev, cfg, tile_cull, min(args.steps, 5), log)
    mixture = None
    if not args.no_mixture:
        log("1-D mixture sweep")
        mixture = mixture_bench(dev, args.mixture_epochs, log)
    serving = None
    if not args.no_serving:
        log("serving (workload 4)")
        serving = serving_bench(dev, args.serve_requests, log)

    cpu = None
    if not args.no_cpu_baseline:
        log("oracle CPU baseline")
        try:
            for wl in (0, 1, 2, 3):
                if wl not in cfgs:
                    cfgs[wl] = synth.make_config(wl)
            cpu = cpu_baseline(cfgs, falloff, tile_cull, log)
        except Exception as e:  # reported, never silently replaced
            cpu = {"error": repr(e)}

    names = {0: "1k splats 64x64", 1: "1M splats 1600x1040", 2: "3M splats 1920x1080 training step",
             3: "5M splats 1920x1080 heavy overlap"}
    res = {
        "metric": "fwd+bwd Mpix/s at 3M splats 1080p; render p50/p99 ms under batched load",
        "value": round(mpix, 3),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "ms_per_step_with_key_readback": round(m["ms_step_readback"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": names[args.workload], "splats": m["n"], "width": W, "height": H,
                   "sh_degree": sc.sh_degree, "falloff": args.falloff, "tile_cull": args.tile_cull,
                   "loss": cfg.get("loss"), "num_keys": m["K"], "candidate_slots": m["C"],
                   "pairs_examined_fwd": m["pairs_exam"], "pairs_composited": m["pairs_blend"],
                   "pairs_walked_bwd": m["bwd_walk"], "stage_ms_per_launch": per_stage,
                   "stage_roofline": rooflines},
        "roofline": roof,
        "cpu_baseline": cpu,
        "other_workloads": others,
        "train_step": train,
        "views_step": views_step,
        "variants": variants,
        "mixture_sweep": mixture,
        "serving": serving,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
