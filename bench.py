#!/usr/bin/env python3
"""Throughput of the SGM hot path on one MI355X.

One step = the whole path on one synthetic 1280x720 road pair already
resident in HBM: census of both images + matching cost (sgm_cost), the
8-direction aggregation (sgm_aggregate_paths) and the summed-cost
selection with sub-pixel refinement (sgm_wta_paths).  Disparities 0..127,
census 7x7, P1 = 10, P2 = 120.

Prints one JSON line with the throughput in Mdisp-evals/s (pixels x
disparities per second), the roofline position of the dominant kernel
(timed live with HIP events on the stream it runs on) and the CPU oracle
timed on the host for reference.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# VALU: 256 CUs x 64 lanes x 2.4 GHz lane-ops; packed 16-bit ops do two each
VALU_PEAK_TOPS_U16 = 256 * 64 * 2.4e9 * 2 / 1e12

METRIC = "SGM Mdisp-evals/s at 1280x720x128; learned-window vs plain at same bad-pixel %"

WORKLOADS = {
    "road1280": "1280x720 uint8 road pair, census 7x7, 8 paths, P1=10, P2=120, disparities 0-127",
    "road320": "320x240 uint8 road pair, census 5x5, 4 paths, P1=10, P2=120, disparities 0-31",
    "road1280_pt": "1280x720 uint8 road pair, census 7x7, 8 paths, P1=10, P2=120, per-row windows of 24 "
                   "disparities centred on the road model (perspective-transformed form)",
    "road_batch64": "64 uint8 road pairs in one batch: 24 x 640x480 (disparities 0-63), "
                    "24 x 1280x720 (0-127), 16 x 1920x1080 (0-191); census 7x7, 8 paths, "
                    "P1=10, P2=120; roll U(0,4) deg",
}

# pairs of each batched workload: (generator config, count)
BATCHES = {
    "road_batch64": [("road640", 24), ("road1280", 24), ("road1920", 16)],
    "road1280": [("road1280", 1)],
}


def kernel_source_digest() -> str:
    """Digest of the device code (kernels and the shared device header)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2012_10802_amd", "csrc")
    for name in ("sgm_device.h", "sgm_kernels.hip", "sgm_batch.hip"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_traffic(workload: str):
    """HBM bytes per aggregation launch from the committed rocprofv3 counter
    summary, or None when the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "aggregate_%s_counters.md" % workload)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    sha = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", text)
    val = re.search(r"traffic_bytes_per_launch:\s*([0-9.e+]+)", text)
    if not sha or not val or sha.group(1) != kernel_source_digest():
        return None
    return float(val.group(1))


def eval_mask(p, w, r, d_lo=None):
    """Pixels scored for accuracy: road, ground truth inside the window and
    away from the image border (census half-window r)."""
    import numpy as np
    H, W = p.gt.shape
    uu = np.arange(W)[None, :]
    lo = np.zeros((H, 1)) if d_lo is None else np.asarray(d_lo, np.float64)[:, None]
    m = p.road & (p.gt >= lo) & (p.gt < lo + w - 1) & (uu - p.gt >= r)
    m[:r] = m[-r:] = False
    m[:, :r] = m[:, -r:] = False
    return m


def host_cpu():
    """The host the CPU oracle runs on: CPU model, logical CPUs, CPUs this
    process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def _median_time(fn, runs):
    import numpy as np
    ts = []
    for _ in range(runs):
        t = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t)
    return float(np.median(ts)), [round(x, 3) for x in ts]


def cpu_baseline_frame(pair, n, w, R, p1, p2, d_lo, runs=3, log=None):
    """The C oracle as it stands on the same frame: its own threading (one
    thread per path direction, so at most R), median of `runs` whole-frame
    runs; and single-threaded on the middle quarter of the rows (same width
    and window), median of `runs`.  Rates in Mdisp-evals/s over the evals
    each run covers."""
    import oracle
    H, W = pair.left.shape
    dl = None if d_lo is None else d_lo
    threads = min(R, oracle.num_threads())
    med, ts = _median_time(lambda: oracle.sgm(pair.left, pair.right, n, w, R, p1, p2, dl), runs)
    if log:
        log("cpu oracle, %d threads: %s s" % (threads, ts))
    v0, v1 = 3 * H // 8, 5 * H // 8
    band_dl = None if dl is None else dl[v0:v1]
    saved = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        med1, ts1 = _median_time(lambda: oracle.sgm(pair.left[v0:v1], pair.right[v0:v1], n, w, R, p1, p2, band_dl),
                                 runs)
    finally:
        oracle.set_num_threads(saved)
    if log:
        log("cpu oracle, 1 thread, rows %d..%d: %s s" % (v0, v1 - 1, ts1))
    evals = W * H * w
    return {"value": round(evals / med / 1e6, 3), "unit": "Mdisp-evals/s", "cores": threads, "kind": "oracle",
            "sample": "the whole %dx%dx%d frame through the C oracle (census, cost, %d paths, selection), "
                      "median of %d runs: %s s; the oracle's threads are its path directions"
                      % (W, H, w, R, runs, ts),
            "single_thread": {"value": round(W * (v1 - v0) * w / med1 / 1e6, 3), "unit": "Mdisp-evals/s",
                              "cores": 1,
                              "sample": "rows %d..%d (the middle quarter, %dx%dx%d), median of %d runs: %s s"
                                        % (v0, v1 - 1, W, v1 - v0, w, runs, ts1)},
            "host": host_cpu()}


def emit(record, args):
    """Print the one JSON line (and append it to --jsonl when given)."""
    line = json.dumps(record)
    print(line, flush=True)
    if getattr(args, "jsonl", None):
        with open(args.jsonl, "a") as f:
            f.write(line + "\n")


def run_batch(args):
    """Batch mode: the whole batch as one captured graph per step; per-stage
    kernel times from eagerly enqueued runs timed with HIP events on the
    same stream; the CPU oracle on a few pairs of each size class,
    extrapolated in evals."""
    import numpy as np
    import torch

    from paper_2012_10802_amd import sgm, synth

    log = lambda msg: print(msg, file=sys.stderr, flush=True)  # noqa: E731
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    pairs, evals, renders, hosts = [], 0, {}, {}
    for name, count in BATCHES[args.workload]:
        c = synth.CONFIGS[name]
        for j in range(count):
            k = (name, j % args.unique)
            if k not in renders:
                seed = args.seed + 97 * j
                p = synth.make_pair(synth.scene_for_config(name, seed), seed)
                hosts[k] = p
                renders[k] = (torch.from_numpy(p.left).to(dev), torch.from_numpy(p.right).to(dev))
            L, R = renders[k]
            pairs.append({"left": L, "right": R, "ndisp": c["ndisp"]})
            evals += c["width"] * c["height"] * c["ndisp"]
    c0 = synth.CONFIGS[BATCHES[args.workload][0][0]]
    n_cen, R_paths, p1, p2 = c0["census"], c0["npaths"], c0["p1"], c0["p2"]
    b = sgm.Batch(pairs, census=n_cen, npaths=R_paths, p1=p1, p2=p2, device=dev)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        tuning = b.autotune(args.tune_cache)
        b.capture(stream)
        for _ in range(args.warmup):
            b.launch(stream)
        stream.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(args.steps):
            b.launch(stream)
        e1.record(stream)
        stream.synchronize()
        t1 = time.perf_counter()
        # the same kernels enqueued eagerly, stages bracketed by HIP events
        stage = np.array([b.run_timed(stream) for _ in range(args.steps)])
    ms = (t1 - t0) * 1e3 / args.steps
    copy_calibration(args, dev)
    census_ms, cost_ms, agg_ms, wta_ms = (float(x) for x in stage.mean(axis=0))
    log("batch stages (ms, mean of %d): census %.3f cost %.3f aggregate %.3f select %.3f"
        % (args.steps, census_ms, cost_ms, agg_ms, wta_ms))
    # algorithmic bytes of the persistent aggregation: every direction reads
    # the cost volume once and writes its uint8 volume (R (1 + 1) B/eval);
    # the selection reads the R volumes back (R B/eval)
    agg_bpe, wta_bpe = R_paths * 2, R_paths
    agg_gbs = evals * agg_bpe / (agg_ms * 1e-3) / 1e9
    wta_gbs = evals * wta_bpe / (wta_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(agg_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(agg_gbs / HBM_PEAK_GBS, 4), "traffic": counter_traffic(args.workload),
                "bytes_per_eval": agg_bpe, "bytes_per_launch": evals * agg_bpe, "kernel": "k_aggregate_batch",
                "launch_ms": round(agg_ms, 4),
                "note": "every volume of the batch (29 GB) exceeds the 256 MB MALL: HBM-clean"}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_batch(args, hosts, n_cen, R_paths, p1, p2, log)
    out = {
        "metric": METRIC,
        "value": round(evals / (ms * 1e-3) / 1e6, 1),
        "unit": "Mdisp-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "ms_per_step_events": round(e0.elapsed_time(e1) / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "storage": "uint8 cost and per-direction volumes, packed u16 arithmetic",
        "data": "synthetic",
        "mode": "batch (one persistent aggregation launch, graph replay)",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload],
                   "pairs": len(pairs), "evals_per_step": evals, "unique_renders": len(renders)},
        "tuning": {"waves_per_cu": tuning[0], "order": ["longest-first", "pair-major",
                                                        "direction-major"][tuning[1]],
                   "lanes_per_scanline": (tuning[2] or 16) if len(tuning) > 2 else 16,
                   "horizontal_lanes_per_scanline": 16},
        "roofline": roofline,
        "kernels_ms": {"census": round(census_ms, 4), "cost": round(cost_ms, 4), "aggregate": round(agg_ms, 4),
                       "wta": round(wta_ms, 4),
                       "timing": "eager runs of the same kernels, HIP events between stages on the run's "
                                 "stream, mean of %d" % args.steps},
        "wta_hbm": {"bytes_per_eval": wta_bpe, "achieved": round(wta_gbs, 1), "unit": "GB/s",
                    "frac": round(wta_gbs / HBM_PEAK_GBS, 4)},
        # whole step: cost written once and read by each of the 8 directions,
        # 8 uint8 volumes written and read back by the selection
        "step_hbm": {"bytes_per_eval": 25, "achieved": round(evals * 25 / (ms * 1e-3) / 1e9, 1), "unit": "GB/s",
                     "frac": round(evals * 25 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "cpu_baseline": cpu,
        "paper_context": PAPER_CONTEXT,
        "kernel_source_sha256": kernel_source_digest(),
    }
    emit(out, args)


# The paper's own timings, quoted as context only: they were taken on
# another GPU, and its frame size and disparity range are not stated, so
# they convert to no Mdisp-evals/s figure and set no target.
PAPER_CONTEXT = {
    "hardware": "NVIDIA RTX 2080 Ti (CUDA)",
    "gpt_sgm_ms_per_frame": 10.1,
    "gpt_sgm_source": "Sec. III-A (disparity estimation: perspective-transformed SGM on KITTI road pairs)",
    "whole_detector_ms_per_frame": 47.48,
    "whole_detector_source": "Table II (all three datasets; SLIC the largest share)",
    "comparable": False,
    "note": "frame size and disparity range not stated: context only, not a baseline",
}


def cpu_baseline_batch(args, hosts, n, R, p1, p2, log):
    """The C oracle on `--cpu-pairs-per-size` pairs of each size class of the
    batch (cycling over the renders the batch uses), at the oracle's own
    threads; the batch's CPU time is extrapolated linearly in evals from the
    median rate of each class."""
    import numpy as np

    import oracle
    from paper_2012_10802_amd import synth
    threads = min(R, oracle.num_threads())
    classes, total_s, total_evals = [], 0.0, 0
    for name, count in BATCHES[args.workload]:
        c = synth.CONFIGS[name]
        rend = [hosts[k] for k in sorted(hosts) if k[0] == name]
        ts = []
        for j in range(args.cpu_pairs_per_size):
            p = rend[j % len(rend)]
            t = time.perf_counter()
            oracle.sgm(p.left, p.right, n, c["ndisp"], R, p1, p2)
            ts.append(time.perf_counter() - t)
        pe = c["width"] * c["height"] * c["ndisp"]
        med = float(np.median(ts))
        log("cpu oracle %s: %s s per pair" % (name, [round(x, 2) for x in ts]))
        classes.append({"class": "%dx%dx%d" % (c["width"], c["height"], c["ndisp"]), "pairs_in_batch": count,
                        "timed_pairs": len(ts), "s_per_pair": [round(x, 3) for x in ts],
                        "value": round(pe / med / 1e6, 3)})
        total_s += count * med
        total_evals += count * pe
    return {"value": round(total_evals / total_s / 1e6, 3), "unit": "Mdisp-evals/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d pairs of each size class through the C oracle (the oracle's threads are its path "
                      "directions); the %d-pair batch's time extrapolated linearly in evals from each class's "
                      "median: %.1f s per batch" % (args.cpu_pairs_per_size, sum(k for _, k in BATCHES[args.workload]),
                                                     total_s),
            "per_class": classes, "host": host_cpu()}


def learned_vs_plain(args, log=None):
    """The learned-window form against plain full-range SGM on held-out
    1920x1080 road pairs (disparities 0..191, census 7x7, 8 paths), batches
    of 16: wall time per batch and the bad-pixel rate (> 1 px) against the
    generator's ground truth over the evaluation mask."""
    import numpy as np
    import torch

    from paper_2012_10802_amd import learned_window as LW
    from paper_2012_10802_amd import sgm, synth

    dev = torch.device("cuda:0")
    c = synth.CONFIGS["road1920"]
    W, H, D = c["width"], c["height"], c["ndisp"]
    n_cen, R, p1, p2 = c["census"], c["npaths"], c["p1"], c["p2"]
    B = 16
    r = n_cen // 2
    net = LW.WindowNet.load(args.weights, device=dev)
    L = torch.empty((B, H, W), dtype=torch.uint8, device=dev)
    Rt = torch.empty_like(L)
    plain = sgm.Batch([dict(left=L[i], right=Rt[i], ndisp=D) for i in range(B)], census=n_cen, npaths=R,
                      p1=p1, p2=p2, device=dev)
    lw = LW.LearnedWindowMatcher(W, H, batch=B, ndisp=D, window=16, census=n_cen, npaths=R, p1=p1, p2=p2,
                                 net=net, tau=args.tau, fallback_margin=args.fallback_margin, device=dev)
    stream = torch.cuda.Stream()
    uu = torch.arange(W, device=dev)[None, :]
    tot = {"pix": 0, "bad_plain": 0, "bad_learned": 0, "miss": 0, "conf_pix": 0, "fallback": 0,
           "rect_area": 0, "fb_scored": 0, "fb_bad_plain": 0, "fb_bad_learned": 0, "fb_differ": 0}
    t_plain, t_learned, stages, rect_shapes = [], [], [], []
    ev_a, ev_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev_stage = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
    nb = max(1, args.eval_pairs // B)
    with torch.cuda.stream(stream):
        L.zero_()
        Rt.zero_()
        plain.autotune(stream=stream)  # both paths with tuned launch shapes
        plain.capture(stream)
        for b in range(nb):
            gts, masks = [], []
            for j in range(B):
                sd = args.seed + 10_000_000 + b * B + j
                l, rr, gt, road = synth.make_pair_torch(synth.scene_for_config("road1920", sd), sd, device=dev)
                L[j].copy_(l)
                Rt[j].copy_(rr)
                m = road & (gt < D - 1) & ((uu - gt) >= r)
                m[:r] = False
                m[-r:] = False
                m[:, :r] = False
                m[:, -r:] = False
                gts.append(gt)
                masks.append(m)
            stream.synchronize()
            # HIP events on the stream around each batch (the learned form
            # includes the time the stream waits while the host plans the
            # fallback rectangles from the window maps)
            reps = []
            for k in range(args.lw_reps + 1):
                stream.synchronize()
                ev_a.record(stream)
                plain.launch(stream)
                ev_b.record(stream)
                stream.synchronize()
                if k:
                    reps.append(ev_a.elapsed_time(ev_b) * 1e-3)
            t_plain.append(float(np.median(reps)))
            reps = []
            for k in range(args.lw_reps + 1):
                stream.synchronize()
                lw.match(L, Rt, stream, events=ev_stage)
                stream.synchronize()
                if k:
                    reps.append(ev_stage[0].elapsed_time(ev_stage[6]) * 1e-3)
                    stages.append([ev_stage[i].elapsed_time(ev_stage[i + 1]) for i in range(6)])
            t_learned.append(float(np.median(reps)))
            for j in range(B):
                m = masks[j]
                e_p = (plain.disp_sub[j] - gts[j]).abs()
                e_l = (lw.dsub[j] - gts[j]).abs()
                tot["pix"] += int(m.sum())
                tot["bad_plain"] += int(((e_p > 1.0) & m).sum())
                tot["bad_learned"] += int(((e_l > 1.0) & m).sum())
                conf = m & (lw.mask[j] == 0)
                d = plain.disp_int[j].int()
                lo = lw.lo[j]
                tot["miss"] += int((conf & ((d < lo) | (d >= lo + 16))).sum())
                tot["conf_pix"] += int(conf.sum())
                tot["fallback"] += int(lw.nfallback[j])
                tot["rect_area"] += sum((y1 - y0) * (x1 - x0) for y0, y1, x0, x1 in lw.last_rects[j])
                for y0, y1, x0, x1 in lw.last_rects[j]:
                    rect_shapes.append((y1 - y0, x1 - x0, x0 == 0))
                # fallback pixels: the crop's full-range SGM against full-frame full-range SGM
                fbm = lw.mask[j] > 0
                tot["fb_differ"] += int((fbm & (lw.dint[j] != plain.disp_int[j])).sum())
                fs = fbm & m
                tot["fb_scored"] += int(fs.sum())
                tot["fb_bad_plain"] += int(((e_p > 1.0) & fs).sum())
                tot["fb_bad_learned"] += int(((e_l > 1.0) & fs).sum())
            if log:
                log("learned-window batch %d/%d: plain %.2f ms, learned %.2f ms"
                    % (b + 1, nb, t_plain[-1] * 1e3, t_learned[-1] * 1e3))
    npairs = nb * B
    st = np.array(stages).mean(axis=0)
    stage_ms = {name: round(float(v), 4) for name, v in zip(LW.LearnedWindowMatcher.STAGES, st)}
    # algorithmic bytes per stage (per batch of B pairs): full-resolution
    # pixels P, quarter-resolution pixels Pc
    P, Pc, Dc = B * W * H, B * (W // 4) * (H // 4), D // 4
    stage_bytes = {
        # both images read, both reductions written
        "reduce": 2 * P + 2 * Pc,
        # plain SGM at quarter scale: 25 B per eval (cost written once and
        # read by 8 directions, 8 uint8 volumes written and read back)
        "coarse_sgm": 25 * Pc * Dc,
        # input prep (5 B in, 32 B out), then the four layers in one launch
        # (32 B in, 8 B out: the hidden activations stay on chip), per
        # quarter-resolution pixel
        "network": Pc * (37 + 40),
        # coarse disparity and two outputs per quarter pixel in, window
        # start (4 B) and fallback flag (1 B) out per pixel
        "window_map": Pc * 12 + P * 5,
        # census (2 B in, 16 B out), cost (16 B codes + 4 B lo in, 16 B out
        # + the window start as a byte), 8 directions x (16 B cost + 1 B
        # window start in, 16 B out), selection (8 x 16 B + 4 B lo in, 6 B
        # out), per pixel
        "windowed_sgm": P * (18 + 37 + 8 * 33 + 138),
    }
    stage_roof = {k: {"bytes": v, "achieved_gbs": round(v / (stage_ms[k] * 1e-3) / 1e9, 1),
                      "frac": round(v / (stage_ms[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
                  for k, v in stage_bytes.items() if stage_ms.get(k, 0) > 0}
    # the network's matrix work: 4 layers x 9 taps x 16 x 16 multiply-adds
    # per quarter-resolution pixel, against the dense bf16 MFMA peak
    if stage_ms.get("network", 0) > 0:
        tflops = Pc * 4 * 9 * 16 * 16 * 2 / (stage_ms["network"] * 1e-3) / 1e12
        stage_roof["network_mfma"] = {"flop": Pc * 4 * 9 * 16 * 16 * 2, "achieved_tflops": round(tflops, 1),
                                      "peak_tflops": 2500.0, "frac": round(tflops / 2500.0, 4)}
    bp = 100.0 * tot["bad_plain"] / tot["pix"]
    bl = 100.0 * tot["bad_learned"] / tot["pix"]
    return {
        "workload": "%d held-out 1920x1080 road pairs in batches of %d, disparities 0-191, census 7x7, "
                    "8 paths, P1=10, P2=120" % (npairs, B),
        "ms_per_batch_plain": round(1e3 * float(np.mean(t_plain)), 3),
        "ms_per_batch_learned": round(1e3 * float(np.mean(t_learned)), 3),
        "speedup": round(float(np.mean(t_plain)) / float(np.mean(t_learned)), 3),
        "bad_1px_pct_plain": round(bp, 4),
        "bad_1px_pct_learned": round(bl, 4),
        "bad_1px_delta_points": round(bl - bp, 4),
        "fallback_pixel_pct": round(100.0 * tot["fallback"] / (npairs * W * H), 4),
        "fallback_area_pct": round(100.0 * tot["rect_area"] / (npairs * W * H), 3),
        "window_miss_pct_vs_full_range": round(100.0 * tot["miss"] / max(1, tot["conf_pix"]), 4),
        "fallback_vs_full_frame": {
            "fallback_pixels": tot["fallback"],
            "integer_disparity_differs_pct": round(100.0 * tot["fb_differ"] / max(1, tot["fallback"]), 4),
            "scored_fallback_pixels": tot["fb_scored"],
            "bad_1px_pct_full_frame": round(100.0 * tot["fb_bad_plain"] / max(1, tot["fb_scored"]), 4),
            "bad_1px_pct_crop": round(100.0 * tot["fb_bad_learned"] / max(1, tot["fb_scored"]), 4),
            "note": "fallback pixels take full-range SGM of a crop around them; compared here with "
                    "full-range SGM of the whole frame on the same pixels"},
        "fallback_rectangles": {
            "per_pair": round(len(rect_shapes) / max(1, nb * B), 2),
            "mean_rows": round(float(np.mean([r[0] for r in rect_shapes])), 1) if rect_shapes else 0,
            "mean_cols": round(float(np.mean([r[1] for r in rect_shapes])), 1) if rect_shapes else 0,
            "at_left_edge_pct": round(100.0 * float(np.mean([r[2] for r in rect_shapes])), 1) if rect_shapes else 0},
        "stages_ms": stage_ms,
        "stage_roofline": stage_roof,
        "tau": args.tau,
        "fallback_margin": args.fallback_margin,
        "window": 16,
        "pixels_scored": tot["pix"],
        "timing": "HIP events on the stream around each batch (the learned form includes the stream's wait "
                  "while the host plans the fallback rectangles), median of %d after one warm-up, mean over "
                  "batches; stages from events between them" % args.lw_reps,
    }


def copy_calibration(args, dev):
    """One device-to-device copy of --copy-calibration-mb MiB: the reference
    kernel whose memory counters scale those of the measured kernels."""
    import torch
    if args.copy_calibration_mb:
        src = torch.ones(args.copy_calibration_mb << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst


def copy_reference(dev, mib=1024, reps=10):
    """Rate of a plain device-to-device copy of `mib` MiB (torch copy_,
    HIP events, median of `reps`): the bandwidth a streaming kernel can
    reach in practice, beside the 8 TB/s peak."""
    import numpy as np
    import torch
    src = torch.ones(mib << 20, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        dst.copy_(src)
        b.record()
    torch.cuda.synchronize()
    ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
    del src, dst
    return {"bytes": 2 * (mib << 20), "ms": round(ms, 4), "achieved": round(2 * (mib << 20) / (ms * 1e-3) / 1e9, 1),
            "unit": "GB/s", "kernel": "torch copy_ of %d MiB, device to device (read + write)" % mib}


def road_model_leg(args, log=None):
    """The road-model stages around the matcher on a batch of 16 full-range
    1920x1080 SGM disparity maps of generated road pairs: the fit of
    Sec. II-C (eq. (11), (12); road pixels from the generator's road mask),
    per-row windows of eq. (6) from the device fits and the disparity
    transformation of eq. (13).  Times each call with HIP events on the
    stream it runs on and reports the HBM rate of the two streaming kernels
    (fit: 4 B disparity + 1 B mask per pixel; transformation: 4 B in + 4 B
    out per pixel) and the fit's error against the scenes' own (a0, a1,
    phi)."""
    import math

    import numpy as np
    import torch

    from paper_2012_10802_amd import sgm, synth

    dev = torch.device("cuda:0")
    c = synth.CONFIGS["road1920"]
    W, H, n = c["width"], c["height"], 16
    L = torch.empty((n, H, W), dtype=torch.uint8, device=dev)
    R = torch.empty_like(L)
    mask = torch.empty((n, H, W), dtype=torch.uint8, device=dev)
    holes = torch.empty((n, H, W), dtype=torch.bool, device=dev)
    truth = []
    for i in range(n):
        seed = 3_000_000 + i
        sc = synth.scene_for_config("road1920", seed)
        l, r, gt, road = synth.make_pair_torch(sc, seed, device=dev)
        L[i].copy_(l)
        R[i].copy_(r)
        cols = torch.arange(W, device=dev)[None, :]
        mask[i].copy_((road & (cols - gt >= 4)).to(torch.uint8))
        a0, a1, phi = sc.road_params
        rows = torch.arange(H, device=dev, dtype=torch.float64)[:, None]
        plane = a0 + a1 * (math.cos(phi) * (rows - sc.cy) - math.sin(phi) * (cols.double() - sc.cx))
        holes[i].copy_(road & (gt.double() < plane - 1e-3))  # the generator's depressions
        truth.append(sc.road_params)
    batch = sgm.Batch([dict(left=L[i], right=R[i], ndisp=c["ndisp"]) for i in range(n)], census=c["census"],
                      npaths=c["npaths"], p1=c["p1"], p2=c["p2"], device=dev)
    batch.run()
    disp = torch.stack([batch.disp_sub[i] for i in range(n)]).contiguous()
    del batch, L, R
    fit = torch.empty((n, sgm.ROAD_FIT_WORDS), dtype=torch.float64, device=dev)
    ws = torch.empty(sgm.road_workspace_size(W, H, n), dtype=torch.uint8, device=dev)
    d_lo = torch.empty((n, H), dtype=torch.int32, device=dev)
    d2 = torch.empty_like(disp)
    torch.cuda.synchronize()

    nbins, delta_pd = 128, 2.36
    pd_res = torch.empty((n, sgm.POTHOLE_WORDS), dtype=torch.float64, device=dev)
    pd_ws = torch.empty(sgm.pothole_workspace_size(nbins, n), dtype=torch.uint8, device=dev)
    labels = torch.empty((n, H, W), dtype=torch.int32, device=dev)
    from paper_2012_10802_amd.pothole_pipeline import SLIC_TOL
    S_slic, m_slic, it_slic = 16, 4.0, 10
    sp_rounds = torch.empty((n,), dtype=torch.int32, device=dev)
    sp_labels = torch.empty((n, H, W), dtype=torch.int32, device=dev)
    d3 = torch.empty((n, H, W), dtype=torch.float32, device=dev)
    centres = torch.empty((n, sgm.slic_num_centres(W, H, S_slic), 3), dtype=torch.float64, device=dev)
    sp_ws = torch.empty(sgm.slic_workspace_size(W, H, S_slic, n), dtype=torch.uint8, device=dev)

    def once(ev=None):
        if ev:
            ev[0].record()
        sgm.road_fit(disp, mask, 0.5, fit=fit, workspace=ws)
        if ev:
            ev[1].record()
        sgm.road_window(fit, W, H, 24, mode=1, delta=2.0, d_lo=d_lo)
        if ev:
            ev[2].record()
        sgm.disparity_transform(disp, fit, 10.0, out=d2)
        if ev:
            ev[3].record()
        # eq. (14), (15) on D2 (road range 10 +- 8 px), then the components
        sgm.pothole_threshold(d2, 2.0, 18.0, nbins, delta_pd, mask=mask, result=pd_res, workspace=pd_ws)
        if ev:
            ev[4].record()
        sgm.pothole_labels(d2, pd_res, mask=mask, labels=labels)
        if ev:
            ev[5].record()
        # superpixels on D2 and the superpixel means D3 (SLIC, at most 10
        # rounds, each map stopping once its centres move by <= SLIC_TOL)
        sgm.slic(d2, S_slic, m_slic, it_slic, mask=mask, tol=SLIC_TOL, labels=sp_labels, d3=d3, centres=centres,
                 workspace=sp_ws, rounds=sp_rounds)
        if ev:
            ev[6].record()

    for _ in range(3):
        once()
    reps = 20
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(7)] for _ in range(reps)]
    torch.cuda.synchronize()
    for e in events:
        once(e)
    torch.cuda.synchronize()
    per = np.array([[e[k].elapsed_time(e[k + 1]) for k in range(6)] for e in events])
    fit_ms, win_ms, tr_ms, thr_ms, lab_ms, slic_ms = (float(x) for x in per.mean(axis=0))
    # the curve E0min(phi) of eq. (12) (Fig. 3) on a 0.1 degree grid over
    # the same maps and pixels as the fit; its minimum against the fit's phi
    nphi = 1800
    phis = torch.linspace(-math.pi / 2, math.pi / 2, nphi + 1, dtype=torch.float64, device=dev)[1:].contiguous()
    energy = torch.empty((n, nphi), dtype=torch.float64, device=dev)
    curve_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(10)]
    sgm.road_energy(disp, phis, mask, 0.5, energy=energy, workspace=ws)
    for a, b in curve_ev:
        a.record()
        sgm.road_energy(disp, phis, mask, 0.5, energy=energy, workspace=ws)
        b.record()
    sgm.road_fit(disp, mask, 0.5, fit=fit, workspace=ws)
    torch.cuda.synchronize()
    curve_ms = float(np.median([a.elapsed_time(b) for a, b in curve_ev]))
    fit_phi = fit[:, 2].cpu().numpy()
    arg_phi = phis.cpu().numpy()[energy.argmin(dim=1).cpu().numpy()]
    curve_dev = float(np.max(np.abs(arg_phi - fit_phi)))
    pd_stat = sgm.pothole_threshold_dicts(pd_res)
    detection = []
    for dpd in (delta_pd, 1.0, 0.5):  # the paper's tolerance, then smaller ones for shallower potholes
        res = pd_res.clone()
        res[:, 1] = res[:, 0] - dpd  # t_s = t_r - delta_PD
        for name, src in (("D2", d2), ("D3", d3)):  # pixel by pixel, then superpixel means
            lab = sgm.pothole_labels(src, res, mask=mask)
            found = lab > 0
            tp = int((found & holes).sum())
            prec = tp / max(1, int(found.sum()))
            rec = tp / max(1, int(holes.sum()))
            detection.append({"map": name, "delta_pd": dpd, "pixel_precision": round(prec, 4),
                              "pixel_recall": round(rec, 4),
                              "pixel_f1": round(2 * prec * rec / max(1e-12, prec + rec), 4),
                              "components_mean": round(float(np.mean(
                                  [torch.unique(lab[i][lab[i] > 0]).numel() for i in range(n)])), 1)})
    copy_calibration(args, dev)
    px = n * W * H
    fit_gbs = px * 5 / (fit_ms * 1e-3) / 1e9
    tr_gbs = px * 8 / (tr_ms * 1e-3) / 1e9
    fits = sgm.road_fit_dicts(fit)
    dphi = [abs(f["phi"] - t[2]) for f, t in zip(fits, truth)]
    da1 = [abs(f["a1"] - t[1]) / t[1] for f, t in zip(fits, truth)]
    da0 = [abs(f["a0"] - t[0]) for f, t in zip(fits, truth)]
    if log:
        log("road model: fit %.4f ms, windows %.4f ms, transformation %.4f ms, pothole threshold %.4f ms, "
            "labels %.4f ms, SLIC %.4f ms per batch of %d" % (fit_ms, win_ms, tr_ms, thr_ms, lab_ms, slic_ms, n))
    return {
        "maps": n, "width": W, "height": H,
        "inputs": "full-range SGM disparity (0-191, census 7x7, 8 paths) of generated road pairs; "
                  "mask = generator road pixels with u - gt >= 4",
        "ms_per_batch": round(fit_ms + win_ms + tr_ms, 4),
        "fit_ms": round(fit_ms, 4), "window_ms": round(win_ms, 4), "transform_ms": round(tr_ms, 4),
        "fit_hbm": {"bytes_per_pixel": 5, "achieved": round(fit_gbs, 1), "unit": "GB/s",
                    "frac": round(fit_gbs / HBM_PEAK_GBS, 4)},
        "transform_hbm": {"bytes_per_pixel": 8, "achieved": round(tr_gbs, 1), "unit": "GB/s",
                          "frac": round(tr_gbs / HBM_PEAK_GBS, 4)},
        "e0min_curve": {"nphi": nphi, "grid_deg": 0.1, "ms_per_batch": round(curve_ms, 4),
                        "argmin_vs_fit_max_deg": round(math.degrees(curve_dev), 4),
                        "note": "eq. (12) at every grid angle from the fit's moments (one pass over the maps)"},
        "fit_error": {"phi_max_deg": round(math.degrees(max(dphi)), 5),
                      "a1_max_rel": round(max(da1), 6), "a0_max_px": round(max(da0), 4)},
        "pothole": {"threshold_ms": round(thr_ms, 4), "label_ms": round(lab_ms, 4),
                    "slic_ms": round(slic_ms, 4),
                    "slic": {"S": S_slic, "m": m_slic, "iters": it_slic, "tol": SLIC_TOL,
                             "rounds_mean": round(float(sp_rounds.double().mean()), 2),
                             "superpixels_per_map": sgm.slic_num_centres(W, H, S_slic)},
                    "threshold_hbm": {"bytes_per_pixel": 5,
                                      "achieved": round(px * 5 / (thr_ms * 1e-3) / 1e9, 1), "unit": "GB/s"},
                    "nbins": nbins, "delta_pd": delta_pd, "range": [2.0, 18.0],
                    "t_r_mean": round(float(np.mean([r["t_r"] for r in pd_stat])), 4),
                    "detection": detection,
                    "note": "threshold t_r from D2 (eq. (14), (15)); potholes = D2 or D3 below t_s, "
                            "8-connected; ground truth = the generator's depressions on road pixels"},
    }


def perspective_leg(args, log=None):
    """The perspective-transformed form from the images alone on a batch of
    16 road1280 pairs (1280x720, disparities 0-127, census 7x7, 8 paths):
    quarter-scale full-range SGM, road fit and refit on it (eq. (11),
    (12)), per-pixel windows of 16 centred on the fitted road plane (and,
    for comparison, per-row windows of 24, Sec. II-A), windowed SGM at full
    resolution, refits on D1 and eq. (13).  Wall time per frame (HIP events
    around whole batches) against plain full-range batched SGM on the same
    frames, and the bad-pixel rate of each on the same pixels (the
    full-range evaluation mask, from the generator's ground truth)."""
    import math

    import numpy as np
    import torch

    from paper_2012_10802_amd import sgm, synth
    from paper_2012_10802_amd.road_pipeline import PerspectiveMatcher

    dev = torch.device("cuda:0")
    c = synth.CONFIGS["road1280"]
    W, H, D, n_cen = c["width"], c["height"], c["ndisp"], c["census"]
    n = 16
    L = torch.empty((n, H, W), dtype=torch.uint8, device=dev)
    R = torch.empty_like(L)
    gts, roads, truth = [], [], []
    for i in range(n):
        seed = args.seed + 100 + i
        sc = synth.scene_for_config("road1280", seed)
        l, r, gt, road = synth.make_pair_torch(sc, seed, device=dev)
        L[i].copy_(l)
        R[i].copy_(r)
        gts.append(gt.cpu().numpy().astype(np.float64))
        roads.append(road.cpu().numpy())
        truth.append(sc.road_params)
    kw = dict(ndisp=D, census=n_cen, npaths=c["npaths"], p1=c["p1"], p2=c["p2"], delta_dt=20.0, device=dev)
    pm = PerspectiveMatcher(W, H, batch=n, windows="pixel", **kw)
    pm_row = PerspectiveMatcher(W, H, batch=n, windows="row", w=24, **kw)
    pdint = torch.empty((n, H, W), dtype=torch.int16, device=dev)
    pdsub = torch.empty((n, H, W), dtype=torch.float32, device=dev)
    plain = sgm.Batch([dict(left=L[i], right=R[i], ndisp=D, disp_int=pdint[i], disp_sub=pdsub[i]) for i in range(n)],
                      census=n_cen, npaths=c["npaths"], p1=c["p1"], p2=c["p2"], device=dev)
    plain.autotune()
    reps = 10
    times = {}
    for name, fn in (("pixel", lambda: pm.match(L, R)), ("row", lambda: pm_row.match(L, R)),
                     ("plain", lambda: plain.run())):
        for _ in range(3):
            fn()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(reps):
            fn()
        ev[1].record()
        torch.cuda.synchronize()
        times[name] = ev[0].elapsed_time(ev[1]) / reps / n
    bad = {"pixel": [], "row": [], "plain": []}
    miss, dphi, da0 = [], [], []
    outs = {"pixel": pm.disp_sub.cpu().numpy(), "row": pm_row.disp_sub.cpu().numpy(), "plain": pdsub.cpu().numpy()}
    lo_all = pm.lo.cpu().numpy().astype(np.float64)
    fits = sgm.road_fit_dicts(pm.coarse_fit)
    r = n_cen // 2
    uu = np.arange(W)[None, :]
    for i in range(n):
        gt = gts[i]
        mask = roads[i] & (gt < D - 1) & (uu - gt >= r)
        mask[:r] = mask[-r:] = False
        mask[:, :r] = mask[:, -r:] = False
        for k in bad:
            bad[k].append(float((np.abs(outs[k][i] - gt)[mask] > 1.0).mean()))
        inside = (gt >= lo_all[i]) & (gt < lo_all[i] + pm.w - 1)
        miss.append(float((~inside[mask]).mean()))
        a0, a1, phi = truth[i]
        dphi.append(abs(fits[i]["phi"] - phi))
        da0.append(abs(4 * fits[i]["a0"] - a0))
    if log:
        log("perspective form: %.4f ms per frame (row windows %.4f) vs plain %.4f ms, batches of %d"
            % (times["pixel"], times["row"], times["plain"], n))
    return {
        "pairs": n, "batch": n, "width": W, "height": H, "ndisp": D,
        "window": "16 per pixel, centred on the fitted road plane",
        "ms_per_frame": round(times["pixel"], 4), "plain_ms_per_frame": round(times["plain"], 4),
        "speedup": round(times["plain"] / times["pixel"], 3),
        "full_range_equivalent": {"value": round(W * H * D / (times["pixel"] * 1e-3) / 1e6, 1),
                                  "unit": "Mdisp-evals/s (pixels x 128 disparities per second)"},
        "bad_1px_pct": round(100 * float(np.mean(bad["pixel"])), 4),
        "plain_bad_1px_pct": round(100 * float(np.mean(bad["plain"])), 4),
        "row_windows_24": {"ms_per_frame": round(times["row"], 4),
                           "bad_1px_pct": round(100 * float(np.mean(bad["row"])), 4)},
        "window_miss_pct": round(100 * float(np.mean(miss)), 4),
        "coarse_fit_error": {"phi_max_deg": round(math.degrees(max(dphi)), 4), "a0_max_px": round(max(da0), 4)},
        "stages": "4x4 reduction, quarter-scale SGM (0-31), road fit and refit, per-pixel windows of 16 from "
                  "the plane, windowed SGM, fit and refits on D1, eq. (13); plain = autotuned batched SGM",
        "timing": "HIP events around 10 batches of 16 after 3 warm-ups, per frame",
    }


def detector_leg(args, log=None):
    """The whole method end to end (PotholeDetector): batches of 16 held-out
    1920x1080 road pairs -> perspective-transformed SGM (the paper's) or
    learned-window SGM -> road fit and refits ->
    road region -> D2 -> threshold -> SLIC / D3 -> labelled potholes, with
    no ground truth used.  Wall time per batch (host clock around
    detect(), synchronised; the learned matcher reads its fallback rows on
    the host once per batch), and the detections against the generator's
    depressions: pixel precision / recall and the share of potholes hit."""
    import torch

    from paper_2012_10802_amd.pothole_pipeline import PotholeDetector

    dev = torch.device("cuda:0")
    n, W, H = 16, 1920, 1080
    return {m: _detector_run(PotholeDetector(W, H, n, matcher=m, delta_pd=0.5, device=dev), n, W, H, m, log)
            for m in ("perspective", "learned")}


def _detector_run(det, n, W, H, matcher, log):
    import math

    import numpy as np
    import torch
    from scipy import ndimage

    from paper_2012_10802_amd import synth

    dev = det.device
    times, tp, fp, fn, hit, holes_total, rounds = [], 0, 0, 0, 0, 0, []
    for b in range(2):
        seeds = [20_000_000 + 100 * b + i for i in range(n)]
        L = torch.empty((n, H, W), dtype=torch.uint8, device=dev)
        R = torch.empty_like(L)
        truth = []
        rows = torch.arange(H, device=dev, dtype=torch.float64)[:, None]
        cols = torch.arange(W, device=dev, dtype=torch.float64)[None, :]
        for i, sd in enumerate(seeds):
            sc = synth.scene_for_config("road1920", sd)
            l, r, gt, road = synth.make_pair_torch(sc, sd, device=dev)
            L[i].copy_(l)
            R[i].copy_(r)
            a0, a1, phi = sc.road_params
            plane = a0 + a1 * (math.cos(phi) * (rows - sc.cy) - math.sin(phi) * (cols - sc.cx))
            truth.append((road & (gt.double() < plane - 1e-3)).cpu().numpy())  # the depressions
        for _ in range(2):
            det.detect(L, R)
        torch.cuda.synchronize()
        reps = []
        for _ in range(3):
            t0 = time.perf_counter()
            det.detect(L, R)
            torch.cuda.synchronize()
            reps.append(time.perf_counter() - t0)
        times.append(sorted(reps)[1])
        rounds += det.slic_rounds.tolist()
        lab = det.labels.cpu().numpy()
        for i, hole in enumerate(truth):
            found = lab[i] > 0
            tp += int((found & hole).sum())
            fp += int((found & ~hole).sum())
            fn += int((~found & hole).sum())
            comps, k = ndimage.label(hole, structure=np.ones((3, 3), int))
            holes_total += k
            hit += sum(1 for c in range(1, k + 1) if found[comps == c].any())
    ms = 1e3 * float(np.mean(times))
    prec, rec = tp / max(1, tp + fp), tp / max(1, tp + fn)
    if log:
        log("pothole detector (%s): %.3f ms per batch of %d (%.0f frames/s)" % (matcher, ms, n, n / (ms * 1e-3)))
    return {
        "matcher": matcher,
        "pairs": 2 * n, "batch": n, "width": W, "height": H,
        "ms_per_batch": round(ms, 3), "frames_per_s": round(n / (ms * 1e-3), 1),
        "pixel_precision": round(prec, 4), "pixel_recall": round(rec, 4),
        "pixel_f1": round(2 * prec * rec / max(1e-12, prec + rec), 4),
        "potholes_hit": hit, "potholes_total": holes_total,
        "slic_rounds_mean": round(float(np.mean(rounds)), 2),
        "settings": "%s SGM (0-191), fit + refits (2, 1 px), road region f >= 2 px, "
                    "delta_DT 10, 128 bins over 2..18, delta_PD 0.5, SLIC S 16 m 4, at most %d rounds, tol %g%s"
                    % ("perspective-transformed (windows of 16 on the fitted plane)" if matcher == "perspective"
                       else "learned-window", det.slic_iters, det.slic_tol,
                       ", potholes in a single superpixel dropped" if det.prune_single else ""),
        "timing": "host wall clock around detect() (synchronised), median of 3 after 2 warm-ups, "
                  "mean over 2 batches",
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="road1280", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="single", choices=["single", "batch"],
                    help="single: the split single-pair calls; batch: the batch calls as a graph")
    ap.add_argument("--unique", type=int, default=2,
                    help="batch mode: distinct rendered pairs per size (inputs are shared)")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file")
    ap.add_argument("--lanes", type=int, default=None, choices=[0, 4, 8, 16],
                    help="single mode: lanes per scanline of the volume kernels (default: autotuned)")
    ap.add_argument("--seed", type=int, default=2001)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-window vs plain comparison")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2012_10802_amd", "window_cnn.npz"))
    ap.add_argument("--no-graph", action="store_true",
                    help="single mode: time eager steps instead of replays of the step captured in a HIP graph")
    ap.add_argument("--tau", type=float, default=0.5, help="confidence threshold of the learned windows")
    ap.add_argument("--fallback-margin", type=int, default=8,
                    help="low-confidence pixels fall back to full range only where x - 4 * coarse disparity is at "
                         "least this (-2147483648: all of them)")
    ap.add_argument("--eval-pairs", type=int, default=64)
    ap.add_argument("--lw-reps", type=int, default=3)
    ap.add_argument("--learned-only", action="store_true", help="print only the learned-window comparison")
    ap.add_argument("--no-road", action="store_true", help="skip the road-model stages (fit, windows, "
                    "disparity transformation)")
    ap.add_argument("--road-only", action="store_true", help="print only the road-model stages")
    ap.add_argument("--perspective-only", action="store_true",
                    help="print only the perspective-transformed form estimated from the images")
    ap.add_argument("--detector-only", action="store_true",
                    help="print only the end-to-end pothole detector")
    ap.add_argument("--jsonl", default=None, help="also append the JSON record to this file")
    ap.add_argument("--cpu-runs", type=int, default=3, help="timed runs of the CPU oracle (median)")
    ap.add_argument("--cpu-pairs-per-size", type=int, default=4,
                    help="batch mode: pairs of each size class the CPU oracle times (extrapolated in evals)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="after timing, run one device-to-device copy of this many MiB "
                         "(reference kernel for scaling memory counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (got --gpus %d): batches shard by independent stereo "
              "pairs, one GPU's share being exactly the single-GPU run, and no multi-GPU path is "
              "implemented here" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.mode == "batch" or args.workload == "road_batch64":
        return run_batch(args)
    if args.road_only:
        import torch
        torch.cuda.set_device(0)
        emit(road_model_leg(args, log=lambda msg: print(msg, file=sys.stderr, flush=True)), args)
        return
    if args.perspective_only:
        import torch
        torch.cuda.set_device(0)
        emit(perspective_leg(args, log=lambda msg: print(msg, file=sys.stderr, flush=True)), args)
        return
    if args.detector_only:
        import torch
        torch.cuda.set_device(0)
        emit(detector_leg(args, log=lambda msg: print(msg, file=sys.stderr, flush=True)), args)
        return
    if args.learned_only:
        import torch
        torch.cuda.set_device(0)
        res = learned_vs_plain(args, log=lambda msg: print(msg, file=sys.stderr, flush=True))
        emit(res, args)
        return

    import numpy as np
    import torch

    from paper_2012_10802_amd import sgm, synth

    cfg = synth.CONFIGS[args.workload]
    W, H, w = cfg["width"], cfg["height"], cfg["ndisp"]
    n, R, p1, p2 = cfg["census"], cfg["npaths"], cfg["p1"], cfg["p2"]
    pair = synth.make_pair(synth.scene_for_config(args.workload, args.seed), args.seed)
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    m = sgm.Matcher(W, H, census=n, ndisp=w, npaths=R, p1=p1, p2=p2, device=dev)
    left = torch.from_numpy(pair.left).to(dev)
    right = torch.from_numpy(pair.right).to(dev)
    d_lo = None
    if args.workload == "road1280_pt":  # per-row windows from the scene's road model, eq. (3), (6)
        a0, a1, phi = pair.road_params
        d_lo = sgm.sgm_window_from_road(a0, a1, phi, W, H, w, mode=0).to(dev)
    # lane mapping of the volume kernels: fixed by --lanes, else timed on
    # this frame (sgm_autotune; cached in --tune-cache when given)
    if args.lanes is not None:
        m = sgm.Matcher(W, H, census=n, ndisp=w, npaths=R, p1=p1, p2=p2, device=dev, lanes=args.lanes)
    else:
        m.autotune(left, right, d_lo=d_lo, cache_path=args.tune_cache)
    cost = m.new_volume(torch.uint8)
    paths = m.new_paths()
    dint = torch.empty((H, W), dtype=torch.int16, device=dev)
    dsub = torch.empty((H, W), dtype=torch.float32, device=dev)

    def step(ev=None):
        if ev:
            ev[0].record()
        m.cost(left, right, d_lo=d_lo, cost=cost)
        if ev:
            ev[1].record()
        m.aggregate_paths(cost, paths)
        if ev:
            ev[2].record()
        m.wta_paths(paths, d_lo=d_lo, disp_int=dint, disp_sub=dsub)
        if ev:
            ev[3].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # eager steps with HIP events between the stages (per-kernel times)
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(events[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_eager = (t1 - t0) * 1e3 / args.steps
    per = np.array([[e[k].elapsed_time(e[k + 1]) for k in range(3)] for e in events])
    cost_ms, agg_ms, wta_ms = (float(x) for x in per.mean(axis=0))
    ms_per_step, graph_info = ms_eager, None
    if not args.no_graph:
        # the same step captured once in a HIP graph and replayed (the calls
        # allocate nothing and issue no memsets); its result must equal the
        # eager one bit for bit before it is timed
        want_i, want_s = dint.clone(), dsub.clone()
        graph = torch.cuda.CUDAGraph()
        try:
            with torch.cuda.graph(graph):
                step()
        except RuntimeError as exc:  # capture unavailable: the eager time stands
            graph = None
            graph_info = {"error": "capture failed (%s); value from the eager steps" % exc}
        if graph is not None:
            dint.fill_(-1)
            dsub.fill_(float("nan"))
            graph.replay()
            torch.cuda.synchronize()
            if not (torch.equal(dint, want_i) and torch.equal(dsub, want_s)):
                raise RuntimeError("graph replay of the step differs from the eager step")
            for _ in range(args.warmup):
                graph.replay()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                graph.replay()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ms_per_step = (t1 - t0) * 1e3 / args.steps
            graph_info = {"ms_per_step_eager": round(ms_eager, 4),
                          "note": "value from replays of the step captured in a HIP graph (checked bit-equal to "
                                  "the eager step); kernels_ms from the eager steps' HIP events"}

    evals = W * H * w
    value = evals / (ms_per_step * 1e-3) / 1e6

    copy_calibration(args, dev)

    # dominant kernel: the one-launch aggregation of all directions.  Its
    # compulsory traffic under this schedule: every direction streams the
    # cost volume once (1 B/eval) and writes its own volume (e B/eval).
    elem_bytes, _, _ = m.path_volumes()
    agg_bytes_per_eval = R * (1 + elem_bytes)
    agg_bytes = evals * agg_bytes_per_eval
    agg_gbs = agg_bytes / (agg_ms * 1e-3) / 1e9
    # packed-u16 ops of the recurrence per eval and direction: neighbour min,
    # +P1, min with L(k), min with P2, +C, running min, -m
    agg_ops = evals * R * 7
    agg_tops = agg_ops / (agg_ms * 1e-3) / 1e12
    traffic = counter_traffic(args.workload)
    hbm = {"bound": "hbm", "achieved": round(agg_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(agg_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
           "bytes_per_eval": agg_bytes_per_eval, "bytes_per_launch": agg_bytes}
    alu = {"bound": "alu", "achieved": round(agg_tops, 2), "peak": round(VALU_PEAK_TOPS_U16, 2),
           "unit": "TOP/s (u16)", "frac": round(agg_tops / VALU_PEAK_TOPS_U16, 4), "traffic": traffic}
    roofline = hbm if hbm["frac"] >= alu["frac"] else alu
    roofline["kernel"] = "k_aggregate"
    if cost.numel() <= (256 << 20):
        roofline["note"] = ("effective rate (algorithmic bytes / kernel time): the %d MB cost volume fits the "
                            "256 MB MALL, which serves most of its 8 reads; the batched workload, whose volumes "
                            "exceed it, gives the HBM-clean figure" % (cost.numel() >> 20))
    copy_ref = copy_reference(torch.device("cuda:0"))
    copy_ref["aggregate_over_copy"] = round(agg_gbs / copy_ref["achieved"], 4)
    # the whole step: cost written once, read once per direction, R volumes
    # written and read back by the selection
    step_bytes_per_eval = 1 + R * (1 + 2 * elem_bytes)
    step_gbs = evals * step_bytes_per_eval / (ms_per_step * 1e-3) / 1e9

    # accuracy against the generator's ground truth (bad-pixel rate, eq. (18))
    torch.cuda.synchronize()
    ds = dsub.cpu().numpy()
    mask = eval_mask(pair, w, n // 2, None if d_lo is None else d_lo.cpu().numpy())
    err = np.abs(ds - pair.gt)[mask]
    accuracy = {"bad_1px_pct": round(float((err > 1.0).mean() * 100), 4),
                "rmse_px": round(float(np.sqrt((err ** 2).mean())), 4),
                "pixels": int(mask.sum())}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_frame(pair, n, w, R, p1, p2, None if d_lo is None else d_lo.cpu().numpy(),
                                 runs=args.cpu_runs, log=lambda msg: print(msg, file=sys.stderr, flush=True))

    learned = None
    if not args.no_learned and os.path.exists(args.weights):
        learned = learned_vs_plain(args, log=lambda msg: print(msg, file=sys.stderr, flush=True))

    road = persp = detector = None
    if not args.no_road:
        road = road_model_leg(args, log=lambda msg: print(msg, file=sys.stderr, flush=True))
        persp = perspective_leg(args, log=lambda msg: print(msg, file=sys.stderr, flush=True))
        if os.path.exists(args.weights):
            detector = detector_leg(args, log=lambda msg: print(msg, file=sys.stderr, flush=True))

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Mdisp-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "storage": "uint8 cost and per-direction volumes, packed u16 arithmetic",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload],
                   "width": W, "height": H, "ndisp": w, "census": n, "npaths": R,
                   "p1": p1, "p2": p2, "evals_per_step": evals},
        "full_range_equivalent": None if d_lo is None else {
            "ndisp": 128, "value": round(W * H * 128 / (ms_per_step * 1e-3) / 1e6, 1),
            "unit": "Mdisp-evals/s (pixels x 128 disparities per second)"},
        "graph": graph_info,
        "tuning": {"lanes_per_scanline": m.lanes, "horizontal_lanes_per_scanline": 16,
                   "slot_order": ["horizontal, diagonal, vertical", "horizontal, vertical, diagonal"][m.order],
                   "chosen_by": "--lanes" if args.lanes is not None else "sgm_autotune"},
        "roofline": roofline,
        "roofline_other_bound": alu if roofline is hbm else hbm,
        "step_hbm": {"bytes_per_eval": step_bytes_per_eval, "achieved": round(step_gbs, 1), "unit": "GB/s",
                     "frac": round(step_gbs / HBM_PEAK_GBS, 4)},
        "hbm_copy_reference": copy_ref,
        "kernels_ms": {"cost": round(cost_ms, 4), "aggregate": round(agg_ms, 4),
                       "wta": round(wta_ms, 4)},
        "accuracy": accuracy,
        "learned_window": learned,
        "road_model": road,
        "perspective_from_images": persp,
        "pothole_detector": detector,
        "cpu_baseline": cpu,
        "paper_context": PAPER_CONTEXT,
        "kernel_source_sha256": kernel_source_digest(),
    }
    emit(out, args)


if __name__ == "__main__":
    main()
