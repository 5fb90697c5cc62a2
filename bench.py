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
}


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2012_10802_amd", "csrc", "sgm_kernels.hip"), "rb") as f:
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


def eval_mask(p, w, r):
    """Pixels scored for accuracy: road, ground truth inside the window and
    away from the image border (census half-window r)."""
    import numpy as np
    H, W = p.gt.shape
    uu = np.arange(W)[None, :]
    m = p.road & (p.gt < w - 1) & (uu - p.gt >= r)
    m[:r] = m[-r:] = False
    m[:, :r] = m[:, -r:] = False
    return m


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="road1280", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=2001)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="after timing, run one device-to-device copy of this many MiB "
                         "(reference kernel for scaling memory counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the SGM path shards by independent stereo pairs and "
              "this build runs and reports a single MI355X (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

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
    cost = m.new_volume(torch.uint8)
    paths = m.new_paths()
    dint = torch.empty((H, W), dtype=torch.int16, device=dev)
    dsub = torch.empty((H, W), dtype=torch.float32, device=dev)

    def step(ev=None):
        if ev:
            ev[0].record()
        m.cost(left, right, cost=cost)
        if ev:
            ev[1].record()
        m.aggregate_paths(cost, paths)
        if ev:
            ev[2].record()
        m.wta_paths(paths, disp_int=dint, disp_sub=dsub)
        if ev:
            ev[3].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(events[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    per = np.array([[e[k].elapsed_time(e[k + 1]) for k in range(3)] for e in events])
    cost_ms, agg_ms, wta_ms = (float(x) for x in per.mean(axis=0))

    evals = W * H * w
    value = evals / (ms_per_step * 1e-3) / 1e6

    if args.copy_calibration_mb:
        src = torch.ones(args.copy_calibration_mb << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # dominant kernel: the one-launch aggregation of all directions
    elem_bytes, _, _ = m.path_volumes()
    agg_bytes = evals * (1 + R * elem_bytes)  # read C once, write R volumes
    agg_gbs = agg_bytes / (agg_ms * 1e-3) / 1e9
    # packed-u16 ops of the recurrence per eval and direction: neighbour min,
    # +P1, min with L(k), min with P2, +C, running min, -m
    agg_ops = evals * R * 7
    agg_tops = agg_ops / (agg_ms * 1e-3) / 1e12
    traffic = counter_traffic(args.workload)
    hbm = {"bound": "hbm", "achieved": round(agg_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(agg_gbs / HBM_PEAK_GBS, 4), "traffic": traffic}
    alu = {"bound": "alu", "achieved": round(agg_tops, 2), "peak": round(VALU_PEAK_TOPS_U16, 2),
           "unit": "TOP/s (u16)", "frac": round(agg_tops / VALU_PEAK_TOPS_U16, 4), "traffic": traffic}
    roofline = hbm if hbm["frac"] >= alu["frac"] else alu
    roofline["kernel"] = "k_aggregate"

    # accuracy against the generator's ground truth (bad-pixel rate, eq. (18))
    torch.cuda.synchronize()
    ds = dsub.cpu().numpy()
    mask = eval_mask(pair, w, n // 2)
    err = np.abs(ds - pair.gt)[mask]
    accuracy = {"bad_1px_pct": round(float((err > 1.0).mean() * 100), 4),
                "rmse_px": round(float(np.sqrt((err ** 2).mean())), 4),
                "pixels": int(mask.sum())}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        oracle.sgm(pair.left, pair.right, n, w, R, p1, p2)
        dt = time.perf_counter() - t
        cpu = {"value": round(evals / dt / 1e6, 3), "unit": "Mdisp-evals/s",
               "cores": min(R, oracle.num_threads()), "kind": "oracle",
               "sample": "one full %dx%dx%d frame through the C oracle (census, cost, %d paths, "
                         "selection), %.1f s wall" % (W, H, w, R, dt)}

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
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload],
                   "width": W, "height": H, "ndisp": w, "census": n, "npaths": R,
                   "p1": p1, "p2": p2, "evals_per_step": evals},
        "roofline": roofline,
        "roofline_other_bound": alu if roofline is hbm else hbm,
        "kernels_ms": {"cost": round(cost_ms, 4), "aggregate": round(agg_ms, 4),
                       "wta": round(wta_ms, 4)},
        "accuracy": accuracy,
        "cpu_baseline": cpu,
        "kernel_source_sha256": kernel_source_digest(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
