"""Train the search-window network on generated road pairs.

    python -m paper_2012_10802_amd.train_window --pairs 20000 --out window_cnn.npz

Data: for each seed, a 1920x1080 pair of the road generator rendered on the
GPU (roll uniform in 0..4 degrees), labelled by full-range plain SGM
(0..191, 8 paths, census 7x7) at full resolution; the network sees the
quarter-resolution level: the coarse full-range SGM disparity (0..47) and
the coarse left image.  The target offset is label - coarse, with the label
the 4x4 block mean of the full-resolution SGM disparity in coarse pixels.
Where the label's match falls off the left edge of the right image (label
>= column) full-range search cannot do better than the coarse estimate, so
the target there is the coarse value itself (offset 0).

Training: Adam, batches of `--batch` quarter-resolution images, epochs over
a seeded permutation.  A checkpoint (`--checkpoint`) is written every
`--save-every` steps and at the end; `--resume` continues from it and
reproduces the uninterrupted run bit for bit (the data are regenerated from
their seeds, the permutation from the seed and the epoch).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import learned_window as LW
from . import sgm as S
from . import synth

W, H, D = 1920, 1080, 192
CENSUS, PATHS, P1, P2 = 7, 8, 10, 120


def generate(seeds, device, chunk=16, log=print):
    """Quarter-resolution training samples for the given seeds: coarse
    disparity (float32), coarse left image (uint8) and coarse label
    (float32), each [n, H/4, W/4], on `device`."""
    Wc, Hc = W // 4, H // 4
    n = len(seeds)
    coarse = torch.empty((n, Hc, Wc), dtype=torch.float32, device=device)
    left_c = torch.empty((n, Hc, Wc), dtype=torch.uint8, device=device)
    label = torch.empty((n, Hc, Wc), dtype=torch.float32, device=device)
    L = torch.empty((chunk, H, W), dtype=torch.uint8, device=device)
    R = torch.empty_like(L)
    cl = torch.empty((chunk, Hc, Wc), dtype=torch.uint8, device=device)
    cr = torch.empty_like(cl)
    full = S.Batch([dict(left=L[i], right=R[i], ndisp=D) for i in range(chunk)], census=CENSUS,
                   npaths=PATHS, p1=P1, p2=P2, device=device)
    small = S.Batch([dict(left=cl[i], right=cr[i], ndisp=D // 4) for i in range(chunk)], census=CENSUS,
                    npaths=PATHS, p1=P1, p2=P2, device=device)
    cols = torch.arange(Wc, dtype=torch.float32, device=device)[None, :]
    t0 = time.time()
    for s0 in range(0, n, chunk):
        k = min(chunk, n - s0)
        for j in range(k):
            sd = int(seeds[s0 + j])
            l, r, _, _ = synth.make_pair_torch(synth.scene_for_config("road1920", sd), sd, device=device)
            L[j].copy_(l)
            R[j].copy_(r)
        for j in range(k, chunk):  # pad a short last chunk
            L[j].copy_(L[0])
            R[j].copy_(R[0])
        full.run()
        for j in range(chunk):
            S.sgm_downsample4(L[j], cl[j])
            S.sgm_downsample4(R[j], cr[j])
        small.run()
        for j in range(k):
            lab = LW.label_downsample4(full.disp_sub[j])
            cd = small.disp_sub[j]
            coarse[s0 + j].copy_(cd)
            left_c[s0 + j].copy_(cl[j])
            label[s0 + j].copy_(torch.where(lab >= cols, cd, lab))
        if (s0 // chunk) % 10 == 0:
            torch.cuda.synchronize()
            log("generated %d/%d pairs (%.1f s)" % (s0 + k, n, time.time() - t0))
    torch.cuda.synchronize()
    return coarse, left_c, label


def permutation(seed, epoch, n):
    return np.random.default_rng([seed, epoch]).permutation(n)


def train(args, log=print):
    dev = torch.device("cuda")
    seeds = np.arange(args.first_seed, args.first_seed + args.pairs)
    coarse, left_c, label = generate(seeds, dev, log=log)
    Hc, Wc = coarse.shape[1:]
    B = args.batch
    steps_per_epoch = args.pairs // B
    total = steps_per_epoch * args.epochs
    if args.resume and os.path.exists(args.checkpoint):
        net = LW.WindowNet.load(args.checkpoint)
        log("resumed at step %d" % net.step)
    else:
        net = LW.WindowNet(seed=args.seed)
    bufs = net.train_buffers(Wc, Hc, B)
    x0 = torch.empty((B, Hc, Wc, LW.CH), dtype=torch.int16, device=dev)
    cb = torch.empty((B, Hc, Wc), dtype=torch.float32, device=dev)
    lb = torch.empty_like(cb)
    ib = torch.empty((B, Hc, Wc), dtype=torch.uint8, device=dev)
    hist = []
    t0 = time.time()
    while net.step < total:
        epoch, k = divmod(net.step, steps_per_epoch)
        perm = permutation(args.seed, epoch, args.pairs)
        idx = torch.from_numpy(perm[k * B:(k + 1) * B]).to(dev)
        torch.index_select(coarse, 0, idx, out=cb)
        torch.index_select(label, 0, idx, out=lb)
        torch.index_select(left_c, 0, idx, out=ib)
        LW.prepare_input(cb, ib, Wc, Hc, B, x0)
        lr = args.lr * (0.1 if net.step >= int(0.8 * total) else 1.0)
        loss = net.train_step(x0, cb, lb, Wc, Hc, B, lr, bufs)
        if net.step % args.log_every == 0 or net.step == total:
            lo = loss.cpu().numpy()
            hist.append([net.step, float(lo[0]), float(lo[1])])
            log("step %d/%d epoch %d loss offset %.4f conf %.4f (%.1f s)"
                % (net.step, total, epoch, lo[0], lo[1], time.time() - t0))
        if args.checkpoint and (net.step % args.save_every == 0 or net.step == total):
            net.save(args.checkpoint, extra={"seed": args.seed, "pairs": args.pairs, "batch": B,
                                             "epochs": args.epochs, "lr": args.lr})
        if args.stop_after and net.step >= args.stop_after:
            break
    torch.cuda.synchronize()
    if args.out and net.step == total:
        net.save(args.out, extra={"seed": args.seed, "pairs": args.pairs, "batch": B, "epochs": args.epochs,
                                  "lr": args.lr, "first_seed": args.first_seed, "loss_history": hist})
    return net


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--pairs", type=int, default=20000)
    ap.add_argument("--first-seed", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=2)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--checkpoint", default="")
    ap.add_argument("--save-every", type=int, default=500)
    ap.add_argument("--resume", action="store_true")
    ap.add_argument("--stop-after", type=int, default=0, help="stop at this step (to test resuming)")
    ap.add_argument("--log-every", type=int, default=100)
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("train_window needs a GPU")

    def log(msg):
        print(msg, flush=True)

    net = train(args, log)
    log(json.dumps({"step": net.step, "out": args.out}))


if __name__ == "__main__":
    main()
