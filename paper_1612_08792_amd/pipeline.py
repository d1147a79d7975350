"""Algorithm 1 end to end on a batch of 8-bit sRGB images, every stage in the
library's kernels, with the time of each stage:

    sRGB -> CIELAB, learned warm start (features, network, theta^0), EM to
    the 1e-5 relative-change stop rule, labels (Eq. obtLi), connectivity
    post-processing, accuracy measures (BR, Eq. ue, Eq. asa) against the
    ground-truth regions.

    python -m paper_1612_08792_amd.pipeline [--images 32] [--steps 3]

Synthetic 3840x2160 images (the 4K workload's Voronoi law drawn in sRGB).
Prints one JSON line."""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from paper_1612_08792_amd import train_warmstart, warmstart  # noqa: E402
from paper_1612_08792_amd.gmmsp import GMMSP, srgb8_to_lab  # noqa: E402


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--images", type=int, default=32)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--regions", type=int, default=2000)
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    W, H = 3840, 2160
    rgbs, gts = [], []
    for i in range(args.images):
        rgb, reg = synth.voronoi_srgb8(W, H, args.regions, (1.0, 6.0), 40000 + i, dev)
        rgbs.append(rgb.reshape(-1, 3))
        gts.append(reg.reshape(-1))
    rgb = torch.cat(rgbs).contiguous()
    gt = torch.cat(gts).to(torch.int32).contiguous()
    del rgbs, gts
    n_pix = W * H * args.images
    params = warmstart.load(train_warmstart.DEFAULT_OUT, dev)
    m = GMMSP([(W, H)] * args.images, K=10000, device=dev)
    lab = torch.empty((n_pix, 3), dtype=torch.float32, device=dev)
    names = ["srgb_to_lab", "warm_start", "em", "labels", "connectivity", "measures"]

    def step():
        t = []

        def mark():
            torch.cuda.synchronize(dev)
            t.append(time.perf_counter())
        mark()
        srgb8_to_lab(rgb, lab)
        mark()
        flat = lab.reshape(-1)
        # the guarded start: the grid seeds wherever they give the higher L(theta^0)
        warmstart.warm_start(m, flat, params, warmstart.APPLY_MASK, guard=True)
        mark()
        it = m.em_iterate(flat, 200, 1e-5)
        mark()
        labels, _ = m.label(flat, want_ll=False)
        mark()
        comp, counts = m.connectivity(flat, labels, compact=True)
        mark()
        vals, _ = m.metrics(comp, gt, args.regions, n_sp=counts[:, 3])
        mark()
        return np.diff(t), it, counts, vals

    # schedules of the EM (waves per cell, gather lanes) timed on this batch
    srgb8_to_lab(rgb, lab)
    m.autotune(lab.reshape(-1), passes=3, cache=None)
    step()                                           # warm-up
    rows = [step() for _ in range(args.steps)]
    ms = np.mean([r[0] for r in rows], axis=0) * 1e3
    _, it, counts, vals = rows[-1]
    out = dict(images=args.images, pixels=n_pix, stage_ms={n: round(float(v), 3) for n, v in zip(names, ms)},
               total_ms=round(float(ms.sum()), 3), mpix_per_s=round(n_pix / ms.sum() / 1e3, 1),
               em_passes_mean=float(np.mean(it)), segments_mean=float(counts[:, 3].mean()),
               BR=float(vals[:, 0].mean()), UE=float(vals[:, 1].mean()), ASA=float(vals[:, 2].mean()))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
