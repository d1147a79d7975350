"""Segmentation quality of the method on held-out synthetic 481x321 images with
ground-truth region maps: boundary recall, under-segmentation error (Eq. ue)
and achievable segmentation accuracy (Eq. asa), before and after the
connectivity post-processing, for the paper's setting (T = 10, lambda = 8,
eps_c = 8), for EM run to the 1e-5 stop rule from the grid and from the
learned warm start, for sweeps of lambda and eps_c (Sec. IV, effect of
lambda and eps_c) at T = 10, and for the other covariance models at T = 10:
the 3x3 colour block, the full 5x5 Sigma (Sec. III-B holds that full matrices
do not improve accuracy), and the L channel alone as a grayscale image.

    python -m paper_1612_08792_amd.quality [--images 256] [--K 400]

Prints one JSON object per setting and a markdown table.  Every step runs in
the library's kernels."""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from paper_1612_08792_amd import train_warmstart, warmstart  # noqa: E402
from paper_1612_08792_amd.gmmsp import GMMSP  # noqa: E402


def measure(m: GMMSP, x, lab, gt, n_regions):
    """x: the EM input; lab: the three channels the connectivity step compares."""
    labels, _ = m.label(x)
    raw, _ = m.metrics(labels, gt, n_regions)
    comp, counts = m.connectivity(lab, labels, compact=True)
    con, _ = m.metrics(comp, gt, n_regions, n_sp=counts[:, 3])
    return dict(BR=float(raw[:, 0].mean()), UE=float(raw[:, 1].mean()), ASA=float(raw[:, 2].mean()),
                BR_conn=float(con[:, 0].mean()), UE_conn=float(con[:, 1].mean()),
                ASA_conn=float(con[:, 2].mean()), segments_conn=float(counts[:, 3].mean()))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--images", type=int, default=256)
    ap.add_argument("--K", type=int, default=400)
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    ims = [synth.config4_image(20000 + i, dev) for i in range(args.images)]
    lab = synth.pack_batch(ims).to(dev)
    gt = torch.cat([im.regions.reshape(-1).to(dev) for im in ims]).to(torch.int32).contiguous()
    sizes = [(im.W, im.H) for im in ims]
    n_regions = 40
    rows = []

    # grayscale: the L channel; the connectivity step compares (L, 0, 0)
    lab3 = lab.reshape(-1, 3)
    gray = lab3[:, 0].contiguous()
    gray3 = torch.zeros_like(lab3)
    gray3[:, 0] = gray

    def run(name, lam=8.0, eps_c=8.0, T=10, tol=0.0, warm=None, cov_mode=0):
        m = GMMSP(sizes, K=args.K, lam=lam, eps_c=eps_c, device=dev, cov_mode=cov_mode)
        x, xc = (gray, gray3.reshape(-1)) if cov_mode == 3 else (lab, lab)
        if warm is not None:
            warmstart.warm_start(m, lab, warm, train_warmstart.MASK)
        else:
            m.init_seeds(x)
        it = m.em_iterate(x, T, tol)
        r = dict(setting=name, lam=lam, eps_c=eps_c, passes=float(np.mean(it)),
                 **measure(m, x, xc, gt, n_regions))
        print(json.dumps(r), flush=True)
        rows.append(r)

    run("paper: T = 10")
    run("plain to rel-tol 1e-5", T=200, tol=1e-5)
    params = warmstart.load(train_warmstart.DEFAULT_OUT, dev)
    run("warm start to rel-tol 1e-5", T=200, tol=1e-5, warm=params)
    for lam in (4.0, 6.0, 10.0, 12.0):
        run(f"lambda = {lam:g}, T = 10", lam=lam)
    for eps_c in (2.0, 4.0, 16.0, 32.0):
        run(f"eps_c = {eps_c:g}, T = 10", eps_c=eps_c)
    run("3x3 colour block (cov_mode 1), T = 10", cov_mode=1)
    run("full 5x5 Sigma (cov_mode 2), T = 10", cov_mode=2)
    run("grayscale L only (cov_mode 3), T = 10", cov_mode=3)
    print("| setting | passes | BR | UE | ASA | BR conn. | UE conn. | ASA conn. | segments conn. |")
    print("|---|---:|---:|---:|---:|---:|---:|---:|---:|")
    for r in rows:
        print(f"| {r['setting']} | {r['passes']:.1f} | {r['BR']:.4f} | {r['UE']:.4f} | {r['ASA']:.4f} | "
              f"{r['BR_conn']:.4f} | {r['UE_conn']:.4f} | {r['ASA_conn']:.4f} | {r['segments_conn']:.1f} |")


if __name__ == "__main__":
    main()
