"""E-step rate of each covariance model on a batch of synthetic 4K images:
split colour blocks (cov_mode 0), the 3x3 colour block (1), the full 5x5 Sigma
(2) and grayscale images (3, the L channel as the intensity).  Each model runs
`--passes` fixed EM passes from the grid seeds; the library times its E-step
launches with HIP events on the launch stream.

    python -m paper_1612_08792_amd.modes_rate [--images 8] [--passes 10]

Prints one JSON line per model."""
from __future__ import annotations

import argparse
import json
import os
import sys

import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from paper_1612_08792_amd.gmmsp import GMMSP  # noqa: E402


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--images", type=int, default=8)
    ap.add_argument("--passes", type=int, default=10)
    ap.add_argument("--modes", type=str, default="0,1,2,3")
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    ims = synth.config5_batch(device=dev, n_images=args.images)
    lab = synth.pack_batch(ims).contiguous()
    gray = lab.reshape(-1, 3)[:, 0].contiguous()
    for mode in (int(x) for x in args.modes.split(",")):
        x = gray if mode == 3 else lab.reshape(-1)
        m = GMMSP([(im.W, im.H) for im in ims], K=10000, device=dev, cov_mode=mode)
        m.init_seeds(x)
        m.em_iterate(x, 2)                      # warm-up
        m.profile(True)
        m.profile_read(True)
        m.init_seeds(x)
        m.em_iterate(x, args.passes)
        p = m.profile_read(True)
        print(json.dumps({
            "cov_mode": mode, "images": args.images, "pixels": m.n_pixels,
            "launches": p["launches"], "estep_ms_per_launch": round(p["estep_ms"] / p["launches"], 4),
            "gpx_per_s": round(p["pixel_evals"] / (p["estep_ms"] / 1e3) / 1e9, 2),
        }), flush=True)
        m.close()
        del m


if __name__ == "__main__":
    main()
