"""Write the stored expected values of the large-image parity test.

Calls only the FP64 oracle (``oracle/``) on the seeded synthetic input of the
1920x1080 workload (300 Voronoi regions, seed 1, K = 2000, T = 20 EM
iterations).  Output: ``cfg2_oracle.npz`` next to this file.

    python tests/golden/make_golden.py
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import gmm_oracle as O  # noqa: E402

N_SAMPLE = 4000


def lab_digest(lab: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(lab, dtype=np.float32).tobytes()).hexdigest()


def main():
    t0 = time.time()
    im = synth.config2_image()
    lab = im.lab.numpy()
    g = O.make_grid(im.W, im.H, K=im.K)
    res = O.run_em(lab, g, O.Params(), max_iters=20)
    rng = np.random.default_rng(2024)
    pix = np.sort(rng.choice(im.W * im.H, N_SAMPLE, replace=False))
    Rs = O.to_slots(g, res["cand"], res["R"]).reshape(-1, 9)[pix]
    # near ties (two largest posteriors within 2e-4) are excluded from the label check
    Rsort = np.sort(res["R"].reshape(-1, 9), axis=1)
    tie = (Rsort[:, -1] - Rsort[:, -2]) <= 2e-4
    np.savez_compressed(
        os.path.join(HERE, "cfg2_oracle.npz"),
        lab_sha256=np.array(lab_digest(lab)),
        grid=np.array([g.vx, g.vy, g.nx, g.ny]),
        theta=O.theta_to_rows(res["theta"]),
        ll_hist=np.array(res["ll_hist"]),
        ll_final=np.array(res["ll_final"]),
        labels=res["labels"].astype(np.int16),
        tie_bits=np.packbits(tie),
        n_pix=np.array(tie.size),
        sample_pix=pix.astype(np.int64),
        sample_R=Rs,
    )
    print(f"cfg2 golden written in {time.time() - t0:.1f} s")


if __name__ == "__main__":
    main()
