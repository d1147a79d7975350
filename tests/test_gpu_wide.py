"""The widest image a batch may hold (2^24 pixels, GMMSP_MAX_WIDTH): two EM
passes of the slot-lane pass on a 2^24 x 64 image made by repeating one
1024 x 64 tile, a 1.07 Gpx image.  With a seed spacing of 32 the seed grid
repeats with the tile, and two passes reach only a few cells, so the
superpixels of the image's first tile have the parameters of the first tile of
a three-tile image, and those of its last-but-one tile (the pixels at the
largest offsets the pass addresses) the parameters of the three-tile image's
middle tile, moved by the tiles between them.  The three-tile image goes
through the FP64 oracle; the bar is the trajectory tolerance."""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import gmm_oracle as O
from paper_1612_08792_amd.gmmsp import GMMSP
from parity_helpers import assert_theta_close

pytestmark = pytest.mark.gpu

TW, H, V = 1024, 64, 32   # tile width, image height, seed spacing
W = 1 << 24               # the widest image


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_widest_image_matches_oracle_at_both_ends():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dev = torch.device("cuda:0")
    tile = synth.voronoi_lab(TW, H, 40, 3.0, 21, (TW // V) * (H // V)).lab  # (H, TW, 3)
    g3 = O.make_grid(3 * TW, H, vx=V, vy=V)
    want = O.theta_to_rows(O.run_em(tile.repeat(1, 3, 1).numpy(), g3, max_iters=2)["theta"])

    say(f"{W}x{H} image ({W * H / 1e9:.2f} Gpx), seed spacing {V}, T 2")
    lab = tile.to(dev).repeat(1, W // TW, 1).reshape(-1).contiguous()
    m = GMMSP([(W, H)], v=V, device=dev)
    m.set_estep_kernel(1)
    m.init_seeds(lab)
    assert list(m.em_iterate(lab, 2)) == [2]
    rows = m.get_params()
    m.close()
    del lab, m
    torch.cuda.empty_cache()

    nx, n3, per = W // V, 3 * TW // V, TW // V
    ky = np.repeat(np.arange(H // V), per)
    kx = np.tile(np.arange(per), H // V)
    e0 = assert_theta_close(rows[ky * nx + kx], want[ky * n3 + kx], 1e-3, what="first tile")
    far = rows[ky * nx + (nx - 2 * per) + kx].copy()
    far[:, 0] -= W - 3 * TW          # x of the last-but-one tile against the middle tile
    e1 = assert_theta_close(far, want[ky * n3 + per + kx], 1e-3, what="last-but-one tile")
    say("first tile", e0, "last-but-one tile", e1)
