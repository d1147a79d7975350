"""GPU sRGB -> CIELAB front end against the FP64 oracle: every one of the 2^24
8-bit colours, ragged lengths, and the HBM rate at 4K batch size.

Tolerance: FP32 arithmetic on values below 130 with a few roundings per step
and the a*, b* differences scaled by 500 and 200: a few 1e-5; the test allows
5e-4 (absolute, in L*a*b* units)."""
import sys
import time

import numpy as np
import pytest
import torch

from oracle import color_oracle as C
from paper_1612_08792_amd.gmmsp import srgb8_to_lab

pytestmark = pytest.mark.gpu
TOL = 5e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def test_every_8bit_colour(dev):
    v = np.arange(1 << 24, dtype=np.uint32)
    rgb = np.stack([(v >> 16) & 255, (v >> 8) & 255, v & 255], -1).astype(np.uint8)
    got = srgb8_to_lab(torch.from_numpy(rgb).to(dev)).cpu().numpy().astype(np.float64)
    want = C.srgb8_to_lab(rgb)
    err = np.abs(got - want).max(axis=0)
    say("max |error| over 2^24 colours (L, a, b):", err)
    assert err.max() <= TOL


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 1001, 4099])
def test_ragged_lengths(dev, n):
    rng = np.random.default_rng(n)
    rgb = rng.integers(0, 256, (n, 3)).astype(np.uint8)
    out = torch.full((n, 3), float("nan"), device=dev)
    srgb8_to_lab(torch.from_numpy(rgb).to(dev), out)
    got = out.cpu().numpy()
    assert np.isfinite(got).all()
    assert np.abs(got - C.srgb8_to_lab(rgb)).max() <= TOL


def test_4k_batch_rate(dev):
    n = 8 * 3840 * 2160
    rgb = torch.randint(0, 256, (n, 3), dtype=torch.uint8, device=dev)
    out = torch.empty((n, 3), dtype=torch.float32, device=dev)
    srgb8_to_lab(rgb, out)
    torch.cuda.synchronize()
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        srgb8_to_lab(rgb, out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    say(f"8 x 4K sRGB -> Lab: {dt * 1e3:.3f} ms, {15 * n / dt / 1e9:.0f} GB/s algorithmic, "
        f"{n / dt / 1e9:.1f} Gpx/s")
    idx = torch.randint(0, n, (4096,), device=dev)
    want = C.srgb8_to_lab(rgb[idx].cpu().numpy())
    assert np.abs(out[idx].cpu().numpy() - want).max() <= TOL
