"""Synthetic Voronoi-CIELAB images (inputs only; no EM arithmetic here).

Stand-in for the natural images the paper segments (BSDS500, 481x321 and
321x481, Sec. IV): the dataset is not available, so every workload is drawn from
one seeded law instead:

* ``n_regions`` sites uniform in [0, W) x [0, H);
* each pixel belongs to the nearest site (Euclidean distance measured at the
  integer pixel position; ties go to the lowest site index);
* region colour = (L0, a0, b0) + g_x (x - s_x) + g_y (y - s_y), with
  L0 ~ U[10, 90], a0, b0 ~ U[-60, 60] and each slope ~ U[-0.05, 0.05] per pixel;
* iid N(0, sigma^2) noise per pixel and channel, no clipping;
* stored as float32, interleaved (L, a, b) per pixel, row-major (index x + W y).

Draw order from ``numpy.random.default_rng(seed)``: site x, site y, L0, a0, b0,
slopes, then (only for a sigma range) sigma, then the noise field.  The region
map is returned as ground truth.  The nearest-site search runs in torch on any
device with exact float64 distances, so CPU and GPU produce the same map.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch


@dataclass
class VoronoiImage:
    lab: torch.Tensor          # (H, W, 3) float32
    regions: torch.Tensor      # (H, W) int32 ground-truth region id
    W: int
    H: int
    K: int                     # requested number of superpixels
    seed: int
    sigma: float


def _nearest_site(W: int, H: int, sx: np.ndarray, sy: np.ndarray,
                  device: torch.device) -> torch.Tensor:
    """Index of the nearest site for every pixel, ties to the lowest index."""
    dev = torch.device(device)
    tsx = torch.from_numpy(sx).to(dev, torch.float64)
    tsy = torch.from_numpy(sy).to(dev, torch.float64)
    xs = torch.arange(W, device=dev, dtype=torch.float64)
    dx2 = (xs[:, None] - tsx[None, :]) ** 2            # (W, S)
    n_sites = sx.shape[0]
    out = torch.empty((H, W), dtype=torch.int32, device=dev)
    # rows per chunk so that the (rows, W, S) distance block stays ~64M doubles
    rows = max(1, min(H, (1 << 26) // max(1, W * n_sites)))
    for y0 in range(0, H, rows):
        y1 = min(H, y0 + rows)
        ys = torch.arange(y0, y1, device=dev, dtype=torch.float64)
        dy2 = (ys[:, None] - tsy[None, :]) ** 2        # (rows, S)
        d2 = dy2[:, None, :] + dx2[None, :, :]         # (rows, W, S)
        # torch.argmin returns the first index among equal minima
        out[y0:y1] = torch.argmin(d2, dim=2).to(torch.int32)
    return out


def voronoi_lab(W: int, H: int, n_regions: int, sigma, seed: int, K: int,
                device="cpu", rng: np.random.Generator | None = None) -> VoronoiImage:
    """One image of the Voronoi-Lab law.  ``sigma`` is a float or a (lo, hi) range."""
    if rng is None:
        rng = np.random.default_rng(seed)
    n = max(1, int(n_regions))
    sx = rng.uniform(0.0, W, n)
    sy = rng.uniform(0.0, H, n)
    L0 = rng.uniform(10.0, 90.0, n)
    a0 = rng.uniform(-60.0, 60.0, n)
    b0 = rng.uniform(-60.0, 60.0, n)
    g = rng.uniform(-0.05, 0.05, (n, 3, 2))            # [region, channel, axis]
    if isinstance(sigma, (tuple, list)):
        sig = float(rng.uniform(sigma[0], sigma[1]))
    else:
        sig = float(sigma)
    noise = rng.standard_normal((H, W, 3))

    dev = torch.device(device)
    reg = _nearest_site(W, H, sx, sy, dev)
    regl = reg.long()
    c0 = torch.from_numpy(np.stack([L0, a0, b0], axis=1)).to(dev)    # (n, 3)
    tg = torch.from_numpy(g).to(dev)
    tsx = torch.from_numpy(sx).to(dev)
    tsy = torch.from_numpy(sy).to(dev)
    xs = torch.arange(W, device=dev, dtype=torch.float64)[None, :]
    ys = torch.arange(H, device=dev, dtype=torch.float64)[:, None]
    relx = xs - tsx[regl]                                             # (H, W)
    rely = ys - tsy[regl]
    col = c0[regl] + tg[regl][..., 0] * relx[..., None] + tg[regl][..., 1] * rely[..., None]
    col = col + sig * torch.from_numpy(noise).to(dev)
    lab = col.to(torch.float32).contiguous()
    return VoronoiImage(lab=lab, regions=reg, W=W, H=H, K=K, seed=seed, sigma=sig)


def voronoi_srgb8(W: int, H: int, n_regions: int, sigma, seed: int,
                  device="cpu") -> tuple[torch.Tensor, torch.Tensor]:
    """The same Voronoi law drawn directly as 8-bit sRGB (for the colour front
    end): per region a colour c0 ~ U[20, 235]^3 and slopes ~ U[-0.05, 0.05]
    per px, N(0, sigma^2) noise, rounded and clipped to [0, 255].  Returns
    ((H, W, 3) uint8, (H, W) int32 region ids)."""
    rng = np.random.default_rng(seed)
    n = max(1, int(n_regions))
    sx = rng.uniform(0.0, W, n)
    sy = rng.uniform(0.0, H, n)
    c0 = rng.uniform(20.0, 235.0, (n, 3))
    g = rng.uniform(-0.05, 0.05, (n, 3, 2))
    sig = float(rng.uniform(sigma[0], sigma[1])) if isinstance(sigma, (tuple, list)) else float(sigma)
    noise = rng.standard_normal((H, W, 3))
    dev = torch.device(device)
    reg = _nearest_site(W, H, sx, sy, dev)
    regl = reg.long()
    tc = torch.from_numpy(c0).to(dev)
    tg = torch.from_numpy(g).to(dev)
    relx = torch.arange(W, device=dev, dtype=torch.float64)[None, :] - torch.from_numpy(sx).to(dev)[regl]
    rely = torch.arange(H, device=dev, dtype=torch.float64)[:, None] - torch.from_numpy(sy).to(dev)[regl]
    col = tc[regl] + tg[regl][..., 0] * relx[..., None] + tg[regl][..., 1] * rely[..., None]
    col = col + sig * torch.from_numpy(noise).to(dev)
    rgb = torch.clamp(torch.round(col), 0, 255).to(torch.uint8).contiguous()
    return rgb, reg


# ---------------------------------------------------------------------------
# The five workloads (sizes and seeds of the benchmark configurations)
# ---------------------------------------------------------------------------

def config1_image(device="cpu") -> VoronoiImage:
    """481x321, seed 0, 40 regions, sigma 3, K = 400 (BSDS-sized)."""
    return voronoi_lab(481, 321, 40, 3.0, 0, 400, device)


def config2_image(device="cpu") -> VoronoiImage:
    """1920x1080, seed 1, 300 regions, sigma 3, K = 2000."""
    return voronoi_lab(1920, 1080, 300, 3.0, 1, 2000, device)


def config3_batch(device="cpu", n_images: int = 64, first_seed: int = 100):
    """Uneven batch: W ~ U{320..1280}, H ~ U{240..720}, regions = WH // 4000,
    K = WH // 600, sigma 3.  W and H are the first two draws of each image's
    generator, the image law continues from the same generator."""
    out = []
    for s in range(first_seed, first_seed + n_images):
        rng = np.random.default_rng(s)
        W = int(rng.integers(320, 1281))
        H = int(rng.integers(240, 721))
        out.append(voronoi_lab(W, H, (W * H) // 4000, 3.0, s, (W * H) // 600,
                               device, rng=rng))
    return out


def config4_image(seed: int, device="cpu") -> VoronoiImage:
    """Warm-start training / held-out image: the 481x321 law of config 1."""
    return voronoi_lab(481, 321, 40, 3.0, seed, 400, device)


def config5_batch(device="cpu", n_images: int = 32, first_seed: int = 30000):
    """32 x 3840x2160, 2000 regions, sigma ~ U[1, 6] per image, K = 10000."""
    return [voronoi_lab(3840, 2160, 2000, (1.0, 6.0), s, 10000, device)
            for s in range(first_seed, first_seed + n_images)]


# 9 CIELAB colours: L in {10, 55, 100} x (a, b) in {(-45,-45), (45,-45), (0,50)};
# every pair is at least 45 apart in Lab.
BLOCK_PALETTE = np.array([[L, a, b] for L in (10.0, 55.0, 100.0)
                          for (a, b) in ((-45.0, -45.0), (45.0, -45.0), (0.0, 50.0))])


def separated_blocks(v: int, nbx: int, nby: int, device="cpu") -> VoronoiImage:
    """Tiling of v x v constant-colour blocks aligned with the seed grid
    (W = nbx v, H = nby v).  Block (bx, by) takes palette entry
    (bx mod 3) + 3 (by mod 3), so the nine blocks of any 3x3 neighbourhood all
    differ in colour.  No noise."""
    W, H = nbx * v, nby * v
    ys, xs = np.mgrid[0:H, 0:W]
    bx, by = xs // v, ys // v
    idx = (bx % 3) + 3 * (by % 3)
    lab = BLOCK_PALETTE[idx].astype(np.float32)
    regions = (by * nbx + bx).astype(np.int32)
    return VoronoiImage(lab=torch.from_numpy(lab).to(device),
                        regions=torch.from_numpy(regions).to(device),
                        W=W, H=H, K=nbx * nby, seed=-1, sigma=0.0)


def pack_batch(images, device=None) -> torch.Tensor:
    """Concatenate images back to back into one flat float32 buffer
    (image b starts at 3 * sum_{c<b} W_c H_c floats)."""
    parts = [im.lab.reshape(-1) for im in images]
    t = torch.cat(parts)
    return t if device is None else t.to(device)
