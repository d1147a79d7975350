"""Learned warm start: training and inference drivers around the library's
network kernels (every forward, backward and optimiser step runs in
libgmmsp.so; this module only orders the calls and holds torch buffers).

The network predicts theta^0 from per-seed-cell colour statistics; EM then
runs unchanged.  Training targets are the converged parameters of plain EM on
the training images, produced by the same library."""
from __future__ import annotations

import os
import time

import numpy as np
import torch

from . import _lib
from .gmmsp import GMMSP

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS_DIR = os.path.join(HERE, "weights")
LAYERS = [(16, 32), (32, 32), (32, 32), (32, 10)]
# outputs the trained network's theta^0 applies: the five mean offsets and the
# two spatial log-scales (the colour variances stay at lambda^2)
APPLY_MASK = 0b0001111111


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights for the ReLU layers, a small last layer (so the first
    predictions stay close to the grid initialisation), zero biases."""
    rng = np.random.default_rng(seed)
    out = []
    for li, (ci, co) in enumerate(LAYERS):
        std = np.sqrt(2.0 / (9 * ci)) if li < 3 else 1e-3
        out.append(rng.normal(0.0, std, co * 9 * ci))
        out.append(np.zeros(co))
    p = np.concatenate(out).astype(np.float32)
    assert p.size == _lib.WS_NPARAM
    return p


def converge_plain(m: GMMSP, lab: torch.Tensor, cap: int, tol: float) -> np.ndarray:
    m.init_seeds(lab)
    return m.em_iterate(lab, cap, tol)


def train(images, device="cuda", epochs: int = 30, batch_images: int = 64, lr: float = 2e-3,
          seed: int = 0, cap: int = 100, tol: float = 1e-5, target_passes: int = 0, log=None):
    """Train on a list of synth.VoronoiImage.  Targets are the parameters of
    plain EM after ``target_passes`` passes, or at convergence (relative LL
    change <= tol, at most cap passes) when target_passes is 0.  Returns
    (params tensor, info)."""
    dev = torch.device(device)
    import synth
    t0 = time.time()
    lab = synth.pack_batch(images).to(dev).contiguous()
    m = GMMSP([(im.W, im.H) for im in images], K=[im.K for im in images], device=dev)
    if target_passes > 0:
        m.init_seeds(lab)
        iters = m.em_iterate(lab, target_passes, 0.0)
    else:
        iters = converge_plain(m, lab, cap, tol)
    m.ws_attach()
    m.ws_features(lab)
    m.ws_targets(lab)
    t_targets = time.time() - t0
    params = torch.from_numpy(init_params(seed)).to(dev)
    mom = torch.zeros_like(params)
    vel = torch.zeros_like(params)
    n = len(images)
    rng = np.random.default_rng(seed + 1)
    starts = list(range(0, n, batch_images))
    losses = []
    step = 0
    for ep in range(epochs):
        order = rng.permutation(len(starts))
        ep_loss = 0.0
        for j in order:
            b0 = starts[j]
            b1 = min(n, b0 + batch_images)
            step += 1
            # cosine decay of the learning rate over the run
            frac = step / (epochs * len(starts))
            lr_t = lr * 0.5 * (1.0 + np.cos(np.pi * min(frac, 1.0)))
            ep_loss += m.ws_train_step(params, mom, vel, step, max(lr_t, lr * 1e-3), b0, b1)
        losses.append(ep_loss / len(starts))
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.5f}")
    torch.cuda.synchronize(dev)
    info = dict(plain_iters_mean=float(np.mean(iters)), losses=losses, steps=step,
                t_targets=t_targets, t_total=time.time() - t0, images=n)
    m.close()
    return params, info


def warm_start(m: GMMSP, lab: torch.Tensor, params: torch.Tensor,
               mask: int = _lib.WS_ALL_OUTPUTS, guard: bool = False, want_flags: bool = False):
    """theta^0 of every image of the handle from the network.  With guard, an
    image whose L(theta^0) would be lower than with the grid seeds keeps the
    seeds (returns the per-image flags when want_flags)."""
    m.ws_attach()
    m.ws_features(lab)
    m.ws_forward(params)
    if guard:
        return m.ws_apply_guarded(lab, mask, want_flags)
    m.ws_apply(lab, mask)
    return None


def save(params: torch.Tensor, path: str, info: dict):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, params=params.detach().cpu().numpy().astype(np.float32),
             losses=np.asarray(info.get("losses", []), dtype=np.float64),
             meta=np.array(repr({k: v for k, v in info.items() if k != "losses"})))


def load(path: str, device="cuda") -> torch.Tensor:
    with np.load(path, allow_pickle=False) as z:
        p = z["params"].astype(np.float32)
    if p.size != _lib.WS_NPARAM:
        raise ValueError(f"{path}: {p.size} parameters, expected {_lib.WS_NPARAM}")
    return torch.from_numpy(p).to(torch.device(device))


def passes_to_target(hist: np.ndarray, target: float, rel: float = 1e-4) -> int:
    """First pass t with L(theta^t) >= target - rel |target| (len(hist) if none)."""
    thr = target - rel * abs(target)
    for t, L in enumerate(hist):
        if L >= thr:
            return t
    return len(hist)
