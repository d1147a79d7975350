"""FP64 CPU oracle of the learned warm start (a small convolutional network on
the seed grid that predicts the initial superpixel parameters for the EM).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library.

The network is not part of the paper: it replaces the grid initialisation of
Sec. III-C (mu_k = seed pixel, Sigma_s = diag(v_x^2, v_y^2), colour variances
lambda^2) by a prediction, after which the EM of Sec. III-B runs unchanged.
Definitions used by both the oracle and the kernels:

* positions: the n_x x n_y seed grid of each image, superpixel order
  k = k_y n_x + k_x;
* features (16 channels) of seed cell k, over the pixels
  [k_x v_x, (k_x+1) v_x) x [k_y v_y, (k_y+1) v_y), with s the seed pixel of
  Sec. III-C and h = floor(v / 2):
  0-2  (mean_L - 50) / 50, mean_a / 64, mean_b / 64,
  3-5  std_L / 16, std_a / 16, std_b / 16 (population standard deviations),
  6    min(k_x, k_y, n_x-1-k_x, n_y-1-k_y, 3) / 3,
  7-9  (colour(s) - mean) / 16,
  10-12 (mean over columns >= v_x - h  -  mean over columns < h) / 32,
  13-15 (mean over rows >= v_y - h  -  mean over rows < h) / 32
  (channels 10-15 are 0 when h = 0);
* network: conv3x3 16->32, ReLU, 32->32, ReLU, 32->32, ReLU, 32->10, zero
  padding at the grid border, out[y][x][o] = b[o] + sum_{t, i} W[o][t][i]
  in[y+dy_t][x+dx_t][i] with tap t = 3 (dy + 1) + (dx + 1);  weights and
  activations rounded to bfloat16 (round to nearest, ties to even), sums
  exact here (FP32 on the GPU);
* outputs o[0..9] -> theta^0 (an output whose bit is clear in the mask counts
  as 0): mu_x = s_x + v_x o0, mu_y = s_y + v_y o1, mu_c = colour(s) +
  lambda o_{2..4}, Sigma = diag(v_x^2 e^{2 o5}, v_y^2 e^{2 o6},
  lambda^2 e^{2 o7}, lambda^2 e^{2 o8}, lambda^2 e^{2 o9}) with every o5..o9
  clipped to [-4, 4], followed by the eigenvalue floors of Eqs. mlams, mlamc;
  a zero output is the grid initialisation of Sec. III-C exactly;
* targets from parameters theta* (of plain EM after some passes): the inverse
  map, each log-scale clipped to [-4, 4];
* loss: mean over positions and the 10 channels of (o - target)^2.
"""
from __future__ import annotations

import math

import numpy as np

C_IN, C_HID, C_OUT = 16, 32, 10
LAYERS = [(C_IN, C_HID), (C_HID, C_HID), (C_HID, C_HID), (C_HID, C_OUT)]
LOG_CLIP = 4.0


def taps():
    return [(t // 3 - 1, t % 3 - 1) for t in range(9)]      # (dy, dx)


def param_count() -> int:
    return sum(co * 9 * ci + co for ci, co in LAYERS)


def unpack(params: np.ndarray):
    """Flat FP32 parameter vector -> [(W (co, 9, ci), b (co,))] per layer."""
    out, o = [], 0
    for ci, co in LAYERS:
        W = params[o:o + co * 9 * ci].reshape(co, 9, ci)
        o += co * 9 * ci
        b = params[o:o + co]
        o += co
        out.append((W, b))
    assert o == params.size
    return out


def bf16_round(x) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(a), a, out)


# ---------------------------------------------------------------------------
# conv3x3 on one (ny, nx, c) grid
# ---------------------------------------------------------------------------

def conv3x3(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    ny, nx, _ = x.shape
    co = W.shape[0]
    xp = np.zeros((ny + 2, nx + 2, x.shape[2]))
    xp[1:-1, 1:-1] = x
    out = np.broadcast_to(b.astype(np.float64), (ny, nx, co)).copy()
    for t, (dy, dx) in enumerate(taps()):
        sh = xp[1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]          # in[y+dy][x+dx]
        out += sh @ W[:, t, :].astype(np.float64).T
    return out


def conv3x3_backward(x: np.ndarray, W: np.ndarray, dy_: np.ndarray):
    """Gradients of sum(dy * conv3x3(x, W, b)) with respect to x, W and b."""
    ny, nx, ci = x.shape
    xp = np.zeros((ny + 2, nx + 2, ci))
    xp[1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dW = np.zeros(W.shape)
    for t, (dy, dx) in enumerate(taps()):
        sh = xp[1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
        dW[:, t, :] = np.einsum("yxo,yxi->oi", dy_, sh)
        dxp[1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx] += dy_ @ W[:, t, :].astype(np.float64)
    db = dy_.sum(axis=(0, 1))
    return dxp[1:-1, 1:-1], dW, db


def forward(params: np.ndarray, x0: np.ndarray, round_bf16: bool = True):
    """Network forward on one grid.  Returns (out (ny, nx, 10), activations)
    where activations[l] is the (bf16-rounded) input of layer l."""
    layers = unpack(params)
    r = bf16_round if round_bf16 else (lambda v: np.asarray(v, np.float64))
    acts = [r(x0).astype(np.float64)]
    h = acts[0]
    for li, (W, b) in enumerate(layers):
        y = conv3x3(h, r(W).astype(np.float64), b.astype(np.float64))
        if li < len(layers) - 1:
            h = r(np.maximum(y, 0.0).astype(np.float32)).astype(np.float64) if round_bf16 \
                else np.maximum(y, 0.0)
            acts.append(h)
        else:
            return y, acts


def loss_and_grads(params: np.ndarray, x0: np.ndarray, target: np.ndarray, count: int,
                   round_bf16: bool = False):
    """Mean-squared error (sum over this grid / (count * 10)) and its gradient
    with respect to the flat parameter vector.  With round_bf16 the forward
    uses bf16-rounded weights and activations (the gradient then treats the
    rounding as identity)."""
    layers = unpack(params)
    r = bf16_round if round_bf16 else (lambda v: np.asarray(v, np.float64))
    out, acts = forward(params, x0, round_bf16)
    diff = out - target
    loss = float(np.sum(diff * diff)) / (count * C_OUT)
    g = 2.0 * diff / (count * C_OUT)
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        dx, dW, db = conv3x3_backward(acts[li], r(W).astype(np.float64), g)
        grads.append((dW, db))
        if li > 0:
            g = dx * (acts[li] > 0)
    flat = []
    for dW, db in reversed(grads):
        flat += [dW.reshape(-1), db]
    return loss, np.concatenate(flat)


# ---------------------------------------------------------------------------
# features, targets and theta^0
# ---------------------------------------------------------------------------

def features(lab: np.ndarray, vx: int, vy: int, nx: int, ny: int) -> np.ndarray:
    lab = np.asarray(lab, dtype=np.float64)
    f = np.zeros((ny, nx, C_IN))
    hx, hy = vx // 2, vy // 2
    for ky in range(ny):
        for kx in range(nx):
            cell = lab[ky * vy:(ky + 1) * vy, kx * vx:(kx + 1) * vx]
            px = cell.reshape(-1, 3)
            m = px.mean(axis=0)
            s = px.std(axis=0)
            sx, sy = seed_xy(vx, vy, kx, ky)
            f[ky, kx, 0:3] = [(m[0] - 50.0) / 50.0, m[1] / 64.0, m[2] / 64.0]
            f[ky, kx, 3:6] = s / 16.0
            f[ky, kx, 6] = min(kx, ky, nx - 1 - kx, ny - 1 - ky, 3) / 3.0
            f[ky, kx, 7:10] = (lab[sy, sx] - m) / 16.0
            if hx > 0:
                f[ky, kx, 10:13] = (cell[:, vx - hx:].reshape(-1, 3).mean(0)
                                    - cell[:, :hx].reshape(-1, 3).mean(0)) / 32.0
            if hy > 0:
                f[ky, kx, 13:16] = (cell[vy - hy:].reshape(-1, 3).mean(0)
                                    - cell[:hy].reshape(-1, 3).mean(0)) / 32.0
    return f


def seed_xy(vx, vy, kx, ky):
    return kx * vx + vx // 2, ky * vy + vy // 2


ALL_OUTPUTS = (1 << C_OUT) - 1


def theta0_rows(out: np.ndarray, lab: np.ndarray, vx: int, vy: int, lam: float,
                mask: int = ALL_OUTPUTS) -> np.ndarray:
    """Rows (mu_x mu_y mu_L mu_a mu_b S_xx S_xy S_yy S_LL S_aa S_ab S_bb N) from
    network outputs (before the eigenvalue floors, which set_params applies)."""
    ny, nx, _ = out.shape
    lab = np.asarray(lab, dtype=np.float64)
    use = np.array([(mask >> c) & 1 for c in range(C_OUT)], dtype=np.float64)
    rows = np.zeros((ny * nx, 13))
    for ky in range(ny):
        for kx in range(nx):
            o = out[ky, kx].astype(np.float64) * use
            sx, sy = seed_xy(vx, vy, kx, ky)
            ls = np.clip(o[5:10], -LOG_CLIP, LOG_CLIP)
            k = ky * nx + kx
            rows[k, 0:5] = [sx + vx * o[0], sy + vy * o[1], *(lab[sy, sx] + lam * o[2:5])]
            rows[k, 5] = vx * vx * math.exp(2 * ls[0])
            rows[k, 7] = vy * vy * math.exp(2 * ls[1])
            rows[k, 8] = lam * lam * math.exp(2 * ls[2])
            rows[k, 9] = lam * lam * math.exp(2 * ls[3])
            rows[k, 11] = lam * lam * math.exp(2 * ls[4])
    return rows


def targets(rows: np.ndarray, lab: np.ndarray, vx: int, vy: int, nx: int, ny: int,
            lam: float) -> np.ndarray:
    rows = np.asarray(rows, dtype=np.float64)
    lab = np.asarray(lab, dtype=np.float64)
    t = np.zeros((ny, nx, C_OUT))
    for ky in range(ny):
        for kx in range(nx):
            r = rows[ky * nx + kx]
            sx, sy = seed_xy(vx, vy, kx, ky)
            t[ky, kx, 0] = (r[0] - sx) / vx
            t[ky, kx, 1] = (r[1] - sy) / vy
            t[ky, kx, 2:5] = (r[2:5] - lab[sy, sx]) / lam
            var = [r[5] / (vx * vx), r[7] / (vy * vy), r[8] / lam ** 2, r[9] / lam ** 2,
                   r[11] / lam ** 2]
            t[ky, kx, 5:10] = np.clip(0.5 * np.log(var), -LOG_CLIP, LOG_CLIP)
    return t
