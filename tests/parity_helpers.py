"""Comparison helpers for GPU-vs-oracle parity.  Tolerances (FP32 E/M arithmetic
with FP64 reductions and FP64 shape control, against the FP64 oracle):

* trajectory after T iterations: posteriors abs <= 1e-4; means
  |d mu_j| / sqrt(Sigma_jj) <= 1e-3 (error in units of the superpixel's own
  standard deviation); each covariance block ||d Sigma_b||_F / ||Sigma_b||_F
  <= 1e-3; labels agree on >= 99.9 % of the pixels whose two largest oracle
  posteriors differ by more than 2e-4 (near ties excepted);
* one step from an identical theta^t: posteriors abs <= 1e-5, theta^(t+1)
  within 1e-5 in the same relative measures;
* integer seed-grid and candidate indexing: bit-exact.
"""
import numpy as np

from oracle import gmm_oracle as O

TIE = 2e-4

BLOCKS = {"s": ([5, 6, 7], [[5, 6], [6, 7]]), "L": ([8], [[8]]),
          "ab": ([9, 10, 11], [[9, 10], [10, 11]])}


def block_matrix(rows, idx2):
    return np.stack([np.stack([rows[:, j] for j in r], -1) for r in idx2], -2)


def theta_errors(gpu_rows: np.ndarray, ora_rows: np.ndarray, mask=None):
    """Largest mean error in std units and largest relative Frobenius error per block."""
    if mask is None:
        mask = np.ones(len(ora_rows), bool)
    g, o = gpu_rows[mask], ora_rows[mask]
    var = np.stack([o[:, 5], o[:, 7], o[:, 8], o[:, 9], o[:, 11]], 1)
    mean_err = np.abs(g[:, :5] - o[:, :5]) / np.sqrt(var)
    out = {"mean": float(mean_err.max()) if len(g) else 0.0}
    for name, (_, idx2) in BLOCKS.items():
        Gm, Om = block_matrix(g, idx2), block_matrix(o, idx2)
        num = np.linalg.norm((Gm - Om).reshape(len(g), -1), axis=1)
        den = np.linalg.norm(Om.reshape(len(g), -1), axis=1)
        out[name] = float((num / den).max()) if len(g) else 0.0
    out["mass"] = float(np.max(np.abs(g[:, 12] - o[:, 12]) / np.maximum(o[:, 12], 1.0))) \
        if len(g) else 0.0
    return out


def assert_theta_close(gpu_rows, ora_rows, tol, mask=None, what=""):
    e = theta_errors(gpu_rows, ora_rows, mask)
    bad = {k: v for k, v in e.items() if k != "mass" and v > tol}
    assert not bad, f"{what} theta errors above {tol}: {e}"
    return e


def label_agreement(gpu_labels: np.ndarray, ora_labels: np.ndarray, margin: np.ndarray):
    """Fraction of non-tie pixels with equal labels, and the tie count."""
    nontie = margin > TIE
    agree = (gpu_labels == ora_labels)[nontie].mean() if nontie.any() else 1.0
    return float(agree), int((~nontie).sum())


def oracle_margin(R: np.ndarray) -> np.ndarray:
    s = np.sort(R.reshape(-1, R.shape[-1]), axis=1)
    return s[:, -1] - s[:, -2]


def oracle_slots(g, cand, values):
    return O.to_slots(g, cand, values).reshape(-1, 9)


def window_step(g, z, cand, theta_t, k, R_gpu_window):
    """Sampled parity on the window I_k (Eq. Ik) of superpixel k: the oracle's
    E-step on the window's pixels at theta_t (Eq. Rik), compared with the GPU
    posteriors of the same pixels in slot layout (R_gpu_window: (h, w, 9)), and
    the oracle's M-step of k from it (Eqs. UpdateMu .. eigdecrc).  Returns (max
    |R_gpu - R_oracle| on the window, the oracle's theta^{t+1} row of k, the
    oracle posteriors and candidates of the window)."""
    xb, xe, yb, ye = O.window(g, int(k))
    zw, cw = z[yb:ye, xb:xe], cand[yb:ye, xb:xe]
    Rw, _, _ = O.estep(zw, cw, theta_t)
    # the oracle's posteriors by neighbour slot s = 3 (dy + 1) + (dx + 1)
    sub = np.zeros((ye - yb, xe - xb, 9))
    cx = (np.arange(xb, xe) // g.vx)[None, :, None]
    cy = (np.arange(yb, ye) // g.vy)[:, None, None]
    s = 3 * (cw // g.nx - cy + 1) + (cw % g.nx - cx + 1)
    yy, xx, jj = np.nonzero(cw >= 0)
    sub[yy, xx, s[yy, xx, jj]] = Rw[yy, xx, jj]
    err = float(np.abs(R_gpu_window - sub).max())
    pos = (cw == k).argmax(-1)
    rk = np.take_along_axis(Rw, pos[..., None], -1).reshape(-1)
    mu, sig, Nk = O.mstep_one(zw.reshape(-1, z.shape[-1]), rk, theta_t.mu[k], theta_t.sigma[k],
                              O.Params())
    row = O.theta_to_rows(O.Theta(mu[None], sig[None], np.array([Nk])))[0]
    return err, row, Rw, cw
