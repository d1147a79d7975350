"""Plain FP64 CPU oracle for the pixel-related GMM superpixel EM
(Ban, Liu and Cao, "Superpixel Segmentation Using Gaussian Mixture Model",
arXiv 1612.08792, Sec. III).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code,
constants or helpers with the HIP library: it is written from the paper's
equations, slowly and in float64, so that it can be read against the paper.

Conventions and readings (the paper is silent or garbled on these):

* pixel index i = x + W y, features z_i = (x_i, y_i, L_i, a_i, b_i) in raw units
  (integer pixel positions, CIELAB values as stored), D = 5 (Sec. III-A, Eq. gaussian);
* grid: v = isqrt(WH // K), which equals floor(sqrt(WH / K)) exactly (Eq. vxy),
  n_x = W // v_x, n_y = H // v_y, K = n_x n_y (Eq. nxyK);
* windows I_k exactly as Eq. Ik, so when W, H are not multiples of v the last
  column / row of windows reach the image border (no re-centring of seeds);
* cov_mode 0 (default): block-diagonal Sigma = diag(Sigma_s (x,y), sigma_L^2,
  Sigma_(a,b)) per Eq. BlockSigma1; cov_mode 1: diag(Sigma_s, Sigma_(L,a,b)) per
  Eq. BlockSigma; cov_mode 2: the full 5 x 5 Sigma of Eq. UpdateSig; cov_mode 3:
  a grayscale image, z_i = (x_i, y_i, I_i) with D = 3 and Sigma = diag(Sigma_s,
  sigma_I^2) (Sec. III-A, III-C);
* shape control clamps each eigenvalue of each block from below:
  lambda~ = max(lambda, eps), eps_s = 2 for the spatial block, eps_c for every
  colour (or intensity) block (Eqs. mlams, mlamc; the first branch keeps
  lambda(j) itself).  The paper defines the floors per block only; for the full
  Sigma (cov_mode 2) the floors act on Sigma scaled by F = diag(eps_s, eps_s,
  eps_c, eps_c, eps_c): the eigenvalues of F^-1/2 Sigma F^-1/2 are raised to 1,
  which is the paper's rule whenever Sigma is block diagonal and the maximum of
  the Gaussian likelihood under Sigma >= F in general;
* init (Sec. III-C): mu_k = z_j at the seed pixel
  j = k_x v_x + v_x // 2 + W (k_y v_y + v_y // 2), Sigma_s = diag(v_x^2, v_y^2),
  every colour variance lambda^2 (lambda = 8), colour covariances 0;
* E-step (Eq. Rik) evaluated in the log domain with the maximum subtracted, which
  is the same quantity and avoids 0/0 for far outliers;
* M-step (Eqs. UpdateMu, UpdateSigS, UpdateSigC): the mean first, then each block
  covariance about the new mean;
* a superpixel whose responsibility mass N_k = sum_{i in I_k} R_ik falls below
  n_min keeps its previous mean and covariance (0/0 guard);
* the objective is L(theta) = sum_i ln sum_{k in K_i} p(z_i; theta_k) (Eq. ftheta,
  second form), the constant sum_i ln P_i left out;
* iteration (Algorithm 1): E-step with theta^0, then T times {M-step, E-step}.
  With a relative tolerance, the loop also stops at the first t >= 1 with
  |L(theta^t) - L(theta^(t-1))| <= tol |L(theta^(t-1))|, keeping theta^t;
* labels (Eq. obtLi): argmax of the posterior over K_i, ties to the smallest k.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

LN_2PI = math.log(2.0 * math.pi)
D = 5                                   # components of z = (x, y, L, a, b) of a colour image
MAXC = 9                                # |K_i| <= 9 (Sec. III-D)


# ---------------------------------------------------------------------------
# Seed grid, windows and candidate sets (Sec. III-A)
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Grid:
    W: int
    H: int
    vx: int
    vy: int
    nx: int
    ny: int

    @property
    def K(self) -> int:
        return self.nx * self.ny


def make_grid(W: int, H: int, K: int | None = None, vx: int | None = None,
              vy: int | None = None) -> Grid:
    """Eq. vxy (from K) or the given v_x, v_y; then Eq. nxyK."""
    if W <= 0 or H <= 0:
        raise ValueError("image must be non-empty")
    if vx is None or vy is None:
        if K is None or K < 1 or K > W * H:
            raise ValueError("K must lie in [1, W*H]")
        # floor(sqrt(W H / K)): for an integer v, v^2 <= WH/K iff v^2 <= WH // K
        vx = vy = math.isqrt((W * H) // K)
    if vx < 1 or vy < 1:
        raise ValueError("seed spacing must be >= 1")
    nx, ny = W // vx, H // vy
    if nx < 1 or ny < 1:
        raise ValueError("seed spacing larger than the image")
    return Grid(W, H, vx, vy, nx, ny)


def superpixel_coords(g: Grid, k):
    """Eq. kxy: k_x = k mod n_x, k_y = floor(k / n_x)."""
    return k % g.nx, k // g.nx


def window(g: Grid, k: int):
    """Eq. Ik: the half-open pixel rectangle [x_b, x_e) x [y_b, y_e) of I_k."""
    kx, ky = superpixel_coords(g, k)
    xb = max(0, g.vx * (kx - 1))
    xe = min(g.W, g.vx * (kx + 2))
    yb = max(0, g.vy * (ky - 1))
    ye = min(g.H, g.vy * (ky + 2))
    return xb, xe, yb, ye


def candidate_sets(g: Grid):
    """K_i = {k : i in I_k} by enumerating every window I_k.

    Returns ``cand`` (H, W, 9) int64 holding K_i in ascending k, padded with -1,
    and ``count`` (H, W) = |K_i|."""
    cand = np.full((g.H, g.W, MAXC), -1, dtype=np.int64)
    count = np.zeros((g.H, g.W), dtype=np.int64)
    for k in range(g.K):
        xb, xe, yb, ye = window(g, k)
        cw = cand[yb:ye, xb:xe]
        nw = count[yb:ye, xb:xe]
        if np.any(nw >= MAXC):
            raise AssertionError("a pixel lies in more than 9 windows")
        np.put_along_axis(cw, nw[..., None], k, axis=-1)
        nw += 1
    return cand, count


def window_positions(g: Grid, cand: np.ndarray):
    """For every k, the position of k inside K_i for each pixel i of I_k."""
    out = []
    for k in range(g.K):
        xb, xe, yb, ye = window(g, k)
        hit = cand[yb:ye, xb:xe] == k
        if not np.all(hit.any(axis=-1)):
            raise AssertionError("window pixel without k among its candidates")
        out.append(hit.argmax(axis=-1))
    return out


def features(lab) -> np.ndarray:
    """z_i = (x_i, y_i, c_i) in float64: (H, W, 5) for a CIELAB image (H, W, 3),
    (H, W, 3) for a grayscale image (H, W) or (H, W, 1)."""
    lab = np.asarray(lab, dtype=np.float32)
    if lab.ndim == 2:
        lab = lab[..., None]
    H, W, C = lab.shape
    z = np.empty((H, W, 2 + C), dtype=np.float64)
    z[..., 0] = np.arange(W, dtype=np.float64)[None, :]
    z[..., 1] = np.arange(H, dtype=np.float64)[:, None]
    z[..., 2:] = lab.astype(np.float64)
    return z


# ---------------------------------------------------------------------------
# Parameters (Sec. III-C)
# ---------------------------------------------------------------------------

@dataclass
class Params:
    eps_s: float = 2.0          # spatial eigenvalue floor (Sec. III-C)
    eps_c: float = 8.0          # colour eigenvalue floor (Sec. IV-A)
    lam: float = 8.0            # initial colour std (Sec. III-C, Sec. IV-A)
    cov_mode: int = 0           # 0: {xy, L, ab}; 1: {xy, Lab}; 2: full 5x5; 3: grayscale {xy, I}
    n_min: float = 1e-3         # mass guard


def blocks(cov_mode: int):
    """Component index sets of the diagonal blocks of Sigma_k."""
    if cov_mode == 0:
        return [(0, 1), (2,), (3, 4)]           # Eq. BlockSigma1
    if cov_mode == 1:
        return [(0, 1), (2, 3, 4)]              # Eq. BlockSigma
    if cov_mode == 2:
        return [(0, 1, 2, 3, 4)]                # Eq. UpdateSig, full
    if cov_mode == 3:
        return [(0, 1), (2,)]                   # grayscale, D = 3
    raise ValueError("cov_mode must be 0, 1, 2 or 3")


def block_eps(cov_mode: int, p: Params):
    return [p.eps_s] + [p.eps_c] * (len(blocks(cov_mode)) - 1)


def component_floors(cov_mode: int, p: Params) -> np.ndarray:
    """The floor of each component's scale: eps_s for x, y, eps_c for colour."""
    n = 3 if cov_mode == 3 else D
    return np.array([p.eps_s, p.eps_s] + [p.eps_c] * (n - 2))


@dataclass
class Theta:
    mu: np.ndarray              # (K, Dz), Dz = 5 (colour) or 3 (grayscale)
    sigma: np.ndarray           # (K, Dz, Dz), block diagonal or full
    mass: np.ndarray = field(default=None)   # (K,) N_k of the M-step that made it

    def copy(self) -> "Theta":
        return Theta(self.mu.copy(), self.sigma.copy(),
                     None if self.mass is None else self.mass.copy())


def seed_index(g: Grid, k):
    """Seed pixel of superpixel k (Sec. III-C)."""
    kx, ky = superpixel_coords(g, k)
    return kx * g.vx + g.vx // 2 + g.W * (ky * g.vy + g.vy // 2)


def init_theta(g: Grid, z: np.ndarray, p: Params) -> Theta:
    dz = z.shape[-1]
    zf = z.reshape(-1, dz)
    ks = np.arange(g.K)
    mu = zf[seed_index(g, ks)].copy()
    sigma = np.zeros((g.K, dz, dz))
    sigma[:, 0, 0] = g.vx ** 2
    sigma[:, 1, 1] = g.vy ** 2
    for c in range(2, dz):
        sigma[:, c, c] = p.lam ** 2
    return Theta(mu, sigma, np.zeros(g.K))


# ---------------------------------------------------------------------------
# E-step (Eqs. gaussian, Rik, ftheta)
# ---------------------------------------------------------------------------

def _block_inverses(theta: Theta, cov_mode: int):
    """Per superpixel and block: the inverse and ln det of Sigma_{k,b}."""
    out = []
    for idx in blocks(cov_mode):
        S = theta.sigma[:, idx][:, :, idx]
        sign, logdet = np.linalg.slogdet(S)
        if np.any(sign <= 0):
            raise FloatingPointError("non positive-definite covariance block")
        out.append((idx, np.linalg.inv(S), logdet))
    return out


def log_density_pairs(zs: np.ndarray, ks: np.ndarray, theta: Theta,
                      cov_mode: int = 0, inv=None) -> np.ndarray:
    """ln p(z; theta_k) (Eq. gaussian, D = zs.shape[1]) for rows zs (n, D) and
    superpixels ks (n,).  With Sigma block diagonal, ln det Sigma is the sum
    over blocks and the quadratic form splits into one form per block."""
    if inv is None:
        inv = _block_inverses(theta, cov_mode)
    d = zs - theta.mu[ks]
    out = np.full(zs.shape[0], -0.5 * zs.shape[1] * LN_2PI)
    for idx, P, logdet in inv:
        db = d[:, idx]
        q = np.einsum("ni,nij,nj->n", db, P[ks], db)
        out -= 0.5 * (logdet[ks] + q)
    return out


def estep(z: np.ndarray, cand: np.ndarray, theta: Theta, cov_mode: int = 0):
    """R_{i,k} = p(z_i; theta_k) / sum_{k' in K_i} p(z_i; theta_k') (Eq. Rik) and
    L(theta) = sum_i ln sum_{k in K_i} p(z_i; theta_k).

    Returns (R, logp, L) with R and logp shaped like ``cand`` (missing
    candidates: R = 0, logp = -inf)."""
    shp = cand.shape
    zf = z.reshape(-1, z.shape[-1])
    cf = cand.reshape(-1, MAXC)
    inv = _block_inverses(theta, cov_mode)
    logp = np.full(cf.shape, -np.inf)
    for j in range(MAXC):
        rows = np.nonzero(cf[:, j] >= 0)[0]
        if rows.size:
            logp[rows, j] = log_density_pairs(zf[rows], cf[rows, j], theta, cov_mode, inv)
    m = logp.max(axis=1)
    e = np.exp(logp - m[:, None])
    s = e.sum(axis=1)
    R = e / s[:, None]
    L = float(np.sum(m + np.log(s)))
    return R.reshape(shp), logp.reshape(shp), L


# ---------------------------------------------------------------------------
# M-step with shape control (Eqs. UpdateMu, UpdateSigS, UpdateSigC,
# eigdecs/eigdecc, mlams/mlamc, eigdecrs/eigdecrc)
# ---------------------------------------------------------------------------

def clamp_eigen(S: np.ndarray, eps: float) -> np.ndarray:
    """Q diag(max(lambda_j, eps)) Q^T for a symmetric block S."""
    if S.shape == (1, 1):
        return np.array([[max(S[0, 0], eps)]])
    w, Q = np.linalg.eigh(S)
    w = np.where(w >= eps, w, eps)
    return (Q * w[None, :]) @ Q.T


def clamp_eigen_scaled(S: np.ndarray, floors) -> np.ndarray:
    """Shape control of a full Sigma: with F = diag(floors), the eigenvalues of
    F^-1/2 S F^-1/2 are raised to at least 1 and the result scaled back."""
    f = np.sqrt(np.asarray(floors, dtype=np.float64))
    T = S / np.outer(f, f)
    w, Q = np.linalg.eigh(T)
    w = np.where(w >= 1.0, w, 1.0)
    return np.outer(f, f) * ((Q * w[None, :]) @ Q.T)


def mstep_one(zw: np.ndarray, rk: np.ndarray, mu_old: np.ndarray,
              sigma_old: np.ndarray, p: Params):
    """M-step for one superpixel from the pixels of its window I_k (rows zw)
    and their responsibilities rk.  Returns (mu, sigma, N_k)."""
    Nk = float(rk.sum())
    if not Nk >= p.n_min:
        return mu_old.copy(), sigma_old.copy(), Nk
    mu = (rk[:, None] * zw).sum(axis=0) / Nk                    # Eq. UpdateMu
    dz = zw.shape[1]
    sigma = np.zeros((dz, dz))
    for idx, eps in zip(blocks(p.cov_mode), block_eps(p.cov_mode, p)):
        db = zw[:, idx] - mu[list(idx)]
        Sb = (rk[:, None, None] * db[:, :, None] * db[:, None, :]).sum(axis=0) / Nk
        if p.cov_mode == 2:
            Sb = clamp_eigen_scaled(Sb, component_floors(2, p))
        else:
            Sb = clamp_eigen(Sb, eps)
        sigma[np.ix_(idx, idx)] = Sb
    return mu, sigma, Nk


def mstep(z: np.ndarray, g: Grid, R: np.ndarray, pos, theta: Theta, p: Params) -> Theta:
    """theta^{t+1} from R^t: every superpixel sums over its own window I_k."""
    new = Theta(np.empty_like(theta.mu), np.empty_like(theta.sigma), np.empty(g.K))
    for k in range(g.K):
        xb, xe, yb, ye = window(g, k)
        zw = z[yb:ye, xb:xe].reshape(-1, z.shape[-1])
        rk = np.take_along_axis(R[yb:ye, xb:xe], pos[k][..., None], axis=-1).reshape(-1)
        new.mu[k], new.sigma[k], new.mass[k] = mstep_one(zw, rk, theta.mu[k],
                                                         theta.sigma[k], p)
    return new


# ---------------------------------------------------------------------------
# Labels and the slot layout used to compare with the GPU export
# ---------------------------------------------------------------------------

def labels_from(R: np.ndarray, cand: np.ndarray) -> np.ndarray:
    """Eq. obtLi: the candidate with the largest posterior; np.argmax returns the
    first maximum and K_i is stored in ascending k, so ties go to the smallest k."""
    Rm = np.where(cand >= 0, R, -1.0)
    j = Rm.argmax(axis=-1)
    return np.take_along_axis(cand, j[..., None], axis=-1)[..., 0]


def to_slots(g: Grid, cand: np.ndarray, values: np.ndarray, fill=0.0) -> np.ndarray:
    """Re-index per-candidate values by neighbour slot s = 3 (dy + 1) + (dx + 1),
    dx = k_x - floor(x / v_x), dy = k_y - floor(y / v_y)."""
    H, W, _ = cand.shape
    out = np.full(cand.shape, fill, dtype=np.asarray(values).dtype)
    cx = (np.arange(W) // g.vx)[None, :, None]
    cy = (np.arange(H) // g.vy)[:, None, None]
    valid = cand >= 0
    kx, ky = cand % g.nx, cand // g.nx
    dx, dy = kx - cx, ky - cy
    if np.any(valid & ((np.abs(dx) > 1) | (np.abs(dy) > 1))):
        raise AssertionError("candidate outside the 3x3 neighbourhood")
    s = 3 * (dy + 1) + (dx + 1)
    yy, xx, jj = np.nonzero(valid)
    out[yy, xx, s[yy, xx, jj]] = values[yy, xx, jj]
    return out


# ---------------------------------------------------------------------------
# Algorithm 1 (steps 1-7)
# ---------------------------------------------------------------------------

def run_em(lab, g: Grid, p: Params | None = None, max_iters: int = 10,
           rel_tol: float = 0.0, theta0: Theta | None = None):
    """Returns a dict with theta (final), ll_hist (L(theta^t) of every E-step
    that was followed by an M-step or by the stop test), ll_final
    (L(theta_final)), iters (M-steps applied), R, logp, cand and labels."""
    p = p or Params()
    z = features(lab)
    cand, _ = candidate_sets(g)
    pos = window_positions(g, cand)
    theta = init_theta(g, z, p) if theta0 is None else theta0.copy()
    ll_hist = []
    iters = 0
    R, logp, L = estep(z, cand, theta, p.cov_mode)
    for t in range(max_iters):
        ll_hist.append(L)
        if rel_tol > 0 and t >= 1 and abs(L - ll_hist[-2]) <= rel_tol * abs(ll_hist[-2]):
            break
        theta = mstep(z, g, R, pos, theta, p)
        iters += 1
        R, logp, L = estep(z, cand, theta, p.cov_mode)
    return dict(theta=theta, ll_hist=ll_hist, ll_final=L, iters=iters, R=R,
                logp=logp, cand=cand, labels=labels_from(R, cand), z=z, pos=pos)


# ---------------------------------------------------------------------------
# Parameter export layout: mu_x mu_y mu_L mu_a mu_b S_xx S_xy S_yy S_LL S_aa S_ab S_bb N_k
# (cov_mode 0); with the 3x3 colour block (cov_mode 1):
# mu_x mu_y mu_L mu_a mu_b S_xx S_xy S_yy S_LL S_La S_Lb S_aa S_ab S_bb N_k
# ---------------------------------------------------------------------------

ROW3 = [(0, 0), (0, 1), (1, 1), (2, 2), (2, 3), (2, 4), (3, 3), (3, 4), (4, 4)]


def theta_to_rows3(theta: Theta) -> np.ndarray:
    K = theta.mu.shape[0]
    out = np.zeros((K, 15))
    out[:, 0:5] = theta.mu
    for c, (i, j) in enumerate(ROW3):
        out[:, 5 + c] = theta.sigma[:, i, j]
    out[:, 14] = 0.0 if theta.mass is None else theta.mass
    return out


def rows3_to_theta(rows: np.ndarray) -> Theta:
    rows = np.asarray(rows, dtype=np.float64)
    K = rows.shape[0]
    s = np.zeros((K, D, D))
    for c, (i, j) in enumerate(ROW3):
        s[:, i, j] = s[:, j, i] = rows[:, 5 + c]
    return Theta(rows[:, 0:5].copy(), s, rows[:, 14].copy())


def theta_to_rows(theta: Theta) -> np.ndarray:
    K = theta.mu.shape[0]
    out = np.zeros((K, 13))
    out[:, 0:5] = theta.mu
    s = theta.sigma
    out[:, 5] = s[:, 0, 0]
    out[:, 6] = s[:, 0, 1]
    out[:, 7] = s[:, 1, 1]
    out[:, 8] = s[:, 2, 2]
    out[:, 9] = s[:, 3, 3]
    out[:, 10] = s[:, 3, 4]
    out[:, 11] = s[:, 4, 4]
    out[:, 12] = 0.0 if theta.mass is None else theta.mass
    return out


# full Sigma (cov_mode 2): mu (5), the upper triangle of Sigma row by row
# (xx xy xL xa xb yy yL ya yb LL La Lb aa ab bb), N_k: 21 values;
# grayscale (cov_mode 3): mu_x mu_y mu_I S_xx S_xy S_yy S_II N_k: 8 values
ROW_FULL = [(i, j) for i in range(D) for j in range(i, D)]
ROW_GRAY = [(0, 0), (0, 1), (1, 1), (2, 2)]


def theta_to_rows_mode(theta: Theta, cov_mode: int) -> np.ndarray:
    """Export rows of any cov_mode (0 and 1 as theta_to_rows, theta_to_rows3)."""
    if cov_mode == 0:
        return theta_to_rows(theta)
    if cov_mode == 1:
        return theta_to_rows3(theta)
    layout = ROW_FULL if cov_mode == 2 else ROW_GRAY
    dz = theta.mu.shape[1]
    out = np.zeros((theta.mu.shape[0], dz + len(layout) + 1))
    out[:, :dz] = theta.mu
    for c, (i, j) in enumerate(layout):
        out[:, dz + c] = theta.sigma[:, i, j]
    out[:, -1] = 0.0 if theta.mass is None else theta.mass
    return out


def rows_mode_to_theta(rows: np.ndarray, cov_mode: int) -> Theta:
    if cov_mode == 0:
        return rows_to_theta(rows)
    if cov_mode == 1:
        return rows3_to_theta(rows)
    rows = np.asarray(rows, dtype=np.float64)
    layout = ROW_FULL if cov_mode == 2 else ROW_GRAY
    dz = D if cov_mode == 2 else 3
    s = np.zeros((rows.shape[0], dz, dz))
    for c, (i, j) in enumerate(layout):
        s[:, i, j] = s[:, j, i] = rows[:, dz + c]
    return Theta(rows[:, :dz].copy(), s, rows[:, -1].copy())


def rows_to_theta(rows: np.ndarray) -> Theta:
    rows = np.asarray(rows, dtype=np.float64)
    K = rows.shape[0]
    mu = rows[:, 0:5].copy()
    s = np.zeros((K, D, D))
    s[:, 0, 0] = rows[:, 5]
    s[:, 0, 1] = s[:, 1, 0] = rows[:, 6]
    s[:, 1, 1] = rows[:, 7]
    s[:, 2, 2] = rows[:, 8]
    s[:, 3, 3] = rows[:, 9]
    s[:, 3, 4] = s[:, 4, 3] = rows[:, 10]
    s[:, 4, 4] = rows[:, 11]
    return Theta(mu, s, rows[:, 12].copy())
