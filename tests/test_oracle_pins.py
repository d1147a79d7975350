"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics:
hand-derived grid integers, closed forms, library routines (scipy, numpy),
invariants stated in the paper and special cases with a textbook answer.
None of these re-types the oracle's own formula."""
import math

import numpy as np
import pytest
from scipy.special import logsumexp
from scipy.stats import multivariate_normal

import synth
from oracle import gmm_oracle as O


# ---------------------------------------------------------------------------
# Grid (Eqs. vxy, nxyK) and candidate sets (Eq. Ik, Eq. kxy, Sec. III-D bounds)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("W,H,K,v,nx,ny", [
    # 481*321 = 154401, //400 = 386, 19^2 = 361 <= 386 < 400 = 20^2
    (481, 321, 400, 19, 25, 16),
    # 1920*1080 = 2073600, //2000 = 1036, 32^2 = 1024 <= 1036 < 1089
    (1920, 1080, 2000, 32, 60, 33),
    # 3840*2160 = 8294400, //10000 = 829, 28^2 = 784 <= 829 < 841
    (3840, 2160, 10000, 28, 137, 77),
    # 640*480 = 307200, K = 307200 // 600 = 512 -> 600 -> 24
    (640, 480, 512, 24, 26, 20),
])
def test_grid_hand_values(W, H, K, v, nx, ny):
    g = O.make_grid(W, H, K=K)
    assert (g.vx, g.vy, g.nx, g.ny, g.K) == (v, v, nx, ny, nx * ny)


def test_grid_floor_sqrt_brute_force():
    rng = np.random.default_rng(7)
    for _ in range(2000):
        W = int(rng.integers(1, 5000))
        H = int(rng.integers(1, 3000))
        K = int(rng.integers(1, W * H + 1))
        # largest v with v^2 K <= W H, i.e. floor(sqrt(WH/K)) by definition
        v = 1
        while (v + 1) * (v + 1) * K <= W * H:
            v += 1
        if v < 10 ** 6:
            try:
                g = O.make_grid(W, H, K=K)
            except ValueError:
                assert W // v < 1 or H // v < 1
                continue
            assert g.vx == v == g.vy


def test_grid_rejects_bad_input():
    for args in [(0, 5, 1), (5, 0, 1), (5, 5, 0), (5, 5, 26)]:
        with pytest.raises(ValueError):
            O.make_grid(*args[:2], K=args[2])
    with pytest.raises(ValueError):
        O.make_grid(10, 10, vx=11, vy=2)


GRIDS = [
    dict(W=57, H=38, vx=19, vy=19),      # divisible, 3 x 2
    dict(W=62, H=45, vx=10, vy=10),      # remainders (2, 5)
    dict(W=60, H=41, vx=12, vy=7),       # anisotropic with remainders
    dict(W=25, H=31, vx=9, vy=9),        # n = 2 x 3 with remainders
    dict(W=13, H=17, vx=13, vy=17),      # one superpixel
    dict(W=100, H=9, vx=9, vy=9),        # one row of superpixels
]


@pytest.mark.parametrize("gd", GRIDS)
def test_candidates_closed_form(gd):
    g = O.make_grid(gd["W"], gd["H"], vx=gd["vx"], vy=gd["vy"])
    cand, count = O.candidate_sets(g)
    # closed form: pixel (x, y) in I_k iff floor(x/v_x) in {k_x-1, k_x, k_x+1}
    # and the same in y, since x_b <= x < x_e with x_b = v(k_x-1), x_e = v(k_x+2)
    for y in range(g.H):
        for x in range(g.W):
            cx, cy = x // g.vx, y // g.vy
            kxs = [k for k in (cx - 1, cx, cx + 1) if 0 <= k < g.nx]
            kys = [k for k in (cy - 1, cy, cy + 1) if 0 <= k < g.ny]
            expect = sorted(ky * g.nx + kx for ky in kys for kx in kxs)
            got = [int(k) for k in cand[y, x] if k >= 0]
            assert got == expect, (x, y)
    assert count.min() >= 1 and count.max() <= 9           # Sec. III-D
    sizes = [(xe - xb) * (ye - yb) for xb, xe, yb, ye in
             (O.window(g, k) for k in range(g.K))]
    vv = g.vx * g.vy
    if g.nx >= 2 and g.ny >= 2:
        assert min(sizes) >= vv and max(sizes) <= 9 * vv    # Sec. III-D
    # double counting: sum_i |K_i| = sum_k |I_k|
    assert int(count.sum()) == sum(sizes)
    if g.nx >= 2 and g.ny >= 2:
        rx, ry = g.W - g.nx * g.vx, g.H - g.ny * g.vy
        wx = g.vx * (3 * g.nx - 2) + rx
        wy = g.vy * (3 * g.ny - 2) + ry
        assert int(count.sum()) == wx * wy


@pytest.mark.parametrize("W,H,K,pairs", [
    (481, 321, 400, 1241163),
    (1920, 1080, 2000, 17817088),
])
def test_pair_counts_of_configs(W, H, K, pairs):
    # (v(3n_x-2)+r_x)(v(3n_y-2)+r_y), evaluated by hand for the two workloads:
    # 481x321: (19*73+6)(19*46+17) = 1393*891; 1920x1080: (32*178+0)(32*97+24) = 5696*3128
    g = O.make_grid(W, H, K=K)
    _, count = O.candidate_sets(g)
    assert int(count.sum()) == pairs


# ---------------------------------------------------------------------------
# E-step: Eq. gaussian against scipy, Eq. Rik invariants, L(theta) brute force
# ---------------------------------------------------------------------------

def _random_spd(rng, n, scale):
    A = rng.normal(size=(n, n))
    return scale * (A @ A.T / n + 0.3 * np.eye(n))


def _random_theta(rng, K, cov_mode, W=60, H=40):
    mu = np.column_stack([rng.uniform(0, W, K), rng.uniform(0, H, K),
                          rng.uniform(10, 90, K), rng.uniform(-60, 60, K),
                          rng.uniform(-60, 60, K)])
    sigma = np.zeros((K, 5, 5))
    for k in range(K):
        for idx in O.blocks(cov_mode):
            sigma[k][np.ix_(idx, idx)] = _random_spd(rng, len(idx),
                                                     40.0 if idx[0] == 0 else 25.0)
    return O.Theta(mu, sigma, np.zeros(K))


@pytest.mark.parametrize("cov_mode", [0, 1])
def test_log_density_matches_scipy(cov_mode):
    rng = np.random.default_rng(3)
    th = _random_theta(rng, 7, cov_mode)
    zs = np.column_stack([rng.uniform(0, 60, 300), rng.uniform(0, 40, 300),
                          rng.uniform(0, 100, 300), rng.uniform(-70, 70, 300),
                          rng.uniform(-70, 70, 300)])
    ks = rng.integers(0, 7, 300)
    got = O.log_density_pairs(zs, ks, th, cov_mode)
    want = np.array([multivariate_normal(th.mu[k], th.sigma[k]).logpdf(z)
                     for z, k in zip(zs, ks)])
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-10)


def test_estep_invariants_and_likelihood_brute_force():
    rng = np.random.default_rng(5)
    g = O.make_grid(31, 23, vx=7, vy=6)
    lab = np.stack([rng.uniform(0, 100, (23, 31)), rng.uniform(-50, 50, (23, 31)),
                    rng.uniform(-50, 50, (23, 31))], -1).astype(np.float32)
    z = O.features(lab)
    cand, count = O.candidate_sets(g)
    th = _random_theta(rng, g.K, 0, 31, 23)
    R, logp, L = O.estep(z, cand, th)
    assert np.all(R >= 0)
    np.testing.assert_allclose(R.sum(-1), 1.0, atol=1e-14)
    assert np.all(R[cand < 0] == 0)
    # L(theta) = sum_i ln sum_{k in K_i} p(z_i; theta_k), every log density from
    # scipy and the sum of densities by scipy's logsumexp
    dens = [multivariate_normal(th.mu[k], th.sigma[k]) for k in range(g.K)]
    tot = 0.0
    for y in range(g.H):
        for x in range(g.W):
            ks = [k for k in cand[y, x] if k >= 0]
            lp = np.array([dens[k].logpdf(z[y, x]) for k in ks])
            lse = logsumexp(lp)
            tot += lse
            np.testing.assert_allclose(R[y, x, :len(ks)], np.exp(lp - lse),
                                       rtol=1e-10, atol=1e-300)
    assert L == pytest.approx(tot, rel=1e-12)


def test_estep_far_outlier_is_finite():
    # a pixel hundreds of standard deviations from every candidate: the direct
    # ratio of Eq. Rik underflows to 0/0, the log-domain form stays exact
    g = O.make_grid(20, 20, vx=10, vy=10)
    lab = np.zeros((20, 20, 3), np.float32)
    lab[5, 5] = (1e4, 0, 0)
    z = O.features(lab)
    cand, _ = O.candidate_sets(g)
    th = O.init_theta(g, z, O.Params())
    R, _, L = O.estep(z, cand, th)
    assert np.isfinite(R).all() and np.isfinite(L)
    np.testing.assert_allclose(R.sum(-1), 1.0, atol=1e-14)


# ---------------------------------------------------------------------------
# M-step (Eqs. UpdateMu, UpdateSigS, UpdateSigC) against numpy statistics
# ---------------------------------------------------------------------------

def _window_pixels(rng, n):
    return np.column_stack([rng.integers(0, 50, n), rng.integers(0, 50, n),
                            rng.uniform(0, 100, n), rng.uniform(-60, 60, n),
                            rng.uniform(-60, 60, n)]).astype(np.float64)


@pytest.mark.parametrize("cov_mode", [0, 1])
def test_mstep_one_hot_is_sample_mean_and_covariance(cov_mode):
    rng = np.random.default_rng(11)
    zw = _window_pixels(rng, 400)
    rk = (rng.uniform(size=400) < 0.4).astype(np.float64)     # a fixed assignment
    p = O.Params(eps_s=1e-9, eps_c=1e-9, cov_mode=cov_mode)
    mu, sigma, Nk = O.mstep_one(zw, rk, np.zeros(5), np.eye(5), p)
    sel = zw[rk == 1]
    assert Nk == sel.shape[0]
    np.testing.assert_allclose(mu, sel.mean(axis=0), rtol=1e-13)
    full = np.cov(sel.T, bias=True)
    for idx in O.blocks(cov_mode):
        np.testing.assert_allclose(sigma[np.ix_(idx, idx)], full[np.ix_(idx, idx)],
                                   rtol=1e-11, atol=1e-9)
    # off-block entries are structurally zero (Eq. BlockSigma)
    mask = np.ones((5, 5), bool)
    for idx in O.blocks(cov_mode):
        mask[np.ix_(idx, idx)] = False
    assert np.all(sigma[mask] == 0)


def test_mstep_weighted_matches_numpy_average_and_cov():
    rng = np.random.default_rng(12)
    zw = _window_pixels(rng, 500)
    rk = rng.uniform(size=500)
    p = O.Params(eps_s=1e-9, eps_c=1e-9)
    mu, sigma, Nk = O.mstep_one(zw, rk, np.zeros(5), np.eye(5), p)
    assert Nk == pytest.approx(rk.sum(), rel=1e-14)
    np.testing.assert_allclose(mu, np.average(zw, axis=0, weights=rk), rtol=1e-13)
    full = np.cov(zw.T, aweights=rk, bias=True)
    for idx in O.blocks(0):
        np.testing.assert_allclose(sigma[np.ix_(idx, idx)], full[np.ix_(idx, idx)],
                                   rtol=1e-10, atol=1e-9)


def test_mstep_zero_mass_keeps_parameters():
    rng = np.random.default_rng(13)
    zw = _window_pixels(rng, 50)
    mu0 = np.arange(5.0)
    s0 = np.diag([4.0, 5.0, 64.0, 64.0, 64.0])
    mu, sigma, Nk = O.mstep_one(zw, np.zeros(50), mu0, s0, O.Params())
    assert Nk == 0.0
    assert np.array_equal(mu, mu0) and np.array_equal(sigma, s0)


# ---------------------------------------------------------------------------
# Shape control (Eqs. eigdecs..eigdecrc)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3])
def test_clamp_eigen(n):
    rng = np.random.default_rng(20 + n)
    for _ in range(200):
        A = rng.normal(size=(n, n)) * rng.uniform(0.1, 10)
        S = A @ A.T
        eps = float(rng.uniform(0.5, 20))
        C = O.clamp_eigen(S, eps)
        assert np.allclose(C, C.T, atol=1e-12)
        np.testing.assert_allclose(np.linalg.eigvalsh(C),
                                   np.maximum(np.linalg.eigvalsh(S), eps),
                                   rtol=1e-10, atol=1e-10)
        if np.linalg.eigvalsh(S).min() >= eps:
            np.testing.assert_allclose(C, S, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(O.clamp_eigen(np.zeros((n, n)), 3.0), 3.0 * np.eye(n))


# ---------------------------------------------------------------------------
# Whole EM: ascent of L(theta), separated blocks, K = 1, 2x2 grid, ties
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("cov_mode", [0, 1])
def test_em_log_likelihood_never_decreases(cov_mode):
    im = synth.voronoi_lab(97, 71, 9, 3.0, 4, 30)
    g = O.make_grid(97, 71, K=30)
    res = O.run_em(im.lab.numpy(), g, O.Params(cov_mode=cov_mode), max_iters=8)
    lls = res["ll_hist"] + [res["ll_final"]]
    for a, b in zip(lls, lls[1:]):
        assert b >= a - 1e-12 * abs(a)


@pytest.mark.parametrize("v,nbx,nby", [(6, 5, 4), (8, 4, 4), (11, 3, 5)])
def test_separated_blocks_are_recovered(v, nbx, nby):
    im = synth.separated_blocks(v, nbx, nby)
    g = O.make_grid(im.W, im.H, vx=v, vy=v)
    res = O.run_em(im.lab.numpy(), g, max_iters=3)
    # labels = block ids exactly
    assert np.array_equal(res["labels"], im.regions.numpy())
    th = res["theta"]
    var = (v * v - 1) / 12.0         # variance of the uniform law on {0..v-1}
    for k in range(g.K):
        kx, ky = k % nbx, k // nbx
        col = synth.BLOCK_PALETTE[(kx % 3) + 3 * (ky % 3)]
        want_mu = [kx * v + (v - 1) / 2, ky * v + (v - 1) / 2, *col]
        np.testing.assert_allclose(th.mu[k], want_mu, rtol=0, atol=1e-9)
        np.testing.assert_allclose(th.sigma[k][:2, :2], np.diag([var, var]), atol=1e-9)
        # constant colour: zero sample variance, clamped to eps_c (Eq. mlamc)
        np.testing.assert_allclose(th.sigma[k][2:, 2:], 8.0 * np.eye(3), atol=1e-9)
        assert th.mass[k] == pytest.approx(v * v, rel=1e-9)


def test_single_superpixel_is_one_gaussian():
    rng = np.random.default_rng(30)
    v = 9
    lab = np.stack([rng.uniform(20, 80, (v, v)), rng.normal(0, 20, (v, v)),
                    rng.normal(0, 15, (v, v))], -1).astype(np.float32)
    g = O.make_grid(v, v, K=1)
    assert g.K == 1
    res = O.run_em(lab, g, max_iters=3)
    assert np.all(res["R"][..., 0] == 1.0)
    z = O.features(lab).reshape(-1, 5)
    mu = z.mean(axis=0)
    S = np.cov(z.T, bias=True)
    want = np.zeros((5, 5))
    want[:2, :2] = O.clamp_eigen(S[:2, :2], 2.0)
    want[2, 2] = max(S[2, 2], 8.0)
    want[3:, 3:] = O.clamp_eigen(S[3:, 3:], 8.0)
    th = res["theta"]
    np.testing.assert_allclose(th.mu[0], mu, rtol=1e-12)
    np.testing.assert_allclose(th.sigma[0], want, rtol=1e-10, atol=1e-10)
    ll = multivariate_normal(mu, want).logpdf(z).sum()
    assert res["ll_final"] == pytest.approx(ll, rel=1e-12)
    # fixed point from t = 1: every later L(theta^t) is the same
    assert res["ll_hist"][1] == pytest.approx(res["ll_final"], rel=1e-13)


def test_two_by_two_grid_is_textbook_equal_weight_gmm():
    rng = np.random.default_rng(31)
    v = 7
    lab = np.stack([rng.uniform(20, 80, (2 * v, 2 * v)),
                    rng.normal(0, 20, (2 * v, 2 * v)),
                    rng.normal(0, 15, (2 * v, 2 * v))], -1).astype(np.float32)
    g = O.make_grid(2 * v, 2 * v, vx=v, vy=v)
    cand, count = O.candidate_sets(g)
    assert np.all(count == 4)
    z = O.features(lab)
    th = _random_theta(rng, 4, 0, 2 * v, 2 * v)
    R, _, L = O.estep(z, cand, th)
    comps = [multivariate_normal(th.mu[k], th.sigma[k]) for k in range(4)]
    zf = z.reshape(-1, 5)
    P = np.stack([0.25 * c.pdf(zf) for c in comps], 1)      # weights 1/4
    post = P / P.sum(1, keepdims=True)
    np.testing.assert_allclose(R.reshape(-1, 9)[:, :4], post, rtol=1e-10)
    # f(theta) = L(theta) + sum_i ln P_i with P_i = 1/4 (Eq. ftheta)
    f = np.log(P.sum(1)).sum()
    assert L + zf.shape[0] * math.log(0.25) == pytest.approx(f, rel=1e-12)


def test_label_ties_go_to_lowest_k():
    g = O.make_grid(20, 20, vx=10, vy=10)
    lab = np.full((20, 20, 3), 50.0, np.float32)
    z = O.features(lab)
    cand, _ = O.candidate_sets(g)
    th = O.init_theta(g, z, O.Params())
    th.mu[:] = th.mu[0]                       # four identical Gaussians
    R, _, _ = O.estep(z, cand, th)
    assert np.all(O.labels_from(R, cand) == 0)


def test_relative_tolerance_stop_rule():
    im = synth.voronoi_lab(120, 90, 12, 3.0, 9, 40)
    g = O.make_grid(120, 90, K=40)
    tol = 1e-3
    res = O.run_em(im.lab.numpy(), g, max_iters=50, rel_tol=tol)
    h = res["ll_hist"]
    assert res["iters"] == len(h) - 1 < 50
    assert abs(h[-1] - h[-2]) <= tol * abs(h[-2])
    for t in range(1, len(h) - 1):
        assert abs(h[t] - h[t - 1]) > tol * abs(h[t - 1])


def test_slot_layout_round_trip():
    g = O.make_grid(62, 45, vx=10, vy=10)
    cand, count = O.candidate_sets(g)
    s = O.to_slots(g, cand, cand, fill=-1)
    assert np.array_equal(np.sort(s, -1), np.sort(cand, -1))
    # slot 4 (dx = dy = 0) holds the pixel's own cell when that cell is a superpixel
    ys, xs = np.mgrid[0:45, 0:62]
    own = (xs // 10 < g.nx) & (ys // 10 < g.ny)
    assert np.array_equal(s[..., 4][own], ((ys // 10) * g.nx + xs // 10)[own])


def test_init_seed_pixels_hand_values():
    # Sec. III-C seeds for the 481x321 grid (v = 19): superpixel 0 at pixel
    # (9, 9); superpixel 26 = (k_x 1, k_y 1) at (28, 28); the last one,
    # 399 = (24, 15), at (465, 294).  Spatial covariance diag(361, 361),
    # colour variances lambda^2 = 64.
    im = synth.config1_image()
    g = O.make_grid(481, 321, K=400)
    z = O.features(im.lab.numpy())
    th = O.init_theta(g, z, O.Params())
    for k, (x, y) in [(0, (9, 9)), (26, (28, 28)), (399, (465, 294))]:
        np.testing.assert_array_equal(th.mu[k], z[y, x])
    np.testing.assert_array_equal(th.sigma[5], np.diag([361.0, 361.0, 64.0, 64.0, 64.0]))


def test_row_layout_of_the_3x3_colour_block():
    im = synth.voronoi_lab(60, 45, 6, 3.0, 9, 12)
    g = O.make_grid(60, 45, K=12)
    res = O.run_em(im.lab.numpy(), g, O.Params(cov_mode=1), max_iters=3)
    th = res["theta"]
    rows = O.theta_to_rows3(th)
    back = O.rows3_to_theta(rows)
    np.testing.assert_array_equal(back.mu, th.mu)
    # the rows hold the upper triangle; the clamped blocks are symmetric to rounding
    np.testing.assert_allclose(back.sigma, th.sigma, rtol=1e-13, atol=1e-12)
    # the colour block is a full 3x3 after the M-step (L-a, L-b correlations kept)
    assert np.any(rows[:, 9] != 0) and np.any(rows[:, 10] != 0)
    assert np.all(th.sigma[:, :2, 2:] == 0)
