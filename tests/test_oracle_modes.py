"""Pins of the oracle's full-covariance (cov_mode 2) and grayscale (cov_mode 3)
modes against what the paper and the mathematics fix:

* the log-density is scipy's multivariate normal (Eq. gaussian, D = 5 full Sigma;
  D = 3 for a grayscale image, Sec. III-A);
* the scaled floor of the full Sigma is the paper's per-block rule (Eqs. mlams,
  mlamc) whenever Sigma is block diagonal, and the constrained maximum of the
  Gaussian likelihood under Sigma >= F in general (checked against random
  feasible covariances);
* the M-step with one-hot responsibilities is numpy's mean and biased covariance
  (Eqs. UpdateMu, UpdateSig);
* EM never lowers L(theta) (Eq. ftheta), since every M-step is the constrained
  maximiser;
* a grayscale image runs exactly like a colour image whose a, b channels are
  constant (cov_mode 0), up to the constant the (a, b) block adds to L."""
import numpy as np
import pytest
from scipy.stats import multivariate_normal

import synth
from oracle import gmm_oracle as O


def random_spd(rng, n, scale):
    A = rng.normal(size=(n, n))
    return A @ A.T * scale + np.eye(n) * 0.5 * scale


def test_full_log_density_is_scipy():
    rng = np.random.default_rng(1)
    K = 4
    mu = rng.normal(size=(K, 5)) * [30, 30, 20, 20, 20]
    sig = np.stack([random_spd(rng, 5, s) for s in (4.0, 9.0, 16.0, 30.0)])
    th = O.Theta(mu, sig)
    zs = mu[rng.integers(0, K, 50)] + rng.normal(size=(50, 5)) * 5
    ks = rng.integers(0, K, 50)
    got = O.log_density_pairs(zs, ks, th, cov_mode=2)
    want = [multivariate_normal(mu[k], sig[k]).logpdf(z) for z, k in zip(zs, ks)]
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-10)


def test_gray_log_density_is_scipy():
    rng = np.random.default_rng(2)
    K = 3
    mu = rng.normal(size=(K, 3)) * [30, 30, 40]
    sig = np.zeros((K, 3, 3))
    for k in range(K):
        sig[k, :2, :2] = random_spd(rng, 2, 20.0)
        sig[k, 2, 2] = rng.uniform(5, 100)
    th = O.Theta(mu, sig)
    zs = mu[rng.integers(0, K, 40)] + rng.normal(size=(40, 3)) * 4
    ks = rng.integers(0, K, 40)
    got = O.log_density_pairs(zs, ks, th, cov_mode=3)
    want = [multivariate_normal(mu[k], sig[k]).logpdf(z) for z, k in zip(zs, ks)]
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-10)


def test_scaled_floor_is_the_block_rule_on_block_diagonal_sigma():
    rng = np.random.default_rng(3)
    p = O.Params()
    floors = O.component_floors(2, p)
    for _ in range(20):
        S = np.zeros((5, 5))
        # small eigenvalues on purpose: both blocks get floored
        S[:2, :2] = random_spd(rng, 2, rng.uniform(0.1, 3.0))
        S[2:, 2:] = random_spd(rng, 3, rng.uniform(0.5, 12.0))
        got = O.clamp_eigen_scaled(S, floors)
        want = np.zeros((5, 5))
        want[:2, :2] = O.clamp_eigen(S[:2, :2], p.eps_s)
        want[2:, 2:] = O.clamp_eigen(S[2:, 2:], p.eps_c)
        np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-10)


def test_scaled_floor_properties():
    rng = np.random.default_rng(4)
    p = O.Params()
    f = O.component_floors(2, p)
    Fh = np.diag(1.0 / np.sqrt(f))
    # zero -> F itself
    np.testing.assert_allclose(O.clamp_eigen_scaled(np.zeros((5, 5)), f), np.diag(f), atol=1e-12)
    for _ in range(20):
        S = random_spd(rng, 5, rng.uniform(0.2, 10.0))
        out = O.clamp_eigen_scaled(S, f)
        np.testing.assert_allclose(out, out.T, atol=1e-12)
        assert np.linalg.eigvalsh(Fh @ out @ Fh).min() >= 1.0 - 1e-10
        # already feasible (S >= F): unchanged
        big = S + np.diag(f) * 1.5
        if np.linalg.eigvalsh(Fh @ big @ Fh).min() >= 1.0:
            np.testing.assert_allclose(O.clamp_eigen_scaled(big, f), big, rtol=1e-10, atol=1e-10)


def test_scaled_floor_maximises_the_constrained_likelihood():
    """Among covariances with Sigma >= F, the scaled floor of the sample
    covariance S maximises -ln det Sigma - tr(Sigma^-1 S): no random feasible
    candidate, nor any small feasible perturbation, does better."""
    rng = np.random.default_rng(5)
    p = O.Params()
    f = O.component_floors(2, p)
    F = np.diag(f)

    def obj(Sig, S):
        return -np.linalg.slogdet(Sig)[1] - np.trace(np.linalg.solve(Sig, S))

    for _ in range(10):
        S = random_spd(rng, 5, rng.uniform(0.3, 4.0))
        best = O.clamp_eigen_scaled(S, f)
        b = obj(best, S)
        for _ in range(200):
            R = rng.normal(size=(5, 5)) * rng.uniform(0.01, 3.0)
            cand = F + R @ R.T
            assert obj(cand, S) <= b + 1e-9
            R2 = rng.normal(size=(5, 5)) * 1e-3
            near = best + R2 @ R2.T          # still >= F
            assert obj(near, S) <= b + 1e-12


def _one_hot_case(cov_mode, rng):
    lab = synth.voronoi_lab(40, 30, 6, 3.0, 7, 1).lab.numpy()
    if cov_mode == 3:
        lab = lab[..., 0]
    z = O.features(lab)
    zw = z.reshape(-1, z.shape[-1])
    rk = np.zeros(zw.shape[0])
    sel = rng.choice(zw.shape[0], 300, replace=False)
    rk[sel] = 1.0
    return zw, rk, sel


@pytest.mark.parametrize("cov_mode", [2, 3])
def test_one_hot_mstep_is_mean_and_biased_covariance(cov_mode):
    rng = np.random.default_rng(6)
    zw, rk, sel = _one_hot_case(cov_mode, rng)
    dz = zw.shape[1]
    p = O.Params(cov_mode=cov_mode)
    mu, sig, N = O.mstep_one(zw, rk, np.zeros(dz), np.eye(dz), p)
    assert N == 300
    np.testing.assert_allclose(mu, zw[sel].mean(axis=0), rtol=1e-12)
    C = np.cov(zw[sel].T, bias=True)
    if cov_mode == 3:      # block diagonal: the cross terms are not part of the model
        C[:2, 2] = C[2, :2] = 0.0
    # the 300 scattered pixels spread far beyond the floors: nothing is clamped
    np.testing.assert_allclose(sig, C, rtol=1e-10, atol=1e-9)


@pytest.mark.parametrize("cov_mode", [2, 3])
def test_em_never_lowers_the_log_likelihood(cov_mode):
    im = synth.voronoi_lab(57, 44, 7, 3.0, 11, 1)
    lab = im.lab.numpy() if cov_mode == 2 else im.lab.numpy()[..., 0]
    g = O.make_grid(57, 44, vx=9, vy=9)
    res = O.run_em(lab, g, O.Params(cov_mode=cov_mode), max_iters=8)
    L = np.array(res["ll_hist"] + [res["ll_final"]])
    assert np.all(np.diff(L) >= -1e-12 * np.abs(L[:-1]))
    assert L[-1] > L[0]


def test_gray_equals_colour_with_constant_ab():
    """cov_mode 3 on I against cov_mode 0 on (I, 12, -7): the (a, b) block is the
    same for every superpixel (lambda^2 I at theta^0, eps_c I after an M-step),
    so R, labels, means and the other blocks agree, and L differs by N (ln 2 pi
    + 1/2 ln det Sigma_ab)."""
    im = synth.voronoi_lab(50, 38, 6, 3.0, 12, 1)
    I = im.lab.numpy()[..., 0]
    lab = np.stack([I, np.full_like(I, 12.0), np.full_like(I, -7.0)], axis=-1)
    g = O.make_grid(50, 38, vx=8, vy=8)
    p0, p3 = O.Params(cov_mode=0), O.Params(cov_mode=3)
    r0 = O.run_em(lab, g, p0, max_iters=5)
    r3 = O.run_em(I, g, p3, max_iters=5)
    np.testing.assert_allclose(r3["R"], r0["R"], atol=1e-12)
    assert np.array_equal(r3["labels"], r0["labels"])
    np.testing.assert_allclose(r3["theta"].mu, r0["theta"].mu[:, :3], rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(r3["theta"].sigma, r0["theta"].sigma[:, :3, :3], rtol=1e-12,
                               atol=1e-9)
    N = I.size
    for t, (l0, l3) in enumerate(zip(r0["ll_hist"], r3["ll_hist"])):
        var_ab = p0.lam ** 2 if t == 0 else p0.eps_c
        assert l3 == pytest.approx(l0 + N * (O.LN_2PI + np.log(var_ab)), rel=1e-12)


@pytest.mark.parametrize("cov_mode,width", [(2, 21), (3, 8)])
def test_row_layout_round_trip(cov_mode, width):
    rng = np.random.default_rng(8)
    dz = 5 if cov_mode == 2 else 3
    K = 6
    sig = np.stack([random_spd(rng, dz, 5.0) for _ in range(K)])
    if cov_mode == 3:
        sig[:, :2, 2] = sig[:, 2, :2] = 0.0
    th = O.Theta(rng.normal(size=(K, dz)), sig, rng.uniform(1, 9, K))
    rows = O.theta_to_rows_mode(th, cov_mode)
    assert rows.shape == (K, width)
    back = O.rows_mode_to_theta(rows, cov_mode)
    np.testing.assert_array_equal(back.mu, th.mu)
    np.testing.assert_allclose(back.sigma, th.sigma, rtol=0, atol=1e-15)
    np.testing.assert_array_equal(back.mass, th.mass)
