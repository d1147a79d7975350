"""Planted mistakes in the FP64 oracle, each of which one of its pins must catch.

Every case below replaces one oracle function (on the CPU, for the duration of the
test) with a plausible wrong version: a dropped term, a wrong sign, an index off by
one, the wrong tie-break, the wrong reference point of a moment.  It then runs the
pins of ``test_oracle_pins`` that cover that part of the method, over all their
parameter sets, and requires at least one of them to fail.  This is the evidence
that the pins constrain the oracle rather than restate it.
"""
import math

import numpy as np
import pytest

import test_oracle_modes as MODES
import test_oracle_pins as PINS
from oracle import gmm_oracle as O

_orig = {name: getattr(O, name) for name in (
    "log_density_pairs", "estep", "clamp_eigen", "mstep_one", "make_grid", "window",
    "labels_from", "init_theta", "seed_index", "block_eps", "clamp_eigen_scaled",
    "component_floors")}


_PARAM_SET = type(pytest.param(0))


def _cases(fn):
    """Keyword sets of every parametrisation of a pin (cartesian over its marks)."""
    combos = [{}]
    for m in getattr(fn, "pytestmark", []):
        if m.name != "parametrize":
            continue
        names = m.args[0]
        names = [n.strip() for n in names.split(",")] if isinstance(names, str) else list(names)
        new = []
        for c in combos:
            for v in m.args[1]:
                v = v.values if isinstance(v, _PARAM_SET) else v
                v = tuple(v) if len(names) > 1 else (v,)
                new.append({**c, **dict(zip(names, v))})
        combos = new
    return combos


def _pin_fails(fn) -> bool:
    for kw in _cases(fn):
        try:
            fn(**kw)
        except Exception:  # an assertion, or the mutant breaking a precondition
            return True
    return False


# ---------------------------------------------------------------------------
# the mutants
# ---------------------------------------------------------------------------

def _logdet_dropped(zs, ks, theta, cov_mode=0, inv=None):
    inv = O._block_inverses(theta, cov_mode) if inv is None else inv
    return _orig["log_density_pairs"](zs, ks, theta, cov_mode,
                                      [(i, P, 0.0 * ld) for i, P, ld in inv])


def _quadratic_sign(zs, ks, theta, cov_mode=0, inv=None):
    inv = O._block_inverses(theta, cov_mode) if inv is None else inv
    d = zs - theta.mu[ks]
    out = np.full(zs.shape[0], -0.5 * zs.shape[1] * O.LN_2PI)
    for idx, P, logdet in inv:
        db = d[:, idx]
        out -= 0.5 * (logdet[ks] - np.einsum("ni,nij,nj->n", db, P[ks], db))
    return out


def _two_pi_dropped(zs, ks, theta, cov_mode=0, inv=None):
    return _orig["log_density_pairs"](zs, ks, theta, cov_mode, inv) + 0.5 * zs.shape[1] * O.LN_2PI


def _normalised_by_max(z, cand, theta, cov_mode=0):
    R, logp, L = _orig["estep"](z, cand, theta, cov_mode)
    return R / R.max(axis=-1, keepdims=True), logp, L


def _likelihood_without_shift(z, cand, theta, cov_mode=0):
    R, logp, L = _orig["estep"](z, cand, theta, cov_mode)
    return R, logp, L - float(logp.reshape(-1, logp.shape[-1]).max(axis=1).sum())


def _clamp_diagonal(S, eps):
    C = S.copy()
    i = np.arange(S.shape[0])
    C[i, i] = np.maximum(C[i, i], eps)
    return C


def _clamp_std(S, eps):
    return _orig["clamp_eigen"](S, math.sqrt(eps))


def _unbiased_covariance(zw, rk, mu_old, sigma_old, p):
    mu, sigma, Nk = _orig["mstep_one"](zw, rk, mu_old, sigma_old, p)
    return mu, (sigma * Nk / (Nk - 1.0) if Nk > 1.0 else sigma), Nk


def _covariance_about_old_mean(zw, rk, mu_old, sigma_old, p):
    Nk = float(rk.sum())
    if not Nk >= p.n_min:
        return mu_old.copy(), sigma_old.copy(), Nk
    mu = (rk[:, None] * zw).sum(axis=0) / Nk
    sigma = np.zeros((zw.shape[1], zw.shape[1]))
    for idx, eps in zip(O.blocks(p.cov_mode), O.block_eps(p.cov_mode, p)):
        db = zw[:, idx] - mu_old[list(idx)]
        Sb = (rk[:, None, None] * db[:, :, None] * db[:, None, :]).sum(axis=0) / Nk
        sigma[np.ix_(idx, idx)] = O.clamp_eigen(Sb, eps)
    return mu, sigma, Nk


def _no_mass_guard(zw, rk, mu_old, sigma_old, p):
    with np.errstate(invalid="ignore", divide="ignore"):
        return _orig["mstep_one"](zw, rk, mu_old, sigma_old, O.Params(
            lam=p.lam, eps_s=p.eps_s, eps_c=p.eps_c, cov_mode=p.cov_mode, n_min=-1.0))


def _spacing_rounded(W, H, K=None, vx=None, vy=None):
    if vx is None or vy is None:
        vx = vy = max(1, int(round(math.sqrt(W * H / K))))
    return _orig["make_grid"](W, H, vx=vx, vy=vy)


def _window_short(g, k):
    xb, xe, yb, ye = _orig["window"](g, k)
    kx, _ = O.superpixel_coords(g, k)
    return xb, min(xe, g.vx * (kx + 1) + g.vx - 1), yb, ye


def _ties_to_largest(R, cand):
    Rm = np.where(cand >= 0, R, -1.0)
    j = Rm.shape[-1] - 1 - np.flip(Rm, axis=-1).argmax(axis=-1)
    return np.take_along_axis(cand, j[..., None], axis=-1)[..., 0]


def _colour_init_lambda(g, z, p):
    th = _orig["init_theta"](g, z, p)
    for c in range(2, z.shape[-1]):
        th.sigma[:, c, c] = p.lam
    return th


def _seed_at_corner(g, k):
    kx, ky = O.superpixel_coords(g, k)
    return kx * g.vx + g.W * (ky * g.vy)


def _colour_floor_spatial(cov_mode, p):
    return [p.eps_s for _ in _orig["block_eps"](cov_mode, p)]


def _scaled_floor_unscaled_back(S, floors):
    """floors applied in the scaled coordinates but the result not scaled back"""
    f = np.sqrt(np.asarray(floors, dtype=np.float64))
    w, Q = np.linalg.eigh(S / np.outer(f, f))
    return (Q * np.maximum(w, 1.0)[None, :]) @ Q.T


def _scaled_floor_by_floors(S, floors):
    """scaled by the floors themselves instead of their square roots"""
    f = np.asarray(floors, dtype=np.float64)
    w, Q = np.linalg.eigh(S / np.outer(f, f))
    return np.outer(f, f) * ((Q * np.maximum(w, 1.0)[None, :]) @ Q.T)


def _floors_colour_first(cov_mode, p):
    fl = _orig["component_floors"](cov_mode, p)
    return fl[::-1].copy()


MUTANTS = [
    ("ln det Sigma dropped from the log density", "log_density_pairs", _logdet_dropped,
     [PINS.test_log_density_matches_scipy]),
    ("quadratic form added instead of subtracted", "log_density_pairs", _quadratic_sign,
     [PINS.test_log_density_matches_scipy]),
    ("(2 pi)^(-D/2) dropped", "log_density_pairs", _two_pi_dropped,
     [PINS.test_log_density_matches_scipy]),
    ("posteriors divided by the largest density, not the sum", "estep", _normalised_by_max,
     [PINS.test_estep_invariants_and_likelihood_brute_force]),
    ("L(theta) without the max shift added back", "estep", _likelihood_without_shift,
     [PINS.test_estep_invariants_and_likelihood_brute_force]),
    ("floor applied to the diagonal, not the eigenvalues", "clamp_eigen", _clamp_diagonal,
     [PINS.test_clamp_eigen]),
    ("floor taken on the standard deviation", "clamp_eigen", _clamp_std,
     [PINS.test_clamp_eigen]),
    ("covariance divided by N - 1", "mstep_one", _unbiased_covariance,
     [PINS.test_mstep_one_hot_is_sample_mean_and_covariance,
      PINS.test_mstep_weighted_matches_numpy_average_and_cov]),
    ("covariance about the previous mean", "mstep_one", _covariance_about_old_mean,
     [PINS.test_mstep_one_hot_is_sample_mean_and_covariance,
      PINS.test_mstep_weighted_matches_numpy_average_and_cov]),
    ("no guard for a superpixel without mass", "mstep_one", _no_mass_guard,
     [PINS.test_mstep_zero_mass_keeps_parameters]),
    ("seed spacing rounded instead of floored", "make_grid", _spacing_rounded,
     [PINS.test_grid_hand_values]),
    ("window one pixel short of its right edge", "window", _window_short,
     [PINS.test_candidates_closed_form, PINS.test_pair_counts_of_configs]),
    ("argmax ties to the largest k", "labels_from", _ties_to_largest,
     [PINS.test_label_ties_go_to_lowest_k]),
    ("colour variances initialised to lambda, not lambda^2", "init_theta", _colour_init_lambda,
     [PINS.test_init_seed_pixels_hand_values]),
    ("seed at the cell corner, not its centre", "seed_index", _seed_at_corner,
     [PINS.test_init_seed_pixels_hand_values]),
    ("colour blocks floored with the spatial epsilon", "block_eps", _colour_floor_spatial,
     [PINS.test_separated_blocks_are_recovered]),
    ("full-Sigma floor not scaled back", "clamp_eigen_scaled", _scaled_floor_unscaled_back,
     [MODES.test_scaled_floor_is_the_block_rule_on_block_diagonal_sigma,
      MODES.test_scaled_floor_properties]),
    ("full-Sigma floor scaled by the floors, not their roots", "clamp_eigen_scaled",
     _scaled_floor_by_floors,
     [MODES.test_scaled_floor_is_the_block_rule_on_block_diagonal_sigma,
      MODES.test_scaled_floor_properties]),
    ("component floors in the wrong order", "component_floors", _floors_colour_first,
     [MODES.test_scaled_floor_is_the_block_rule_on_block_diagonal_sigma,
      MODES.test_scaled_floor_maximises_the_constrained_likelihood]),
]


@pytest.mark.parametrize("what,name,mutant,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(monkeypatch, what, name, mutant, pins):
    monkeypatch.setattr(O, name, mutant)
    assert any(_pin_fails(pin) for pin in pins), f"no pin caught: {what}"


def test_pins_pass_on_the_oracle_itself():
    """The same harness over the unmodified oracle: every pin used above passes."""
    used = {pin for *_, pins in MUTANTS for pin in pins}
    assert not [p.__name__ for p in used if _pin_fails(p)]
