"""Planted mistakes in the oracles of the connectivity step, the warm-start
network, the colour front end and the accuracy measures, each of which one of their pins must catch (the same
harness as ``test_oracle_mutations``: the mutant replaces one function on the CPU
and at least one listed pin, over all its parameter sets, has to fail)."""
import numpy as np
import pytest

import test_color_oracle as CP
import test_conn_oracle as KP
import test_metrics_oracle as MP
import test_ws_oracle as WP
from oracle import color_oracle as C
from oracle import conn_oracle as K
from oracle import metrics_oracle as M
from oracle import ws_oracle as WS
from test_oracle_mutations import _pin_fails

_conv, _bwd, _bf16 = WS.conv3x3, WS.conv3x3_backward, WS.bf16_round
_br, _ue_asa = M.boundary_recall, M.ue_asa_sums
_segments, _seg_colours = K.segments, K.segment_colours
_features, _theta0, _targets = WS.features, WS.theta0_rows, WS.targets


def _conv_flipped(x, W, b):
    """true convolution (taps mirrored) instead of the correlation of the kernels"""
    return _conv(x, W[:, ::-1, :], b)


def _bwd_dx_wrong_shift(x, W, dy_):
    ny, nx, ci = x.shape
    dxp = np.zeros((ny + 2, nx + 2, ci))
    _, dW, db = _bwd(x, W, dy_)
    for t, (dy, dx) in enumerate(WS.taps()):
        dxp[1 - dy:1 - dy + ny, 1 - dx:1 - dx + nx] += dy_ @ W[:, t, :].astype(np.float64)
    return dxp[1:-1, 1:-1], dW, db


def _bwd_dw_unshifted(x, W, dy_):
    dx, dW, db = _bwd(x, W, dy_)
    dW = np.repeat(np.einsum("yxo,yxi->oi", dy_, x)[:, None, :], 9, axis=1)
    return dx, dW, db


def _bf16_truncate(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    return ((a.view(np.uint32) >> 16) << 16).view(np.float32)


def _gamma_22(c):
    return np.asarray(c, dtype=np.float64) ** 2.2


def _lab_f_slope(t):
    t = np.asarray(t, dtype=np.float64)
    return np.where(t > C.DELTA ** 3, np.cbrt(t), t / (C.DELTA ** 2) + 4.0 / 29.0)


def _boundaries_right_only(labels):
    b = np.zeros(labels.shape, bool)
    b[:, :-1] |= labels[:, :-1] != labels[:, 1:]
    return b


def _recall_radius_one(sp, gt, r=2):
    return _br(sp, gt, 1)


def _ue_without_tolerance(sp, gt):
    ov = M.overlaps(sp, gt)
    size = {}
    for (k, g), c in ov.items():
        size[k] = size.get(k, 0) + c
    return sum(size[k] for (k, g), c in ov.items()), _ue_asa(sp, gt)[1]


def _asa_smallest_overlap(sp, gt):
    ov = M.overlaps(sp, gt)
    worst = {}
    for (k, g), c in ov.items():
        worst[k] = min(worst.get(k, c), c)
    return _ue_asa(sp, gt)[0], sum(worst.values())


def _segments_8_connected(labels):
    H, W = labels.shape
    seg = np.full((H, W), -1, dtype=np.int64)
    ids = []
    for y0 in range(H):
        for x0 in range(W):
            if seg[y0, x0] >= 0:
                continue
            sid = y0 * W + x0
            ids.append(sid)
            seg[y0, x0] = sid
            stack = [(y0, x0)]
            while stack:
                y, x = stack.pop()
                for yy in (y - 1, y, y + 1):
                    for xx in (x - 1, x, x + 1):
                        if (0 <= yy < H and 0 <= xx < W and seg[yy, xx] < 0
                                and labels[yy, xx] == labels[y0, x0]):
                            seg[yy, xx] = sid
                            stack.append((yy, xx))
    return seg, ids


def _colour_sums_not_means(lab, seg, ids):
    size, col = _seg_colours(lab, seg, ids)
    return size, {s: tuple(c * size[s] for c in col[s]) for s in ids}


def _distance_without_b(a, b):
    dL, da = a[0] - b[0], a[1] - b[1]
    return dL * dL + da * da


def _features_uncapped(lab, vx, vy, nx, ny):
    f = _features(lab, vx, vy, nx, ny)
    for ky in range(ny):
        for kx in range(nx):
            f[ky, kx, 6] = min(kx, ky, nx - 1 - kx, ny - 1 - ky) / 3.0
    return f


def _features_sample_std(lab, vx, vy, nx, ny):
    f = _features(lab, vx, vy, nx, ny)
    lab = np.asarray(lab, dtype=np.float64)
    for ky in range(ny):
        for kx in range(nx):
            px = lab[ky * vy:(ky + 1) * vy, kx * vx:(kx + 1) * vx].reshape(-1, 3)
            f[ky, kx, 3:6] = px.std(axis=0, ddof=1) / 16.0
    return f


def _features_half_cells_reversed(lab, vx, vy, nx, ny):
    f = _features(lab, vx, vy, nx, ny)
    f[..., 10:16] *= -1.0
    return f


def _theta0_log_variance(out, lab, vx, vy, lam, mask=WS.ALL_OUTPUTS):
    o = np.array(out, dtype=np.float64)
    o[..., 5:10] *= 0.5           # e^(s) where the law has e^(2 s)
    return _theta0(o, lab, vx, vy, lam, mask)


def _targets_log_variance(rows, lab, vx, vy, nx, ny, lam):
    t = _targets(rows, lab, vx, vy, nx, ny, lam)
    t[..., 5:10] *= 2.0
    return t


MUTANTS = [
    ("8- instead of 4-connected segments", K, "segments", _segments_8_connected,
     [KP.test_segments_match_scipy, KP.test_invariants_on_fragmented_labels]),
    ("segment colour sums instead of means", K, "segment_colours", _colour_sums_not_means,
     [KP.test_quantised_means_are_the_means, KP.test_fragment_joins_the_closer_colour]),
    ("colour distance without the b* term", K, "colour_dist2", _distance_without_b,
     [KP.test_colour_distance_counts_a_and_b]),
    ("border channel without its cap at 3 cells", WS, "features", _features_uncapped,
     [WP.test_border_channel_caps_at_three]),
    ("cell standard deviation with N - 1", WS, "features", _features_sample_std,
     [WP.test_half_cell_and_seed_channels_by_hand]),
    ("half-cell differences left minus right", WS, "features", _features_half_cells_reversed,
     [WP.test_half_cell_and_seed_channels_by_hand]),
    ("conv3x3 with mirrored taps", WS, "conv3x3", _conv_flipped,
     [WP.test_conv3x3_matches_scipy_correlate, WP.test_backward_matches_finite_differences]),
    ("data gradient shifted the wrong way", WS, "conv3x3_backward", _bwd_dx_wrong_shift,
     [WP.test_backward_matches_finite_differences]),
    ("weight gradient from the unshifted input", WS, "conv3x3_backward", _bwd_dw_unshifted,
     [WP.test_backward_matches_finite_differences]),
    ("bfloat16 by truncation, not round-to-nearest-even", WS, "bf16_round", _bf16_truncate,
     [WP.test_bf16_round_matches_torch]),
    ("sRGB decoded with a pure 2.2 power", C, "srgb_to_linear", _gamma_22,
     [CP.test_reference_colours, CP.test_piecewise_functions_are_continuous]),
    ("CIE f linear segment without its factor 3", C, "lab_f", _lab_f_slope,
     [CP.test_piecewise_functions_are_continuous]),
    ("sRGB-to-XYZ matrix transposed", C, "M_RGB_TO_XYZ", np.ascontiguousarray(C.M_RGB_TO_XYZ.T),
     [CP.test_reference_colours, CP.test_grey_axis_has_no_chroma]),
    ("D50 white instead of D65", C, "WHITE_D65", np.array([0.96422, 1.0, 0.82521]),
     [CP.test_grey_axis_has_no_chroma, CP.test_reference_colours]),
    ("boundary map without the lower neighbour", M, "boundaries", _boundaries_right_only,
     [MP.test_boundary_recall_window_across_rows]),
    ("boundary recall within one pixel, not two", M, "boundary_recall", _recall_radius_one,
     [MP.test_boundary_recall_window]),
    ("under-segmentation error without the 5 % tolerance", M, "ue_asa_sums",
     _ue_without_tolerance, [MP.test_one_superpixel_over_two_regions]),
    ("ASA with the smallest overlap", M, "ue_asa_sums", _asa_smallest_overlap,
     [MP.test_one_superpixel_over_two_regions, MP.test_identical_maps_are_perfect]),
]


@pytest.mark.parametrize("what,mod,name,mutant,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(monkeypatch, what, mod, name, mutant, pins):
    monkeypatch.setattr(mod, name, mutant)
    assert any(_pin_fails(pin) for pin in pins), f"no pin caught: {what}"


def test_pins_pass_on_the_oracles_themselves():
    used = {pin for *_, pins in MUTANTS for pin in pins}
    assert not [p.__name__ for p in used if _pin_fails(p)]


def test_log_variance_reading_in_both_directions_is_caught(monkeypatch):
    """Outputs read as log-variances in theta^0 and in the targets alike: the two
    stay inverse to each other, so only the hand pin of the scale law catches it."""
    monkeypatch.setattr(WS, "theta0_rows", _theta0_log_variance)
    monkeypatch.setattr(WS, "targets", _targets_log_variance)
    assert not _pin_fails(WP.test_targets_invert_theta0)
    assert _pin_fails(WP.test_log_scales_are_log_standard_deviations)
