"""Pins of the warm-start network oracle: convolution against scipy, backward
against central finite differences, bfloat16 rounding against torch, and the
exact inverse relation between targets and theta^0."""
import math

import numpy as np
import pytest
import torch
from scipy.signal import correlate2d

from oracle import ws_oracle as WS


def test_param_count():
    # 16*9*32+32 + 2*(32*9*32+32) + 32*9*10+10
    assert WS.param_count() == 4640 + 2 * 9248 + 2890


def test_conv3x3_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(6, 7, 3))
    W = rng.normal(size=(4, 9, 3))
    b = rng.normal(size=4)
    got = WS.conv3x3(x, W, b)
    for o in range(4):
        want = b[o] + sum(correlate2d(x[:, :, i], W[o, :, i].reshape(3, 3), mode="same")
                          for i in range(3))
        np.testing.assert_allclose(got[:, :, o], want, rtol=1e-12, atol=1e-12)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    ny, nx = 4, 5
    params = rng.normal(scale=0.3, size=WS.param_count())
    x0 = rng.normal(size=(ny, nx, WS.C_IN))
    tgt = rng.normal(size=(ny, nx, WS.C_OUT))
    loss, g = WS.loss_and_grads(params, x0, tgt, ny * nx)
    idx = rng.choice(params.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        p1, p2 = params.copy(), params.copy()
        p1[i] += h
        p2[i] -= h
        l1, _ = WS.loss_and_grads(p1, x0, tgt, ny * nx)
        l2, _ = WS.loss_and_grads(p2, x0, tgt, ny * nx)
        fd = (l1 - l2) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.normal(size=5000).astype(np.float32) * 10.0 ** rng.integers(-6, 6, 5000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 65504.0], np.float32)])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(WS.bf16_round(x), want)


def test_features_of_constant_cells_and_border_channel():
    lab = np.zeros((12, 20, 3), np.float32)
    lab[..., 0], lab[..., 1], lab[..., 2] = 70.0, -32.0, 16.0
    f = WS.features(lab, 4, 4, 5, 3)
    np.testing.assert_allclose(f[..., 0], 0.4)
    np.testing.assert_allclose(f[..., 1], -0.5)
    np.testing.assert_allclose(f[..., 2], 0.25)
    np.testing.assert_allclose(f[..., 3:6], 0.0, atol=1e-12)
    np.testing.assert_allclose(f[..., 7:16], 0.0, atol=1e-12)
    # distance to the border in cells, capped at 3, over 3: a 5 x 3 grid
    np.testing.assert_allclose(f[..., 6] * 3, [[0, 0, 0, 0, 0], [0, 1, 1, 1, 0], [0, 0, 0, 0, 0]])


def test_border_channel_caps_at_three():
    # a 9 x 9 grid of 2 x 2 cells: the centre cell is 4 cells from every border,
    # capped at 3; the ring next to the border is 1
    f = WS.features(np.zeros((18, 18, 3), np.float32), 2, 2, 9, 9)
    d = np.minimum(np.minimum(np.arange(9)[:, None], np.arange(9)[None, :]),
                   np.minimum(8 - np.arange(9)[:, None], 8 - np.arange(9)[None, :]))
    np.testing.assert_allclose(f[..., 6] * 3, np.minimum(d, 3))
    assert f[4, 4, 6] == 1.0


def test_half_cell_and_seed_channels_by_hand():
    # one 5 x 5 cell: L = 10 x (column), a = 4 x (row), b = 0; h = 2
    lab = np.zeros((5, 5, 3), np.float32)
    lab[..., 0] = 10.0 * np.arange(5)[None, :]
    lab[..., 1] = 4.0 * np.arange(5)[:, None]
    f = WS.features(lab, 5, 5, 1, 1)[0, 0]
    # right columns {3, 4} minus left {0, 1}: L 35 - 5 = 30; rows likewise for a: 14 - 2 = 12
    np.testing.assert_allclose(f[10:13], [30 / 32, 0, 0], atol=1e-12)
    np.testing.assert_allclose(f[13:16], [0, 12 / 32, 0], atol=1e-12)
    # seed (2, 2): colour (20, 8, 0), cell mean (20, 8, 0)
    np.testing.assert_allclose(f[7:10], 0.0, atol=1e-12)
    np.testing.assert_allclose(f[3], np.std(10.0 * np.arange(5)) / 16)


def test_zero_output_is_the_grid_init():
    rng = np.random.default_rng(3)
    lab = rng.uniform(0, 50, (19 * 2, 19 * 3, 3)).astype(np.float32)
    rows = WS.theta0_rows(np.zeros((2, 3, 10)), lab, 19, 19, 8.0)
    assert rows[4, 0] == 19 + 9 and rows[4, 1] == 19 + 9          # k = (1, 1)
    np.testing.assert_array_equal(rows[4, 2:5], lab[28, 28])
    np.testing.assert_allclose(rows[:, [5, 7, 8, 9, 11]], [[361, 361, 64, 64, 64]] * 6)
    assert np.all(rows[:, [6, 10]] == 0)


def test_log_scales_are_log_standard_deviations():
    # Sigma^0 = diag(v_x^2 e^(2 s_x), v_y^2 e^(2 s_y), lambda^2 e^(2 s_L), ...): an
    # output s = ln 2 doubles the standard deviation (four times the variance),
    # and a mean output of 1/2 moves the mean by half a cell / half of lambda
    lab = np.zeros((20, 30, 3), np.float32)
    out = np.zeros((2, 3, 10))
    out[1, 2] = [0.5, -0.5, 0.5, 0, 0, math.log(2), 0, 0, math.log(2), 0]
    rows = WS.theta0_rows(out, lab, 10, 10, 8.0)
    r = rows[1 * 3 + 2]
    assert r[0] == 25 + 5 and r[1] == 15 - 5 and r[2] == 4.0
    np.testing.assert_allclose(r[[5, 7, 8, 9, 11]], [400, 100, 64, 256, 64], rtol=1e-12)


def test_output_mask_zeroes_outputs():
    rng = np.random.default_rng(5)
    lab = rng.uniform(0, 50, (30, 40, 3)).astype(np.float32)
    out = rng.uniform(-1, 1, (3, 4, 10))
    mask = 0b0001100011          # mu_x, mu_y, S_xx, S_yy only
    got = WS.theta0_rows(out, lab, 10, 10, 8.0, mask)
    kept = out * np.array([(mask >> c) & 1 for c in range(10)])
    np.testing.assert_array_equal(got, WS.theta0_rows(kept, lab, 10, 10, 8.0))


def test_targets_invert_theta0():
    rng = np.random.default_rng(4)
    lab = rng.uniform(0, 50, (45, 68, 3)).astype(np.float32)
    out = rng.uniform(-2, 2, (3, 4, 10))
    rows = WS.theta0_rows(out, lab, 17, 15, 8.0)
    np.testing.assert_allclose(WS.targets(rows, lab, 17, 15, 4, 3, 8.0), out, rtol=1e-10,
                               atol=1e-12)
