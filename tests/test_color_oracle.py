"""Pins of the sRGB -> CIELAB oracle: published reference colours, the grey
axis, the continuity of both piecewise functions at their breakpoints, and a
round trip through the closed-form inverse."""
import numpy as np
import pytest

from oracle import color_oracle as C


# sRGB primaries, white and black in CIELAB (D65, 2 degrees) as commonly tabulated
@pytest.mark.parametrize("rgb,lab", [
    ((255, 0, 0), (53.2408, 80.0925, 67.2032)),
    ((0, 255, 0), (87.7347, -86.1827, 83.1793)),
    ((0, 0, 255), (32.2970, 79.1875, -107.8602)),
    ((255, 255, 255), (100.0, 0.0, 0.0)),
    ((0, 0, 0), (0.0, 0.0, 0.0)),
])
def test_reference_colours(rgb, lab):
    np.testing.assert_allclose(C.srgb8_to_lab(np.array(rgb, np.uint8)), lab, atol=2e-3)


def test_grey_axis_has_no_chroma():
    g = np.repeat(np.arange(256, dtype=np.uint8)[:, None], 3, axis=1)
    lab = C.srgb8_to_lab(g)
    assert np.abs(lab[:, 1:]).max() < 1e-3
    assert np.all(np.diff(lab[:, 0]) > 0)              # L* increases with the grey level


def test_piecewise_functions_are_continuous():
    c = 0.04045
    assert abs(C.srgb_to_linear(c) - ((c + 0.055) / 1.055) ** 2.4) < 1e-7
    t = C.DELTA ** 3
    assert abs(C.lab_f(t) - np.cbrt(t)) < 1e-12


def lab_to_srgb(lab):
    """Closed-form inverse, for the round trip."""
    L, a, b = lab[..., 0], lab[..., 1], lab[..., 2]
    fy = (L + 16.0) / 116.0
    fx, fz = fy + a / 500.0, fy - b / 200.0

    def finv(f):
        return np.where(f > C.DELTA, f ** 3, 3.0 * C.DELTA ** 2 * (f - 4.0 / 29.0))

    xyz = np.stack([finv(fx), finv(fy), finv(fz)], -1) * C.WHITE_D65
    lin = xyz @ np.linalg.inv(C.M_RGB_TO_XYZ).T
    c = np.where(lin <= 0.04045 / 12.92, lin * 12.92, 1.055 * np.abs(lin) ** (1 / 2.4) - 0.055)
    return c * 255.0


def test_round_trip():
    rng = np.random.default_rng(0)
    rgb = rng.integers(0, 256, (5000, 3)).astype(np.uint8)
    back = lab_to_srgb(C.srgb8_to_lab(rgb))
    np.testing.assert_allclose(back, rgb, atol=1e-6)
