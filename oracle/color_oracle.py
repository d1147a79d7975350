"""Plain FP64 CPU oracle of the colour front end: 8-bit sRGB to CIELAB.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library.

The paper runs the method in CIELAB (Sec. IV) without stating the conversion.
Reading (the HIP path follows it): sRGB per IEC 61966-2-1 (8-bit code / 255,
the piecewise transfer function with the 0.04045 breakpoint), linear RGB to
XYZ with the sRGB primaries and the D65 white, CIE 1976 L*a*b* relative to the
D65 white of the 2-degree observer (X_n, Y_n, Z_n) = (0.95047, 1, 1.08883).
"""
from __future__ import annotations

import numpy as np

M_RGB_TO_XYZ = np.array([[0.4124564, 0.3575761, 0.1804375],
                         [0.2126729, 0.7151522, 0.0721750],
                         [0.0193339, 0.1191920, 0.9503041]])
WHITE_D65 = np.array([0.95047, 1.0, 1.08883])
DELTA = 6.0 / 29.0


def srgb_to_linear(c: np.ndarray) -> np.ndarray:
    """The sRGB transfer function inverted, c in [0, 1]."""
    c = np.asarray(c, dtype=np.float64)
    return np.where(c <= 0.04045, c / 12.92, ((c + 0.055) / 1.055) ** 2.4)


def lab_f(t: np.ndarray) -> np.ndarray:
    """CIE 1976 f: cube root above delta^3, the linear segment below."""
    t = np.asarray(t, dtype=np.float64)
    return np.where(t > DELTA ** 3, np.cbrt(t), t / (3.0 * DELTA ** 2) + 4.0 / 29.0)


def srgb8_to_lab(rgb: np.ndarray) -> np.ndarray:
    """(..., 3) uint8 sRGB -> (..., 3) float64 L*, a*, b*."""
    lin = srgb_to_linear(np.asarray(rgb, dtype=np.float64) / 255.0)
    xyz = lin @ M_RGB_TO_XYZ.T
    f = lab_f(xyz / WHITE_D65)
    L = 116.0 * f[..., 1] - 16.0
    a = 500.0 * (f[..., 0] - f[..., 1])
    b = 200.0 * (f[..., 1] - f[..., 2])
    return np.stack([L, a, b], -1)
