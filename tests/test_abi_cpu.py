"""Host-side checks of the C ABI: the library loads, exports every entry point
that include/gmmsp.h declares, computes the seed grid bit-exactly like the
oracle and rejects bad arguments with the documented codes.  No GPU needed:
nothing here launches a kernel."""
import ctypes
import os
import re
from ctypes import byref, c_int32, c_size_t, c_void_p

import numpy as np
import pytest

from oracle import gmm_oracle as O
from paper_1612_08792_amd import _lib
from paper_1612_08792_amd.gmmsp import make_params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gmmsp.h")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gmmsp_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    L = _lib.lib()
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert sorted(_lib.exported_symbols()) == names


def test_params_struct_layout_matches_header():
    # int32 W H K vx vy | pad | double eps_s eps_c lambda | int32 cov_mode | pad | double n_min
    assert ctypes.sizeof(_lib.GmmspParams) == 64
    assert _lib.GmmspParams.eps_s.offset == 24
    assert _lib.GmmspParams.n_min.offset == 56


def _grid(W, H, K=0, vx=0, vy=0):
    g = _lib.GmmspGridInfo()
    rc = _lib.lib().gmmsp_grid(byref(make_params(W, H, K, vx, vy)), byref(g))
    return rc, g


def test_grid_bit_exact_against_oracle():
    rng = np.random.default_rng(1)
    cases = [(481, 321, 400), (1920, 1080, 2000), (3840, 2160, 10000), (1, 1, 1),
             (7, 3, 21), (5000, 1, 17)]
    for _ in range(3000):
        W = int(rng.integers(1, 6000))
        H = int(rng.integers(1, 4000))
        cases.append((W, H, int(rng.integers(1, W * H + 1))))
    for W, H, K in cases:
        rc, g = _grid(W, H, K)
        try:
            og = O.make_grid(W, H, K=K)
        except ValueError:
            assert rc == _lib.GMMSP_E_SIZE
            continue
        assert rc == 0
        assert (g.vx, g.vy, g.nx, g.ny, g.K) == (og.vx, og.vy, og.nx, og.ny, og.K)
        assert g.ncx == -(-W // og.vx) and g.ncy == -(-H // og.vy)


def test_grid_explicit_spacing():
    rc, g = _grid(60, 41, vx=12, vy=7)
    og = O.make_grid(60, 41, vx=12, vy=7)
    assert rc == 0 and (g.nx, g.ny, g.K, g.ncx, g.ncy) == (og.nx, og.ny, og.K, 5, 6)


@pytest.mark.parametrize("args,code", [
    ((0, 5, 1), _lib.GMMSP_E_INVAL),
    ((5, 0, 1), _lib.GMMSP_E_INVAL),
    ((5, 5, 0), _lib.GMMSP_E_INVAL),
    ((5, 5, 26), _lib.GMMSP_E_INVAL),
    ((5, 5, 0, -1, 2), _lib.GMMSP_E_INVAL),
    ((5, 5, 0, 6, 2), _lib.GMMSP_E_SIZE),
])
def test_grid_error_codes(args, code):
    rc, _ = _grid(*args)
    assert rc == code
    assert len(_lib.lib().gmmsp_last_error()) > 0


def test_workspace_bytes_and_validation():
    L = _lib.lib()
    arr = (_lib.GmmspParams * 2)(make_params(481, 321, 400), make_params(640, 480, 512))
    n = c_size_t(0)
    assert L.gmmsp_workspace_bytes(2, arr, byref(n)) == 0
    n1 = c_size_t(0)
    assert L.gmmsp_workspace_bytes(1, arr, byref(n1)) == 0
    assert n.value > n1.value > 154401 // 10
    for m in (-1, 4):
        bad = (_lib.GmmspParams * 1)(make_params(481, 321, 400, cov_mode=m))
        assert L.gmmsp_workspace_bytes(1, bad, byref(n)) == _lib.GMMSP_E_INVAL
    # the 3x3 colour block and the full Sigma need wider records and rows, the
    # grayscale model narrower ones; one cov_mode per batch
    sizes = {}
    for m in (0, 1, 2, 3):
        arr_m = (_lib.GmmspParams * 1)(make_params(481, 321, 400, cov_mode=m))
        nm = c_size_t(0)
        assert L.gmmsp_workspace_bytes(1, arr_m, byref(nm)) == 0
        sizes[m] = nm.value
    assert sizes[3] < sizes[0] < sizes[1] < sizes[2]
    mixed = (_lib.GmmspParams * 2)(make_params(481, 321, 400), make_params(481, 321, 400, cov_mode=1))
    assert L.gmmsp_workspace_bytes(2, mixed, byref(n)) == _lib.GMMSP_E_INVAL
    bad = (_lib.GmmspParams * 1)(make_params(481, 321, 400, eps_c=0.0))
    assert L.gmmsp_workspace_bytes(1, bad, byref(n)) == _lib.GMMSP_E_INVAL
    assert L.gmmsp_workspace_bytes(0, arr, byref(n)) == _lib.GMMSP_E_INVAL
    # the widest image the E-step addresses with 32-bit offsets is 2^24 pixels
    wide = (_lib.GmmspParams * 1)(make_params(1 << 24, 64, 1 << 20))
    assert L.gmmsp_workspace_bytes(1, wide, byref(n)) == 0
    wide = (_lib.GmmspParams * 1)(make_params((1 << 24) + 1, 64, 1 << 20))
    assert L.gmmsp_workspace_bytes(1, wide, byref(n)) == _lib.GMMSP_E_SIZE


def test_create_rejects_bad_arguments_before_any_device_work():
    L = _lib.lib()
    arr = (_lib.GmmspParams * 1)(make_params(481, 321, 400))
    h = c_void_p()
    assert L.gmmsp_create(1, arr, None, 1 << 20, None, byref(h)) == _lib.GMMSP_E_INVAL
    # misaligned workspace pointer
    assert L.gmmsp_create(1, arr, c_void_p(0x1001), 1 << 20, None, byref(h)) == _lib.GMMSP_E_INVAL
    # too small a workspace
    assert L.gmmsp_create(1, arr, c_void_p(0x1000), 16, None, byref(h)) == _lib.GMMSP_E_SIZE
    assert L.gmmsp_em_iterate(None, None, 1, 0.0, None, None) == _lib.GMMSP_E_INVAL
    assert L.gmmsp_label(None, None, None, None, None) == _lib.GMMSP_E_INVAL
    assert L.gmmsp_init_seeds(None, None, None) == _lib.GMMSP_E_INVAL
    assert L.gmmsp_set_gather_lanes(None, 16) == _lib.GMMSP_E_INVAL
    assert L.gmmsp_get_gather_lanes(None, byref(c_int32())) == _lib.GMMSP_E_INVAL
    assert L.gmmsp_autotune_gather(None, None, 1, None, byref(c_int32()), None) == _lib.GMMSP_E_INVAL
    assert L.gmmsp_set_persistent(None, 1) == _lib.GMMSP_E_INVAL
    assert L.gmmsp_get_persistent(None, byref(c_int32())) == _lib.GMMSP_E_INVAL
    assert L.gmmsp_autotune_persistent(None, None, 1, None, byref(c_int32()), None) == _lib.GMMSP_E_INVAL


def test_connectivity_rejects_bad_arguments_before_any_device_work():
    L = _lib.lib()
    p = c_void_p(0x1000)
    assert L.gmmsp_conn_workspace_bytes(None, byref(c_size_t(0))) == _lib.GMMSP_E_INVAL
    assert L.gmmsp_connectivity(None, p, p, p, p, 1 << 20, 0, None, None) == _lib.GMMSP_E_INVAL


def test_metrics_rejects_bad_arguments_before_any_device_work():
    L = _lib.lib()
    p = c_void_p(0x1000)
    assert L.gmmsp_metrics_workspace_bytes(None, None, p, byref(c_size_t(0))) == _lib.GMMSP_E_INVAL
    assert L.gmmsp_metrics(None, p, p, None, p, p, 1 << 20, p, None, None) == _lib.GMMSP_E_INVAL


def test_colour_front_end_rejects_bad_arguments():
    L = _lib.lib()
    assert L.gmmsp_srgb8_to_lab(None, 4, c_void_p(0x1000), None) == _lib.GMMSP_E_INVAL
    assert L.gmmsp_srgb8_to_lab(c_void_p(0x1001), 4, c_void_p(0x1000), None) == _lib.GMMSP_E_INVAL
    assert L.gmmsp_srgb8_to_lab(c_void_p(0x1000), 4, c_void_p(0x1004), None) == _lib.GMMSP_E_INVAL
    assert L.gmmsp_srgb8_to_lab(c_void_p(0x1000), -1, c_void_p(0x1000), None) == _lib.GMMSP_E_INVAL
    assert L.gmmsp_srgb8_to_lab(c_void_p(0x1000), 0, c_void_p(0x1000), None) == 0
