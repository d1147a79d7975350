"""Persistent T-mode passes (one cooperative launch per em_iterate call, grid
barriers between the statistics pass and the gather): bitwise equal to the
per-pass launches of the same schedule, on single images, uneven batches with
stopped images, a grid larger than the GPU keeps resident, and after the
launch-form autotuner."""
import sys

import numpy as np
import pytest
import torch

import synth
from paper_1612_08792_amd import _lib
from paper_1612_08792_amd._lib import GmmspError
from paper_1612_08792_amd.gmmsp import GMMSP

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def make(ims, dev, rows=None, wpc=1, lanes=1, persistent=False):
    m = GMMSP([(im.W, im.H) for im in ims], K=[im.K for im in ims], device=dev)
    m.set_estep_kernel(1)
    if rows is not None:
        m.set_slot_rows(rows)
    m.set_schedule(wpc)
    m.set_gather_lanes(lanes)
    m.set_persistent(persistent)
    lab = synth.pack_batch(ims).to(dev).contiguous()
    return m, lab


def outcome(m, lab):
    labels, ll = m.label(lab)
    return dict(theta=m.get_params(), labels=labels.cpu().numpy(), ll=np.array(ll),
                hist=[m.ll_history(b) for b in range(m.n_images)])


def assert_same(a, b, what):
    assert np.array_equal(a["theta"], b["theta"]), what
    assert np.array_equal(a["labels"], b["labels"]), what
    assert np.array_equal(a["ll"], b["ll"]), what
    for ha, hb in zip(a["hist"], b["hist"]):
        assert np.array_equal(ha, hb), what


@pytest.mark.parametrize("rows,wpc,lanes", [(3, 1, 1), (2, 2, 4), (1, 4, 16), (3, 1, 16)])
def test_single_image_equals_per_pass_launches(dev, rows, wpc, lanes):
    im = synth.config1_image()
    say(f"481x321 K 400, rows {rows}, waves per cell {wpc}, gather lanes {lanes}, T 10")
    res = []
    for pers in (False, True):
        m, lab = make([im], dev, rows, wpc, lanes, pers)
        m.init_seeds(lab)
        assert list(m.em_iterate(lab, 10)) == [10]
        res.append(outcome(m, lab))
    assert_same(res[0], res[1], f"rows {rows} wpc {wpc} lanes {lanes}")


def test_uneven_batch_with_stopped_images(dev):
    ims = [synth.voronoi_lab(333, 217, 18, 3.0, 5, 150),
           synth.voronoi_lab(97, 180, 6, 2.0, 6, 40),
           synth.voronoi_lab(640, 481, 60, 4.0, 7, 512)]
    say("3 uneven images: EM with the stop rule (per-pass launches), then 6 T-mode passes")
    res = []
    for pers in (False, True):
        m, lab = make(ims, dev, wpc=2, lanes=4, persistent=pers)
        m.init_seeds(lab)
        it = m.em_iterate(lab, 40, 2e-3)   # the stop rule: never the persistent launch
        assert min(it) < 40                # some images have stopped
        m.em_iterate(lab, 6)               # stopped images stay stopped
        res.append((list(it), outcome(m, lab)))
    assert res[0][0] == res[1][0]
    assert_same(res[0][1], res[1][1], "uneven batch")


def test_grid_beyond_resident_blocks(dev):
    # one 3840x2160 image, K 10000 -> 10549 cells: 2638 blocks of the statistics
    # pass, more than the GPU keeps resident, so each block takes several cells
    im = synth.config5_batch(device="cpu", n_images=1)[0]
    say("3840x2160 K 10549, T 3: a grid-stride persistent launch")
    res = []
    for pers in (False, True):
        m, lab = make([im], dev, persistent=pers)
        m.init_seeds(lab)
        m.em_iterate(lab, 3)
        res.append(outcome(m, lab))
    assert_same(res[0], res[1], "4K grid-stride")


def test_profiled_calls_keep_per_pass_launches(dev):
    im = synth.config1_image()
    m, lab = make([im], dev, persistent=True)
    assert m.get_persistent() == 1
    m.init_seeds(lab)
    m.profile(True)
    m.profile_read(reset=True)
    m.em_iterate(lab, 4)
    p = m.profile_read(reset=True)
    m.profile(False)
    assert p["launches"] == 4          # per-pass launches, each timed
    a = outcome(m, lab)
    m2, _ = make([im], dev, persistent=False)
    m2.init_seeds(lab)
    m2.em_iterate(lab, 4)
    assert_same(a, outcome(m2, lab), "profiled")


def test_launch_form_autotuner(dev):
    im = synth.config1_image()
    m = GMMSP([(im.W, im.H)], K=im.K, device=dev)
    lab = im.lab.reshape(-1).to(dev)
    m.autotune(lab, passes=3, cache=None)
    s = m.schedule()
    say(f"tuned schedule {s}, launch-form times {m.tune_persistent_ms}")
    assert m.tune_persistent_ms["per_pass"] > 0
    assert all(v > 0 for v in m.tune_persistent_ms.values())
    assert s["persistent"] in (0, 1)
    if s["persistent"]:
        assert s["estep_kernel"] == 1
    m.init_seeds(lab)
    m.em_iterate(lab, 10)
    a = outcome(m, lab)
    # the same schedule with per-pass launches
    m2 = GMMSP([(im.W, im.H)], K=im.K, device=dev)
    m2.set_estep_kernel(s["estep_kernel"])
    if s["estep_kernel"] == 1:
        m2.set_slot_rows(s["rows_per_chunk"])
    m2.set_schedule(s["waves_per_cell"])
    m2.set_gather_lanes(s["gather_lanes"])
    m2.init_seeds(lab)
    m2.em_iterate(lab, 10)
    assert_same(a, outcome(m2, lab), "tuned")


def test_persistent_needs_the_slot_lane_pass(dev):
    im = synth.config1_image()
    m = GMMSP([(im.W, im.H)], K=im.K, device=dev, cov_mode=1)
    with pytest.raises(GmmspError) as e:
        m.set_persistent(True)
    assert e.value.code == _lib.GMMSP_E_INVAL
    assert m.get_persistent() == 0
