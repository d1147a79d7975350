"""Schedules (statistics-pass kind, rows per chunk and waves per cell, lanes
per superpixel of the gather), the autotuners, graph replay and the 64-image
uneven batch: every path against the oracle or bitwise against the eager
single-image path."""
import os
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import gmm_oracle as O
from paper_1612_08792_amd.gmmsp import GMMSP
from parity_helpers import window_step, assert_theta_close, oracle_slots

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def cfg1():
    im = synth.config1_image()
    g = O.make_grid(im.W, im.H, K=im.K)
    ref = O.run_em(im.lab.numpy(), g, max_iters=10)
    return im, g, ref


def run(im, dev, T, wpc=1, graph=0, rel_tol=0.0, K=None, lanes=1, kind=None, rows=None):
    m = GMMSP([(im.W, im.H)], K=K or im.K, device=dev)
    if kind is not None:
        m.set_estep_kernel(kind)
    if rows is not None:
        m.set_slot_rows(rows)
    m.set_schedule(wpc)
    m.set_gather_lanes(lanes)
    m.set_graph_passes(graph)
    lab = im.lab.reshape(-1).to(dev)
    m.init_seeds(lab)
    it = m.em_iterate(lab, T, rel_tol)
    labels, ll = m.label(lab)
    return dict(theta=m.get_params(), hist=m.ll_history(0), labels=labels.cpu().numpy(),
                iters=it, R=m.export_responsibilities(lab).cpu().numpy(), ll=ll[0])


@pytest.mark.parametrize("wpc", [1, 2, 4])
def test_schedule_matches_oracle_and_repeats(dev, cfg1, wpc):
    im, g, ref = cfg1
    a = run(im, dev, 10, wpc)
    b = run(im, dev, 10, wpc)
    assert np.array_equal(a["theta"], b["theta"]) and np.array_equal(a["hist"], b["hist"])
    assert_theta_close(a["theta"], O.theta_to_rows(ref["theta"]), 1e-3, what=f"wpc {wpc}")
    np.testing.assert_allclose(a["hist"], ref["ll_hist"], rtol=1e-6)
    assert np.abs(a["R"] - oracle_slots(g, ref["cand"], ref["R"])).max() <= 1e-4


# every candidate the autotuner times on the 481x321 grid (v = 19: J = 3 columns
# per lane, rows per chunk 3, 2, 1)
CANDIDATES = [(1, r, w) for r in (3, 2, 1) for w in (1, 2, 4)] + [(0, None, w) for w in (1, 2, 4)]


@pytest.mark.parametrize("kind,rows,wpc", CANDIDATES)
def test_every_tuned_candidate_matches_oracle(dev, cfg1, kind, rows, wpc):
    im, g, ref = cfg1
    a = run(im, dev, 10, wpc, kind=kind, rows=rows)
    assert_theta_close(a["theta"], O.theta_to_rows(ref["theta"]), 1e-3,
                       what=f"kind {kind} rows {rows} wpc {wpc}")
    np.testing.assert_allclose(a["hist"], ref["ll_hist"], rtol=1e-6)
    assert np.abs(a["R"] - oracle_slots(g, ref["cand"], ref["R"])).max() <= 1e-4
    b = run(im, dev, 10, wpc, kind=kind, rows=rows)
    assert np.array_equal(a["theta"], b["theta"]) and np.array_equal(a["hist"], b["hist"])
    if kind == 1 and wpc == 1 and rows != 3:
        # one wave per cell: every rows value gives the same passes bit for bit
        base = run(im, dev, 10, 1, kind=1, rows=3)
        assert np.array_equal(a["theta"], base["theta"])
        assert np.array_equal(a["hist"], base["hist"])


def test_slot_rows_restrictions(dev):
    im = synth.config1_image()                 # v = 19: J = 3
    m = GMMSP([(im.W, im.H)], K=im.K, device=dev)
    assert m.get_estep_kernel() == 1 and m.get_slot_rows() == 3
    for bad in (0, 4, 8, -1):
        with pytest.raises(Exception):
            m.set_slot_rows(bad)
    big = GMMSP([(640, 480)], v=60, device=dev)  # cells wider than 56 pixels
    assert big.get_estep_kernel() == 0 and big.get_slot_rows() == 0
    with pytest.raises(Exception):
        big.set_slot_rows(1)


@pytest.mark.parametrize("wpc,graph,tol", [(1, 4, 0.0), (2, 3, 0.0), (1, 5, 1e-4), (4, 2, 1e-4)])
def test_graph_replay_is_bitwise_eager(dev, wpc, graph, tol):
    im = synth.voronoi_lab(320, 240, 19, 3.0, 77, 200)
    eager = run(im, dev, 30 if tol else 10, wpc, 0, tol)
    m = GMMSP([(im.W, im.H)], K=im.K, device=dev)
    m.set_schedule(wpc)
    m.set_graph_passes(graph)
    lab = im.lab.reshape(-1).to(dev)
    for rep in range(3):                       # replays, with eager work between them
        m.init_seeds(lab)
        it = m.em_iterate(lab, 30 if tol else 10, tol)
        torch.cuda.synchronize()
        _ = torch.ones(1000, device=dev).sum().item()
        assert np.array_equal(m.get_params(), eager["theta"]), rep
        assert np.array_equal(m.ll_history(0), eager["hist"]), rep
        assert np.array_equal(it, eager["iters"]), rep


def test_graph_replay_follows_schedule_changes(dev):
    """A captured graph holds the kernels of its schedule: after the rows per
    chunk, the pass kind or the gather lanes change, replay re-captures and
    matches an eager run of the new schedule bit for bit."""
    im = synth.voronoi_lab(320, 240, 19, 3.0, 77, 200)
    lab = im.lab.reshape(-1).to(dev)
    m = GMMSP([(im.W, im.H)], K=im.K, device=dev)
    m.set_schedule(2)
    m.set_graph_passes(4)
    for kind, rows, lanes in [(1, 3, 1), (1, 1, 1), (0, 1, 4), (1, 2, 16)]:
        m.set_estep_kernel(kind)
        m.set_slot_rows(rows)
        m.set_gather_lanes(lanes)
        m.init_seeds(lab)
        it = m.em_iterate(lab, 30, 1e-4)
        eager = run(im, dev, 30, 2, 0, 1e-4, kind=kind, rows=rows, lanes=lanes)
        assert np.array_equal(m.get_params(), eager["theta"]), (kind, rows, lanes)
        assert np.array_equal(m.ll_history(0), eager["hist"]), (kind, rows, lanes)
        assert np.array_equal(it, eager["iters"]), (kind, rows, lanes)


@pytest.mark.parametrize("wpc,lanes", [(1, 16), (4, 16), (1, 4), (2, 4)])
def test_gather_lanes_match_one_lane_and_oracle(dev, cfg1, wpc, lanes):
    """4 or 16 lanes per superpixel: the FP64 sums group differently from one
    lane, so theta agrees to FP64 rounding after one pass and to the oracle's
    tolerances after ten; the schedule is bitwise repeatable and replays
    bitwise under graph capture."""
    im, g, ref = cfg1
    one1 = run(im, dev, 1, wpc)
    ln_1 = run(im, dev, 1, wpc, lanes=lanes)
    np.testing.assert_allclose(ln_1["theta"], one1["theta"], rtol=1e-12, atol=1e-9)
    a = run(im, dev, 10, wpc, lanes=lanes)
    b = run(im, dev, 10, wpc, lanes=lanes)
    c = run(im, dev, 10, wpc, graph=4, lanes=lanes)
    assert np.array_equal(a["theta"], b["theta"]) and np.array_equal(a["hist"], b["hist"])
    assert np.array_equal(a["theta"], c["theta"]) and np.array_equal(a["hist"], c["hist"])
    assert_theta_close(a["theta"], O.theta_to_rows(ref["theta"]), 1e-3,
                       what=f"lanes {lanes}, wpc {wpc}")
    np.testing.assert_allclose(a["hist"], ref["ll_hist"], rtol=1e-6)
    assert np.abs(a["R"] - oracle_slots(g, ref["cand"], ref["R"])).max() <= 1e-4


def test_gather_lanes_restrictions(dev):
    im = synth.voronoi_lab(64, 48, 4, 3.0, 5, 12)
    m = GMMSP([(im.W, im.H)], K=im.K, device=dev)
    assert m.get_gather_lanes() == 1
    for bad in (0, 2, 8, 32):
        with pytest.raises(Exception):
            m.set_gather_lanes(bad)
    for mode in (1, 2, 3):
        mm = GMMSP([(im.W, im.H)], K=im.K, device=dev, cov_mode=mode)
        for lanes in (4, 16):
            with pytest.raises(Exception):
                mm.set_gather_lanes(lanes)


def test_autotune_picks_a_schedule(dev, tmp_path):
    ims = synth.config3_batch(n_images=6)
    lab = synth.pack_batch(ims).to(dev)
    m = GMMSP([(im.W, im.H) for im in ims], K=[im.K for im in ims], device=dev)
    cache = str(tmp_path / "schedules.json")
    w = m.autotune(lab, passes=2, cache=cache)
    assert w in (1, 2, 4) and m.get_schedule() == w
    vmax = max(g.vx for g in m.grids)
    J = -(-vmax // 7)
    n_rows = {1: 3, 2: 3, 3: 3, 4: 2, 5: 2 if vmax <= 32 else 1}.get(J, 1)
    assert os.path.exists(cache) and len(m.tune_ms) == 3 * (n_rows + 1)
    assert all(v > 0 for v in m.tune_ms.values())
    assert set(m.tune_gather_ms) == {1, 4, 16} and m.get_gather_lanes() in (1, 4, 16)
    assert all(v > 0 for v in m.tune_gather_ms.values())
    say("autotune ms", m.tune_ms, "picked", w, "gather ms", m.tune_gather_ms,
        "lanes", m.get_gather_lanes())
    # the handle is initialised: EM runs and matches a fresh run with that schedule
    it = m.em_iterate(lab, 3)
    assert list(it) == [3] * 6
    m2 = GMMSP([(im.W, im.H) for im in ims], K=[im.K for im in ims], device=dev)
    assert m2.autotune(lab, passes=2, cache=cache) == w          # from the cache
    assert m2.tune_cached and m2.schedule() == m.schedule()
    m2.em_iterate(lab, 3)
    assert np.array_equal(m.get_params(), m2.get_params())


def test_uneven_batch_of_64_images(dev):
    say("64-image uneven batch, T = 15")
    ims = synth.config3_batch(device=dev)
    assert len(ims) == 64
    for im in ims:
        assert O.make_grid(im.W, im.H, K=im.K).vx == 24
    lab = synth.pack_batch(ims).to(dev)
    sizes = [(im.W, im.H) for im in ims]
    m = GMMSP(sizes, K=[im.K for im in ims], device=dev)
    m.init_seeds(lab)
    m.em_iterate(lab, 14)
    th14 = m.get_params()
    R = m.export_responsibilities(lab).cpu().numpy()
    m.em_iterate(lab, 1)
    th15 = m.get_params()
    labels, _ = m.label(lab)
    labels = labels.cpu().numpy()
    # the batch equals each image run alone
    for b in (0, 31, 63):
        one = run(ims[b], dev, 15)
        assert np.array_equal(th15[m.sp_slice(b)], one["theta"]), b
        assert np.array_equal(labels[m.image_slice(b)], one["labels"]), b
    # one EM step from the GPU's theta^14 against the oracle, whole image
    for b in (0, 63):
        im = ims[b]
        g = O.make_grid(im.W, im.H, K=im.K)
        z = O.features(im.lab.cpu().numpy())
        cand, _ = O.candidate_sets(g)
        th = O.rows_to_theta(th14[m.sp_slice(b)])
        Ro, _, _ = O.estep(z, cand, th)
        assert np.abs(R[m.image_slice(b)] - oracle_slots(g, cand, Ro)).max() <= 1e-5
        th1 = O.mstep(z, g, Ro, O.window_positions(g, cand), th, O.Params())
        assert_theta_close(th15[m.sp_slice(b)], O.theta_to_rows(th1), 1e-5, what=f"image {b}")
    # one EM step on sampled windows of every image of the batch
    rng = np.random.default_rng(64)
    worst = 0.0
    for b, im in enumerate(ims):
        g = O.make_grid(im.W, im.H, K=im.K)
        z = O.features(im.lab.cpu().numpy())
        cand, _ = O.candidate_sets(g)
        sl = m.sp_slice(b)
        th = O.rows_to_theta(th14[sl])
        Rimg = R[m.image_slice(b)].reshape(im.H, im.W, 9)
        ks = rng.choice(g.K, 4, replace=False)
        got, want = np.empty((4, 13)), np.empty((4, 13))
        for j, k in enumerate(ks):
            xb, xe, yb, ye = O.window(g, int(k))
            err, want[j], _, _ = window_step(g, z, cand, th, k, Rimg[yb:ye, xb:xe])
            worst = max(worst, err)
            assert err <= 1e-5, (b, k, err)
            got[j] = th15[sl][k]
        assert_theta_close(got, want, 1e-5, what=f"image {b}, sampled windows")
    say(f"64 images, 256 sampled windows: R err {worst:.2e}")
