"""GPU parity of the unified 3x3 colour block (cov_mode 1, Eq. BlockSigma) with
the FP64 oracle, through the C ABI: one step from an identical theta,
trajectories, separated blocks, edge shapes, the far-outlier path,
determinism, graph replay and the schedule restrictions.  Tolerances as for
the split colour blocks; the colour block error is the relative Frobenius
error of the whole 3x3 block."""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import gmm_oracle as O
from paper_1612_08792_amd.gmmsp import GMMSP
from parity_helpers import label_agreement, oracle_margin, oracle_slots

pytestmark = pytest.mark.gpu
P3 = O.Params(cov_mode=1)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def theta3_errors(g, o):
    """Largest mean error in std units; relative Frobenius error per block."""
    var = np.stack([o[:, 5], o[:, 7], o[:, 8], o[:, 11], o[:, 13]], 1)
    out = {"mean": float((np.abs(g[:, :5] - o[:, :5]) / np.sqrt(var)).max())}
    for name, idx in (("s", [[5, 6], [6, 7]]), ("Lab", [[8, 9, 10], [9, 11, 12], [10, 12, 13]])):
        Gm = np.stack([np.stack([g[:, j] for j in r], -1) for r in idx], -2)
        Om = np.stack([np.stack([o[:, j] for j in r], -1) for r in idx], -2)
        num = np.linalg.norm((Gm - Om).reshape(len(g), -1), axis=1)
        out[name] = float((num / np.linalg.norm(Om.reshape(len(g), -1), axis=1)).max())
    return out


def assert_close3(g, o, tol, what):
    e = theta3_errors(g, o)
    assert max(e.values()) <= tol, f"{what}: {e}"
    return e


def run_gpu(im, dev, T, K=None, v=None, rel_tol=0.0, graph=0):
    m = GMMSP([(im.W, im.H)], K=K if K is not None else im.K, v=v, device=dev, cov_mode=1)
    m.set_graph_passes(graph)
    lab = im.lab.reshape(-1).to(dev)
    m.init_seeds(lab)
    it = m.em_iterate(lab, T, rel_tol)
    labels, ll = m.label(lab)
    return dict(theta=m.get_params(), hist=m.ll_history(0), iters=it, ll_final=ll[0],
                labels=labels.cpu().numpy(), R=m.export_responsibilities(lab).cpu().numpy())


def test_init_rows(dev):
    im = synth.config1_image()
    g = O.make_grid(im.W, im.H, K=im.K)
    m = GMMSP([(im.W, im.H)], K=im.K, device=dev, cov_mode=1)
    assert m.theta_row == 15
    m.init_seeds(im.lab.reshape(-1).to(dev))
    want = O.theta_to_rows3(O.init_theta(g, O.features(im.lab.numpy()), P3))
    np.testing.assert_array_equal(m.get_params()[:, :14], want[:, :14])


def test_one_step_parity(dev):
    im = synth.config1_image()
    g = O.make_grid(im.W, im.H, K=im.K)
    res = O.run_em(im.lab.numpy(), g, P3, max_iters=3)
    m = GMMSP([(im.W, im.H)], K=im.K, device=dev, cov_mode=1)
    lab = im.lab.reshape(-1).to(dev)
    m.set_params(O.theta_to_rows3(res["theta"]))
    R = m.export_responsibilities(lab).cpu().numpy()
    assert np.abs(R - oracle_slots(g, res["cand"], res["R"])).max() <= 1e-5
    m.em_iterate(lab, 1)
    assert m.ll_history(0)[0] == pytest.approx(res["ll_final"], rel=1e-7)
    th1 = O.mstep(res["z"], g, res["R"], res["pos"], res["theta"], P3)
    e = assert_close3(m.get_params(), O.theta_to_rows3(th1), 1e-5, "one step")
    say("3x3 one-step errors", e)


def test_trajectory_T10(dev):
    im = synth.config1_image()
    g = O.make_grid(im.W, im.H, K=im.K)
    ref = O.run_em(im.lab.numpy(), g, P3, max_iters=10)
    out = run_gpu(im, dev, 10)
    e = assert_close3(out["theta"], O.theta_to_rows3(ref["theta"]), 1e-3, "T=10")
    r_err = np.abs(out["R"] - oracle_slots(g, ref["cand"], ref["R"])).max()
    assert r_err <= 1e-4
    agree, ties = label_agreement(out["labels"], ref["labels"].reshape(-1), oracle_margin(ref["R"]))
    assert agree >= 0.999
    np.testing.assert_allclose(out["hist"], ref["ll_hist"], rtol=1e-6)
    assert out["ll_final"] == pytest.approx(ref["ll_final"], rel=1e-6)
    say("3x3 T=10 errors", e, "R", r_err, "labels", agree, "ties", ties)


def test_separated_blocks(dev):
    for v, nbx, nby in [(6, 5, 4), (11, 3, 5)]:
        im = synth.separated_blocks(v, nbx, nby)
        out = run_gpu(im, dev, 4, v=v)
        assert np.array_equal(out["labels"], im.regions.numpy().reshape(-1))
        var = (v * v - 1) / 12.0
        th = out["theta"]
        for k in range(nbx * nby):
            kx, ky = k % nbx, k // nbx
            col = synth.BLOCK_PALETTE[(kx % 3) + 3 * (ky % 3)]
            np.testing.assert_allclose(th[k, :5], [kx * v + (v - 1) / 2, ky * v + (v - 1) / 2, *col],
                                       atol=1e-4)
            # constant colour: the 3x3 block is clamped to eps_c I
            np.testing.assert_allclose(th[k, 5:14], [var, 0, var, 8, 0, 0, 8, 0, 8], atol=1e-4 * var)


@pytest.mark.parametrize("W,H,K,v", [(9, 9, 1, None), (62, 45, None, 10), (60, 41, None, (12, 7))])
def test_edge_shapes(dev, W, H, K, v):
    im = synth.voronoi_lab(W, H, 3, 3.0, 11, K or 1)
    vx, vy = (v if isinstance(v, tuple) else (v, v)) if v else (None, None)
    g = O.make_grid(W, H, K=K, vx=vx, vy=vy)
    ref = O.run_em(im.lab.numpy(), g, P3, max_iters=4)
    out = run_gpu(im, dev, 4, K=K, v=v)
    assert_close3(out["theta"], O.theta_to_rows3(ref["theta"]), 1e-3, f"{W}x{H}")
    assert np.abs(out["R"] - oracle_slots(g, ref["cand"], ref["R"])).max() <= 1e-4


def test_far_outlier_and_determinism(dev):
    im = synth.voronoi_lab(64, 48, 4, 2.0, 12, 12)
    lab = im.lab.clone()
    lab[10, 10] = torch.tensor([900.0, -800.0, 700.0])
    im.lab = lab
    g = O.make_grid(64, 48, K=12)
    ref = O.run_em(lab.numpy(), g, P3, max_iters=2)
    a = run_gpu(im, dev, 2)
    b = run_gpu(im, dev, 2)
    assert np.isfinite(a["R"]).all()
    assert np.abs(a["R"] - oracle_slots(g, ref["cand"], ref["R"])).max() <= 1e-4
    assert np.array_equal(a["theta"], b["theta"]) and np.array_equal(a["hist"], b["hist"])


def test_graph_replay_and_schedules(dev):
    im = synth.voronoi_lab(320, 240, 19, 3.0, 77, 200)
    eager = run_gpu(im, dev, 12)
    graph = run_gpu(im, dev, 12, graph=5)
    assert np.array_equal(eager["theta"], graph["theta"])
    assert np.array_equal(eager["hist"], graph["hist"])
    m = GMMSP([(im.W, im.H)], K=im.K, device=dev, cov_mode=1)
    with pytest.raises(Exception):
        m.set_schedule(2)
    assert m.autotune(im.lab.reshape(-1).to(dev), passes=1, cache=None) == 1
    with pytest.raises(Exception):
        m.ws_attach()
