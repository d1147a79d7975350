"""The benchmarked path at full size, against the FP64 oracle.

Two images of the 4K batch workload (3840x2160 Voronoi-Lab, 2000 regions, noise
sigma ~ U[1, 6], K = 10000 requested -> v = 28, 137 x 77 = 10549 superpixels)
run exactly the benchmark's step in its launch configuration: the library's
schedule autotuners, the learned warm start with the benchmark's output mask
(features, network, theta^0, and the guard that keeps the grid seeds where
they give the higher L(theta^0)), EM until the relative change of L is <= 1e-5
(cap 200; Algorithm 1 with the stop rule), and the labels (Eq. obtLi).  Checked:

* theta^0 from the network's outputs against the oracle's map (ws_oracle) with
  the eigenvalue floors, at v = 28;
* one oracle step (Eq. Rik, Eqs. UpdateMu .. eigdecrc) from the GPU's final
  theta on sampled windows: posteriors abs <= 1e-5, theta^{t+1} <= 1e-5;
* the GPU's final labels against the oracle's argmax on the same windows:
  >= 99.9 % of the non-tie pixels.
"""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import gmm_oracle as O
from oracle import ws_oracle as WS
from paper_1612_08792_amd import train_warmstart, warmstart
from paper_1612_08792_amd.gmmsp import GMMSP
from parity_helpers import TIE, assert_theta_close, window_step

pytestmark = pytest.mark.gpu

SEEDS = (30000, 30017)
WINDOWS = 24   # sampled superpixel windows per image


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def run(dev):
    say("headline path: 2 x 3840x2160, warm start, EM to rel-tol 1e-5, labels")
    ims = [synth.config5_batch(device="cpu", n_images=1, first_seed=s)[0] for s in SEEDS]
    lab = synth.pack_batch(ims).to(dev).contiguous()
    m = GMMSP([(im.W, im.H) for im in ims], K=ims[0].K, device=dev)
    m.autotune(lab, passes=3, cache=None)
    params = warmstart.load(train_warmstart.DEFAULT_OUT, dev)
    flags = warmstart.warm_start(m, lab, params, warmstart.APPLY_MASK, guard=True,
                                 want_flags=True)
    theta0 = m.get_params()
    out = m.ws_read("out")
    iters = m.em_iterate(lab, 200, 1e-5)
    labels, _ = m.label(lab)
    theta_f = m.get_params()
    R = m.export_responsibilities(lab)          # at the final theta
    # one more pass from the final theta (the stop rule has ended the run)
    m.set_params(theta_f)
    assert list(m.em_iterate(lab, 1)) == [1, 1]
    theta_f1 = m.get_params()
    say(f"passes {list(iters)}, schedule: kernel {m.get_estep_kernel()}, "
        f"{m.get_schedule()} waves per cell, {m.get_gather_lanes()} gather lanes")
    return dict(ims=ims, m=m, flags=flags, theta0=theta0, out=out, iters=iters, labels=labels,
                theta_f=theta_f, theta_f1=theta_f1, R=R)


def test_warm_start_theta0_matches_oracle(run):
    m = run["m"]
    for b, im in enumerate(run["ims"]):
        g = m.grids[b]
        assert (g.vx, g.vy, g.nx, g.ny) == (28, 28, 137, 77)
        sl = m.sp_slice(b)
        if run["flags"][b]:   # the guard kept the grid seeds for this image
            og = O.make_grid(im.W, im.H, K=im.K)
            seeds = O.theta_to_rows(O.init_theta(og, O.features(im.lab.numpy()), O.Params()))
            np.testing.assert_array_equal(run["theta0"][sl, :12], seeds[:, :12])
            continue
        want = WS.theta0_rows(run["out"][sl].reshape(g.ny, g.nx, 16)[..., :10], im.lab.numpy(),
                              g.vx, g.vy, 8.0, warmstart.APPLY_MASK)
        want[:, 5] = np.maximum(want[:, 5], 2.0)
        want[:, 7] = np.maximum(want[:, 7], 2.0)
        want[:, [8, 9, 11]] = np.maximum(want[:, [8, 9, 11]], 8.0)
        np.testing.assert_allclose(run["theta0"][sl, :12], want[:, :12], rtol=1e-12, atol=1e-9)


def test_converged_run_one_step_and_labels_match_oracle(run):
    m = run["m"]
    assert all(20 <= int(t) <= 200 for t in run["iters"])
    for b, im in enumerate(run["ims"]):
        g = O.make_grid(im.W, im.H, K=im.K)
        z = O.features(im.lab.numpy())
        cand, _ = O.candidate_sets(g)
        sl = m.sp_slice(b)
        th = O.rows_to_theta(run["theta_f"][sl])
        Rimg = run["R"][m.image_slice(b)].view(im.H, im.W, 9)
        Limg = run["labels"][m.image_slice(b)].view(im.H, im.W)
        rng = np.random.default_rng(b)
        ks = rng.choice(g.K, WINDOWS, replace=False)
        got, want = np.empty((WINDOWS, 13)), np.empty((WINDOWS, 13))
        r_err, n_nontie, n_agree, n_tie = 0.0, 0, 0, 0
        for j, k in enumerate(ks):
            xb, xe, yb, ye = O.window(g, int(k))
            err, want[j], Rw, cw = window_step(g, z, cand, th, k,
                                               Rimg[yb:ye, xb:xe].cpu().numpy())
            r_err = max(r_err, err)
            got[j] = run["theta_f1"][sl][k]
            lo = O.labels_from(Rw, cw)
            srt = np.sort(Rw, axis=-1)
            nontie = (srt[..., -1] - srt[..., -2]) > TIE
            lg = Limg[yb:ye, xb:xe].cpu().numpy()
            n_nontie += int(nontie.sum())
            n_agree += int((lg == lo)[nontie].sum())
            n_tie += int((~nontie).sum())
        e = assert_theta_close(got, want, 1e-5, what=f"image {b} one step from the final theta")
        agree = n_agree / max(1, n_nontie)
        say(f"image {b}: R err {r_err:.2e}, theta errors {e}, labels {agree:.5f} of "
            f"{n_nontie} non-tie pixels ({n_tie} ties)")
        assert r_err <= 1e-5
        assert agree >= 0.999
