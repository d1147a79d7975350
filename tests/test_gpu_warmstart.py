"""GPU parity of the warm-start network kernels (through the C ABI) against the
FP64 oracle.  Each layer is checked on the GPU's own bfloat16 inputs and
bf16-rounded weights, so the only difference left is FP32 versus FP64
accumulation: FP32 results within 1e-5 (normwise), bf16 results within one
bf16 rounding step."""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import gmm_oracle as O
from oracle import ws_oracle as WS
from paper_1612_08792_amd import warmstart
from paper_1612_08792_amd.gmmsp import GMMSP

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def grids_of(m):
    return [(g.nx, g.ny, g.vx, g.vy) for g in m.grids]


def split(arr, m):
    """(n_sp, C) batch array -> list of (ny, nx, C) grids."""
    out = []
    for b, (nx, ny, _, _) in enumerate(grids_of(m)):
        out.append(arr[m.sp_slice(b)].reshape(ny, nx, -1).astype(np.float64))
    return out


def normwise(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


@pytest.fixture(scope="module")
def batch(dev):
    ims = [synth.voronoi_lab(481, 321, 40, 3.0, 10000, 400),
           synth.voronoi_lab(250, 190, 15, 5.0, 10001, 150)]
    lab = synth.pack_batch(ims).to(dev)
    m = GMMSP([(im.W, im.H) for im in ims], K=[im.K for im in ims], device=dev)
    m.ws_attach()
    m.ws_features(lab)
    return ims, lab, m


def test_features_match_oracle(batch):
    ims, lab, m = batch
    feat = m.ws_read("feat")
    for b, im in enumerate(ims):
        g = m.grids[b]
        want = WS.features(im.lab.numpy(), g.vx, g.vy, g.nx, g.ny)
        got = feat[m.sp_slice(b)].reshape(g.ny, g.nx, 16)
        np.testing.assert_allclose(got, want, rtol=1e-5, atol=1e-5)
    x0 = m.ws_read("x0")
    np.testing.assert_array_equal(x0, WS.bf16_round(feat))


def _params(dev, seed=3, last_std=0.2):
    p = warmstart.init_params(seed)
    rng = np.random.default_rng(seed)
    off = sum(co * 9 * ci + co for ci, co in WS.LAYERS[:3])
    p[off:off + 10 * 9 * 32] = rng.normal(0, last_std, 10 * 9 * 32)
    p[-10:] = rng.normal(0, 0.1, 10)
    # non-zero biases for the hidden layers too
    o = 0
    for ci, co in WS.LAYERS:
        o += co * 9 * ci
        p[o:o + co] = rng.normal(0, 0.05, co)
        o += co
    return p


def test_forward_layers_match_oracle(batch, dev):
    ims, lab, m = batch
    p = _params(dev)
    m.ws_forward(torch.from_numpy(p).to(dev))
    layers = WS.unpack(p.astype(np.float64))
    acts = [split(m.ws_read(n), m) for n in ("x0", "y1", "y2", "y3")]
    out = split(m.ws_read("out"), m)
    for b in range(len(ims)):
        for li in range(3):
            W, bias = layers[li]
            ref = WS.conv3x3(acts[li][b], WS.bf16_round(W).astype(np.float64), bias)
            want = WS.bf16_round(np.maximum(ref, 0).astype(np.float32)).astype(np.float64)
            got = acts[li + 1][b]
            exact = np.mean(got == want)
            ulp = np.abs(got - want) <= np.abs(want) * 2.0 ** -7 + 1e-30
            assert exact >= 0.999 and ulp.all(), (b, li, exact)
        W, bias = layers[3]
        ref = WS.conv3x3(acts[3][b], WS.bf16_round(W).astype(np.float64), bias)
        assert normwise(out[b][..., :10], ref) <= 1e-5
        assert np.all(out[b][..., 10:] == 0)


def test_backward_matches_oracle(batch, dev):
    ims, lab, m = batch
    p = _params(dev, seed=5)
    rng = np.random.default_rng(6)
    tgt = np.zeros((m.n_superpixels, 16), np.float32)
    tgt[:, :10] = rng.normal(0, 0.5, (m.n_superpixels, 10))
    m.ws_write("tgt", tgt)
    params = torch.from_numpy(p).to(dev)
    mom, vel = torch.zeros_like(params), torch.zeros_like(params)
    loss = m.ws_train_step(params, mom, vel, 1, 1e-3)
    layers = WS.unpack(p.astype(np.float64))
    xs = [split(m.ws_read(n), m) for n in ("x0", "y1", "y2", "y3")]
    gs = [split(m.ws_read(n), m) for n in ("g1", "g2", "g3", "g4")]
    out = split(m.ws_read("out"), m)
    grad = m.ws_read("grad")
    count = m.n_superpixels
    # loss and the output gradient 2 (o - t) / 10
    want_loss = sum(float(np.sum((o[..., :10] - t) ** 2)) for o, t in
                    zip(out, split(tgt[:, :10], m))) / (count * 10)
    assert loss == pytest.approx(want_loss, rel=1e-6)
    ogrid = split(tgt, m)
    for b in range(len(ims)):
        g4 = WS.bf16_round((0.2 * (out[b] - ogrid[b])).astype(np.float32))
        g4[..., 10:] = 0
        np.testing.assert_array_equal(gs[3][b], g4)
    # weight and bias gradients: sum over positions of g (x) shifted input
    o = 0
    for li, (ci, co) in enumerate(WS.LAYERS):
        dW = np.zeros((co, 9, ci))
        db = np.zeros(co)
        for b in range(len(ims)):
            gl = gs[li][b][..., :co]
            _, dWb, dbb = WS.conv3x3_backward(xs[li][b], np.zeros((co, 9, ci)), gl)
            dW += dWb
            db += dbb
        got_W = grad[o:o + co * 9 * ci].reshape(co, 9, ci)
        got_b = grad[o + co * 9 * ci:o + co * 9 * ci + co]
        assert normwise(got_W, dW / count) <= 1e-5, li
        assert normwise(got_b, db / count) <= 1e-5, li
        o += co * 9 * ci + co
    # input gradients through the ReLU: g_{l-1} = bf16((W^T g_l) * (y_{l-1} > 0))
    for li in (3, 2, 1):
        W, _ = layers[li]
        ci, co = WS.LAYERS[li]
        for b in range(len(ims)):
            dx, _, _ = WS.conv3x3_backward(xs[li][b], WS.bf16_round(W).astype(np.float64),
                                           gs[li][b][..., :co])
            want = dx * (xs[li][b] > 0)
            assert normwise(gs[li - 1][b], want) <= 1e-2, li
            rounded = WS.bf16_round(want.astype(np.float32))
            assert np.mean(gs[li - 1][b] == rounded) >= 0.99, li


@pytest.mark.parametrize("mask", [0x3FF, 0b0001100011])
def test_apply_and_targets_match_oracle(batch, dev, mask):
    ims, lab, m = batch
    p = _params(dev, seed=7, last_std=0.05)
    m.ws_forward(torch.from_numpy(p).to(dev))
    m.ws_apply(lab, mask)
    rows = m.get_params()
    out = m.ws_read("out")
    for b, im in enumerate(ims):
        g = m.grids[b]
        want = WS.theta0_rows(out[m.sp_slice(b)].reshape(g.ny, g.nx, 16)[..., :10],
                              im.lab.numpy(), g.vx, g.vy, 8.0, mask)
        want[:, 5] = np.maximum(want[:, 5], 2.0)
        want[:, 7] = np.maximum(want[:, 7], 2.0)
        want[:, [8, 9, 11]] = np.maximum(want[:, [8, 9, 11]], 8.0)
        np.testing.assert_allclose(rows[m.sp_slice(b), :12], want[:, :12], rtol=1e-12, atol=1e-9)
    # targets from the theta just set: the inverse map gives back the used
    # outputs wherever no floor or clip was active
    m.ws_targets(lab)
    tgt = m.ws_read("tgt")
    use = np.array([(mask >> c) & 1 for c in range(10)], dtype=np.float32)
    o = out[:, :10] * use
    ls = np.clip(o[:, 5:10], -4, 4)
    free = (np.abs(o[:, 5:10]) < 4).all(1)
    for b, im in enumerate(ims):
        g = m.grids[b]
        sl = m.sp_slice(b)
        floors = np.array([2.0 / g.vx ** 2, 2.0 / g.vy ** 2, 8.0 / 64, 8.0 / 64, 8.0 / 64])
        ok = free[sl] & (np.exp(2 * ls[sl]) > floors).all(1)
        np.testing.assert_allclose(tgt[sl][ok, :10], np.concatenate([o[sl][ok, :5], ls[sl][ok]], 1),
                                   rtol=1e-5, atol=1e-5)
        want_t = WS.targets(rows[sl], im.lab.numpy(), g.vx, g.vy, g.nx, g.ny, 8.0)
        np.testing.assert_allclose(tgt[sl, :10], want_t.reshape(-1, 10), rtol=1e-5, atol=1e-5)


def test_non_finite_outputs_fall_back_to_grid_init(batch, dev):
    ims, lab, m = batch
    p = _params(dev, seed=8)
    p[-10:] = np.nan                           # every output becomes NaN
    m.ws_forward(torch.from_numpy(p).to(dev))
    m.ws_apply(lab)
    rows = m.get_params()
    for b, im in enumerate(ims):
        g = O.make_grid(im.W, im.H, K=im.K)
        th = O.init_theta(g, O.features(im.lab.numpy()), O.Params())
        np.testing.assert_array_equal(rows[m.sp_slice(b), :12], O.theta_to_rows(th)[:, :12])


def test_guarded_warm_start_keeps_the_better_start(batch, dev):
    """gmmsp_ws_apply_guarded: per image, the start with the higher L(theta^0)
    (the oracle's L of the grid seeds and of the network's theta^0 decides
    wherever the two differ clearly), and exactly that start's theta^0; weights
    scaled up 40-fold put every mean far off, and every image keeps the seeds."""
    from paper_1612_08792_amd import train_warmstart
    ims, lab, m = batch
    trained = warmstart.load(train_warmstart.DEFAULT_OUT, dev)
    for name, params in (("trained", trained), ("corrupted", trained * 40.0)):
        m.ws_forward(params)
        m.ws_apply(lab, warmstart.APPLY_MASK)            # the network's theta^0, unguarded
        warm_rows = m.get_params()
        flags = m.ws_apply_guarded(lab, warmstart.APPLY_MASK, want_flags=True)
        rows = m.get_params()
        for b, im in enumerate(ims):
            sl = m.sp_slice(b)
            g = O.make_grid(im.W, im.H, K=im.K)
            z = O.features(im.lab.numpy())
            cand, _ = O.candidate_sets(g)
            seeds = O.theta_to_rows(O.init_theta(g, z, O.Params()))
            L_seed = O.estep(z, cand, O.rows_to_theta(seeds))[2]
            L_warm = O.estep(z, cand, O.rows_to_theta(warm_rows[sl]))[2]
            say(f"{name} image {b}: L(seeds) {L_seed:.6e} L(network) {L_warm:.6e} "
                f"fallback {flags[b]}")
            if abs(L_warm - L_seed) > 1e-6 * abs(L_seed):
                assert flags[b] == int(L_warm < L_seed)
            want = seeds if flags[b] else warm_rows[sl]
            np.testing.assert_array_equal(rows[sl, :12], want[:, :12])
        if name == "corrupted":
            assert flags.tolist() == [1] * len(ims)


def test_training_lowers_loss_and_warm_start_gains(dev):
    say("warm start: train on 512 images, evaluate 32 held out")
    train_ims = [synth.config4_image(10000 + i, dev) for i in range(512)]
    params, info = warmstart.train(train_ims, dev, epochs=100, batch_images=32, lr=2e-3,
                                   target_passes=24)
    say("losses", [round(x, 4) for x in info["losses"][::10]])
    assert info["losses"][-1] < 0.7 * info["losses"][0]
    test_ims = [synth.config4_image(20000 + i, dev) for i in range(32)]
    lab = synth.pack_batch(test_ims).to(dev)
    sizes = [(im.W, im.H) for im in test_ims]
    plain = GMMSP(sizes, K=400, device=dev)
    plain.init_seeds(lab)
    plain.em_iterate(lab, 150, 1e-5)
    warm = GMMSP(sizes, K=400, device=dev)
    warmstart.warm_start(warm, lab, params, warmstart.APPLY_MASK, guard=True)
    warm.em_iterate(lab, 150, 1e-5)
    tp, tw, dl, np_, nw = [], [], [], [], []
    for b in range(len(test_ims)):
        hp, hw = plain.ll_history(b), warm.ll_history(b)
        tp.append(warmstart.passes_to_target(hp, hp[-1]))
        tw.append(warmstart.passes_to_target(hw, hp[-1]))
        dl.append((hw[-1] - hp[-1]) / abs(hp[-1]))
        np_.append(len(hp) - 1)
        nw.append(len(hw) - 1)
    dl, np_, nw = np.array(dl), np.array(np_), np.array(nw)
    # per image: an image whose warm-started optimum ends more than 1e-4 below the
    # plain one is charged a plain run on top of its warm one
    worse = dl < -1e-4
    charged = np.where(worse, nw + np_, nw)
    say("passes to the plain optimum within 1e-4: plain", np.mean(tp), "warm", np.mean(tw),
        "final L rel diff mean", dl.mean(), "min", dl.min(), "images below 1e-4:",
        int(worse.sum()), "passes to the stop rule: plain", np_.mean(), "warm, charged",
        charged.mean())
    assert np.mean(tw) < np.mean(tp)
    assert dl.mean() > -1e-4
    assert worse.sum() <= len(dl) // 8
    assert charged.mean() < np_.mean()
