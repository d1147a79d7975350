"""The row-strip sharding rule for one image over several GPUs, validated on
the CPU with the oracle: two strips of cell rows, each evaluating the E-step of
its own pixels with the parameters of its own superpixel rows plus one halo row
on each side, and forming partial M-step sums for the superpixels whose
windows reach it.  Only the two superpixel rows at the strip boundary receive
sums from both strips (the exchange), the log-likelihood is the sum of the
strips' values (an all-reduce), and the combined step equals the whole-image
oracle step."""
import numpy as np
import pytest

import synth
from oracle import gmm_oracle as O


@pytest.mark.parametrize("W,H,v,split", [(97, 120, 10, 6), (64, 50, 8, 3)])
def test_two_strip_step_equals_whole_image(W, H, v, split):
    im = synth.voronoi_lab(W, H, 9, 3.0, 21, 1)
    g = O.make_grid(W, H, vx=v, vy=v)
    res = O.run_em(im.lab.numpy(), g, max_iters=3)
    z, cand, theta = res["z"], res["cand"], res["theta"]
    p = O.Params()
    y_cut = split * g.vy                      # first pixel row of the second strip
    strips = [(0, y_cut), (y_cut, H)]
    ky_of = np.arange(g.K) // g.nx
    Ls, partial = [], []
    for s, (y0, y1) in enumerate(strips):
        c = cand[y0:y1]
        rows = np.unique(ky_of[c[c >= 0]])
        # parameters needed: the strip's own superpixel rows and one halo row
        own = (0, split - 1) if s == 0 else (split, g.ny - 1)
        assert rows.min() >= own[0] - 1 and rows.max() <= own[1] + 1
        R, _, L = O.estep(z[y0:y1], c, theta)
        Ls.append(L)
        # partial sums per superpixel about its current mean: N, S1, S2
        N = np.zeros(g.K)
        S1 = np.zeros((g.K, 5))
        S2 = np.zeros((g.K, 5, 5))
        zf = z[y0:y1].reshape(-1, 5)
        for j in range(9):
            sel = c.reshape(-1, 9)[:, j] >= 0
            k = c.reshape(-1, 9)[sel, j]
            r = R.reshape(-1, 9)[sel, j]
            d = zf[sel] - theta.mu[k]
            np.add.at(N, k, r)
            np.add.at(S1, k, r[:, None] * d)
            np.add.at(S2, k, r[:, None, None] * d[:, :, None] * d[:, None, :])
        partial.append((N, S1, S2))
    # the log-likelihood is the sum of the strips' values
    _, _, L_all = O.estep(z, cand, theta)
    assert sum(Ls) == pytest.approx(L_all, rel=1e-13)
    # only the two boundary superpixel rows receive sums from both strips
    both = (partial[0][0] > 0) & (partial[1][0] > 0)
    assert set(np.unique(ky_of[both])) == {split - 1, split}
    # combining the partials gives the whole-image M-step
    N = partial[0][0] + partial[1][0]
    S1 = partial[0][1] + partial[1][1]
    S2 = partial[0][2] + partial[1][2]
    want = O.mstep(z, g, *O.estep(z, cand, theta)[:1], O.window_positions(g, cand), theta, p)
    for k in range(g.K):
        m = S1[k] / N[k]
        mu = theta.mu[k] + m
        np.testing.assert_allclose(mu, want.mu[k], rtol=1e-10, atol=1e-9)
        for idx, eps in zip(O.blocks(0), O.block_eps(0, p)):
            Sb = S2[k][np.ix_(idx, idx)] / N[k] - np.outer(m[list(idx)], m[list(idx)])
            np.testing.assert_allclose(O.clamp_eigen(Sb, eps), want.sigma[k][np.ix_(idx, idx)],
                                       rtol=1e-8, atol=1e-8)
