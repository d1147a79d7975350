"""Pins of the connectivity post-processing oracle: components against
scipy.ndimage.label, hand-built cases for each rule of the paper's procedure
(colour-nearest destination, ascending size order, size update, inherited
neighbours, ties), and invariants on fragment-heavy label maps."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import conn_oracle as C


def partition(seg):
    """Canonical form of a partition: relabel by first appearance."""
    _, inv = np.unique(seg.ravel(), return_inverse=True)
    first = {}
    out = np.empty(inv.size, np.int64)
    for i, v in enumerate(inv):
        out[i] = first.setdefault(v, len(first))
    return out


def scipy_partition(labels):
    """4-connected components of equal label with scipy, one label value at a time."""
    out = np.zeros(labels.shape, np.int64)
    nxt = 1
    for v in np.unique(labels):
        cc, n = ndimage.label(labels == v)            # 4-connectivity by default
        out[cc > 0] = cc[cc > 0] + nxt - 1
        nxt += n
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_segments_match_scipy(seed):
    rng = np.random.default_rng(seed)
    labels = rng.integers(0, 4, (23, 31))
    labels[5:15, 3:20] = 7                            # a large blob with holes
    labels[8, 5:18] = rng.integers(0, 4, 13)
    seg, ids = C.segments(labels)
    assert np.array_equal(partition(seg), partition(scipy_partition(labels)))
    # ids are the raster index of each segment's first pixel
    H, W = labels.shape
    for s in ids:
        y, x = divmod(s, W)
        assert seg[y, x] == s
        assert not np.any(seg.ravel()[:s] == s)


def test_quantised_means_are_the_means():
    rng = np.random.default_rng(3)
    labels = rng.integers(0, 3, (12, 9))
    lab = rng.uniform(-100, 100, (12, 9, 3)).astype(np.float32)
    seg, ids = C.segments(labels)
    size, col = C.segment_colours(lab, seg, ids)
    for s in ids:
        m = lab[seg == s].astype(np.float64).mean(0)
        assert size[s] == int((seg == s).sum())
        np.testing.assert_allclose(col[s], m, rtol=0, atol=2.0 ** -20)


def flat_image(H, W, colour):
    lab = np.zeros((H, W, 3), np.float32)
    lab[..., 0] = colour
    return lab


def test_fragment_joins_the_closer_colour():
    # left half L = 50, right half L = 60, a 2 x 2 fragment of L = 58 on the seam
    labels = np.zeros((12, 12), np.int64)
    labels[:, 6:] = 1
    labels[5:7, 5:7] = 2
    lab = flat_image(12, 12, 50.0)
    lab[:, 6:, 0] = 60.0
    lab[5:7, 5:7, 0] = 58.0
    out, info = C.enforce_connectivity(labels, lab, 6, 6)
    assert info["merged"] == 1
    assert np.all(out[5:7, 5:7] == 6)                 # id of the right half: pixel (0, 6)
    assert np.all(out[:, :6][labels[:, :6] == 0] == 0)


def test_colour_distance_counts_a_and_b():
    # equal L everywhere; the right half differs from the left only in a* (then
    # only in b*), and the fragment is 2 from the right half and 8 from the left
    # in that channel alone, so it must join the right half both times
    for ch in (1, 2):
        labels = np.zeros((12, 12), np.int64)
        labels[:, 6:] = 1
        labels[5:7, 5:7] = 2
        lab = flat_image(12, 12, 50.0)
        lab[:, 6:, ch] = 10.0
        lab[5:7, 5:7, ch] = 8.0
        out, info = C.enforce_connectivity(labels, lab, 6, 6)
        assert info["merged"] == 1, ch
        assert np.all(out[5:7, 5:7] == 6), ch


def test_size_update_keeps_a_grown_segment():
    # A (2 px, L 50) merges into B (7 px, L 52); B then has 9 px, 4 * 9 >= 36,
    # so B stays although its own 7 px are below a quarter of 6 x 6
    labels = np.zeros((10, 10), np.int64)
    lab = flat_image(10, 10, 10.0)
    labels[0, 0:2] = 1
    lab[0, 0:2, 0] = 50.0
    labels[1, 0:7] = 2
    lab[1, 0:7, 0] = 52.0
    out, info = C.enforce_connectivity(labels, lab, 6, 6)
    assert info["merged"] == 1
    assert np.all(out[0, 0:2] == 10) and np.all(out[1, 0:7] == 10)   # B's id: pixel (1, 0)
    # without the grown size B (7 px) would have been merged into the background
    labels2 = labels.copy()
    labels2[0, 0:2] = 0
    lab2 = lab.copy()
    lab2[0, 0:2, 0] = 10.0
    out2, info2 = C.enforce_connectivity(labels2, lab2, 6, 6)
    assert info2["merged"] == 1 and np.all(out2 == 0)


def test_merged_pixels_bring_their_neighbours():
    # A (1 px, L 50.0) touches Y (row 0, L 51), B and the background X (L 10);
    # B (6 px, L 50.2) touches only A and X.  A joins B; B, still small, then
    # sees Y through A's pixel and joins Y instead of X.
    labels = np.zeros((10, 10), np.int64)
    lab = flat_image(10, 10, 10.0)
    labels[0, :] = 3
    lab[0, :, 0] = 51.0
    labels[1, 0] = 1
    lab[1, 0, 0] = 50.0
    labels[2:4, 0:3] = 2
    lab[2:4, 0:3, 0] = 50.2
    out, info = C.enforce_connectivity(labels, lab, 6, 6)
    assert info["small"] == 2 and info["merged"] == 2
    assert out[1, 0] == 0 and np.all(out[2:4, 0:3] == 0)              # all in Y (id 0)
    assert np.all(out[4:, :] == 11)                                   # X keeps its id: pixel (1, 1)


def test_equal_distances_go_to_the_smaller_id():
    labels = np.zeros((8, 8), np.int64)
    labels[:, 4:] = 1
    labels[3, 3] = 2
    lab = flat_image(8, 8, 40.0)
    lab[:, 4:, 0] = 60.0
    lab[3, 3, 0] = 50.0                               # 10 from both halves
    out, _ = C.enforce_connectivity(labels, lab, 4, 4)
    assert out[3, 3] == 0


def test_single_segment_and_no_small_segments():
    labels = np.zeros((5, 7), np.int64)
    lab = flat_image(5, 7, 33.0)
    out, info = C.enforce_connectivity(labels, lab, 5, 7)
    assert info["merged"] == 0 and np.all(out == 0)
    # a tiny image that is one small segment has no neighbour and stays
    out, info = C.enforce_connectivity(labels[:1, :1], lab[:1, :1], 5, 5)
    assert info["small"] == 1 and info["merged"] == 0


@pytest.mark.parametrize("seed", [4, 5])
def test_invariants_on_fragmented_labels(seed):
    rng = np.random.default_rng(seed)
    H, W, v = 30, 41, 6
    # blocky labels with 15 % of the pixels flipped to a random neighbour label
    labels = (np.arange(H)[:, None] // v) * 10 + (np.arange(W)[None, :] // v)
    flip = rng.random((H, W)) < 0.15
    labels = np.where(flip, labels + rng.integers(-1, 2, (H, W)), labels)
    lab = rng.normal(50, 10, (H, W, 3)).astype(np.float32)
    out, info = C.enforce_connectivity(labels, lab, v, v)
    assert info["merged"] > 0
    seg0, _ = C.segments(labels)
    for s in np.unique(out):
        region = out == s
        cc, n = ndimage.label(region)
        assert n == 1                                 # every output segment is connected
        assert 4 * region.sum() >= v * v or len(np.unique(out)) == 1
        y, x = divmod(int(s), W)
        assert out[y, x] == s                          # the id is one of its own pixels
    # segments that were not small keep all their pixels and their id
    sizes = np.bincount(seg0.ravel(), minlength=H * W)
    for s in np.unique(seg0):
        if 4 * sizes[s] >= v * v:
            assert np.all(out[seg0 == s] == s)
