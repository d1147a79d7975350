"""Pins of the accuracy-measure oracle (BR, UE Eq. ue, ASA Eq. asa): closed
forms on hand-built maps, a distance-transform form of the boundary recall,
and an independent pair count for the overlap sums."""
import numpy as np
import pytest
from scipy import ndimage

import synth
from oracle import metrics_oracle as M


def test_identical_maps_are_perfect():
    im = synth.voronoi_lab(60, 45, 12, 3.0, 7, 20)
    gt = im.regions.numpy()
    m = M.metrics(gt, gt)
    assert m["BR"] == 1.0 and m["UE"] == 0.0 and m["ASA"] == 1.0


def test_one_superpixel_over_two_regions():
    gt = np.zeros((10, 20), np.int64)
    gt[:, 7:] = 1                                   # 70 and 130 pixels
    sp = np.zeros_like(gt)
    m = M.metrics(sp, gt)
    assert m["UE"] == 1.0                           # both overlaps exceed 5 %: 2 N / N - 1
    assert m["ASA"] == 130 / 200
    # an overlap of at most 5 % is not a leak: 10 of 200 pixels, 20 * 10 = 200
    gt2 = np.zeros((10, 20), np.int64)
    gt2[0, :10] = 1
    assert M.metrics(sp, gt2)["UE"] == 0.0
    gt2[1, 0] = 1                                   # 11 pixels: 220 > 200
    assert M.metrics(sp, gt2)["UE"] == 1.0


@pytest.mark.parametrize("d,hit", [(0, True), (1, True), (2, True), (3, False), (-2, True), (-3, False)])
def test_boundary_recall_window(d, hit):
    gt = np.zeros((12, 24), np.int64)
    gt[:, 10:] = 1                                  # ground-truth boundary pixels at x = 9
    sp = np.zeros_like(gt)
    sp[:, 10 + d:] = 1                              # superpixel boundary pixels at x = 9 + d
    hits, total = M.boundary_recall(sp, gt)
    assert total == 12 and hits == (12 if hit else 0)


@pytest.mark.parametrize("d,hit", [(0, True), (2, True), (3, False), (-2, True), (-3, False)])
def test_boundary_recall_window_across_rows(d, hit):
    # the transposed case: a boundary between rows, found through the lower neighbour
    gt = np.zeros((24, 12), np.int64)
    gt[10:, :] = 1                                  # ground-truth boundary pixels at y = 9
    sp = np.zeros_like(gt)
    sp[10 + d:, :] = 1                              # superpixel boundary pixels at y = 9 + d
    hits, total = M.boundary_recall(sp, gt)
    assert total == 12 and hits == (12 if hit else 0)


@pytest.mark.parametrize("seed", [0, 1])
def test_boundary_recall_by_distance_transform(seed):
    a = synth.voronoi_lab(70, 50, 15, 3.0, seed, 30).regions.numpy()
    b = synth.voronoi_lab(70, 50, 25, 3.0, seed + 10, 30).regions.numpy()
    hits, total = M.boundary_recall(a, b)
    gb, sb = M.boundaries(b), M.boundaries(a)
    dist = ndimage.distance_transform_cdt(~sb, metric="chessboard")
    assert total == int(gb.sum())
    assert hits == int((dist[gb] <= 2).sum())


@pytest.mark.parametrize("seed", [2, 3])
def test_overlap_sums_by_pair_counting(seed):
    sp = synth.voronoi_lab(64, 48, 30, 3.0, seed, 30).regions.numpy()
    gt = synth.voronoi_lab(64, 48, 9, 3.0, seed + 20, 30).regions.numpy()
    ue, asa = M.ue_asa_sums(sp, gt)
    keys, counts = np.unique(sp.astype(np.int64) * 1000 + gt, return_counts=True)
    k = keys // 1000
    size = {kk: counts[k == kk].sum() for kk in np.unique(k)}
    want_ue = sum(size[kk] for kk, c in zip(k, counts) if c * 20 > size[kk])
    want_asa = sum(counts[k == kk].max() for kk in np.unique(k))
    assert ue == want_ue and asa == want_asa
    m = M.metrics(sp, gt)
    assert 0.0 <= m["UE"] and 0.0 < m["ASA"] <= 1.0 and 0.0 <= m["BR"] <= 1.0
