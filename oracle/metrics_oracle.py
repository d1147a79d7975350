"""Plain CPU oracle of the segmentation accuracy measures the paper reports
(Sec. IV: boundary recall, under-segmentation error Eq. ue, achievable
segmentation accuracy Eq. asa), for a superpixel label map against a
ground-truth region map.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library.

Readings (the paper is silent or garbled on these; the HIP path follows them):

* M-1 a boundary pixel of a label map is a pixel whose right or lower
  4-neighbour carries another label; a ground-truth boundary pixel counts as
  recovered when a superpixel boundary pixel lies in the (2r+1) x (2r+1)
  square around it, r = 2 ("within two pixels"); BR = recovered / all
  ground-truth boundary pixels (1 when there are none);
* M-2 Eq. ue, garbled in the text, reads UE = (1/N) sum_g sum_{k :
  |s_k n s_g| > eps |s_k|} |s_k| - 1 with eps = 0.05, the comparison taken
  exactly as 20 |s_k n s_g| > |s_k|;
* M-3 Eq. asa: ASA = (1/N) sum_k max_g |s_k n s_g|;
* all three are ratios of integer counts, formed once in FP64.
"""
from __future__ import annotations

import numpy as np


def boundaries(labels: np.ndarray) -> np.ndarray:
    """M-1 boundary map: right or lower neighbour differs."""
    H, W = labels.shape
    b = np.zeros((H, W), bool)
    b[:, :-1] |= labels[:, :-1] != labels[:, 1:]
    b[:-1, :] |= labels[:-1, :] != labels[1:, :]
    return b


def boundary_recall(sp: np.ndarray, gt: np.ndarray, r: int = 2):
    """(recovered, total) ground-truth boundary pixels, by explicit windows."""
    H, W = sp.shape
    gb, sb = boundaries(gt), boundaries(sp)
    hits = total = 0
    for y, x in zip(*np.nonzero(gb)):
        total += 1
        win = sb[max(0, y - r):min(H, y + r + 1), max(0, x - r):min(W, x + r + 1)]
        hits += bool(win.any())
    return hits, total


def overlaps(sp: np.ndarray, gt: np.ndarray):
    """|s_k n s_g| for every pair that meets, as a dict {(k, g): count}."""
    out = {}
    for k, g in zip(sp.ravel().tolist(), gt.ravel().tolist()):
        out[(k, g)] = out.get((k, g), 0) + 1
    return out


def ue_asa_sums(sp: np.ndarray, gt: np.ndarray):
    """The integer sums of Eqs. ue and asa: (sum_g sum_{k: 20 c > |s_k|} |s_k|,
    sum_k max_g c) with c = |s_k n s_g|."""
    ov = overlaps(sp, gt)
    size, best = {}, {}
    for (k, g), c in ov.items():
        size[k] = size.get(k, 0) + c
        best[k] = max(best.get(k, 0), c)
    ue = sum(size[k] for (k, g), c in ov.items() if 20 * c > size[k])
    asa = sum(best.values())
    return ue, asa


def metrics(sp: np.ndarray, gt: np.ndarray):
    """BR, UE, ASA of one image (M-1 .. M-3)."""
    n = sp.size
    hits, total = boundary_recall(sp, gt)
    ue, asa = ue_asa_sums(sp, gt)
    br = hits / total if total else 1.0
    return dict(BR=br, UE=ue / n - 1.0, ASA=asa / n, br_hits=hits, br_total=total,
                ue_sum=ue, asa_sum=asa)
