"""Plain CPU oracle of the connectivity post-processing that ends the
superpixel algorithm (Algorithm 1, last step; the paragraph on enforcing
connectivity in Sec. III-C).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library.

What the paper fixes: the labelled superpixels may be disconnected; the
isolated pieces are sorted by size, ascending, and each piece smaller than a
quarter of the desired superpixel size is merged, in that order, into the
neighbouring superpixel closest to it in colour; the merged piece's size is
then zero and the destination's size grows by it.

Readings (the paper is silent on these; the HIP path follows the same ones):

* C-1 pieces ("segments") are the 4-connected components of equal label;
  every segment takes part, the main body of a superpixel included;
* C-2 a segment's id is the raster index y W + x of its first pixel in raster
  order; equal sizes sort by id;
* C-3 small means 4 size < v_x v_y (the desired size of Eq. vxy); the test
  uses the segment's current size when its turn comes, the order is fixed by
  the initial sizes;
* C-4 the colour of a segment is the mean Lab colour of its own pixels, fixed
  for the whole procedure (only sizes are updated), computed from the float32
  pixel values quantised to multiples of 2^-20 (exact integer sums), and the
  distance is the squared Euclidean distance in FP64, summed L, a, b in that
  order with no fused multiply-add;
* C-5 the neighbours of a segment are the segments, as merged so far, that
  contain a 4-neighbour of any pixel merged into it so far (its own pixels and
  those of the segments merged into it); the destination is the neighbour of
  smallest distance, ties to the smallest id; a segment with no neighbour
  stays;
* C-6 the output label of a pixel is the id of the segment it ends in (every
  output segment is connected).
"""
from __future__ import annotations

from collections import deque

import numpy as np

QUANT = 2.0 ** 20


def segments(labels: np.ndarray):
    """4-connected components of equal label (C-1), by breadth-first search in
    raster order.  Returns seg (H, W) holding each pixel's segment id (C-2) and
    the ids in increasing order."""
    H, W = labels.shape
    seg = np.full((H, W), -1, dtype=np.int64)
    ids = []
    for y0 in range(H):
        for x0 in range(W):
            if seg[y0, x0] >= 0:
                continue
            sid = y0 * W + x0
            ids.append(sid)
            lab = labels[y0, x0]
            seg[y0, x0] = sid
            q = deque([(y0, x0)])
            while q:
                y, x = q.popleft()
                for yy, xx in ((y - 1, x), (y + 1, x), (y, x - 1), (y, x + 1)):
                    if 0 <= yy < H and 0 <= xx < W and seg[yy, xx] < 0 and labels[yy, xx] == lab:
                        seg[yy, xx] = sid
                        q.append((yy, xx))
    return seg, ids


def segment_colours(lab: np.ndarray, seg: np.ndarray, ids):
    """Size and mean colour of every segment (C-4): integer sums of the
    quantised pixel colours, mean = sum / size / 2^20 in FP64."""
    q = np.rint(lab.astype(np.float64) * QUANT).astype(np.int64)
    size, col = {}, {}
    flat_seg = seg.ravel()
    flat_q = q.reshape(-1, 3)
    sums = {}
    for i in range(flat_seg.size):
        s = int(flat_seg[i])
        size[s] = size.get(s, 0) + 1
        t = sums.setdefault(s, [0, 0, 0])
        for c in range(3):
            t[c] += int(flat_q[i, c])
    for s in ids:
        col[s] = tuple(float(sums[s][c]) / float(size[s]) / QUANT for c in range(3))
    return size, col


def colour_dist2(a, b) -> float:
    """Squared Euclidean distance, L then a then b (C-4)."""
    dL = a[0] - b[0]
    da = a[1] - b[1]
    db = a[2] - b[2]
    return (dL * dL + da * da) + db * db


def enforce_connectivity(labels: np.ndarray, lab: np.ndarray, vx: int, vy: int):
    """The post-processing step, in the paper's order.  labels (H, W) ints,
    lab (H, W, 3) float32.  Returns (out (H, W) int64 segment ids, info)."""
    H, W = labels.shape
    seg, ids = segments(labels)
    size0, col = segment_colours(lab, seg, ids)
    pixels = {s: [] for s in ids}
    for y in range(H):
        for x in range(W):
            pixels[int(seg[y, x])].append((y, x))
    parent = {s: s for s in ids}

    def find(s):
        while parent[s] != s:
            s = parent[s]
        return s

    size = dict(size0)
    members = {s: [s] for s in ids}
    # the isolated superpixels that can be merged, ascending by size (C-2, C-3)
    order = sorted((s for s in ids if 4 * size0[s] < vx * vy), key=lambda s: (size0[s], s))
    merged = 0
    for s in order:
        if 4 * size[s] >= vx * vy:
            continue
        best, best_d = None, None
        for m in members[s]:
            for y, x in pixels[m]:
                for yy, xx in ((y - 1, x), (y + 1, x), (y, x - 1), (y, x + 1)):
                    if not (0 <= yy < H and 0 <= xx < W):
                        continue
                    t = find(int(seg[yy, xx]))
                    if t == s:
                        continue
                    d = colour_dist2(col[s], col[t])
                    if best is None or d < best_d or (d == best_d and t < best):
                        best, best_d = t, d
        if best is None:
            continue
        parent[s] = best
        size[best] += size[s]
        size[s] = 0
        members[best].extend(members[s])
        members[s] = []
        merged += 1
    out = np.empty((H, W), dtype=np.int64)
    for y in range(H):
        for x in range(W):
            out[y, x] = find(int(seg[y, x]))
    info = dict(segments=len(ids), small=len(order), merged=merged,
                final=len({find(s) for s in ids}))
    return out, info
