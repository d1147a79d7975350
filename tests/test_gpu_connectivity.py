"""GPU connectivity post-processing (Algorithm 1, last step) through the C ABI
against the CPU oracle: bit-exact output ids and counts on the oracle EM's
labels, on fragment-heavy and checkerboard label maps, on hand-built cases, in
uneven batches; at 4K, the properties that hold at any size."""
import sys
import time

import numpy as np
import pytest
import torch
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import synth
from oracle import conn_oracle as C
from oracle import gmm_oracle as O
from paper_1612_08792_amd.gmmsp import GMMSP

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def run_gpu(dev, items, v):
    """items: list of (labels (H, W) ints, lab (H, W, 3) float32); grid spacing v."""
    sizes = [(l.shape[1], l.shape[0]) for l, _ in items]
    m = GMMSP(sizes, v=v, device=dev)
    labels = torch.from_numpy(np.concatenate([l.astype(np.int32).ravel() for l, _ in items])).to(dev)
    lab = torch.from_numpy(np.concatenate([x.astype(np.float32).reshape(-1) for _, x in items])).to(dev)
    out, counts = m.connectivity(lab, labels)
    out = out.cpu().numpy()
    res = [out[m.image_slice(b)].reshape(items[b][0].shape) for b in range(len(items))]
    return res, counts, m


def check_exact(dev, items, v):
    got, counts, m = run_gpu(dev, items, v)
    labels = torch.from_numpy(np.concatenate([l.astype(np.int32).ravel() for l, _ in items])).to(dev)
    lab = torch.from_numpy(np.concatenate([x.astype(np.float32).reshape(-1) for _, x in items])).to(dev)
    comp, _ = m.connectivity(lab, labels, compact=True)
    comp = comp.cpu().numpy()
    for b, (labels, lab) in enumerate(items):
        want, info = C.enforce_connectivity(labels, lab, v, v)
        assert np.array_equal(got[b], want), b
        assert list(counts[b]) == [info["segments"], info["small"], info["merged"], info["final"]], b
        # compact form: the rank of each final segment id in the image
        ranks = np.searchsorted(np.unique(want), want)
        assert np.array_equal(comp[m.image_slice(b)].reshape(want.shape), ranks), b
    return counts


def fragmented(seed, H, W, v, p=0.15):
    rng = np.random.default_rng(seed)
    labels = (np.arange(H)[:, None] // v) * 1000 + (np.arange(W)[None, :] // v)
    flip = rng.random((H, W)) < p
    labels = np.where(flip, labels + rng.integers(-1, 2, (H, W)), labels)
    lab = rng.normal(50, 12, (H, W, 3)).astype(np.float32)
    return labels, lab


def test_oracle_em_labels_481x321(dev):
    im = synth.config1_image()
    g = O.make_grid(im.W, im.H, K=im.K)
    ref = O.run_em(im.lab.numpy(), g, max_iters=10)
    labels = ref["labels"].reshape(im.H, im.W)
    counts = check_exact(dev, [(labels, im.lab.numpy())], g.vx)
    say("481x321 after T = 10: segments, small, merged, final =", list(counts[0]))


def test_fragmented_uneven_batch(dev):
    items = [fragmented(10, 97, 131, 9), fragmented(11, 40, 27, 9, 0.3), fragmented(12, 9, 9, 9, 0.5)]
    check_exact(dev, items, 9)


def small_cluster_sizes(labels, v):
    """Sizes (in segments) and pixel counts of the clusters of 4-adjacent small
    segments, from scipy's component labelling on the CPU."""
    from scipy import ndimage
    seg = np.full(labels.shape, -1, np.int64)
    n = 0
    for val in np.unique(labels):
        comp, k = ndimage.label(labels == val)
        seg[comp > 0] = comp[comp > 0] - 1 + n
        n += k
    size = np.bincount(seg.ravel(), minlength=n)
    small = 4 * size < v * v
    a = np.concatenate([seg[:, :-1].ravel(), seg[:-1, :].ravel()])
    b = np.concatenate([seg[:, 1:].ravel(), seg[1:, :].ravel()])
    keep = (a != b) & small[a] & small[b]
    g = coo_matrix((np.ones(keep.sum()), (a[keep], b[keep])), shape=(n, n))
    _, cl = connected_components(g, directed=False)
    members = np.bincount(cl[small])
    pixels = np.bincount(cl[small], weights=size[small])
    return members[members > 0], pixels[members > 0]


def test_large_clusters_bit_exact(dev):
    """Clusters of more than 16 small segments run one wave each with their
    state in LDS (up to 768 members and external neighbours, 2048 member
    pixels); larger ones on one lane with the state in memory.  Both against
    the oracle, bit for bit: two fragment fields (clusters of 17 to 695
    segments) and 25 adjacent 30 x 30 blocks under v = 64 (one cluster of 25
    segments and 22 500 pixels, too many pixels for LDS)."""
    frag = [fragmented(31, 200, 240, 16, 0.5), fragmented(34, 256, 256, 16, 0.55)]
    sizes = [small_cluster_sizes(l, 16) for l, _ in frag]
    members = np.concatenate([m for m, _ in sizes])
    pixels = np.concatenate([p for _, p in sizes])
    lds = (members > 16) & (members <= 768) & (pixels <= 2048)
    assert lds.sum() >= 100 and members[lds].max() >= 600, (lds.sum(), members.max())
    check_exact(dev, frag, 16)
    H = W = 150
    blocks = (np.arange(H)[:, None] // 30) * 10 + (np.arange(W)[None, :] // 30)
    m, p = small_cluster_sizes(blocks, 64)
    assert list(m) == [25] and p[0] == 22500
    rng = np.random.default_rng(5)
    check_exact(dev, [(blocks, rng.uniform(0, 100, (H, W, 3)).astype(np.float32))], 64)


def test_checkerboard_is_one_cluster(dev):
    # every pixel is its own segment, all small, all in one cluster
    H, W = 40, 48
    labels = (np.arange(H)[:, None] + np.arange(W)[None, :]) % 2
    rng = np.random.default_rng(13)
    lab = rng.uniform(0, 100, (H, W, 3)).astype(np.float32)
    counts = check_exact(dev, [(labels, lab)], 8)
    assert counts[0][0] == H * W


def serpentine(H, W, period=4):
    """A one-pixel path snaking over the whole image in a field of 0: rows
    y = 0 mod period are full, joined at alternating ends, so the path crosses
    every tile border many times and its union-find chains are long."""
    labels = np.zeros((H, W), np.int64)
    for y in range(0, H, period):
        labels[y, :] = 1
        if y + period < H:
            x = W - 1 if (y // period) % 2 == 0 else 0
            labels[y:y + period, x] = 1
    return labels


def test_long_components_across_tiles(dev):
    rng = np.random.default_rng(17)
    items = []
    for H, W in [(150, 200), (129, 65)]:
        items.append((serpentine(H, W), rng.uniform(0, 100, (H, W, 3)).astype(np.float32)))
    # one-pixel vertical stripes (each a segment crossing every tile row) and a staircase
    H, W = 140, 131
    items.append(((np.arange(W)[None, :] % 2).repeat(H, 0), rng.uniform(0, 100, (H, W, 3)).astype(np.float32)))
    H, W = 100, 100
    stair = ((np.arange(H)[:, None] + np.arange(W)[None, :]) // 3) % 2
    items.append((stair, rng.uniform(0, 100, (H, W, 3)).astype(np.float32)))
    check_exact(dev, items, 8)


def test_degenerate_shapes(dev):
    """Images one pixel wide or tall, a single pixel, and thin strips that cross
    the 64-pixel tile borders, in one uneven batch; the seed spacing (vx, vy) of
    each keeps its grid valid while single pixels still count as small."""
    rng = np.random.default_rng(19)
    cases = [((50, 1), (1, 8)), ((1, 70), (8, 1)), ((1, 1), (1, 1)), ((2, 130), (8, 2)),
             ((130, 2), (2, 8)), ((65, 65), (4, 4))]            # (H, W), (vx, vy)
    items = [(rng.integers(0, 3, hw), rng.uniform(0, 100, (*hw, 3)).astype(np.float32))
             for hw, _ in cases]
    m = GMMSP([(l.shape[1], l.shape[0]) for l, _ in items], v=[v for _, v in cases], device=dev)
    labels = torch.from_numpy(np.concatenate([l.astype(np.int32).ravel() for l, _ in items])).to(dev)
    lab = torch.from_numpy(np.concatenate([x.reshape(-1) for _, x in items])).to(dev)
    out, counts = m.connectivity(lab, labels)
    out = out.cpu().numpy()
    merged = 0
    for b, ((l, x), (_, (vx, vy))) in enumerate(zip(items, cases)):
        want, info = C.enforce_connectivity(l, x, vx, vy)
        assert np.array_equal(out[m.image_slice(b)].reshape(l.shape), want), b
        assert list(counts[b]) == [info["segments"], info["small"], info["merged"], info["final"]], b
        merged += info["merged"]
    assert merged > 0


def test_hand_cases(dev):
    # inherited neighbours: A joins B, B then joins Y through A's pixel
    labels = np.zeros((10, 10), np.int64)
    lab = np.zeros((10, 10, 3), np.float32)
    lab[..., 0] = 10.0
    labels[0, :] = 3
    lab[0, :, 0] = 51.0
    labels[1, 0] = 1
    lab[1, 0, 0] = 50.0
    labels[2:4, 0:3] = 2
    lab[2:4, 0:3, 0] = 50.2
    # equal distances: the smaller id wins
    l2 = np.zeros((8, 8), np.int64)
    l2[:, 4:] = 1
    l2[3, 3] = 2
    x2 = np.zeros((8, 8, 3), np.float32)
    x2[..., 0] = 40.0
    x2[:, 4:, 0] = 60.0
    x2[3, 3, 0] = 50.0
    check_exact(dev, [(labels, lab)], 6)
    check_exact(dev, [(l2, x2)], 4)
    # a single segment
    check_exact(dev, [(np.zeros((5, 7), np.int64), x2[:5, :7])], 5)


def components_of(values: np.ndarray):
    """Number of 4-connected components of equal value (scipy sparse graph)."""
    H, W = values.shape
    idx = np.arange(H * W).reshape(H, W)
    e1 = values[:, 1:] == values[:, :-1]
    e2 = values[1:, :] == values[:-1, :]
    rows = np.concatenate([idx[:, 1:][e1], idx[1:, :][e2]])
    cols = np.concatenate([idx[:, :-1][e1], idx[:-1, :][e2]])
    g = coo_matrix((np.ones(rows.size, np.int8), (rows, cols)), shape=(H * W, H * W))
    return connected_components(g, directed=False)[0]


def test_4k_gpu_labels_properties(dev):
    say("two 3840x2160 images of the 4K law: EM to rel-tol 1e-5, labels, connectivity")
    ims = synth.config5_batch(device=dev, n_images=2)
    lab = synth.pack_batch(ims).to(dev)
    m = GMMSP([(im.W, im.H) for im in ims], K=10000, device=dev)
    m.init_seeds(lab)
    m.em_iterate(lab, 200, 1e-5)
    labels, _ = m.label(lab)
    out, counts = m.connectivity(lab, labels)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out2, counts2 = m.connectivity(lab, labels)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert torch.equal(out, out2) and np.array_equal(counts, counts2)     # deterministic
    say("connectivity on 2 x 4K:", f"{dt * 1e3:.1f} ms;", "counts", counts.tolist())
    g = m.grids[0]
    lab_np = labels.cpu().numpy()
    out_np = out.cpu().numpy()
    for b in range(2):
        L = lab_np[m.image_slice(b)].reshape(2160, 3840)
        Oq = out_np[m.image_slice(b)].reshape(2160, 3840)
        assert counts[b][0] == components_of(L)
        vals, sizes = np.unique(Oq, return_counts=True)
        assert counts[b][3] == vals.size == components_of(Oq)             # every segment connected
        assert np.all(4 * sizes >= g.vx * g.vy)
        assert np.all(Oq.ravel()[vals] == vals)                           # ids are own pixels
        assert counts[b][2] == counts[b][0] - counts[b][3]
