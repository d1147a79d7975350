// Connectivity post-processing (Algorithm 1, last step; the paragraph on
// enforcing connectivity in Sec. III-C) for a batch of label maps on gfx950.
//
// The paper sorts the isolated pieces of the superpixels by size, ascending,
// and merges each piece smaller than a quarter of the desired superpixel size,
// in that order, into the neighbouring superpixel closest in colour; a merged
// piece's size becomes zero and its destination's size grows by it.
//
// Definitions (pieces are "segments"):
//   * a segment is a 4-connected component of equal label; its id is the
//     raster index of its first pixel; small means 4 size < v_x v_y;
//   * colours are the segments' own mean Lab colours, fixed for the whole
//     procedure, from integer sums of the pixel colours quantised to 2^-20;
//   * the neighbours of a segment are the current segments holding a
//     4-neighbour of any pixel merged into it so far; the destination is the
//     one at the smallest squared colour distance (FP64, no fused
//     multiply-add), ties to the smallest id.
//
// Parallel form of the sequential procedure.  A small segment's decision
// reads only (a) its own size and pixels, which change only when small
// segments adjacent to it are merged into it, and (b) the current owner of
// each neighbouring pixel, which changes only for neighbouring small
// segments.  So the clusters of small segments joined by adjacency never
// influence each other: each cluster runs the procedure sequentially, in the
// global order restricted to it, on one thread, and all clusters run in
// parallel.  Merges into a large segment from several clusters only add to
// its size, which no decision reads (a large segment is never merged).
//
// Steps: pixel union-find of equal-label 4-neighbours, in 64 x 64 tiles in
// LDS and then across tile borders (roots are the minimum index, so the
// partition and ids are unique whatever the order of the atomics); ranks of
// the roots in raster order (segment indices, in id order); sizes and integer
// colour sums, gathered per block in LDS and added with integer atomics
// (exact); cluster union-find over adjacent small segments; per-cluster lists
// sorted by (size, id); per-source pixel lists; the sequential merge per
// cluster (one thread for small clusters, one wave for large ones); the
// output ids.
#include "gmmsp_internal.h"

#include <math.h>

namespace gmmsp {

namespace {

constexpr int kT = 256;
constexpr int kScanPer = 16;                // elements per thread of the scan
constexpr int kScanBlock = kScanPer * 256;  // elements per block of the scan

// loads and stores of state other threads update (device-coherent: served by
// the L2, never by a possibly stale L1 line)
__device__ __forceinline__ int ld_dev(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// root of x in a forest with parent[x] <= x (every link points to a smaller
// index, so the walk strictly decreases and ends)
__device__ int uf_find(int* par, int x) {
  int y = ld_dev(par + x);
  while (y != x) {
    x = y;
    y = ld_dev(par + x);
  }
  return x;
}

// join the sets of a and b by hanging the larger root under the smaller; a
// failed compare-and-swap returns the newer, strictly smaller parent, so the
// loop ends
__device__ void uf_unite(int* par, int a, int b) {
  a = uf_find(par, a);
  b = uf_find(par, b);
  while (a != b) {
    if (a < b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old = atomicCAS(par + a, a, b);
    if (old == a) return;
    a = uf_find(par, old);
    b = uf_find(par, b);
  }
}

__device__ __forceinline__ bool img_pixel(const ImgDesc* img, int& b, int& j, int& W, int& H,
                                          int64_t& off) {
  b = blockIdx.y;
  const ImgDesc I = img[b];
  W = I.W;
  H = I.H;
  off = I.pix_off;
  j = blockIdx.x * kT + threadIdx.x;
  return j < W * H;
}

__device__ __forceinline__ bool is_small(const ImgDesc* img, const int* seg_img,
                                         const int* size0, int s) {
  const ImgDesc& I = img[seg_img[s]];
  return 4LL * size0[s] < (int64_t)I.vx * I.vy;
}

__device__ double colour_dist2(const double* a, const double* b) {
#pragma clang fp contract(off)
  const double dL = a[0] - b[0];
  const double da = a[1] - b[1];
  const double db = a[2] - b[2];
  return (dL * dL + da * da) + db * db;
}

// merge parent walk: a segment points to the segment it was merged into
__device__ __forceinline__ int m_find(const int* mpar, int t) {
  int u = ld_dev(mpar + t);
  while (u != t) {
    t = u;
    u = ld_dev(mpar + t);
  }
  return t;
}

// ---- pixel components ------------------------------------------------------
// A block labels a 64 x 64 tile in LDS, one tile row per wave at a time:
// every pixel first points at the head of its horizontal run of equal label
// (found with a ballot), then each overlap of two equal runs on adjacent rows
// is joined once, by its first pixel (union-find with LDS atomics, roots the
// smallest tile-local raster index, which is also the smallest global index).
// The block writes each pixel's tile root as a global index and keeps the
// labels and roots of the tile's first and last columns in a side buffer; the
// tile borders are then joined in global memory from those and from the
// tiles' first rows.  Roots stay the minimum index of their set throughout.

constexpr int kTW = 64, kTH = 64;  // tile of the component labelling
constexpr int kSide = 4 * kTH;     // first-column labels, roots; last-column labels, roots
constexpr int kTileWaves = kT / 64;

__device__ int lds_find(int* lp, int x) {
  int y = __hip_atomic_load(lp + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  while (y != x) {
    x = y;
    y = __hip_atomic_load(lp + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  return x;
}

__device__ void lds_unite(int* lp, int a, int b) {
  a = lds_find(lp, a);
  b = lds_find(lp, b);
  while (a != b) {
    if (a < b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old = atomicCAS(lp + a, a, b);
    if (old == a) return;
    a = lds_find(lp, old);
    b = lds_find(lp, b);
  }
}

__global__ __launch_bounds__(kT) void k_cc_tile(const ImgDesc* img, const int32_t* labels,
                                                int* par, int* side, int max_tiles) {
  __shared__ int lp[kTW * kTH];
  __shared__ int32_t ll[kTW * kTH];
  const int b = blockIdx.y;
  const ImgDesc& I = img[b];
  const int W = I.W, H = I.H;
  const int tiles_x = (W + kTW - 1) / kTW, tiles_y = (H + kTH - 1) / kTH;
  if ((int)blockIdx.x >= tiles_x * tiles_y) return;  // the whole block
  const int x0 = (blockIdx.x % tiles_x) * kTW, y0 = (blockIdx.x / tiles_x) * kTH;
  const int64_t off = I.pix_off;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int x = x0 + lane;
  const bool xin = x < W;
  // labels and run heads (pixels outside the image are runs of their own);
  // the wave's rows are loaded first, so their loads are in flight together
  constexpr int kRows = kTH / kTileWaves;
  int32_t labs[kRows];
#pragma unroll
  for (int q = 0; q < kRows; ++q) {
    const int ty = wv + q * kTileWaves;
    labs[q] = xin && y0 + ty < H ? labels[off + (int64_t)(y0 + ty) * W + x] : 0;
  }
#pragma unroll
  for (int q = 0; q < kRows; ++q) {
    const int ty = wv + q * kTileWaves;
    const bool in = xin && y0 + ty < H;
    const int l = ty * kTW + lane;
    const int32_t lab = labs[q];
    ll[l] = lab;
    const int32_t left = __shfl_up(lab, 1, 64);
    const unsigned long long heads = __ballot(lane == 0 || left != lab || !in);
    const unsigned long long upto = heads & ((2ull << lane) - 1ull);  // bits 0..lane
    lp[l] = ty * kTW + 63 - __builtin_clzll(upto);
  }
  __syncthreads();
  // vertical joins: the first pixel of each overlap of equal runs
  for (int ty = 1 + wv; ty < kTH; ty += kTileWaves) {
    if (!xin || y0 + ty >= H) continue;
    const int l = ty * kTW + lane;
    const int32_t lab = ll[l];
    if (ll[l - kTW] != lab) continue;
    if (lane > 0 && ll[l - 1] == lab && ll[l - kTW - 1] == lab) continue;
    lds_unite(lp, l, l - kTW);
  }
  __syncthreads();
  int* sd = side + ((size_t)b * max_tiles + blockIdx.x) * kSide;
  const int xl = min(kTW, W - x0) - 1;  // the tile's last column
  for (int ty = wv; ty < kTH; ty += kTileWaves) {
    if (!xin || y0 + ty >= H) continue;
    const int l = ty * kTW + lane;
    const int r = lds_find(lp, l);
    const int g = (int)(off + (int64_t)(y0 + r / kTW) * W + x0 + r % kTW);
    par[off + (int64_t)(y0 + ty) * W + x] = g;
    if (lane == 0) {
      sd[ty] = ll[l];
      sd[kTH + ty] = g;
    }
    if (lane == xl) {
      sd[2 * kTH + ty] = ll[l];
      sd[3 * kTH + ty] = g;
    }
  }
}

// Joins across tile borders, one block per tile: wave 0 joins the tile's first
// row to the row above it, wave 1 its first column to the column on its left
// (from the side buffer).  As inside the tiles, only the first pixel of each
// overlap of equal runs along the border joins.
__global__ __launch_bounds__(128) void k_cc_border(const ImgDesc* img, const int32_t* labels,
                                                   int* par, const int* side, int max_tiles) {
  const int b = blockIdx.y;
  const ImgDesc& I = img[b];
  const int W = I.W, H = I.H;
  const int tiles_x = (W + kTW - 1) / kTW, tiles_y = (H + kTH - 1) / kTH;
  if ((int)blockIdx.x >= tiles_x * tiles_y) return;
  const int x0 = (blockIdx.x % tiles_x) * kTW, y0 = (blockIdx.x / tiles_x) * kTH;
  const int t = threadIdx.x & 63;
  int32_t a = 0, c = 0;
  int ra = 0, rc = 0;
  bool in;
  if (threadIdx.x < 64) {  // first row against the row above
    if (y0 == 0) return;
    in = x0 + t < W;
    const int64_t i = I.pix_off + (int64_t)y0 * W + x0 + t;
    if (in) {
      a = labels[i];
      c = labels[i - W];
      ra = ld_dev(par + i);
      rc = ld_dev(par + i - W);
    }
  } else {  // first column against the last column of the tile on the left
    if (x0 == 0) return;
    in = y0 + t < H;
    const int* me = side + ((size_t)b * max_tiles + blockIdx.x) * kSide;
    const int* lf = me - kSide;
    if (in) {
      a = me[t];
      ra = me[kTH + t];
      c = lf[2 * kTH + t];
      rc = lf[3 * kTH + t];
    }
  }
  const int32_t ap = __shfl_up(a, 1, 64), cp = __shfl_up(c, 1, 64);
  if (!in || a != c) return;
  if (t > 0 && ap == a && cp == a) return;  // joined through the previous pixel
  uf_unite(par, ra, rc);
}

// Segment numbering: the roots of the pixel forest (par[i] == i) in raster
// order.  Each block of kScanBlock pixels counts its roots and writes each
// root's rank within the block (at the root only); a root's segment index is
// that rank plus the exclusive scan of the block counts.
__global__ __launch_bounds__(kT) void k_root_rank(const int* par, int n, int* rank, int* bsum) {
  __shared__ int sh[kT];
  const int base = blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
  int v[kScanPer];
  if (base + kScanPer <= n) {  // par is 256-byte aligned: four 16-byte loads
#pragma unroll
    for (int k = 0; k < kScanPer / 4; ++k) {
      const int4 w = reinterpret_cast<const int4*>(par + base)[k];
      v[4 * k] = w.x == base + 4 * k;
      v[4 * k + 1] = w.y == base + 4 * k + 1;
      v[4 * k + 2] = w.z == base + 4 * k + 2;
      v[4 * k + 3] = w.w == base + 4 * k + 3;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) v[k] = base + k < n && par[base + k] == base + k;
  }
  int t = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) t += v[k];
  sh[threadIdx.x] = t;
  __syncthreads();
  for (int o = 1; o < kT; o <<= 1) {
    const int u = (int)threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += u;
    __syncthreads();
  }
  int run = sh[threadIdx.x] - t;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if (v[k]) rank[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == kT - 1) bsum[blockIdx.x] = sh[kT - 1];
}

// ---- exclusive scan of int32 (in place), total to *total ---------------------

__global__ __launch_bounds__(kT) void k_scan_blocks(int* a, int n, int* bsum) {
  __shared__ int sh[kT];
  const int base = blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
  int v[kScanPer];
  const bool whole = base + kScanPer <= n;
  if (whole) {  // a is 256-byte aligned: four 16-byte loads
#pragma unroll
    for (int k = 0; k < kScanPer / 4; ++k) {
      const int4 w = reinterpret_cast<const int4*>(a + base)[k];
      v[4 * k] = w.x;
      v[4 * k + 1] = w.y;
      v[4 * k + 2] = w.z;
      v[4 * k + 3] = w.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) v[k] = base + k < n ? a[base + k] : 0;
  }
  int t = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) t += v[k];
  sh[threadIdx.x] = t;
  __syncthreads();
  // Hillis-Steele inclusive scan of the per-thread totals
  for (int o = 1; o < kT; o <<= 1) {
    const int u = (int)threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += u;
    __syncthreads();
  }
  int run = sh[threadIdx.x] - t;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int e = run;
    run += v[k];
    v[k] = e;
  }
  if (whole) {
#pragma unroll
    for (int k = 0; k < kScanPer / 4; ++k)
      reinterpret_cast<int4*>(a + base)[k] = make_int4(v[4 * k], v[4 * k + 1], v[4 * k + 2],
                                                       v[4 * k + 3]);
  } else {
#pragma unroll
    for (int k = 0; k < kScanPer; ++k)
      if (base + k < n) a[base + k] = v[k];
  }
  if (threadIdx.x == kT - 1) bsum[blockIdx.x] = sh[kT - 1];
}

// one block: exclusive scan of the nb block totals, in chunks of kScanBlock
__global__ __launch_bounds__(kT) void k_scan_totals(int* bsum, int nb, int* total) {
  __shared__ int sh[kT];
  int carry = 0;
  for (int c0 = 0; c0 < nb; c0 += kScanBlock) {
    const int base = c0 + threadIdx.x * kScanPer;
    int v[kScanPer];
    int t = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      v[k] = base + k < nb ? bsum[base + k] : 0;
      t += v[k];
    }
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int o = 1; o < kT; o <<= 1) {
      const int u = (int)threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
      __syncthreads();
      sh[threadIdx.x] += u;
      __syncthreads();
    }
    int run = carry + sh[threadIdx.x] - t;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      if (base + k < nb) bsum[base + k] = run;
      run += v[k];
    }
    carry += sh[kT - 1];
    __syncthreads();  // sh is rewritten by the next chunk
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kT) void k_scan_add(int* a, int n, const int* bsum) {
  const int add = bsum[blockIdx.x];
  // consecutive threads on consecutive elements
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int i = blockIdx.x * kScanBlock + k * kT + threadIdx.x;
    if (i < n) a[i] += add;
  }
}

// ---- segments ---------------------------------------------------------------

__global__ __launch_bounds__(kT) void k_seg_zero(int n_seg, int* size0,
                                                 unsigned long long* colsum, int* ccnt) {
  const int s = blockIdx.x * kT + threadIdx.x;
  if (s >= n_seg) return;
  size0[s] = 0;
  colsum[3 * s] = 0ull;
  colsum[3 * s + 1] = 0ull;
  colsum[3 * s + 2] = 0ull;
  ccnt[s] = 0;
}

// Segment of each pixel, segment roots, and the sizes and integer colour sums
// (exact, so the order of the additions does not matter).  A block covers a
// 64 x 16 tile, one row of 64 pixels per wave at a time: each run of equal
// segment in the row is summed across its lanes, the run totals are gathered
// per segment in an LDS table, and the block adds each table entry to the
// segment once.  Entries that do not fit the table go to memory directly.
constexpr int kSW = 64, kSH = 16;  // tile of the segment statistics
constexpr int kHash = 128;         // LDS table entries (a power of two)

__device__ __forceinline__ void add_stats(int s, int cnt, const long long (&q)[3], int* size0,
                                          unsigned long long* colsum) {
  atomicAdd(size0 + s, cnt);
#pragma unroll
  for (int c = 0; c < 3; ++c) atomicAdd(colsum + 3 * s + c, (unsigned long long)q[c]);
}

__global__ __launch_bounds__(kT) void k_seg_assign(const ImgDesc* img, const float* lab,
                                                   const int* par, const int* rank,
                                                   const int* boff, int* segid,
                                                   int* seg_root, int* seg_img, int* size0,
                                                   unsigned long long* colsum) {
  __shared__ int hkey[kHash];
  __shared__ int hcnt[kHash];
  __shared__ unsigned long long hsum[3][kHash];
  const int b = blockIdx.y;
  const ImgDesc& I = img[b];
  const int W = I.W, H = I.H;
  const int tiles_x = (W + kSW - 1) / kSW;
  if ((int)blockIdx.x >= tiles_x * ((H + kSH - 1) / kSH)) return;  // the whole block
  for (int e = threadIdx.x; e < kHash; e += kT) {
    hkey[e] = -1;
    hcnt[e] = 0;
    hsum[0][e] = hsum[1][e] = hsum[2][e] = 0ull;
  }
  __syncthreads();
  const int x0 = (blockIdx.x % tiles_x) * kSW, y0 = (blockIdx.x / tiles_x) * kSH;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const bool xin = x0 + lane < W;
  // the wave's rows: loads first (colours, parents), then the roots and the
  // segment indices, each step's loads in flight together
  constexpr int kRows = kSH / kTileWaves;
  int pi[kRows], pr[kRows], ps[kRows];
  float pc[kRows][3];
#pragma unroll
  for (int u = 0; u < kRows; ++u) {
    const int ty = wv + u * kTileWaves;
    const bool in = xin && y0 + ty < H;
    pi[u] = in ? (int)(I.pix_off + (int64_t)(y0 + ty) * W + x0 + lane) : -1;
    pr[u] = in ? par[pi[u]] : 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) pc[u][c] = in ? lab[3 * (int64_t)pi[u] + c] : 0.f;
  }
#pragma unroll
  for (int u = 0; u < kRows; ++u) {
    if (pi[u] < 0) continue;
    int y = par[pr[u]];
    while (y != pr[u]) {
      pr[u] = y;
      y = par[y];
    }
  }
#pragma unroll
  for (int u = 0; u < kRows; ++u) ps[u] = pi[u] >= 0 ? rank[pr[u]] + boff[pr[u] / kScanBlock] : -1;
#pragma unroll
  for (int u = 0; u < kRows; ++u) {
    const bool in = pi[u] >= 0;
    const int s = ps[u];
    int cnt = 0;
    long long q[3] = {0, 0, 0};
    if (in) {
      const int i = pi[u];
      segid[i] = s;
      if (pr[u] == i) {
        seg_root[s] = i;
        seg_img[s] = b;
      }
      cnt = 1;
#pragma unroll
      for (int c = 0; c < 3; ++c) q[c] = (long long)rint((double)pc[u][c] * 1048576.0);
    }
    // runs of equal segment: the head lane of each, then sums within runs
    const int sl = __shfl_up(s, 1, 64);
    const unsigned long long heads = __ballot(lane == 0 || sl != s);
    const int hp = 63 - __builtin_clzll(heads & ((2ull << lane) - 1ull));
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int c0 = __shfl_up(cnt, o, 64);
      const long long a0 = __shfl_up(q[0], o, 64), a1 = __shfl_up(q[1], o, 64),
                      a2 = __shfl_up(q[2], o, 64);
      if (lane - o >= hp) {
        cnt += c0;
        q[0] += a0;
        q[1] += a1;
        q[2] += a2;
      }
    }
    const bool last = lane == 63 || ((heads >> (lane + 1)) & 1ull);
    if (!in || !last) continue;
    // the run's totals into the table (open addressing, linear probing)
    const int h0 = (int)(((unsigned)s * 2654435761u) >> 25);  // top 7 bits: 0 .. kHash - 1
    bool done = false;
    for (int p = 0; p < kHash && !done; ++p) {
      const int e = (h0 + p) & (kHash - 1);
      const int k = atomicCAS(hkey + e, -1, s);
      if (k == -1 || k == s) {
        atomicAdd(hcnt + e, cnt);
#pragma unroll
        for (int c = 0; c < 3; ++c) atomicAdd(&hsum[c][e], (unsigned long long)q[c]);
        done = true;
      }
    }
    if (!done) add_stats(s, cnt, q, size0, colsum);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kHash; e += kT) {
    const int k = hkey[e];
    if (k < 0) continue;
    const long long q[3] = {(long long)hsum[0][e], (long long)hsum[1][e], (long long)hsum[2][e]};
    add_stats(k, hcnt[e], q, size0, colsum);
  }
}

// means (in place of the sums), working sizes, parents, chains; the cluster
// parent of a large segment is -1, which marks it large from here on
__global__ __launch_bounds__(kT) void k_seg_prep(const ImgDesc* img, int n_seg,
                                                 const int* seg_img, const int* size0,
                                                 unsigned long long* colsum, int* size,
                                                 int* mpar, int* cpar, int* next, int* tail) {
  const int s = blockIdx.x * kT + threadIdx.x;
  if (s >= n_seg) return;
  const int n = size0[s];
  double* mean = reinterpret_cast<double*>(colsum + 3 * s);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const long long q = (long long)colsum[3 * s + c];
    mean[c] = (double)q / (double)n * 0x1p-20;
  }
  size[s] = n;
  mpar[s] = s;
  cpar[s] = is_small(img, seg_img, size0, s) ? s : -1;
  next[s] = -1;
  tail[s] = s;
}

// clusters: union of 4-adjacent small segments
// (a small segment's cluster parent is never negative, a large one's is -1)
__global__ __launch_bounds__(kT) void k_cl_link(const ImgDesc* img, const int* segid, int* cpar) {
  int b, j, W, H;
  int64_t off;
  if (!img_pixel(img, b, j, W, H, off)) return;
  const int i = (int)(off + j);
  const int s = segid[i];
  const int x = j % W, y = j / W;
  const int tl = x > 0 ? segid[i - 1] : s, tu = y > 0 ? segid[i - W] : s;
  if ((tl == s && tu == s) || cpar[s] < 0) return;
  if (tl != s && cpar[tl] >= 0) uf_unite(cpar, s, tl);
  if (tu != s && cpar[tu] >= 0) uf_unite(cpar, s, tu);
}

__global__ __launch_bounds__(kT) void k_cl_count(int n_seg, int* cpar, int* ccnt) {
  const int s = blockIdx.x * kT + threadIdx.x;
  if (s >= n_seg || cpar[s] < 0) return;
  const int r = uf_find(cpar, s);
  cpar[s] = r;
  atomicAdd(ccnt + r, 1);
}

// cluster lists (any order) and the sources' pixel-list sizes
__global__ __launch_bounds__(kT) void k_cl_fill(int n_seg, const int* size0, const int* cpar,
                                                const int* coff, int* cursor, int* list,
                                                int* psz) {
  const int s = blockIdx.x * kT + threadIdx.x;
  if (s >= n_seg) return;
  const bool small = cpar[s] >= 0;
  psz[s] = small ? size0[s] : 0;
  if (!small) return;
  const int r = cpar[s];
  const int pos = atomicAdd(cursor + r, 1);
  list[coff[r] + pos] = s;
}

__global__ __launch_bounds__(kT) void k_zero(int n, int* a) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i < n) a[i] = 0;
}

__global__ __launch_bounds__(kT) void k_px_fill(const ImgDesc* img, const int* segid,
                                                const int* cpar, const int* poff, int* cursor,
                                                int* plist) {
  int b, j, W, H;
  int64_t off;
  if (!img_pixel(img, b, j, W, H, off)) return;
  const int i = (int)(off + j);
  const int s = segid[i];
  if (cpar[s] < 0) return;
  plist[poff[s] + atomicAdd(cursor + s, 1)] = i;
}

__device__ __forceinline__ bool key_less(const int* size0, int a, int b) {
  return size0[a] < size0[b] || (size0[a] == size0[b] && a < b);
}

__device__ void sift_down(int* v, const int* size0, int root, int n) {
  while (true) {
    int c = 2 * root + 1;
    if (c >= n) return;
    if (c + 1 < n && key_less(size0, v[c], v[c + 1])) ++c;
    if (!key_less(size0, v[root], v[c])) return;
    const int t = v[root];
    v[root] = v[c];
    v[c] = t;
    root = c;
  }
}

// The colour-nearest neighbour among the 4-neighbours of pixel j (image-local
// index) for segment s: updates (best, bd); ties to the smaller id.
__device__ __forceinline__ void scan_pixel(int j, int W, int H, int off, int s, const double* ms,
                                           const int* segid, const int* mpar, const double* mean,
                                           int& best, double& bd) {
  const int x = j % W, y = j / W;
  int nb[4];
  int k = 0;
  if (y > 0) nb[k++] = j - W;
  if (y + 1 < H) nb[k++] = j + W;
  if (x > 0) nb[k++] = j - 1;
  if (x + 1 < W) nb[k++] = j + 1;
  for (int e = 0; e < k; ++e) {
    const int t = m_find(mpar, segid[off + nb[e]]);
    if (t == s) continue;
    const double d = colour_dist2(ms, mean + 3 * (int64_t)t);
    if (best < 0 || d < bd || (d == bd && t < best)) {
      best = t;
      bd = d;
    }
  }
}

// merge s into best: size transfer and, inside the cluster, the hand-over of
// the member chain
__device__ __forceinline__ void merge_into(const ImgDesc* img, const int* seg_img, const int* size0,
                                           int s, int best, int* size, int* mpar, int* next,
                                           int* tail) {
  st_dev(mpar + s, best);
  atomicAdd(size + best, ld_dev(size + s));  // a large destination is shared by clusters
  st_dev(size + s, 0);
  if (is_small(img, seg_img, size0, best)) {
    st_dev(next + ld_dev(tail + best), s);
    st_dev(tail + best, ld_dev(tail + s));
  }
}

// The procedure on one cluster, one thread: heap sort of its sources by
// (size, id), then the visits in that order.
__device__ void merge_cluster(const ImgDesc* img, int r, const int* seg_img, const int* size0,
                              const int* ccnt, const int* coff, int* list, const int* poff,
                              const int* plist, const int* segid, const double* mean, int* size,
                              int* mpar, int* next, int* tail) {
  const int n = ccnt[r];
  int* v = list + coff[r];
  for (int k = n / 2 - 1; k >= 0; --k) sift_down(v, size0, k, n);
  for (int e = n - 1; e > 0; --e) {
    const int t = v[0];
    v[0] = v[e];
    v[e] = t;
    sift_down(v, size0, 0, e);
  }
  const ImgDesc& I = img[seg_img[r]];
  const int W = I.W, H = I.H;
  const int off = (int)I.pix_off;
  const int64_t desired = (int64_t)I.vx * I.vy;
  for (int q = 0; q < n; ++q) {
    const int s = v[q];
    if (4LL * ld_dev(size + s) >= desired) continue;
    const double* ms = mean + 3 * (int64_t)s;
    int best = -1;
    double bd = 0.0;
    for (int m = s; m >= 0; m = ld_dev(next + m)) {
      const int p0 = poff[m], np = size0[m];
      for (int u = 0; u < np; ++u)
        scan_pixel(plist[p0 + u] - off, W, H, off, s, ms, segid, mpar, mean, best, bd);
    }
    if (best >= 0) merge_into(img, seg_img, size0, s, best, size, mpar, next, tail);
  }
}

// clusters of at most kBig sources run here, one thread each; larger ones are
// listed for k_merge_big
constexpr int kBig = 16;

__global__ __launch_bounds__(kT) void k_merge(const ImgDesc* img, int n_seg, const int* seg_img,
                                              const int* size0, const int* cpar, const int* ccnt,
                                              const int* coff, int* list, const int* poff,
                                              const int* plist, const int* segid,
                                              const double* mean, int* size, int* mpar, int* next,
                                              int* tail, int* big, int* n_big) {
  const int r = blockIdx.x * kT + threadIdx.x;
  if (r >= n_seg || cpar[r] != r) return;  // cluster roots only (a large segment's is -1)
  if (ccnt[r] > kBig) {
    big[atomicAdd(n_big, 1)] = r;
    return;
  }
  merge_cluster(img, r, seg_img, size0, ccnt, coff, list, poff, plist, segid, mean, size, mpar,
                next, tail);
}

// Large clusters, one wave each, with the cluster's whole merge state in LDS.
// The sources are sorted by (size, id) with a bitonic sort; each source gets a
// local index in that order, and so does every large segment adjacent to the
// cluster (its "external" neighbours), through an LDS table from segment id to
// local index.  Before the first visit the wave records, for every pixel of
// every source, the local indices of the segments holding its 4-neighbours
// (4 entries per pixel); a visit then reads only LDS: the member chain of the
// source, the entries of the members' pixels, the current owner of each entry
// (merge-parent walk), the colour means of the source and the owners.  The
// owner set of a visit is exactly the set of current owners of the 4-neighbours
// of every pixel merged into the source, so the decision is the one of the
// sequential procedure.  A cluster that does not fit (members and externals,
// or neighbour entries) runs on one lane with the state in memory.
constexpr int kLCap = 768;     // members + external neighbours held in LDS
constexpr int kLSort = 1024;   // bitonic sort width (power of two >= kLCap)
constexpr int kLAdj = 8192;    // neighbour entries: 4 per member pixel
constexpr int kLHash = 2048;   // segment id -> local index table
constexpr int kLWaves = 2;     // waves (clusters) per block
constexpr unsigned short kNone = 0xFFFF;

struct ClusterLds {
  unsigned long long key[kLSort];
  double mean[kLCap][3];
  int gid[kLCap];                // segment id of each local index
  int sz[kLCap];                 // current size of each member
  int pref[kLCap + 1];           // first pixel of each member, in member order
  int cum[kLCap + 1];            // entry offsets along the chain of a visit
  int hkey[kLHash];
  short hval[kLHash];
  short mp[kLCap], nx[kLCap], tl[kLCap], chain[kLCap];
  unsigned short adj[kLAdj];
  int n_ext, overflow, n_chain;
};

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int hash_slot(int id) {
  return (int)(((unsigned)id * 2654435761u) >> 21) & (kLHash - 1);
}

// local index of segment t, inserting it as an external neighbour when new
__device__ int lds_index(ClusterLds& S, int t) {
  int e = hash_slot(t);
  for (int probe = 0; probe < kLHash; ++probe, e = (e + 1) & (kLHash - 1)) {
    const int k = atomicCAS(&S.hkey[e], -1, t);
    if (k == -1) {  // this lane inserted t: a new external slot
      const int slot = atomicAdd(&S.n_ext, 1);
      S.hval[e] = (short)(slot < kLCap ? slot : -1);
      if (slot < kLCap) S.gid[slot] = t;
      else S.overflow = 1;
    }
    if (k == -1 || k == t) return e;  // the value is read once every lane has stored
  }
  S.overflow = 1;
  return -1;
}

__device__ __forceinline__ int lds_owner(const ClusterLds& S, int n, int x) {
  while (x < n && S.mp[x] != x) x = S.mp[x];
  return x;
}

__global__ __launch_bounds__(64 * kLWaves) void k_merge_big(
    const ImgDesc* img, const int* seg_img, const int* size0, const int* ccnt, const int* coff,
    int* list, const int* poff, const int* plist, const int* segid, const double* mean, int* size,
    int* mpar, int* next, int* tail, const int* big, const int* n_big) {
  __shared__ ClusterLds lds[kLWaves];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  ClusterLds& S = lds[wv];
  const int nbig = *n_big;
  for (int c = blockIdx.x * kLWaves + wv; c < nbig; c += gridDim.x * kLWaves) {
    const int r = big[c];
    const int n = ccnt[r];
    const int* v = list + coff[r];
    const ImgDesc& I = img[seg_img[r]];
    const int W = I.W, H = I.H;
    const int off = (int)I.pix_off;
    const int64_t desired = (int64_t)I.vx * I.vy;
    bool fits = n <= kLCap;
    if (fits) {
      // sort the sources by (size, id)
      int P = 1;
      while (P < n) P <<= 1;
      for (int i = lane; i < P; i += 64)
        S.key[i] = i < n ? ((unsigned long long)size0[v[i]] << 32) | (unsigned)v[i] : ~0ull;
      for (int e = lane; e < kLHash; e += 64) {
        S.hkey[e] = -1;
        S.hval[e] = -1;
      }
      if (lane == 0) {
        S.n_ext = n;
        S.overflow = 0;
      }
      wave_sync_lds();
      for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
          for (int i = lane; i < P; i += 64) {
            const int l = i ^ j;
            if (l > i) {
              const unsigned long long a = S.key[i], b = S.key[l];
              if ((a > b) == ((i & k) == 0)) {
                S.key[i] = b;
                S.key[l] = a;
              }
            }
          }
          wave_sync_lds();
        }
      }
      // members: ids, sizes, chains, means, table entries
      for (int q = lane; q < n; q += 64) {
        const int g = (int)(unsigned)(S.key[q] & 0xFFFFFFFFull);
        S.gid[q] = g;
        S.sz[q] = size0[g];
        S.mp[q] = (short)q;
        S.nx[q] = -1;
        S.tl[q] = (short)q;
        int e = hash_slot(g);
        while (atomicCAS(&S.hkey[e], -1, g) != -1) e = (e + 1) & (kLHash - 1);
        S.hval[e] = (short)q;
      }
      // first pixel of each member: per-lane chunk sums, then a wave scan
      const int chunk = (n + 63) / 64;
      const int q0 = min(n, lane * chunk), q1 = min(n, q0 + chunk);
      int part = 0;
      for (int q = q0; q < q1; ++q) part += size0[(int)(unsigned)(S.key[q] & 0xFFFFFFFFull)];
      int incl = part;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
      }
      int run = incl - part;
      for (int q = q0; q < q1; ++q) {
        S.pref[q] = run;
        run += size0[(int)(unsigned)(S.key[q] & 0xFFFFFFFFull)];
      }
      const int total = __shfl(incl, 63, 64);
      if (lane == 0) S.pref[n] = total;
      wave_sync_lds();
      fits = 4 * total <= kLAdj;
    }
    if (fits) {
      // the 4-neighbour entries of every member pixel (up, down, left, right)
      const int total = S.pref[n];
      for (int u = lane; u < total; u += 64) {
        int lo = 0, hi = n;  // the member q with pref[q] <= u < pref[q + 1]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (S.pref[mid] <= u) lo = mid;
          else hi = mid;
        }
        const int g = S.gid[lo];
        const int j = plist[poff[g] + (u - S.pref[lo])] - off;
        const int x = j % W, y = j / W;
        int t[4];
        t[0] = y > 0 ? segid[off + j - W] : g;
        t[1] = y + 1 < H ? segid[off + j + W] : g;
        t[2] = x > 0 ? segid[off + j - 1] : g;
        t[3] = x + 1 < W ? segid[off + j + 1] : g;
        int e[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) e[k] = t[k] != g ? lds_index(S, t[k]) : -1;
        wave_sync_lds();  // every inserting lane has stored its value
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int idx = e[k] >= 0 ? S.hval[e[k]] : -1;
          S.adj[4 * u + k] = idx >= 0 ? (unsigned short)idx : kNone;
        }
      }
      wave_sync_lds();
      // colour means of the members and the external neighbours
      const int nl = min(S.n_ext, kLCap);
      for (int i = lane; i < nl; i += 64) {
        const double* m = mean + 3 * (int64_t)S.gid[i];
        S.mean[i][0] = m[0];
        S.mean[i][1] = m[1];
        S.mean[i][2] = m[2];
      }
      wave_sync_lds();
      fits = S.overflow == 0;
    }
    if (!fits) {  // the state in memory, one lane
      if (lane == 0)
        merge_cluster(img, r, seg_img, size0, ccnt, coff, list, poff, plist, segid, mean, size,
                      mpar, next, tail);
      continue;
    }
    // the visits, in (size, id) order
    for (int q = 0; q < n; ++q) {
      if (4LL * S.sz[q] >= desired) continue;
      if (lane == 0) {  // the members merged into q so far, and their entry offsets
        int nc = 0, acc = 0;
        for (int m = q; m >= 0; m = S.nx[m]) {
          S.chain[nc] = (short)m;
          S.cum[nc] = acc;
          acc += 4 * (S.pref[m + 1] - S.pref[m]);
          ++nc;
        }
        S.cum[nc] = acc;
        S.n_chain = nc;
      }
      wave_sync_lds();
      const int nc = S.n_chain, T = S.cum[nc];
      const double ms[3] = {S.mean[q][0], S.mean[q][1], S.mean[q][2]};
      int best = -1, bidx = -1;
      double bd = 0.0;
      for (int u = lane; u < T; u += 64) {
        int lo = 0, hi = nc;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (S.cum[mid] <= u) lo = mid;
          else hi = mid;
        }
        const int m = S.chain[lo];
        const unsigned short a = S.adj[4 * S.pref[m] + (u - S.cum[lo])];
        if (a == kNone) continue;
        const int o = lds_owner(S, n, a);
        if (o == q) continue;
        const double d = colour_dist2(ms, S.mean[o]);
        const int go = S.gid[o];
        if (best < 0 || d < bd || (d == bd && go < best)) {
          best = go;
          bidx = o;
          bd = d;
        }
      }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const double od = __shfl_xor(bd, o, 64);
        const int ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bidx, o, 64);
        if (ob >= 0 && (best < 0 || od < bd || (od == bd && ob < best))) {
          best = ob;
          bidx = oi;
          bd = od;
        }
      }
      if (best < 0) continue;  // every lane holds the same result
      if (lane == 0) {
        S.mp[q] = (short)bidx;
        if (bidx < n) {  // into a member: size and member chain move over
          S.sz[bidx] += S.sz[q];
          S.nx[S.tl[bidx]] = (short)q;
          S.tl[bidx] = S.tl[q];
        }
        S.sz[q] = 0;
      }
      wave_sync_lds();
    }
    // merge parents back to memory, as segment ids (a large destination's size
    // is read by no decision and no output)
    for (int q = lane; q < n; q += 64) mpar[S.gid[q]] = S.gid[S.mp[q]];
    wave_sync_lds();  // the table and arrays are rewritten by the next cluster
  }
}

__global__ __launch_bounds__(kT) void k_root_flags(int n_seg, const int* mpar, int* flag) {
  const int s = blockIdx.x * kT + threadIdx.x;
  if (s < n_seg) flag[s] = mpar[s] == s;
}

// output value of each segment: the id of its final segment (compact = 0),
// or the rank of that segment among the image's final segments in id order
// (compact = 1; rank = final roots before it in the batch minus those before
// the image's first segment)
__global__ __launch_bounds__(kT) void k_seg_out(const ImgDesc* img, int n_seg, const int* seg_img,
                                                const int* segid, const int* mpar,
                                                const int* seg_root, const int* rank, int compact,
                                                int* val) {
  const int s = blockIdx.x * kT + threadIdx.x;
  if (s >= n_seg) return;
  const int t = m_find(mpar, s);
  const int64_t off = img[seg_img[s]].pix_off;
  val[s] = compact ? rank[t] - rank[segid[off]] : (int)(seg_root[t] - off);
}

__global__ __launch_bounds__(kT) void k_final(const ImgDesc* img, const int* segid,
                                              const int* val, int32_t* out) {
  int b, j, W, H;
  int64_t off;
  if (!img_pixel(img, b, j, W, H, off)) return;
  const int i = (int)(off + j);
  out[i] = val[segid[i]];
}

// per-image counts of small and merged segments: each block sums its
// segments per image in LDS (a block's 256 consecutive segments span few
// images) and adds each image's sums with one atomic per counter; the segment
// count per image comes from the image's first segment index
__global__ __launch_bounds__(kT) void k_counts(const ImgDesc* img, int n_seg, const int* seg_img,
                                               const int* size0, const int* mpar, int* counts) {
  __shared__ int sb[kT], sc[kT][2];
  const int s = blockIdx.x * kT + threadIdx.x;
  const bool valid = s < n_seg;
  sb[threadIdx.x] = valid ? seg_img[s] : -1;
  sc[threadIdx.x][0] = valid && is_small(img, seg_img, size0, s);
  sc[threadIdx.x][1] = valid && mpar[s] != s;
  __syncthreads();
  const int b = sb[threadIdx.x];
  // the first thread of each run of equal image sums the run and adds it
  if (b < 0 || (threadIdx.x > 0 && sb[threadIdx.x - 1] == b)) return;
  int c0 = 0, c1 = 0, c2 = 0;
  for (int t = threadIdx.x; t < kT && sb[t] == b; ++t) {
    ++c0;
    c1 += sc[t][0];
    c2 += sc[t][1];
  }
  atomicAdd(counts + 4 * b + 0, c0);
  atomicAdd(counts + 4 * b + 1, c1);
  atomicAdd(counts + 4 * b + 2, c2);
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

hipError_t scan(int* a, int n, int* bsum, int* total, hipStream_t s) {
  const int nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb > 0) hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(kT), 0, s, a, n, bsum);
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kT), 0, s, bsum, nb, total);
  if (nb > 0) hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kT), 0, s, a, n, bsum);
  return hipGetLastError();
}

}  // namespace

size_t conn_scan_blocks(int64_t n) { return (size_t)((n + kScanBlock - 1) / kScanBlock); }

size_t conn_tiles(int W, int H) {
  return (size_t)((W + kTW - 1) / kTW) * (size_t)((H + kTH - 1) / kTH);
}

size_t conn_side_ints(int n_img, int max_tiles) { return (size_t)n_img * max_tiles * kSide; }

hipError_t conn_launch_components(const ConnPtrs& C, const ImgDesc* img, int n_img,
                                  int max_pixels, int max_tiles, const int32_t* labels,
                                  hipStream_t s) {
  (void)max_pixels;
  hipLaunchKernelGGL(k_cc_tile, dim3(max_tiles, n_img), dim3(kT), 0, s, img, labels, C.par,
                     C.side, max_tiles);
  hipLaunchKernelGGL(k_cc_border, dim3(max_tiles, n_img), dim3(128), 0, s, img, labels, C.par,
                     C.side, max_tiles);
  // roots in raster order: ranks within blocks, then the scan of the block counts
  const int n = (int)C.n_pix;
  const int nb = (n + kScanBlock - 1) / kScanBlock;
  hipLaunchKernelGGL(k_root_rank, dim3(nb), dim3(kT), 0, s, C.par, n, C.scan, C.bsum);
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kT), 0, s, C.bsum, nb, C.total);
  return hipGetLastError();
}

hipError_t conn_launch_merge(const ConnPtrs& C, const ImgDesc* img, int n_img, int max_pixels,
                             int max_w, int max_h, int n_seg, const float* lab, int compact,
                             int32_t* out, hipStream_t s) {
  const dim3 g(blocks(max_pixels), n_img);
  const unsigned max_stat_tiles = (unsigned)(((max_w + kSW - 1) / kSW) * ((max_h + kSH - 1) / kSH));
  const unsigned gs = blocks(n_seg);
  hipLaunchKernelGGL(k_seg_zero, dim3(gs), dim3(kT), 0, s, n_seg, C.size0, C.colsum, C.ccnt);
  // (bsum still holds the block offsets of the root ranks here)
  hipLaunchKernelGGL(k_seg_assign, dim3(max_stat_tiles, n_img), dim3(kT), 0, s, img, lab, C.par,
                     C.scan, C.bsum, C.segid, C.seg_root, C.seg_img, C.size0, C.colsum);
  hipLaunchKernelGGL(k_seg_prep, dim3(gs), dim3(kT), 0, s, img, n_seg, C.seg_img, C.size0,
                     C.colsum, C.size, C.mpar, C.cpar, C.next, C.tail);
  hipLaunchKernelGGL(k_cl_link, g, dim3(kT), 0, s, img, C.segid, C.cpar);
  hipLaunchKernelGGL(k_cl_count, dim3(gs), dim3(kT), 0, s, n_seg, C.cpar, C.ccnt);
  hipError_t e = hipMemcpyAsync(C.coff, C.ccnt, sizeof(int) * (size_t)n_seg,
                                hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  e = scan(C.coff, n_seg, C.bsum, C.total, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_zero, dim3(gs), dim3(kT), 0, s, n_seg, C.cursor);
  hipLaunchKernelGGL(k_cl_fill, dim3(gs), dim3(kT), 0, s, n_seg, C.size0, C.cpar, C.coff,
                     C.cursor, C.list, C.poff);
  e = scan(C.poff, n_seg, C.bsum, C.total, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_zero, dim3(gs), dim3(kT), 0, s, n_seg, C.cursor);
  // the pixel union-find array is free now: it holds the sources' pixel lists
  hipLaunchKernelGGL(k_px_fill, g, dim3(kT), 0, s, img, C.segid, C.cpar, C.poff, C.cursor,
                     C.par);
  // the root-rank array is free until the final ranks: it lists the large clusters
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(kT), 0, s, 1, C.n_big);
  hipLaunchKernelGGL(k_merge, dim3(gs), dim3(kT), 0, s, img, n_seg, C.seg_img, C.size0, C.cpar,
                     C.ccnt, C.coff, C.list, C.poff, C.par, C.segid,
                     reinterpret_cast<const double*>(C.colsum), C.size, C.mpar, C.next, C.tail,
                     C.scan, C.n_big);
  hipLaunchKernelGGL(k_merge_big, dim3(1024), dim3(64 * kLWaves), 0, s, img, C.seg_img,
                     C.size0, C.ccnt, C.coff, C.list, C.poff, C.par, C.segid,
                     reinterpret_cast<const double*>(C.colsum), C.size, C.mpar, C.next, C.tail,
                     C.scan, C.n_big);
  // final segments ranked in id order; each segment's output value (into the
  // working sizes, no longer needed); the output
  hipLaunchKernelGGL(k_root_flags, dim3(gs), dim3(kT), 0, s, n_seg, C.mpar, C.scan);
  e = scan(C.scan, n_seg, C.bsum, C.total, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_seg_out, dim3(gs), dim3(kT), 0, s, img, n_seg, C.seg_img, C.segid, C.mpar,
                     C.seg_root, C.scan, compact, C.size);
  hipLaunchKernelGGL(k_final, g, dim3(kT), 0, s, img, C.segid, C.size, out);
  hipLaunchKernelGGL(k_zero, dim3(blocks(4 * n_img)), dim3(kT), 0, s, 4 * n_img, C.counts);
  hipLaunchKernelGGL(k_counts, dim3(gs), dim3(kT), 0, s, img, n_seg, C.seg_img, C.size0, C.mpar,
                     C.counts);
  return hipGetLastError();
}

}  // namespace gmmsp
