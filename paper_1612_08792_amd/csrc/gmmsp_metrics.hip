// Segmentation accuracy measures of Sec. IV on gfx950, per image of a batch:
// boundary recall (BR), under-segmentation error (Eq. ue) and achievable
// segmentation accuracy (Eq. asa) of a superpixel label map against a
// ground-truth region map.
//
//   * a boundary pixel of a map is one whose right or lower neighbour carries
//     another value; a ground-truth boundary pixel is recovered when a
//     superpixel boundary pixel lies in the 5 x 5 square around it;
//   * UE = (1/N) sum_g sum_{k : 20 |s_k n s_g| > |s_k|} |s_k| - 1 (eps = 0.05
//     compared exactly), ASA = (1/N) sum_k max_g |s_k n s_g|.
//
// Superpixel labels lie in [0, S_b) (S_b given per image, by default the
// image's seed-grid size K_b) and region ids in [0, G_b); the overlaps
// |s_k n s_g| are a dense S_b x G_b count table per image (S_b G_b < 2^31).
// The pixel pass runs on 64 x 16 tiles: the superpixel boundary map of the
// tile and a 2-pixel halo is built in LDS, the runs of equal (k, g) along each
// row are gathered per block in an LDS table, and the block adds each entry to
// the count table once.  Every result is a ratio of exact integer counts.
#include "gmmsp_internal.h"

#include <algorithm>

namespace gmmsp {

namespace {

constexpr int kT = 256;
constexpr int kR = 2;  // boundary tolerance in pixels (square window)

__global__ __launch_bounds__(kT) void k_m_fill(int64_t n, int* a) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    a[i] = 0;
}

constexpr int kMW = 64, kMH = 16;        // tile of the pixel pass
constexpr int kBW = kMW + 2 * kR;        // boundary map of the tile and its halo
constexpr int kBH = kMH + 2 * kR;
constexpr int kHW = kBW + 1, kHH = kBH + 1;  // labels needed for it (right, lower neighbour)
constexpr int kMHash = 128;              // LDS table entries (a power of two)

__host__ __device__ inline int m_tiles(int W, int H) {
  return ((W + kMW - 1) / kMW) * ((H + kMH - 1) / kMH);
}

// overlap counts, and per block the boundary recall counts
__global__ __launch_bounds__(kT) void k_m_pix(const ImgDesc* img, const int32_t* sp,
                                              const int32_t* gt, const int32_t* n_lab,
                                              const int32_t* n_gt, const int64_t* tab_off,
                                              int* tab, int* br_part, int max_blocks, int* err) {
  __shared__ int32_t hs[kHH * kHW];
  __shared__ uint8_t hb[kBH * kBW];
  __shared__ int hkey[kMHash], hcnt[kMHash];
  __shared__ int wsum[kT / 64][2];
  const int b = blockIdx.y;
  const ImgDesc& I = img[b];
  const int W = I.W, H = I.H;
  const int tiles_x = (W + kMW - 1) / kMW;
  if ((int)blockIdx.x >= m_tiles(W, H)) return;  // the whole block
  const int x0 = (blockIdx.x % tiles_x) * kMW, y0 = (blockIdx.x / tiles_x) * kMH;
  const int64_t off = I.pix_off;
  // superpixel labels of the tile and its halo (0 outside the image, never read as such)
  for (int e = threadIdx.x; e < kHH * kHW; e += kT) {
    const int x = x0 - kR + e % kHW, y = y0 - kR + e / kHW;
    hs[e] = (x >= 0 && x < W && y >= 0 && y < H) ? sp[off + (int64_t)y * W + x] : 0;
  }
  for (int e = threadIdx.x; e < kMHash; e += kT) {
    hkey[e] = -1;
    hcnt[e] = 0;
  }
  __syncthreads();
  // superpixel boundary pixels: the right or lower neighbour carries another label
  for (int e = threadIdx.x; e < kBH * kBW; e += kT) {
    const int rx = e % kBW, ry = e / kBW;
    const int x = x0 - kR + rx, y = y0 - kR + ry;
    bool v = false;
    if (x >= 0 && x < W && y >= 0 && y < H) {
      const int32_t h = hs[ry * kHW + rx];
      v = (x + 1 < W && hs[ry * kHW + rx + 1] != h) || (y + 1 < H && hs[(ry + 1) * kHW + rx] != h);
    }
    hb[e] = v;
  }
  __syncthreads();
  const int G = n_gt[b], K = n_lab[b];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int x = x0 + lane;
  int nhit = 0, ngb = 0;
  // the wave's rows of region ids (and their right and lower neighbours) first
  constexpr int kRows = kMH / (kT / 64);
  int gq[kRows][3];
#pragma unroll
  for (int u = 0; u < kRows; ++u) {
    const int y = y0 + wv + u * (kT / 64);
    const int64_t i = off + (int64_t)y * W + x;
    const bool in = x < W && y < H;
    gq[u][0] = in ? gt[i] : 0;
    gq[u][1] = in && x + 1 < W ? gt[i + 1] : gq[u][0];
    gq[u][2] = in && y + 1 < H ? gt[i + W] : gq[u][0];
  }
#pragma unroll
  for (int u = 0; u < kRows; ++u) {
    const int ty = wv + u * (kT / 64);
    const int y = y0 + ty;
    const bool in = x < W && y < H;
    int key = -1;
    bool gb = false, hit = false;
    if (in) {
      const int k = hs[(ty + kR) * kHW + lane + kR], g = gq[u][0];
      if (k < 0 || k >= K || g < 0 || g >= G) {
        atomicOr(err, 1);
      } else {
        key = k * G + g;
      }
      gb = gq[u][1] != g || gq[u][2] != g;
      if (gb) {  // a superpixel boundary pixel in the 5 x 5 square (the halo is 0 outside)
        const uint8_t* c = hb + ty * kBW + lane;
#pragma unroll
        for (int dy = 0; dy <= 2 * kR; ++dy)
#pragma unroll
          for (int dx = 0; dx <= 2 * kR; ++dx) hit |= c[dy * kBW + dx] != 0;
      }
    }
    nhit += __popcll(__ballot(hit));
    ngb += __popcll(__ballot(gb));
    // runs of equal key along the row: the run's length, gathered per block
    const int kl = __shfl_up(key, 1, 64);
    const unsigned long long heads = __ballot(lane == 0 || kl != key);
    const int hp = 63 - __builtin_clzll(heads & ((2ull << lane) - 1ull));
    const bool last = lane == 63 || ((heads >> (lane + 1)) & 1ull);
    if (key < 0 || !last) continue;
    const int len = lane - hp + 1;
    const int h0 = (int)(((unsigned)key * 2654435761u) >> 25);  // top 7 bits
    bool done = false;
    for (int p = 0; p < kMHash && !done; ++p) {
      const int e = (h0 + p) & (kMHash - 1);
      const int q = atomicCAS(hkey + e, -1, key);
      if (q == -1 || q == key) {
        atomicAdd(hcnt + e, len);
        done = true;
      }
    }
    if (!done) atomicAdd(tab + tab_off[b] + key, len);
  }
  if (lane == 0) {
    wsum[wv][0] = nhit;
    wsum[wv][1] = ngb;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kMHash; e += kT)
    if (hkey[e] >= 0) atomicAdd(tab + tab_off[b] + hkey[e], hcnt[e]);
  if (threadIdx.x < 2) {
    int t = 0;
    for (int w = 0; w < kT / 64; ++w) t += wsum[w][threadIdx.x];
    br_part[((int64_t)b * max_blocks + blockIdx.x) * 2 + threadIdx.x] = t;
  }
}

// one wave per superpixel k (a row of its image's count table): |s_k|, the
// leaking overlaps, the largest overlap.  Rows are numbered image by image
// (row_off[b] .. row_off[b + 1]).
__global__ __launch_bounds__(kT) void k_m_rows(int n_img, const int64_t* row_off,
                                               const int32_t* n_gt, const int64_t* tab_off,
                                               const int* tab, int64_t* row_ue, int64_t* row_asa) {
  const int64_t row = (int64_t)blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= row_off[n_img]) return;  // whole wave
  int lo = 0, hi = n_img - 1;  // the image b with row_off[b] <= row < row_off[b + 1]
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (row_off[mid] <= row) lo = mid;
    else hi = mid - 1;
  }
  const int b = lo;
  const int G = n_gt[b];
  const int* r = tab + tab_off[b] + (row - row_off[b]) * G;
  // the row's first 64 kRowCache entries stay in registers for the second pass
  constexpr int kRowCache = 32;
  int c[kRowCache];
  int size = 0, best = 0;
#pragma unroll
  for (int q = 0; q < kRowCache; ++q) {
    const int g = 64 * q + lane;
    c[q] = g < G ? r[g] : 0;
    size += c[q];
    best = max(best, c[q]);
  }
  for (int g = 64 * kRowCache + lane; g < G; g += 64) {
    const int v = r[g];
    size += v;
    best = max(best, v);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    size += __shfl_xor(size, o, 64);
    best = max(best, __shfl_xor(best, o, 64));
  }
  int leak = 0;
#pragma unroll
  for (int q = 0; q < kRowCache; ++q) leak += 20LL * c[q] > (int64_t)size;
  for (int g = 64 * kRowCache + lane; g < G; g += 64) leak += 20LL * r[g] > (int64_t)size;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) leak += __shfl_xor(leak, o, 64);
  if (lane == 0) {
    row_ue[row] = (int64_t)size * leak;
    row_asa[row] = best;
  }
}

// one block per image: fixed-order sums of the block and row partials
__global__ __launch_bounds__(kT) void k_m_reduce(const ImgDesc* img, const int* br_part,
                                                 int max_blocks, const int64_t* row_off,
                                                 const int64_t* row_ue, const int64_t* row_asa,
                                                 int64_t* sums) {
  __shared__ int64_t red[4][kT];
  const int b = blockIdx.x;
  const ImgDesc& I = img[b];
  const int nb = m_tiles(I.W, I.H);
  const int64_t r0 = row_off[b], r1 = row_off[b + 1];
  int64_t a[4] = {0, 0, 0, 0};
  for (int t = threadIdx.x; t < nb; t += kT) {
    a[0] += br_part[((int64_t)b * max_blocks + t) * 2 + 0];
    a[1] += br_part[((int64_t)b * max_blocks + t) * 2 + 1];
  }
  for (int64_t k = r0 + threadIdx.x; k < r1; k += kT) {
    a[2] += row_ue[k];
    a[3] += row_asa[k];
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) red[c][threadIdx.x] = a[c];
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
#pragma unroll
      for (int c = 0; c < 4; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 4) sums[4 * b + threadIdx.x] = red[threadIdx.x][0];
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

}  // namespace

int metrics_max_blocks(int max_w, int max_h) { return m_tiles(max_w, max_h); }

hipError_t metrics_launch(const DevPtrs& P, int max_blocks, const int32_t* sp, const int32_t* gt,
                          const int32_t* n_lab, const int32_t* n_gt, const int64_t* row_off,
                          int64_t n_rows, const int64_t* tab_off, int64_t tab_n, int* tab,
                          int* br_part, int64_t* row_ue, int64_t* row_asa, int64_t* sums,
                          int* err, hipStream_t s) {
  const unsigned fill_blocks = (unsigned)std::min<int64_t>(blocks(tab_n), 65536);
  hipLaunchKernelGGL(k_m_fill, dim3(std::max(1u, fill_blocks)), dim3(kT), 0, s, tab_n, tab);
  hipLaunchKernelGGL(k_m_fill, dim3(1), dim3(kT), 0, s, (int64_t)1, err);
  const int mb = max_blocks;
  hipLaunchKernelGGL(k_m_pix, dim3(mb, P.n_img), dim3(kT), 0, s, P.img, sp, gt, n_lab, n_gt,
                     tab_off, tab, br_part, mb, err);
  hipLaunchKernelGGL(k_m_rows, dim3((unsigned)((n_rows + 3) / 4)), dim3(kT), 0, s, P.n_img,
                     row_off, n_gt, tab_off, tab, row_ue, row_asa);
  hipLaunchKernelGGL(k_m_reduce, dim3(P.n_img), dim3(kT), 0, s, P.img, br_part, mb, row_off,
                     row_ue, row_asa, sums);
  return hipGetLastError();
}

}  // namespace gmmsp
