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
// |s_k n s_g| are a dense S_b x G_b count table per image (S_b G_b < 2^31),
// filled with integer atomics after a per-wave aggregation of runs of equal
// (k, g) along the pixel row.  Every result is a ratio of exact integer
// counts.
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

// superpixel boundary map (bytes)
__global__ __launch_bounds__(kT) void k_m_bnd(const ImgDesc* img, const int32_t* sp,
                                              uint8_t* sb) {
  const int b = blockIdx.y;
  const ImgDesc& I = img[b];
  const int W = I.W, H = I.H;
  const int j = blockIdx.x * kT + threadIdx.x;
  if (j >= W * H) return;
  const int64_t i = I.pix_off + j;
  const int x = j % W, y = j / W;
  const int32_t v = sp[i];
  sb[i] = (x + 1 < W && sp[i + 1] != v) || (y + 1 < H && sp[i + W] != v);
}

// overlap counts, and per block the boundary recall counts
__global__ __launch_bounds__(kT) void k_m_pix(const ImgDesc* img, const int32_t* sp,
                                              const int32_t* gt, const uint8_t* sb,
                                              const int32_t* n_lab, const int32_t* n_gt,
                                              const int64_t* tab_off, int* tab, int* br_part,
                                              int max_blocks, int* err) {
  __shared__ int wsum[kT / 64][2];
  const int b = blockIdx.y;
  const ImgDesc& I = img[b];
  const int W = I.W, H = I.H, n = W * H;
  if ((int)(blockIdx.x * kT) >= n) return;  // whole block beyond the image
  const int j = blockIdx.x * kT + threadIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const bool in = j < n;
  const int64_t i = I.pix_off + j;
  const int G = n_gt[b];
  const int K = n_lab[b];
  int key = -1;
  bool gb = false, hit = false;
  if (in) {
    const int k = sp[i], g = gt[i];
    if (k < 0 || k >= K || g < 0 || g >= G) {
      atomicOr(err, 1);
    } else {
      key = k * G + g;
    }
    const int x = j % W, y = j / W;
    gb = (x + 1 < W && gt[i + 1] != g) || (y + 1 < H && gt[i + W] != g);
    if (gb) {
      for (int yy = max(0, y - kR); yy <= min(H - 1, y + kR) && !hit; ++yy)
        for (int xx = max(0, x - kR); xx <= min(W - 1, x + kR); ++xx)
          if (sb[I.pix_off + (int64_t)yy * W + xx]) {
            hit = true;
            break;
          }
    }
  }
  // runs of equal key along the wave: one atomic per run
  const int kl = __shfl_up(key, 1, 64);
  int hp = (lane == 0 || kl != key) ? lane : 0;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(hp, o, 64);
    if (lane >= o) hp = max(hp, t);
  }
  const int kr = __shfl_down(key, 1, 64);
  if (key >= 0 && (lane == 63 || kr != key)) atomicAdd(tab + tab_off[b] + key, lane - hp + 1);
  const unsigned long long mh = __ballot(hit), mt = __ballot(gb);
  if (lane == 0) {
    wsum[wv][0] = __popcll(mh);
    wsum[wv][1] = __popcll(mt);
  }
  __syncthreads();
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
  int size = 0, best = 0;
  for (int g = lane; g < G; g += 64) {
    const int c = r[g];
    size += c;
    best = max(best, c);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    size += __shfl_xor(size, o, 64);
    best = max(best, __shfl_xor(best, o, 64));
  }
  int leak = 0;
  for (int g = lane; g < G; g += 64) leak += 20LL * r[g] > (int64_t)size;
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
  const int nb = (I.W * I.H + kT - 1) / kT;
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

int metrics_max_blocks(int max_pixels) { return (int)blocks(max_pixels); }

hipError_t metrics_launch(const DevPtrs& P, int max_pixels, const int32_t* sp, const int32_t* gt,
                          const int32_t* n_lab, const int32_t* n_gt, const int64_t* row_off,
                          int64_t n_rows, const int64_t* tab_off, int64_t tab_n, int* tab,
                          uint8_t* sb, int* br_part, int64_t* row_ue, int64_t* row_asa,
                          int64_t* sums, int* err, hipStream_t s) {
  const unsigned fill_blocks = (unsigned)std::min<int64_t>(blocks(tab_n), 65536);
  hipLaunchKernelGGL(k_m_fill, dim3(std::max(1u, fill_blocks)), dim3(kT), 0, s, tab_n, tab);
  hipLaunchKernelGGL(k_m_fill, dim3(1), dim3(kT), 0, s, (int64_t)1, err);
  const int mb = metrics_max_blocks(max_pixels);
  const dim3 g(mb, P.n_img);
  hipLaunchKernelGGL(k_m_bnd, g, dim3(kT), 0, s, P.img, sp, sb);
  hipLaunchKernelGGL(k_m_pix, g, dim3(kT), 0, s, P.img, sp, gt, sb, n_lab, n_gt, tab_off, tab,
                     br_part, mb, err);
  hipLaunchKernelGGL(k_m_rows, dim3((unsigned)((n_rows + 3) / 4)), dim3(kT), 0, s, P.n_img,
                     row_off, n_gt, tab_off, tab, row_ue, row_asa);
  hipLaunchKernelGGL(k_m_reduce, dim3(P.n_img), dim3(kT), 0, s, P.img, br_part, mb, row_off,
                     row_ue, row_asa, sums);
  return hipGetLastError();
}

}  // namespace gmmsp
