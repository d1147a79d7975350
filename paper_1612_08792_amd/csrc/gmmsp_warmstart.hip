// Learned warm start for the EM (gfx950): seed-grid features, a 4-layer
// conv3x3 network on v_mfma_f32_16x16x32_bf16 (BF16 operands, FP32
// accumulation), its backward pass, the loss and Adam, and the map from the
// network outputs to theta^0.
//
// Positions are the superpixels of the batch in batch order (image b's
// superpixel k = k_y n_x + k_x at sp_off + k); a precomputed table gives the
// nine 3x3 neighbours of each position inside its own image (-1 past the
// grid border, i.e. zero padding).  Activations are stored position-major
// (NHWC) in bfloat16 with 8, 16 or 32 channels per position.
//
// MFMA operand layout (16x16x32 bf16): lane l holds A[l % 16][8 (l / 16) + j]
// and B[8 (l / 16) + j][l % 16] for j = 0..7, and receives C[4 (l / 16) + i]
// [l % 16] for i = 0..3.  For a conv, the GEMM row is the position, the K
// index runs over (tap, input channel) in chunks of 32, the column is the
// output channel.
#include "gmmsp_internal.h"

#include <math.h>

namespace gmmsp {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ uint16_t f2bf(float f) {
  const __bf16 b = (__bf16)f;  // round to nearest, ties to even
  return __builtin_bit_cast(uint16_t, b);
}
__device__ __forceinline__ float bf2f(uint16_t u) { return __uint_as_float((uint32_t)u << 16); }

__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}
__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }

// ---------------------------------------------------------------------------
// neighbour table and features
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_ws_nbr(DevPtrs P, int32_t* __restrict__ nbr) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= P.n_sp) return;
  const SpDesc d = P.sp[p];
  const ImgDesc* I = P.img + d.img;
  const int nx = I->nx, ny = I->ny, off = I->sp_off;
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int kx = d.kx + t % 3 - 1, ky = d.ky + t / 3 - 1;
    nbr[(size_t)p * 9 + t] = (kx >= 0 && kx < nx && ky >= 0 && ky < ny) ? off + ky * nx + kx : -1;
  }
}

// One wave per seed cell: Lab mean and population std over the cell's v_x x v_y
// pixels (moments about the cell's first pixel), the border channel, the seed
// colour minus the mean, and the differences of the half-cell means (last h
// columns minus first h, last h rows minus first h, h = floor(v / 2)).
constexpr int kWsIn = 16;

__global__ __launch_bounds__(256) void k_ws_features(DevPtrs P, const float* __restrict__ lab,
                                                     float* __restrict__ feat,
                                                     uint16_t* __restrict__ x0) {
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (p >= P.n_sp) return;
  const SpDesc d = P.sp[p];
  const ImgDesc I = P.img[d.img];
  const int vx = I.vx, vy = I.vy, n = vx * vy, hx = vx / 2, hy = vy / 2;
  const float* base = lab + 3 * (I.pix_off + (int64_t)d.ky * vy * I.W + (int64_t)d.kx * vx);
  const float r0 = base[0], r1 = base[1], r2 = base[2];
  // 0-2 sums, 3-5 sums of squares, 6-8 left, 9-11 right, 12-14 top, 15-17 bottom
  float s[18];
#pragma unroll
  for (int j = 0; j < 18; ++j) s[j] = 0.f;
  for (int q = lane; q < n; q += 64) {
    const int row = q / vx, col = q - row * vx;
    const float* px = base + 3 * ((int64_t)row * I.W + col);
    const float c[3] = {px[0] - r0, px[1] - r1, px[2] - r2};
    const bool lf = col < hx, rt = col >= vx - hx, tp = row < hy, bt = row >= vy - hy;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      s[j] += c[j];
      s[3 + j] = fmaf(c[j], c[j], s[3 + j]);
      s[6 + j] += lf ? c[j] : 0.f;
      s[9 + j] += rt ? c[j] : 0.f;
      s[12 + j] += tp ? c[j] : 0.f;
      s[15 + j] += bt ? c[j] : 0.f;
    }
  }
  double t[18];
#pragma unroll
  for (int j = 0; j < 18; ++j) {
    t[j] = (double)s[j];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) t[j] += __shfl_xor(t[j], m, 64);
  }
  if (lane != 0) return;
  const double inv = 1.0 / n;
  const double r[3] = {r0, r1, r2};
  double mean[3], sd[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double m = t[j] * inv;
    mean[j] = r[j] + m;
    sd[j] = sqrt(fmax(t[3 + j] * inv - m * m, 0.0));
  }
  const int bd = min(min(min(d.kx, d.ky), min(I.nx - 1 - d.kx, I.ny - 1 - d.ky)), 3);
  const int sx = d.kx * vx + vx / 2, sy = d.ky * vy + vy / 2;
  const float* sp = lab + 3 * (I.pix_off + (int64_t)sy * I.W + sx);
  float f[kWsIn];
  f[0] = (float)((mean[0] - 50.0) / 50.0);
  f[1] = (float)(mean[1] / 64.0);
  f[2] = (float)(mean[2] / 64.0);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    f[3 + j] = (float)(sd[j] / 16.0);
    f[7 + j] = (float)(((double)sp[j] - mean[j]) / 16.0);
    // moments about the first pixel cancel in the differences of half means
    f[10 + j] = hx > 0 ? (float)((t[9 + j] - t[6 + j]) / ((double)hx * vy) / 32.0) : 0.f;
    f[13 + j] = hy > 0 ? (float)((t[15 + j] - t[12 + j]) / ((double)hy * vx) / 32.0) : 0.f;
  }
  f[6] = (float)bd / 3.0f;
#pragma unroll
  for (int j = 0; j < kWsIn; ++j) {
    feat[(size_t)p * kWsIn + j] = f[j];
    x0[(size_t)p * kWsIn + j] = f2bf(f[j]);
  }
}

// ---------------------------------------------------------------------------
// weights: FP32 master -> BF16 B operands
// ---------------------------------------------------------------------------

// B operand of a conv whose input has CINP (padded) channels: element j of lane
// l in chunk kc, column tile nt.  transposed = false: W[n][tap][ci] (forward).
// transposed = true: W[ci][8 - tap][n] (gradient with respect to the input:
// the input channel of that conv is the layer's output channel).
__global__ __launch_bounds__(256) void k_ws_prep(const float* __restrict__ W, int cout, int cin,
                                                 int cinp, int nk, int nt, int transposed,
                                                 uint16_t* __restrict__ wb) {
  const int i = blockIdx.x * 256 + threadIdx.x;  // element index
  const int total = nk * nt * 64 * 8;
  if (i >= total) return;
  const int j = i & 7, lane = (i >> 3) & 63, tile = i >> 9;
  const int kc = tile / nt, ntile = tile % nt;
  const int kb = lane >> 4, n = ntile * 16 + (lane & 15);
  const int cpb = cinp / 8, tpc = 4 / cpb;
  const int tap = kc * tpc + kb / cpb;
  const int ci = 8 * (kb % cpb) + j;
  float v = 0.f;
  if (tap < 9) {
    if (!transposed) {
      if (n < cout && ci < cin) v = W[((size_t)n * 9 + tap) * cin + ci];
    } else {
      // this conv's input channel ci is the layer's output channel, its output
      // channel n the layer's input channel
      if (ci < cout && n < cin) v = W[((size_t)ci * 9 + (8 - tap)) * cin + n];
    }
  }
  wb[i] = f2bf(v);
}

// ---------------------------------------------------------------------------
// conv3x3 as an MFMA GEMM over positions [p0, p1): one wave per 16 positions
// MODE 0: out = relu(acc + bias) in bf16 (NT * 16 channels)
// MODE 1: out = acc + bias in fp32, 16 channels per position (cout real ones)
// MODE 2: out = acc * (mask > 0) in bf16 (gradient through the ReLU of the
//         layer input; mask has NT * 16 channels)
// ---------------------------------------------------------------------------
template <int CINP, int NT, int MODE>
__global__ __launch_bounds__(256) void k_ws_conv(const int32_t* __restrict__ nbr,
                                                 const uint16_t* __restrict__ in,
                                                 const uint16_t* __restrict__ wb,
                                                 const float* __restrict__ bias, int cout,
                                                 const uint16_t* __restrict__ mask,
                                                 uint16_t* __restrict__ out_bf,
                                                 float* __restrict__ out_f, int p0, int p1) {
  constexpr int CPB = CINP / 8, TPC = 4 / CPB, NK = (9 * CINP + 31) / 32, CO = NT * 16;
  const int lane = threadIdx.x & 63;
  const int pt = p0 + (int)(blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  if (pt >= p1) return;  // whole wave
  const int col = lane & 15, kb = lane >> 4;
  const int p = pt + col;
  f32x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kc = 0; kc < NK; ++kc) {
    const int tap = kc * TPC + kb / CPB;
    const int cib = 8 * (kb % CPB);
    bf16x8 a = zero8();
    if (p < p1 && tap < 9) {
      const int q = nbr[(size_t)p * 9 + tap];
      if (q >= 0) a = load8(in + (size_t)q * CINP + cib);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const bf16x8 b = load8(wb + ((size_t)(kc * NT + t) * 64 + lane) * 8);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int pp = pt + 4 * kb + i;
      if (pp >= p1) continue;
      const int c = t * 16 + col;
      float v = acc[t][i];
      if (MODE == 0) {
        v = fmaxf(v + bias[c], 0.f);
        out_bf[(size_t)pp * CO + c] = f2bf(v);
      } else if (MODE == 1) {
        out_f[(size_t)pp * 16 + c] = c < cout ? v + bias[c] : 0.f;
      } else {
        v = bf2f(mask[(size_t)pp * CO + c]) > 0.f ? v : 0.f;
        out_bf[(size_t)pp * CO + c] = f2bf(v);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// weight gradient: dW[co][tap][ci] = sum_p g[p][co] x[nbr(p, tap)][ci] as an
// MFMA GEMM (rows co, columns (tap, ci), K = positions).  Block s reduces the
// positions of chunks [s cps, (s+1) cps) of 32 and writes its partial sums;
// k_ws_reduce_dw adds the partials in split order.
// ---------------------------------------------------------------------------
template <int CINP, int MT>
__global__ __launch_bounds__(64) void k_ws_dw(const int32_t* __restrict__ nbr,
                                              const uint16_t* __restrict__ g,
                                              const uint16_t* __restrict__ x,
                                              float* __restrict__ part, int p0, int p1, int cps) {
  constexpr int NCOL = 9 * CINP, NTN = (NCOL + 15) / 16, GC = MT * 16;
  const int lane = threadIdx.x;
  const int col = lane & 15, kb = lane >> 4;
  const int split = blockIdx.x;
  f32x4 acc[MT][NTN];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NTN; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int ch = 0; ch < cps; ++ch) {
    const int pb = p0 + (split * cps + ch) * 32;
    if (pb >= p1) break;  // whole wave
    int q[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) q[j] = pb + 8 * kb + j;
    bf16x8 a[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const uint16_t u = q[j] < p1 ? g[(size_t)q[j] * GC + m * 16 + col] : (uint16_t)0;
        a[m][j] = __builtin_bit_cast(__bf16, u);
      }
    }
#pragma unroll
    for (int t = 0; t < NTN; ++t) {
      const int n = t * 16 + col;
      const int tap = n / CINP, ci = n - (n / CINP) * CINP;
      bf16x8 b;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        uint16_t u = 0;
        if (n < NCOL && q[j] < p1) {
          const int r = nbr[(size_t)q[j] * 9 + tap];
          if (r >= 0) u = x[(size_t)r * CINP + ci];
        }
        b[j] = __builtin_bit_cast(__bf16, u);
      }
#pragma unroll
      for (int m = 0; m < MT; ++m)
        acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b, acc[m][t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NTN; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int co = m * 16 + 4 * kb + i, n = t * 16 + col;
        if (n < NCOL) part[((size_t)split * GC + co) * NCOL + n] = acc[m][t][i];
      }
}

// grad[co][n] = scale * sum_s part[s][co][n] for co < cout, n < ncol
__global__ __launch_bounds__(256) void k_ws_reduce_dw(const float* __restrict__ part, int splits,
                                                      int gc, int cout, int ncol, float scale,
                                                      float* __restrict__ grad) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= cout * ncol) return;
  const int co = i / ncol, n = i - co * ncol;
  double s = 0.0;
  for (int k = 0; k < splits; ++k) s += part[((size_t)k * gc + co) * ncol + n];
  grad[i] = (float)(s * scale);
}

// db[co] = scale * sum_p g[p][co]; one block per output channel, fixed order
__global__ __launch_bounds__(256) void k_ws_db(const uint16_t* __restrict__ g, int gc, int p0,
                                               int p1, float scale, float* __restrict__ db) {
  __shared__ double red[256];
  const int co = blockIdx.x;
  double s = 0.0;
  for (int p = p0 + threadIdx.x; p < p1; p += 256) s += bf2f(g[(size_t)p * gc + co]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[co] = (float)(red[0] * scale);
}

// squared error of the 10 outputs and the per-position gradient 2 d / 10 (the
// 1 / count of the mean is applied in the weight and bias reductions)
__global__ __launch_bounds__(256) void k_ws_loss(const float* __restrict__ out,
                                                 const float* __restrict__ tgt,
                                                 uint16_t* __restrict__ g4, int p0, int p1,
                                                 double* __restrict__ loss_part) {
  __shared__ double red[256];
  const int p = p0 + blockIdx.x * 256 + threadIdx.x;
  double s = 0.0;
  if (p < p1) {
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      float gv = 0.f;
      if (c < 10) {
        const float d = out[(size_t)p * 16 + c] - tgt[(size_t)p * 16 + c];
        s += (double)d * d;
        gv = 0.2f * d;
      }
      g4[(size_t)p * 16 + c] = f2bf(gv);
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

__global__ void k_ws_sum(const double* __restrict__ part, int n, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  *out = s;
}

__global__ __launch_bounds__(256) void k_ws_adam(float* __restrict__ w, float* __restrict__ m,
                                                 float* __restrict__ v,
                                                 const float* __restrict__ grad, int n, float lr,
                                                 float b1, float b2, float eps, float c1,
                                                 float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float g = grad[i];
  const float mi = b1 * m[i] + (1.f - b1) * g;
  const float vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
// outputs -> theta^0 rows, and converged theta -> targets
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ws_apply(DevPtrs P, const float* __restrict__ lab,
                                                  const float* __restrict__ out, uint32_t mask,
                                                  double* __restrict__ rows) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= P.n_sp) return;
  const SpDesc d = P.sp[p];
  const ImgDesc I = P.img[d.img];
  const int sx = d.kx * I.vx + I.vx / 2, sy = d.ky * I.vy + I.vy / 2;
  const float* px = lab + 3 * (I.pix_off + (int64_t)sy * I.W + sx);
  const double vx = I.vx, vy = I.vy, lam = I.lam;
  double o[10];
  bool finite = true;
#pragma unroll
  for (int c = 0; c < 10; ++c) {
    o[c] = ((mask >> c) & 1u) ? (double)out[(size_t)p * 16 + c] : 0.0;
    finite = finite && isfinite(o[c]);
  }
  if (!finite) {
    // grid initialisation of Sec. III-C for this superpixel
#pragma unroll
    for (int c = 0; c < 10; ++c) o[c] = 0.0;
  }
  double ls[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) ls[c] = fmin(fmax(o[5 + c], -4.0), 4.0);
  double* r = rows + (size_t)p * kThetaRow;
  r[0] = sx + vx * o[0];
  r[1] = sy + vy * o[1];
  r[2] = (double)px[0] + lam * o[2];
  r[3] = (double)px[1] + lam * o[3];
  r[4] = (double)px[2] + lam * o[4];
  r[5] = vx * vx * exp(2.0 * ls[0]);
  r[6] = 0.0;
  r[7] = vy * vy * exp(2.0 * ls[1]);
  r[8] = lam * lam * exp(2.0 * ls[2]);
  r[9] = lam * lam * exp(2.0 * ls[3]);
  r[10] = 0.0;
  r[11] = lam * lam * exp(2.0 * ls[4]);
  r[12] = 0.0;
}

__global__ __launch_bounds__(256) void k_ws_targets(DevPtrs P, const float* __restrict__ lab,
                                                    float* __restrict__ tgt) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= P.n_sp) return;
  const SpDesc d = P.sp[p];
  const ImgDesc I = P.img[d.img];
  const double* r = P.theta + (size_t)p * kThetaRow;
  const double vx = I.vx, vy = I.vy, lam = I.lam;
  const int sx = d.kx * I.vx + I.vx / 2, sy = d.ky * I.vy + I.vy / 2;
  const float* px = lab + 3 * (I.pix_off + (int64_t)sy * I.W + sx);
  float* t = tgt + (size_t)p * 16;
  t[0] = (float)((r[0] - sx) / vx);
  t[1] = (float)((r[1] - sy) / vy);
  t[2] = (float)((r[2] - (double)px[0]) / lam);
  t[3] = (float)((r[3] - (double)px[1]) / lam);
  t[4] = (float)((r[4] - (double)px[2]) / lam);
  const double var[5] = {r[5] / (vx * vx), r[7] / (vy * vy), r[8] / (lam * lam),
                         r[9] / (lam * lam), r[11] / (lam * lam)};
#pragma unroll
  for (int c = 0; c < 5; ++c) t[5 + c] = (float)fmin(fmax(0.5 * log(var[c]), -4.0), 4.0);
#pragma unroll
  for (int c = 10; c < 16; ++c) t[c] = 0.f;
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
static inline unsigned nblk(size_t n, unsigned per) { return (unsigned)((n + per - 1) / per); }

hipError_t ws_launch_nbr(const DevPtrs& P, int32_t* nbr, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_nbr, dim3(nblk(P.n_sp, 256)), dim3(256), 0, s, P, nbr);
  return hipGetLastError();
}

hipError_t ws_launch_features(const DevPtrs& P, const float* lab, float* feat, uint16_t* x0,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_ws_features, dim3(nblk(P.n_sp, 4)), dim3(256), 0, s, P, lab, feat, x0);
  return hipGetLastError();
}

hipError_t ws_launch_prep(const float* W, int cout, int cin, int cinp, int nk, int nt,
                          int transposed, uint16_t* wb, hipStream_t s) {
  const int total = nk * nt * 64 * 8;
  hipLaunchKernelGGL(k_ws_prep, dim3(nblk(total, 256)), dim3(256), 0, s, W, cout, cin, cinp, nk,
                     nt, transposed, wb);
  return hipGetLastError();
}

hipError_t ws_launch_conv(int layer, int mode, const int32_t* nbr, const uint16_t* in,
                          const uint16_t* wb, const float* bias, int cout, const uint16_t* mask,
                          uint16_t* out_bf, float* out_f, int p0, int p1, hipStream_t s) {
  const unsigned grid = nblk((size_t)nblk(p1 - p0, 16), 4);
  if (grid == 0) return hipSuccess;
  if (mode == 0 && layer == 1)
    hipLaunchKernelGGL((k_ws_conv<16, 2, 0>), dim3(grid), dim3(256), 0, s, nbr, in, wb, bias, cout,
                       mask, out_bf, out_f, p0, p1);
  else if (mode == 0)
    hipLaunchKernelGGL((k_ws_conv<32, 2, 0>), dim3(grid), dim3(256), 0, s, nbr, in, wb, bias,
                       cout, mask, out_bf, out_f, p0, p1);
  else if (mode == 1)
    hipLaunchKernelGGL((k_ws_conv<32, 1, 1>), dim3(grid), dim3(256), 0, s, nbr, in, wb, bias,
                       cout, mask, out_bf, out_f, p0, p1);
  else if (layer == 4)  // gradient input has 16 channels (10 real)
    hipLaunchKernelGGL((k_ws_conv<16, 2, 2>), dim3(grid), dim3(256), 0, s, nbr, in, wb, bias,
                       cout, mask, out_bf, out_f, p0, p1);
  else
    hipLaunchKernelGGL((k_ws_conv<32, 2, 2>), dim3(grid), dim3(256), 0, s, nbr, in, wb, bias,
                       cout, mask, out_bf, out_f, p0, p1);
  return hipGetLastError();
}

hipError_t ws_launch_dw(int layer, const int32_t* nbr, const uint16_t* g, const uint16_t* x,
                        float* part, int splits, int cps, int p0, int p1, hipStream_t s) {
  if (layer == 1)
    hipLaunchKernelGGL((k_ws_dw<16, 2>), dim3(splits), dim3(64), 0, s, nbr, g, x, part, p0, p1, cps);
  else if (layer == 4)
    hipLaunchKernelGGL((k_ws_dw<32, 1>), dim3(splits), dim3(64), 0, s, nbr, g, x, part, p0, p1, cps);
  else
    hipLaunchKernelGGL((k_ws_dw<32, 2>), dim3(splits), dim3(64), 0, s, nbr, g, x, part, p0, p1, cps);
  return hipGetLastError();
}

hipError_t ws_launch_reduce_dw(const float* part, int splits, int gc, int cout, int ncol,
                               float scale, float* grad, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_reduce_dw, dim3(nblk((size_t)cout * ncol, 256)), dim3(256), 0, s, part,
                     splits, gc, cout, ncol, scale, grad);
  return hipGetLastError();
}

hipError_t ws_launch_db(const uint16_t* g, int gc, int cout, int p0, int p1, float scale,
                        float* db, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_db, dim3(cout), dim3(256), 0, s, g, gc, p0, p1, scale, db);
  return hipGetLastError();
}

hipError_t ws_launch_loss(const float* out, const float* tgt, uint16_t* g4, int p0, int p1,
                          double* loss_part, double* loss_sum, hipStream_t s) {
  const unsigned nb = nblk(p1 - p0, 256);
  hipLaunchKernelGGL(k_ws_loss, dim3(nb), dim3(256), 0, s, out, tgt, g4, p0, p1, loss_part);
  hipLaunchKernelGGL(k_ws_sum, dim3(1), dim3(64), 0, s, loss_part, (int)nb, loss_sum);
  return hipGetLastError();
}

hipError_t ws_launch_adam(float* w, float* m, float* v, const float* grad, int n, float lr,
                          float b1, float b2, float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_adam, dim3(nblk(n, 256)), dim3(256), 0, s, w, m, v, grad, n, lr, b1, b2,
                     eps, c1, c2);
  return hipGetLastError();
}

hipError_t ws_launch_apply(const DevPtrs& P, const float* lab, const float* out, uint32_t mask,
                           double* rows, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_apply, dim3(nblk(P.n_sp, 256)), dim3(256), 0, s, P, lab, out, mask, rows);
  return hipGetLastError();
}

hipError_t ws_launch_targets(const DevPtrs& P, const float* lab, float* tgt, hipStream_t s) {
  hipLaunchKernelGGL(k_ws_targets, dim3(nblk(P.n_sp, 256)), dim3(256), 0, s, P, lab, tgt);
  return hipGetLastError();
}

}  // namespace gmmsp
