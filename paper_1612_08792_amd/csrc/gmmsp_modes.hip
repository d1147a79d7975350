// Two more covariance models on gfx950, with the same work decomposition as the
// split-colour kernels (one wave per v_x x v_y cell, its nine records read by
// scalar loads, FP32 statistics reduced across the wave and written in FP64,
// a fixed-order per-superpixel gather with FP64 shape control):
//
//   * cov_mode 2, the full 5 x 5 Sigma of Eq. UpdateSig.  The paper defines its
//     eigenvalue floors per block (Eqs. mlams, mlamc); on a full Sigma they act
//     on Sigma scaled by F = diag(eps_s, eps_s, eps_c, eps_c, eps_c): the
//     eigenvalues of F^-1/2 Sigma F^-1/2 are raised to at least 1 (cyclic
//     Jacobi in FP64).  On a block-diagonal Sigma this is the per-block rule.
//   * cov_mode 3, grayscale images: z = (x, y, I), D = 3 (Sec. III-A), Sigma =
//     diag(Sigma_s, sigma_I^2) with floors eps_s and eps_c (Sec. III-C); the
//     input holds one float per pixel.
//
// Also the dispatch of every covariance model other than the split colour
// blocks (cov_mode 1 runs the kernels of gmmsp_cov3.hip).
#include "gmmsp_internal.h"
#include "gmmsp_wave.h"

#include <math.h>

namespace gmmsp {

namespace {

// position of (i, j), i <= j, in the row-by-row upper triangle of a 5 x 5 matrix
__host__ __device__ constexpr int ut(int i, int j) { return i * 5 - i * (i - 1) / 2 + (j - i); }

// Symmetric eigen-decomposition by cyclic Jacobi rotations (at most 30
// sweeps): A ends diagonal (its eigenvalues), V holds the eigenvectors.
template <int N>
__device__ void jacobi(double (&A)[N][N], double (&V)[N][N]) {
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) V[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int i = 0; i < N; ++i) {
      dia += A[i][i] * A[i][i];
      for (int j = i + 1; j < N; ++j) off += A[i][j] * A[i][j];
    }
    if (!(off > 1e-36 * dia)) break;
    for (int p = 0; p < N - 1; ++p) {
      for (int q = p + 1; q < N; ++q) {
        const double apq = A[p][q];
        if (apq == 0.0) continue;
        const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
        const double at = fabs(theta);
        double t = at > 1e150 ? 0.5 / at : 1.0 / (at + sqrt(at * at + 1.0));
        if (theta < 0.0) t = -t;
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < N; ++k) {  // A <- A J
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < N; ++k) {  // A <- J^T A
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < N; ++k) {  // V <- V J
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
    }
  }
}

// 2 x 2 spatial block (xx, xy, yy) with every eigenvalue floored at eps; a
// block already above the floor is kept as it is
__device__ void clamp_sym2(double xx, double xy, double yy, double eps, double out[3]) {
  double A[2][2] = {{xx, xy}, {xy, yy}}, V[2][2];
  jacobi<2>(A, V);
  if (A[0][0] >= eps && A[1][1] >= eps) {
    out[0] = xx;
    out[1] = xy;
    out[2] = yy;
    return;
  }
  const double l0 = fmax(A[0][0], eps), l1 = fmax(A[1][1], eps);
  out[0] = V[0][0] * l0 * V[0][0] + V[0][1] * l1 * V[0][1];
  out[1] = V[0][0] * l0 * V[1][0] + V[0][1] * l1 * V[1][1];
  out[2] = V[1][0] * l0 * V[1][0] + V[1][1] * l1 * V[1][1];
}

// the folded spatial factor of a record: t1 = l11 xr + l12 yr + o1, t2 =
// l22 yr + o2 with t1^2 + t2^2 = (d^T Sigma_s^-1 d) / (2 ln 2), d the offset
// from (mx, my) given relative to the cell origin
__device__ void spatial_factor(double sxx, double sxy, double syy, double mx, double my,
                               float* r /* l11 l12 o1 o2 l22 */) {
  const double s2 = sqrt(0.5 * kLog2e);
  const double det = sxx * syy - sxy * sxy;
  const double l11 = s2 * sqrt(syy / det);
  const double l12 = -s2 * sxy / sqrt(det * syy);
  const double l22 = s2 / sqrt(syy);
  r[0] = (float)l11;
  r[1] = (float)l12;
  r[2] = (float)(-(l11 * mx + l12 * my));
  r[3] = (float)(-l22 * my);
  r[4] = (float)l22;
}

// ===========================================================================
// cov_mode 2: full 5 x 5 Sigma
// ===========================================================================

// Record of a cell slot (float32): u = U (z - mu) with U upper triangular and
// U^T U = Sigma^-1 / (2 ln 2), folded with the cell origin, so for a pixel
// z = (xr, yr, L, a, b) (position relative to the cell origin)
//   u_i = sum_{j >= i} U_ij z_j + O_i,  l = C - |u|^2 = log2 p(z; theta_k) - cmax2,
// and (ML, MA, MB) the float32 colour mean, the origin of the colour statistics.
constexpr int F_U = 0;  // 15 entries, ut(i, j) order
constexpr int F_O = 15;  // 5 offsets
enum RecFull { F_C = 20, F_ML = 21, F_MA = 22, F_MB = 23 };

// statistics of a cell slot: spatial about the cell origin, colour about ML..MB
enum StatFull {
  G_N = 0, G_X, G_Y, G_L, G_A, G_B, G_XX, G_XY, G_YY, G_LL, G_LA, G_LB, G_AA, G_AB, G_BB,
  G_XL, G_XA, G_XB, G_YL, G_YA, G_YB
};
static_assert(G_YB + 1 == kStatsF, "statistics of the full model");

// Shape control of a full Sigma (upper triangle s, ut order) with floors
// f[5]: the eigenvalues of F^-1/2 Sigma F^-1/2 are raised to at least 1.
// Returns the clamped Sigma, its inverse (ut order) and ln det.
__device__ void clamp_full(const double s[15], const double f[5], double out[15], double prec[15],
                           double* lndet) {
  double sf[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) sf[i] = sqrt(f[i]);
  double A[5][5], V[5][5];
  for (int i = 0; i < 5; ++i)
    for (int j = i; j < 5; ++j) A[i][j] = A[j][i] = s[ut(i, j)] / (sf[i] * sf[j]);
  jacobi<5>(A, V);
  double t[5];
  bool keep = true;
  double lnd = 0.0;
  for (int k = 0; k < 5; ++k) {
    keep = keep && A[k][k] >= 1.0;
    t[k] = fmax(A[k][k], 1.0);
    lnd += log(t[k]) + 2.0 * log(sf[k]);
  }
  for (int i = 0; i < 5; ++i) {
    for (int j = i; j < 5; ++j) {
      double v = 0.0, w = 0.0;
      for (int k = 0; k < 5; ++k) {
        v += V[i][k] * t[k] * V[j][k];
        w += V[i][k] * V[j][k] / t[k];
      }
      out[ut(i, j)] = keep ? s[ut(i, j)] : v * sf[i] * sf[j];
      prec[ut(i, j)] = w / (sf[i] * sf[j]);
    }
  }
  *lndet = lnd;
}

struct SpFull {
  double mu[5];
  double s[15];     // clamped Sigma, ut order
  double prec[15];  // its inverse
  double lndet;
};

__device__ inline void full_floors(const ImgDesc& I, double f[5]) {
  f[0] = f[1] = I.eps_s;
  f[2] = f[3] = f[4] = I.eps_c;
}

__device__ inline void store_row_full(double* row, const SpFull& q, double mass) {
#pragma unroll
  for (int i = 0; i < 5; ++i) row[i] = q.mu[i];
#pragma unroll
  for (int i = 0; i < 15; ++i) row[5 + i] = q.s[i];
  row[20] = mass;
}

__device__ void write_record_full(const DevPtrs& P, const ImgDesc& I, int kx, int ky,
                                  const SpFull& q, int dx, int dy) {
  const int cx = kx - dx, cy = ky - dy;
  if (cx < 0 || cx >= I.ncx || cy < 0 || cy >= I.ncy) return;
  const int slot = 3 * (dy + 1) + (dx + 1);
  // Cholesky P = L L^T (lower L); U = L^T
  double Lm[5][5];
  for (int j = 0; j < 5; ++j) {
    double d = q.prec[ut(j, j)];
    for (int k = 0; k < j; ++k) d -= Lm[j][k] * Lm[j][k];
    Lm[j][j] = sqrt(d);
    for (int i = j + 1; i < 5; ++i) {
      double v = q.prec[ut(j, i)];
      for (int k = 0; k < j; ++k) v -= Lm[i][k] * Lm[j][k];
      Lm[i][j] = v / Lm[j][j];
    }
  }
  const double s2 = sqrt(0.5 * kLog2e);
  const double m[5] = {q.mu[0] - (double)cx * I.vx, q.mu[1] - (double)cy * I.vy, q.mu[2], q.mu[3],
                       q.mu[4]};
  float r[kRecF];
#pragma unroll
  for (int i = 0; i < kRecF; ++i) r[i] = 0.f;
  for (int i = 0; i < 5; ++i) {
    double o = 0.0;
    for (int j = i; j < 5; ++j) {
      const double u = s2 * Lm[j][i];
      r[F_U + ut(i, j)] = (float)u;
      o -= u * m[j];
    }
    r[F_O + i] = (float)o;
  }
  r[F_C] = (float)(kLog2e * (-2.5 * kLn2Pi - 0.5 * q.lndet - I.lncmax));
  r[F_ML] = (float)q.mu[2];
  r[F_MA] = (float)q.mu[3];
  r[F_MB] = (float)q.mu[4];
  float4* dst = reinterpret_cast<float4*>(
      P.rec + ((size_t)(I.cell_off + cy * I.ncx + cx) * kSlots + slot) * kRecF);
#pragma unroll
  for (int j = 0; j < kRecF / 4; ++j)
    dst[j] = make_float4(r[4 * j], r[4 * j + 1], r[4 * j + 2], r[4 * j + 3]);
}

// ===========================================================================
// cov_mode 3: grayscale, D = 3
// ===========================================================================

// Record of a cell slot (float32): the spatial factor as in the colour modes,
// w = UI I + PI with UI^2 = 1 / (2 ln 2 sigma_I^2), l = C - t1^2 - t2^2 - w^2,
// MI the float32 intensity mean, the origin of the intensity statistics.
enum RecGray {
  H_L11 = 0, H_L12 = 1, H_O1 = 2, H_O2 = 3, H_L22 = 4, H_C = 5, H_UI = 6, H_PI = 7, H_MI = 8
};
enum StatGray { J_N = 0, J_X, J_Y, J_I, J_XX, J_XY, J_YY, J_II };
static_assert(J_II + 1 == kStatsG, "statistics of the grayscale model");

struct SpGray {
  double mx, my, mI, sxx, sxy, syy, sII;
};

__device__ inline void store_row_gray(double* row, const SpGray& q, double mass) {
  row[0] = q.mx; row[1] = q.my; row[2] = q.mI;
  row[3] = q.sxx; row[4] = q.sxy; row[5] = q.syy; row[6] = q.sII;
  row[7] = mass;
}

__device__ void write_record_gray(const DevPtrs& P, const ImgDesc& I, int kx, int ky,
                                  const SpGray& q, int dx, int dy) {
  const int cx = kx - dx, cy = ky - dy;
  if (cx < 0 || cx >= I.ncx || cy < 0 || cy >= I.ncy) return;
  const int slot = 3 * (dy + 1) + (dx + 1);
  float r[kRecG];
#pragma unroll
  for (int i = 0; i < kRecG; ++i) r[i] = 0.f;
  spatial_factor(q.sxx, q.sxy, q.syy, q.mx - (double)cx * I.vx, q.my - (double)cy * I.vy,
                 r + H_L11);
  const double ui = sqrt(0.5 * kLog2e / q.sII);
  r[H_UI] = (float)ui;
  r[H_PI] = (float)(-ui * q.mI);
  const double lndet = log(q.sxx * q.syy - q.sxy * q.sxy) + log(q.sII);
  r[H_C] = (float)(kLog2e * (-1.5 * kLn2Pi - 0.5 * lndet - I.lncmax));
  r[H_MI] = (float)q.mI;
  float4* dst = reinterpret_cast<float4*>(
      P.rec + ((size_t)(I.cell_off + cy * I.ncx + cx) * kSlots + slot) * kRecG);
#pragma unroll
  for (int j = 0; j < kRecG / 4; ++j)
    dst[j] = make_float4(r[4 * j], r[4 * j + 1], r[4 * j + 2], r[4 * j + 3]);
}

__device__ inline SpGray clamp_gray(double mx, double my, double mI, double sxx, double sxy,
                                    double syy, double sII, const ImgDesc& I) {
  SpGray q;
  q.mx = mx;
  q.my = my;
  q.mI = mI;
  double s[3];
  clamp_sym2(sxx, sxy, syy, I.eps_s, s);
  q.sxx = s[0];
  q.sxy = s[1];
  q.syy = s[2];
  q.sII = fmax(sII, I.eps_c);
  return q;
}

// ===========================================================================
// The two models for the per-cell kernel
// ===========================================================================

struct FullModel {
  static constexpr int kRec = kRecF, kStat = kStatsF, kPart = kPartF, kCh = 3, kC = F_C;
  static constexpr int kNOff = 5;  // the offsets of the five whitened coordinates
  static constexpr int kOffIdx[kNOff] = {F_O, F_O + 1, F_O + 2, F_O + 3, F_O + 4};
  static __device__ __forceinline__ float eval(const AS4 float* f, const float (&o)[kNOff],
                                               float xr, float yr, const float (&c)[kCh]) {
    const float z[5] = {xr, yr, c[0], c[1], c[2]};
    float l = f[F_C];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      float u = o[i];
#pragma unroll
      for (int j = i; j < 5; ++j) u = fmaf(f[F_U + ut(i, j)], z[j], u);
      l = fmaf(-u, u, l);
    }
    return l;
  }
  static __device__ __forceinline__ void accumulate(float* a, float R, const AS4 float* f,
                                                    float xr, float yr, const float (&c)[kCh],
                                                    float xx, float xy, float yy) {
    const float dL = c[0] - f[F_ML], da = c[1] - f[F_MA], db = c[2] - f[F_MB];
    a[G_N] += R;
    a[G_X] = fmaf(R, xr, a[G_X]);
    a[G_Y] = fmaf(R, yr, a[G_Y]);
    a[G_XX] = fmaf(R, xx, a[G_XX]);
    a[G_XY] = fmaf(R, xy, a[G_XY]);
    a[G_YY] = fmaf(R, yy, a[G_YY]);
    const float rL = R * dL, ra = R * da, rb = R * db;
    a[G_L] += rL;
    a[G_A] += ra;
    a[G_B] += rb;
    a[G_LL] = fmaf(rL, dL, a[G_LL]);
    a[G_LA] = fmaf(rL, da, a[G_LA]);
    a[G_LB] = fmaf(rL, db, a[G_LB]);
    a[G_AA] = fmaf(ra, da, a[G_AA]);
    a[G_AB] = fmaf(ra, db, a[G_AB]);
    a[G_BB] = fmaf(rb, db, a[G_BB]);
    a[G_XL] = fmaf(rL, xr, a[G_XL]);
    a[G_XA] = fmaf(ra, xr, a[G_XA]);
    a[G_XB] = fmaf(rb, xr, a[G_XB]);
    a[G_YL] = fmaf(rL, yr, a[G_YL]);
    a[G_YA] = fmaf(ra, yr, a[G_YA]);
    a[G_YB] = fmaf(rb, yr, a[G_YB]);
  }
};

struct GrayModel {
  static constexpr int kRec = kRecG, kStat = kStatsG, kPart = kPartG, kCh = 1, kC = H_C;
  static constexpr int kNOff = 3;  // the offsets of t1, t2 and w
  static constexpr int kOffIdx[kNOff] = {H_O1, H_O2, H_PI};
  static __device__ __forceinline__ float eval(const AS4 float* f, const float (&o)[kNOff],
                                               float xr, float yr, const float (&c)[kCh]) {
    const float t1 = fmaf(f[H_L11], xr, fmaf(f[H_L12], yr, o[0]));
    const float t2 = fmaf(f[H_L22], yr, o[1]);
    const float w = fmaf(f[H_UI], c[0], o[2]);
    float l = fmaf(-t1, t1, f[H_C]);
    l = fmaf(-t2, t2, l);
    return fmaf(-w, w, l);
  }
  static __device__ __forceinline__ void accumulate(float* a, float R, const AS4 float* f,
                                                    float xr, float yr, const float (&c)[kCh],
                                                    float xx, float xy, float yy) {
    const float dI = c[0] - f[H_MI];
    a[J_N] += R;
    a[J_X] = fmaf(R, xr, a[J_X]);
    a[J_Y] = fmaf(R, yr, a[J_Y]);
    a[J_XX] = fmaf(R, xx, a[J_XX]);
    a[J_XY] = fmaf(R, xy, a[J_XY]);
    a[J_YY] = fmaf(R, yy, a[J_YY]);
    const float rI = R * dI;
    a[J_I] += rI;
    a[J_II] = fmaf(rI, dI, a[J_II]);
  }
};

enum CellModeM { CM_STATS = 0, CM_LABEL = 1, CM_EXPORT_R = 2, CM_EXPORT_CAND = 3 };

template <class M>
__global__ __launch_bounds__(256) void km_clear_records(float* rec, size_t n_rec) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n_rec) return;
  float* d = rec + i * M::kRec;
  for (int j = 0; j < M::kRec; ++j) d[j] = 0.f;
  d[M::kC] = -INFINITY;
}

// One wave per cell, one pixel per lane per round of 64; the record offsets
// are read from the wave's LDS block.
template <class M, int MODE>
__global__ __launch_bounds__(256) void km_cells(DevPtrs P, const float* __restrict__ in,
                                                int32_t* __restrict__ out_i,
                                                float* __restrict__ out_f) {
  constexpr int kCh = M::kCh, kRec = M::kRec, kStat = M::kStat;
  const int lane = threadIdx.x & 63;
  const int cell = __builtin_amdgcn_readfirstlane(
      (int)(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6)));
  if (cell >= P.n_cell) return;
  const AS4 CellDesc* cdp = cptr(P.cell) + cell;
  const int b = cdp->img, ccx = cdp->cx, ccy = cdp->cy;
  const AS4 ImgDesc* Ip = cptr(P.img) + b;
  if (MODE == CM_STATS && cptr(P.state)[b].done) return;
  const int W = Ip->W, H = Ip->H, vx = Ip->vx, vy = Ip->vy;
  const int x0 = ccx * vx, y0 = ccy * vy;
  const int w = min(vx, W - x0), h = min(vy, H - y0);
  const int npix = w * h;
  const int64_t pix0 = Ip->pix_off + (int64_t)y0 * W + x0;
  const AS4 float* rec0 = cptr(P.rec) + (size_t)cell * (kSlots * kRec);

  if (MODE == CM_EXPORT_CAND) {
    const int nx = Ip->nx, ny = Ip->ny;
    for (int p = lane; p < npix; p += 64) {
      const int row = p / w, col = p - row * w;
      int32_t* dst = out_i + (size_t)(pix0 + (int64_t)row * W + col) * kSlots;
#pragma unroll
      for (int s = 0; s < kSlots; ++s) {
        const int kx = ccx + (s % 3) - 1, ky = ccy + (s / 3) - 1;
        const bool idx_ok = kx >= 0 && kx < nx && ky >= 0 && ky < ny;
        const bool rec_ok = rec0[s * kRec + M::kC] != -INFINITY;
        dst[s] = (idx_ok != rec_ok) ? -2 : (idx_ok ? ky * nx + kx : -1);
      }
    }
    return;
  }

  constexpr int NS = kSlots * kStat;
  constexpr int CAP = 2 * ((NS + 1) / 2);
  float acc[CAP];
  if (MODE == CM_STATS) {
#pragma unroll
    for (int i = 0; i < CAP; ++i) acc[i] = 0.f;
  }
  float llacc = 0.f;
  const float* img = in + (size_t)kCh * pix0;
  __shared__ float s_off[kWavesPerBlock * kOffBlock];
  float* woff0 = s_off + (threadIdx.x >> 6) * kOffBlock;
  stage_offsets(woff0, P.rec + (size_t)cell * (kSlots * kRec), kRec, M::kOffIdx, lane);
  for (int p = lane; p < npix; p += 64) {
    // opaque zero offsets: the records are re-read each round by scalar loads
    // and the offsets by LDS reads, rather than held in registers
    int zero = 0, vz = 0;
    asm volatile("" : "+s"(zero));
    asm volatile("" : "+v"(vz));
    const AS4 float* rec = rec0 + zero;
    const float* woff = woff0 + vz;
    const int row = p / w, col = p - row * w;
    const float* px = img + (size_t)kCh * ((int64_t)row * W + col);
    float c[kCh];
#pragma unroll
    for (int k = 0; k < kCh; ++k) c[k] = px[k];
    const float xr = (float)col, yr = (float)row;
    float e[kSlots];
    float sum = 0.f;
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
      float o[M::kNOff];
      load_offsets(woff, s, o);
      e[s] = __builtin_amdgcn_exp2f(M::eval(rec + s * kRec, o, xr, yr, c));
      sum += e[s];
    }
    float shift = 0.f;
    if (sum < 0x1p-100f) {
      // every candidate is far away: subtract the largest exponent first
      float lv[kSlots];
      float m = -INFINITY;
#pragma unroll
      for (int s = 0; s < kSlots; ++s) {
        float o[M::kNOff];
        load_offsets(woff, s, o);
        lv[s] = M::eval(rec + s * kRec, o, xr, yr, c);
        m = fmaxf(m, lv[s]);
      }
      sum = 0.f;
#pragma unroll
      for (int s = 0; s < kSlots; ++s) {
        e[s] = __builtin_amdgcn_exp2f(lv[s] - m);
        sum += e[s];
      }
      shift = m;
    }
    const float inv = __builtin_amdgcn_rcpf(sum);
    llacc += __builtin_amdgcn_logf(sum) + shift;
    if (MODE == CM_STATS) {
      const float xx = xr * xr, xy = xr * yr, yy = yr * yr;
#pragma unroll
      for (int s = 0; s < kSlots; ++s)
        M::accumulate(acc + s * kStat, e[s] * inv, rec + s * kRec, xr, yr, c, xx, xy, yy);
    } else if (MODE == CM_LABEL) {
      // Eq. obtLi: the largest posterior, ties to the smallest k
      int best = 0;
      float be = e[0];
#pragma unroll
      for (int s = 1; s < kSlots; ++s) {
        if (e[s] > be) {
          be = e[s];
          best = s;
        }
      }
      const int kx = ccx + (best % 3) - 1, ky = ccy + (best / 3) - 1;
      out_i[pix0 + (int64_t)row * W + col] = ky * Ip->nx + kx;
    } else {
      float* dst = out_f + (size_t)(pix0 + (int64_t)row * W + col) * kSlots;
#pragma unroll
      for (int s = 0; s < kSlots; ++s) dst[s] = e[s] * inv;
    }
  }
  if (MODE == CM_STATS) {
    wave_reduce_scatter<NS>(acc, lane);
    const int r = (int)(__builtin_bitreverse32((unsigned)lane) >> 26);
    double* part = P.part + (size_t)cell * M::kPart;
#pragma unroll
    for (int q = 0; q < (NS + 63) / 64; ++q)
      if (64 * q + r < NS) part[64 * q + r] = (double)acc[q];
  }
  if (MODE == CM_STATS || MODE == CM_LABEL) {
    double ll = (double)llacc;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) ll += __shfl_xor(ll, m, 64);
    if (lane == 0) P.llp[cell] = kLn2 * ll + (double)npix * Ip->lncmax;
  }
}

// ---- per-superpixel kernels of the full model ------------------------------

__device__ void write_records_full(const DevPtrs& P, const ImgDesc& I, int kx, int ky,
                                   const SpFull& q) {
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) write_record_full(P, I, kx, ky, q, dx, dy);
}

// theta^0 or a given row: the shape control applied, the records written
__device__ void full_from(const DevPtrs& P, const SpDesc& d, const ImgDesc& I, const double mu[5],
                          const double s[15], double mass, int sp) {
  SpFull q;
  double f[5];
  full_floors(I, f);
#pragma unroll
  for (int i = 0; i < 5; ++i) q.mu[i] = mu[i];
  clamp_full(s, f, q.s, q.prec, &q.lndet);
  store_row_full(P.theta + (size_t)sp * kThetaRowF, q, mass);
  write_records_full(P, I, d.kx, d.ky, q);
}

__global__ __launch_bounds__(256) void kf_init_seeds(DevPtrs P, const float* __restrict__ lab) {
  const int sp = blockIdx.x * 256 + threadIdx.x;
  if (sp >= P.n_sp) return;
  const SpDesc d = P.sp[sp];
  const ImgDesc I = P.img[d.img];
  const int x = d.kx * I.vx + I.vx / 2, y = d.ky * I.vy + I.vy / 2;
  const float* px = lab + 3 * (I.pix_off + (int64_t)y * I.W + x);
  const double mu[5] = {(double)x, (double)y, px[0], px[1], px[2]};
  double s[15];
#pragma unroll
  for (int i = 0; i < 15; ++i) s[i] = 0.0;
  const double l2 = I.lam * I.lam;
  s[ut(0, 0)] = (double)I.vx * I.vx;
  s[ut(1, 1)] = (double)I.vy * I.vy;
  s[ut(2, 2)] = s[ut(3, 3)] = s[ut(4, 4)] = l2;
  full_from(P, d, I, mu, s, 0.0, sp);
}

__global__ __launch_bounds__(256) void kf_set_params(DevPtrs P, const double* __restrict__ rows) {
  const int sp = blockIdx.x * 256 + threadIdx.x;
  if (sp >= P.n_sp) return;
  const SpDesc d = P.sp[sp];
  const ImgDesc I = P.img[d.img];
  const double* row = rows + (size_t)sp * kThetaRowF;
  full_from(P, d, I, row, row + 5, row[20], sp);
}

// M-step: fixed-order gather of the window's cell partials, the mean (Eq.
// UpdateMu), the full covariance about it (Eq. UpdateSig), shape control, FP64
__global__ __launch_bounds__(256) void kf_finalize(DevPtrs P) {
  const int sp = blockIdx.x * 256 + threadIdx.x;
  if (sp >= P.n_sp) return;
  const SpDesc d = P.sp[sp];
  if (P.state[d.img].done) return;
  const ImgDesc I = P.img[d.img];
  double a[kStatsF];
#pragma unroll
  for (int j = 0; j < kStatsF; ++j) a[j] = 0.0;
  for (int dy = -1; dy <= 1; ++dy) {
    for (int dx = -1; dx <= 1; ++dx) {
      const int cx = d.kx - dx, cy = d.ky - dy;
      if (cx < 0 || cx >= I.ncx || cy < 0 || cy >= I.ncy) continue;
      const int slot = 3 * (dy + 1) + (dx + 1);
      // positions move from the cell's origin to the superpixel's own cell origin
      const double ox = (double)(-dx) * I.vx, oy = (double)(-dy) * I.vy;
      const double* q =
          P.part + (size_t)(I.cell_off + cy * I.ncx + cx) * kPartF + slot * kStatsF;
      const double n = q[G_N], sx = q[G_X], sy = q[G_Y];
      a[G_N] += n;
      a[G_X] += sx + ox * n;
      a[G_Y] += sy + oy * n;
      a[G_XX] += q[G_XX] + 2.0 * ox * sx + ox * ox * n;
      a[G_XY] += q[G_XY] + ox * sy + oy * sx + ox * oy * n;
      a[G_YY] += q[G_YY] + 2.0 * oy * sy + oy * oy * n;
#pragma unroll
      for (int j = G_L; j <= G_B; ++j) a[j] += q[j];
#pragma unroll
      for (int j = G_LL; j <= G_BB; ++j) a[j] += q[j];
      a[G_XL] += q[G_XL] + ox * q[G_L];
      a[G_XA] += q[G_XA] + ox * q[G_A];
      a[G_XB] += q[G_XB] + ox * q[G_B];
      a[G_YL] += q[G_YL] + oy * q[G_L];
      a[G_YA] += q[G_YA] + oy * q[G_A];
      a[G_YB] += q[G_YB] + oy * q[G_B];
    }
  }
  double* row = P.theta + (size_t)sp * kThetaRowF;
  const double N = a[G_N];
  if (!(N >= I.n_min)) {
    row[20] = N;  // 0/0 guard: theta_k keeps its value
    return;
  }
  const double iN = 1.0 / N;
  const double m[5] = {a[G_X] * iN, a[G_Y] * iN, a[G_L] * iN, a[G_A] * iN, a[G_B] * iN};
  // second moments in ut order: x y L a b against x y L a b
  const double s2[15] = {a[G_XX], a[G_XY], a[G_XL], a[G_XA], a[G_XB], a[G_YY], a[G_YL],
                         a[G_YA], a[G_YB], a[G_LL], a[G_LA], a[G_LB], a[G_AA], a[G_AB], a[G_BB]};
  double s[15];
  for (int i = 0; i < 5; ++i)
    for (int j = i; j < 5; ++j) s[ut(i, j)] = s2[ut(i, j)] * iN - m[i] * m[j];
  // colour moments were taken about the float32 record mean
  const double mu[5] = {(double)d.kx * I.vx + m[0], (double)d.ky * I.vy + m[1],
                        (double)(float)row[2] + m[2], (double)(float)row[3] + m[3],
                        (double)(float)row[4] + m[4]};
  full_from(P, d, I, mu, s, N, sp);
}

// ---- per-superpixel kernels of the grayscale model -------------------------

__device__ void gray_from(const DevPtrs& P, const SpDesc& d, const ImgDesc& I, const SpGray& q,
                          double mass, int sp) {
  store_row_gray(P.theta + (size_t)sp * kThetaRowG, q, mass);
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) write_record_gray(P, I, d.kx, d.ky, q, dx, dy);
}

__global__ __launch_bounds__(256) void kg_init_seeds(DevPtrs P, const float* __restrict__ gray) {
  const int sp = blockIdx.x * 256 + threadIdx.x;
  if (sp >= P.n_sp) return;
  const SpDesc d = P.sp[sp];
  const ImgDesc I = P.img[d.img];
  const int x = d.kx * I.vx + I.vx / 2, y = d.ky * I.vy + I.vy / 2;
  const double v = gray[I.pix_off + (int64_t)y * I.W + x];
  const double l2 = I.lam * I.lam;
  gray_from(P, d, I,
            clamp_gray(x, y, v, (double)I.vx * I.vx, 0.0, (double)I.vy * I.vy, l2, I), 0.0, sp);
}

__global__ __launch_bounds__(256) void kg_set_params(DevPtrs P, const double* __restrict__ rows) {
  const int sp = blockIdx.x * 256 + threadIdx.x;
  if (sp >= P.n_sp) return;
  const SpDesc d = P.sp[sp];
  const ImgDesc I = P.img[d.img];
  const double* r = rows + (size_t)sp * kThetaRowG;
  gray_from(P, d, I, clamp_gray(r[0], r[1], r[2], r[3], r[4], r[5], r[6], I), r[7], sp);
}

__global__ __launch_bounds__(256) void kg_finalize(DevPtrs P) {
  const int sp = blockIdx.x * 256 + threadIdx.x;
  if (sp >= P.n_sp) return;
  const SpDesc d = P.sp[sp];
  if (P.state[d.img].done) return;
  const ImgDesc I = P.img[d.img];
  double a[kStatsG];
#pragma unroll
  for (int j = 0; j < kStatsG; ++j) a[j] = 0.0;
  for (int dy = -1; dy <= 1; ++dy) {
    for (int dx = -1; dx <= 1; ++dx) {
      const int cx = d.kx - dx, cy = d.ky - dy;
      if (cx < 0 || cx >= I.ncx || cy < 0 || cy >= I.ncy) continue;
      const int slot = 3 * (dy + 1) + (dx + 1);
      const double ox = (double)(-dx) * I.vx, oy = (double)(-dy) * I.vy;
      const double* q =
          P.part + (size_t)(I.cell_off + cy * I.ncx + cx) * kPartG + slot * kStatsG;
      const double n = q[J_N], sx = q[J_X], sy = q[J_Y];
      a[J_N] += n;
      a[J_X] += sx + ox * n;
      a[J_Y] += sy + oy * n;
      a[J_XX] += q[J_XX] + 2.0 * ox * sx + ox * ox * n;
      a[J_XY] += q[J_XY] + ox * sy + oy * sx + ox * oy * n;
      a[J_YY] += q[J_YY] + 2.0 * oy * sy + oy * oy * n;
      a[J_I] += q[J_I];
      a[J_II] += q[J_II];
    }
  }
  double* row = P.theta + (size_t)sp * kThetaRowG;
  const double N = a[J_N];
  if (!(N >= I.n_min)) {
    row[7] = N;  // 0/0 guard: theta_k keeps its value
    return;
  }
  const double iN = 1.0 / N;
  const double mx = a[J_X] * iN, my = a[J_Y] * iN, mI = a[J_I] * iN;
  const SpGray q = clamp_gray((double)d.kx * I.vx + mx, (double)d.ky * I.vy + my,
                              (double)(float)row[2] + mI, a[J_XX] * iN - mx * mx,
                              a[J_XY] * iN - mx * my, a[J_YY] * iN - my * my,
                              a[J_II] * iN - mI * mI, I);
  gray_from(P, d, I, q, N, sp);
}

inline unsigned blocks_of(size_t n, unsigned per) { return (unsigned)((n + per - 1) / per); }

template <class M>
hipError_t cells(const DevPtrs& P, int mode, const float* in, int32_t* out_i, float* out_f,
                 hipStream_t s) {
  const dim3 grid(blocks_of(P.n_cell, kWavesPerBlock)), blk(256);
  switch (mode) {
    case 0: hipLaunchKernelGGL((km_cells<M, CM_STATS>), grid, blk, 0, s, P, in, out_i, out_f); break;
    case 1: hipLaunchKernelGGL((km_cells<M, CM_LABEL>), grid, blk, 0, s, P, in, out_i, out_f); break;
    case 2:
      hipLaunchKernelGGL((km_cells<M, CM_EXPORT_R>), grid, blk, 0, s, P, in, out_i, out_f);
      break;
    default:
      hipLaunchKernelGGL((km_cells<M, CM_EXPORT_CAND>), grid, blk, 0, s, P, in, out_i, out_f);
  }
  return hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------------------
// Dispatch of the covariance models other than the split colour blocks
// ---------------------------------------------------------------------------

hipError_t launch_alt_clear_records(const DevPtrs& P, hipStream_t s) {
  if (P.cov_mode == 1) return launch3_clear_records(P, s);
  const size_t n = (size_t)P.n_cell * kSlots;
  if (P.cov_mode == 2)
    hipLaunchKernelGGL(km_clear_records<FullModel>, dim3(blocks_of(n, 256)), dim3(256), 0, s,
                       P.rec, n);
  else
    hipLaunchKernelGGL(km_clear_records<GrayModel>, dim3(blocks_of(n, 256)), dim3(256), 0, s,
                       P.rec, n);
  return hipGetLastError();
}

hipError_t launch_alt_init_seeds(const DevPtrs& P, const float* in, hipStream_t s) {
  if (P.cov_mode == 1) return launch3_init_seeds(P, in, s);
  if (P.cov_mode == 2)
    hipLaunchKernelGGL(kf_init_seeds, dim3(blocks_of(P.n_sp, 256)), dim3(256), 0, s, P, in);
  else
    hipLaunchKernelGGL(kg_init_seeds, dim3(blocks_of(P.n_sp, 256)), dim3(256), 0, s, P, in);
  return hipGetLastError();
}

hipError_t launch_alt_set_params(const DevPtrs& P, const double* rows, hipStream_t s) {
  if (P.cov_mode == 1) return launch3_set_params(P, rows, s);
  if (P.cov_mode == 2)
    hipLaunchKernelGGL(kf_set_params, dim3(blocks_of(P.n_sp, 256)), dim3(256), 0, s, P, rows);
  else
    hipLaunchKernelGGL(kg_set_params, dim3(blocks_of(P.n_sp, 256)), dim3(256), 0, s, P, rows);
  return hipGetLastError();
}

hipError_t launch_alt_cells(const DevPtrs& P, int mode, const float* in, int32_t* out_i,
                            float* out_f, hipStream_t s) {
  if (P.cov_mode == 1) return launch3_cells(P, mode, in, out_i, out_f, s);
  if (P.cov_mode == 2) return cells<FullModel>(P, mode, in, out_i, out_f, s);
  return cells<GrayModel>(P, mode, in, out_i, out_f, s);
}

hipError_t launch_alt_finalize(const DevPtrs& P, hipStream_t s) {
  if (P.cov_mode == 1) return launch3_finalize(P, s);
  if (P.cov_mode == 2)
    hipLaunchKernelGGL(kf_finalize, dim3(blocks_of(P.n_sp, 256)), dim3(256), 0, s, P);
  else
    hipLaunchKernelGGL(kg_finalize, dim3(blocks_of(P.n_sp, 256)), dim3(256), 0, s, P);
  return hipGetLastError();
}

}  // namespace gmmsp
