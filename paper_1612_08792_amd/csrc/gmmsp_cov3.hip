// The unified 3x3 colour block (cov_mode 1): Sigma_k = diag(Sigma_s (x, y),
// Sigma_c (L, a, b)) as in Eq. BlockSigma, with shape control of both blocks
// (Eqs. eigdecs .. eigdecrc: every eigenvalue floored, eps_s spatial, eps_c
// colour).  Same work decomposition as the split-colour kernels: one wave per
// v_x x v_y cell with its nine records read by scalar loads, the statistics
// reduced across the wave in FP32 and written in FP64, then a per-superpixel
// fixed-order gather with FP64 shape control.  One pixel per lane (the 9 x 15
// statistics fill the registers).
#include "gmmsp_internal.h"
#include "gmmsp_wave.h"

#include <math.h>

namespace gmmsp {

namespace {

// Record of slot s of a cell (float32, kRec3 floats), folded with the cell
// origin: for a pixel at (xr, yr) relative to the origin with colour (L, a, b)
//   t1 = L11 xr + L12 yr + O1,  t2 = L22 yr + O2,
//   u1 = U11 L + U12 a + U13 b + P1,  u2 = U22 a + U23 b + P2,  u3 = U33 b + P3,
//   l  = C - t1^2 - t2^2 - u1^2 - u2^2 - u3^2 = log2 p(z; theta_k) - cmax2
// (U upper triangular with U^T U = Sigma_c^-1 / (2 ln 2)); (ML, MA, MB) is
// the float32 colour mean, the origin of the colour statistics.
enum Rec3 {
  Q_L11 = 0, Q_L12 = 1, Q_O1 = 2, Q_O2 = 3, Q_L22 = 4, Q_C = 5, Q_U11 = 6, Q_U12 = 7,
  Q_P1 = 8, Q_P2 = 9, Q_U13 = 10, Q_U22 = 11, Q_U23 = 12, Q_U33 = 13, Q_P3 = 14,
  Q_ML = 15, Q_MA = 16, Q_MB = 17
};

// statistics of a cell slot: spatial about the cell origin, colour about ML..MB
enum Stat3 {
  T_N = 0, T_X = 1, T_Y = 2, T_L = 3, T_A = 4, T_B = 5, T_XX = 6, T_XY = 7, T_YY = 8,
  T_LL = 9, T_LA = 10, T_LB = 11, T_AA = 12, T_AB = 13, T_BB = 14
};

// FP64 parameters of one superpixel; colour block c = (LL, La, Lb, aa, ab, bb)
struct Sp3 {
  double mx, my, mL, ma, mb;
  double sxx, sxy, syy;
  double c[6];
};

// Symmetric 3x3 shape control: cyclic Jacobi rotations (at most 16 sweeps)
// give Q and the eigenvalues; each eigenvalue below eps is raised to eps and
// the block rebuilt on the same eigenvectors.  A block whose eigenvalues all
// reach eps is kept as it is.
__device__ void clamp3(const double in[6], double eps, double out[6]) {
  double A[3][3] = {{in[0], in[1], in[2]}, {in[1], in[3], in[4]}, {in[2], in[4], in[5]}};
  double V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int sweep = 0; sweep < 16; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (!(off > 1e-36 * dia)) break;
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
      const double apq = A[p][q];
      if (apq == 0.0) continue;
      const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
      const double at = fabs(theta);
      double t = at > 1e150 ? 0.5 / at : 1.0 / (at + sqrt(at * at + 1.0));
      if (theta < 0.0) t = -t;
      const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
      for (int k = 0; k < 3; ++k) {  // A <- A J
        const double akp = A[k][p], akq = A[k][q];
        A[k][p] = c * akp - s * akq;
        A[k][q] = s * akp + c * akq;
      }
      for (int k = 0; k < 3; ++k) {  // A <- J^T A
        const double apk = A[p][k], aqk = A[q][k];
        A[p][k] = c * apk - s * aqk;
        A[q][k] = s * apk + c * aqk;
      }
      for (int k = 0; k < 3; ++k) {  // V <- V J
        const double vkp = V[k][p], vkq = V[k][q];
        V[k][p] = c * vkp - s * vkq;
        V[k][q] = s * vkp + c * vkq;
      }
    }
  }
  const double l[3] = {A[0][0], A[1][1], A[2][2]};
  if (l[0] >= eps && l[1] >= eps && l[2] >= eps) {
#pragma unroll
    for (int i = 0; i < 6; ++i) out[i] = in[i];
    return;
  }
  const double lc[3] = {fmax(l[0], eps), fmax(l[1], eps), fmax(l[2], eps)};
  const int ii[6] = {0, 0, 0, 1, 1, 2}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) v += V[ii[e]][k] * lc[k] * V[jj[e]][k];
    out[e] = v;
  }
}

__device__ inline void store_row3(double* row, const Sp3& q, double mass) {
  row[0] = q.mx; row[1] = q.my; row[2] = q.mL; row[3] = q.ma; row[4] = q.mb;
  row[5] = q.sxx; row[6] = q.sxy; row[7] = q.syy;
#pragma unroll
  for (int i = 0; i < 6; ++i) row[8 + i] = q.c[i];
  row[14] = mass;
}

// theta row -> parameters with both blocks' shape control applied
__device__ inline Sp3 from_row3(const double* row, const ImgDesc& I) {
  Sp3 q;
  q.mx = row[0]; q.my = row[1]; q.mL = row[2]; q.ma = row[3]; q.mb = row[4];
  const double s3[6] = {row[5], row[6], 0.0, row[7], 0.0, 1.0};
  // the spatial block through the 2x2 path of clamp3 (third axis decoupled at 1)
  double s_out[6];
  const double sp_in[6] = {s3[0], s3[1], 0.0, s3[3], 0.0, fmax(I.eps_s, 1.0)};
  clamp3(sp_in, I.eps_s, s_out);
  q.sxx = s_out[0]; q.sxy = s_out[1]; q.syy = s_out[3];
  const double c_in[6] = {row[8], row[9], row[10], row[11], row[12], row[13]};
  clamp3(c_in, I.eps_c, q.c);
  return q;
}

// the record of superpixel (kx, ky) for cell (kx - dx, ky - dy)
__device__ void write_record3(const DevPtrs& P, const ImgDesc& I, int kx, int ky, const Sp3& q,
                              int dx, int dy) {
  const int cx = kx - dx, cy = ky - dy;
  if (cx < 0 || cx >= I.ncx || cy < 0 || cy >= I.ncy) return;
  const int slot = 3 * (dy + 1) + (dx + 1);
  const double s2 = sqrt(0.5 * kLog2e);
  const double det_s = q.sxx * q.syy - q.sxy * q.sxy;
  const double l11 = s2 * sqrt(q.syy / det_s);
  const double l12 = -s2 * q.sxy / sqrt(det_s * q.syy);
  const double l22 = s2 / sqrt(q.syy);
  // colour precision by cofactors, then its upper Cholesky factor
  const double c00 = q.c[0], c01 = q.c[1], c02 = q.c[2], c11 = q.c[3], c12 = q.c[4], c22 = q.c[5];
  const double a00 = c11 * c22 - c12 * c12, a01 = c02 * c12 - c01 * c22, a02 = c01 * c12 - c02 * c11;
  const double a11 = c00 * c22 - c02 * c02, a12 = c01 * c02 - c00 * c12, a22 = c00 * c11 - c01 * c01;
  const double det_c = c00 * a00 + c01 * a01 + c02 * a02;
  const double p00 = a00 / det_c, p01 = a01 / det_c, p02 = a02 / det_c;
  const double p11 = a11 / det_c, p12 = a12 / det_c, p22 = a22 / det_c;
  const double u11 = sqrt(p00), u12 = p01 / u11, u13 = p02 / u11;
  const double u22 = sqrt(p11 - u12 * u12), u23 = (p12 - u12 * u13) / u22;
  const double u33 = sqrt(p22 - u13 * u13 - u23 * u23);
  const double lndet = log(det_s) + log(det_c);
  const double cc = kLog2e * (-2.5 * kLn2Pi - 0.5 * lndet - I.lncmax);
  const double mxs = q.mx - (double)cx * I.vx, mys = q.my - (double)cy * I.vy;
  float r[kRec3];
#pragma unroll
  for (int i = 0; i < kRec3; ++i) r[i] = 0.f;
  r[Q_L11] = (float)l11;
  r[Q_L12] = (float)l12;
  r[Q_O1] = (float)(-(l11 * mxs + l12 * mys));
  r[Q_O2] = (float)(-l22 * mys);
  r[Q_L22] = (float)l22;
  r[Q_C] = (float)cc;
  r[Q_U11] = (float)(s2 * u11);
  r[Q_U12] = (float)(s2 * u12);
  r[Q_U13] = (float)(s2 * u13);
  r[Q_U22] = (float)(s2 * u22);
  r[Q_U23] = (float)(s2 * u23);
  r[Q_U33] = (float)(s2 * u33);
  r[Q_P1] = (float)(-s2 * (u11 * q.mL + u12 * q.ma + u13 * q.mb));
  r[Q_P2] = (float)(-s2 * (u22 * q.ma + u23 * q.mb));
  r[Q_P3] = (float)(-s2 * u33 * q.mb);
  r[Q_ML] = (float)q.mL;
  r[Q_MA] = (float)q.ma;
  r[Q_MB] = (float)q.mb;
  float4* dst = reinterpret_cast<float4*>(
      P.rec + ((size_t)(I.cell_off + cy * I.ncx + cx) * kSlots + slot) * kRec3);
#pragma unroll
  for (int j = 0; j < kRec3 / 4; ++j)
    dst[j] = make_float4(r[4 * j], r[4 * j + 1], r[4 * j + 2], r[4 * j + 3]);
}

__device__ void write_records3(const DevPtrs& P, const ImgDesc& I, int kx, int ky, const Sp3& q) {
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) write_record3(P, I, kx, ky, q, dx, dy);
}

__global__ __launch_bounds__(256) void k3_clear_records(float* rec, size_t n_rec) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n_rec) return;
  float* d = rec + i * kRec3;
  for (int j = 0; j < kRec3; ++j) d[j] = 0.f;
  d[Q_C] = -INFINITY;
}

__global__ __launch_bounds__(256) void k3_init_seeds(DevPtrs P, const float* __restrict__ lab) {
  const int sp = blockIdx.x * 256 + threadIdx.x;
  if (sp >= P.n_sp) return;
  const SpDesc d = P.sp[sp];
  const ImgDesc I = P.img[d.img];
  const int x = d.kx * I.vx + I.vx / 2;
  const int y = d.ky * I.vy + I.vy / 2;
  const float* px = lab + 3 * (I.pix_off + (int64_t)y * I.W + x);
  Sp3 q;
  q.mx = x; q.my = y; q.mL = px[0]; q.ma = px[1]; q.mb = px[2];
  const double l2 = I.lam * I.lam;
  q.sxx = (double)I.vx * I.vx; q.sxy = 0.0; q.syy = (double)I.vy * I.vy;
  q.c[0] = l2; q.c[1] = 0.0; q.c[2] = 0.0; q.c[3] = l2; q.c[4] = 0.0; q.c[5] = l2;
  store_row3(P.theta + (size_t)sp * kThetaRow3, q, 0.0);
  write_records3(P, I, d.kx, d.ky, q);
}

__global__ __launch_bounds__(256) void k3_set_params(DevPtrs P, const double* __restrict__ rows) {
  const int sp = blockIdx.x * 256 + threadIdx.x;
  if (sp >= P.n_sp) return;
  const SpDesc d = P.sp[sp];
  const ImgDesc I = P.img[d.img];
  const double* row = rows + (size_t)sp * kThetaRow3;
  const Sp3 q = from_row3(row, I);
  store_row3(P.theta + (size_t)sp * kThetaRow3, q, row[14]);
  write_records3(P, I, d.kx, d.ky, q);
}

// the offsets of t1, t2, u1, u2, u3, read from the wave's LDS block
constexpr int kOffIdx3[5] = {Q_O1, Q_O2, Q_P1, Q_P2, Q_P3};

__device__ __forceinline__ float eval3(const AS4 float* f, const float (&o)[5], float xr, float yr,
                                       float L, float A, float B) {
  const float t1 = fmaf(f[Q_L11], xr, fmaf(f[Q_L12], yr, o[0]));
  const float t2 = fmaf(f[Q_L22], yr, o[1]);
  const float u1 = fmaf(f[Q_U11], L, fmaf(f[Q_U12], A, fmaf(f[Q_U13], B, o[2])));
  const float u2 = fmaf(f[Q_U22], A, fmaf(f[Q_U23], B, o[3]));
  const float u3 = fmaf(f[Q_U33], B, o[4]);
  float l = fmaf(-t1, t1, f[Q_C]);
  l = fmaf(-t2, t2, l);
  l = fmaf(-u1, u1, l);
  l = fmaf(-u2, u2, l);
  l = fmaf(-u3, u3, l);
  return l;
}

enum CellMode3 { C3_STATS = 0, C3_LABEL = 1, C3_EXPORT_R = 2, C3_EXPORT_CAND = 3 };

template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k3_cells(DevPtrs P, const float* __restrict__ lab,
                                                int32_t* __restrict__ out_i,
                                                float* __restrict__ out_f) {
  const int lane = threadIdx.x & 63;
  const int cell = __builtin_amdgcn_readfirstlane(
      (int)(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6)));
  if (cell >= P.n_cell) return;
  const AS4 CellDesc* cdp = cptr(P.cell) + cell;
  const int b = cdp->img, ccx = cdp->cx, ccy = cdp->cy;
  const AS4 ImgDesc* Ip = cptr(P.img) + b;
  if (MODE == C3_STATS && cptr(P.state)[b].done) return;
  const int W = Ip->W, H = Ip->H, vx = Ip->vx, vy = Ip->vy;
  const int x0 = ccx * vx, y0 = ccy * vy;
  const int w = min(vx, W - x0), h = min(vy, H - y0);
  const int npix = w * h;
  const int64_t pix0 = Ip->pix_off + (int64_t)y0 * W + x0;
  const float* img = lab + 3 * pix0;
  const AS4 float* rec0 = cptr(P.rec) + (size_t)cell * (kSlots * kRec3);

  if (MODE == C3_EXPORT_CAND) {
    const int nx = Ip->nx, ny = Ip->ny;
    for (int p = lane; p < npix; p += 64) {
      const int row = p / w, col = p - row * w;
      int32_t* dst = out_i + (size_t)(pix0 + (int64_t)row * W + col) * kSlots;
#pragma unroll
      for (int s = 0; s < kSlots; ++s) {
        const int kx = ccx + (s % 3) - 1, ky = ccy + (s / 3) - 1;
        const bool idx_ok = kx >= 0 && kx < nx && ky >= 0 && ky < ny;
        const bool rec_ok = rec0[s * kRec3 + Q_C] != -INFINITY;
        dst[s] = (idx_ok != rec_ok) ? -2 : (idx_ok ? ky * nx + kx : -1);
      }
    }
    return;
  }

  constexpr int NS = kSlots * kStats3;  // 135
  float acc[NS + 1];
  if (MODE == C3_STATS) {
#pragma unroll
    for (int i = 0; i < NS + 1; ++i) acc[i] = 0.f;
  }
  float llacc = 0.f;
  __shared__ float s_off[kWavesPerBlock * kOffBlock];
  float* woff0 = s_off + (threadIdx.x >> 6) * kOffBlock;
  stage_offsets(woff0, P.rec + (size_t)cell * (kSlots * kRec3), kRec3, kOffIdx3, lane);
  for (int p = lane; p < npix; p += 64) {
    // opaque zero offsets: the records are re-read each round by scalar loads
    // and the offsets by LDS reads, rather than held in (too few) registers
    int zero = 0, vz = 0;
    asm volatile("" : "+s"(zero));
    asm volatile("" : "+v"(vz));
    const AS4 float* rec = rec0 + zero;
    const float* woff = woff0 + vz;
    const int row = p / w, col = p - row * w;
    const float* px = img + 3 * ((int64_t)row * W + col);
    const float L = px[0], A = px[1], B = px[2];
    const float xr = (float)col, yr = (float)row;
    float e[kSlots];
    float sum = 0.f;
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
      float o[5];
      load_offsets(woff, s, o);
      e[s] = __builtin_amdgcn_exp2f(eval3(rec + s * kRec3, o, xr, yr, L, A, B));
      sum += e[s];
    }
    float shift = 0.f;
    if (sum < 0x1p-100f) {
      // every candidate is far away: subtract the largest exponent first
      float lv[kSlots];
      float m = -INFINITY;
#pragma unroll
      for (int s = 0; s < kSlots; ++s) {
        float o[5];
        load_offsets(woff, s, o);
        lv[s] = eval3(rec + s * kRec3, o, xr, yr, L, A, B);
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
    if (MODE == C3_STATS) {
      const float xx = xr * xr, xy = xr * yr, yy = yr * yr;
#pragma unroll
      for (int s = 0; s < kSlots; ++s) {
        const AS4 float* f = rec + s * kRec3;
        float* a = acc + s * kStats3;
        const float R = e[s] * inv;
        const float dL = L - f[Q_ML], da = A - f[Q_MA], db = B - f[Q_MB];
        a[T_N] += R;
        a[T_X] = fmaf(R, xr, a[T_X]);
        a[T_Y] = fmaf(R, yr, a[T_Y]);
        a[T_XX] = fmaf(R, xx, a[T_XX]);
        a[T_XY] = fmaf(R, xy, a[T_XY]);
        a[T_YY] = fmaf(R, yy, a[T_YY]);
        const float rL = R * dL, ra = R * da, rb = R * db;
        a[T_L] += rL;
        a[T_A] += ra;
        a[T_B] += rb;
        a[T_LL] = fmaf(rL, dL, a[T_LL]);
        a[T_LA] = fmaf(rL, da, a[T_LA]);
        a[T_LB] = fmaf(rL, db, a[T_LB]);
        a[T_AA] = fmaf(ra, da, a[T_AA]);
        a[T_AB] = fmaf(ra, db, a[T_AB]);
        a[T_BB] = fmaf(rb, db, a[T_BB]);
      }
    } else if (MODE == C3_LABEL) {
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
  if (MODE == C3_STATS) {
    wave_reduce_scatter<NS>(acc, lane);
    const int r = (int)(__builtin_bitreverse32((unsigned)lane) >> 26);
    double* part = P.part + (size_t)cell * kPart3;
    part[r] = (double)acc[0];
    part[64 + r] = (double)acc[1];
    if (128 + r < NS) part[128 + r] = (double)acc[2];
  }
  if (MODE == C3_STATS || MODE == C3_LABEL) {
    double ll = (double)llacc;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) ll += __shfl_xor(ll, m, 64);
    if (lane == 0) P.llp[cell] = kLn2 * ll + (double)npix * Ip->lncmax;
  }
}

// M-step: fixed-order gather of the window's cell partials, means (Eq.
// UpdateMu), the spatial and the 3x3 colour covariance (Eqs. UpdateSigS,
// UpdateSigC) about the new mean, shape control of both blocks, in FP64
__global__ __launch_bounds__(256) void k3_finalize(DevPtrs P) {
  const int sp = blockIdx.x * 256 + threadIdx.x;
  if (sp >= P.n_sp) return;
  const SpDesc d = P.sp[sp];
  if (P.state[d.img].done) return;
  const ImgDesc I = P.img[d.img];
  double acc[kStats3];
#pragma unroll
  for (int j = 0; j < kStats3; ++j) acc[j] = 0.0;
  for (int dy = -1; dy <= 1; ++dy) {
    for (int dx = -1; dx <= 1; ++dx) {
      const int cx = d.kx - dx, cy = d.ky - dy;
      if (cx < 0 || cx >= I.ncx || cy < 0 || cy >= I.ncy) continue;
      const int slot = 3 * (dy + 1) + (dx + 1);
      const double ox = (double)(-dx) * I.vx, oy = (double)(-dy) * I.vy;
      const double* q = P.part + (size_t)(I.cell_off + cy * I.ncx + cx) * kPart3 + slot * kStats3;
      const double n = q[T_N], sx = q[T_X], sy = q[T_Y];
      acc[T_N] += n;
      acc[T_X] += sx + ox * n;
      acc[T_Y] += sy + oy * n;
      acc[T_XX] += q[T_XX] + 2.0 * ox * sx + ox * ox * n;
      acc[T_XY] += q[T_XY] + ox * sy + oy * sx + ox * oy * n;
      acc[T_YY] += q[T_YY] + 2.0 * oy * sy + oy * oy * n;
#pragma unroll
      for (int j = T_L; j <= T_B; ++j) acc[j] += q[j];
#pragma unroll
      for (int j = T_LL; j <= T_BB; ++j) acc[j] += q[j];
    }
  }
  double* row = P.theta + (size_t)sp * kThetaRow3;
  const double N = acc[T_N];
  if (!(N >= I.n_min)) {
    row[14] = N;  // 0/0 guard: theta_k keeps its value
    return;
  }
  const double iN = 1.0 / N;
  const double mx = acc[T_X] * iN, my = acc[T_Y] * iN;
  const double mL = acc[T_L] * iN, ma = acc[T_A] * iN, mb = acc[T_B] * iN;
  Sp3 q;
  q.mx = (double)d.kx * I.vx + mx;
  q.my = (double)d.ky * I.vy + my;
  // colour moments were taken about the float32 record mean
  q.mL = (double)(float)row[2] + mL;
  q.ma = (double)(float)row[3] + ma;
  q.mb = (double)(float)row[4] + mb;
  const double s_in[6] = {acc[T_XX] * iN - mx * mx, acc[T_XY] * iN - mx * my, 0.0,
                          acc[T_YY] * iN - my * my, 0.0, fmax(I.eps_s, 1.0)};
  double s_out[6];
  clamp3(s_in, I.eps_s, s_out);
  q.sxx = s_out[0]; q.sxy = s_out[1]; q.syy = s_out[3];
  const double c_in[6] = {acc[T_LL] * iN - mL * mL, acc[T_LA] * iN - mL * ma,
                          acc[T_LB] * iN - mL * mb, acc[T_AA] * iN - ma * ma,
                          acc[T_AB] * iN - ma * mb, acc[T_BB] * iN - mb * mb};
  clamp3(c_in, I.eps_c, q.c);
  store_row3(row, q, N);
  write_records3(P, I, d.kx, d.ky, q);
}

inline unsigned blocks_of(size_t n, unsigned per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch3_clear_records(const DevPtrs& P, hipStream_t s) {
  const size_t n = (size_t)P.n_cell * kSlots;
  hipLaunchKernelGGL(k3_clear_records, dim3(blocks_of(n, 256)), dim3(256), 0, s, P.rec, n);
  return hipGetLastError();
}

hipError_t launch3_init_seeds(const DevPtrs& P, const float* lab, hipStream_t s) {
  hipLaunchKernelGGL(k3_init_seeds, dim3(blocks_of(P.n_sp, 256)), dim3(256), 0, s, P, lab);
  return hipGetLastError();
}

hipError_t launch3_set_params(const DevPtrs& P, const double* rows, hipStream_t s) {
  hipLaunchKernelGGL(k3_set_params, dim3(blocks_of(P.n_sp, 256)), dim3(256), 0, s, P, rows);
  return hipGetLastError();
}

hipError_t launch3_cells(const DevPtrs& P, int mode, const float* lab, int32_t* out_i,
                         float* out_f, hipStream_t s) {
  const dim3 grid(blocks_of(P.n_cell, kWavesPerBlock)), blk(256);
  switch (mode) {
    case 0: hipLaunchKernelGGL(k3_cells<C3_STATS>, grid, blk, 0, s, P, lab, out_i, out_f); break;
    case 1: hipLaunchKernelGGL(k3_cells<C3_LABEL>, grid, blk, 0, s, P, lab, out_i, out_f); break;
    case 2: hipLaunchKernelGGL(k3_cells<C3_EXPORT_R>, grid, blk, 0, s, P, lab, out_i, out_f); break;
    default: hipLaunchKernelGGL(k3_cells<C3_EXPORT_CAND>, grid, blk, 0, s, P, lab, out_i, out_f);
  }
  return hipGetLastError();
}

hipError_t launch3_finalize(const DevPtrs& P, hipStream_t s) {
  hipLaunchKernelGGL(k3_finalize, dim3(blocks_of(P.n_sp, 256)), dim3(256), 0, s, P);
  return hipGetLastError();
}

}  // namespace gmmsp
