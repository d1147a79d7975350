// Device functions of the M-step gather (Eqs. UpdateMu .. eigdecrc), the
// record writer and the per-image L(theta^t) reduction, shared by the
// per-pass kernels and the persistent T-mode kernel so that both compute the
// same arithmetic in the same order.
#pragma once

#include "gmmsp_internal.h"
#include "gmmsp_wave.h"

#include <math.h>

namespace gmmsp {

// ---------------------------------------------------------------------------
// FP64 shape control of one symmetric 2x2 block [[a, b], [b, c]]
// (Eqs. eigdecs, mlams, eigdecrs and their colour counterparts): both
// eigenvalues floored at eps, the block rebuilt on the same eigenvectors.
// ---------------------------------------------------------------------------
struct Sym2 {
  double a, b, c, det;
};

__device__ inline Sym2 clamp2(double a, double b, double c, double eps) {
  const double h = 0.5 * (a - c);
  const double r = sqrt(h * h + b * b);
  const double m = 0.5 * (a + c);
  const double l1 = m + r;  // larger eigenvalue
  const double l2 = m - r;  // smaller eigenvalue
  Sym2 o;
  if (l2 >= eps) {
    o.a = a;
    o.b = b;
    o.c = c;
    o.det = a * c - b * b;
    return o;
  }
  const double l1c = fmax(l1, eps);
  if (r > 0.0) {
    // S~ = eps I + (l1c - eps) v v^T, v v^T = (S - l2 I) / (l1 - l2)
    const double inv = 1.0 / (2.0 * r);
    const double d = l1c - eps;
    o.a = eps + d * ((h + r) * inv);
    o.b = d * (b * inv);
    o.c = eps + d * ((r - h) * inv);
  } else {
    o.a = l1c;
    o.b = 0.0;
    o.c = l1c;
  }
  o.det = l1c * eps;
  return o;
}

// FP64 parameters of one superpixel after shape control.
struct SpTheta {
  double mx, my, mL, ma, mb;          // absolute mean
  double sxx, sxy, syy, sLL, saa, sab, sbb;
  double det_s, det_ab;               // determinants of the 2x2 blocks
};

__device__ inline void store_theta_row(double* row, const SpTheta& q, double mass) {
  row[0] = q.mx;  row[1] = q.my;  row[2] = q.mL;  row[3] = q.ma;  row[4] = q.mb;
  row[5] = q.sxx; row[6] = q.sxy; row[7] = q.syy; row[8] = q.sLL;
  row[9] = q.saa; row[10] = q.sab; row[11] = q.sbb; row[12] = mass;
}

// The float32 record of superpixel (kx, ky) for the cell (kx - dx, ky - dy),
// in which it is candidate slot 3 (dy + 1) + (dx + 1); nothing if that cell is
// outside the grid.
__device__ inline void write_record_slot(const DevPtrs& P, const ImgDesc& I, int kx, int ky,
                                         const SpTheta& q, int dx, int dy) {
  const int cx = kx - dx, cy = ky - dy;
  if (cx < 0 || cx >= I.ncx || cy < 0 || cy >= I.ncy) return;
  const int slot = 3 * (dy + 1) + (dx + 1);
  const double s2 = sqrt(0.5 * kLog2e);  // l in log2 units: l = c - |whitened d|^2
  // spatial block: P_s = Sigma_s^-1, factored as t1^2 + t2^2
  const double l11 = s2 * sqrt(q.syy / q.det_s);
  const double l12 = -s2 * q.sxy / sqrt(q.det_s * q.syy);
  const double l22 = s2 / sqrt(q.syy);
  const double sL = s2 / sqrt(q.sLL);
  const double a11 = s2 * sqrt(q.sbb / q.det_ab);
  const double a12 = -s2 * q.sab / sqrt(q.det_ab * q.sbb);
  const double a22 = s2 / sqrt(q.sbb);
  const double lndet = log(q.det_s) + log(q.sLL) + log(q.det_ab);
  const double c = kLog2e * (-2.5 * kLn2Pi - 0.5 * lndet - I.lncmax);
  // spatial offsets about the cell origin
  const double mxs = q.mx - (double)cx * I.vx;
  const double mys = q.my - (double)cy * I.vy;
  float r[kRecFloats];
  r[R_L11] = (float)l11;
  r[R_L12] = (float)l12;
  r[R_O1] = (float)(-(l11 * mxs + l12 * mys));
  r[R_O2] = (float)(-l22 * mys);
  r[R_L22] = (float)l22;
  r[R_SL] = (float)sL;
  r[R_O3] = (float)(-(a11 * q.ma + a12 * q.mb));
  r[R_O4] = (float)(-a22 * q.mb);
  r[R_OL] = (float)(-sL * q.mL);
  r[R_A11] = (float)a11;
  r[R_A12] = (float)a12;
  r[R_A22] = (float)a22;
  r[R_C] = (float)c;
  r[R_ML] = (float)q.mL;
  r[R_MA] = (float)q.ma;
  r[R_MB] = (float)q.mb;
  float4* dst = reinterpret_cast<float4*>(P.rec + rec_index(P.n_cell, I.cell_off + cy * I.ncx + cx, slot));
#pragma unroll
  for (int j = 0; j < kRecFloats / 4; ++j)
    dst[j] = make_float4(r[4 * j], r[4 * j + 1], r[4 * j + 2], r[4 * j + 3]);
}

// All (up to) nine records of superpixel (kx, ky), one thread.
__device__ inline void write_records(const DevPtrs& P, const ImgDesc& I, int kx, int ky,
                                     const SpTheta& q) {
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) write_record_slot(P, I, kx, ky, q, dx, dy);
}

__device__ inline SpTheta theta_from_row(const double* row, const ImgDesc& I) {
  SpTheta q;
  q.mx = row[0]; q.my = row[1]; q.mL = row[2]; q.ma = row[3]; q.mb = row[4];
  const Sym2 s = clamp2(row[5], row[6], row[7], I.eps_s);
  const Sym2 ab = clamp2(row[9], row[10], row[11], I.eps_c);
  q.sxx = s.a; q.sxy = s.b; q.syy = s.c; q.det_s = s.det;
  q.sLL = fmax(row[8], I.eps_c);
  q.saa = ab.a; q.sab = ab.b; q.sbb = ab.c; q.det_ab = ab.det;
  return q;
}

// ---------------------------------------------------------------------------
// L(theta^t) per image and the stop rule; one block per image
// ---------------------------------------------------------------------------
constexpr int kLLThreads = 256;

// L(theta^t) of image b from its cell waves' terms, committed in `mode` (see
// ll_commit); one block of kLLThreads threads.  Fixed order: thread i adds
// cells i, i + kLLThreads, ... of each wave set in turn, then a fixed tree.
// With LL_EM an image that has stopped is skipped.
__device__ inline void ll_reduce_block(const DevPtrs& P, int b, double rel_tol, int mode,
                                       int nsub) {
  __shared__ double red[kLLThreads];
  const ImgDesc* I = P.img + b;
  if (mode == LL_EM && P.state[b].done) return;
  const int ncells = I->ncells;
  double s = 0.0;
  for (int u = 0; u < nsub; ++u) {
    const double* llp = P.llp + (size_t)u * P.n_cell + I->cell_off;
    for (int c = threadIdx.x; c < ncells; c += kLLThreads) s += llp[c];
  }
  red[threadIdx.x] = s;
  __syncthreads();
#pragma unroll
  for (int o = kLLThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) ll_commit(P, b, red[0], mode, rel_tol);
}

// ---------------------------------------------------------------------------
// M-step: per superpixel gather of the window's cell partials in a fixed
// order, mean (Eq. UpdateMu), block covariances (Eqs. UpdateSigS, UpdateSigC)
// and shape control (Eqs. eigdecs .. eigdecrc), all in FP64.
// ---------------------------------------------------------------------------
// The statistics of slot (dx, dy) of the window cell (kx - dx, ky - dy), every
// wave set of it in order, added to acc with the spatial moments moved from the
// cell origin to the superpixel's own cell origin: x' = x + ox, ox = (cx - kx) v_x.
__device__ inline void add_cell_stats(const DevPtrs& P, const ImgDesc& I, int kx, int ky, int dx,
                                      int dy, double (&acc)[kStats]) {
  const int cx = kx - dx, cy = ky - dy;
  if (cx < 0 || cx >= I.ncx || cy < 0 || cy >= I.ncy) return;
  const int slot = 3 * (dy + 1) + (dx + 1);
  const double ox = (double)(-dx) * I.vx, oy = (double)(-dy) * I.vy;
  for (int u = 0; u < P.wpc; ++u) {
    const float* q = reinterpret_cast<const float*>(P.part) +
                     ((size_t)u * P.n_cell + I.cell_off + cy * I.ncx + cx) * kPartStride +
                     slot * kStats;
    const double n = q[S_N], sx = q[S_X], sy = q[S_Y];
    acc[S_N] += n;
    acc[S_X] += sx + ox * n;
    acc[S_Y] += sy + oy * n;
    acc[S_L] += q[S_L];
    acc[S_A] += q[S_A];
    acc[S_B] += q[S_B];
    acc[S_XX] += q[S_XX] + 2.0 * ox * sx + ox * ox * n;
    acc[S_XY] += q[S_XY] + ox * sy + oy * sx + ox * oy * n;
    acc[S_YY] += q[S_YY] + 2.0 * oy * sy + oy * oy * n;
    acc[S_LL] += q[S_LL];
    acc[S_AA] += q[S_AA];
    acc[S_AB] += q[S_AB];
    acc[S_BB] += q[S_BB];
  }
}

// Colour factors of a superpixel's record (its own cell, slot 4), in FP64:
// w = SL L + OL, u1 = A11 a + A12 b + O3, u2 = A22 b + O4.  The slot-lane
// statistics pass takes the colour moments in these coordinates.
struct ColourFrame {
  double sl, ol, a11, a12, a22, o3, o4;
};

__device__ inline ColourFrame colour_frame(const DevPtrs& P, const ImgDesc& I, const SpDesc& d) {
  const float* f = P.rec + rec_index(P.n_cell, I.cell_off + d.ky * I.ncx + d.kx, 4);
  return ColourFrame{f[R_SL], f[R_OL], f[R_A11], f[R_A12], f[R_A22], f[R_O3], f[R_O4]};
}

// theta^{t+1} of superpixel d from its window statistics: the mean (Eq.
// UpdateMu), the block covariances about it (Eqs. UpdateSigS, UpdateSigC) and
// the shape control; false when the mass is below n_min (theta^t is kept).
// The colour moments are about the superpixel's float32 mean (row: its FP64
// master row), or, with cf, whitened moments in the frame cf, which are mapped
// back to Lab first: d_L = w / SL, d_b = u2 / A22, d_a = (u1 - A12 d_b) / A11,
// about the colour at which w, u1 and u2 vanish.
__device__ inline bool theta_from_stats(double (&acc)[kStats], const SpDesc& d,
                                        const ImgDesc& I, const double* row, SpTheta& q,
                                        const ColourFrame* cf) {
  const double N = acc[S_N];
  if (!(N >= I.n_min)) return false;
  double oL, oa, ob;
  if (cf) {
    const double k = cf->a12 / cf->a22;
    const double sw = acc[S_L], s1 = acc[S_A], s2 = acc[S_B];
    const double sww = acc[S_LL], s11 = acc[S_AA], s12 = acc[S_AB], s22 = acc[S_BB];
    acc[S_L] = sw / cf->sl;
    acc[S_B] = s2 / cf->a22;
    acc[S_A] = (s1 - k * s2) / cf->a11;
    acc[S_LL] = sww / (cf->sl * cf->sl);
    acc[S_BB] = s22 / (cf->a22 * cf->a22);
    acc[S_AB] = (s12 - k * s22) / (cf->a11 * cf->a22);
    acc[S_AA] = (s11 - 2.0 * k * s12 + k * k * s22) / (cf->a11 * cf->a11);
    oL = -cf->ol / cf->sl;
    ob = -cf->o4 / cf->a22;
    oa = (-cf->o3 - cf->a12 * ob) / cf->a11;
  } else {
    oL = (double)(float)row[2];
    oa = (double)(float)row[3];
    ob = (double)(float)row[4];
  }
  const double iN = 1.0 / N;
  const double mx = acc[S_X] * iN, my = acc[S_Y] * iN;
  const double mL = acc[S_L] * iN, ma = acc[S_A] * iN, mb = acc[S_B] * iN;
  q.mx = (double)d.kx * I.vx + mx;
  q.my = (double)d.ky * I.vy + my;
  q.mL = oL + mL;
  q.ma = oa + ma;
  q.mb = ob + mb;
  const Sym2 s = clamp2(acc[S_XX] * iN - mx * mx, acc[S_XY] * iN - mx * my,
                        acc[S_YY] * iN - my * my, I.eps_s);
  const Sym2 c = clamp2(acc[S_AA] * iN - ma * ma, acc[S_AB] * iN - ma * mb,
                        acc[S_BB] * iN - mb * mb, I.eps_c);
  q.sxx = s.a; q.sxy = s.b; q.syy = s.c; q.det_s = s.det;
  q.sLL = fmax(acc[S_LL] * iN - mL * mL, I.eps_c);
  q.saa = c.a; q.sab = c.b; q.sbb = c.c; q.det_ab = c.det;
  return true;
}

// theta^{t+1} of superpixel sp, one thread: the window cells in fixed (dy, dx)
// order, then the row and the (up to) nine records.
__device__ inline void finalize_one(const DevPtrs& P, int sp) {
  if (sp >= P.n_sp) return;
  const SpDesc d = P.sp[sp];
  if (P.state[d.img].done) return;
  const ImgDesc I = P.img[d.img];
  double acc[kStats];
#pragma unroll
  for (int j = 0; j < kStats; ++j) acc[j] = 0.0;
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) add_cell_stats(P, I, d.kx, d.ky, dx, dy, acc);
  double* row = P.theta + (size_t)sp * kThetaRow;
  SpTheta q;
  ColourFrame cf;
  if (P.estep == 1) cf = colour_frame(P, I, d);
  if (!theta_from_stats(acc, d, I, row, q, P.estep == 1 ? &cf : nullptr)) {
    row[12] = acc[S_N];  // 0/0 guard: theta_k keeps its value
    return;
  }
  store_theta_row(row, q, acc[S_N]);
  write_records(P, I, d.kx, d.ky, q);
}

// theta^{t+1} of superpixel sp with G lanes (G = 4 or 16, lane = 0 .. G-1 of
// an aligned group of the wave): lane j reads window cells j, j + G, ... in
// that order, the G lanes add in a fixed butterfly order, every lane forms
// theta, and lane j writes the records of cells j, j + G, ...  The sums group
// differently from finalize_one, so the two agree up to FP64 rounding; each is
// bitwise repeatable.  The whole group leaves together.
template <int G>
__device__ inline void finalize_group(const DevPtrs& P, int sp, int lane) {
  static_assert(G == 4 || G == 16, "4 or 16 lanes per superpixel");
  if (sp >= P.n_sp) return;
  const SpDesc d = P.sp[sp];
  if (P.state[d.img].done) return;
  const ImgDesc I = P.img[d.img];
  double acc[kStats];
#pragma unroll
  for (int j = 0; j < kStats; ++j) acc[j] = 0.0;
  for (int c = lane; c < kSlots; c += G) add_cell_stats(P, I, d.kx, d.ky, c % 3 - 1, c / 3 - 1, acc);
#pragma unroll
  for (int m = 1; m < G; m <<= 1)
#pragma unroll
    for (int j = 0; j < kStats; ++j) acc[j] += __shfl_xor(acc[j], m, G);
  double* row = P.theta + (size_t)sp * kThetaRow;
  SpTheta q;
  ColourFrame cf;
  if (P.estep == 1) cf = colour_frame(P, I, d);
  const bool ok = theta_from_stats(acc, d, I, row, q, P.estep == 1 ? &cf : nullptr);
  if (!ok) {
    if (lane == 0) row[12] = acc[S_N];  // 0/0 guard: theta_k keeps its value
    return;
  }
  // every lane has read row[2..4] and the record's colour frame before lane 0
  // rewrites the row and the lanes rewrite the records
  __builtin_amdgcn_wave_barrier();
  if (lane == 0) store_theta_row(row, q, acc[S_N]);
  for (int c = lane; c < kSlots; c += G) write_record_slot(P, I, d.kx, d.ky, q, c % 3 - 1, c / 3 - 1);
}

// Block `blk` of the gather launch (256 threads; superpixels blk * 256 / G ..),
// with G = P.glanes.
__device__ inline void finalize_block(const DevPtrs& P, int blk) {
  if (P.glanes == 16)
    finalize_group<16>(P, blk * 16 + (int)threadIdx.x / 16, threadIdx.x & 15);
  else if (P.glanes == 4)
    finalize_group<4>(P, blk * 64 + (int)threadIdx.x / 4, threadIdx.x & 3);
  else
    finalize_one(P, blk * 256 + (int)threadIdx.x);
}

}  // namespace gmmsp
