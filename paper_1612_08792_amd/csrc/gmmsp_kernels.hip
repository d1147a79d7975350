// HIP kernels (gfx950) of the GMM superpixel EM: E-step with fused M-step
// statistics, log-likelihood reduction with the stop rule, per-superpixel
// gather and FP64 shape control, initialisation and labelling.
//
// Work decomposition.  The image is cut into v_x x v_y pixel cells (plus the
// partial remainder column / row).  All pixels of a cell share the same
// candidate set K_i: the superpixels of the 3 x 3 neighbouring seed cells
// (Eq. Ik), so one 64-lane wave owns one cell, reads its nine cell-slot records
// with scalar loads, evaluates the E-step of each pixel in registers and keeps
// the 9 x 13 sufficient statistics of the M-step in registers.  A butterfly
// reduce-scatter across the wave leaves two totals per lane, written in FP64 as
// the cell's partials.  Superpixel k then sums the partials of the (at most)
// nine cells of its window I_k in a fixed order: no atomics, bitwise
// repeatable.
#include "gmmsp_gather.h"
#include "gmmsp_internal.h"
#include "gmmsp_wave.h"

#include <math.h>

namespace gmmsp {

// ---------------------------------------------------------------------------
// Set-up kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_clear_records(float* rec, size_t n_rec) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n_rec) return;
  float4* d = reinterpret_cast<float4*>(rec + i * kRecFloats);
  d[0] = make_float4(0.f, 0.f, 0.f, 0.f);
  d[1] = d[0];
  d[2] = d[0];
  d[3] = make_float4(-INFINITY, 0.f, 0.f, 0.f);
}

__global__ __launch_bounds__(256) void k_reset_state(DevPtrs P) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b == 0) *P.n_done = 0;
  if (b >= P.n_img) return;
  ImgState* st = P.state + b;
  st->t = 0;
  st->done = 0;
  st->iters = 0;
  st->ll_final = 0.0;
}

// Sec. III-C: mu_k = z_j at the seed pixel, Sigma_s = diag(v_x^2, v_y^2),
// colour variances lambda^2.  With `guarded`, only the images whose
// L(theta^0) (ll_final) is below the seeds' (ll_seed) or not finite are
// re-seeded, and every image's fallback flag records the choice.
__device__ inline void seed_superpixel(DevPtrs& P, const float* __restrict__ lab, int sp,
                                       const SpDesc& d, const ImgDesc& I) {
  const int x = d.kx * I.vx + I.vx / 2;
  const int y = d.ky * I.vy + I.vy / 2;
  const float* px = lab + 3 * (I.pix_off + (int64_t)y * I.W + x);
  SpTheta q;
  q.mx = x; q.my = y; q.mL = px[0]; q.ma = px[1]; q.mb = px[2];
  const double l2 = I.lam * I.lam;
  q.sxx = (double)I.vx * I.vx; q.sxy = 0.0; q.syy = (double)I.vy * I.vy;
  q.sLL = l2; q.saa = l2; q.sab = 0.0; q.sbb = l2;
  q.det_s = q.sxx * q.syy;
  q.det_ab = l2 * l2;
  store_theta_row(P.theta + (size_t)sp * kThetaRow, q, 0.0);
  write_records(P, I, d.kx, d.ky, q);
}

__global__ __launch_bounds__(256) void k_init_seeds(DevPtrs P, const float* __restrict__ lab,
                                                    int guarded) {
  const int sp = blockIdx.x * 256 + threadIdx.x;
  if (sp >= P.n_sp) return;
  const SpDesc d = P.sp[sp];
  const ImgDesc I = P.img[d.img];
  if (guarded) {
    ImgState* st = P.state + d.img;
    const bool keep = st->ll_final >= st->ll_seed;  // false for NaN
    if (d.kx == 0 && d.ky == 0) st->fallback = keep ? 0 : 1;
    if (keep) return;
  }
  seed_superpixel(P, lab, sp, d, I);
}

__global__ __launch_bounds__(256) void k_set_params(DevPtrs P, const double* __restrict__ rows) {
  const int sp = blockIdx.x * 256 + threadIdx.x;
  if (sp >= P.n_sp) return;
  const SpDesc d = P.sp[sp];
  const ImgDesc I = P.img[d.img];
  const double* row = rows + (size_t)sp * kThetaRow;
  const SpTheta q = theta_from_row(row, I);
  store_theta_row(P.theta + (size_t)sp * kThetaRow, q, row[12]);
  write_records(P, I, d.kx, d.ky, q);
}

// ---------------------------------------------------------------------------
// Per-cell E-step kernel
// ---------------------------------------------------------------------------

enum CellMode { M_STATS = 0, M_LABEL = 1, M_EXPORT_R = 2, M_EXPORT_CAND = 3 };

// log2 p(z; theta_k) - cmax2 for the record at f (Eq. gaussian, block diagonal)
__device__ __forceinline__ float eval_l(const AS4 float* f, float xr, float yr, float L,
                                        float A, float B) {
  const float t1 = fmaf(f[R_L11], xr, fmaf(f[R_L12], yr, f[R_O1]));
  const float t2 = fmaf(f[R_L22], yr, f[R_O2]);
  const float w = fmaf(f[R_SL], L, f[R_OL]);
  const float u1 = fmaf(f[R_A11], A, fmaf(f[R_A12], B, f[R_O3]));
  const float u2 = fmaf(f[R_A22], B, f[R_O4]);
  float l = fmaf(-t1, t1, f[R_C]);
  l = fmaf(-t2, t2, l);
  l = fmaf(-w, w, l);
  l = fmaf(-u1, u1, l);
  l = fmaf(-u2, u2, l);
  return l;
}

// 3 waves per SIMD measured fastest for the statistics pass (168 VGPRs)
#define CELLS_ATTR __attribute__((amdgpu_waves_per_eu(3)))

// E-step of NP pixels per lane against the nine records of the wave's cell:
// e[p][s] is proportional to R_(i_p, s) (Eq. Rik), sum[p] = sum_s e[p][s], and
// shift[p] is the log2 offset of e (0 unless all nine densities underflowed).
// Each record value is read once (scalar load) for all NP pixels; with kLdsOff
// the offsets (O1, O2, O3, O4, OL) come from the wave's LDS block loff (the
// statistics pass), otherwise from the records.

// log2 p(z; theta_k) - cmax2 with the five offsets in vector registers
__device__ __forceinline__ float eval_l_o(const AS4 float* f, float o1, float o2, float oL,
                                          float o3, float o4, float xr, float yr, float L,
                                          float A, float B) {
  const float t1 = fmaf(f[R_L11], xr, fmaf(f[R_L12], yr, o1));
  const float t2 = fmaf(f[R_L22], yr, o2);
  const float w = fmaf(f[R_SL], L, oL);
  const float u1 = fmaf(f[R_A11], A, fmaf(f[R_A12], B, o3));
  const float u2 = fmaf(f[R_A22], B, o4);
  float l = fmaf(-t1, t1, f[R_C]);
  l = fmaf(-t2, t2, l);
  l = fmaf(-w, w, l);
  l = fmaf(-u1, u1, l);
  l = fmaf(-u2, u2, l);
  return l;
}

template <int NP, bool kLdsOff = false>
__device__ __forceinline__ void estep_pixels(const AS4 float* rec, size_t rs, const float (&xr)[NP],
                                             const float (&yr)[NP], const float (&L)[NP],
                                             const float (&A)[NP], const float (&B)[NP],
                                             float (&e)[NP][kSlots], float (&sum)[NP],
                                             float (&shift)[NP], const float* loff = nullptr) {
#pragma unroll
  for (int p = 0; p < NP; ++p) sum[p] = 0.f;
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    const AS4 float* f = rec + s * rs;
    float l[NP];
    if constexpr (kLdsOff) {
      float o[5];
      load_offsets(loff, s, o);
#pragma unroll
      for (int p = 0; p < NP; ++p)
        l[p] = eval_l_o(f, o[0], o[1], o[4], o[2], o[3], xr[p], yr[p], L[p], A[p], B[p]);
    } else {
#pragma unroll
      for (int p = 0; p < NP; ++p) l[p] = eval_l(f, xr[p], yr[p], L[p], A[p], B[p]);
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      e[p][s] = __builtin_amdgcn_exp2f(l[p]);
      sum[p] += e[p][s];
    }
  }
  // one branch for all NP pixels, so the compiler keeps their evaluations together
  float smin = sum[0];
#pragma unroll
  for (int p = 1; p < NP; ++p) smin = fminf(smin, sum[p]);
#pragma unroll
  for (int p = 0; p < NP; ++p) shift[p] = 0.f;
  if (smin < 0x1p-100f) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      if (sum[p] < 0x1p-100f) {
        // every candidate is far away: subtract the largest exponent first
        float lv[kSlots];
        float m = -INFINITY;
#pragma unroll
        for (int s = 0; s < kSlots; ++s) {
          lv[s] = eval_l(rec + s * rs, xr[p], yr[p], L[p], A[p], B[p]);
          m = fmaxf(m, lv[s]);
        }
        float t = 0.f;
#pragma unroll
        for (int s = 0; s < kSlots; ++s) {
          e[p][s] = __builtin_amdgcn_exp2f(lv[s] - m);
          t += e[p][s];
        }
        sum[p] = t;
        shift[p] = m;
      }
    }
  }
}

// M-step sufficient statistics of NP pixels (weights inv[p] = 1 / sum[p], or 0
// for a masked pixel) added to the 9 x 13 per-lane accumulators.
template <int NP>
__device__ __forceinline__ void accumulate_stats(const AS4 float* rec, size_t rs, float* acc,
                                                 const float (&e)[NP][kSlots],
                                                 const float (&inv)[NP], const float (&xr)[NP],
                                                 const float (&yr)[NP], const float (&L)[NP],
                                                 const float (&A)[NP], const float (&B)[NP]) {
  float xx[NP], xy[NP], yy[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    xx[p] = xr[p] * xr[p];
    xy[p] = xr[p] * yr[p];
    yy[p] = yr[p] * yr[p];
  }
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    const AS4 float* f = rec + s * rs;
    const float mL = f[R_ML], ma = f[R_MA], mb = f[R_MB];
    float* a = acc + s * kStats;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const float R = e[p][s] * inv[p];
      a[S_N] += R;
      a[S_X] = fmaf(R, xr[p], a[S_X]);
      a[S_Y] = fmaf(R, yr[p], a[S_Y]);
      a[S_XX] = fmaf(R, xx[p], a[S_XX]);
      a[S_XY] = fmaf(R, xy[p], a[S_XY]);
      a[S_YY] = fmaf(R, yy[p], a[S_YY]);
      const float dL = L[p] - mL;
      const float da = A[p] - ma;
      const float db = B[p] - mb;
      const float rL = R * dL;
      a[S_L] += rL;
      a[S_LL] = fmaf(rL, dL, a[S_LL]);
      const float ra = R * da;
      a[S_A] += ra;
      a[S_AA] = fmaf(ra, da, a[S_AA]);
      a[S_AB] = fmaf(ra, db, a[S_AB]);
      const float rb = R * db;
      a[S_B] += rb;
      a[S_BB] = fmaf(rb, db, a[S_BB]);
    }
  }
}

// advance a lane's (row, col) inside a cell of width w by the step (dr, dc)
__device__ __forceinline__ void advance(int& row, int& col, int dr, int dc, int w) {
  col += dc;
  row += dr;
  if (col >= w) {
    col -= w;
    row += 1;
  }
}

template <int MODE, int WPC = 1>
__global__ __launch_bounds__(256) CELLS_ATTR void k_cells(DevPtrs P, const float* __restrict__ lab,
                                                          int32_t* __restrict__ out_i,
                                                          float* __restrict__ out_f) {
  const int lane = threadIdx.x & 63;
  // the statistics pass may share a cell among WPC waves (wave sub takes the
  // pixel rounds sub, sub + WPC, ...); the other modes use one wave per cell
  constexpr int wpc = WPC;
  const int gw = __builtin_amdgcn_readfirstlane(
      (int)(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6)));
  const int cell = __builtin_amdgcn_readfirstlane(gw / wpc);
  const int sub = __builtin_amdgcn_readfirstlane(gw - cell * wpc);
  if (cell >= P.n_cell) return;
  const AS4 CellDesc* cdp = cptr(P.cell) + cell;
  const int b = cdp->img, ccx = cdp->cx, ccy = cdp->cy;
  const AS4 ImgDesc* Ip = cptr(P.img) + b;
  if (MODE == M_STATS && cptr(P.state)[b].done) return;
  const int W = Ip->W, H = Ip->H, vx = Ip->vx, vy = Ip->vy;
  const int x0 = ccx * vx, y0 = ccy * vy;
  const int w = min(vx, W - x0), h = min(vy, H - y0);
  const int npix = w * h;
  const int64_t pix0 = Ip->pix_off + (int64_t)y0 * W + x0;
  const float* img = lab + 3 * pix0;
  // the cell's slot-0 record; slot s is s * rs floats further (rec_index)
  const AS4 float* rec0 = cptr(P.rec) + rec_index(P.n_cell, cell, 0);
  const AS4 float* rec = rec0;
  const size_t rs = (size_t)P.n_cell * kRecFloats;

  if (MODE == M_EXPORT_CAND) {
    const int nx = Ip->nx, ny = Ip->ny;
    for (int p = lane; p < npix; p += 64) {
      const int row = p / w, col = p - row * w;
      int32_t* dst = out_i + (size_t)(pix0 + (int64_t)row * W + col) * kSlots;
#pragma unroll
      for (int s = 0; s < kSlots; ++s) {
        const int kx = ccx + (s % 3) - 1, ky = ccy + (s / 3) - 1;
        const bool idx_ok = kx >= 0 && kx < nx && ky >= 0 && ky < ny;
        const bool rec_ok = rec[s * rs + R_C] != -INFINITY;
        dst[s] = (idx_ok != rec_ok) ? -2 : (idx_ok ? ky * nx + kx : -1);
      }
    }
    return;
  }

  float llacc = 0.f;

  if (MODE == M_STATS) {
    // 117 statistics plus one zero pad, so every butterfly step reads pairs
    float acc[kSlots * kStats + 1];
#pragma unroll
    for (int i = 0; i < kSlots * kStats + 1; ++i) acc[i] = 0.f;
    // Rounds of 128 pixels: lane l takes pixels 128 r + l and 128 r + 64 + l.
    // Rounds that hold more than 64 pixels run as pairs (the second pixel of a
    // lane masked past the end); a last round of at most 64 pixels runs after
    // the loop, one pixel per lane, so the loop body has a single path and the
    // accumulators stay in place.
    const int q0 = 128 * sub + lane;  // this wave's first pixel
    int r1 = q0 / w, c1 = q0 - r1 * w;
    int r2 = (q0 + 64) / w, c2 = (q0 + 64) - r2 * w;
    const int step = 128 * wpc;
    const int dr = step / w, dc = step - (step / w) * w;
    const int n_pair = npix > 64 ? (npix - 64 + 127) >> 7 : 0;  // rounds with base + 64 < npix
    // the nine slots' offsets in this wave's own LDS block
    __shared__ float s_off[kWavesPerBlock * kOffBlock];
    float* woff = s_off + (threadIdx.x >> 6) * kOffBlock;
    constexpr int kOffIdx[5] = {R_O1, R_O2, R_O3, R_O4, R_OL};
    stage_offsets(woff, P.rec + rec_index(P.n_cell, cell, 0), rs, kOffIdx, lane);
    for (int rd = sub; rd < n_pair; rd += wpc) {
      const int base = rd << 7;
      // The 144 record floats do not fit the scalar registers; an opaque zero
      // offset keeps the compiler from hoisting them out of the loop, so each
      // round re-reads them with scalar loads instead of spilling them to
      // vector-register lanes.
      int zero = 0;
      asm volatile("" : "+s"(zero));
      const AS4 float* rec = rec0 + zero;
      const bool v2 = base + 64 + lane < npix;
      const float* q1 = img + 3 * ((int64_t)r1 * W + c1);
      const float* q2 = img + (v2 ? 3 * ((int64_t)r2 * W + c2) : 3 * ((int64_t)r1 * W + c1));
      const float L[2] = {q1[0], q2[0]}, A[2] = {q1[1], q2[1]}, B[2] = {q1[2], q2[2]};
      const float xr[2] = {(float)c1, (float)c2}, yr[2] = {(float)r1, (float)r2};
      float e[2][kSlots], sum[2], shift[2];
      // likewise an opaque zero keeps the LDS offsets from being hoisted into
      // 45 vector registers
      int vz = 0;
      asm volatile("" : "+v"(vz));
      estep_pixels<2, true>(rec, rs, xr, yr, L, A, B, e, sum, shift, woff + vz);
      const float inv[2] = {__builtin_amdgcn_rcpf(sum[0]), v2 ? __builtin_amdgcn_rcpf(sum[1]) : 0.f};
      llacc += __builtin_amdgcn_logf(sum[0]) + shift[0];
      llacc += v2 ? __builtin_amdgcn_logf(sum[1]) + shift[1] : 0.f;
      accumulate_stats<2>(rec, rs, acc, e, inv, xr, yr, L, A, B);
      advance(r1, c1, dr, dc, w);
      advance(r2, c2, dr, dc, w);
    }
    // the last round (at most 64 pixels) falls to the wave whose turn it is
    if (n_pair % wpc == sub && (n_pair << 7) + lane < npix) {
      const float* q1 = img + 3 * ((int64_t)r1 * W + c1);
      const float xr[1] = {(float)c1}, yr[1] = {(float)r1};
      const float L[1] = {q1[0]}, A[1] = {q1[1]}, B[1] = {q1[2]};
      float e[1][kSlots], sum[1], shift[1];
      estep_pixels<1, true>(rec, rs, xr, yr, L, A, B, e, sum, shift, woff);
      const float inv[1] = {__builtin_amdgcn_rcpf(sum[0])};
      llacc += __builtin_amdgcn_logf(sum[0]) + shift[0];
      accumulate_stats<1>(rec, rs, acc, e, inv, xr, yr, L, A, B);
    }
    wave_reduce_scatter<kSlots * kStats>(acc, lane);
    const int r = (int)(__builtin_bitreverse32((unsigned)lane) >> 26);
    // the FP32 wave totals, stored as they are; the gather adds them in FP64
    float* part = reinterpret_cast<float*>(P.part) + ((size_t)sub * P.n_cell + cell) * kPartStride;
    part[r] = acc[0];
    if (64 + r < kSlots * kStats) part[64 + r] = acc[1];
  } else if (MODE == M_LABEL) {
    // Eq. obtLi: rounds of 128 pixels, two per lane as in the statistics pass
    // (the second masked past the end; a masked pixel evaluates the cell's
    // first pixel and is neither stored nor counted)
    __shared__ float s_off[kWavesPerBlock * kOffBlock];
    float* woff = s_off + (threadIdx.x >> 6) * kOffBlock;
    constexpr int kOffIdx[5] = {R_O1, R_O2, R_O3, R_O4, R_OL};
    stage_offsets(woff, P.rec + rec_index(P.n_cell, cell, 0), rs, kOffIdx, lane);
    int r1 = lane / w, c1 = lane - r1 * w;
    int r2 = (lane + 64) / w, c2 = (lane + 64) - r2 * w;
    const int dr = 128 / w, dc = 128 - (128 / w) * w;
    const int nx = Ip->nx;
    for (int base = 0; base < npix; base += 128) {
      int zero = 0;
      asm volatile("" : "+s"(zero));
      const AS4 float* rec = rec0 + zero;
      const bool v1 = base + lane < npix, v2 = base + 64 + lane < npix;
      const int y1 = v1 ? r1 : 0, x1 = v1 ? c1 : 0;
      const int y2 = v2 ? r2 : y1, x2 = v2 ? c2 : x1;
      const float* q1 = img + 3 * ((int64_t)y1 * W + x1);
      const float* q2 = img + 3 * ((int64_t)y2 * W + x2);
      const float L[2] = {q1[0], q2[0]}, A[2] = {q1[1], q2[1]}, B[2] = {q1[2], q2[2]};
      const float xr[2] = {(float)x1, (float)x2}, yr[2] = {(float)y1, (float)y2};
      float e[2][kSlots], sum[2], shift[2];
      int vz = 0;
      asm volatile("" : "+v"(vz));
      estep_pixels<2, true>(rec, rs, xr, yr, L, A, B, e, sum, shift, woff + vz);
      int best[2];
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        // the largest posterior, ties to the smallest k (slots ascend in k
        // and the comparison is strict)
        best[p] = 0;
        float be = e[p][0];
#pragma unroll
        for (int s = 1; s < kSlots; ++s) {
          if (e[p][s] > be) {
            be = e[p][s];
            best[p] = s;
          }
        }
      }
      if (v1)
        out_i[pix0 + (int64_t)y1 * W + x1] =
            (ccy + best[0] / 3 - 1) * nx + (ccx + best[0] % 3 - 1);
      if (v2)
        out_i[pix0 + (int64_t)y2 * W + x2] =
            (ccy + best[1] / 3 - 1) * nx + (ccx + best[1] % 3 - 1);
      llacc += v1 ? __builtin_amdgcn_logf(sum[0]) + shift[0] : 0.f;
      llacc += v2 ? __builtin_amdgcn_logf(sum[1]) + shift[1] : 0.f;
      advance(r1, c1, dr, dc, w);
      advance(r2, c2, dr, dc, w);
    }
  } else {
    // the posteriors R (export), one pixel per lane per step of 64
    int row = lane / w, col = lane - (lane / w) * w;
    const int drow = 64 / w, dcol = 64 - (64 / w) * w;
    for (int p = lane; p < npix; p += 64) {
      const float* px = img + 3 * ((int64_t)row * W + col);
      const float xr[1] = {(float)col}, yr[1] = {(float)row};
      const float L[1] = {px[0]}, A[1] = {px[1]}, B[1] = {px[2]};
      float e[1][kSlots], sum[1], shift[1];
      estep_pixels<1>(rec, rs, xr, yr, L, A, B, e, sum, shift);
      const float inv = __builtin_amdgcn_rcpf(sum[0]);
      float* dst = out_f + (size_t)(pix0 + (int64_t)row * W + col) * kSlots;
#pragma unroll
      for (int s = 0; s < kSlots; ++s) dst[s] = e[0][s] * inv;
      advance(row, col, drow, dcol, w);
    }
  }

  if (MODE == M_STATS || MODE == M_LABEL) {
    // cell log-likelihood: sum_i ln sum_k p = ln2 (sum_i l2_i) + npix ln(cmax)
    double ll = (double)llacc;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) ll += __shfl_xor(ll, m, 64);
    // each wave of a cell adds its own pixels' share; the constant term once
    const double cst = sub == 0 ? (double)npix * Ip->lncmax : 0.0;
    if (lane == 0) P.llp[(size_t)sub * P.n_cell + cell] = kLn2 * ll + cst;
  }
}

// ---------------------------------------------------------------------------
// L(theta^t) per image and the stop rule (ll_reduce_block); the M-step gather
// (finalize_one, finalize_group)
// ---------------------------------------------------------------------------
// mode: LL_EM the EM pass (history, stop rule), LL_FINAL L into ll_final,
// LL_SEED L into ll_seed (the last two change no EM state)
__global__ __launch_bounds__(kLLThreads) void k_ll_reduce(DevPtrs P, double rel_tol, int mode,
                                                          int nsub) {
  ll_reduce_block(P, blockIdx.x, rel_tol, mode, nsub);
}

// One thread per superpixel (finalize_one).  Blocks from n_fin on take
// L(theta^t) of image blockIdx.x - n_fin in the EM pass without the stop rule
// (nothing in this pass depends on it then).
__global__ __launch_bounds__(256) void k_finalize(DevPtrs P, int n_fin) {
  if ((int)blockIdx.x >= n_fin) {
    ll_reduce_block(P, blockIdx.x - n_fin, 0.0, LL_EM, P.wpc);
    return;
  }
  finalize_one(P, blockIdx.x * 256 + threadIdx.x);
}

// G lanes per superpixel (finalize_group; G = 4 or 16), for batches that one
// thread per superpixel leaves short of waves.
template <int G>
__global__ __launch_bounds__(256) void k_finalize_lanes(DevPtrs P, int n_fin) {
  if ((int)blockIdx.x >= n_fin) {
    ll_reduce_block(P, blockIdx.x - n_fin, 0.0, LL_EM, P.wpc);
    return;
  }
  finalize_group<G>(P, blockIdx.x * (256 / G) + threadIdx.x / G, threadIdx.x & (G - 1));
}

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(size_t n, unsigned per) {
  return (unsigned)((n + per - 1) / per);
}

hipError_t launch_clear_records(const DevPtrs& P, hipStream_t s) {
  if (P.cov_mode) return launch_alt_clear_records(P, s);
  const size_t n = (size_t)P.n_cell * kSlots;
  hipLaunchKernelGGL(k_clear_records, dim3(blocks_for(n, 256)), dim3(256), 0, s, P.rec, n);
  return hipGetLastError();
}

hipError_t launch_reset_state(const DevPtrs& P, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_state, dim3(blocks_for(P.n_img, 256)), dim3(256), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_init_seeds(const DevPtrs& P, const float* lab, hipStream_t s) {
  if (P.cov_mode) return launch_alt_init_seeds(P, lab, s);
  hipLaunchKernelGGL(k_init_seeds, dim3(blocks_for(P.n_sp, 256)), dim3(256), 0, s, P, lab, 0);
  return hipGetLastError();
}

hipError_t launch_seed_fallback(const DevPtrs& P, const float* lab, hipStream_t s) {
  if (P.cov_mode) return hipErrorInvalidValue;  // the warm start serves cov_mode 0
  hipLaunchKernelGGL(k_init_seeds, dim3(blocks_for(P.n_sp, 256)), dim3(256), 0, s, P, lab, 1);
  return hipGetLastError();
}

hipError_t launch_ll_eval(const DevPtrs& P, const float* lab, int to_seed, hipStream_t s) {
  // L(theta) per cell wave: the slot-lane pass without its statistics, else the
  // statistics pass (its partials are scratch until the next pass); images
  // marked done are evaluated too
  const int mode = to_seed ? LL_SEED : LL_FINAL;
  hipError_t e = launch_reset_state(P, s);
  if (e != hipSuccess) return e;
  if (P.cov_mode == 0 && P.slot_j) {
    e = launch_ll_slots(P, lab, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ll_reduce, dim3(P.n_img), dim3(kLLThreads), 0, s, P, 0.0, mode, 1);
    return hipGetLastError();
  }
  return launch_estep_ll(P, lab, mode, 0.0, s);
}

hipError_t launch_set_params(const DevPtrs& P, const double* rows, hipStream_t s) {
  if (P.cov_mode) return launch_alt_set_params(P, rows, s);
  hipLaunchKernelGGL(k_set_params, dim3(blocks_for(P.n_sp, 256)), dim3(256), 0, s, P, rows);
  return hipGetLastError();
}

hipError_t launch_estep_stats(const DevPtrs& P, const float* lab, hipStream_t s) {
  if (P.cov_mode) return launch_alt_cells(P, 0, lab, nullptr, nullptr, s);
  if (P.estep == 1) return launch_estep_slots(P, lab, s);
  const dim3 grid(blocks_for((size_t)P.n_cell * P.wpc, kWavesPerBlock));
  if (P.wpc == 4)
    hipLaunchKernelGGL((k_cells<M_STATS, 4>), grid, dim3(256), 0, s, P, lab, (int32_t*)nullptr,
                       (float*)nullptr);
  else if (P.wpc == 2)
    hipLaunchKernelGGL((k_cells<M_STATS, 2>), grid, dim3(256), 0, s, P, lab, (int32_t*)nullptr,
                       (float*)nullptr);
  else
    hipLaunchKernelGGL((k_cells<M_STATS, 1>), grid, dim3(256), 0, s, P, lab, (int32_t*)nullptr,
                       (float*)nullptr);
  return hipGetLastError();
}

hipError_t launch_ll_update(const DevPtrs& P, double rel_tol, hipStream_t s) {
  hipLaunchKernelGGL(k_ll_reduce, dim3(P.n_img), dim3(kLLThreads), 0, s, P, rel_tol, (int)LL_EM,
                     P.wpc);
  return hipGetLastError();
}

hipError_t launch_estep_ll(const DevPtrs& P, const float* lab, int mode, double rel_tol,
                           hipStream_t s) {
  hipError_t e = launch_estep_stats(P, lab, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ll_reduce, dim3(P.n_img), dim3(kLLThreads), 0, s, P, rel_tol, mode, P.wpc);
  return hipGetLastError();
}

hipError_t launch_finalize(const DevPtrs& P, hipStream_t s, bool with_ll) {
  if (P.cov_mode) {
    hipError_t e = hipSuccess;
    if (with_ll) e = launch_ll_update(P, 0.0, s);
    return e == hipSuccess ? launch_alt_finalize(P, s) : e;
  }
  const int per = 256 / P.glanes;  // superpixels per block
  const int n_fin = (int)blocks_for(P.n_sp, per);
  const dim3 grid(n_fin + (with_ll ? P.n_img : 0));
  if (P.glanes == 16)
    hipLaunchKernelGGL(k_finalize_lanes<16>, grid, dim3(256), 0, s, P, n_fin);
  else if (P.glanes == 4)
    hipLaunchKernelGGL(k_finalize_lanes<4>, grid, dim3(256), 0, s, P, n_fin);
  else
    hipLaunchKernelGGL(k_finalize, grid, dim3(256), 0, s, P, n_fin);
  return hipGetLastError();
}

hipError_t launch_label(const DevPtrs& P, const float* lab, int32_t* labels, hipStream_t s) {
  if (P.cov_mode) {
    const hipError_t e = launch_alt_cells(P, 1, lab, labels, nullptr, s);
    if (e != hipSuccess) return e;
  } else {
    hipLaunchKernelGGL(k_cells<M_LABEL>, dim3(blocks_for(P.n_cell, kWavesPerBlock)), dim3(256), 0,
                       s, P, lab, labels, (float*)nullptr);
  }
  hipLaunchKernelGGL(k_ll_reduce, dim3(P.n_img), dim3(kLLThreads), 0, s, P, 0.0, (int)LL_FINAL, 1);
  return hipGetLastError();
}

hipError_t launch_export_R(const DevPtrs& P, const float* lab, float* R, hipStream_t s) {
  if (P.cov_mode) return launch_alt_cells(P, 2, lab, nullptr, R, s);
  hipLaunchKernelGGL(k_cells<M_EXPORT_R>, dim3(blocks_for(P.n_cell, kWavesPerBlock)), dim3(256),
                     0, s, P, lab, (int32_t*)nullptr, R);
  return hipGetLastError();
}

hipError_t launch_export_candidates(const DevPtrs& P, int32_t* cand, hipStream_t s) {
  if (P.cov_mode) return launch_alt_cells(P, 3, nullptr, cand, nullptr, s);
  hipLaunchKernelGGL(k_cells<M_EXPORT_CAND>, dim3(blocks_for(P.n_cell, kWavesPerBlock)),
                     dim3(256), 0, s, P, (const float*)nullptr, cand, (float*)nullptr);
  return hipGetLastError();
}

}  // namespace gmmsp
