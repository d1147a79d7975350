// Slot-lane E-step with fused M-step statistics, for the split colour blocks
// (Eqs. gaussian, Rik; the numerators and denominators of Eqs. UpdateMu,
// UpdateSigS, UpdateSigC).
//
// Work decomposition.  One 64-lane wave owns one v_x x v_y cell (Eq. Ik: all
// pixels of a cell share the candidate set of the 3 x 3 neighbouring seeds).
// Lane l owns candidate slot s = l / 7 and column phase q = l % 7 (lane 63
// idles): it evaluates slot s for the cell pixels of columns q, q + 7, ...,
// so the slot's record factors live in the lane's own vector registers and
// every density and statistics instruction reads vector registers only (on
// gfx950 such instructions issue at twice the rate of those that read a
// scalar register).  Rows are processed in chunks of RC rows:
//   phase 0  one lane per pixel stages the chunk's pixels in the wave's LDS;
//   phase 1  every (slot, phase) lane evaluates its slot's log density for
//            its RC x J pixels, exponentiates and writes e = 2^l to LDS;
//   phase 2  one lane per pixel adds the nine e of its pixel (Eq. Rik's
//            denominator), takes the reciprocal and the log-likelihood term;
//   phase 3  every (slot, phase) lane forms R = e / sum for its pixels and
//            adds them to its slot's statistics.
// Spatial statistics use per-column accumulators (a lane's columns are fixed,
// its row is wave-uniform); colour statistics are taken in the record's
// whitened colour coordinates (w, u1, u2), which the density computes anyway,
// and are mapped back to Lab by the FP64 gather.  At the end of the cell the
// seven lanes of each slot are added in a fixed order through LDS.
#include "gmmsp_gather.h"
#include "gmmsp_internal.h"
#include "gmmsp_wave.h"

#include <math.h>

namespace gmmsp {

namespace {

constexpr int kQ = 7;  // column phases per slot: 9 x 7 = 63 lanes

// The smallest stride (a multiple of 4 floats, at least `need`) at which the
// seven column phases' reads of `width` consecutive floats fall in distinct
// LDS banks (64 banks of 4 bytes).
constexpr int bank_stride(int need, int width) {
  for (int s = ((need + 3) / 4) * 4;; s += 4) {
    bool ok = true;
    for (int k = 1; k < kQ && ok; ++k) {
      const int d = (k * s) % 64;
      if (d < width || 64 - d < width) ok = false;
    }
    if (ok) return s;
  }
}

// LDS of one wave for J columns per lane and RC rows per chunk.  The e rows
// of consecutive lanes are 4 x odd floats apart, so that 16 lanes' 16-byte
// writes fall in distinct banks.
template <int J, int RC>
struct SlotLds {
  static constexpr int kPB = bank_stride(RC * J * 3, 3);  // pixel floats per column phase
  static constexpr int kEB = ((RC * J + 3) / 8) * 8 + 4;  // e floats per (slot, phase)
  static constexpr int kPix = kQ * kPB;
  static constexpr int kE = (kSlots + 1) * kQ * kEB;       // + the idle lane's row
  static constexpr int kInv = kQ * kEB;
  static constexpr int kRed = 64 * kStats;                 // end-of-cell reduction
  static constexpr int kTail = kE + 2 * kInv > kRed ? kE + 2 * kInv : kRed;
  static constexpr int kWave = kPix + kTail;
};

// LDS writes of this wave become visible to all of its lanes.  Wavefront
// scope: a wave's LDS operations are carried out in the order it issues them,
// so the fences only keep the compiler from moving LDS accesses across the
// barrier, and no wait for the LDS is needed (a workgroup-scope fence would
// wait for every outstanding LDS operation, four times per chunk).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// keep a wave-uniform value in a vector register, so that the instructions
// that read it stay in the all-vector-register form
__device__ __forceinline__ float vreg(float x) {
  asm volatile("" : "+v"(x));
  return x;
}

// an LDS address that the compiler keeps in a register as an opaque value,
// instead of recomputing it from the lane index in every chunk
__device__ __forceinline__ float* lds_hold(float* p) {
  auto q = (__attribute__((address_space(3))) float*)p;
  asm volatile("" : "+v"(q));
  return (float*)q;
}

}  // namespace

// One wave's share of one cell: wave `sub` of the cell's `wpc` waves (WPC, or
// the run-time P.wpc when WPC is 0) takes chunks sub, sub + wpc, ...  PIX is
// the wave's LDS (SlotLds<J, RC>::kWave floats).  STATS false: only the
// log-likelihood terms (phase 3, the partials and the shifted e of the
// fallback are skipped), for evaluating L(theta) alone.
template <int J, int RC, int WPC, bool STATS>
__device__ __forceinline__ void slot_cell(const DevPtrs& P, const float* __restrict__ lab,
                                          float* PIX, int cell, int sub) {
  // products are rounded where written: every shape of the kernel rounds alike
#pragma clang fp contract(off)
  using LL = SlotLds<J, RC>;
  const int wpc = WPC > 0 ? WPC : P.wpc;
  const int lane = threadIdx.x & 63;
  float* E = PIX + LL::kPix;
  float* INV = E + LL::kE;
  float* SH = INV + LL::kInv;
  float* RED = E;
  const AS4 CellDesc* cdp = cptr(P.cell) + cell;
  const int b = cdp->img, ccx = cdp->cx, ccy = cdp->cy;
  if (cptr(P.state)[b].done) return;
  const AS4 ImgDesc* Ip = cptr(P.img) + b;
  const int W = Ip->W, H = Ip->H, vx = Ip->vx, vy = Ip->vy;
  const int x0 = ccx * vx, y0 = ccy * vy;
  const int w = min(vx, W - x0), h = min(vy, H - y0);
  const float* img = lab + 3 * (Ip->pix_off + (int64_t)y0 * W + x0);

  // this lane's slot and column phase; lane 63 idles on a copy of slot 8
  const int s = lane / kQ;
  const int q = lane - kQ * s;
  const bool live = s < kSlots;
  const float4* rp = reinterpret_cast<const float4*>(
      P.rec + rec_index(P.n_cell, cell, live ? s : kSlots - 1));
  const float4 f0 = rp[0], f1 = rp[1], f2 = rp[2], f3 = rp[3];
  const float L11 = f0.x, L12 = f0.y, O1 = f0.z, O2 = f0.w;
  const float L22 = f1.x, SL = f1.y, O3 = f1.z, O4 = f1.w;
  const float OL = f2.x, A11 = f2.y, A12 = f2.z, A22 = f2.w;
  const float C = f3.x;
  // t1 = L11 x + L12 y + O1 = ax[j] + L12 y for the lane's column x = q + 7 j;
  // a column outside the cell (or the idle lane) gets +inf, so its density is 0
  float ax[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int c = q + kQ * j;
    ax[j] = (live && c < w) ? fmaf(L11, (float)c, O1) : INFINITY;
  }

  // the pixel this lane stages and normalises in phases 0 and 2
  const int p_r = lane / w;
  const int p_c = lane - p_r * w;
  const int p_q = p_c % kQ, p_j = p_c / kQ;
  const int p_e = p_q * LL::kEB + p_r * J + p_j;        // index in E (slot 0), INV, SH
  const int p_x = p_q * LL::kPB + (p_r * J + p_j) * 3;  // index in PIX

  // entries that no pixel writes stay finite (0): a masked column reads them
  for (int i = lane; i < LL::kPix; i += 64) PIX[i] = 0.f;
  for (int i = lane; i < 2 * LL::kInv; i += 64) INV[i] = 0.f;

  float Nj[J], Mj[J], Qj[J];
#pragma unroll
  for (int j = 0; j < J; ++j) Nj[j] = Mj[j] = Qj[j] = 0.f;
  float Sw = 0.f, Su1 = 0.f, Su2 = 0.f, Sww = 0.f, S11 = 0.f, S12 = 0.f, S22 = 0.f;
  double ll64 = 0.0;  // sum of the pixels' log2 terms, in units of 2^-22

  const int n_chunks = (h + RC - 1) / RC;
  // the lane's staged pixel: byte offset from the first pixel of its chunk,
  // below 12 RC W, a 32-bit offset from a wave-uniform row address
  static_assert(12LL * RC * kMaxWidth < (1LL << 32), "32-bit pixel offsets");
  const uint32_t p_ofs = 12u * ((uint32_t)p_r * (uint32_t)W + (uint32_t)p_c);
  float pf0 = 0.f, pf1 = 0.f, pf2 = 0.f;
  auto fetch = [&](int c) {
    if (c < n_chunks && p_r < min(RC, h - c * RC)) {
      const char* row = reinterpret_cast<const char*>(img + (size_t)3 * W * (c * RC));
      const float* src = reinterpret_cast<const float*>(row + p_ofs);
      pf0 = src[0];
      pf1 = src[1];
      pf2 = src[2];
    }
  };
  fetch(sub);  // prefetch of the first chunk's pixel
  // loop-invariant LDS addresses of phases 2 and 3: the pixel's e in slots
  // 0-2, 3-5 and 6-8, and the lane's column phase of 1/sum
  constexpr int kSE = kQ * LL::kEB;  // e floats per slot
  static_assert(kSlots == 9, "phase 2 adds nine slots");
  const float* const e0 = lds_hold(E + p_e);
  const float* const e3 = lds_hold(E + 3 * kSE + p_e);
  const float* const e6 = lds_hold(E + 6 * kSE + p_e);
  // (16-byte aligned: kEB and the offset of INV are multiples of 4 floats,
  // and a row of kEB floats holds the RC J values rounded up to 4)
  const float4* const ivs = reinterpret_cast<const float4*>(lds_hold(INV + q * LL::kEB));
  static_assert(LL::kEB % 4 == 0 && (LL::kPix + LL::kE) % 4 == 0 &&
                (RC * J + 3) / 4 * 4 <= LL::kEB, "16-byte reads of 1/sum");
  for (int ch = sub; ch < n_chunks; ch += wpc) {
    const int r0 = ch * RC;
    const int nr = min(RC, h - r0);
    // phase 0: stage this chunk's pixels, then fetch the next chunk's
    wave_sync();  // the previous chunk's reads of PIX are done
    if (p_r < nr) {
      PIX[p_x] = pf0;
      PIX[p_x + 1] = pf1;
      PIX[p_x + 2] = pf2;
    }
    if constexpr (STATS) {
      // a position past the cell's last row (in the cell's last chunk) gets
      // 1/sum = 0, so its finite e (from a stale pixel) has R = 0 in phase 3
      if (nr < RC) {
        if (p_r >= nr && p_r < RC) INV[p_e] = 0.f;
      }
    }
    wave_sync();
    fetch(ch + wpc);
    // phase 1: log densities (log2 units, Eq. gaussian) and e = 2^l
    float e[RC][J], tw[RC][J], tu1[RC][J], tu2[RC][J];
    float cr[RC], rrv[RC];
#pragma unroll
    for (int i = 0; i < RC; ++i) {
      rrv[i] = vreg((float)(r0 + i));
      const float t2 = fmaf(L22, rrv[i], O2);
      cr[i] = fmaf(-t2, t2, C);
      const float* px = PIX + q * LL::kPB + i * J * 3;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const float Lv = px[3 * j], Av = px[3 * j + 1], Bv = px[3 * j + 2];
        tw[i][j] = fmaf(SL, Lv, OL);
        tu1[i][j] = fmaf(A11, Av, fmaf(A12, Bv, O3));
        tu2[i][j] = fmaf(A22, Bv, O4);
      }
    }
    // l = C - t1^2 - t2^2 - w^2 - u1^2 - u2^2 with t1 = L11 x + L12 y + O1,
    // each square taken off the running value by one fused multiply-add
    auto log_density = [&](int i, int j) {
      const float t1 = fmaf(L12, rrv[i], ax[j]);
      float l = fmaf(-t1, t1, cr[i]);
      l = fmaf(-tw[i][j], tw[i][j], l);
      l = fmaf(-tu1[i][j], tu1[i][j], l);
      return fmaf(-tu2[i][j], tu2[i][j], l);
    };
#pragma unroll
    for (int i = 0; i < RC; ++i)
#pragma unroll
      for (int j = 0; j < J; ++j) e[i][j] = __builtin_amdgcn_exp2f(log_density(i, j));
    {
      float* dst = E + (s * kQ + q) * LL::kEB;
#pragma unroll
      for (int i = 0; i < RC; ++i)
#pragma unroll
        for (int j = 0; j < J; ++j) dst[i * J + j] = e[i][j];
    }
    wave_sync();
    // phase 2: the denominator of Eq. Rik for each pixel of the chunk
    const bool pv = p_r < nr;
    // a lane without a pixel gets sum 1 (log-likelihood term 0)
    float sm = 1.f;
    if (pv) {
      sm = e0[0];
      sm += e0[kSE];
      sm += e0[2 * kSE];
      sm += e3[0];
      sm += e3[kSE];
      sm += e3[2 * kSE];
      sm += e6[0];
      sm += e6[kSE];
      sm += e6[2 * kSE];
    }
    const bool small = sm < 0x1p-100f;  // only a pixel's sum can be small
    float inv = __builtin_amdgcn_rcpf(sm), lg = __builtin_amdgcn_logf(sm);
    if (__builtin_amdgcn_ballot_w64(small) != 0) {
      // A pixel whose nine densities all underflow is normalised with its
      // largest log density subtracted first (the same posterior, Eq. Rik,
      // without 0/0); every other pixel keeps its e, inv and lg.  The log
      // densities replace e in LDS.
      float* dst = E + (s * kQ + q) * LL::kEB;
#pragma unroll
      for (int i = 0; i < RC; ++i)
#pragma unroll
        for (int j = 0; j < J; ++j) dst[i * J + j] = log_density(i, j);
      wave_sync();
      if (p_r < RC) SH[p_e] = INFINITY;  // not shifted (also every position past the last row)
      if (small) {
        float m = E[p_e];
#pragma unroll
        for (int k = 1; k < kSlots; ++k) m = fmaxf(m, E[k * kQ * LL::kEB + p_e]);
        float t = 0.f;
#pragma unroll
        for (int k = 0; k < kSlots; ++k) t += __builtin_amdgcn_exp2f(E[k * kQ * LL::kEB + p_e] - m);
        inv = __builtin_amdgcn_rcpf(t);
        lg = __builtin_amdgcn_logf(t) + m;
        SH[p_e] = m;
      }
      if constexpr (STATS) {
        wave_sync();
        const float* sh = SH + q * LL::kEB;
#pragma unroll
        for (int i = 0; i < RC; ++i)
#pragma unroll
          for (int j = 0; j < J; ++j) {
            const float m = sh[i * J + j];
            if (m != INFINITY) e[i][j] = __builtin_amdgcn_exp2f(log_density(i, j) - m);
          }
      }
    }
    if constexpr (STATS) {
      if (pv) INV[p_e] = inv;
    }
    // the log-likelihood term of the pixel (log2 units) on a 2^-22 grid: the
    // integer-valued FP64 sums are exact, so L does not depend on how pixels
    // are grouped into chunks and lanes.  lg * 2^22 is exact in FP32, so
    // rounding it there equals rounding it in FP64.
    ll64 += (double)rintf(lg * 0x1p22f);
    if constexpr (!STATS) continue;
    wave_sync();
    // phase 3: R = e / sum and the slot's sufficient statistics
    {
      float iv[(RC * J + 3) / 4 * 4];
#pragma unroll
      for (int k = 0; k < (RC * J + 3) / 4; ++k) {
        const float4 v = ivs[k];
        iv[4 * k] = v.x;
        iv[4 * k + 1] = v.y;
        iv[4 * k + 2] = v.z;
        iv[4 * k + 3] = v.w;
      }
#pragma unroll
      for (int i = 0; i < RC; ++i) {
        const float rr = rrv[i];
        const float r2 = vreg(rr * rr);
#pragma unroll
        for (int j = 0; j < J; ++j) {
          const float R = e[i][j] * iv[i * J + j];
          Nj[j] += R;
          Mj[j] = fmaf(rr, R, Mj[j]);
          Qj[j] = fmaf(r2, R, Qj[j]);
          const float rw = R * tw[i][j];
          Sw += rw;
          Sww = fmaf(rw, tw[i][j], Sww);
          const float r1 = R * tu1[i][j];
          Su1 += r1;
          S11 = fmaf(r1, tu1[i][j], S11);
          S12 = fmaf(r1, tu2[i][j], S12);
          const float rb = R * tu2[i][j];
          Su2 += rb;
          S22 = fmaf(rb, tu2[i][j], S22);
        }
      }
    }
  }

  if constexpr (STATS) {
    // this lane's statistics of its slot over its columns: spatial moments
    // about the cell origin from the per-column sums
    float st[kStats];
    st[S_N] = 0.f;
    st[S_X] = 0.f;
    st[S_Y] = 0.f;
    st[S_XX] = 0.f;
    st[S_XY] = 0.f;
    st[S_YY] = 0.f;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const float c = (float)(q + kQ * j);
      st[S_N] += Nj[j];
      st[S_X] = fmaf(c, Nj[j], st[S_X]);
      st[S_XX] = fmaf(c * c, Nj[j], st[S_XX]);
      st[S_Y] += Mj[j];
      st[S_XY] = fmaf(c, Mj[j], st[S_XY]);
      st[S_YY] += Qj[j];
    }
    // colour moments in the whitened coordinates of the slot's record
    st[S_L] = Sw;
    st[S_A] = Su1;
    st[S_B] = Su2;
    st[S_LL] = Sww;
    st[S_AA] = S11;
    st[S_AB] = S12;
    st[S_BB] = S22;
    wave_sync();  // the last chunk's reads of E, INV and SH are done
#pragma unroll
    for (int t = 0; t < kStats; ++t) RED[lane * kStats + t] = st[t];
    wave_sync();
    // the cell's totals: the seven lanes of each slot in ascending phase order
    float* part = reinterpret_cast<float*>(P.part) + ((size_t)sub * P.n_cell + cell) * kPartStride;
    for (int o = lane; o < kSlots * kStats; o += 64) {
      const int so = o / kStats, t = o - so * kStats;
      float a = 0.f;
#pragma unroll
      for (int k = 0; k < kQ; ++k) a += RED[(so * kQ + k) * kStats + t];
      part[o] = a;
    }
  }
  // cell log-likelihood: ln 2 (sum of log2 terms) + pixels x ln(cmax); the
  // integer-valued sums stay exact
  double ll = ll64;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) ll += __shfl_xor(ll, m, 64);
  const double cst = sub == 0 ? (double)(w * h) * Ip->lncmax : 0.0;
  if (lane == 0) P.llp[(size_t)sub * P.n_cell + cell] = kLn2 * (ll * 0x1p-22) + cst;
}

// One wave per (cell, sub) pair: WPC waves per cell.  The blocks of a launch
// go to the eight XCDs in turn (block b to XCD b mod 8).  Block b takes the
// cells of logical block lb: runs of kG consecutive logical blocks (4 kG
// consecutive cells) go to one XCD, the runs to the XCDs in turn.  Within a
// run the cache lines that neighbouring cells share (pixel rows that cross a
// cell border) are fetched into one L2 rather than two; across runs every
// image is spread over all XCDs, so images that have stopped leave no XCD
// idle (whole XCD-sized ranges of cells made the converging 4K batch 4.5 %
// slower).  The last partial round of runs keeps launch order.
template <int J, int RC, int WPC, bool STATS = true>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_slots(
    DevPtrs P, const float* __restrict__ lab) {
  using LL = SlotLds<J, RC>;
  __shared__ __align__(16) float lds[kWavesPerBlock * LL::kWave];
  const int wv = threadIdx.x >> 6;
  constexpr int kG = 8;  // blocks per run
  const int nb = (int)gridDim.x, b = (int)blockIdx.x;
  const int full = nb / (8 * kG) * (8 * kG);
  const int x = b % 8, i = b / 8;
  const int lb = b < full ? ((i / kG) * 8 + x) * kG + i % kG : b;  // a bijection of [0, nb)
  const int gw = __builtin_amdgcn_readfirstlane(lb * kWavesPerBlock + wv);
  const int cell = __builtin_amdgcn_readfirstlane(gw / WPC);
  const int sub = __builtin_amdgcn_readfirstlane(gw - cell * WPC);
  if (cell >= P.n_cell) return;
  slot_cell<J, RC, WPC, STATS>(P, lab, lds + wv * LL::kWave, cell, sub);
}

// Columns per lane and rows per chunk for cells up to max_w wide: J = ceil(max_w / 7),
// RC x max_w <= 64 (one lane per pixel in phases 0 and 2).  0 when the slot-lane
// kernel does not cover this width.
int slots_shape(int max_w, int* J, int* RC) {
  if (max_w < 1 || max_w > 8 * kQ) return 0;
  const int j = (max_w + kQ - 1) / kQ;
  int rc;
  switch (j) {
    case 1: rc = 8; break;
    case 2: rc = 4; break;
    case 3: rc = 3; break;
    case 4: rc = 2; break;
    case 5: rc = max_w <= 32 ? 2 : 1; break;
    default: rc = 1; break;
  }
  *J = j;
  *RC = rc;
  return 1;
}

namespace {
template <int J, int RC>
hipError_t launch_jrc(const DevPtrs& P, const float* lab, hipStream_t s) {
  const dim3 grid((unsigned)(((size_t)P.n_cell * P.wpc + kWavesPerBlock - 1) / kWavesPerBlock));
  if (P.wpc == 4)
    hipLaunchKernelGGL((k_slots<J, RC, 4>), grid, dim3(256), 0, s, P, lab);
  else if (P.wpc == 2)
    hipLaunchKernelGGL((k_slots<J, RC, 2>), grid, dim3(256), 0, s, P, lab);
  else
    hipLaunchKernelGGL((k_slots<J, RC, 1>), grid, dim3(256), 0, s, P, lab);
  return hipGetLastError();
}
}  // namespace

// Rows per chunk built for J columns per lane: every value of the shape
// table down to 1 row (J = 1: 8, 4, 2), largest first.
int slots_rows(int J, int max_rc, int* rows, int cap) {
  static const int kBuilt[8][3] = {{8, 4, 2}, {4, 2, 1}, {3, 2, 1}, {2, 1, 0},
                                   {2, 1, 0}, {1, 0, 0}, {1, 0, 0}, {1, 0, 0}};
  if (J < 1 || J > 8) return 0;
  int n = 0;
  for (int i = 0; i < 3 && n < cap; ++i)
    if (kBuilt[J - 1][i] > 0 && kBuilt[J - 1][i] <= max_rc) rows[n++] = kBuilt[J - 1][i];
  return n;
}

namespace {
template <int J, int RC>
hipError_t launch_ll_jrc(const DevPtrs& P, const float* lab, hipStream_t s) {
  const dim3 grid((unsigned)(((size_t)P.n_cell + kWavesPerBlock - 1) / kWavesPerBlock));
  hipLaunchKernelGGL((k_slots<J, RC, 1, false>), grid, dim3(256), 0, s, P, lab);
  return hipGetLastError();
}
}  // namespace

// The log-likelihood terms alone, one wave per cell (llp set 0), with the
// largest rows-per-chunk value of the batch's shape.
hipError_t launch_ll_slots(const DevPtrs& P, const float* lab, hipStream_t s) {
  switch (P.slot_j) {
    case 1: return launch_ll_jrc<1, 8>(P, lab, s);
    case 2: return launch_ll_jrc<2, 4>(P, lab, s);
    case 3: return launch_ll_jrc<3, 3>(P, lab, s);
    case 4: return launch_ll_jrc<4, 2>(P, lab, s);
    case 5: return P.slot_rc_max == 2 ? launch_ll_jrc<5, 2>(P, lab, s) : launch_ll_jrc<5, 1>(P, lab, s);
    case 6: return launch_ll_jrc<6, 1>(P, lab, s);
    case 7: return launch_ll_jrc<7, 1>(P, lab, s);
    case 8: return launch_ll_jrc<8, 1>(P, lab, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_estep_slots(const DevPtrs& P, const float* lab, hipStream_t s) {
  const int J = P.slot_j, RC = P.slot_rc;
#define GMMSP_JRC(j, rc) \
  if (J == j && RC == rc) return launch_jrc<j, rc>(P, lab, s);
  GMMSP_JRC(1, 8) GMMSP_JRC(1, 4) GMMSP_JRC(1, 2)
  GMMSP_JRC(2, 4) GMMSP_JRC(2, 2) GMMSP_JRC(2, 1)
  GMMSP_JRC(3, 3) GMMSP_JRC(3, 2) GMMSP_JRC(3, 1)
  GMMSP_JRC(4, 2) GMMSP_JRC(4, 1)
  GMMSP_JRC(5, 2) GMMSP_JRC(5, 1)
  GMMSP_JRC(6, 1) GMMSP_JRC(7, 1) GMMSP_JRC(8, 1)
#undef GMMSP_JRC
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Persistent T-mode passes (Algorithm 1 without the stop rule): one
// cooperative launch runs `iters` em passes.  Each pass is the statistics
// pass over every (cell, sub) pair, a grid barrier, the gather of every
// superpixel and L(theta^t) of every image (the work of the gather launch's
// blocks, taken block by block), and a grid barrier.  Every work item runs the
// per-pass kernels' code, so the passes are bitwise those of the eager
// launches with the same schedule.
// ---------------------------------------------------------------------------
namespace {

constexpr long kBarrierSpins = 1l << 25;  // sleeps of about 50 ns: about 2 s

// Grid-wide barrier of a cooperative launch (every block resident).  Every
// wave first waits until its stores have reached the L2 (the vector memory
// counter counts stores on this GPU); thread 0 of each block then arrives
// with a device-scope acquire-release atomic add (its release writes the
// XCD's L2 back, so the whole block's writes reach the device), waits with
// relaxed loads and takes one device-scope acquire fence, whose invalidation
// of the CU's L1 and the XCD's L2 serves the block's other waves too (they
// share them), which __syncthreads orders after it.  A wait beyond
// kBarrierSpins, or one that finds the error flag set, sets the flag and
// returns false; the caller then leaves the kernel, so every block ends.
__device__ bool grid_sync(GridBar* gb, uint32_t& gen) {
  __shared__ int ok_s;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t g = gen;
    int ok = 1;
    if (__hip_atomic_fetch_add(&gb->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) ==
        gridDim.x - 1) {
      __hip_atomic_store(&gb->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&gb->gen, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      // relaxed polls: an acquire per poll would invalidate the XCD's L2 under
      // the blocks still working; one acquire fence follows the wait
      for (long n = 0;
           __hip_atomic_load(&gb->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g; ++n) {
        if (n >= kBarrierSpins ||
            __hip_atomic_load(&gb->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          __hip_atomic_store(&gb->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    gen = g + 1u;
    ok_s = ok;
    __builtin_amdgcn_s_waitcnt(0);  // the acquire's cache invalidation has completed
  }
  __syncthreads();
  return ok_s != 0;
}

// The gather phase's block blk (a call, so that its FP64 registers do not
// crowd the statistics pass's)
__device__ __noinline__ void persist_gather(const DevPtrs& P, int blk, int n_fin) {
  if (blk < n_fin)
    finalize_block(P, blk);
  else
    ll_reduce_block(P, blk - n_fin, 0.0, LL_EM, P.wpc);
}

}  // namespace

// Pd: a device copy of the pass's DevPtrs (read-only here), so that the
// gather's call takes it by reference without a private copy
template <int J, int RC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_persist(
    const DevPtrs* __restrict__ Pd, const float* __restrict__ lab, int iters, int n_fin,
    GridBar* gb) {
  const DevPtrs& P = *Pd;
  using LL = SlotLds<J, RC>;
  __shared__ __align__(16) float lds[kWavesPerBlock * LL::kWave];
  const int wv = threadIdx.x >> 6;
  const int n_units = P.n_cell * P.wpc;
  const int n_waves = (int)gridDim.x * kWavesPerBlock;
  uint32_t gen = 0;
  for (int t = 0; t < iters; ++t) {
    for (int u = (int)blockIdx.x * kWavesPerBlock + wv; u < n_units; u += n_waves) {
      const int gw = __builtin_amdgcn_readfirstlane(u);
      const int cell = __builtin_amdgcn_readfirstlane(gw / P.wpc);
      const int sub = __builtin_amdgcn_readfirstlane(gw - cell * P.wpc);
      slot_cell<J, RC, 0, true>(P, lab, lds + wv * LL::kWave, cell, sub);
    }
    if (!grid_sync(gb, gen)) return;
    for (int blk = blockIdx.x; blk < n_fin + P.n_img; blk += gridDim.x)
      persist_gather(P, blk, n_fin);
    if (!grid_sync(gb, gen)) return;
  }
}

namespace {
template <int J, int RC>
hipError_t launch_persist_jrc(const DevPtrs& P, const DevPtrs* Pd, const float* lab, int iters,
                              GridBar* gb, hipStream_t s) {
  // resident blocks of this kernel per device, queried once (0: not yet)
  constexpr int kMaxDev = 64;
  static int resident[kMaxDev] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
  if (resident[dev] == 0) {
    int n_cu = 0, coop = 0, per_cu = 0;
    e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persist<J, RC>, 256, 0);
    if (e != hipSuccess) return e;
    if (!coop || per_cu < 1) return hipErrorCooperativeLaunchTooLarge;
    resident[dev] = per_cu * n_cu;
  }
  const int per = 256 / P.glanes;  // superpixels per gather block
  int n_fin = (int)((P.n_sp + per - 1) / per);
  const long need_e = ((long)P.n_cell * P.wpc + kWavesPerBlock - 1) / kWavesPerBlock;
  const long need = need_e > (long)n_fin + P.n_img ? need_e : (long)n_fin + P.n_img;
  const long cap = resident[dev];
  const unsigned grid = (unsigned)(need < cap ? need : cap);
  const float* l = lab;
  void* args[] = {&Pd, &l, &iters, &n_fin, &gb};
  e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_persist<J, RC>), dim3(grid),
                                 dim3(256), args, 0, s);
  return e != hipSuccess ? e : hipGetLastError();
}
}  // namespace

hipError_t launch_persist(const DevPtrs& P, const DevPtrs* Pd, const float* lab, int iters,
                          GridBar* gb, hipStream_t s) {
  const int J = P.slot_j, RC = P.slot_rc;
#define GMMSP_JRC(j, rc) \
  if (J == j && RC == rc) return launch_persist_jrc<j, rc>(P, Pd, lab, iters, gb, s);
  GMMSP_JRC(1, 8) GMMSP_JRC(1, 4) GMMSP_JRC(1, 2)
  GMMSP_JRC(2, 4) GMMSP_JRC(2, 2) GMMSP_JRC(2, 1)
  GMMSP_JRC(3, 3) GMMSP_JRC(3, 2) GMMSP_JRC(3, 1)
  GMMSP_JRC(4, 2) GMMSP_JRC(4, 1)
  GMMSP_JRC(5, 2) GMMSP_JRC(5, 1)
  GMMSP_JRC(6, 1) GMMSP_JRC(7, 1) GMMSP_JRC(8, 1)
#undef GMMSP_JRC
  return hipErrorInvalidValue;
}

}  // namespace gmmsp
