// Internal layout shared by the host API (gmmsp_api.cpp) and the kernels
// (gmmsp_*.hip).  Not part of the public ABI.
#pragma once

#include <stdint.h>
#include <stddef.h>
#include <hip/hip_runtime.h>

namespace gmmsp {

constexpr int kSlots = 9;          // |K_i| <= 9: neighbour slots (dx, dy) in {-1,0,1}^2
constexpr int kStats = 13;         // N, S1 (5), S2 (xx xy yy LL aa ab bb)
constexpr int kPartStride = 120;   // FP32 values per cell wave: 9 x 13 statistics, 3 pad
constexpr int kRecFloats = 16;     // floats per cell-slot record
constexpr int kThetaRow = 13;      // doubles per superpixel in the FP64 master
constexpr int kLLCap = 4096;       // log-likelihood history entries per image
constexpr int kWavesPerBlock = 4;  // 64-lane waves per block of the per-cell kernels
constexpr int kMaxWpc = 4;         // largest number of waves sharing one cell
constexpr int kMaxWidth = 1 << 24; // widest image: a chunk's byte offsets fit 32 bits
// the unified 3x3 colour block (cov_mode 1)
constexpr int kRec3 = 20;          // floats per cell-slot record
constexpr int kStats3 = 15;        // N, S1 (5), S2 (xx xy yy LL La Lb aa ab bb)
constexpr int kPart3 = 136;        // doubles per cell: 9 x 15 statistics, 1 pad
constexpr int kThetaRow3 = 15;     // doubles per superpixel in the FP64 master
// the full 5 x 5 Sigma (cov_mode 2)
constexpr int kRecF = 24;          // floats per cell-slot record
constexpr int kStatsF = 21;        // N, S1 (5), S2 (15)
constexpr int kPartF = 192;        // doubles per cell: 9 x 21 statistics, 3 pad
constexpr int kThetaRowF = 21;     // mu (5), Sigma upper triangle (15), N
// grayscale images, D = 3 (cov_mode 3)
constexpr int kRecG = 12;          // floats per cell-slot record
constexpr int kStatsG = 8;         // N, S1 (x y I), S2 (xx xy yy II)
constexpr int kPartG = 72;         // doubles per cell: 9 x 8 statistics
constexpr int kThetaRowG = 8;      // mu (3), Sxx Sxy Syy SII, N
// the partials of one cell wave fit every model (the split model has kMaxWpc
// sets of kPartStride per cell, the others one set)
static_assert(kPart3 <= kPartStride * kMaxWpc && kPartF <= kPartStride * kMaxWpc, "partials");

// FP64 master row and record sizes of a covariance model
inline int theta_row_of(int cov_mode) {
  return cov_mode == 0 ? kThetaRow : cov_mode == 1 ? kThetaRow3 : cov_mode == 2 ? kThetaRowF
                                                                                : kThetaRowG;
}
inline int rec_floats_of(int cov_mode) {
  return cov_mode == 0 ? kRecFloats : cov_mode == 1 ? kRec3 : cov_mode == 2 ? kRecF : kRecG;
}

// First float of the split-colour-block record of candidate slot `slot` of batch
// cell `cell`.  Slot-major: the gather's threads (consecutive superpixels of a
// grid row) write the records of consecutive cells for each slot, whole lines.
__host__ __device__ inline size_t rec_index(int n_cell, int cell, int slot) {
  return ((size_t)slot * n_cell + cell) * kRecFloats;
}

// Cell-slot record: the parameters of the superpixel in slot s of cell c, in
// float32 and folded with the cell's origin, so that for a pixel at (xr, yr)
// relative to the cell origin with colour (L, a, b):
//   t1 = L11 xr + L12 yr + O1,  t2 = L22 yr + O2,
//   w  = SL L + OL,
//   u1 = A11 a + A12 b + O3,    u2 = A22 b + O4,
//   l  = C - t1^2 - t2^2 - w^2 - u1^2 - u2^2 = log2 p(z; theta_k) - cmax2
// and (ML, MA, MB) = (mu_L, mu_a, mu_b) rounded to float32, the colour origin
// of the statistics.  The offset pairs (O1, O2) and (O3, O4) sit at 8-byte
// aligned positions so that each pair moves to vector registers in one 64-bit
// move.  An empty slot has C = -inf and zeros elsewhere.
enum RecField {
  R_L11 = 0, R_L12 = 1, R_O1 = 2, R_O2 = 3, R_L22 = 4, R_SL = 5, R_O3 = 6, R_O4 = 7,
  R_OL = 8, R_A11 = 9, R_A12 = 10, R_A22 = 11, R_C = 12,
  R_ML = 13, R_MA = 14, R_MB = 15
};

// Statistic index inside a cell-slot partial.  Spatial moments are taken about
// the cell origin, colour moments about the slot's float32 record mean.
enum StatField {
  S_N = 0, S_X = 1, S_Y = 2, S_L = 3, S_A = 4, S_B = 5,
  S_XX = 6, S_XY = 7, S_YY = 8, S_LL = 9, S_AA = 10, S_AB = 11, S_BB = 12
};

struct ImgDesc {            // 96 bytes
  int32_t W, H, vx, vy;
  int32_t nx, ny, ncx, ncy;
  int64_t pix_off;          // first pixel of the image in the packed batch
  int32_t cell_off;         // first cell of the image in batch cell order
  int32_t sp_off;           // first superpixel of the image in batch order
  int32_t K, ncells;
  double eps_s, eps_c, lam, n_min;
  double lncmax;            // ln of the largest density the floors allow
};

struct ImgState {           // 40 bytes
  int32_t t;                // passes evaluated since the last initialisation
  int32_t done;             // 1 once the stop rule held
  int32_t iters;            // M-steps applied
  int32_t fallback;         // 1: the guarded warm start kept the grid seeds
  double ll_final;          // L(theta) of the last labelling (or evaluation) pass
  double ll_seed;           // L(theta^0) of the grid seeds (guarded warm start)
  double pad;
};

struct CellDesc { int32_t img, cx, cy, pad; };
struct SpDesc { int32_t img, kx, ky, pad; };

struct DevPtrs {
  const ImgDesc* img;
  ImgState* state;
  double* ll_hist;          // [n_img][kLLCap]
  const CellDesc* cell;
  const SpDesc* sp;
  double* theta;            // [n_sp][kThetaRow] FP64 master
  float* rec;               // split colour blocks: [9][n_cell][kRecFloats] (rec_index);
                            // other models [n_cell][9][their record floats]
  double* part;             // cell partials: split colour blocks FP32, [kMaxWpc][n_cell]
                            // [kPartStride] (one set per cell wave); other models FP64,
                            // one set per cell (kPart3, kPartF, kPartG doubles)
  double* llp;              // [kMaxWpc][n_cell]: log-likelihood of each cell wave's pixels
  int32_t* n_done;          // images that have stopped
  int32_t n_img, n_cell, n_sp;
  int32_t wpc;              // waves per cell of the statistics pass (1, 2 or 4)
  int32_t glanes;           // lanes per superpixel of the gather (1, 4 or 16)
  int32_t cov_mode;         // 0 split colour blocks; 1 3x3 colour block (gmmsp_cov3.hip);
                            // 2 full 5x5, 3 grayscale (gmmsp_modes.hip)
  int32_t estep;            // statistics pass of the split colour blocks: 0 one pixel per
                            // lane (k_cells), 1 one candidate slot per lane (k_slots,
                            // gmmsp_slots.hip; its colour statistics are whitened)
  int32_t slot_j, slot_rc;  // k_slots shape: columns per lane, rows per chunk
  int32_t slot_rc_max;      // the largest rows per chunk of this batch's shape
};

// How a per-image log-likelihood L(theta^t) is committed: LL_EM appends it to
// the image's history and applies the stop rule; LL_FINAL and LL_SEED store it
// (ll_final, ll_seed) and change no EM state.
enum LLMode { LL_EM = 0, LL_FINAL = 1, LL_SEED = 2 };

// The stop rule of Algorithm 1 on image b's L = L(theta^t): the run stops when
// |L - L(theta^(t-1))| <= rel_tol |L(theta^(t-1))| (rel_tol > 0); otherwise
// the M-step of this pass counts as applied.  One thread per image.
__device__ inline void ll_commit(const DevPtrs& P, int b, double L, int mode, double rel_tol) {
  ImgState* st = P.state + b;
  if (mode == LL_SEED) {
    st->ll_seed = L;
    return;
  }
  if (mode == LL_FINAL) {
    st->ll_final = L;
    return;
  }
  const int t = st->t;
  double* hist = P.ll_hist + (size_t)b * kLLCap;
  if (t < kLLCap) hist[t] = L;
  bool conv = false;
  if (rel_tol > 0.0 && t >= 1) {
    const double Lp = hist[t - 1];
    conv = fabs(L - Lp) <= rel_tol * fabs(Lp);
  }
  if (conv) {
    st->done = 1;
    atomicAdd(P.n_done, 1);
  } else {
    st->iters = t + 1;
  }
  st->t = t + 1;
}

// Grid barrier state of the persistent launch (device memory, zeroed before
// each launch): arrivals at the current barrier, barriers completed, and an
// error flag that a wait beyond its bound sets.
struct GridBar {
  uint32_t count;
  uint32_t gen;
  int32_t err;
  int32_t pad;
};

// The persistent launch's region of the workspace: its barrier and the device
// copy of the DevPtrs it runs with.
struct PersistArea {
  GridBar bar;
  DevPtrs P;
};

// Launch wrappers (gmmsp_kernels.hip).  All return hipError_t of the launch.
hipError_t launch_clear_records(const DevPtrs& P, hipStream_t s);
hipError_t launch_init_seeds(const DevPtrs& P, const float* lab, hipStream_t s);
// the grid seeds again for the images whose L(theta^0) (ll_final) is below that
// of the seeds (ll_seed) or not finite; sets their fallback flag, clears it elsewhere
hipError_t launch_seed_fallback(const DevPtrs& P, const float* lab, hipStream_t s);
// L(theta) of the current theta per image into ll_final (to_seed = 0) or
// ll_seed (to_seed = 1): one E-step, no M-step, no change of the EM state
hipError_t launch_ll_eval(const DevPtrs& P, const float* lab, int to_seed, hipStream_t s);
hipError_t launch_set_params(const DevPtrs& P, const double* rows, hipStream_t s);
hipError_t launch_reset_state(const DevPtrs& P, hipStream_t s);
hipError_t launch_estep_stats(const DevPtrs& P, const float* lab, hipStream_t s);
hipError_t launch_ll_update(const DevPtrs& P, double rel_tol, hipStream_t s);
// the statistics pass, then L(theta^t) per image (k_ll_reduce) committed in `mode`
hipError_t launch_estep_ll(const DevPtrs& P, const float* lab, int mode, double rel_tol,
                           hipStream_t s);
// the M-step gather; with_ll: also L(theta^t) of every image in the EM pass
// without the stop rule (rel_tol 0), as extra blocks of the same launch
hipError_t launch_finalize(const DevPtrs& P, hipStream_t s, bool with_ll = false);
hipError_t launch_label(const DevPtrs& P, const float* lab, int32_t* labels, hipStream_t s);
hipError_t launch_export_R(const DevPtrs& P, const float* lab, float* R, hipStream_t s);
hipError_t launch_export_candidates(const DevPtrs& P, int32_t* cand, hipStream_t s);

// The slot-lane statistics pass (gmmsp_slots.hip).  slots_shape gives the
// columns per lane and the largest rows per chunk for cells up to max_w pixels
// wide (0 when the kernel does not cover that width); slots_rows lists the
// rows-per-chunk values built for J columns per lane (largest first) and
// returns their count.
int slots_shape(int max_w, int* J, int* RC);
int slots_rows(int J, int max_rc, int* rows, int cap);
hipError_t launch_estep_slots(const DevPtrs& P, const float* lab, hipStream_t s);
// the slot-lane pass's log-likelihood terms alone (no statistics), one wave per
// cell: per-cell L terms in llp set 0
hipError_t launch_ll_slots(const DevPtrs& P, const float* lab, hipStream_t s);
// `iters` em passes without the stop rule in one cooperative launch of the
// slot-lane pass (P.estep 1, P.cov_mode 0) and the gather; Pd a device copy
// of P, gb zeroed, both written before the launch on stream s
hipError_t launch_persist(const DevPtrs& P, const DevPtrs* Pd, const float* lab, int iters,
                          GridBar* gb, hipStream_t s);

// The 3x3 colour block (gmmsp_cov3.hip); mode: 0 statistics, 1 labels,
// 2 responsibilities, 3 candidates.
hipError_t launch3_clear_records(const DevPtrs& P, hipStream_t s);
hipError_t launch3_init_seeds(const DevPtrs& P, const float* lab, hipStream_t s);
hipError_t launch3_set_params(const DevPtrs& P, const double* rows, hipStream_t s);
hipError_t launch3_cells(const DevPtrs& P, int mode, const float* lab, int32_t* out_i,
                         float* out_f, hipStream_t s);
hipError_t launch3_finalize(const DevPtrs& P, hipStream_t s);

// Every covariance model but the split colour blocks (gmmsp_modes.hip: the
// full 5x5 and grayscale kernels, and the 3x3 block's above); same modes.  The
// launchers of gmmsp_kernels.hip dispatch to these when P.cov_mode != 0.
hipError_t launch_alt_clear_records(const DevPtrs& P, hipStream_t s);
hipError_t launch_alt_init_seeds(const DevPtrs& P, const float* in, hipStream_t s);
hipError_t launch_alt_set_params(const DevPtrs& P, const double* rows, hipStream_t s);
hipError_t launch_alt_cells(const DevPtrs& P, int mode, const float* in, int32_t* out_i,
                            float* out_f, hipStream_t s);
hipError_t launch_alt_finalize(const DevPtrs& P, hipStream_t s);

// Warm-start network launchers (gmmsp_warmstart.hip).
hipError_t ws_launch_nbr(const DevPtrs& P, int32_t* nbr, hipStream_t s);
hipError_t ws_launch_features(const DevPtrs& P, const float* lab, float* feat, uint16_t* x0,
                              hipStream_t s);
hipError_t ws_launch_prep(const float* W, int cout, int cin, int cinp, int nk, int nt,
                          int transposed, uint16_t* wb, hipStream_t s);
hipError_t ws_launch_conv(int layer, int mode, const int32_t* nbr, const uint16_t* in,
                          const uint16_t* wb, const float* bias, int cout, const uint16_t* mask,
                          uint16_t* out_bf, float* out_f, int p0, int p1, hipStream_t s);
hipError_t ws_launch_dw(int layer, const int32_t* nbr, const uint16_t* g, const uint16_t* x,
                        float* part, int splits, int cps, int p0, int p1, hipStream_t s);
hipError_t ws_launch_reduce_dw(const float* part, int splits, int gc, int cout, int ncol,
                               float scale, float* grad, hipStream_t s);
hipError_t ws_launch_db(const uint16_t* g, int gc, int cout, int p0, int p1, float scale,
                        float* db, hipStream_t s);
hipError_t ws_launch_loss(const float* out, const float* tgt, uint16_t* g4, int p0, int p1,
                          double* loss_part, double* loss_sum, hipStream_t s);
hipError_t ws_launch_adam(float* w, float* m, float* v, const float* grad, int n, float lr,
                          float b1, float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t ws_launch_apply(const DevPtrs& P, const float* lab, const float* out, uint32_t mask,
                           double* rows, hipStream_t s);
hipError_t ws_launch_targets(const DevPtrs& P, const float* lab, float* tgt, hipStream_t s);

// Connectivity post-processing (gmmsp_connect.hip).  Per-pixel arrays hold
// n_pix entries; per-segment arrays hold n_pix entries (a segment has at least
// one pixel).
struct ConnPtrs {
  int64_t n_pix;
  int* par;                 // pixel union-find, then the small segments' pixel lists
  int* segid;               // segment index of each pixel (segments in id order)
  int* scan;                // root flags, then their exclusive scan
  int* bsum;                // scan block totals
  int* total;               // scan total (the number of segments after the first scan)
  int* n_big;               // number of clusters handled one wave each
  int* side;                // per tile: labels and roots of its first and last columns
  int* counts;              // [n_img][4]: segments, small, merged, (unused)
  int *seg_root, *seg_img, *size0, *size, *ccnt, *coff, *cursor, *list, *poff;
  int *cpar, *mpar, *next, *tail;
  unsigned long long* colsum;  // [n_seg][3] quantised colour sums, then FP64 means
};
size_t conn_scan_blocks(int64_t n);
size_t conn_tiles(int W, int H);  // 64 x 64 tiles of the component labelling
size_t conn_side_ints(int n_img, int max_tiles);  // side buffer of the tile borders
hipError_t conn_launch_components(const ConnPtrs& C, const ImgDesc* img, int n_img,
                                  int max_pixels, int max_tiles, const int32_t* labels,
                                  hipStream_t s);
hipError_t conn_launch_merge(const ConnPtrs& C, const ImgDesc* img, int n_img, int max_pixels,
                             int max_w, int max_h, int n_seg, const float* lab, int compact,
                             int32_t* out, hipStream_t s);

// Colour front end (gmmsp_color.hip).
hipError_t launch_srgb8_to_lab(const uint8_t* rgb, int64_t n, float* lab, hipStream_t s);

// Accuracy measures (gmmsp_metrics.hip).
int metrics_max_blocks(int max_w, int max_h);  // pixel-pass tiles of the largest image
hipError_t metrics_launch(const DevPtrs& P, int max_blocks, const int32_t* sp, const int32_t* gt,
                          const int32_t* n_lab, const int32_t* n_gt, const int64_t* row_off,
                          int64_t n_rows, const int64_t* tab_off, int64_t tab_n, int* tab,
                          int* br_part, int64_t* row_ue, int64_t* row_asa, int64_t* sums,
                          int* err, hipStream_t s);

}  // namespace gmmsp
