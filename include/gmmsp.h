/*
 * gmmsp.h -- C ABI of the MI355X (gfx950) GMM superpixel EM library.
 *
 * The library runs the data-parallel hot path of the pixel-related Gaussian
 * mixture superpixel method of Ban, Liu and Cao (arXiv 1612.08792, Sec. III):
 * seed grid (Eqs. vxy, nxyK), candidate windows (Eq. Ik), initialisation
 * (Sec. III-C), EM iterations made of the E-step (Eq. Rik) and the M-step
 * (Eqs. UpdateMu, UpdateSigS, UpdateSigC) with shape control (Eqs. eigdecs to
 * eigdecrc), the log-likelihood L(theta) (Eq. ftheta), and the final labelling
 * (Eq. obtLi).  It handles a batch of images of different sizes in one set of
 * launches; one image is a batch of one.  Around the EM: a learned warm start
 * for theta^0 (gmmsp_ws_*), the connectivity post-processing that ends
 * Algorithm 1 (gmmsp_connectivity), the accuracy measures of Sec. IV
 * (gmmsp_metrics) and an sRGB to CIELAB front end (gmmsp_srgb8_to_lab).
 *
 * Conventions shared by every entry point
 *   - Image data: interleaved float32 CIELAB (L, a, b) per pixel, row-major,
 *     pixel index i = x + W y.  A batch is packed back to back: image b starts
 *     at pixel offset P_b = sum_{c<b} W_c H_c, i.e. at float 3 P_b.  With
 *     cov_mode 3 (grayscale) the EM entry points take one float32 intensity per
 *     pixel instead (image b at float P_b); the connectivity step always takes
 *     three channels (pass (I, 0, 0) for a grayscale image).
 *   - Superpixel k of an image is k = k_y n_x + k_x (Eq. kxy); batch-wide
 *     tables list the superpixels of image 0, then of image 1, and so on.
 *   - Device pointers (suffix _dev) are owned by the caller, who allocates
 *     them (e.g. with PyTorch) and keeps them alive during the call and the
 *     work it enqueues.  Host pointers (suffix _host) likewise.
 *   - Every launch goes to the caller's HIP stream, passed as an opaque
 *     pointer (a hipStream_t; NULL is the legacy default stream).  Calls that
 *     return host values synchronise that stream before returning.
 *   - Return value: GMMSP_OK or a negative gmmsp_status.  Nothing else crosses
 *     the ABI; gmmsp_last_error() returns a message for the calling thread.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Non-finite input pixels give undefined results.
 */
#ifndef GMMSP_H
#define GMMSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gmmsp_status {
  GMMSP_OK = 0,
  GMMSP_E_INVAL = -1,   /* bad argument: null pointer, non-positive size or constant */
  GMMSP_E_SIZE = -2,    /* sizes that give an empty grid, or workspace too small    */
  GMMSP_E_HIP = -3,     /* a HIP runtime call failed                                */
  GMMSP_E_NOMEM = -4,   /* host memory for the handle's tables, pinned host memory or
                           a HIP object could not be allocated (the library allocates
                           no device memory; a caller's buffers that are too small
                           give E_SIZE)                                             */
  GMMSP_E_STATE = -5    /* call out of order, or iteration history exhausted        */
} gmmsp_status;

/* Per-image parameters.  Every field is explicit: there are no hidden defaults. */
typedef struct gmmsp_params {
  int32_t W, H;         /* image size in pixels, both >= 1                           */
  int32_t K;            /* requested superpixels; used iff vx == 0 and vy == 0       */
  int32_t vx, vy;       /* seed spacing; 0, 0 => v_x = v_y = floor(sqrt(W H / K))    */
  double eps_s;         /* spatial eigenvalue floor (paper: 2, Sec. III-C)           */
  double eps_c;         /* colour eigenvalue floor (paper: 8, Sec. IV-A)             */
  double lambda;        /* initial colour standard deviation (paper: 8, Sec. IV-A)   */
  int32_t cov_mode;     /* 0: blocks {(x,y), L, (a,b)} (Eq. BlockSigma1);            */
                        /* 1: blocks {(x,y), (L,a,b)} (Eq. BlockSigma);              */
                        /* 2: the full 5x5 Sigma (Eq. UpdateSig), its eigenvalue     */
                        /*    floors applied to Sigma scaled by diag(eps_s, eps_s,   */
                        /*    eps_c, eps_c, eps_c) (the per-block rule of Eqs.       */
                        /*    mlams, mlamc whenever Sigma is block diagonal);        */
                        /* 3: a grayscale image, z = (x, y, I), D = 3 (Sec. III-A),  */
                        /*    blocks {(x,y), I}; the image buffer holds one float    */
                        /*    per pixel instead of three.                            */
                        /* One value for every image of a batch.                     */
  double n_min;         /* a superpixel with mass sum_i R_ik < n_min keeps theta_k   */
} gmmsp_params;

/* Seed grid of one image (Eqs. vxy, nxyK).  ncx = ceil(W / vx), ncy = ceil(H / vy)
 * count the v_x x v_y pixel cells including the partial remainder column / row. */
typedef struct gmmsp_grid_info {
  int32_t vx, vy, nx, ny, K, ncx, ncy;
} gmmsp_grid_info;

typedef struct gmmsp_handle gmmsp_handle;

/* Parameter row exported per superpixel, 13 doubles with cov_mode 0:
 *   mu_x mu_y mu_L mu_a mu_b  S_xx S_xy S_yy  S_LL  S_aa S_ab S_bb  N_k
 * (mean, the blocks of Sigma_k per Eq. BlockSigma1, and the mass
 * N_k = sum_{i in I_k} R_ik of the M-step that produced them); 15 doubles with
 * cov_mode 1 (the 3x3 colour block of Eq. BlockSigma):
 *   mu_x mu_y mu_L mu_a mu_b  S_xx S_xy S_yy  S_LL S_La S_Lb S_aa S_ab S_bb  N_k
 * 21 doubles with cov_mode 2 (the upper triangle of the full Sigma row by row):
 *   mu (5)  S_xx S_xy S_xL S_xa S_xb S_yy S_yL S_ya S_yb S_LL S_La S_Lb S_aa S_ab S_bb  N_k
 * 8 doubles with cov_mode 3 (grayscale):
 *   mu_x mu_y mu_I  S_xx S_xy S_yy  S_II  N_k */
#define GMMSP_THETA_ROW 13
#define GMMSP_THETA_ROW3 15
#define GMMSP_THETA_ROW_FULL 21
#define GMMSP_THETA_ROW_GRAY 8

/* Largest number of E-steps whose log-likelihood one handle records per image
 * between two initialisations. */
#define GMMSP_LL_CAP 4096

/* Widest image a batch may hold (2^24 pixels). */
#define GMMSP_MAX_WIDTH 16777216

/* Host only.  Seed grid of one image by Eqs. vxy and nxyK.
 * Errors: E_INVAL (null pointer, W or H < 1, K outside [1, W H] when v is
 * derived, v_x or v_y < 1), E_SIZE (n_x or n_y would be 0). */
int gmmsp_grid(const gmmsp_params* params, gmmsp_grid_info* out);

/* Host only.  Device workspace, in bytes, for a batch of n_images images with
 * parameters params[0..n_images-1].  Errors: those of gmmsp_grid, E_INVAL for
 * cov_mode outside 0..3, different cov_mode values in one batch, or a
 * non-positive eps_s, eps_c, lambda; E_SIZE for an image wider than
 * GMMSP_MAX_WIDTH pixels. */
int gmmsp_workspace_bytes(int32_t n_images, const gmmsp_params* params, size_t* bytes);

/* Create a handle over caller-owned device workspace (at least
 * gmmsp_workspace_bytes, 256-byte aligned).  Uploads the batch tables and clears
 * the parameter records on `stream`, then synchronises it.  The handle must be
 * initialised with gmmsp_init_seeds or gmmsp_set_params before it iterates.
 * Errors: those of gmmsp_workspace_bytes; E_INVAL for a null or misaligned
 * workspace or a null out; E_SIZE for a workspace smaller than
 * gmmsp_workspace_bytes; E_NOMEM when host memory for the tables runs out;
 * E_HIP when an upload fails. */
int gmmsp_create(int32_t n_images, const gmmsp_params* params, void* workspace_dev,
                 size_t workspace_bytes, void* stream, gmmsp_handle** out);

int gmmsp_destroy(gmmsp_handle* h);

/* Information about the batch: number of images, total pixels, total
 * superpixels, and the grid of image b. */
int gmmsp_batch_info(const gmmsp_handle* h, int32_t* n_images, int64_t* n_pixels,
                     int64_t* n_superpixels);
int gmmsp_image_grid(const gmmsp_handle* h, int32_t b, gmmsp_grid_info* out);

/* Sec. III-C initialisation: mu_k = z_j at the seed pixel
 * j = k_x v_x + floor(v_x/2) + W (k_y v_y + floor(v_y/2)), Sigma_s = diag(v_x^2,
 * v_y^2), colour variances lambda^2.  Resets the iteration state of every
 * image.  lab_dev: packed batch (see above). */
int gmmsp_init_seeds(gmmsp_handle* h, const float* lab_dev, void* stream);

/* Set theta for every superpixel from rows of the cov_mode's width
 * (GMMSP_THETA_ROW, _ROW3, _ROW_FULL, _ROW_GRAY) doubles (device
 * memory, batch order; N_k ignored), applying the shape-control eigenvalue floors
 * of Eqs. mlams and mlamc, and reset the iteration state.  This is the warm-start
 * entry point and the resume hook. */
int gmmsp_set_params_dev(gmmsp_handle* h, const double* theta_dev, void* stream);

/* The same from host memory (copied on `stream`, which is synchronised). */
int gmmsp_set_params(gmmsp_handle* h, const double* theta_host, void* stream);

/* Copy theta (rows of the cov_mode's width, doubles, batch order) to the host. */
int gmmsp_get_params(gmmsp_handle* h, double* theta_host, void* stream);

/* EM iterations (Algorithm 1, steps 2-6).  Each pass t evaluates the E-step
 * with theta^t (Eq. Rik) together with L(theta^t) and the sufficient statistics
 * of the M-step, then forms theta^(t+1) (Eqs. UpdateMu, UpdateSigS, UpdateSigC
 * with shape control).  At most max_iters passes run.  With rel_tol > 0 an image
 * stops at the first pass t >= 1 with |L_t - L_(t-1)| <= rel_tol |L_(t-1)| and
 * keeps theta^t; with rel_tol <= 0 every image runs exactly max_iters passes
 * (the paper's fixed T).  Images that have stopped are skipped by every kernel.
 * A pass is three launches (statistics, L with the stop rule, gather), or two
 * with rel_tol <= 0, where nothing in the pass waits for L and the gather's
 * launch also forms it (the same fixed-order sum either way); with the
 * persistent flag (gmmsp_set_persistent) and rel_tol <= 0, all passes are one
 * cooperative launch.  Calls accumulate: a second call continues from the
 * current theta; E_STATE, before any launch, for a call that could take an
 * image past 4096 passes since the last initialisation.
 * iters_host (nullable, n_images int32): M-steps applied per image since the
 * last initialisation.  Synchronises `stream` at the end (and before the
 * passes only when the pass count must be read to check the 4096 cap, or with
 * kernel timing on). */
int gmmsp_em_iterate(gmmsp_handle* h, const float* lab_dev, int32_t max_iters,
                     double rel_tol, int32_t* iters_host, void* stream);

/* Log-likelihood history of image b: L(theta^0), L(theta^1), ... for every pass
 * run since the last initialisation (at most cap values); *n receives the count. */
int gmmsp_ll_history(gmmsp_handle* h, int32_t b, double* out_host, int32_t cap,
                     int32_t* n, void* stream);

/* Final E-step with the current theta and the labelling of Eq. obtLi: labels_dev
 * (int32, one per pixel, packed like the image) receives argmax_k R_ik, ties to
 * the smallest k; k is the superpixel's index within its own image, k_y n_x + k_x.  ll_host (nullable, n_images doubles) receives L(theta) of this
 * E-step.  Synchronises `stream` only when ll_host is given. */
int gmmsp_label(gmmsp_handle* h, const float* lab_dev, int32_t* labels_dev,
                double* ll_host, void* stream);

/* Parity hooks.  R_dev (float32, 9 per pixel): R_ik of the E-step with the
 * current theta, stored by neighbour slot s = 3 (d_y + 1) + (d_x + 1) with
 * d_x = k_x - floor(x / v_x), d_y = k_y - floor(y / v_y); slots that are not
 * candidates hold 0.  cand_dev (int32, 9 per pixel): the superpixel of each slot
 * as the kernels index it, or -1. */
int gmmsp_export_responsibilities(gmmsp_handle* h, const float* lab_dev, float* R_dev,
                                  void* stream);
int gmmsp_export_candidates(gmmsp_handle* h, int32_t* cand_dev, void* stream);

/* Schedule of the statistics pass: how many 64-lane waves share one v_x x v_y
 * cell (1, 2 or 4; default 1).  More waves per cell raise the parallelism of
 * small batches; every schedule gives the same result up to the grouping of the
 * FP64 sums (each schedule is itself bitwise repeatable).  With cov_mode 1, 2
 * or 3 only 1 is accepted (E_INVAL otherwise). */
#define GMMSP_MAX_WAVES_PER_CELL 4
int gmmsp_set_schedule(gmmsp_handle* h, int32_t waves_per_cell);
int gmmsp_get_schedule(const gmmsp_handle* h, int32_t* waves_per_cell);

/* Work split of the statistics pass (E-step of Eqs. gaussian and Rik with the
 * sums of Eqs. UpdateMu .. UpdateSigC), cov_mode 0 only.  kind 0: every lane of
 * a cell's wave takes whole pixels and evaluates all nine candidates of each;
 * kind 1 (the default where it applies): every lane takes one candidate slot
 * and one column phase of the cell, so the slot's Gaussian stays in that lane's
 * registers, and the nine densities of a pixel meet in LDS for the normalisation
 * of Eq. Rik.  Kind 1 covers cells up to 56 pixels wide (v_x <= 56); E_INVAL for
 * kind 1 with another cov_mode or a wider grid.  Both give the method's result
 * (FP32 arithmetic, FP64 gather; they differ in the rounding of the FP32 sums)
 * and each is bitwise repeatable. */
int gmmsp_set_estep_kernel(gmmsp_handle* h, int32_t kind);
int gmmsp_get_estep_kernel(const gmmsp_handle* h, int32_t* kind);

/* Tile height of the slot-lane pass (kind 1): the cell rows each chunk takes
 * (every lane evaluates rows x J pixels of its slot per chunk, J = ceil(v_x /
 * 7) columns).  Built values: J = 1: 8, 4, 2; J = 2: 4, 2, 1; J = 3: 3, 2, 1;
 * J = 4 and J = 5 (v_x <= 32): 2, 1; otherwise 1.  The default is the
 * largest.  E_INVAL for a value not built for this batch's widest cell, or
 * when the batch has no slot-lane pass.  With one wave per cell every value
 * gives the same result bit for bit (the per-pixel arithmetic and the order of
 * every sum are the same); with more, the value decides which rows each wave
 * takes, so the FP32 sums group differently.  get returns 0 without a
 * slot-lane pass. */
int gmmsp_set_slot_rows(gmmsp_handle* h, int32_t rows);
int gmmsp_get_slot_rows(const gmmsp_handle* h, int32_t* rows);

/* Autotuner of the statistics pass: for each candidate schedule, `passes` em
 * passes (statistics, L, gather; after three untimed) from the grid
 * initialisation, timed with HIP events on `stream`, in two rounds over all
 * candidates (each candidate's faster round counts).  Candidates, in order of
 * preference: the slot-lane pass (kind 1) with each built rows-per-chunk value,
 * largest first, then the pixel-lane pass (kind 0); 1, 2 and 4 waves per cell
 * each.  A later candidate is kept only if it is more than 3 % faster than the
 * best before it.  Sets the kind, rows per chunk and waves per cell; leaves the
 * handle initialised by gmmsp_init_seeds; *chosen = the waves per cell.
 * ms_host (nullable, GMMSP_TUNE_CANDIDATES doubles): the time of candidate
 * 3 v + w, v = 0, 1, 2 the slot-lane pass with the v-th rows value, v = 3 the
 * pixel-lane pass, w = 0, 1, 2 for 1, 2, 4 waves per cell; -1 where not timed
 * (with cov_mode 1, 2 or 3 only entry 9, one wave per cell, is). */
#define GMMSP_TUNE_CANDIDATES 12
int gmmsp_autotune(gmmsp_handle* h, const float* lab_dev, int32_t passes, double* ms_host,
                   int32_t* chosen, void* stream);

/* Schedule of the per-superpixel gather of the M-step (Eqs. UpdateMu,
 * UpdateSigS, UpdateSigC and the shape control): 1 lane per superpixel
 * (default; the window cells are added in a fixed sequential order), or G = 4
 * or 16 lanes per superpixel (lane j adds window cells j, j + G, ... in that
 * order, the G lanes add in a fixed butterfly order, and lane j writes the
 * records of the same cells), for batches that one lane per superpixel leaves
 * short of waves.  The schedules group the FP64 sums differently; each is
 * bitwise repeatable.  With cov_mode 1, 2 or 3 only 1 is accepted (E_INVAL
 * otherwise). */
int gmmsp_set_gather_lanes(gmmsp_handle* h, int32_t lanes_per_superpixel);
int gmmsp_get_gather_lanes(const gmmsp_handle* h, int32_t* lanes_per_superpixel);

/* Autotuner of the gather: for 1, 4 and 16 lanes per superpixel, `passes`
 * whole em passes (after three untimed) from the grid initialisation with the
 * statistics-pass schedule in effect, timed with HIP events on `stream`, in two
 * rounds (each candidate's faster round counts); more lanes are kept only if
 * more than 3 % faster than the best with fewer.  Leaves the handle
 * initialised by gmmsp_init_seeds.  Run it after gmmsp_autotune.  ms_host
 * (nullable, 3 doubles, in the order 1, 4, 16): the measured times (-1 for a
 * schedule not timed). */
int gmmsp_autotune_gather(gmmsp_handle* h, const float* lab_dev, int32_t passes,
                          double* ms_host, int32_t* chosen, void* stream);

/* Graph replay: with passes > 0, gmmsp_em_iterate runs whole chunks of
 * `passes` em passes as one captured hipGraph launch each (captured on first
 * use for the given image buffer, tolerance and schedule, on a private stream
 * ordered after the caller's), the stop test being read between chunks; the
 * remainder of max_iters runs as single launches.  0 (default) turns it off.
 * Not used while kernel timing is enabled. */
int gmmsp_set_graph_passes(gmmsp_handle* h, int32_t passes);

/* Persistent T-mode passes (Algorithm 1 without the stop rule): with on = 1,
 * gmmsp_em_iterate with rel_tol <= 0 runs all max_iters passes in one
 * cooperative launch when the statistics pass is the slot-lane kind (kind 1):
 * each pass is the statistics pass over every cell, a grid-wide barrier, the
 * gather of every superpixel and L(theta^t) of every image, and a barrier.
 * The grid holds at most as many blocks as the GPU keeps resident; every
 * work item runs the per-pass kernels' code, so the passes equal the per-pass
 * launches with the same schedule bit for bit.  Calls with the stop rule, with
 * kind 0, or with kernel timing enabled keep the per-pass launches.  Uses the
 * handle's workspace (its barrier and a device copy of the schedule) and
 * waits for the launch before returning; E_STATE if a barrier wait ran out
 * (about 2 s; the passes are then incomplete).  0 (default) turns it off;
 * E_INVAL for 1 when the batch has no slot-lane pass. */
int gmmsp_set_persistent(gmmsp_handle* h, int32_t on);
int gmmsp_get_persistent(const gmmsp_handle* h, int32_t* on);

/* Autotuner of the launch form of T-mode passes: `passes` passes (after three
 * untimed) from the grid initialisation as per-pass launches with the schedule
 * in effect, against the persistent launch of the slot-lane pass with each
 * built rows-per-chunk value (largest first; waves per cell and gather lanes
 * as in effect), each timed on the host clock from its first launch to the
 * end of its last pass on `stream` (what the launch form changes is mostly
 * host launch cost), in two rounds (each candidate's faster round counts).  The persistent form is kept only if more
 * than 3 % faster than the per-pass launches; it then sets kind 1, its rows
 * value and the persistent flag, else it leaves the schedule and clears the
 * flag.  Run it after gmmsp_autotune and gmmsp_autotune_gather.  Leaves the
 * handle initialised by gmmsp_init_seeds; *chosen = the flag.  ms_host
 * (nullable, 4 doubles): per-pass launches, then the persistent launch with
 * the rows values largest first (-1 where not timed, e.g. every persistent
 * entry for a batch without a slot-lane pass). */
int gmmsp_autotune_persistent(gmmsp_handle* h, const float* lab_dev, int32_t passes,
                              double* ms_host, int32_t* chosen, void* stream);

/* Kernel timing for roofline reporting.  While enabled, gmmsp_em_iterate
 * brackets every launch of the E-step/statistics kernel with HIP events on the
 * caller's stream.  gmmsp_profile_read returns, since the last reset: the summed
 * kernel time in ms, the number of launches, and the pixels and (pixel,
 * candidate) pairs those launches evaluated (images that had stopped excluded);
 * reset != 0 clears the counters afterwards. */
int gmmsp_profile_enable(gmmsp_handle* h, int32_t enable);
int gmmsp_profile_read(gmmsp_handle* h, double* estep_ms, int32_t* launches,
                       int64_t* pixel_evals, int64_t* pair_evals, int32_t reset);

/* ------------------------------------------------------------------------
 * Learned warm start (not part of the paper): a conv3x3 network on the seed
 * grid, BF16 weights and activations with FP32 accumulation on the matrix
 * cores, predicts theta^0 in place of the grid initialisation of Sec. III-C;
 * the EM above then runs unchanged.  Layers: 16 -> 32 -> 32 -> 32 -> 10, ReLU
 * between them, zero padding at the grid border.
 *   inputs (16 per superpixel, over its own v_x x v_y seed cell, s its seed
 *   pixel, h = floor(v / 2)): (mean_L - 50)/50, mean_a/64, mean_b/64,
 *     std_L/16, std_a/16, std_b/16, min(k_x, k_y, n_x-1-k_x, n_y-1-k_y, 3)/3,
 *     (colour(s) - mean)/16 (3), (mean of the last h columns - mean of the
 *     first h)/32 (3), the same for rows (3)
 *   outputs o[0..9] -> theta^0: mu_x = s_x + v_x o0, mu_y = s_y + v_y o1,
 *     mu_c = colour(s) + lambda o_{2..4}, Sigma = diag(v_x^2 e^{2 o5},
 *     v_y^2 e^{2 o6}, lambda^2 e^{2 o7..9}) (log-scales clipped to [-4, 4]),
 *     then the eigenvalue floors; outputs outside the caller's mask count as
 *     0, so the all-zero output is the grid initialisation exactly, and a
 *     superpixel with a non-finite output gets the grid initialisation.
 * Parameters: one flat FP32 vector (caller-owned device memory), per layer
 * W[cout][9][cin] (tap t = 3 (dy + 1) + (dx + 1)) then b[cout].
 * ------------------------------------------------------------------------ */
#define GMMSP_WS_NPARAM 26026

/* Buffers of the warm-start workspace that gmmsp_ws_read / gmmsp_ws_write reach. */
typedef enum gmmsp_ws_buffer {
  GMMSP_WS_FEAT = 0,   /* float32 [n_sp][16] inputs                        */
  GMMSP_WS_X0 = 1,     /* bf16 [n_sp][16] inputs as the first layer reads   */
  GMMSP_WS_Y1 = 2,     /* bf16 [n_sp][32] activation after layer 1 (ReLU)   */
  GMMSP_WS_Y2 = 3,
  GMMSP_WS_Y3 = 4,
  GMMSP_WS_OUT = 5,    /* float32 [n_sp][16] outputs (10 used)              */
  GMMSP_WS_TGT = 6,    /* float32 [n_sp][16] training targets (10 used)     */
  GMMSP_WS_G4 = 7,     /* bf16 [n_sp][16] gradient at the outputs, 2 (o - t) / 10 */
  GMMSP_WS_G3 = 8,     /* bf16 [n_sp][32] gradient at layer-3 output, ReLU applied */
  GMMSP_WS_G2 = 9,
  GMMSP_WS_G1 = 10,
  GMMSP_WS_GRAD = 11   /* float32 [GMMSP_WS_NPARAM] gradient of the last step */
} gmmsp_ws_buffer;

/* Device workspace of the warm start for this handle's batch, and attaching it
 * (builds the seed-grid neighbour table on `stream`, then synchronises it).
 * The network predicts the split colour blocks: E_INVAL with cov_mode 1, 2, 3. */
int gmmsp_ws_workspace_bytes(const gmmsp_handle* h, size_t* bytes);
int gmmsp_ws_attach(gmmsp_handle* h, void* ws_dev, size_t bytes, void* stream);

/* Network inputs of every superpixel of the batch from the Lab images. */
int gmmsp_ws_features(gmmsp_handle* h, const float* lab_dev, void* stream);

/* Forward pass over the superpixels of images [b0, b1) with parameters
 * params_dev (GMMSP_WS_NPARAM floats). */
int gmmsp_ws_forward(gmmsp_handle* h, const float* params_dev, int32_t b0, int32_t b1,
                     void* stream);

/* theta^0 of every image from the last forward outputs (see above; bit c of
 * output_mask selects output c), with the eigenvalue floors, and reset of the
 * iteration state: the handle is then initialised as by gmmsp_init_seeds. */
int gmmsp_ws_apply(gmmsp_handle* h, const float* lab_dev, uint32_t output_mask, void* stream);

/* gmmsp_ws_apply with the grid seeds of Sec. III-C as the fallback, judged by
 * the objective L(theta) of Sec. III-B (Eq. ftheta's log-likelihood): one
 * E-step evaluates L(theta^0) for the grid seeds and one for the network's
 * theta^0; every image whose network start has the lower L, or a non-finite
 * one, starts from the grid seeds instead.  fallback_host (nullable,
 * n_images int32): 1 where the seeds were kept; when given, `stream` is
 * synchronised.  Costs two E-steps over the batch. */
int gmmsp_ws_apply_guarded(gmmsp_handle* h, const float* lab_dev, uint32_t output_mask,
                           int32_t* fallback_host, void* stream);

/* Training targets from the handle's current theta (for instance plain EM
 * after some passes): the inverse of the map above. */
int gmmsp_ws_targets(gmmsp_handle* h, const float* lab_dev, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with
 * step >= 1) on the mean squared error over images [b0, b1): forward, loss,
 * backward (input and weight gradients on the matrix cores, fixed-order
 * reductions) and the update of params_dev, m_dev, v_dev (caller-owned,
 * GMMSP_WS_NPARAM floats each).  loss_host (nullable): the loss before the
 * update; when given, `stream` is synchronised. */
int gmmsp_ws_train_step(gmmsp_handle* h, float* params_dev, float* m_dev, float* v_dev,
                        int32_t step, float lr, int32_t b0, int32_t b1, double* loss_host,
                        void* stream);

/* Copy a workspace buffer to or from the host (synchronises `stream`); bytes
 * must not exceed the buffer's size. */
int gmmsp_ws_read(gmmsp_handle* h, int32_t which, void* host, size_t bytes, void* stream);
int gmmsp_ws_write(gmmsp_handle* h, int32_t which, const void* host, size_t bytes, void* stream);

/* ------------------------------------------------------------------------
 * Connectivity post-processing (Algorithm 1, last step; the paragraph on
 * enforcing connectivity in Sec. III-C).
 *
 * The labelled superpixels may be disconnected.  Segments are the
 * 4-connected components of equal label in each image of the batch; a
 * segment's id is the raster index y W + x (inside its image) of its first
 * pixel.  Segments smaller than a quarter of the desired superpixel size
 * (4 size < v_x v_y of the image's grid) are visited in ascending order of
 * their size (ties: ascending id) and each one still small when visited is
 * merged into the neighbouring segment (as merged so far) whose mean Lab
 * colour is closest: squared Euclidean distance in FP64 between the
 * segments' own mean colours, each the mean of the pixels' colours
 * quantised to multiples of 2^-20, ties to the smaller id; the destination's
 * size grows by the merged size.  The neighbours of a segment are those
 * holding a 4-neighbour of any pixel merged into it so far.  A segment with
 * no neighbour stays.  The result is a partition into connected segments.
 *
 * gmmsp_conn_workspace_bytes: size of the caller-allocated device workspace
 *   (256-byte aligned), about 88 bytes per pixel of the batch (the worst case
 *   of one segment per pixel).
 * gmmsp_connectivity: labels_dev (int32 per pixel of the batch, any values:
 *   only equality matters, e.g. the output of gmmsp_label) and lab_dev (the
 *   batch's Lab pixels) in; out_dev (int32 per pixel) receives the id of the
 *   segment the pixel ends in (compact = 0), or its rank among the image's
 *   final segments in id order, 0 .. final - 1 (compact != 0, e.g. as labels
 *   for gmmsp_metrics).  Needs the handle's geometry only (no
 *   initialisation).  counts_host (nullable, 4 int32 per image): segments,
 *   small segments, merged segments, final segments.  Synchronises `stream`
 *   (the segment count is read back between two groups of launches).
 *   Errors: E_INVAL for null or misaligned pointers, E_SIZE for a short
 *   workspace or a batch of 2^31 - 1 pixels or more.
 * ------------------------------------------------------------------------ */
int gmmsp_conn_workspace_bytes(const gmmsp_handle* h, size_t* bytes);
int gmmsp_connectivity(gmmsp_handle* h, const float* lab_dev, const int32_t* labels_dev,
                       int32_t* out_dev, void* ws_dev, size_t ws_bytes, int32_t compact,
                       int32_t* counts_host, void* stream);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc: serving loops, harnesses that forbid allocation).  The same as
 * gmmsp_connectivity, with the workspace taken from a scratch array of
 * GMMSP_CONN_STATIC_BYTES that the library keeps on each GPU it runs on until
 * the process ends (its address is looked up on the first call on a device,
 * with that device current).  The entry point allocates nothing: no hipMalloc,
 * hipFree or host heap.  E_SIZE when the batch needs more than
 * GMMSP_CONN_STATIC_BYTES (gmmsp_conn_workspace_bytes; about 88 bytes per
 * pixel, so about 1.1 million pixels).  Every call on a GPU uses that GPU's
 * one array and leaves its contents behind: calls that overlap on one GPU
 * (several threads or streams) race, and the caller must serialise them.
 * Synchronises `stream`. */
#define GMMSP_CONN_STATIC_BYTES (96u << 20)
int gmmsp_connectivity_static(gmmsp_handle* h, const float* lab_dev, const int32_t* labels_dev,
                              int32_t* out_dev, int32_t compact, int32_t* counts_host,
                              void* stream);

/* ------------------------------------------------------------------------
 * Accuracy measures of Sec. IV for each image of the batch: boundary recall
 * (BR), under-segmentation error (Eq. ue) and achievable segmentation
 * accuracy (Eq. asa) of a superpixel label map against a ground-truth region
 * map.
 *
 * A boundary pixel of a map is one whose right or lower neighbour carries
 * another value.  BR = the fraction of ground-truth boundary pixels with a
 * superpixel boundary pixel in the 5 x 5 square around them (1 when there
 * is no ground-truth boundary).  UE = (1/N) sum_g sum_{k : |s_k n s_g| >
 * 0.05 |s_k|} |s_k| - 1 (the comparison taken exactly as 20 |s_k n s_g| >
 * |s_k|), ASA = (1/N) sum_k max_g |s_k n s_g|; N = W H.
 *
 * labels_dev: int32 per pixel of the batch with values in [0, S_b), where
 * S_b = n_sp_host[b], or the image's n_x n_y when n_sp_host is NULL (the
 * output of gmmsp_label); gt_dev: int32 per pixel with values in
 * [0, n_gt_host[b]).  Workspace (caller-allocated, 256-byte aligned):
 * gmmsp_metrics_workspace_bytes, dominated by an S_b x n_gt[b] int32 count
 * table per image.  out_host: 3 doubles per image (BR, UE, ASA);
 * sums_host (nullable): 4 int64 per image (recovered boundary pixels,
 * ground-truth boundary pixels, the sum of Eq. ue, the sum of Eq. asa).
 * Synchronises `stream`.  Errors: E_INVAL for null or misaligned pointers,
 * S_b or n_gt < 1, or a value outside its range (found on the device;
 * nothing is written out of bounds); E_SIZE for a short workspace or
 * S_b n_gt >= 2^31.
 * ------------------------------------------------------------------------ */
int gmmsp_metrics_workspace_bytes(const gmmsp_handle* h, const int32_t* n_sp_host,
                                  const int32_t* n_gt_host, size_t* bytes);
int gmmsp_metrics(gmmsp_handle* h, const int32_t* labels_dev, const int32_t* gt_dev,
                  const int32_t* n_sp_host, const int32_t* n_gt_host, void* ws_dev,
                  size_t ws_bytes, double* out_host, int64_t* sums_host, void* stream);

/* ------------------------------------------------------------------------
 * Colour front end: the method runs in CIELAB (Sec. IV); this converts 8-bit
 * sRGB (IEC 61966-2-1 transfer function, sRGB primaries, D65 white) to CIE
 * 1976 L*a*b* relative to D65 (2-degree observer), in float32.
 * rgb_dev: n_pixels x 3 uint8 (R, G, B interleaved), 4-byte aligned;
 * lab_dev: n_pixels x 3 float32 (L, a, b interleaved, the layout every entry
 * point above reads), 16-byte aligned.  Needs no handle.  Errors: E_INVAL for
 * null or misaligned pointers or n_pixels < 0.
 * ------------------------------------------------------------------------ */
int gmmsp_srgb8_to_lab(const uint8_t* rgb_dev, int64_t n_pixels, float* lab_dev, void* stream);

const char* gmmsp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GMMSP_H */
