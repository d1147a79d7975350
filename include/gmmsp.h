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
 * launches; one image is a batch of one.
 *
 * Conventions shared by every entry point
 *   - Image data: interleaved float32 CIELAB (L, a, b) per pixel, row-major,
 *     pixel index i = x + W y.  A batch is packed back to back: image b starts
 *     at pixel offset P_b = sum_{c<b} W_c H_c, i.e. at float 3 P_b.
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
  int32_t cov_mode;     /* 0: blocks {(x,y), L, (a,b)} (Eq. BlockSigma1); only 0     */
  double n_min;         /* a superpixel with mass sum_i R_ik < n_min keeps theta_k   */
} gmmsp_params;

/* Seed grid of one image (Eqs. vxy, nxyK).  ncx = ceil(W / vx), ncy = ceil(H / vy)
 * count the v_x x v_y pixel cells including the partial remainder column / row. */
typedef struct gmmsp_grid_info {
  int32_t vx, vy, nx, ny, K, ncx, ncy;
} gmmsp_grid_info;

typedef struct gmmsp_handle gmmsp_handle;

/* Parameter row exported per superpixel, 13 doubles:
 *   mu_x mu_y mu_L mu_a mu_b  S_xx S_xy S_yy  S_LL  S_aa S_ab S_bb  N_k
 * (mean, the blocks of Sigma_k per Eq. BlockSigma1, and the mass
 * N_k = sum_{i in I_k} R_ik of the M-step that produced them). */
#define GMMSP_THETA_ROW 13

/* Largest number of E-steps whose log-likelihood one handle records per image
 * between two initialisations. */
#define GMMSP_LL_CAP 4096

/* Host only.  Seed grid of one image by Eqs. vxy and nxyK.
 * Errors: E_INVAL (null pointer, W or H < 1, K outside [1, W H] when v is
 * derived, v_x or v_y < 1), E_SIZE (n_x or n_y would be 0). */
int gmmsp_grid(const gmmsp_params* params, gmmsp_grid_info* out);

/* Host only.  Device workspace, in bytes, for a batch of n_images images with
 * parameters params[0..n_images-1].  Errors: those of gmmsp_grid, E_INVAL for
 * cov_mode != 0 or a non-positive eps_s, eps_c, lambda. */
int gmmsp_workspace_bytes(int32_t n_images, const gmmsp_params* params, size_t* bytes);

/* Create a handle over caller-owned device workspace (at least
 * gmmsp_workspace_bytes, 256-byte aligned).  Uploads the batch tables and clears
 * the parameter records on `stream`, then synchronises it.  The handle must be
 * initialised with gmmsp_init_seeds or gmmsp_set_params before it iterates. */
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

/* Set theta for every superpixel from rows of GMMSP_THETA_ROW doubles (device
 * memory, batch order; N_k ignored), applying the shape-control eigenvalue floors
 * of Eqs. mlams and mlamc, and reset the iteration state.  This is the warm-start
 * entry point and the resume hook. */
int gmmsp_set_params_dev(gmmsp_handle* h, const double* theta_dev, void* stream);

/* The same from host memory (copied on `stream`, which is synchronised). */
int gmmsp_set_params(gmmsp_handle* h, const double* theta_host, void* stream);

/* Copy theta (rows of GMMSP_THETA_ROW doubles, batch order) to the host. */
int gmmsp_get_params(gmmsp_handle* h, double* theta_host, void* stream);

/* EM iterations (Algorithm 1, steps 2-6).  Each pass t evaluates the E-step
 * with theta^t (Eq. Rik) together with L(theta^t) and the sufficient statistics
 * of the M-step, then forms theta^(t+1) (Eqs. UpdateMu, UpdateSigS, UpdateSigC
 * with shape control).  At most max_iters passes run.  With rel_tol > 0 an image
 * stops at the first pass t >= 1 with |L_t - L_(t-1)| <= rel_tol |L_(t-1)| and
 * keeps theta^t; with rel_tol <= 0 every image runs exactly max_iters passes
 * (the paper's fixed T).  Images that have stopped are skipped by every kernel.
 * Calls accumulate: a second call continues from the current theta.
 * iters_host (nullable, n_images int32): M-steps applied per image since the
 * last initialisation.  Synchronises `stream`. */
int gmmsp_em_iterate(gmmsp_handle* h, const float* lab_dev, int32_t max_iters,
                     double rel_tol, int32_t* iters_host, void* stream);

/* Log-likelihood history of image b: L(theta^0), L(theta^1), ... for every pass
 * run since the last initialisation (at most cap values); *n receives the count. */
int gmmsp_ll_history(gmmsp_handle* h, int32_t b, double* out_host, int32_t cap,
                     int32_t* n, void* stream);

/* Final E-step with the current theta and the labelling of Eq. obtLi: labels_dev
 * (int32, one per pixel, packed like the image) receives argmax_k R_ik, ties to
 * the smallest k.  ll_host (nullable, n_images doubles) receives L(theta) of this
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

/* Kernel timing for roofline reporting.  While enabled, gmmsp_em_iterate
 * brackets every launch of the E-step/statistics kernel with HIP events on the
 * caller's stream.  gmmsp_profile_read returns, since the last reset: the summed
 * kernel time in ms, the number of launches, and the pixels and (pixel,
 * candidate) pairs those launches evaluated (images that had stopped excluded);
 * reset != 0 clears the counters afterwards. */
int gmmsp_profile_enable(gmmsp_handle* h, int32_t enable);
int gmmsp_profile_read(gmmsp_handle* h, double* estep_ms, int32_t* launches,
                       int64_t* pixel_evals, int64_t* pair_evals, int32_t reset);

const char* gmmsp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GMMSP_H */
