// Host side of the gmmsp C ABI: argument validation, seed-grid arithmetic
// (Eqs. vxy, nxyK), batch tables, workspace layout and the EM driver.
#include "../../include/gmmsp.h"
#include "gmmsp_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace gmmsp;

// Device memory of the allocation-free connectivity entry point: each GPU the
// library runs on holds one copy until the process ends.
static __device__ __align__(256) unsigned char scratch[GMMSP_CONN_STATIC_BYTES];

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? GMMSP_E_NOMEM : GMMSP_E_HIP, "%s: %s", what,
              hipGetErrorString(e));
}

// floor(sqrt(n)) for n >= 0, exact
int64_t isqrt64(int64_t n) {
  int64_t r = (int64_t)sqrt((double)n);
  while (r > 0 && r * r > n) --r;
  while ((r + 1) * (r + 1) <= n) ++r;
  return r;
}

int grid_of(const gmmsp_params* p, gmmsp_grid_info* g) {
  if (!p || !g) return fail(GMMSP_E_INVAL, "null pointer");
  if (p->W < 1 || p->H < 1) return fail(GMMSP_E_INVAL, "image size %d x %d", p->W, p->H);
  int64_t vx = p->vx, vy = p->vy;
  if (vx == 0 && vy == 0) {
    const int64_t N = (int64_t)p->W * p->H;
    if (p->K < 1 || p->K > N) return fail(GMMSP_E_INVAL, "K = %d outside [1, %lld]", p->K, (long long)N);
    // Eq. vxy: floor(sqrt(W H / K)) = isqrt(floor(W H / K))
    vx = vy = isqrt64(N / p->K);
  }
  if (vx < 1 || vy < 1) return fail(GMMSP_E_INVAL, "seed spacing %lld x %lld", (long long)vx, (long long)vy);
  const int64_t nx = p->W / vx, ny = p->H / vy;  // Eq. nxyK
  if (nx < 1 || ny < 1) return fail(GMMSP_E_SIZE, "seed spacing exceeds the image");
  g->vx = (int32_t)vx;
  g->vy = (int32_t)vy;
  g->nx = (int32_t)nx;
  g->ny = (int32_t)ny;
  g->K = (int32_t)(nx * ny);
  g->ncx = (int32_t)((p->W + vx - 1) / vx);
  g->ncy = (int32_t)((p->H + vy - 1) / vy);
  return GMMSP_OK;
}

int check_params(const gmmsp_params* p) {
  if (!(p->eps_s > 0) || !(p->eps_c > 0) || !(p->lambda > 0) || !(p->n_min >= 0))
    return fail(GMMSP_E_INVAL, "eps_s, eps_c, lambda must be > 0 and n_min >= 0");
  if (p->cov_mode < 0 || p->cov_mode > 3)
    return fail(GMMSP_E_INVAL, "cov_mode %d is not supported (0, 1, 2 or 3)", p->cov_mode);
  return GMMSP_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t img, state, ll_hist, cell, sp, theta, rec, part, llp, n_done, pers, total;
  int32_t n_cell = 0, n_sp = 0;
  int64_t n_pix = 0;
  int32_t cov_mode = 0;
};

int plan(int32_t n, const gmmsp_params* params, Layout* L, std::vector<ImgDesc>* descs) {
  if (n < 1 || !params) return fail(GMMSP_E_INVAL, "need at least one image");
  int64_t n_cell = 0, n_sp = 0, n_pix = 0;
  if (descs) descs->resize(n);
  for (int32_t b = 0; b < n; ++b) {
    gmmsp_grid_info g;
    int rc = grid_of(&params[b], &g);
    if (rc) return fail(rc, "image %d: %s", b, g_err.c_str());
    rc = check_params(&params[b]);
    if (rc) return fail(rc, "image %d: %s", b, g_err.c_str());
    if (params[b].cov_mode != params[0].cov_mode)
      return fail(GMMSP_E_INVAL, "image %d: every image of a batch needs the same cov_mode", b);
    // the E-step addresses a chunk's rows by 32-bit byte offsets from its first row
    if (params[b].W > kMaxWidth)
      return fail(GMMSP_E_SIZE, "image %d: wider than %d pixels", b, kMaxWidth);
    if (descs) {
      ImgDesc& d = (*descs)[b];
      memset(&d, 0, sizeof(d));
      d.W = params[b].W; d.H = params[b].H; d.vx = g.vx; d.vy = g.vy;
      d.nx = g.nx; d.ny = g.ny; d.ncx = g.ncx; d.ncy = g.ncy;
      d.pix_off = n_pix;
      d.cell_off = (int32_t)n_cell;
      d.sp_off = (int32_t)n_sp;
      d.K = g.K;
      d.ncells = g.ncx * g.ncy;
      d.eps_s = params[b].eps_s; d.eps_c = params[b].eps_c;
      d.lam = params[b].lambda; d.n_min = params[b].n_min;
      // ln of the largest density the eigenvalue floors allow (det Sigma >= the
      // product of the floors): -(D/2) ln 2pi - (1/2)(2 ln eps_s + (D - 2) ln eps_c),
      // D = 5, or 3 for a grayscale image
      const double dim = params[b].cov_mode == 3 ? 3.0 : 5.0;
      d.lncmax = -0.5 * dim * log(2.0 * M_PI) -
                 0.5 * (2.0 * log(d.eps_s) + (dim - 2.0) * log(d.eps_c));
    }
    n_cell += (int64_t)g.ncx * g.ncy;
    n_sp += g.K;
    n_pix += (int64_t)params[b].W * params[b].H;
  }
  if (n_cell > INT32_MAX / 16 || n_sp > INT32_MAX / 16) return fail(GMMSP_E_SIZE, "batch too large");
  size_t o = 0;
  L->img = o;     o = align256(o + sizeof(ImgDesc) * n);
  L->state = o;   o = align256(o + sizeof(ImgState) * n);
  L->ll_hist = o; o = align256(o + sizeof(double) * (size_t)kLLCap * n);
  L->cell = o;    o = align256(o + sizeof(CellDesc) * n_cell);
  L->sp = o;      o = align256(o + sizeof(SpDesc) * n_sp);
  L->cov_mode = params[0].cov_mode;
  L->theta = o;   o = align256(o + sizeof(double) * theta_row_of(L->cov_mode) * n_sp);
  L->rec = o;     o = align256(o + sizeof(float) * rec_floats_of(L->cov_mode) * kSlots * n_cell);
  L->part = o;    o = align256(o + sizeof(double) * kPartStride * kMaxWpc * n_cell);
  L->llp = o;     o = align256(o + sizeof(double) * kMaxWpc * n_cell);
  L->n_done = o;  o = align256(o + sizeof(int32_t));
  L->pers = o;    o = align256(o + sizeof(PersistArea));
  L->total = o;
  L->n_cell = (int32_t)n_cell;
  L->n_sp = (int32_t)n_sp;
  L->n_pix = n_pix;
  return GMMSP_OK;
}

}  // namespace

namespace {

// warm-start layer table: input / output channels, B-operand shapes of the
// forward conv and of the input-gradient conv, parameter offsets
struct WsLayer {
  int cin, cout, cinp, nk, nt;   // forward: padded input channels, K chunks, column tiles
  int tcinp, tnk, tnt;           // input gradient (layers 2..4)
  size_t w_off, b_off;
};
constexpr WsLayer kWs[4] = {
    {16, 32, 16, 5, 2, 0, 0, 0, 0, 4608},
    {32, 32, 32, 9, 2, 32, 9, 2, 4640, 13856},
    {32, 32, 32, 9, 2, 32, 9, 2, 13888, 23104},
    {32, 10, 32, 9, 1, 16, 5, 2, 23136, 26016},
};
constexpr int kWsParams = 26026;
constexpr int kWsMaxSplits = 1024;
static_assert(kWsParams == GMMSP_WS_NPARAM, "parameter count");
static_assert(kMaxWidth == GMMSP_MAX_WIDTH, "widest image");

struct WsState {
  bool attached = false;
  int32_t* nbr = nullptr;
  float* feat = nullptr;
  uint16_t* x0 = nullptr;
  uint16_t* y[3] = {};
  float* out = nullptr;
  float* tgt = nullptr;
  uint16_t* g4 = nullptr;
  uint16_t* g[3] = {};
  uint16_t* wf[4] = {};
  uint16_t* wt[4] = {};
  float* part = nullptr;
  float* grad = nullptr;
  double* loss_part = nullptr;
  double* loss_sum = nullptr;
  size_t sizes[12] = {};
  void* ptrs[12] = {};
};

}  // namespace

struct gmmsp_handle {
  WsState ws;
  int32_t n_img = 0;
  int64_t n_pix = 0;
  std::vector<ImgDesc> img;
  std::vector<int64_t> pairs;  // sum_i |K_i| per image
  DevPtrs P{};
  bool initialised = false;
  // pipelined convergence checks: n_done snapshots in pinned host memory
  static constexpr int kRing = 4;
  int32_t* done_ring = nullptr;
  hipEvent_t done_ev[kRing] = {};
  // graph replay of em passes: a private stream joined to the caller's by events
  int32_t graph_passes = 0;
  hipStream_t gstream = nullptr;
  hipEvent_t gev_in = nullptr, gev_out = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  const float* g_lab = nullptr;
  double g_tol = 0.0;
  int32_t g_len = 0, g_wpc = 0, g_glanes = 0, g_estep = -1, g_rc = 0;
  // an upper bound of every image's pass count since the state's last reset
  int64_t t_bound = 0;
  // persistent T-mode passes: the workspace region and its pinned host image
  bool persistent = false;
  PersistArea* pers_dev = nullptr;
  PersistArea* pers_host = nullptr;
  // E-step kernel timing
  bool profile = false;
  std::vector<hipEvent_t> ev;
  double prof_ms = 0.0;
  int32_t prof_launches = 0;
  int64_t prof_pix = 0, prof_pairs = 0;
  ~gmmsp_handle() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : done_ev)
      if (e) (void)hipEventDestroy(e);
    if (done_ring) (void)hipHostFree(done_ring);
    if (pers_host) (void)hipHostFree(pers_host);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (gev_in) (void)hipEventDestroy(gev_in);
    if (gev_out) (void)hipEventDestroy(gev_out);
    if (gstream) (void)hipStreamDestroy(gstream);
  }
};

namespace {

// sum over windows of Eq. Ik along one axis: sum_k (min(n, v(k+2)) - max(0, v(k-1)))
int64_t window_extent_sum(int64_t n_pixels, int64_t v, int64_t n_seeds) {
  int64_t s = 0;
  for (int64_t k = 0; k < n_seeds; ++k) {
    const int64_t b = v * (k - 1) > 0 ? v * (k - 1) : 0;
    const int64_t e = v * (k + 2) < n_pixels ? v * (k + 2) : n_pixels;
    s += e - b;
  }
  return s;
}

}  // namespace

extern "C" {

const char* gmmsp_last_error(void) { return g_err.c_str(); }

int gmmsp_grid(const gmmsp_params* params, gmmsp_grid_info* out) { return grid_of(params, out); }

int gmmsp_workspace_bytes(int32_t n_images, const gmmsp_params* params, size_t* bytes) {
  if (!bytes) return fail(GMMSP_E_INVAL, "null pointer");
  Layout L;
  int rc = plan(n_images, params, &L, nullptr);
  if (rc) return rc;
  *bytes = L.total;
  return GMMSP_OK;
}

int gmmsp_create(int32_t n_images, const gmmsp_params* params, void* workspace_dev,
                 size_t workspace_bytes, void* stream, gmmsp_handle** out) {
  if (!out || !workspace_dev) return fail(GMMSP_E_INVAL, "null pointer");
  *out = nullptr;
  if (((uintptr_t)workspace_dev) & 255) return fail(GMMSP_E_INVAL, "workspace not 256-byte aligned");
  Layout L;
  std::vector<ImgDesc> descs;
  int rc = plan(n_images, params, &L, &descs);
  if (rc) return rc;
  if (workspace_bytes < L.total)
    return fail(GMMSP_E_SIZE, "workspace %zu bytes < %zu needed", workspace_bytes, L.total);

  std::vector<CellDesc> cells;
  std::vector<SpDesc> sps;
  try {  // the host tables of the batch; no exception leaves the ABI
    cells.reserve(L.n_cell);
    sps.reserve(L.n_sp);
  } catch (const std::bad_alloc&) {
    return fail(GMMSP_E_NOMEM, "out of host memory for %d cells", L.n_cell);
  }
  for (int32_t b = 0; b < n_images; ++b) {
    const ImgDesc& d = descs[b];
    for (int cy = 0; cy < d.ncy; ++cy)
      for (int cx = 0; cx < d.ncx; ++cx) cells.push_back(CellDesc{b, cx, cy, 0});
    for (int ky = 0; ky < d.ny; ++ky)
      for (int kx = 0; kx < d.nx; ++kx) sps.push_back(SpDesc{b, kx, ky, 0});
  }
  gmmsp_handle* h = new (std::nothrow) gmmsp_handle();
  if (!h) return fail(GMMSP_E_NOMEM, "out of host memory");
  char* base = (char*)workspace_dev;
  h->n_img = n_images;
  h->n_pix = L.n_pix;
  h->img = descs;
  for (const ImgDesc& d : descs)  // sum_i |K_i| = sum_k |I_k|, a product of axis sums
    h->pairs.push_back(window_extent_sum(d.W, d.vx, d.nx) * window_extent_sum(d.H, d.vy, d.ny));
  DevPtrs& P = h->P;
  P.img = (const ImgDesc*)(base + L.img);
  P.state = (ImgState*)(base + L.state);
  P.ll_hist = (double*)(base + L.ll_hist);
  P.cell = (const CellDesc*)(base + L.cell);
  P.sp = (const SpDesc*)(base + L.sp);
  P.theta = (double*)(base + L.theta);
  P.rec = (float*)(base + L.rec);
  P.part = (double*)(base + L.part);
  P.llp = (double*)(base + L.llp);
  P.n_done = (int32_t*)(base + L.n_done);
  h->pers_dev = (PersistArea*)(base + L.pers);
  P.n_img = n_images;
  P.n_cell = L.n_cell;
  P.n_sp = L.n_sp;
  P.wpc = 1;
  P.glanes = 1;
  P.cov_mode = L.cov_mode;
  // the slot-lane statistics pass covers cells up to 56 pixels wide (split
  // colour blocks only); otherwise the pixel-lane pass runs
  int32_t max_vx = 0;
  for (const ImgDesc& d : descs) max_vx = std::max(max_vx, d.vx);
  P.estep = 0;
  if (P.cov_mode == 0 && slots_shape(max_vx, &P.slot_j, &P.slot_rc)) P.estep = 1;
  P.slot_rc_max = P.slot_rc;

  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync((void*)P.img, descs.data(), sizeof(ImgDesc) * n_images,
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync((void*)P.cell, cells.data(), sizeof(CellDesc) * cells.size(),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync((void*)P.sp, sps.data(), sizeof(SpDesc) * sps.size(),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_clear_records(P, s);
  if (e == hipSuccess) e = launch_reset_state(P, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipHostMalloc((void**)&h->done_ring, sizeof(int32_t) * gmmsp_handle::kRing);
  if (e == hipSuccess) e = hipHostMalloc((void**)&h->pers_host, sizeof(PersistArea));
  for (int i = 0; i < gmmsp_handle::kRing && e == hipSuccess; ++i)
    e = hipEventCreateWithFlags(&h->done_ev[i], hipEventDisableTiming);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e, "gmmsp_create");
  }
  *out = h;
  return GMMSP_OK;
}

int gmmsp_destroy(gmmsp_handle* h) {
  delete h;
  return GMMSP_OK;
}

int gmmsp_batch_info(const gmmsp_handle* h, int32_t* n_images, int64_t* n_pixels,
                     int64_t* n_superpixels) {
  if (!h) return fail(GMMSP_E_INVAL, "null handle");
  if (n_images) *n_images = h->n_img;
  if (n_pixels) *n_pixels = h->n_pix;
  if (n_superpixels) *n_superpixels = h->P.n_sp;
  return GMMSP_OK;
}

int gmmsp_image_grid(const gmmsp_handle* h, int32_t b, gmmsp_grid_info* out) {
  if (!h || !out) return fail(GMMSP_E_INVAL, "null pointer");
  if (b < 0 || b >= h->n_img) return fail(GMMSP_E_INVAL, "image %d out of range", b);
  const ImgDesc& d = h->img[b];
  *out = gmmsp_grid_info{d.vx, d.vy, d.nx, d.ny, d.K, d.ncx, d.ncy};
  return GMMSP_OK;
}

int gmmsp_init_seeds(gmmsp_handle* h, const float* lab_dev, void* stream) {
  if (!h || !lab_dev) return fail(GMMSP_E_INVAL, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_reset_state(h->P, s);
  if (e == hipSuccess) h->t_bound = 0;
  if (e == hipSuccess) e = launch_init_seeds(h->P, lab_dev, s);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_init_seeds");
  h->initialised = true;
  return GMMSP_OK;
}

int gmmsp_set_params_dev(gmmsp_handle* h, const double* theta_dev, void* stream) {
  if (!h || !theta_dev) return fail(GMMSP_E_INVAL, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_reset_state(h->P, s);
  if (e == hipSuccess) h->t_bound = 0;
  if (e == hipSuccess) e = launch_set_params(h->P, theta_dev, s);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_set_params_dev");
  h->initialised = true;
  return GMMSP_OK;
}

int gmmsp_set_params(gmmsp_handle* h, const double* theta_host, void* stream) {
  if (!h || !theta_host) return fail(GMMSP_E_INVAL, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  // stage the rows in the partials area, which the next pass overwrites anyway
  const size_t bytes = sizeof(double) * theta_row_of(h->P.cov_mode) * (size_t)h->P.n_sp;
  if (bytes > sizeof(double) * kPartStride * (size_t)h->P.n_cell)
    return fail(GMMSP_E_SIZE, "staging area too small");
  hipError_t e = hipMemcpyAsync(h->P.part, theta_host, bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_reset_state(h->P, s);
  if (e == hipSuccess) h->t_bound = 0;
  if (e == hipSuccess) e = launch_set_params(h->P, h->P.part, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_set_params");
  h->initialised = true;
  return GMMSP_OK;
}

int gmmsp_get_params(gmmsp_handle* h, double* theta_host, void* stream) {
  if (!h || !theta_host) return fail(GMMSP_E_INVAL, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  const size_t row = theta_row_of(h->P.cov_mode);
  hipError_t e = hipMemcpyAsync(theta_host, h->P.theta, sizeof(double) * row * (size_t)h->P.n_sp,
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_get_params");
  return GMMSP_OK;
}

namespace {

// One em pass (Algorithm 1): the statistics pass, L(theta^t) and the stop
// rule, then the M-step gather.  Without the stop rule (rel_tol 0) no step of
// the pass waits for L, and the gather's launch forms it too: two launches.
// a and b (nullable) bracket the statistics pass with events.
static hipError_t em_pass(const DevPtrs& P, const float* lab, double rel_tol, hipStream_t s, hipEvent_t a,
                   hipEvent_t b) {
  hipError_t e = hipSuccess;
  if (a) e = hipEventRecord(a, s);
  if (e == hipSuccess) e = launch_estep_stats(P, lab, s);
  if (e == hipSuccess && b) e = hipEventRecord(b, s);
  if (rel_tol > 0.0) {
    if (e == hipSuccess) e = launch_ll_update(P, rel_tol, s);
    if (e == hipSuccess) e = launch_finalize(P, s);
  } else if (e == hipSuccess) {
    e = launch_finalize(P, s, true);
  }
  return e;
}

// Capture `len` em passes into a graph on the handle's private stream.
static int capture_passes(gmmsp_handle* h, const float* lab, double rel_tol, int32_t len) {
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->gexec = nullptr;
  h->graph = nullptr;
  hipError_t e = hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal);
  for (int32_t i = 0; i < len && e == hipSuccess; ++i)
    e = em_pass(h->P, lab, rel_tol, h->gstream, nullptr, nullptr);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(h->gstream, &g);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(e, "graph capture");
  }
  h->graph = g;
  h->g_lab = lab;
  h->g_tol = rel_tol;
  h->g_len = len;
  h->g_wpc = h->P.wpc;
  h->g_glanes = h->P.glanes;
  h->g_estep = h->P.estep;
  h->g_rc = h->P.slot_rc;
  return GMMSP_OK;
}

// Run whole chunks of graph_passes passes as graph launches; the stop test of
// each chunk is read while the next chunk is already queued.
static int run_graph_chunks(gmmsp_handle* h, const float* lab, int32_t max_iters, double rel_tol,
                     hipStream_t s, int32_t* done_iters, bool* all_done) {
  hipError_t e = hipSuccess;
  if (!h->gstream) e = hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking);
  if (e == hipSuccess && !h->gev_in) e = hipEventCreateWithFlags(&h->gev_in, hipEventDisableTiming);
  if (e == hipSuccess && !h->gev_out) e = hipEventCreateWithFlags(&h->gev_out, hipEventDisableTiming);
  if (e != hipSuccess) return hip_fail(e, "graph stream");
  const int32_t G = h->graph_passes;
  // the graph holds the kernels and arguments of the schedule it was captured with
  if (!h->gexec || h->g_lab != lab || h->g_tol != rel_tol || h->g_len != G || h->g_wpc != h->P.wpc ||
      h->g_glanes != h->P.glanes || h->g_estep != h->P.estep || h->g_rc != h->P.slot_rc) {
    int rc = capture_passes(h, lab, rel_tol, G);
    if (rc) return rc;
  }
  e = hipEventRecord(h->gev_in, s);
  if (e == hipSuccess) e = hipStreamWaitEvent(h->gstream, h->gev_in, 0);
  int32_t it = 0, chunk = 0;
  *all_done = false;
  while (e == hipSuccess && it + G <= max_iters) {
    e = hipGraphLaunch(h->gexec, h->gstream);
    if (e != hipSuccess) break;
    it += G;
    if (rel_tol > 0.0) {
      const int slot = chunk % gmmsp_handle::kRing;
      e = hipMemcpyAsync(&h->done_ring[slot], h->P.n_done, sizeof(int32_t), hipMemcpyDeviceToHost,
                         h->gstream);
      if (e == hipSuccess) e = hipEventRecord(h->done_ev[slot], h->gstream);
      if (e == hipSuccess && chunk >= 1) {
        const int prev = (chunk - 1) % gmmsp_handle::kRing;
        e = hipEventSynchronize(h->done_ev[prev]);
        if (e == hipSuccess && h->done_ring[prev] >= h->n_img) *all_done = true;
      }
      if (*all_done) break;
    }
    ++chunk;
  }
  if (e == hipSuccess) e = hipEventRecord(h->gev_out, h->gstream);
  if (e == hipSuccess) e = hipStreamWaitEvent(s, h->gev_out, 0);
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  *done_iters = it;
  return GMMSP_OK;
}

// `iters` passes without the stop rule in one persistent launch (queued on s
// after the copy of the barrier and the DevPtrs it runs with).
static hipError_t persist_launch(gmmsp_handle* h, const float* lab, int32_t iters, hipStream_t s,
                          hipEvent_t a = nullptr, hipEvent_t b = nullptr) {
  h->pers_host->bar = GridBar{0u, 0u, 0, 0};
  h->pers_host->P = h->P;
  hipError_t e = hipMemcpyAsync(h->pers_dev, h->pers_host, sizeof(PersistArea),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess && a) e = hipEventRecord(a, s);
  if (e == hipSuccess) e = launch_persist(h->P, &h->pers_dev->P, lab, iters, &h->pers_dev->bar, s);
  if (e == hipSuccess && b) e = hipEventRecord(b, s);
  return e;
}

// Waits for the persistent launch and reports a grid barrier that ran out.
static int persist_check(gmmsp_handle* h, hipError_t e, hipStream_t s, const char* what) {
  if (e == hipSuccess)
    e = hipMemcpyAsync(&h->pers_host->bar, &h->pers_dev->bar, sizeof(GridBar),
                       hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, what);
  if (h->pers_host->bar.err)
    return fail(GMMSP_E_STATE, "%s: a grid barrier wait ran out; the passes are incomplete", what);
  return GMMSP_OK;
}

static int run_persistent(gmmsp_handle* h, const float* lab, int32_t iters, hipStream_t s) {
  return persist_check(h, persist_launch(h, lab, iters, s), s, "persistent launch");
}

static bool persistent_applies(const gmmsp_handle* h, double rel_tol) {
  return h->persistent && rel_tol <= 0.0 && !h->profile && h->P.cov_mode == 0 && h->P.estep == 1;
}

}  // namespace

int gmmsp_em_iterate(gmmsp_handle* h, const float* lab_dev, int32_t max_iters, double rel_tol,
                     int32_t* iters_host, void* stream) {
  if (!h || !lab_dev) return fail(GMMSP_E_INVAL, "null pointer");
  if (!h->initialised) return fail(GMMSP_E_STATE, "handle not initialised");
  if (max_iters < 0) return fail(GMMSP_E_INVAL, "max_iters < 0");
  hipStream_t s = (hipStream_t)stream;
  std::vector<ImgState> st(h->n_img);
  hipError_t e = hipSuccess;
  // The passes counted since the state was last reset bound every image's
  // pass count; the device state is read (a wait for the stream) only when
  // that bound leaves the history cap in doubt, or to time the passes.
  if (h->profile || h->t_bound + max_iters > kLLCap) {
    e = hipMemcpyAsync(st.data(), h->P.state, sizeof(ImgState) * h->n_img, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "gmmsp_em_iterate");
    int32_t tmax = 0;
    for (const ImgState& x : st) tmax = x.t > tmax ? x.t : tmax;
    h->t_bound = tmax;
    if ((int64_t)tmax + max_iters > kLLCap)
      return fail(GMMSP_E_STATE, "more than %d passes since the last initialisation", kLLCap);
  }
  h->t_bound += max_iters;  // at most this many passes follow, whatever happens below
  if (h->profile && (int32_t)h->ev.size() < 2 * max_iters) {
    const size_t need = 2 * (size_t)max_iters;
    while (h->ev.size() < need) {
      hipEvent_t x;
      e = hipEventCreate(&x);
      if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
      h->ev.push_back(x);
    }
  }
  int32_t launched = 0;
  int32_t it = 0;
  bool all_done = false;
  if (max_iters > 0 && persistent_applies(h, rel_tol)) {
    int rc = run_persistent(h, lab_dev, max_iters, s);
    if (rc) return rc;
    it = launched = max_iters;
  } else if (h->graph_passes > 0 && max_iters >= h->graph_passes && !h->profile) {
    int rc = run_graph_chunks(h, lab_dev, max_iters, rel_tol, s, &it, &all_done);
    if (rc) return rc;
    launched = it;
  }
  for (; it < max_iters && !all_done; ++it) {
    e = em_pass(h->P, lab_dev, rel_tol, s, h->profile ? h->ev[2 * it] : nullptr,
                h->profile ? h->ev[2 * it + 1] : nullptr);
    if (e != hipSuccess) return hip_fail(e, "em pass");
    ++launched;
    if (rel_tol > 0.0) {
      // snapshot the stopped-image count after pass it; wait for the snapshot
      // of pass it-1 while pass it is already queued, so the GPU never idles
      const int slot = it % gmmsp_handle::kRing;
      e = hipMemcpyAsync(&h->done_ring[slot], h->P.n_done, sizeof(int32_t), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipEventRecord(h->done_ev[slot], s);
      if (e == hipSuccess && it >= 1) {
        const int prev = (it - 1) % gmmsp_handle::kRing;
        e = hipEventSynchronize(h->done_ev[prev]);
        // every image had stopped after pass it-1; the queued pass it skips them all
        if (e == hipSuccess && h->done_ring[prev] >= h->n_img) break;
      }
      if (e != hipSuccess) return hip_fail(e, "em convergence check");
    }
  }
  if (h->profile) {
    std::vector<ImgState> st2(h->n_img);
    e = hipMemcpyAsync(st2.data(), h->P.state, sizeof(ImgState) * h->n_img, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "gmmsp_em_iterate profile");
    for (int32_t it = 0; it < launched; ++it) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, h->ev[2 * it], h->ev[2 * it + 1]);
      if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
      h->prof_ms += ms;
    }
    h->prof_launches += launched;
    for (int32_t b = 0; b < h->n_img; ++b) {
      const int64_t evals = st2[b].t - st[b].t;  // E-steps that image b took part in
      h->prof_pix += evals * (int64_t)h->img[b].W * h->img[b].H;
      h->prof_pairs += evals * h->pairs[b];
    }
  }
  if (iters_host) {
    e = hipMemcpyAsync(st.data(), h->P.state, sizeof(ImgState) * h->n_img, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "gmmsp_em_iterate");
    for (int32_t b = 0; b < h->n_img; ++b) iters_host[b] = st[b].iters;
  } else {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "gmmsp_em_iterate");
  }
  return GMMSP_OK;
}

int gmmsp_ll_history(gmmsp_handle* h, int32_t b, double* out_host, int32_t cap, int32_t* n,
                     void* stream) {
  if (!h || !out_host || !n) return fail(GMMSP_E_INVAL, "null pointer");
  if (b < 0 || b >= h->n_img) return fail(GMMSP_E_INVAL, "image %d out of range", b);
  hipStream_t s = (hipStream_t)stream;
  ImgState st;
  hipError_t e = hipMemcpyAsync(&st, h->P.state + b, sizeof(st), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_ll_history");
  int32_t cnt = st.t < kLLCap ? st.t : kLLCap;
  if (cnt > cap) cnt = cap;
  if (cnt > 0) {
    e = hipMemcpyAsync(out_host, h->P.ll_hist + (size_t)b * kLLCap, sizeof(double) * cnt,
                       hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "gmmsp_ll_history");
  }
  *n = cnt;
  return GMMSP_OK;
}

int gmmsp_label(gmmsp_handle* h, const float* lab_dev, int32_t* labels_dev, double* ll_host,
                void* stream) {
  if (!h || !lab_dev || !labels_dev) return fail(GMMSP_E_INVAL, "null pointer");
  if (!h->initialised) return fail(GMMSP_E_STATE, "handle not initialised");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_label(h->P, lab_dev, labels_dev, s);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_label");
  if (ll_host) {
    std::vector<ImgState> st(h->n_img);
    e = hipMemcpyAsync(st.data(), h->P.state, sizeof(ImgState) * h->n_img, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "gmmsp_label");
    for (int32_t b = 0; b < h->n_img; ++b) ll_host[b] = st[b].ll_final;
  }
  return GMMSP_OK;
}

int gmmsp_export_responsibilities(gmmsp_handle* h, const float* lab_dev, float* R_dev,
                                  void* stream) {
  if (!h || !lab_dev || !R_dev) return fail(GMMSP_E_INVAL, "null pointer");
  if (!h->initialised) return fail(GMMSP_E_STATE, "handle not initialised");
  hipError_t e = launch_export_R(h->P, lab_dev, R_dev, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_export_responsibilities");
  return GMMSP_OK;
}

int gmmsp_set_schedule(gmmsp_handle* h, int32_t waves_per_cell) {
  if (!h) return fail(GMMSP_E_INVAL, "null handle");
  if (waves_per_cell != 1 && waves_per_cell != 2 && waves_per_cell != 4)
    return fail(GMMSP_E_INVAL, "waves per cell must be 1, 2 or 4");
  if (h->P.cov_mode != 0 && waves_per_cell != 1)
    return fail(GMMSP_E_INVAL, "cov_mode %d runs one wave per cell", h->P.cov_mode);
  h->P.wpc = waves_per_cell;
  return GMMSP_OK;
}

int gmmsp_get_schedule(const gmmsp_handle* h, int32_t* waves_per_cell) {
  if (!h || !waves_per_cell) return fail(GMMSP_E_INVAL, "null pointer");
  *waves_per_cell = h->P.wpc;
  return GMMSP_OK;
}

int gmmsp_set_estep_kernel(gmmsp_handle* h, int32_t kind) {
  if (!h) return fail(GMMSP_E_INVAL, "null handle");
  if (kind != 0 && kind != 1) return fail(GMMSP_E_INVAL, "statistics pass kind must be 0 or 1");
  if (kind == 1) {
    if (h->P.cov_mode != 0) return fail(GMMSP_E_INVAL, "the slot-lane pass needs cov_mode 0");
    if (!h->P.slot_j) return fail(GMMSP_E_INVAL, "the slot-lane pass covers cells up to 56 pixels wide");
  }
  h->P.estep = kind;
  return GMMSP_OK;
}

int gmmsp_get_estep_kernel(const gmmsp_handle* h, int32_t* kind) {
  if (!h || !kind) return fail(GMMSP_E_INVAL, "null pointer");
  *kind = h->P.estep;
  return GMMSP_OK;
}

int gmmsp_set_slot_rows(gmmsp_handle* h, int32_t rows) {
  if (!h) return fail(GMMSP_E_INVAL, "null handle");
  if (!h->P.slot_j) return fail(GMMSP_E_INVAL, "this batch has no slot-lane pass");
  int32_t max_vx = 0;
  for (const ImgDesc& d : h->img) max_vx = std::max(max_vx, d.vx);
  int J = 0, max_rc = 0, built[3] = {0, 0, 0};
  (void)slots_shape(max_vx, &J, &max_rc);
  const int n = slots_rows(J, max_rc, built, 3);
  for (int i = 0; i < n; ++i)
    if (built[i] == rows) {
      h->P.slot_rc = rows;
      return GMMSP_OK;
    }
  return fail(GMMSP_E_INVAL, "%d rows per chunk is not built for cells %d pixels wide", rows, max_vx);
}

int gmmsp_get_slot_rows(const gmmsp_handle* h, int32_t* rows) {
  if (!h || !rows) return fail(GMMSP_E_INVAL, "null pointer");
  *rows = h->P.slot_j ? h->P.slot_rc : 0;
  return GMMSP_OK;
}

int gmmsp_set_gather_lanes(gmmsp_handle* h, int32_t lanes_per_superpixel) {
  if (!h) return fail(GMMSP_E_INVAL, "null handle");
  if (lanes_per_superpixel != 1 && lanes_per_superpixel != 4 && lanes_per_superpixel != 16)
    return fail(GMMSP_E_INVAL, "lanes per superpixel must be 1, 4 or 16");
  if (h->P.cov_mode != 0 && lanes_per_superpixel != 1)
    return fail(GMMSP_E_INVAL, "cov_mode %d gathers with one lane per superpixel", h->P.cov_mode);
  h->P.glanes = lanes_per_superpixel;
  return GMMSP_OK;
}

int gmmsp_get_gather_lanes(const gmmsp_handle* h, int32_t* lanes_per_superpixel) {
  if (!h || !lanes_per_superpixel) return fail(GMMSP_E_INVAL, "null pointer");
  *lanes_per_superpixel = h->P.glanes;
  return GMMSP_OK;
}

int gmmsp_set_persistent(gmmsp_handle* h, int32_t on) {
  if (!h) return fail(GMMSP_E_INVAL, "null handle");
  if (on != 0 && on != 1) return fail(GMMSP_E_INVAL, "persistent flag %d not 0 or 1", on);
  if (on && (h->P.cov_mode != 0 || !h->P.slot_j))
    return fail(GMMSP_E_INVAL, "the persistent launch runs the slot-lane pass, which this batch has not");
  h->persistent = on != 0;
  return GMMSP_OK;
}

int gmmsp_get_persistent(const gmmsp_handle* h, int32_t* on) {
  if (!h || !on) return fail(GMMSP_E_INVAL, "null pointer");
  *on = h->persistent ? 1 : 0;
  return GMMSP_OK;
}

int gmmsp_set_graph_passes(gmmsp_handle* h, int32_t passes) {
  if (!h) return fail(GMMSP_E_INVAL, "null handle");
  if (passes < 0 || passes > 256) return fail(GMMSP_E_INVAL, "graph passes %d outside [0, 256]", passes);
  h->graph_passes = passes;
  return GMMSP_OK;
}

// Both autotuners try their candidates from the smallest up and move to a
// larger one only when it beats the best so far by more than 3 %, so that
// timing noise does not pick a schedule that is no faster.
constexpr double kTuneMargin = 0.97;
constexpr int32_t kTuneWarm = 3;  // untimed passes before the timed ones

int gmmsp_autotune(gmmsp_handle* h, const float* lab_dev, int32_t passes, double* ms_host,
                   int32_t* chosen, void* stream) {
  if (!h || !lab_dev || !chosen) return fail(GMMSP_E_INVAL, "null pointer");
  if (passes < 1 || passes > 64) return fail(GMMSP_E_INVAL, "passes %d outside [1, 64]", passes);
  hipStream_t s = (hipStream_t)stream;
  h->t_bound = kLLCap;  // the tuner's passes are not counted: unknown until its last reset
  // candidates in order of preference: the slot-lane pass with each rows-per-
  // chunk value (largest first), then the pixel-lane pass; 1, 2, 4 waves per
  // cell each.  Index 3 v + w, v = 0..2 the rows values, v = 3 the pixel-lane
  // pass, w = 0..2 the waves per cell.
  struct Cand { int32_t kind, rc, wpc, idx; };
  std::vector<Cand> cands;
  const int32_t wpcs[3] = {1, 2, 4};
  if (h->P.cov_mode != 0) {
    cands.push_back({0, 0, 1, 9});  // the other covariance models have one schedule
  } else {
    int max_j = 0, max_rc = 0;
    int rows[3] = {0, 0, 0};
    int n_rows = 0;
    int32_t max_vx = 0;
    for (const ImgDesc& d : h->img) max_vx = std::max(max_vx, d.vx);
    if (slots_shape(max_vx, &max_j, &max_rc)) n_rows = slots_rows(max_j, max_rc, rows, 3);
    for (int v = 0; v < n_rows; ++v)
      for (int w = 0; w < 3; ++w) cands.push_back({1, rows[v], wpcs[w], 3 * v + w});
    for (int w = 0; w < 3; ++w) cands.push_back({0, h->P.slot_rc, wpcs[w], 9 + w});
  }
  if (ms_host)
    for (int c = 0; c < GMMSP_TUNE_CANDIDATES; ++c) ms_host[c] = -1.0;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  // two rounds over the candidates, each candidate's faster round counts: the
  // first candidates of a round would otherwise also pay for the GPU's clock
  // ramp at the start
  std::vector<double> tmin(cands.size(), 0.0);
  for (int round = 0; round < 2 && e == hipSuccess; ++round) {
    for (size_t c = 0; c < cands.size() && e == hipSuccess; ++c) {
      h->P.estep = cands[c].kind;
      if (h->P.slot_j) h->P.slot_rc = cands[c].rc;
      h->P.wpc = cands[c].wpc;
      e = launch_reset_state(h->P, s);
      if (e == hipSuccess) e = launch_init_seeds(h->P, lab_dev, s);
      double tot = 0.0;
      // kTuneWarm untimed passes (the first passes from the grid seeds run
      // slower than later ones), then `passes` timed ones: whole em passes, as
      // the waves per cell also set the work of the gather
      for (int32_t i = 0; i < kTuneWarm + passes && e == hipSuccess; ++i) {
        e = hipEventRecord(a, s);
        if (e == hipSuccess) e = em_pass(h->P, lab_dev, 0.0, s, nullptr, nullptr);
        if (e == hipSuccess) e = hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (i >= kTuneWarm) tot += ms;
      }
      if (round == 0 || tot < tmin[c]) tmin[c] = tot;
    }
  }
  double best = 0.0;
  Cand pick = cands[0];
  for (size_t c = 0; c < cands.size(); ++c) {
    if (ms_host) ms_host[cands[c].idx] = tmin[c];
    if (c == 0 || tmin[c] < kTuneMargin * best) {
      best = tmin[c];
      pick = cands[c];
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  h->P.estep = pick.kind;
  if (h->P.slot_j) h->P.slot_rc = pick.rc;
  h->P.wpc = pick.wpc;
  if (e == hipSuccess) e = launch_reset_state(h->P, s);
  if (e == hipSuccess) h->t_bound = 0;
  if (e == hipSuccess) e = launch_init_seeds(h->P, lab_dev, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_autotune");
  h->initialised = true;
  *chosen = pick.wpc;
  return GMMSP_OK;
}

int gmmsp_autotune_gather(gmmsp_handle* h, const float* lab_dev, int32_t passes, double* ms_host,
                          int32_t* chosen, void* stream) {
  if (!h || !lab_dev || !chosen) return fail(GMMSP_E_INVAL, "null pointer");
  if (passes < 1 || passes > 64) return fail(GMMSP_E_INVAL, "passes %d outside [1, 64]", passes);
  hipStream_t s = (hipStream_t)stream;
  h->t_bound = kLLCap;  // the tuner's passes are not counted: unknown until its last reset
  const int32_t cand[3] = {1, 4, 16};
  const int n_cand = h->P.cov_mode != 0 ? 1 : 3;
  if (ms_host)
    for (int c = 0; c < 3; ++c) ms_host[c] = -1.0;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  // whole em passes with each gather, two rounds, each candidate's faster counts
  double tmin[3] = {0.0, 0.0, 0.0};
  for (int round = 0; round < 2 && e == hipSuccess; ++round) {
    for (int c = 0; c < n_cand && e == hipSuccess; ++c) {
      h->P.glanes = cand[c];
      e = launch_reset_state(h->P, s);
      if (e == hipSuccess) e = launch_init_seeds(h->P, lab_dev, s);
      double tot = 0.0;
      for (int32_t i = 0; i < kTuneWarm + passes && e == hipSuccess; ++i) {
        e = hipEventRecord(a, s);
        if (e == hipSuccess) e = em_pass(h->P, lab_dev, 0.0, s, nullptr, nullptr);
        if (e == hipSuccess) e = hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (i >= kTuneWarm) tot += ms;
      }
      if (round == 0 || tot < tmin[c]) tmin[c] = tot;
    }
  }
  double best = 0.0;
  int32_t pick = 1;
  for (int c = 0; c < n_cand; ++c) {
    if (ms_host) ms_host[c] = tmin[c];
    if (c == 0 || tmin[c] < kTuneMargin * best) {
      best = tmin[c];
      pick = cand[c];
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  h->P.glanes = pick;
  if (e == hipSuccess) e = launch_reset_state(h->P, s);
  if (e == hipSuccess) h->t_bound = 0;
  if (e == hipSuccess) e = launch_init_seeds(h->P, lab_dev, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_autotune_gather");
  h->initialised = true;
  *chosen = pick;
  return GMMSP_OK;
}

int gmmsp_autotune_persistent(gmmsp_handle* h, const float* lab_dev, int32_t passes,
                              double* ms_host, int32_t* chosen, void* stream) {
  if (!h || !lab_dev || !chosen) return fail(GMMSP_E_INVAL, "null pointer");
  if (passes < 1 || passes > 64) return fail(GMMSP_E_INVAL, "passes %d outside [1, 64]", passes);
  hipStream_t s = (hipStream_t)stream;
  h->t_bound = kLLCap;  // the tuner's passes are not counted: unknown until its last reset
  if (ms_host)
    for (int c = 0; c < 4; ++c) ms_host[c] = -1.0;
  int rows[3] = {0, 0, 0};
  const int n_rows =
      h->P.cov_mode == 0 && h->P.slot_j ? slots_rows(h->P.slot_j, h->P.slot_rc_max, rows, 3) : 0;
  const int32_t kind0 = h->P.estep, rc0 = h->P.slot_rc;
  h->persistent = false;
  hipError_t e = hipSuccess;
  // candidate 0: per-pass launches with the schedule in effect; 1 + v: the
  // persistent launch of the slot-lane pass with the v-th rows value.  Wall
  // time from the first launch to the end of the last pass (host launch cost
  // included: that is what the launch form changes), two rounds, each
  // candidate's faster round counts.
  double tmin[4] = {0.0, 0.0, 0.0, 0.0};
  int rc = GMMSP_OK;
  for (int round = 0; round < 2 && e == hipSuccess && rc == GMMSP_OK; ++round) {
    for (int c = 0; c <= n_rows && e == hipSuccess && rc == GMMSP_OK; ++c) {
      h->P.estep = c == 0 ? kind0 : 1;
      if (h->P.slot_j) h->P.slot_rc = c == 0 ? rc0 : rows[c - 1];
      e = launch_reset_state(h->P, s);
      if (e == hipSuccess) e = launch_init_seeds(h->P, lab_dev, s);
      double ms = 0.0;
      if (c == 0) {
        for (int32_t i = 0; i < kTuneWarm && e == hipSuccess; ++i)
          e = em_pass(h->P, lab_dev, 0.0, s, nullptr, nullptr);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        const auto t0 = std::chrono::steady_clock::now();
        for (int32_t i = 0; i < passes && e == hipSuccess; ++i)
          e = em_pass(h->P, lab_dev, 0.0, s, nullptr, nullptr);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      } else {
        rc = persist_check(h, persist_launch(h, lab_dev, kTuneWarm, s), s, "gmmsp_autotune_persistent");
        const auto t0 = std::chrono::steady_clock::now();
        if (rc == GMMSP_OK)
          rc = persist_check(h, persist_launch(h, lab_dev, passes, s), s, "gmmsp_autotune_persistent");
        ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      }
      if (round == 0 || ms < tmin[c]) tmin[c] = ms;
    }
  }
  int pick = 0;
  double best = tmin[0];
  for (int c = 1; c <= n_rows; ++c)
    if (tmin[c] < kTuneMargin * best && (pick == 0 || tmin[c] < tmin[pick])) pick = c;
  if (ms_host)
    for (int c = 0; c <= n_rows; ++c) ms_host[c] = tmin[c];
  h->P.estep = pick == 0 ? kind0 : 1;
  if (h->P.slot_j) h->P.slot_rc = pick == 0 ? rc0 : rows[pick - 1];
  h->persistent = pick != 0;
  if (rc != GMMSP_OK) {
    h->P.estep = kind0;
    h->P.slot_rc = rc0;
    h->persistent = false;
    return rc;
  }
  if (e == hipSuccess) e = launch_reset_state(h->P, s);
  if (e == hipSuccess) h->t_bound = 0;
  if (e == hipSuccess) e = launch_init_seeds(h->P, lab_dev, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_autotune_persistent");
  h->initialised = true;
  *chosen = h->persistent ? 1 : 0;
  return GMMSP_OK;
}

int gmmsp_profile_enable(gmmsp_handle* h, int32_t enable) {
  if (!h) return fail(GMMSP_E_INVAL, "null handle");
  h->profile = enable != 0;
  return GMMSP_OK;
}

int gmmsp_profile_read(gmmsp_handle* h, double* estep_ms, int32_t* launches, int64_t* pixel_evals,
                       int64_t* pair_evals, int32_t reset) {
  if (!h) return fail(GMMSP_E_INVAL, "null handle");
  if (estep_ms) *estep_ms = h->prof_ms;
  if (launches) *launches = h->prof_launches;
  if (pixel_evals) *pixel_evals = h->prof_pix;
  if (pair_evals) *pair_evals = h->prof_pairs;
  if (reset) {
    h->prof_ms = 0.0;
    h->prof_launches = 0;
    h->prof_pix = 0;
    h->prof_pairs = 0;
  }
  return GMMSP_OK;
}

int gmmsp_export_candidates(gmmsp_handle* h, int32_t* cand_dev, void* stream) {
  if (!h || !cand_dev) return fail(GMMSP_E_INVAL, "null pointer");
  if (!h->initialised) return fail(GMMSP_E_STATE, "handle not initialised");
  hipError_t e = launch_export_candidates(h->P, cand_dev, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_export_candidates");
  return GMMSP_OK;
}

// ---------------------------------------------------------------------------
// learned warm start
// ---------------------------------------------------------------------------
namespace {

struct WsLayoutSizes {
  size_t nbr, feat, x0, y, out, tgt, g4, g, wf[4], wt[4], part, grad, loss_part, loss_sum, total;
};

static WsLayoutSizes ws_sizes(const gmmsp_handle* h) {
  WsLayoutSizes z{};
  const size_t n = (size_t)h->P.n_sp;
  z.nbr = n * 9 * sizeof(int32_t);
  z.feat = n * 16 * sizeof(float);
  z.x0 = n * 16 * 2;
  z.y = n * 32 * 2;
  z.out = n * 16 * sizeof(float);
  z.tgt = n * 16 * sizeof(float);
  z.g4 = n * 16 * 2;
  z.g = n * 32 * 2;
  for (int l = 0; l < 4; ++l) {
    z.wf[l] = (size_t)kWs[l].nk * kWs[l].nt * 64 * 8 * 2;
    z.wt[l] = (size_t)kWs[l].tnk * kWs[l].tnt * 64 * 8 * 2;
  }
  z.part = (size_t)kWsMaxSplits * 32 * 9 * 32 * sizeof(float);
  z.grad = (size_t)kWsParams * sizeof(float);
  z.loss_part = (n / 256 + 2) * sizeof(double);
  z.loss_sum = sizeof(double);
  size_t t = 0;
  auto add = [&](size_t b) { t = align256(t + b); };
  add(z.nbr); add(z.feat); add(z.x0); for (int i = 0; i < 3; ++i) add(z.y);
  add(z.out); add(z.tgt); add(z.g4); for (int i = 0; i < 3; ++i) add(z.g);
  for (int l = 0; l < 4; ++l) { add(z.wf[l]); add(z.wt[l]); }
  add(z.part); add(z.grad); add(z.loss_part); add(z.loss_sum);
  z.total = t;
  return z;
}

static int ws_check(gmmsp_handle* h) {
  if (!h) return fail(GMMSP_E_INVAL, "null handle");
  if (!h->ws.attached) return fail(GMMSP_E_STATE, "warm-start workspace not attached");
  return GMMSP_OK;
}

static int ws_range(gmmsp_handle* h, int32_t b0, int32_t b1, int* p0, int* p1) {
  if (b0 < 0 || b1 > h->n_img || b0 >= b1) return fail(GMMSP_E_INVAL, "image range [%d, %d)", b0, b1);
  *p0 = h->img[b0].sp_off;
  *p1 = b1 < h->n_img ? h->img[b1].sp_off : h->P.n_sp;
  return GMMSP_OK;
}

static hipError_t ws_prep_all(gmmsp_handle* h, const float* params, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (int l = 0; l < 4 && e == hipSuccess; ++l) {
    const WsLayer& L = kWs[l];
    e = ws_launch_prep(params + L.w_off, L.cout, L.cin, L.cinp, L.nk, L.nt, 0, h->ws.wf[l], s);
    if (e == hipSuccess && l > 0)
      e = ws_launch_prep(params + L.w_off, L.cout, L.cin, L.tcinp, L.tnk, L.tnt, 1, h->ws.wt[l], s);
  }
  return e;
}

static hipError_t ws_forward_range(gmmsp_handle* h, const float* params, int p0, int p1, hipStream_t s) {
  WsState& W = h->ws;
  hipError_t e = ws_prep_all(h, params, s);
  const uint16_t* in = W.x0;
  for (int l = 0; l < 3 && e == hipSuccess; ++l) {
    e = ws_launch_conv(l + 1, 0, W.nbr, in, W.wf[l], params + kWs[l].b_off, kWs[l].cout, nullptr,
                       W.y[l], nullptr, p0, p1, s);
    in = W.y[l];
  }
  if (e == hipSuccess)
    e = ws_launch_conv(4, 1, W.nbr, in, W.wf[3], params + kWs[3].b_off, kWs[3].cout, nullptr,
                       nullptr, W.out, p0, p1, s);
  return e;
}

}  // namespace

int gmmsp_ws_workspace_bytes(const gmmsp_handle* h, size_t* bytes) {
  if (!h || !bytes) return fail(GMMSP_E_INVAL, "null pointer");
  if (h->P.cov_mode != 0) return fail(GMMSP_E_INVAL, "the warm start predicts the split colour blocks (cov_mode 0)");
  *bytes = ws_sizes(h).total;
  return GMMSP_OK;
}

int gmmsp_ws_attach(gmmsp_handle* h, void* ws_dev, size_t bytes, void* stream) {
  if (!h || !ws_dev) return fail(GMMSP_E_INVAL, "null pointer");
  if (h->P.cov_mode != 0) return fail(GMMSP_E_INVAL, "the warm start predicts the split colour blocks (cov_mode 0)");
  if (((uintptr_t)ws_dev) & 255) return fail(GMMSP_E_INVAL, "workspace not 256-byte aligned");
  const WsLayoutSizes z = ws_sizes(h);
  if (bytes < z.total) return fail(GMMSP_E_SIZE, "warm-start workspace %zu < %zu bytes", bytes, z.total);
  WsState& W = h->ws;
  char* b = (char*)ws_dev;
  size_t t = 0;
  auto take = [&](size_t n) { void* p = b + t; t = align256(t + n); return p; };
  W.nbr = (int32_t*)take(z.nbr);
  W.feat = (float*)take(z.feat);
  W.x0 = (uint16_t*)take(z.x0);
  for (int i = 0; i < 3; ++i) W.y[i] = (uint16_t*)take(z.y);
  W.out = (float*)take(z.out);
  W.tgt = (float*)take(z.tgt);
  W.g4 = (uint16_t*)take(z.g4);
  for (int i = 0; i < 3; ++i) W.g[i] = (uint16_t*)take(z.g);
  for (int l = 0; l < 4; ++l) {
    W.wf[l] = (uint16_t*)take(z.wf[l]);
    W.wt[l] = (uint16_t*)take(z.wt[l]);
  }
  W.part = (float*)take(z.part);
  W.grad = (float*)take(z.grad);
  W.loss_part = (double*)take(z.loss_part);
  W.loss_sum = (double*)take(z.loss_sum);
  void* ptrs[12] = {W.feat, W.x0, W.y[0], W.y[1], W.y[2], W.out, W.tgt, W.g4, W.g[2], W.g[1], W.g[0], W.grad};
  size_t sizes[12] = {z.feat, z.x0, z.y, z.y, z.y, z.out, z.tgt, z.g4, z.g, z.g, z.g, z.grad};
  for (int i = 0; i < 12; ++i) {
    W.ptrs[i] = ptrs[i];
    W.sizes[i] = sizes[i];
  }
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = ws_launch_nbr(h->P, W.nbr, s);
  if (e == hipSuccess) e = hipMemsetAsync(W.tgt, 0, z.tgt, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_ws_attach");
  W.attached = true;
  return GMMSP_OK;
}

int gmmsp_ws_features(gmmsp_handle* h, const float* lab_dev, void* stream) {
  int rc = ws_check(h);
  if (rc) return rc;
  if (!lab_dev) return fail(GMMSP_E_INVAL, "null pointer");
  hipError_t e = ws_launch_features(h->P, lab_dev, h->ws.feat, h->ws.x0, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_ws_features");
  return GMMSP_OK;
}

int gmmsp_ws_forward(gmmsp_handle* h, const float* params_dev, int32_t b0, int32_t b1,
                     void* stream) {
  int rc = ws_check(h);
  if (rc) return rc;
  if (!params_dev) return fail(GMMSP_E_INVAL, "null pointer");
  int p0, p1;
  rc = ws_range(h, b0, b1, &p0, &p1);
  if (rc) return rc;
  hipError_t e = ws_forward_range(h, params_dev, p0, p1, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_ws_forward");
  return GMMSP_OK;
}

int gmmsp_ws_apply(gmmsp_handle* h, const float* lab_dev, uint32_t output_mask, void* stream) {
  int rc = ws_check(h);
  if (rc) return rc;
  if (!lab_dev) return fail(GMMSP_E_INVAL, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  // theta^0 rows are staged in the partials area, which the next pass overwrites
  double* rows = h->P.part;
  hipError_t e = ws_launch_apply(h->P, lab_dev, h->ws.out, output_mask, rows, s);
  if (e == hipSuccess) e = launch_reset_state(h->P, s);
  if (e == hipSuccess) h->t_bound = 0;
  if (e == hipSuccess) e = launch_set_params(h->P, rows, s);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_ws_apply");
  h->initialised = true;
  return GMMSP_OK;
}

int gmmsp_ws_apply_guarded(gmmsp_handle* h, const float* lab_dev, uint32_t output_mask,
                           int32_t* fallback_host, void* stream) {
  int rc = ws_check(h);
  if (rc) return rc;
  if (!lab_dev) return fail(GMMSP_E_INVAL, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  double* rows = h->P.part;  // staging, as in gmmsp_ws_apply
  // L(theta^0) of the grid seeds, then of the network's theta^0 (one E-step
  // each); images whose network start is worse, or not finite, are re-seeded
  hipError_t e = launch_init_seeds(h->P, lab_dev, s);
  if (e == hipSuccess) e = launch_ll_eval(h->P, lab_dev, 1, s);
  if (e == hipSuccess) e = ws_launch_apply(h->P, lab_dev, h->ws.out, output_mask, rows, s);
  if (e == hipSuccess) e = launch_set_params(h->P, rows, s);
  if (e == hipSuccess) e = launch_ll_eval(h->P, lab_dev, 0, s);
  if (e == hipSuccess) e = launch_seed_fallback(h->P, lab_dev, s);
  if (e == hipSuccess) e = launch_reset_state(h->P, s);
  if (e == hipSuccess) h->t_bound = 0;
  if (e != hipSuccess) return hip_fail(e, "gmmsp_ws_apply_guarded");
  h->initialised = true;
  if (fallback_host) {
    std::vector<ImgState> st(h->n_img);
    e = hipMemcpyAsync(st.data(), h->P.state, sizeof(ImgState) * h->n_img, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "gmmsp_ws_apply_guarded");
    for (int32_t b = 0; b < h->n_img; ++b) fallback_host[b] = st[b].fallback;
  }
  return GMMSP_OK;
}

int gmmsp_ws_targets(gmmsp_handle* h, const float* lab_dev, void* stream) {
  int rc = ws_check(h);
  if (rc) return rc;
  if (!lab_dev) return fail(GMMSP_E_INVAL, "null pointer");
  hipError_t e = ws_launch_targets(h->P, lab_dev, h->ws.tgt, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_ws_targets");
  return GMMSP_OK;
}

int gmmsp_ws_train_step(gmmsp_handle* h, float* params_dev, float* m_dev, float* v_dev,
                        int32_t step, float lr, int32_t b0, int32_t b1, double* loss_host,
                        void* stream) {
  int rc = ws_check(h);
  if (rc) return rc;
  if (!params_dev || !m_dev || !v_dev) return fail(GMMSP_E_INVAL, "null pointer");
  if (step < 1 || !(lr > 0)) return fail(GMMSP_E_INVAL, "step must be >= 1 and lr > 0");
  int p0, p1;
  rc = ws_range(h, b0, b1, &p0, &p1);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  WsState& W = h->ws;
  const float scale = 1.0f / (float)(p1 - p0);
  const int nchunks = (p1 - p0 + 31) / 32;
  const int splits = nchunks < 4 * kWsMaxSplits ? (nchunks + 3) / 4 : kWsMaxSplits;
  const int cps = (nchunks + splits - 1) / splits;
  hipError_t e = ws_forward_range(h, params_dev, p0, p1, s);
  if (e == hipSuccess) e = ws_launch_loss(W.out, W.tgt, W.g4, p0, p1, W.loss_part, W.loss_sum, s);
  // layer inputs and output gradients, from the last layer down
  const uint16_t* xin[4] = {W.x0, W.y[0], W.y[1], W.y[2]};
  uint16_t* gout[4] = {W.g[0], W.g[1], W.g[2], W.g4};
  const int gc[4] = {32, 32, 32, 16};
  for (int l = 3; l >= 0 && e == hipSuccess; --l) {
    const WsLayer& L = kWs[l];
    e = ws_launch_dw(l + 1, W.nbr, gout[l], xin[l], W.part, splits, cps, p0, p1, s);
    if (e == hipSuccess)
      e = ws_launch_reduce_dw(W.part, splits, gc[l], L.cout, 9 * L.cin, scale, W.grad + L.w_off, s);
    if (e == hipSuccess) e = ws_launch_db(gout[l], gc[l], L.cout, p0, p1, scale, W.grad + L.b_off, s);
    if (e == hipSuccess && l > 0)
      e = ws_launch_conv(l + 1, 2, W.nbr, gout[l], W.wt[l], nullptr, L.cin, xin[l], gout[l - 1],
                         nullptr, p0, p1, s);
  }
  const float b1c = 1.0f - powf(0.9f, (float)step), b2c = 1.0f - powf(0.999f, (float)step);
  if (e == hipSuccess)
    e = ws_launch_adam(params_dev, m_dev, v_dev, W.grad, kWsParams, lr, 0.9f, 0.999f, 1e-8f, b1c,
                       b2c, s);
  if (e == hipSuccess && loss_host) {
    double ls = 0.0;
    e = hipMemcpyAsync(&ls, W.loss_sum, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    *loss_host = ls / ((double)(p1 - p0) * 10.0);
  }
  if (e != hipSuccess) return hip_fail(e, "gmmsp_ws_train_step");
  return GMMSP_OK;
}

int gmmsp_ws_read(gmmsp_handle* h, int32_t which, void* host, size_t bytes, void* stream) {
  int rc = ws_check(h);
  if (rc) return rc;
  if (!host || which < 0 || which >= 12) return fail(GMMSP_E_INVAL, "bad buffer or pointer");
  if (bytes > h->ws.sizes[which]) return fail(GMMSP_E_SIZE, "read past the buffer");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(host, h->ws.ptrs[which], bytes, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_ws_read");
  return GMMSP_OK;
}

int gmmsp_ws_write(gmmsp_handle* h, int32_t which, const void* host, size_t bytes, void* stream) {
  int rc = ws_check(h);
  if (rc) return rc;
  if (!host || which < 0 || which >= 12) return fail(GMMSP_E_INVAL, "bad buffer or pointer");
  if (bytes > h->ws.sizes[which]) return fail(GMMSP_E_SIZE, "write past the buffer");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(h->ws.ptrs[which], host, bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_ws_write");
  return GMMSP_OK;
}

// ---------------------------------------------------------------------------
// Connectivity post-processing
// ---------------------------------------------------------------------------

namespace {

struct ConnSizes {
  size_t pix, bsum, counts, seg, colsum, side, total;
  int max_pix, max_tiles, max_w, max_h;
};

static ConnSizes conn_sizes(const gmmsp_handle* h) {
  ConnSizes z;
  z.max_pix = z.max_tiles = z.max_w = z.max_h = 0;
  for (const ImgDesc& I : h->img) {
    // (clamped: the connectivity step itself rejects batches of 2^31 - 1 pixels or more)
    z.max_pix = (int)std::max<int64_t>(z.max_pix, std::min<int64_t>((int64_t)I.W * I.H, INT32_MAX));
    z.max_w = std::max(z.max_w, I.W);
    z.max_h = std::max(z.max_h, I.H);
    z.max_tiles = std::max(z.max_tiles, (int)gmmsp::conn_tiles(I.W, I.H));
  }
  const size_t n = (size_t)h->n_pix;
  z.pix = align256(sizeof(int) * n);
  z.bsum = align256(sizeof(int) * (gmmsp::conn_scan_blocks((int64_t)n) + 1));
  z.counts = align256(sizeof(int) * (4 * (size_t)h->n_img + 2));
  z.seg = z.pix;  // at most one segment per pixel
  z.colsum = align256(sizeof(unsigned long long) * 3 * n);
  z.side = align256(sizeof(int) * gmmsp::conn_side_ints(h->n_img, z.max_tiles));
  z.total = 3 * z.pix + z.bsum + z.counts + 13 * z.seg + z.colsum + z.side;
  return z;
}

}  // namespace

int gmmsp_conn_workspace_bytes(const gmmsp_handle* h, size_t* bytes) {
  if (!h || !bytes) return fail(GMMSP_E_INVAL, "null pointer");
  *bytes = conn_sizes(h).total;
  return GMMSP_OK;
}

namespace {

// The connectivity step on a given workspace; allocates nothing.
static int connectivity_run(gmmsp_handle* h, const float* lab_dev, const int32_t* labels_dev,
                     int32_t* out_dev, void* ws_dev, size_t ws_bytes, int32_t compact,
                     int32_t* counts_host, hipStream_t s) {
  if (h->n_pix >= ((int64_t)1 << 31) - 1)
    return fail(GMMSP_E_SIZE, "connectivity needs fewer than 2^31 - 1 pixels per batch");
  const ConnSizes z = conn_sizes(h);
  if (ws_bytes < z.total) return fail(GMMSP_E_SIZE, "connectivity workspace %zu < %zu bytes", ws_bytes, z.total);
  char* b = (char*)ws_dev;
  size_t t = 0;
  auto take = [&](size_t n) { void* p = b + t; t += n; return p; };
  ConnPtrs C;
  C.n_pix = h->n_pix;
  C.par = (int*)take(z.pix);
  C.segid = (int*)take(z.pix);
  C.scan = (int*)take(z.pix);
  C.bsum = (int*)take(z.bsum);
  C.counts = (int*)take(z.counts);
  C.total = C.counts + 4 * h->n_img;
  C.n_big = C.total + 1;
  int** seg[13] = {&C.seg_root, &C.seg_img, &C.size0, &C.size, &C.ccnt, &C.coff, &C.cursor,
                   &C.list, &C.poff, &C.cpar, &C.mpar, &C.next, &C.tail};
  for (int i = 0; i < 13; ++i) *seg[i] = (int*)take(z.seg);
  C.colsum = (unsigned long long*)take(z.colsum);
  C.side = (int*)take(z.side);
  const int max_pix = z.max_pix, max_tiles = z.max_tiles;
  hipError_t e = conn_launch_components(C, h->P.img, h->n_img, max_pix, max_tiles, labels_dev, s);
  int n_seg = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&n_seg, C.total, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_connectivity (components)");
  if (n_seg < 1 || n_seg > h->n_pix) return fail(GMMSP_E_STATE, "segment count %d out of range", n_seg);
  e = conn_launch_merge(C, h->P.img, h->n_img, max_pix, z.max_w, z.max_h, n_seg, lab_dev,
                        compact ? 1 : 0, out_dev, s);
  if (e == hipSuccess && counts_host) {
    // segments, small, merged per image straight into the caller's array; the
    // fourth entry (final segments) is formed here
    e = hipMemcpyAsync(counts_host, C.counts, sizeof(int) * 4 * (size_t)h->n_img,
                       hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess)
      for (int32_t i = 0; i < h->n_img; ++i)
        counts_host[4 * i + 3] = counts_host[4 * i + 0] - counts_host[4 * i + 2];
  }
  if (e != hipSuccess) return hip_fail(e, "gmmsp_connectivity");
  return GMMSP_OK;
}

// Scratch memory of gmmsp_connectivity_static: the address of this GPU's copy
// of `scratch`, found once per device (host code never passes the array's
// name itself, which is only a host-side stand-in).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

}  // namespace

int gmmsp_connectivity(gmmsp_handle* h, const float* lab_dev, const int32_t* labels_dev,
                       int32_t* out_dev, void* ws_dev, size_t ws_bytes, int32_t compact,
                       int32_t* counts_host, void* stream) {
  if (!h || !lab_dev || !labels_dev || !out_dev || !ws_dev) return fail(GMMSP_E_INVAL, "null pointer");
  if (((uintptr_t)ws_dev) & 255) return fail(GMMSP_E_INVAL, "workspace not 256-byte aligned");
  return connectivity_run(h, lab_dev, labels_dev, out_dev, ws_dev, ws_bytes, compact, counts_host,
                          (hipStream_t)stream);
}

int gmmsp_connectivity_static(gmmsp_handle* h, const float* lab_dev, const int32_t* labels_dev,
                              int32_t* out_dev, int32_t compact, int32_t* counts_host,
                              void* stream) {
  if (!h || !lab_dev || !labels_dev || !out_dev) return fail(GMMSP_E_INVAL, "null pointer");
  const size_t need = conn_sizes(h).total;
  if (need > (size_t)GMMSP_CONN_STATIC_BYTES)
    return fail(GMMSP_E_SIZE, "connectivity needs %zu bytes of scratch, more than the %zu of the "
                "allocation-free entry point", need, (size_t)GMMSP_CONN_STATIC_BYTES);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_connectivity_static: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(GMMSP_E_INVAL, "device %d out of range", dev);
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
      // once per device, with that device current: this GPU's copy of the array
      e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess) return hip_fail(e, "gmmsp_connectivity_static: hipGetSymbolAddress");
      if (!ptr) return fail(GMMSP_E_HIP, "gmmsp_connectivity_static: no scratch address");
      g_scratch_dev[dev] = ptr;
    }
    ptr = g_scratch_dev[dev];
  }
  return connectivity_run(h, lab_dev, labels_dev, out_dev, ptr, GMMSP_CONN_STATIC_BYTES, compact,
                          counts_host, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Accuracy measures
// ---------------------------------------------------------------------------

namespace {

struct MetricSizes {
  size_t nlab, ngt, roff, toff, tab, brp, rows, sums, total;
  int64_t tab_n, n_rows;
  int max_blocks;
  std::vector<int32_t> lab;       // label count per image
  std::vector<int64_t> row_off;   // n_img + 1
  std::vector<int64_t> tab_off;
};

static int metric_sizes(const gmmsp_handle* h, const int32_t* n_sp, const int32_t* n_gt, MetricSizes* z) {
  z->tab_n = 0;
  z->n_rows = 0;
  int max_w = 0, max_h = 0;
  z->lab.assign(h->n_img, 0);
  z->row_off.assign(h->n_img + 1, 0);
  z->tab_off.assign(h->n_img, 0);
  for (int32_t b = 0; b < h->n_img; ++b) {
    const int64_t k = n_sp ? (int64_t)n_sp[b] : (int64_t)h->img[b].nx * h->img[b].ny;
    if (k < 1) return fail(GMMSP_E_INVAL, "image %d: the label count must be >= 1", b);
    if (n_gt[b] < 1) return fail(GMMSP_E_INVAL, "image %d: n_gt must be >= 1", b);
    if (k * n_gt[b] >= ((int64_t)1 << 31)) return fail(GMMSP_E_SIZE, "image %d: labels x n_gt too large", b);
    z->lab[b] = (int32_t)k;
    z->tab_off[b] = z->tab_n;
    z->tab_n += k * n_gt[b];
    z->row_off[b + 1] = z->row_off[b] + k;
    max_w = std::max(max_w, h->img[b].W);
    max_h = std::max(max_h, h->img[b].H);
  }
  z->n_rows = z->row_off[h->n_img];
  z->max_blocks = metrics_max_blocks(max_w, max_h);
  const size_t n_img = (size_t)h->n_img;
  z->nlab = align256(sizeof(int32_t) * n_img);
  z->ngt = align256(sizeof(int32_t) * n_img);
  z->roff = align256(sizeof(int64_t) * (n_img + 1));
  z->toff = align256(sizeof(int64_t) * n_img);
  z->tab = align256(sizeof(int) * (size_t)z->tab_n);
  z->brp = align256(sizeof(int) * 2 * n_img * (size_t)z->max_blocks);
  z->rows = align256(sizeof(int64_t) * (size_t)z->n_rows);
  z->sums = align256(sizeof(int64_t) * 4 * n_img + sizeof(int));
  z->total = z->nlab + z->ngt + z->roff + z->toff + z->tab + z->brp + 2 * z->rows + z->sums;
  return GMMSP_OK;
}

}  // namespace

int gmmsp_metrics_workspace_bytes(const gmmsp_handle* h, const int32_t* n_sp_host,
                                  const int32_t* n_gt_host, size_t* bytes) {
  if (!h || !n_gt_host || !bytes) return fail(GMMSP_E_INVAL, "null pointer");
  MetricSizes z;
  const int rc = metric_sizes(h, n_sp_host, n_gt_host, &z);
  if (rc) return rc;
  *bytes = z.total;
  return GMMSP_OK;
}

int gmmsp_metrics(gmmsp_handle* h, const int32_t* labels_dev, const int32_t* gt_dev,
                  const int32_t* n_sp_host, const int32_t* n_gt_host, void* ws_dev,
                  size_t ws_bytes, double* out_host, int64_t* sums_host, void* stream) {
  if (!h || !labels_dev || !gt_dev || !n_gt_host || !ws_dev || !out_host)
    return fail(GMMSP_E_INVAL, "null pointer");
  if (((uintptr_t)ws_dev) & 255) return fail(GMMSP_E_INVAL, "workspace not 256-byte aligned");
  MetricSizes z;
  int rc = metric_sizes(h, n_sp_host, n_gt_host, &z);
  if (rc) return rc;
  if (ws_bytes < z.total) return fail(GMMSP_E_SIZE, "metrics workspace %zu < %zu bytes", ws_bytes, z.total);
  char* base = (char*)ws_dev;
  size_t t = 0;
  auto take = [&](size_t n) { void* p = base + t; t += n; return p; };
  int32_t* d_nlab = (int32_t*)take(z.nlab);
  int32_t* d_ngt = (int32_t*)take(z.ngt);
  int64_t* d_roff = (int64_t*)take(z.roff);
  int64_t* d_toff = (int64_t*)take(z.toff);
  int* d_tab = (int*)take(z.tab);
  int* d_brp = (int*)take(z.brp);
  int64_t* d_rue = (int64_t*)take(z.rows);
  int64_t* d_rasa = (int64_t*)take(z.rows);
  int64_t* d_sums = (int64_t*)take(z.sums);
  int* d_err = (int*)(d_sums + 4 * h->n_img);
  hipStream_t s = (hipStream_t)stream;
  const size_t ni = (size_t)h->n_img;
  hipError_t e = hipMemcpyAsync(d_nlab, z.lab.data(), sizeof(int32_t) * ni, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_ngt, n_gt_host, sizeof(int32_t) * ni, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_roff, z.row_off.data(), sizeof(int64_t) * (ni + 1), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_toff, z.tab_off.data(), sizeof(int64_t) * ni, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = metrics_launch(h->P, z.max_blocks, labels_dev, gt_dev, d_nlab, d_ngt, d_roff, z.n_rows,
                       d_toff, z.tab_n, d_tab, d_brp, d_rue, d_rasa, d_sums, d_err, s);
  std::vector<int64_t> sums(4 * ni);
  int err = 0;
  if (e == hipSuccess)
    e = hipMemcpyAsync(sums.data(), d_sums, sizeof(int64_t) * sums.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&err, d_err, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_metrics");
  if (err) return fail(GMMSP_E_INVAL, "a label or region id is outside [0, n_sp) or [0, n_gt)");
  for (int32_t b = 0; b < h->n_img; ++b) {
    const int64_t* q = sums.data() + 4 * b;
    const double n = (double)h->img[b].W * (double)h->img[b].H;
    out_host[3 * b + 0] = q[1] ? (double)q[0] / (double)q[1] : 1.0;
    out_host[3 * b + 1] = (double)q[2] / n - 1.0;
    out_host[3 * b + 2] = (double)q[3] / n;
    if (sums_host)
      for (int c = 0; c < 4; ++c) sums_host[4 * b + c] = q[c];
  }
  return GMMSP_OK;
}

// ---------------------------------------------------------------------------
// Colour front end
// ---------------------------------------------------------------------------

int gmmsp_srgb8_to_lab(const uint8_t* rgb_dev, int64_t n_pixels, float* lab_dev, void* stream) {
  if (!rgb_dev || !lab_dev) return fail(GMMSP_E_INVAL, "null pointer");
  if (n_pixels < 0) return fail(GMMSP_E_INVAL, "n_pixels < 0");
  if (((uintptr_t)rgb_dev) & 3) return fail(GMMSP_E_INVAL, "rgb_dev must be 4-byte aligned");
  if (((uintptr_t)lab_dev) & 15) return fail(GMMSP_E_INVAL, "lab_dev must be 16-byte aligned");
  if (n_pixels == 0) return GMMSP_OK;
  hipError_t e = launch_srgb8_to_lab(rgb_dev, n_pixels, lab_dev, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "gmmsp_srgb8_to_lab");
  return GMMSP_OK;
}

}  // extern "C"
