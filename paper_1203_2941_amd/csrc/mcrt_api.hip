// mcrt_api.hip - host side of the C ABI declared in include/mcrt.h.
//
// Owns device memory per context, validates inputs, builds the packed
// per-model tables (frequency quadrature, mixture opacities, Planck
// constants, source spectra, ln Phi(ln T) tables for Eq. 4) and sequences
// the kernels: epochs of the Bjorkman & Wood mode, passes of the iterative
// scheme, the PAH second stage, the ray-tracer and its adjoint, and the
// batched launch captured in a HIP graph.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>
#include <mutex>

#include "../../include/mcrt.h"
#include "mcrt_rtargs.h"

namespace mcrt {
size_t transport_lds_bytes(int nl, int ns, int nsrc, int nrows, int ntheta, bool fp64);
hipError_t launch_epoch_snapshot(const ModelDev *d, hipStream_t st);
hipError_t launch_finalize_T(const ModelDev *d, bool fp64, double *T, double *E, hipStream_t st);
hipError_t launch_init_T(const ModelDev *d, bool fp64, double *T, hipStream_t st);
hipError_t launch_build_S(const ModelDev *d, bool fp64, bool lit, bool sh, void *S,
                          hipStream_t st);
hipError_t launch_brick(bool fp64, const void *rho, void *rb, int nx, int ny, int nz, int nbx,
                        int nby, hipStream_t st);
hipError_t launch_wf_round(const ModelDev *d_models, int nmodels, bool fp64, bool rec, int fcur,
                           int grid_full, int grid_walk, size_t lds_full, size_t lds_walk,
                           bool idx32, bool per_cell, bool refined, int fast,
                           const hipEvent_t *ev, hipStream_t st);
hipError_t launch_mrw_cand(const ModelDev *d_models, int nmodels, int ncu, hipStream_t st);
size_t walk_lds_bytes(int nl, int ns, int nsrc, int nrows, int ntheta, int occ_words, bool fp64);
hipError_t launch_occ(bool fp64, const void *rb, uint32_t *occ, uint64_t ncell_b, int osh,
                      hipStream_t st);
hipError_t launch_wf_finish(const ModelDev *d_models, int nmodels, bool fp64, bool rec, int fcur,
                            int grid, size_t lds, bool idx32, bool per_cell, bool refined,
                            hipStream_t st);
hipError_t launch_wf_busy(const ModelDev *d_models, int nmodels, int fcur, uint32_t *busy,
                          uint32_t *left,
                          hipStream_t st);
hipError_t launch_sample_reem(const ModelDev *d, bool fp64, int s, double T, uint64_t n,
                              uint64_t seed, unsigned long long *counts, size_t lds,
                              hipStream_t st);
hipError_t launch_vox_torus(bool fp64, int nx, int ny, int nz, const double o[3], double dc,
                            int ncl, const double *dC, double r_clump, double rho_cl,
                            double rho_int, double r_in, double r_out, double s1, void *rho,
                            hipStream_t st);
hipError_t launch_vox_shell(bool fp64, int nx, int ny, int nz, const double o[3], double dc,
                            double rho0, double r_in, double r_out, double power, int ng,
                            const double *dgx, const double *dgw, void *rho, hipStream_t st);
hipError_t launch_rt_fwd(const RtArgs *dA, const RtArgs &hA, bool fp64, void *img, double *sed,
                         hipEvent_t ev_main, hipStream_t st);
hipError_t launch_rt_adj(const RtArgs *dA, const RtArgs &hA, bool fp64, const void *w_img,
                         const double *w_sed, void *drho, hipEvent_t ev_main, hipStream_t st);
}  // namespace mcrt

using namespace mcrt;

struct mcrt_ctx {
  int device = 0;
  bool fp64 = true;
  std::string err;
  // grid
  bool has_grid = false;
  int nx = 0, ny = 0, nz = 0;
  double origin[3] = {0, 0, 0}, dcell = 0;
  uint64_t ncell = 0;          // leaf cells: cubes plus sub-cubes (every per-cell array)
  uint64_t ncube = 0;          // cubes of the grid
  uint64_t nsub = 0;           // sub-cubes of the divided cubes (one refinement level)
  uint8_t *d_ref = nullptr;    // [ncube] sub-cubes per edge (0/1: whole)
  uint64_t *d_suboff = nullptr;  // [ncube] exclusive prefix sum of r^3 over divided cubes
  int max_r = 1;
  void *d_rho = nullptr;       // [ncell]: cube densities, then sub-cube densities
  void *d_rho_b = nullptr;  // density in 4x4x4 bricks for the walk
  int nbx = 0, nby = 0, nbz = 0;
  uint32_t *d_occ = nullptr;  // brick-run occupancy bits for the walk
  int osh = 0, ow = 0;
  // dust
  bool has_dust = false;
  int nl = 0, ns = 0, pah = -1, nrows = 0;
  std::vector<double> lam, frac, kabs, ksca, g, pah_emis, pah_edges;
  // sources
  bool has_src = false;
  int nsrc = 0;
  std::vector<double> src_pos, src_lum, src_lnu;  // lnu [nsrc][nl] erg/s/Hz
  // views
  int nview = 0, nimg = 0;
  std::vector<double> views;
  std::vector<int32_t> img_idx;
  double distance = 1.0;
  // tables
  std::vector<double> h_tab;
  double kext_max = 0.0, ltot = 0.0;
  double kr_gmax = 0.0, phi_tmin = 0.0;  // MRW pre-test bounds (see build_tables)
  double herm_pmin[MAX_NS] = {0.0, 0.0, 0.0, 0.0};  // lower ends of the Hermite tables
  double *d_tab = nullptr;
  void *d_rtab = nullptr;
  int32_t *d_imgmap = nullptr;
  double *d_herm = nullptr;
  double *d_mrw_ub = nullptr;  // MRW pre-test bound per herm node interval (FP32 walk)
  uint32_t *d_mrw_flags = nullptr;  // candidate and current diffusion bits, [2][words]
  size_t mrw_flags_cap = 0;         // words per half
  float *d_rej_pe = nullptr;   // FP32 re-emission proposal tables (alias prob, envelope)
  uint8_t *d_rej_al = nullptr;
  size_t tab_cap = 0, rtab_cap = 0;
  bool tables_ok = false;
  // state
  uint64_t state_cells = 0;
  int state_ns = 0;
  uint64_t *d_k = nullptr;
  double *d_epath = nullptr, *d_T = nullptr, *d_esnap = nullptr, *d_tt = nullptr, *d_tmp = nullptr;
  uint8_t *d_dirty = nullptr;
  uint32_t *d_kpah = nullptr;
  uint64_t *d_prefix = nullptr;
  uint64_t *d_sed = nullptr;
  int sed_cap = 0, ntheta = 10;
  void *d_ssca = nullptr;
  size_t ssca_cap = 0;
  void *d_rec = nullptr;
  uint64_t rec_cap = 0, rec_n = 0;
  WfCtl *d_ctl = nullptr;   // wavefront queue counters (ctl->emitted is the packet counter)
  // events bracketing the emission, walk and interaction kernels of every
  // round since the last phase_reset (4 per round), and the phase totals
  std::vector<hipEvent_t> pev;
  size_t pev_used = 0;
  double t_phase[3] = {0, 0, 0};
  uint64_t n_rounds = 0;
  WfCtl *h_ctl = nullptr;   // pinned copy read between rounds
  void *d_q = nullptr;      // the two packet queues
  uint32_t qcap = 0;
  QBuf q[2] = {};
  unsigned long long *d_stats = nullptr;
  ModelDev *d_model = nullptr;
  ModelDev h_model;
  double xi = 0.0;
  uint64_t n_total = 0;
  double ssca_unit = 1.0;  // erg/s/sr per stored unit of the scattering sums
  // scattering law (Henyey-Greenstein or the g-factor approximation)
  int scat_law = MCRT_SCAT_HG;
  // scattering moments [cell][img][order^2] (context precision, units of
  // ssca_unit), kept for the imaged wavelengths sh_img
  void *d_sh = nullptr;
  size_t sh_cap = 0;
  int sh_have = 0;            // order of the moments in d_sh (0: none)
  std::vector<int32_t> sh_img;
  int ssca_src = MCRT_SSCA_PEELOFF;
  // ray-tracer
  int rt_mode = MCRT_RT_EXT;
  void *d_S = nullptr;
  size_t S_cap = 0;
  bool S_ok = false;
  // tallies changed by a run outside B&W epochs, which keeps no dirty flags:
  // the next epoch snapshot must then cover every cell
  bool snap_stale = false;
  RtArgs *d_rt = nullptr;
  void *d_img_tmp = nullptr;
  size_t img_cap = 0;
  double *d_sed_tmp = nullptr;
  // staging (pinned) for small structures
  void *h_stage = nullptr;
  hipEvent_t ev_stage = nullptr, ev0 = nullptr, ev1 = nullptr;
  hipEvent_t evf0 = nullptr, evf1 = nullptr, eva0 = nullptr, eva1 = nullptr;
  hipEvent_t evs0 = nullptr, evs1 = nullptr;  // around the last source-function build
  bool have_s = false;
  hipStream_t cap_stream = nullptr;  // graph capture (the caller's stream may be the legacy one)
  bool have_f = false, have_a = false;
  double t_transport = 0.0;
  size_t sed_tmp_cap = 0;
  size_t lds_max = 65536;
  int num_cu = 256;
  // batch
  ModelDev *d_batch = nullptr;
  int batch_cap = 0;
  void *d_temp = nullptr;
  size_t temp_cap = 0;
};

static thread_local std::string g_create_err;

static mcrt_status fail(mcrt_ctx *c, mcrt_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf; else g_create_err = buf;
  return s;
}

#define HIPCHK(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(ctx, e_ == hipErrorOutOfMemory ? MCRT_ENOMEM : MCRT_EDEVICE, "%s: %s", \
                  #call, hipGetErrorString(e_));                                      \
  } while (0)

static hipError_t dev_alloc(void **p, size_t bytes) {
  if (*p) {
    (void)hipFree(*p);
    *p = nullptr;
  }
  if (bytes == 0) return hipSuccess;
  hipError_t e = hipMalloc(p, bytes);
  // a failed allocation must not linger as the runtime's last error (a
  // later hipGetLastError check would report it against another call)
  if (e != hipSuccess) (void)hipGetLastError();
  return e;
}

template <typename T>
static hipError_t fill(T *p, T v, uint64_t n, hipStream_t st) {
  if (!p || n == 0) return hipSuccess;
  unsigned g = (unsigned)((n + 255) / 256);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_fill<T>, dim3(g), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

// Small structures go through one pinned buffer; the event guards reuse.
static hipError_t stage_copy(mcrt_ctx *ctx, void *dst, const void *src, size_t bytes,
                             hipStream_t st) {
  hipError_t e = hipEventSynchronize(ctx->ev_stage);
  if (e != hipSuccess) return e;
  memcpy(ctx->h_stage, src, bytes);
  e = hipMemcpyAsync(dst, ctx->h_stage, bytes, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  return hipEventRecord(ctx->ev_stage, st);
}

static const size_t STAGE_BYTES = 1 << 20;
static hipError_t scratch_init(int device);

extern "C" mcrt_status mcrt_create(mcrt_ctx **out, int device, int precision) {
  mcrt_ctx *ctx = nullptr;
  if (!out) return fail(nullptr, MCRT_EINVAL, "out is NULL");
  *out = nullptr;
  if (precision != MCRT_FP64 && precision != MCRT_FP32)
    return fail(nullptr, MCRT_EINVAL, "precision must be MCRT_FP64 or MCRT_FP32");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(nullptr, MCRT_EDEVICE, "no HIP device available");
  if (device < 0 || device >= ndev) return fail(nullptr, MCRT_EINVAL, "device %d out of range", device);
  if (hipSetDevice(device) != hipSuccess) return fail(nullptr, MCRT_EDEVICE, "hipSetDevice failed");
  ctx = new mcrt_ctx();
  ctx->device = device;
  ctx->fp64 = (precision == MCRT_FP64);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    ctx->num_cu = prop.multiProcessorCount;
    ctx->lds_max = prop.sharedMemPerBlock;
  }
  if (hipHostMalloc(&ctx->h_stage, STAGE_BYTES, hipHostMallocDefault) != hipSuccess ||
      hipEventCreate(&ctx->ev_stage) != hipSuccess || hipEventCreate(&ctx->ev0) != hipSuccess ||
      hipEventCreate(&ctx->ev1) != hipSuccess || hipEventCreate(&ctx->evf0) != hipSuccess ||
      hipEventCreate(&ctx->evf1) != hipSuccess || hipEventCreate(&ctx->eva0) != hipSuccess ||
      hipEventCreate(&ctx->eva1) != hipSuccess || hipEventCreate(&ctx->evs0) != hipSuccess ||
      hipEventCreate(&ctx->evs1) != hipSuccess ||
      hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess ||
      hipMalloc((void **)&ctx->d_ctl, sizeof(WfCtl)) != hipSuccess ||
      hipHostMalloc((void **)&ctx->h_ctl, sizeof(WfCtl), hipHostMallocDefault) != hipSuccess ||
      hipMalloc((void **)&ctx->d_stats, sizeof(unsigned long long) * NSTAT) != hipSuccess ||
      hipMalloc((void **)&ctx->d_model, sizeof(ModelDev)) != hipSuccess ||
      hipMalloc((void **)&ctx->d_rt, sizeof(RtArgs)) != hipSuccess) {
    mcrt_destroy(ctx);
    return fail(nullptr, MCRT_ENOMEM, "context allocation failed");
  }
  (void)hipEventRecord(ctx->ev_stage, 0);
  if (scratch_init(device) != hipSuccess) {
    mcrt_destroy(ctx);
    return fail(nullptr, MCRT_EDEVICE, "hipGetSymbolAddress failed for the scratch array");
  }
  *out = ctx;
  return MCRT_OK;
}

extern "C" void mcrt_destroy(mcrt_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  void *ps[] = {ctx->d_rho, ctx->d_rho_b, ctx->d_occ, ctx->d_tab, ctx->d_rtab, ctx->d_imgmap, ctx->d_herm, ctx->d_mrw_ub, ctx->d_mrw_flags, ctx->d_rej_pe, ctx->d_rej_al, ctx->d_k, ctx->d_epath,
                ctx->d_T, ctx->d_esnap, ctx->d_tt, ctx->d_tmp, ctx->d_dirty, ctx->d_kpah,
                ctx->d_prefix, ctx->d_sed, ctx->d_ssca, ctx->d_rec, ctx->d_ctl, ctx->d_q, ctx->d_stats,
                ctx->d_model, ctx->d_S, ctx->d_rt, ctx->d_img_tmp, ctx->d_sed_tmp, ctx->d_batch,
                ctx->d_temp, ctx->d_sh, ctx->d_ref, ctx->d_suboff};
  for (void *p : ps)
    if (p) (void)hipFree(p);
  if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
  if (ctx->h_ctl) (void)hipHostFree(ctx->h_ctl);
  for (hipEvent_t e : ctx->pev) (void)hipEventDestroy(e);
  if (ctx->ev_stage) (void)hipEventDestroy(ctx->ev_stage);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  hipEvent_t evs[] = {ctx->evf0, ctx->evf1, ctx->eva0, ctx->eva1, ctx->evs0, ctx->evs1};
  for (hipEvent_t e : evs)
    if (e) (void)hipEventDestroy(e);
  delete ctx;
}

extern "C" const char *mcrt_last_error(const mcrt_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

static size_t rsize(const mcrt_ctx *c) { return c->fp64 ? 8 : 4; }

// ----------------------------------------------------------------- state

static mcrt_status ensure_state(mcrt_ctx *ctx, hipStream_t st) {
  if (ctx->state_cells == ctx->ncell && ctx->state_ns == ctx->ns && ctx->d_k) return MCRT_OK;
  uint64_t n = ctx->ncell * (uint64_t)ctx->ns;
  HIPCHK(dev_alloc((void **)&ctx->d_k, n * 8));
  HIPCHK(dev_alloc((void **)&ctx->d_epath, n * 8));
  HIPCHK(dev_alloc((void **)&ctx->d_T, n * 8));
  HIPCHK(dev_alloc((void **)&ctx->d_esnap, n * 8));
  HIPCHK(dev_alloc((void **)&ctx->d_tt, n * 8));
  HIPCHK(dev_alloc((void **)&ctx->d_tmp, n * 8));
  HIPCHK(dev_alloc((void **)&ctx->d_dirty, ctx->ncell));
  HIPCHK(dev_alloc((void **)&ctx->d_kpah, ctx->ncell * 4));
  HIPCHK(dev_alloc((void **)&ctx->d_prefix, ctx->ncell * 8));
  ctx->state_cells = ctx->ncell;
  ctx->state_ns = ctx->ns;
  HIPCHK(fill<double>(ctx->d_T, 0.0, n, st));
  HIPCHK(fill<uint64_t>(ctx->d_k, 0ull, n, st));
  HIPCHK(fill<double>(ctx->d_epath, 0.0, n, st));
  HIPCHK(fill<uint32_t>(ctx->d_kpah, 0u, ctx->ncell, st));
  HIPCHK(fill<double>(ctx->d_esnap, 0.0, n, st));
  HIPCHK(fill<double>(ctx->d_tt, -1.0, n, st));
  HIPCHK(fill<uint8_t>(ctx->d_dirty, (uint8_t)0, ctx->ncell, st));
  ctx->ssca_cap = 0;
  ctx->S_ok = false;
  return MCRT_OK;
}

static mcrt_status ensure_ssca(mcrt_ctx *ctx) {
  size_t need = (size_t)ctx->nview * ctx->nimg * ctx->ncell * rsize(ctx);
  if (need == 0) return MCRT_OK;
  if (ctx->ssca_cap == need && ctx->d_ssca) return MCRT_OK;
  ctx->ssca_cap = 0;
  HIPCHK(dev_alloc(&ctx->d_ssca, need));
  ctx->ssca_cap = need;
  HIPCHK(hipMemset(ctx->d_ssca, 0, need));
  HIPCHK(hipDeviceSynchronize());
  return MCRT_OK;
}

static mcrt_status ensure_sed(mcrt_ctx *ctx, int ntheta) {
  int need = ntheta * ctx->nl;
  if (ctx->sed_cap == need && ctx->d_sed) return MCRT_OK;
  ctx->sed_cap = 0;
  HIPCHK(dev_alloc((void **)&ctx->d_sed, (size_t)need * 8));
  ctx->sed_cap = need;
  HIPCHK(hipMemset(ctx->d_sed, 0, (size_t)need * 8));
  HIPCHK(hipDeviceSynchronize());
  return MCRT_OK;
}

static mcrt_status zero_tallies(mcrt_ctx *ctx, hipStream_t st) {
  uint64_t n = ctx->ncell * (uint64_t)ctx->ns;
  HIPCHK(fill<uint64_t>(ctx->d_k, 0ull, n, st));
  HIPCHK(fill<double>(ctx->d_epath, 0.0, n, st));
  HIPCHK(fill<uint32_t>(ctx->d_kpah, 0u, ctx->ncell, st));
  HIPCHK(fill<uint64_t>(ctx->d_sed, 0ull, (uint64_t)ctx->sed_cap, st));
  if (ctx->d_ssca) {
    uint64_t m = (uint64_t)ctx->nview * ctx->nimg * ctx->ncell;
    if (ctx->fp64) HIPCHK(fill<double>((double *)ctx->d_ssca, 0.0, m, st));
    else HIPCHK(fill<float>((float *)ctx->d_ssca, 0.0f, m, st));
  }
  if (ctx->d_sh && ctx->sh_have > 0) {
    uint64_t m = (uint64_t)ctx->ncell * ctx->nimg * (uint64_t)(ctx->sh_have * ctx->sh_have);
    if (ctx->fp64) HIPCHK(fill<double>((double *)ctx->d_sh, 0.0, m, st));
    else HIPCHK(fill<float>((float *)ctx->d_sh, 0.0f, m, st));
  }
  ctx->S_ok = false;
  return MCRT_OK;
}

// Moments of order `order` for the current imaged wavelengths, zeroed when
// the buffer is (re)made; kept across runs otherwise (runs add to them).
static mcrt_status ensure_sh(mcrt_ctx *ctx, int order, hipStream_t st) {
  if (order <= 0 || ctx->nimg == 0) return MCRT_OK;
  if (ctx->sh_have == order && ctx->d_sh && ctx->sh_img == ctx->img_idx) return MCRT_OK;
  uint64_t m = (uint64_t)ctx->ncell * ctx->nimg * (uint64_t)(order * order);
  size_t need = m * rsize(ctx);
  if (need > ctx->sh_cap || !ctx->d_sh) {
    ctx->sh_cap = 0;
    ctx->sh_have = 0;
    HIPCHK(dev_alloc(&ctx->d_sh, need));
    ctx->sh_cap = need;
  }
  if (ctx->fp64) HIPCHK(fill<double>((double *)ctx->d_sh, 0.0, m, st));
  else HIPCHK(fill<float>((float *)ctx->d_sh, 0.0f, m, st));
  ctx->sh_have = order;
  ctx->sh_img = ctx->img_idx;
  ctx->S_ok = false;
  return MCRT_OK;
}

static mcrt_status zero_epoch(mcrt_ctx *ctx, hipStream_t st) {
  uint64_t n = ctx->ncell * (uint64_t)ctx->ns;
  HIPCHK(fill<double>(ctx->d_esnap, 0.0, n, st));
  HIPCHK(fill<double>(ctx->d_tt, -1.0, n, st));
  HIPCHK(fill<uint8_t>(ctx->d_dirty, (uint8_t)0, ctx->ncell, st));
  ctx->snap_stale = false;
  return MCRT_OK;
}

// ---------------------------------------------------------------- tables

// Vose's alias table for weights v[0..n-1] (all >= 0): prob[j] in [0, 1] and
// alias[j] such that bin j0 drawn uniformly, kept when a second uniform is
// below prob[j0] and replaced by alias[j0] otherwise, has probability
// v_j / sum v. A zero sum gives a uniform table.
static void alias_table(const double *v, int n, float *prob, uint8_t *alias) {
  double sum = 0.0;
  for (int j = 0; j < n; ++j) sum += v[j];
  std::vector<double> q(n);
  std::vector<int> small, large;
  for (int j = 0; j < n; ++j) {
    q[j] = sum > 0.0 ? v[j] * n / sum : 1.0;
    (q[j] < 1.0 ? small : large).push_back(j);
  }
  while (!small.empty() && !large.empty()) {
    const int l = small.back(), g = large.back();
    small.pop_back();
    large.pop_back();
    prob[l] = (float)q[l];
    alias[l] = (uint8_t)g;
    q[g] = (q[g] + q[l]) - 1.0;
    (q[g] < 1.0 ? small : large).push_back(g);
  }
  for (int j : small) { prob[j] = 1.0f; alias[j] = (uint8_t)j; }
  for (int j : large) { prob[j] = 1.0f; alias[j] = (uint8_t)j; }
}

static double h_planck(double nu, double T) {
  if (!(T > 0.0)) return 0.0;
  double x = H_PL * nu / (K_BO * T);
  if (x > 700.0) return 0.0;
  return 2.0 * H_PL * nu * nu * nu / (C_LI * C_LI) / expm1(x);
}

static mcrt_status build_tables(mcrt_ctx *ctx) {
  if (!(ctx->has_dust && ctx->has_src)) return MCRT_OK;
  const int nl = ctx->nl, ns = ctx->ns;
  TabOff o = tab_offsets(nl, ns, ctx->nsrc, ctx->nrows);
  std::vector<double> t(o.dtotal, 0.0);
  std::vector<double> nu(nl), w(nl);
  for (int j = 0; j < nl; ++j) nu[j] = C_LI / (ctx->lam[j] * 1e-4);
  for (int j = 0; j < nl; ++j) {
    const double *L = ctx->lam.data();
    double lo = (j == 0) ? L[0] * std::sqrt(L[0] / L[1]) : std::sqrt(L[j - 1] * L[j]);
    double hi = (j == nl - 1) ? L[nl - 1] * std::sqrt(L[nl - 1] / L[nl - 2]) : std::sqrt(L[j] * L[j + 1]);
    w[j] = C_LI / (lo * 1e-4) - C_LI / (hi * 1e-4);
  }
  // scattering as transported: the model's, or under the g-factor
  // approximation isotropic with kappa_sca (1 - g)
  const bool gfac = ctx->scat_law == MCRT_SCAT_GFACTOR;
  auto ksca_eff = [&](int i) { return gfac ? (1.0 - ctx->g[i]) * ctx->ksca[i] : ctx->ksca[i]; };
  auto g_eff = [&](int i) { return gfac ? 0.0 : ctx->g[i]; };
  std::vector<double> kabsm(nl), kscam(nl), kext(nl);
  ctx->kext_max = 0.0;
  for (int j = 0; j < nl; ++j) {
    double a = 0.0, s = 0.0;
    for (int q = 0; q < ns; ++q) {
      a += ctx->frac[q] * ctx->kabs[q * nl + j];
      s += ctx->frac[q] * ksca_eff(q * nl + j);
    }
    kabsm[j] = a;
    kscam[j] = s;
    kext[j] = a + s;
    if (kext[j] > ctx->kext_max) ctx->kext_max = kext[j];
  }
  for (int j = 0; j < nl; ++j) {
    t[o.w + j] = w[j];
    t[o.hnu + j] = H_PL * nu[j];
    t[o.a + j] = 2.0 * H_PL * nu[j] * nu[j] * nu[j] / (C_LI * C_LI);
    t[o.kext + j] = kext[j];
    for (int s = 0; s < ns; ++s) {
      t[o.wk + s * nl + j] = w[j] * ctx->kabs[s * nl + j];
      t[o.wfk + s * nl + j] = w[j] * ctx->frac[s] * ctx->kabs[s * nl + j];
      t[o.kabs + s * nl + j] = ctx->kabs[s * nl + j];
    }
  }
  for (int s = 0; s < ns; ++s) t[o.frac + s] = ctx->frac[s];
  ctx->ltot = 0.0;
  // source and PAH emission spectra as running sums of w_j L_j taken from
  // the highest index down (the order of the inverse-CDF walk), so that a
  // binary search finds the same bin as the sequential walk
  for (int s = 0; s < ctx->nsrc; ++s) {
    double c = 0.0;
    for (int j = nl - 1; j >= 0; --j) {
      c += w[j] * ctx->src_lnu[s * nl + j];
      t[o.srccum + s * nl + j] = c;
    }
    for (int j = 0; j < nl; ++j) t[o.lnu + s * nl + j] = ctx->src_lnu[s * nl + j];
    t[o.lum + s] = ctx->src_lum[s];
    for (int k = 0; k < 3; ++k) t[o.srcpos + 3 * s + k] = ctx->src_pos[3 * s + k];
    ctx->ltot += ctx->src_lum[s];
  }
  for (int r = 0; r < ctx->nrows; ++r) {
    double c = 0.0;
    for (int j = nl - 1; j >= 0; --j) {
      c += w[j] * ctx->pah_emis[r * nl + j];
      t[o.pahcum + r * nl + j] = c;
    }
    if (r < ctx->nrows - 1) t[o.pahe + r] = ctx->pah_edges[r];
  }
  const double lt0 = std::log(T_TAB_MIN), dlt = (std::log(T_MAX) - lt0) / (NT_TAB - 1);
  for (int s = 0; s < ns; ++s)
    for (int k = 0; k < NT_TAB; ++k) {
      double T = std::exp(lt0 + k * dlt), ph = 0.0;
      for (int j = nl - 1; j >= 0; --j) ph += t[o.wk + s * nl + j] * h_planck(nu[j], T);
      t[o.logphi + s * NT_TAB + k] = std::log(ph);  // -inf where Phi underflows
    }
  // Upper bound of the mixture Rosseland mean on each interval [T_k, T_k+1]
  // of the ln T grid. kappa_R = num/den with num = sum_j w_j dB_j/dT and
  // den = sum_j w_j (dB_j/dT)/kext_j; at fixed nu, dB/dT grows with T
  // (x^2 e^x/(e^x - 1)^2 falls with x = h nu/kT), so on the interval
  // num(T) <= num(T_k+1) and den(T) >= den(T_k), hence
  // kappa_R(T) <= num(T_k+1)/den(T_k). The factor 1 + 1e-9 covers the
  // rounding of the sums here and in the device's exact mean.
  {
    auto sums = [&](double T, double &num, double &den) {
      num = den = 0.0;
      for (int j = nl - 1; j >= 0; --j) {
        double x = H_PL * nu[j] / (K_BO * T);
        if (x > 700.0) continue;
        double em = std::expm1(x);
        double B = t[o.a + j] / em;
        double db = w[j] * (B * (x / T) * (1.0 + 1.0 / em));
        num += db;
        den += db / kext[j];
      }
    };
    bool pos = true;
    for (int j = 0; j < nl; ++j) pos = pos && kext[j] > 0.0;
    double gmax = 0.0;
    for (int k = 0; k < NT_TAB - 1; ++k) {
      double nlo, dlo, nhi, dhi;
      sums(std::exp(lt0 + k * dlt), nlo, dlo);
      sums(std::exp(lt0 + (k + 1) * dlt), nhi, dhi);
      // a zero extinction anywhere makes the exact mean 0 (no diffusion);
      // an empty lower sum leaves only the hard bound kext_max
      double b = !pos ? 0.0 : (dlo > 0.0 ? (1.0 + 1e-9) * nhi / dlo : ctx->kext_max);
      if (b > ctx->kext_max) b = ctx->kext_max;
      t[o.krmax + k] = b;
      if (b > gmax) gmax = b;
    }
    t[o.krmax + NT_TAB - 1] = ctx->kext_max;  // outside the grid: the hard bound
    ctx->kr_gmax = gmax;
  }
  {
    int s0 = 0;
    while (s0 < ns && s0 == ctx->pah) ++s0;
    ctx->phi_tmin = s0 < ns ? std::exp(t[o.logphi + s0 * NT_TAB]) : 0.0;
  }
  // walk-precision table
  std::vector<double> r(o.r_total, 0.0);
  for (int j = 0; j < nl; ++j) {
    r[o.r_kext + j] = kext[j];
    r[o.r_kabsm + j] = kabsm[j];
    r[o.r_alb + j] = (kext[j] > 0.0) ? kscam[j] / kext[j] : 0.0;
    r[o.r_hnu + j] = t[o.hnu + j];
    r[o.r_a + j] = t[o.a + j];
    for (int s = 0; s < ns; ++s) {
      r[o.r_fsca + s * nl + j] = ctx->frac[s] * ksca_eff(s * nl + j);
      r[o.r_fabs + s * nl + j] = ctx->frac[s] * ctx->kabs[s * nl + j];
      r[o.r_g + s * nl + j] = g_eff(s * nl + j);
      r[o.r_lucy + s * nl + j] =
          (s != ctx->pah && kabsm[j] > 0.0) ? ctx->frac[s] * ctx->kabs[s * nl + j] / kabsm[j] : 0.0;
      r[o.r_wk + s * nl + j] = t[o.wk + s * nl + j];
    }
  }
  // Hermite table of ln T(ln Phi) per species (see invert_T_fast)
  const int HS = 3 + 2 * NH_TAB;
  std::vector<double> herm((size_t)ns * HS, 0.0);
  for (int s = 0; s < ns; ++s) {
    const double *wk = &t[o.wk + s * nl];
    auto phi = [&](double T, double *dphi) {
      double sum = 0.0, ds = 0.0;
      for (int j = nl - 1; j >= 0; --j) {
        double x = H_PL * nu[j] / (K_BO * T);
        if (x > 700.0) continue;
        double em = std::expm1(x);
        double B = t[o.a + j] / em;
        sum += wk[j] * B;
        ds += wk[j] * (B * (x / T) * (1.0 + 1.0 / em));
      }
      *dphi = ds;
      return sum;
    };
    double d0, d1;
    double p0 = phi(T_HERM_MIN, &d0), p1 = phi(T_MAX, &d1);
    double *hh = &herm[(size_t)s * HS];
    if (!(p0 > 0.0) || !(p1 > p0)) {
      hh[0] = 0.0; hh[1] = 1.0; hh[2] = 0.0;  // empty table: always the Newton path
      ctx->herm_pmin[s] = HUGE_VAL;
      continue;
    }
    double u0 = std::log(p0), u1 = std::log(p1), du = (u1 - u0) / (NH_TAB - 1);
    hh[0] = u0; hh[1] = du; hh[2] = NH_TAB;
    // a right-hand side at or above this inverts by the table alone: the
    // table index (ln rhs - u0)/du of any such value is at least 0
    ctx->herm_pmin[s] = std::exp(u0) * (1.0 + 1e-12);
    double T = T_HERM_MIN;
    for (int k = 0; k < NH_TAB; ++k) {
      double target = u0 + k * du;
      if (k == NH_TAB - 1) T = T_MAX;
      // Newton on ln Phi(ln T) from the previous node (monotone, smooth)
      for (int it = 0; it < 60 && k > 0 && k < NH_TAB - 1; ++it) {
        double dp, p = phi(T, &dp);
        double g = std::log(p) - target;
        double step = g / (T * dp / p);
        double Tn = T * std::exp(-step);
        if (!(Tn > 0.0)) break;
        T = Tn;
        if (std::fabs(step) < 1e-15) break;
      }
      double dp, p = phi(T, &dp);
      hh[3 + 2 * k] = std::log(T);
      hh[4 + 2 * k] = p / (T * dp);  // d ln T / d ln Phi
    }
  }
  // FP32 walk: re-emission proposals. For each mode (0: Eq. 5, weights
  // w kabs B; 1: Eq. 10, weights w kabs dB/dT), species and ln T bin, the
  // spectrum at the bin's upper temperature as an envelope (B and dB/dT grow
  // with T at fixed nu, so it bounds the spectrum anywhere in the bin; 2e-4
  // headroom covers FP32 evaluation on the GPU) and its alias table.
  std::vector<float> rej_pe;
  std::vector<uint8_t> rej_al;
  if (!ctx->fp64 && nl <= 256) {
    const size_t per = (size_t)NK_REJ * nl, tot = 2 * (size_t)ns * per;
    rej_pe.assign(2 * tot, 0.0f);
    rej_al.assign(tot, 0);
    const double lt0 = std::log(T_TAB_MIN), dlt = (std::log(T_MAX) - lt0) / NK_REJ;
    std::vector<double> env(nl);
    std::vector<float> prob(nl);
    std::vector<uint8_t> al(nl);
    for (int mode = 0; mode < 2; ++mode)
      for (int s = 0; s < ns; ++s)
        for (int k = 0; k < NK_REJ; ++k) {
          const double T = std::exp(lt0 + (k + 1) * dlt);
          for (int j = 0; j < nl; ++j) {
            const double x = H_PL * nu[j] / (K_BO * T);
            double d = 0.0;
            if (x <= 700.0) {
              const double em = std::expm1(x), B = t[o.a + j] / em;
              d = mode == 0 ? B : B * (x / T) * (1.0 + 1.0 / em);
            }
            env[j] = t[o.wk + s * nl + j] * d * (1.0 + 2e-4);
          }
          alias_table(env.data(), nl, prob.data(), al.data());
          const size_t base = ((size_t)mode * ns + s) * per + (size_t)k * nl;
          for (int j = 0; j < nl; ++j) {
            rej_pe[2 * (base + j)] = prob[j];
            rej_pe[2 * (base + j) + 1] = (float)env[j];
            rej_al[base + j] = al[j];
          }
        }
  }
  std::vector<int32_t> im(nl, -1);
  for (int q = 0; q < ctx->nimg; ++q) im[ctx->img_idx[q]] = q;
  mcrt_ctx *c = ctx;
  size_t tb = (size_t)o.dtotal * 8, rb = (size_t)o.r_total * rsize(c);
  if (tb > ctx->tab_cap) {
    ctx->tab_cap = 0;
    HIPCHK(dev_alloc((void **)&ctx->d_tab, tb));
    ctx->tab_cap = tb;
  }
  if (rb > ctx->rtab_cap) {
    ctx->rtab_cap = 0;
    HIPCHK(dev_alloc(&ctx->d_rtab, rb));
    ctx->rtab_cap = rb;
  }
  HIPCHK(dev_alloc((void **)&ctx->d_imgmap, (size_t)nl * 4));
  HIPCHK(dev_alloc((void **)&ctx->d_herm, herm.size() * 8));
  HIPCHK(hipMemcpy(ctx->d_herm, herm.data(), herm.size() * 8, hipMemcpyHostToDevice));
  // MRW pre-test without the temperature: for node interval k of the first
  // thermal species' table, the largest Rosseland bound (krmax) of every
  // T-interval that ln T from nodes k-1 .. k+2 falls in. The Hermite value
  // on interval k lies between nodes k and k+1 up to ~1e-10; the extra node
  // on each side covers that and an interval index taken from an FP32 log.
  {
    int s0 = 0;
    while (s0 < ns && s0 == ctx->pah) ++s0;
    const double *hh = s0 < ns ? &herm[(size_t)s0 * HS] : nullptr;
    if (hh && (int)hh[2] == NH_TAB) {
      auto tidx = [&](double lnT) {  // T-interval of krmax as the MRW test takes it
        const double xk = (lnT - lt0) / dlt;
        return (xk >= 0.0 && xk < (double)(NT_TAB - 1)) ? (int)xk : NT_TAB - 1;
      };
      std::vector<double> ub(NH_TAB - 1);
      for (int k = 0; k < NH_TAB - 1; ++k) {
        const int a = k > 0 ? k - 1 : 0, b = k + 2 < NH_TAB ? k + 2 : NH_TAB - 1;
        const double la = hh[3 + 2 * a] - 1e-9, lb = hh[3 + 2 * b] + 1e-9;
        int ka = tidx(la), kb = tidx(lb);
        double mx = 0.0;
        if (ka > kb || la < lt0) mx = t[o.krmax + NT_TAB - 1];
        if (ka <= kb)
          for (int kk = ka; kk <= kb; ++kk) mx = std::max(mx, t[o.krmax + kk]);
        else
          for (int kk = 0; kk < NT_TAB; ++kk) mx = std::max(mx, t[o.krmax + kk]);
        ub[k] = mx;
      }
      HIPCHK(dev_alloc((void **)&ctx->d_mrw_ub, ub.size() * 8));
      HIPCHK(hipMemcpy(ctx->d_mrw_ub, ub.data(), ub.size() * 8, hipMemcpyHostToDevice));
    } else if (ctx->d_mrw_ub) {
      (void)hipFree(ctx->d_mrw_ub);
      ctx->d_mrw_ub = nullptr;
    }
  }
  HIPCHK(dev_alloc((void **)&ctx->d_rej_pe, rej_pe.size() * 4));
  HIPCHK(dev_alloc((void **)&ctx->d_rej_al, rej_al.size()));
  if (!rej_pe.empty()) {
    HIPCHK(hipMemcpy(ctx->d_rej_pe, rej_pe.data(), rej_pe.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_rej_al, rej_al.data(), rej_al.size(), hipMemcpyHostToDevice));
  }
  HIPCHK(hipMemcpy(ctx->d_tab, t.data(), tb, hipMemcpyHostToDevice));
  if (ctx->fp64) {
    HIPCHK(hipMemcpy(ctx->d_rtab, r.data(), rb, hipMemcpyHostToDevice));
  } else {
    std::vector<float> rf(r.begin(), r.end());
    HIPCHK(hipMemcpy(ctx->d_rtab, rf.data(), rb, hipMemcpyHostToDevice));
  }
  HIPCHK(hipMemcpy(ctx->d_imgmap, im.data(), (size_t)nl * 4, hipMemcpyHostToDevice));
  ctx->h_tab = t;
  ctx->tables_ok = true;
  ctx->S_ok = false;
  return MCRT_OK;
}

// ------------------------------------------------------------------- set

// Bricked copy of the density read by the walk, and the occupancy bits of
// its brick runs; rebuilt whenever the density changes.
static uint64_t brick_cells(const mcrt_ctx *ctx) {
  return (uint64_t)ctx->nbx * ctx->nby * ctx->nbz * 64;
}

// The walk may use 32-bit brick indices (brick_index32).
static bool idx32_ok(const mcrt_ctx *ctx) {
  return brick_cells(ctx) < (1ull << 32) && (uint64_t)ctx->nby * ctx->nbz < (1ull << 24);
}

static mcrt_status build_brick(mcrt_ctx *ctx) {
  ctx->nbx = (ctx->nx + 3) / 4;
  ctx->nby = (ctx->ny + 3) / 4;
  ctx->nbz = (ctx->nz + 3) / 4;
  const uint64_t nb = (uint64_t)ctx->nbx * ctx->nby * ctx->nbz * 64;
  HIPCHK(dev_alloc(&ctx->d_rho_b, nb * rsize(ctx)));
  HIPCHK(hipMemset(ctx->d_rho_b, 0, nb * rsize(ctx)));
  HIPCHK(launch_brick(ctx->fp64, ctx->d_rho, ctx->d_rho_b, ctx->nx, ctx->ny, ctx->nz, ctx->nbx,
                      ctx->nby, 0));
  // shortest run of 2^m bricks whose bits fit OCC_MAX_WORDS words
  const uint64_t nbrick = nb / 64;
  int m = 0;
  while (((nbrick + (1ull << m) - 1) >> m) > (uint64_t)OCC_MAX_WORDS * 32) ++m;
  ctx->osh = 6 + m;
  const uint64_t nrun = (nbrick + (1ull << m) - 1) >> m;
  ctx->ow = (int)((nrun + 31) / 32);
  HIPCHK(dev_alloc((void **)&ctx->d_occ, (nrun + 63) / 64 * 8));
  HIPCHK(launch_occ(ctx->fp64, ctx->d_rho_b, ctx->d_occ, nb, ctx->osh, 0));
  HIPCHK(hipDeviceSynchronize());
  return MCRT_OK;
}

static bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }

extern "C" mcrt_status mcrt_set_grid(mcrt_ctx *ctx, int nx, int ny, int nz, const double origin[3],
                                     double dcell, const void *rho, int dtype, int mem) {
  if (!ctx) return MCRT_EINVAL;
  if (nx <= 0 || ny <= 0 || nz <= 0) return fail(ctx, MCRT_EINVAL, "grid dimensions must be > 0");
  if (nx > MAX_AXIS || ny > MAX_AXIS || nz > MAX_AXIS)
    return fail(ctx, MCRT_EINVAL, "at most %d cells per axis", MAX_AXIS);
  if (!origin || !rho) return fail(ctx, MCRT_EINVAL, "origin and rho must be non-NULL");
  if (!(dcell > 0.0) || !std::isfinite(dcell)) return fail(ctx, MCRT_EINVAL, "dcell must be > 0");
  if (dtype != MCRT_FP64 && dtype != MCRT_FP32) return fail(ctx, MCRT_EINVAL, "bad dtype");
  if (mem != MCRT_HOST && mem != MCRT_DEVICE) return fail(ctx, MCRT_EINVAL, "bad mem flag");
  uint64_t n = (uint64_t)nx * ny * nz;
  if (n > (1ull << 34)) return fail(ctx, MCRT_EINVAL, "grid too large");
  HIPCHK(hipSetDevice(ctx->device));
  // copy to host for validation and conversion
  std::vector<double> h(n);
  size_t es = dtype == MCRT_FP64 ? 8 : 4;
  std::vector<unsigned char> raw(n * es);
  if (mem == MCRT_DEVICE) HIPCHK(hipMemcpy(raw.data(), rho, n * es, hipMemcpyDeviceToHost));
  else memcpy(raw.data(), rho, n * es);
  for (uint64_t i = 0; i < n; ++i) {
    double v = dtype == MCRT_FP64 ? ((double *)raw.data())[i] : (double)((float *)raw.data())[i];
    if (!finite_nonneg(v)) return fail(ctx, MCRT_EINVAL, "rho[%llu] is negative or not finite", (unsigned long long)i);
    h[i] = v;
  }
  HIPCHK(dev_alloc(&ctx->d_rho, n * rsize(ctx)));
  if (ctx->fp64) {
    HIPCHK(hipMemcpy(ctx->d_rho, h.data(), n * 8, hipMemcpyHostToDevice));
  } else {
    std::vector<float> f(h.begin(), h.end());
    HIPCHK(hipMemcpy(ctx->d_rho, f.data(), n * 4, hipMemcpyHostToDevice));
  }
  ctx->nx = nx; ctx->ny = ny; ctx->nz = nz;
  for (int k = 0; k < 3; ++k) ctx->origin[k] = origin[k];
  ctx->dcell = dcell;
  ctx->ncell = ctx->ncube = n;
  ctx->nsub = 0;
  ctx->max_r = 1;
  {
    mcrt_status sb = build_brick(ctx);
    if (sb) return sb;
  }
  ctx->has_grid = true;
  ctx->S_ok = false;
  if (ctx->has_dust) {
    mcrt_status s = ensure_state(ctx, 0);
    if (s) return s;
    s = zero_tallies(ctx, 0);
    if (s) return s;
    s = zero_epoch(ctx, 0);
    if (s) return s;
    HIPCHK(hipDeviceSynchronize());
  }
  return MCRT_OK;
}

extern "C" mcrt_status mcrt_set_refinement(mcrt_ctx *ctx, const uint8_t *ref, const void *rho_sub,
                                           uint64_t nsub, int dtype) {
  if (!ctx) return MCRT_EINVAL;
  if (!ctx->has_grid) return fail(ctx, MCRT_ESTATE, "set the grid before its refinement");
  if (dtype != MCRT_FP64 && dtype != MCRT_FP32) return fail(ctx, MCRT_EINVAL, "bad dtype");
  HIPCHK(hipSetDevice(ctx->device));
  const uint64_t nc = ctx->ncube;
  std::vector<uint64_t> off(nc, 0);
  uint64_t tot = 0;
  int rmax = 1;
  if (ref) {
    for (uint64_t c = 0; c < nc; ++c) {
      off[c] = tot;
      const int r = ref[c];
      if (r > MAX_REF) return fail(ctx, MCRT_EINVAL, "ref[%llu] = %d exceeds %d", (unsigned long long)c, r, MAX_REF);
      if (r >= 2) {
        tot += (uint64_t)r * r * r;
        if (r > rmax) rmax = r;
      }
    }
  }
  if (tot != nsub) return fail(ctx, MCRT_EINVAL, "nsub = %llu, the divided cubes hold %llu", (unsigned long long)nsub, (unsigned long long)tot);
  if (tot > 0 && !rho_sub) return fail(ctx, MCRT_EINVAL, "rho_sub is NULL");
  if (nc + tot > (1ull << 34)) return fail(ctx, MCRT_EINVAL, "too many cells");
  std::vector<double> h(tot);
  for (uint64_t i = 0; i < tot; ++i) {
    double v = dtype == MCRT_FP64 ? ((const double *)rho_sub)[i] : (double)((const float *)rho_sub)[i];
    if (!finite_nonneg(v)) return fail(ctx, MCRT_EINVAL, "rho_sub[%llu] is negative or not finite", (unsigned long long)i);
    h[i] = v;
  }
  // cube densities stay first; sub-cube densities follow them
  void *nr = nullptr;
  HIPCHK(dev_alloc(&nr, (nc + tot) * rsize(ctx)));
  HIPCHK(hipMemcpy(nr, ctx->d_rho, nc * rsize(ctx), hipMemcpyDeviceToDevice));
  if (tot > 0) {
    char *dst = (char *)nr + nc * rsize(ctx);
    if (ctx->fp64) {
      HIPCHK(hipMemcpy(dst, h.data(), tot * 8, hipMemcpyHostToDevice));
    } else {
      std::vector<float> f(h.begin(), h.end());
      HIPCHK(hipMemcpy(dst, f.data(), tot * 4, hipMemcpyHostToDevice));
    }
  }
  (void)hipFree(ctx->d_rho);
  ctx->d_rho = nr;
  if (tot > 0) {
    HIPCHK(dev_alloc((void **)&ctx->d_ref, nc));
    HIPCHK(hipMemcpy(ctx->d_ref, ref, nc, hipMemcpyHostToDevice));
    HIPCHK(dev_alloc((void **)&ctx->d_suboff, nc * 8));
    HIPCHK(hipMemcpy(ctx->d_suboff, off.data(), nc * 8, hipMemcpyHostToDevice));
  } else {
    if (ctx->d_ref) (void)hipFree(ctx->d_ref);
    if (ctx->d_suboff) (void)hipFree(ctx->d_suboff);
    ctx->d_ref = nullptr;
    ctx->d_suboff = nullptr;
  }
  ctx->nsub = tot;
  ctx->max_r = rmax;
  ctx->ncell = nc + tot;
  ctx->S_ok = false;
  ctx->sh_have = 0;
  if (ctx->d_ssca) {
    (void)hipFree(ctx->d_ssca);
    ctx->d_ssca = nullptr;
  }
  ctx->ssca_cap = 0;
  if (ctx->has_dust) {
    mcrt_status s = ensure_state(ctx, 0);
    if (s) return s;
    s = ensure_ssca(ctx);
    if (s) return s;
    s = zero_tallies(ctx, 0);
    if (s) return s;
    s = zero_epoch(ctx, 0);
    if (s) return s;
  }
  HIPCHK(hipDeviceSynchronize());
  return MCRT_OK;
}

static mcrt_status grid_geom(mcrt_ctx *ctx, int nx, int ny, int nz, const double origin[3], double dcell) {
  if (nx <= 0 || ny <= 0 || nz <= 0) return fail(ctx, MCRT_EINVAL, "grid dimensions must be > 0");
  if (nx > MAX_AXIS || ny > MAX_AXIS || nz > MAX_AXIS)
    return fail(ctx, MCRT_EINVAL, "at most %d cells per axis", MAX_AXIS);
  if (!origin) return fail(ctx, MCRT_EINVAL, "origin is NULL");
  if (!(dcell > 0.0) || !std::isfinite(dcell)) return fail(ctx, MCRT_EINVAL, "dcell must be > 0");
  uint64_t n = (uint64_t)nx * ny * nz;
  if (n > (1ull << 34)) return fail(ctx, MCRT_EINVAL, "grid too large");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(dev_alloc(&ctx->d_rho, n * rsize(ctx)));
  ctx->nx = nx; ctx->ny = ny; ctx->nz = nz;
  for (int k = 0; k < 3; ++k) ctx->origin[k] = origin[k];
  ctx->dcell = dcell;
  ctx->ncell = ctx->ncube = n;
  ctx->nsub = 0;
  ctx->max_r = 1;
  return MCRT_OK;
}

static mcrt_status grid_done(mcrt_ctx *ctx) {
  mcrt_status sb = build_brick(ctx);
  if (sb) return sb;
  ctx->has_grid = true;
  ctx->S_ok = false;
  if (ctx->has_dust) {
    mcrt_status s = ensure_state(ctx, 0);
    if (s) return s;
    s = zero_tallies(ctx, 0);
    if (s) return s;
    s = zero_epoch(ctx, 0);
    if (s) return s;
  }
  HIPCHK(hipDeviceSynchronize());
  return MCRT_OK;
}

extern "C" mcrt_status mcrt_voxelize_torus(mcrt_ctx *ctx, int nx, int ny, int nz,
                                           const double origin[3], double dcell, int n_clumps,
                                           const double *centres, double r_clump,
                                           double rho_clump, double rho_inter, double r_in,
                                           double r_out, double sin_theta1) {
  if (!ctx) return MCRT_EINVAL;
  if (n_clumps < 0 || (n_clumps > 0 && !centres)) return fail(ctx, MCRT_EINVAL, "bad clump list");
  if (!finite_nonneg(rho_clump) || !finite_nonneg(rho_inter) || !finite_nonneg(r_clump) ||
      !finite_nonneg(r_in) || !(r_out >= r_in) || !(sin_theta1 >= 0.0 && sin_theta1 <= 1.0))
    return fail(ctx, MCRT_EINVAL, "bad torus parameters");
  mcrt_status s = grid_geom(ctx, nx, ny, nz, origin, dcell);
  if (s) return s;
  double *dC = nullptr;
  if (n_clumps > 0) {
    HIPCHK(hipMalloc((void **)&dC, (size_t)n_clumps * 24));
    HIPCHK(hipMemcpy(dC, centres, (size_t)n_clumps * 24, hipMemcpyHostToDevice));
  }
  hipError_t e = launch_vox_torus(ctx->fp64, nx, ny, nz, origin, dcell, n_clumps, dC, r_clump,
                                  rho_clump, rho_inter, r_in, r_out, sin_theta1, ctx->d_rho, 0);
  hipError_t e2 = hipDeviceSynchronize();
  if (dC) (void)hipFree(dC);
  if (e != hipSuccess || e2 != hipSuccess)
    return fail(ctx, MCRT_EDEVICE, "torus voxelizer: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  return grid_done(ctx);
}

// Gauss-Legendre rule: roots of P_n by Newton from Chebyshev-like guesses.
static void gl_rule(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double pm = 1.0, pc = z;  // P_0, P_1
      for (int k = 2; k <= n; ++k) {
        double pn = ((2.0 * k - 1.0) * z * pc - (k - 1.0) * pm) / k;
        pm = pc;
        pc = pn;
      }
      dp = n * (z * pc - pm) / (z * z - 1.0);
      double dz = pc / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-15) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

extern "C" mcrt_status mcrt_voxelize_shell(mcrt_ctx *ctx, int nx, int ny, int nz,
                                           const double origin[3], double dcell, double rho0,
                                           double r_in, double r_out, double power) {
  if (!ctx) return MCRT_EINVAL;
  if (!finite_nonneg(rho0) || !(r_in > 0.0) || !(r_out >= r_in) || !std::isfinite(r_out) ||
      !std::isfinite(power))
    return fail(ctx, MCRT_EINVAL, "bad shell parameters");
  mcrt_status s = grid_geom(ctx, nx, ny, nz, origin, dcell);
  if (s) return s;
  std::vector<double> gx, gw;
  gl_rule(8, gx, gw);
  double *dg = nullptr;
  HIPCHK(hipMalloc((void **)&dg, 16 * 8));
  HIPCHK(hipMemcpy(dg, gx.data(), 64, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(dg + 8, gw.data(), 64, hipMemcpyHostToDevice));
  hipError_t e = launch_vox_shell(ctx->fp64, nx, ny, nz, origin, dcell, rho0, r_in, r_out, power,
                                  8, dg, dg + 8, ctx->d_rho, 0);
  hipError_t e2 = hipDeviceSynchronize();
  (void)hipFree(dg);
  if (e != hipSuccess || e2 != hipSuccess)
    return fail(ctx, MCRT_EDEVICE, "shell voxelizer: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  return grid_done(ctx);
}

extern "C" mcrt_status mcrt_set_dust(mcrt_ctx *ctx, int n_lambda, const double *lambda_um,
                                     int n_species, const double *mass_frac, const double *kabs,
                                     const double *ksca, const double *g, int pah_species,
                                     int n_pah_rows, const double *pah_emis,
                                     const double *pah_row_edges) {
  if (!ctx) return MCRT_EINVAL;
  if (n_lambda < 2 || n_lambda > MAX_NL) return fail(ctx, MCRT_EINVAL, "n_lambda must be 2..%d", MAX_NL);
  if (n_species < 1 || n_species > MAX_NS) return fail(ctx, MCRT_EINVAL, "n_species must be 1..%d", MAX_NS);
  if (!lambda_um || !mass_frac || !kabs || !ksca || !g) return fail(ctx, MCRT_EINVAL, "NULL dust array");
  for (int j = 0; j < n_lambda; ++j) {
    if (!(lambda_um[j] > 0.0) || !std::isfinite(lambda_um[j]))
      return fail(ctx, MCRT_EINVAL, "lambda must be positive");
    if (j > 0 && !(lambda_um[j] > lambda_um[j - 1]))
      return fail(ctx, MCRT_EINVAL, "lambda must be strictly increasing");
  }
  for (int s = 0; s < n_species; ++s) {
    if (!finite_nonneg(mass_frac[s])) return fail(ctx, MCRT_EINVAL, "mass fractions must be >= 0");
    for (int j = 0; j < n_lambda; ++j) {
      int q = s * n_lambda + j;
      if (!finite_nonneg(kabs[q]) || !finite_nonneg(ksca[q]))
        return fail(ctx, MCRT_EINVAL, "kappa must be finite and >= 0");
      if (!(std::fabs(g[q]) < 1.0)) return fail(ctx, MCRT_EINVAL, "|g| must be < 1");
    }
  }
  if (pah_species >= n_species || pah_species < -1) return fail(ctx, MCRT_EINVAL, "bad pah_species");
  if (pah_species >= 0) {
    if (n_pah_rows < 1 || !pah_emis || (n_pah_rows > 1 && !pah_row_edges))
      return fail(ctx, MCRT_EINVAL, "PAH species needs emissivity rows and edges");
    for (int i = 0; i < n_pah_rows * n_lambda; ++i)
      if (!finite_nonneg(pah_emis[i])) return fail(ctx, MCRT_EINVAL, "PAH emissivity must be >= 0");
  }
  HIPCHK(hipSetDevice(ctx->device));
  ctx->nl = n_lambda;
  ctx->ns = n_species;
  ctx->lam.assign(lambda_um, lambda_um + n_lambda);
  ctx->frac.assign(mass_frac, mass_frac + n_species);
  ctx->kabs.assign(kabs, kabs + n_species * n_lambda);
  ctx->ksca.assign(ksca, ksca + n_species * n_lambda);
  ctx->g.assign(g, g + n_species * n_lambda);
  ctx->pah = pah_species;
  ctx->nrows = pah_species >= 0 ? n_pah_rows : 0;
  ctx->pah_emis.assign(pah_species >= 0 ? pah_emis : nullptr,
                       pah_species >= 0 ? pah_emis + n_pah_rows * n_lambda : nullptr);
  ctx->pah_edges.clear();
  if (pah_species >= 0 && n_pah_rows > 1) ctx->pah_edges.assign(pah_row_edges, pah_row_edges + n_pah_rows - 1);
  ctx->has_dust = true;
  ctx->has_src = false;  // source spectra live on the wavelength grid
  if (ctx->has_grid) {
    mcrt_status s = ensure_state(ctx, 0);
    if (s) return s;
  }
  HIPCHK(hipDeviceSynchronize());
  return MCRT_OK;
}

extern "C" mcrt_status mcrt_set_sources(mcrt_ctx *ctx, int n_src, const double *pos_cm,
                                        const double *lum, const double *lnu_shape,
                                        const double *t_bb) {
  if (!ctx) return MCRT_EINVAL;
  if (!ctx->has_dust) return fail(ctx, MCRT_ESTATE, "set_dust before set_sources");
  if (!ctx->has_grid) return fail(ctx, MCRT_ESTATE, "set the grid before set_sources");
  if (n_src < 1 || n_src > MAX_SRC) return fail(ctx, MCRT_EINVAL, "n_src must be 1..%d", MAX_SRC);
  if (!pos_cm || !lum || (!lnu_shape && !t_bb)) return fail(ctx, MCRT_EINVAL, "NULL source array");
  const int nl = ctx->nl;
  std::vector<double> nu(nl), w(nl);
  for (int j = 0; j < nl; ++j) nu[j] = C_LI / (ctx->lam[j] * 1e-4);
  for (int j = 0; j < nl; ++j) {
    const double *L = ctx->lam.data();
    double lo = (j == 0) ? L[0] * std::sqrt(L[0] / L[1]) : std::sqrt(L[j - 1] * L[j]);
    double hi = (j == nl - 1) ? L[nl - 1] * std::sqrt(L[nl - 1] / L[nl - 2]) : std::sqrt(L[j] * L[j + 1]);
    w[j] = C_LI / (lo * 1e-4) - C_LI / (hi * 1e-4);
  }
  std::vector<double> lnu((size_t)n_src * nl);
  for (int s = 0; s < n_src; ++s) {
    if (!finite_nonneg(lum[s])) return fail(ctx, MCRT_EINVAL, "luminosity must be >= 0");
    for (int k = 0; k < 3; ++k) {
      double p = pos_cm[3 * s + k];
      double lo = ctx->origin[k];
      double hi = ctx->origin[k] + (double)(k == 0 ? ctx->nx : k == 1 ? ctx->ny : ctx->nz) * ctx->dcell;
      if (!(p >= lo && p <= hi)) return fail(ctx, MCRT_EINVAL, "source %d lies outside the grid", s);
    }
    std::vector<double> shape(nl);
    for (int j = 0; j < nl; ++j) {
      shape[j] = lnu_shape ? lnu_shape[s * nl + j] : h_planck(nu[j], t_bb[s]);
      if (!finite_nonneg(shape[j])) return fail(ctx, MCRT_EINVAL, "source spectrum must be >= 0");
    }
    double norm = 0.0;
    for (int j = nl - 1; j >= 0; --j) norm += w[j] * shape[j];
    if (!(norm > 0.0)) return fail(ctx, MCRT_EINVAL, "source %d has an empty spectrum", s);
    for (int j = 0; j < nl; ++j) lnu[s * nl + j] = lum[s] * shape[j] / norm;
  }
  ctx->nsrc = n_src;
  ctx->src_pos.assign(pos_cm, pos_cm + 3 * n_src);
  ctx->src_lum.assign(lum, lum + n_src);
  ctx->src_lnu = lnu;
  ctx->has_src = true;
  return build_tables(ctx);
}

extern "C" mcrt_status mcrt_set_views(mcrt_ctx *ctx, int n_views, const double *theta_phi_deg,
                                      int n_img, const int32_t *lambda_idx, double distance_cm) {
  if (!ctx) return MCRT_EINVAL;
  if (!ctx->has_dust) return fail(ctx, MCRT_ESTATE, "set_dust before set_views");
  if (n_views < 0 || n_views > MAX_VIEW) return fail(ctx, MCRT_EINVAL, "n_views must be 0..%d", MAX_VIEW);
  if (n_img < 0 || n_img > MAX_IMG) return fail(ctx, MCRT_EINVAL, "n_img must be 0..%d", MAX_IMG);
  if ((n_views > 0 && !theta_phi_deg) || (n_img > 0 && !lambda_idx))
    return fail(ctx, MCRT_EINVAL, "NULL view arrays");
  if (!(distance_cm > 0.0) || !std::isfinite(distance_cm)) return fail(ctx, MCRT_EINVAL, "distance must be > 0");
  std::vector<int> seen(ctx->nl, 0);
  for (int q = 0; q < n_img; ++q) {
    if (lambda_idx[q] < 0 || lambda_idx[q] >= ctx->nl) return fail(ctx, MCRT_EINVAL, "imaged index out of range");
    if (seen[lambda_idx[q]]++) return fail(ctx, MCRT_EINVAL, "imaged indices must be distinct");
  }
  ctx->nview = n_views;
  ctx->nimg = n_img;
  ctx->views.assign(theta_phi_deg, theta_phi_deg + 2 * n_views);
  ctx->img_idx.assign(lambda_idx, lambda_idx + n_img);
  ctx->distance = distance_cm;
  ctx->ssca_cap = 0;
  if (ctx->d_ssca) {
    (void)hipFree(ctx->d_ssca);
    ctx->d_ssca = nullptr;
  }
  if (ctx->has_grid) {
    mcrt_status s = ensure_ssca(ctx);
    if (s) return s;
    uint64_t m = (uint64_t)ctx->nview * ctx->nimg * ctx->ncell;
    if (ctx->d_ssca) {
      if (ctx->fp64) HIPCHK(fill<double>((double *)ctx->d_ssca, 0.0, m, 0));
      else HIPCHK(fill<float>((float *)ctx->d_ssca, 0.0f, m, 0));
    }
  }
  // moments are kept for their imaged wavelengths (valid for any views)
  if (ctx->sh_have > 0 && ctx->sh_img != ctx->img_idx) ctx->sh_have = 0;
  ctx->S_ok = false;
  mcrt_status s = build_tables(ctx);
  if (s) return s;
  HIPCHK(hipDeviceSynchronize());
  return MCRT_OK;
}

static mcrt_status ready(mcrt_ctx *ctx) {
  if (!ctx) return MCRT_EINVAL;
  if (!ctx->has_grid) return fail(ctx, MCRT_ESTATE, "grid not set");
  if (!ctx->has_dust) return fail(ctx, MCRT_ESTATE, "dust not set");
  if (!ctx->has_src) return fail(ctx, MCRT_ESTATE, "sources not set");
  if (!ctx->tables_ok) return fail(ctx, MCRT_ESTATE, "tables not built");
  return MCRT_OK;
}

// Host image of the model descriptor for a launch.
// The fast interaction kernel (with its slow list) serves the FP32 walk in
// immediate B&W without packet records or scattering moments.
static bool fast_interactions(const mcrt_ctx *ctx, const mcrt_run_opts *o) {
  return !ctx->fp64 && o && o->record == 0 && o->mode == MCRT_BW_TICKET &&
         !(o->sh_order > 0 && ctx->nimg > 0);
}

// Round variant: 0 general interaction kernel, 1 fast kernel, 2 fast kernel
// with the per-cell diffusion flags (diffusion steps armed).
static int fast_mode(const mcrt_ctx *ctx, const mcrt_run_opts *o) {
  if (!fast_interactions(ctx, o)) return 0;
  return o->mrw_tau > 0.0 ? 2 : 1;
}

// Blocks per compute unit of the emission and interaction kernels when the
// caller leaves it open: the fast interaction kernel fits three waves per
// SIMD (158 VGPRs) and waits on memory, so a third block hides more of it
// (measured on the 256^3 torus: interaction 73 -> 65 ms per step, no gain
// from a fourth); the general kernels fit two.
static int default_bpc(int fast) { return fast ? 3 : 2; }

static mcrt_status ensure_mrw_flags(mcrt_ctx *ctx) {
  const size_t nw = (ctx->ncell + 31) / 32;
  if (ctx->d_mrw_flags && ctx->mrw_flags_cap >= nw) return MCRT_OK;
  ctx->mrw_flags_cap = 0;
  HIPCHK(dev_alloc((void **)&ctx->d_mrw_flags, 2 * nw * 4));
  ctx->mrw_flags_cap = nw;
  return MCRT_OK;
}

// Ray-tracer source terms: printed form of Eqs. 13-14, and the order of the
// scattering moments the scattered light is formed from (0: per-view sums).
static bool rt_lit(const mcrt_ctx *ctx) { return ctx->rt_mode == MCRT_RT_ABS_LITERAL; }
static int sh_read(const mcrt_ctx *ctx) {
  return ctx->ssca_src == MCRT_SSCA_MOMENTS ? ctx->sh_have : 0;
}

static void fill_model(mcrt_ctx *ctx, ModelDev &M, const mcrt_run_opts *o, int model_id) {
  memset(&M, 0, sizeof(M));
  M.nx = ctx->nx; M.ny = ctx->ny; M.nz = ctx->nz;
  M.nl = ctx->nl; M.ns = ctx->ns; M.nsrc = ctx->nsrc; M.pah = ctx->pah; M.nrows = ctx->nrows;
  M.nview = ctx->nview; M.nimg = ctx->nimg; M.ntheta = ctx->ntheta; M.model_id = model_id;
  M.mode = o ? o->mode : M_BW_TICKET;
  M.record = o ? o->record : 0;
  M.tau_mode = o ? o->tau_mode : 0;
  M.src_strata = o ? o->src_strata : 0;
  M.pah_nc = o ? o->pah_nc : 0.0;
  M.pah_tcool = o ? o->pah_tcool : 0.0;
  M.sh_order = (o && o->sh_order > 0 && ctx->nimg > 0) ? o->sh_order : 0;
  M.sh = ctx->d_sh;
  M.sh_read = o ? 0 : sh_read(ctx);
  M.rt_lit = rt_lit(ctx) ? 1 : 0;
  M.pass = 1;
  M.iter = 0;
  for (int k = 0; k < 3; ++k) M.origin[k] = ctx->origin[k];
  M.dcell = ctx->dcell;
  M.V = ctx->dcell * ctx->dcell * ctx->dcell;
  M.xi = ctx->xi;
  M.lucy_tau = o ? o->lucy_tau : 0.0;
  M.mrw_tau = o ? o->mrw_tau : 0.0;
  M.mrw_gamma = o ? o->mrw_gamma : 2.0;
  M.kext_max = ctx->kext_max;
  M.ssca_unit = ctx->ssca_unit;
  M.kr_gmax = ctx->kr_gmax;
  M.phi_tmin = ctx->phi_tmin;
  for (int k = 0; k < MAX_NS; ++k) M.herm_pmin[k] = ctx->herm_pmin[k];
  M.max_int = o ? o->max_interactions : 0;
  M.ncell = ctx->ncell;
  M.ncube = ctx->ncube;
  M.ref = ctx->nsub > 0 ? ctx->d_ref : nullptr;
  M.sub_off = ctx->nsub > 0 ? ctx->d_suboff : nullptr;
  M.rho = ctx->d_rho;
  M.rho_b = ctx->d_rho_b;
  M.nbx = ctx->nbx; M.nby = ctx->nby; M.nbz = ctx->nbz;
  M.occ = ctx->d_occ;
  M.osh = ctx->osh; M.ow = ctx->ow;
  M.tab = ctx->d_tab;
  M.rtab = ctx->d_rtab;
  M.imgmap = ctx->d_imgmap;
  M.herm = ctx->d_herm;
  M.mrw_ub = ctx->d_mrw_ub;
  const bool flags = fast_mode(ctx, o) == 2 && ctx->d_mrw_flags;
  M.mrw_cand = flags ? ctx->d_mrw_flags : nullptr;
  M.mrw_bits = flags ? ctx->d_mrw_flags + ctx->mrw_flags_cap : nullptr;
  M.rej_pe = ctx->d_rej_pe;
  M.rej_al = ctx->d_rej_al;
  for (int q = 0; q < ctx->nimg; ++q) M.img_j[q] = ctx->img_idx[q];
  M.k = ctx->d_k; M.epath = ctx->d_epath; M.T = ctx->d_T; M.esnap = ctx->d_esnap; M.tt = ctx->d_tt;
  M.dirty = ctx->d_dirty; M.kpah = ctx->d_kpah; M.kpah_prefix = ctx->d_prefix;
  M.sed = ctx->d_sed;
  M.ssca = ctx->d_ssca;
  M.rec = nullptr;
  M.ctl = ctx->d_ctl;
  M.counter = &ctx->d_ctl->emitted;  // address arithmetic only
  for (int k = 0; k < 2; ++k) {
    M.q[k] = ctx->q[k];
    if (ctx->nsub == 0) M.q[k].fine = nullptr;  // whole cubes only: no sub-cube indices
  }
  M.qcap = ctx->qcap;
  M.qseg = ctx->qcap / NSEG;
  M.stats = ctx->d_stats;
  for (int v = 0; v < ctx->nview; ++v) {
    double th = ctx->views[2 * v] * PI_D / 180.0, ph = ctx->views[2 * v + 1] * PI_D / 180.0;
    M.kv[v][0] = std::sin(th) * std::cos(ph);
    M.kv[v][1] = std::sin(th) * std::sin(ph);
    M.kv[v][2] = std::cos(th);
  }
}

static mcrt_status check_opts(mcrt_ctx *ctx, const mcrt_run_opts *o) {
  if (!o) return fail(ctx, MCRT_EINVAL, "opts is NULL");
  if (o->mode < MCRT_FROZEN || o->mode > MCRT_BW_TICKET) return fail(ctx, MCRT_EINVAL, "bad mode");
  if (o->mode == MCRT_FROZEN && o->n_iter < 1) return fail(ctx, MCRT_EINVAL, "n_iter must be >= 1");
  if (o->mode == MCRT_BW_EPOCH && o->epoch_packets < 1) return fail(ctx, MCRT_EINVAL, "epoch_packets must be >= 1");
  if (o->sed_theta_bins < 1 || o->sed_theta_bins > 180) return fail(ctx, MCRT_EINVAL, "sed_theta_bins must be 1..180");
  if (o->mrw_tau > 0.0 && !(o->mrw_gamma > 0.0)) return fail(ctx, MCRT_EINVAL, "mrw_gamma must be > 0");
  if (!std::isfinite(o->lucy_tau) || !std::isfinite(o->mrw_tau)) return fail(ctx, MCRT_EINVAL, "non-finite threshold");
  if (o->blocks_per_cu < 0 || o->blocks_per_cu > 32) return fail(ctx, MCRT_EINVAL, "blocks_per_cu must be 0..32");
  if (o->walk_blocks_per_cu < 0 || o->walk_blocks_per_cu > 32)
    return fail(ctx, MCRT_EINVAL, "walk_blocks_per_cu must be 0..32");
  if (o->queue_depth != 0 && (o->queue_depth < 64 || o->queue_depth > (1 << 26)))
    return fail(ctx, MCRT_EINVAL, "queue_depth must be 0 or 64..2^26");
  if (o->tau_mode != MCRT_TAU_FLIGHT && o->tau_mode != MCRT_TAU_PER_CELL)
    return fail(ctx, MCRT_EINVAL, "tau_mode must be MCRT_TAU_FLIGHT or MCRT_TAU_PER_CELL");
  if (!std::isfinite(o->pah_nc) || !std::isfinite(o->pah_tcool) || o->pah_tcool < 0.0)
    return fail(ctx, MCRT_EINVAL, "pah_nc and pah_tcool must be finite, pah_tcool >= 0");
  if (o->sh_order < 0 || o->sh_order > MAX_SH_ORDER)
    return fail(ctx, MCRT_EINVAL, "sh_order must be 0..%d", MAX_SH_ORDER);
  return MCRT_OK;
}

// Packet range of the next launch (device-side, in stream order).
// Every queue counter of a model back to zero (one block).
__device__ void wf_zero(WfCtl *c) {
  uint32_t *w = (uint32_t *)c;
  for (size_t i = threadIdx.x; i < sizeof(WfCtl) / 4; i += blockDim.x) w[i] = 0u;
}

__global__ void k_set_range(ModelDev *m, uint64_t first, uint64_t n) {
  if (threadIdx.x == 0) {
    m->first = first;
    m->n = n;
  }
  wf_zero(m->ctl);
}

static mcrt_status set_range(mcrt_ctx *ctx, uint64_t first, uint64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_set_range, dim3(1), dim3(256), 0, st, ctx->d_model, first, n);
  HIPCHK(hipGetLastError());
  return MCRT_OK;
}


// Wavefront queues: two queues of Q packets as structures of arrays,
// carved from one allocation (256-byte aligned arrays).
static mcrt_status ensure_queues(mcrt_ctx *ctx, const mcrt_run_opts *o, uint64_t n) {
  uint64_t want = (o && o->queue_depth > 0) ? (uint64_t)o->queue_depth : (1ull << 25);
  if (want > (1ull << 26)) want = 1ull << 26;
  uint64_t need = (n + 4095) / 4096 * 4096;
  if (need < 4096) need = 4096;
  uint32_t Q = (uint32_t)(want < need ? want : need);
  Q = Q / NSEG * NSEG;  // whole segments
  if (Q < NSEG) Q = NSEG;
  if (Q <= ctx->qcap && ctx->d_q) return MCRT_OK;
  const size_t rs = rsize(ctx);
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t per = 8 * al(Q * rs) + 2 * al(Q * 8) + 9 * al(Q * 4) + al(Q * 8);
  HIPCHK(dev_alloc(&ctx->d_q, 2 * per));
  char *b = (char *)ctx->d_q;
  for (int k = 0; k < 2; ++k) {
    QBuf &q = ctx->q[k];
    void **rv[8] = {&q.px, &q.py, &q.pz, &q.dx, &q.dy, &q.dz, &q.rho, &q.tau};
    for (void **r : rv) { *r = b; b += al(Q * rs); }
    q.cj = (uint64_t *)b; b += al(Q * 8);
    q.pid = (uint64_t *)b; b += al(Q * 8);
    uint32_t **uv[9] = {&q.rngd, &q.nint, &q.ncross, &q.nscat, &q.nabs, &q.nmrw, &q.nlucy,
                        &q.fine, &q.slow};
    for (uint32_t **r : uv) { *r = (uint32_t *)b; b += al(Q * 4); }
    q.mm = (double *)b; b += al(Q * 8);
  }
  ctx->qcap = Q;
  return MCRT_OK;
}

// Four fresh events for the next round's phase timing (null when the
// pool cannot grow; timing is then skipped for that round).
static const hipEvent_t *phase_events(mcrt_ctx *ctx) {
  if (ctx->pev_used + 4 > ctx->pev.size()) {
    for (int k = 0; k < 64; ++k) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      ctx->pev.push_back(e);
    }
  }
  const hipEvent_t *e = ctx->pev.data() + ctx->pev_used;
  ctx->pev_used += 4;
  return e;
}

// Adds the recorded rounds' kernel times to the phase totals (after a sync).
static void phase_collect(mcrt_ctx *ctx) {
  for (size_t i = 0; i + 3 < ctx->pev_used; i += 4) {
    for (int k = 0; k < 3; ++k) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, ctx->pev[i + k], ctx->pev[i + k + 1]) == hipSuccess)
        ctx->t_phase[k] += ms;
    }
    ctx->n_rounds++;
  }
  ctx->pev_used = 0;
}

// Transport of the n packets set by set_range: wavefront rounds until every
// packet has been started and has ended. The host reads the queue counters
// every few rounds to stop.
static mcrt_status transport_launch(mcrt_ctx *ctx, const mcrt_run_opts *o, uint64_t n,
                                    hipStream_t st) {
  size_t lds = transport_lds_bytes(ctx->nl, ctx->ns, ctx->nsrc, ctx->nrows, ctx->ntheta, ctx->fp64);
  size_t lds_w = walk_lds_bytes(ctx->nl, ctx->ns, ctx->nsrc, ctx->nrows, ctx->ntheta, ctx->ow,
                                ctx->fp64);
  if (lds > ctx->lds_max || lds_w > ctx->lds_max)
    return fail(ctx, MCRT_EINVAL, "tables need %zu bytes of LDS (limit %zu): fewer wavelengths, species or SED bins", lds > lds_w ? lds : lds_w, ctx->lds_max);
  const bool rec = o->record != 0;
  const bool per_cell = o->tau_mode == MCRT_TAU_PER_CELL;
  const int fast = fast_mode(ctx, o);
  const int gfull = ctx->num_cu * (o->blocks_per_cu > 0 ? o->blocks_per_cu : default_bpc(fast));
  const int gwalk = ctx->num_cu * (o->walk_blocks_per_cu > 0 ? o->walk_blocks_per_cu : 4);
  if (fast == 2) HIPCHK(launch_mrw_cand(ctx->d_model, 1, ctx->num_cu, st));
  const int every = 4;
  // the finishing kernel takes over once every packet has been started and
  // the survivors fit one lane each at two blocks of 256 per CU
  const size_t lds_f = lds + (size_t)ctx->ow * 4;
  const uint32_t fin_max = (uint32_t)ctx->num_cu * 2u * 256u;
  for (uint64_t r = 0;; ++r) {
    const int fcur = (int)(r & 1);
    const hipEvent_t *ev = phase_events(ctx);
    HIPCHK(launch_wf_round(ctx->d_model, 1, ctx->fp64, rec, fcur, gfull, gwalk, lds, lds_w,
                           idx32_ok(ctx), per_cell, ctx->nsub > 0, fast, ev, st));
    if ((r + 1) % every == 0) {
      HIPCHK(launch_wf_busy(ctx->d_model, 1, fcur, &ctx->d_ctl->busy, &ctx->d_ctl->left, st));
      // emitted .. left: the header of the counters
      HIPCHK(hipMemcpyAsync(ctx->h_ctl, ctx->d_ctl, offsetof(WfCtl, pad), hipMemcpyDeviceToHost,
                            st));
      HIPCHK(hipStreamSynchronize(st));
      phase_collect(ctx);
      if (ctx->h_ctl->busy == 0u) break;
      if (ctx->h_ctl->emitted >= n && ctx->h_ctl->left <= fin_max && lds_f <= ctx->lds_max) {
        // timed as one more round whose walk phase is the finishing kernel
        const hipEvent_t *fe = phase_events(ctx);
        if (fe) {
          HIPCHK(hipEventRecord(fe[0], st));
          HIPCHK(hipEventRecord(fe[1], st));
        }
        HIPCHK(launch_wf_finish(ctx->d_model, 1, ctx->fp64, rec, 1 - fcur, gfull, lds_f,
                                idx32_ok(ctx), per_cell, ctx->nsub > 0, st));
        if (fe) {
          HIPCHK(hipEventRecord(fe[2], st));
          HIPCHK(hipEventRecord(fe[3], st));
        }
        HIPCHK(hipStreamSynchronize(st));
        phase_collect(ctx);
        break;
      }
    }
    if (r > (1ull << 32)) return fail(ctx, MCRT_EDEVICE, "transport did not finish");
  }
  if (o->mode != MCRT_BW_EPOCH) ctx->snap_stale = true;
  return MCRT_OK;
}

static mcrt_status read_stats(mcrt_ctx *ctx, mcrt_run_stats *stats, hipStream_t st) {
  unsigned long long h[NSTAT];
  HIPCHK(hipMemcpyAsync(h, ctx->d_stats, sizeof h, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  float ms = 0.0f;
  HIPCHK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  ctx->t_transport = ms;
  if (stats) {
    stats->packets = h[0]; stats->escaped = h[1]; stats->killed = h[2]; stats->pah_stopped = h[3];
    stats->crossings = h[4]; stats->scatters = h[5]; stats->absorptions = h[6];
    stats->mrw_steps = h[7]; stats->lucy_deposits = h[8]; stats->clamped_T = h[9];
    stats->kernel_ms = ms;
  }
  return MCRT_OK;
}

template <typename T>
__global__ void k_scale(T *p, double f, uint64_t n) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = (T)((double)p[i] * f);
}

// Scattering sums are stored in units of the packet energy of the run that
// accumulates them; a change of unit rescales what is already stored.
static mcrt_status set_ssca_unit(mcrt_ctx *ctx, double unit, hipStream_t st) {
  if (!(unit > 0.0) || unit == ctx->ssca_unit) return MCRT_OK;
  uint64_t m = (uint64_t)ctx->nview * ctx->nimg * ctx->ncell;
  if (ctx->d_ssca && m) {
    double f = ctx->ssca_unit / unit;
    if (ctx->fp64) hipLaunchKernelGGL(k_scale<double>, dim3(4096), dim3(256), 0, st, (double *)ctx->d_ssca, f, m);
    else hipLaunchKernelGGL(k_scale<float>, dim3(4096), dim3(256), 0, st, (float *)ctx->d_ssca, f, m);
    HIPCHK(hipGetLastError());
  }
  if (ctx->d_sh && ctx->sh_have > 0) {
    uint64_t ms = (uint64_t)ctx->ncell * ctx->nimg * (uint64_t)(ctx->sh_have * ctx->sh_have);
    double f = ctx->ssca_unit / unit;
    if (ctx->fp64) hipLaunchKernelGGL(k_scale<double>, dim3(4096), dim3(256), 0, st, (double *)ctx->d_sh, f, ms);
    else hipLaunchKernelGGL(k_scale<float>, dim3(4096), dim3(256), 0, st, (float *)ctx->d_sh, f, ms);
    HIPCHK(hipGetLastError());
  }
  ctx->ssca_unit = unit;
  return MCRT_OK;
}

static mcrt_status prepare_run(mcrt_ctx *ctx, const mcrt_run_opts *o, uint64_t n, hipStream_t st) {
  mcrt_status s = ready(ctx);
  if (s) return s;
  s = check_opts(ctx, o);
  if (s) return s;
  HIPCHK(hipSetDevice(ctx->device));
  s = ensure_state(ctx, st);
  if (s) return s;
  s = ensure_ssca(ctx);
  if (s) return s;
  if (o->sed_theta_bins != ctx->ntheta || !ctx->d_sed) {
    ctx->ntheta = o->sed_theta_bins;
    s = ensure_sed(ctx, ctx->ntheta);
    if (s) return s;
    HIPCHK(fill<uint64_t>(ctx->d_sed, 0ull, (uint64_t)ctx->sed_cap, st));
  }
  s = ensure_sh(ctx, o->sh_order, st);
  if (s) return s;
  if (fast_mode(ctx, o) == 2) {
    s = ensure_mrw_flags(ctx);
    if (s) return s;
  }
  uint64_t nt = o->n_total ? o->n_total : n;
  if (nt == 0) return fail(ctx, MCRT_EINVAL, "n_total is 0");
  ctx->n_total = nt;
  ctx->xi = ctx->ltot / (double)nt;
  s = set_ssca_unit(ctx, ctx->xi, st);
  if (s) return s;
  HIPCHK(fill<unsigned long long>(ctx->d_stats, 0ull, NSTAT, st));
  ctx->t_phase[0] = ctx->t_phase[1] = ctx->t_phase[2] = 0.0;
  ctx->n_rounds = 0;
  ctx->pev_used = 0;
  return MCRT_OK;
}

static mcrt_status ensure_records(mcrt_ctx *ctx, uint64_t n) {
  size_t need = (size_t)n * sizeof(mcrt_packet_record);
  if (ctx->rec_cap < need) {
    ctx->rec_cap = 0;
    HIPCHK(dev_alloc(&ctx->d_rec, need));
    ctx->rec_cap = need;
  }
  ctx->rec_n = n;
  return MCRT_OK;
}

extern "C" mcrt_status mcrt_run_packets(mcrt_ctx *ctx, uint64_t first, uint64_t n, uint64_t seed,
                                        const mcrt_run_opts *opts, mcrt_run_stats *stats,
                                        void *stream) {
  hipStream_t st = (hipStream_t)stream;
  mcrt_status s = prepare_run(ctx, opts, n, st);
  if (s) return s;
  if (first + n > (1ull << 48)) return fail(ctx, MCRT_EINVAL, "packet ids must stay below 2^48");
  if (opts->record) {
    s = ensure_records(ctx, n);
    if (s) return s;
  }
  s = ensure_queues(ctx, opts, opts->mode == MCRT_BW_EPOCH && opts->epoch_packets < n ? opts->epoch_packets : n);
  if (s) return s;
  ModelDev &M = ctx->h_model;
  fill_model(ctx, M, opts, 0);
  M.seed = seed;
  M.rec = opts->record ? ctx->d_rec : nullptr;
  M.first = first;
  M.n = n;
  M.id_base = 0;
  M.rec_first = first;
  HIPCHK(hipEventRecord(ctx->ev0, st));
  if (opts->mode == MCRT_FROZEN) {
    for (int it = 0; it < opts->n_iter; ++it) {
      s = zero_tallies(ctx, st);
      if (s) return s;
      M.iter = it;
      HIPCHK(stage_copy(ctx, ctx->d_model, &M, sizeof M, st));
      s = set_range(ctx, first, n, st);
      if (s) return s;
      s = transport_launch(ctx, opts, n, st);
      if (s) return s;
      HIPCHK(launch_finalize_T(ctx->d_model, ctx->fp64, ctx->d_T, nullptr, st));
    }
  } else {
    HIPCHK(stage_copy(ctx, ctx->d_model, &M, sizeof M, st));
    if (opts->mode == MCRT_BW_TICKET) {
      s = set_range(ctx, first, n, st);
      if (s) return s;
      s = transport_launch(ctx, opts, n, st);
      if (s) return s;
    } else {
      const uint64_t P = opts->epoch_packets;
      uint64_t a = first, end = first + n;
      while (a < end) {
        uint64_t b = (a / P + 1) * P;
        if (b > end) b = end;
        if (ctx->snap_stale) {
          HIPCHK(fill<uint8_t>(ctx->d_dirty, (uint8_t)1, ctx->ncell, st));
          ctx->snap_stale = false;
        }
        HIPCHK(launch_epoch_snapshot(ctx->d_model, st));
        s = set_range(ctx, a, b - a, st);
        if (s) return s;
        s = transport_launch(ctx, opts, b - a, st);
        if (s) return s;
        a = b;
      }
    }
  }
  HIPCHK(hipEventRecord(ctx->ev1, st));
  ctx->S_ok = false;
  ctx->err.clear();
  if (stats) return read_stats(ctx, stats, st);
  return MCRT_OK;
}

__global__ void k_u32_to_u64(const uint32_t *a, uint64_t *b, uint64_t n) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) b[i] = a[i];
}

extern "C" mcrt_status mcrt_run_pah(mcrt_ctx *ctx, uint64_t seed, const mcrt_run_opts *opts,
                                    mcrt_run_stats *stats, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  if (ctx && ctx->pah < 0) return fail(ctx, MCRT_ESTATE, "no PAH species");
  if (ctx && ctx->n_total == 0) return fail(ctx, MCRT_ESTATE, "run_packets before run_pah");
  if (opts && opts->n_total && ctx && opts->n_total != ctx->n_total)
    return fail(ctx, MCRT_EINVAL, "n_total differs from the source pass");
  uint64_t nt = ctx ? ctx->n_total : 0;
  mcrt_run_opts o2 = opts ? *opts : mcrt_run_opts{};
  o2.n_total = nt;
  mcrt_status s = prepare_run(ctx, &o2, nt, st);
  if (s) return s;
  // exclusive prefix of the pass-1 PAH counts (u64)
  const uint64_t nc = ctx->ncell;
  hipLaunchKernelGGL(k_u32_to_u64, dim3(4096), dim3(256), 0, st, ctx->d_kpah, (uint64_t *)ctx->d_tmp, nc);
  HIPCHK(hipGetLastError());
  size_t tb = 0;
  HIPCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, (uint64_t *)ctx->d_tmp, ctx->d_prefix, (int)nc, st));
  if (tb > ctx->temp_cap) {
    ctx->temp_cap = 0;
    HIPCHK(dev_alloc(&ctx->d_temp, tb));
    ctx->temp_cap = tb;
  }
  HIPCHK(hipcub::DeviceScan::ExclusiveSum(ctx->d_temp, tb, (uint64_t *)ctx->d_tmp, ctx->d_prefix, (int)nc, st));
  uint64_t last[2];
  HIPCHK(hipMemcpyAsync(&last[0], ctx->d_prefix + nc - 1, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&last[1], (uint64_t *)ctx->d_tmp + nc - 1, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const uint64_t total = last[0] + last[1];
  if (o2.record) {
    s = ensure_records(ctx, total);
    if (s) return s;
  }
  s = ensure_queues(ctx, &o2, o2.mode == MCRT_BW_EPOCH && o2.epoch_packets < total ? o2.epoch_packets : total);
  if (s) return s;
  ModelDev &M = ctx->h_model;
  fill_model(ctx, M, &o2, 0);
  M.seed = seed;
  M.pass = 2;
  M.id_base = nt;
  M.rec_first = 0;
  M.rec = o2.record ? ctx->d_rec : nullptr;
  HIPCHK(hipEventRecord(ctx->ev0, st));
  HIPCHK(stage_copy(ctx, ctx->d_model, &M, sizeof M, st));
  if (total > 0) {
    if (o2.mode == MCRT_BW_EPOCH) {
      const uint64_t P = o2.epoch_packets;
      for (uint64_t a = 0; a < total;) {
        uint64_t b = (a / P + 1) * P;
        if (b > total) b = total;
        if (ctx->snap_stale) {
          HIPCHK(fill<uint8_t>(ctx->d_dirty, (uint8_t)1, ctx->ncell, st));
          ctx->snap_stale = false;
        }
        HIPCHK(launch_epoch_snapshot(ctx->d_model, st));
        s = set_range(ctx, a, b - a, st);
        if (s) return s;
        s = transport_launch(ctx, &o2, b - a, st);
        if (s) return s;
        a = b;
      }
    } else {
      s = set_range(ctx, 0, total, st);
      if (s) return s;
      s = transport_launch(ctx, &o2, total, st);
      if (s) return s;
    }
  }
  HIPCHK(hipEventRecord(ctx->ev1, st));
  ctx->S_ok = false;
  if (stats) return read_stats(ctx, stats, st);
  return MCRT_OK;
}

// ---------------------------------------------------------------- outputs

static mcrt_status to_caller(mcrt_ctx *ctx, void *dst, const void *src, size_t bytes, int mem,
                             hipStream_t st) {
  if (!dst) return MCRT_OK;
  if (mem == MCRT_DEVICE) {
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st));
  } else {
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  return MCRT_OK;
}

static mcrt_status upload_model_only(mcrt_ctx *ctx, hipStream_t st) {
  fill_model(ctx, ctx->h_model, nullptr, 0);
  HIPCHK(stage_copy(ctx, ctx->d_model, &ctx->h_model, sizeof(ModelDev), st));
  return MCRT_OK;
}

extern "C" mcrt_status mcrt_reset(mcrt_ctx *ctx, void *stream) {
  mcrt_status s = ready(ctx);
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device));
  s = ensure_state(ctx, st);
  if (s) return s;
  s = ensure_ssca(ctx);
  if (s) return s;
  s = ensure_sed(ctx, ctx->ntheta);
  if (s) return s;
  s = zero_tallies(ctx, st);
  if (s) return s;
  return zero_epoch(ctx, st);
}

extern "C" mcrt_status mcrt_init_temperatures(mcrt_ctx *ctx, void *stream) {
  mcrt_status s = ready(ctx);
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device));
  s = ensure_state(ctx, st);
  if (s) return s;
  s = upload_model_only(ctx, st);
  if (s) return s;
  HIPCHK(launch_init_T(ctx->d_model, ctx->fp64, ctx->d_T, st));
  ctx->S_ok = false;
  return MCRT_OK;
}

extern "C" mcrt_status mcrt_set_temperatures(mcrt_ctx *ctx, const double *T, int mem, void *stream) {
  if (!ctx) return MCRT_EINVAL;
  if (!ctx->has_grid || !ctx->has_dust) return fail(ctx, MCRT_ESTATE, "grid and dust must be set");
  if (!T) return fail(ctx, MCRT_EINVAL, "T is NULL");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device));
  mcrt_status s = ensure_state(ctx, st);
  if (s) return s;
  size_t bytes = ctx->ncell * (size_t)ctx->ns * 8;
  HIPCHK(hipMemcpyAsync(ctx->d_T, T, bytes, mem == MCRT_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  if (mem != MCRT_DEVICE) HIPCHK(hipStreamSynchronize(st));
  ctx->S_ok = false;
  return MCRT_OK;
}

__global__ void k_d2f(const double *a, float *b, uint64_t n) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) b[i] = (float)a[i];
}
// Scattering sums from the device layout [cell][view][img] (in units of
// `unit`) to the API layout [view][img][cell] in erg/s/sr.
template <typename R>
__global__ void k_ssca_out(const R *a, double *b, double unit, int nview, uint64_t ncell,
                           int nq) {
  const uint64_t n = (uint64_t)nview * nq * ncell;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    const uint64_t c = i % ncell, r = i / ncell;
    const uint64_t q = r % (uint64_t)nq, v = r / (uint64_t)nq;
    b[i] = (double)a[(c * (uint64_t)nview + v) * (uint64_t)nq + q] * unit;
  }
}

extern "C" mcrt_status mcrt_set_scattering(mcrt_ctx *ctx, const double *ssca, int mem, void *stream) {
  if (!ctx) return MCRT_EINVAL;
  if (!ctx->has_grid || !ctx->has_dust) return fail(ctx, MCRT_ESTATE, "grid and dust must be set");
  if (!ssca) return fail(ctx, MCRT_EINVAL, "ssca is NULL");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device));
  mcrt_status s = ensure_ssca(ctx);
  if (s) return s;
  uint64_t m = (uint64_t)ctx->nview * ctx->nimg * ctx->ncell;
  if (m == 0) return MCRT_OK;
  std::vector<double> h(m);
  if (mem == MCRT_DEVICE) {
    HIPCHK(hipMemcpyAsync(h.data(), ssca, m * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  } else {
    memcpy(h.data(), ssca, m * 8);
  }
  double mx = 0.0;
  for (uint64_t i = 0; i < m; ++i) {
    if (!finite_nonneg(h[i])) return fail(ctx, MCRT_EINVAL, "scattering sums must be finite and >= 0");
    if (h[i] > mx) mx = h[i];
  }
  // store in units that keep the largest value near 2^20, in the device
  // layout [cell][view][img]
  double unit = mx > 0.0 ? mx / 1048576.0 : 1.0;
  const uint64_t nc = ctx->ncell, nq = (uint64_t)ctx->nimg, nv = (uint64_t)ctx->nview;
  auto dev_index = [&](uint64_t i) {  // API index [view][img][cell] -> device index
    const uint64_t c = i % nc, r = i / nc;
    return (c * nv + r / nq) * nq + r % nq;
  };
  if (ctx->fp64) {
    std::vector<double> d(m);
    for (uint64_t i = 0; i < m; ++i) d[dev_index(i)] = h[i] / unit;
    HIPCHK(hipMemcpy(ctx->d_ssca, d.data(), m * 8, hipMemcpyHostToDevice));
  } else {
    std::vector<float> f(m);
    for (uint64_t i = 0; i < m; ++i) f[dev_index(i)] = (float)(h[i] / unit);
    HIPCHK(hipMemcpy(ctx->d_ssca, f.data(), m * 4, hipMemcpyHostToDevice));
  }
  ctx->ssca_unit = unit;
  ctx->S_ok = false;
  return MCRT_OK;
}

extern "C" mcrt_status mcrt_temperatures(mcrt_ctx *ctx, double *T_out, double *E_out, int mem,
                                         void *stream) {
  mcrt_status s = ready(ctx);
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device));
  if (!ctx->d_k) return fail(ctx, MCRT_ESTATE, "no tallies");
  fill_model(ctx, ctx->h_model, nullptr, 0);
  HIPCHK(stage_copy(ctx, ctx->d_model, &ctx->h_model, sizeof(ModelDev), st));
  HIPCHK(launch_finalize_T(ctx->d_model, ctx->fp64, ctx->d_T, ctx->d_tmp, st));
  size_t bytes = ctx->ncell * (size_t)ctx->ns * 8;
  s = to_caller(ctx, T_out, ctx->d_T, bytes, mem, st);
  if (s) return s;
  s = to_caller(ctx, E_out, ctx->d_tmp, bytes, mem, st);
  if (s) return s;
  ctx->S_ok = false;
  return MCRT_OK;
}

__global__ void k_invert(const double *tab, const double *herm, int nl, int ns, int nsrc, int nrows,
                         int s, uint64_t n, const double *rhs, double *T, int method) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  TabOff o = tab_offsets(nl, ns, nsrc, nrows);
  bool cl = false;
  T[i] = method == 1 ? invert_T_fast(herm, tab, o, nl, s, rhs[i], &cl)
                     : invert_T(tab, o, nl, s, rhs[i], &cl);
}

extern "C" mcrt_status mcrt_invert_temperature(mcrt_ctx *ctx, int species, uint64_t n,
                                               const double *rhs, double *T_out, int method) {
  mcrt_status s = ready(ctx);
  if (s) return s;
  if (species < 0 || species >= ctx->ns) return fail(ctx, MCRT_EINVAL, "bad species");
  if (!rhs || !T_out) return fail(ctx, MCRT_EINVAL, "NULL array");
  if (method != 0 && method != 1) return fail(ctx, MCRT_EINVAL, "method must be 0 or 1");
  if (n == 0) return MCRT_OK;
  HIPCHK(hipSetDevice(ctx->device));
  double *d = nullptr;
  HIPCHK(hipMalloc((void **)&d, n * 16));
  HIPCHK(hipMemcpy(d, rhs, n * 8, hipMemcpyHostToDevice));
  hipLaunchKernelGGL(k_invert, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, 0, ctx->d_tab,
                     ctx->d_herm, ctx->nl, ctx->ns, ctx->nsrc, ctx->nrows, species, n, d, d + n,
                     method);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpy(T_out, d + n, n * 8, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(ctx, MCRT_EDEVICE, "invert: %s", hipGetErrorString(e));
  return MCRT_OK;
}

extern "C" mcrt_status mcrt_get_temperatures(mcrt_ctx *ctx, double *T_out, int mem, void *stream) {
  if (!ctx) return MCRT_EINVAL;
  if (!ctx->d_T) return fail(ctx, MCRT_ESTATE, "no temperature field yet");
  if (!T_out) return fail(ctx, MCRT_EINVAL, "T_out is NULL");
  return to_caller(ctx, T_out, ctx->d_T, ctx->ncell * (size_t)ctx->ns * 8, mem, (hipStream_t)stream);
}

extern "C" mcrt_status mcrt_density(mcrt_ctx *ctx, void *rho_out, int mem, void *stream) {
  if (!ctx) return MCRT_EINVAL;
  if (!ctx->has_grid) return fail(ctx, MCRT_ESTATE, "grid not set");
  if (!rho_out) return fail(ctx, MCRT_EINVAL, "rho_out is NULL");
  return to_caller(ctx, rho_out, ctx->d_rho, ctx->ncell * rsize(ctx), mem, (hipStream_t)stream);
}

extern "C" mcrt_status mcrt_tallies(mcrt_ctx *ctx, uint64_t *k_out, double *epath_out,
                                    uint32_t *kpah_out, int mem, void *stream) {
  mcrt_status s = ready(ctx);
  if (s) return s;
  if (!ctx->d_k) return fail(ctx, MCRT_ESTATE, "no tallies");
  hipStream_t st = (hipStream_t)stream;
  size_t b = ctx->ncell * (size_t)ctx->ns * 8;
  s = to_caller(ctx, k_out, ctx->d_k, b, mem, st);
  if (s) return s;
  s = to_caller(ctx, epath_out, ctx->d_epath, b, mem, st);
  if (s) return s;
  return to_caller(ctx, kpah_out, ctx->d_kpah, ctx->ncell * 4, mem, st);
}

__global__ void k_sed_flux(const uint64_t *cnt, const double *w, int nl, int nt, double xi,
                           double D2, double *out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nl * nt) return;
  int j = i % nl;
  double dOmega = 4.0 * PI_D / (double)nt;
  out[i] = (double)cnt[i] * xi / (dOmega * D2 * w[j]);
}

extern "C" mcrt_status mcrt_sed(mcrt_ctx *ctx, double *sed_out, uint64_t *counts_out, int mem,
                                void *stream) {
  mcrt_status s = ready(ctx);
  if (s) return s;
  if (!ctx->d_sed) return fail(ctx, MCRT_ESTATE, "no SED yet");
  hipStream_t st = (hipStream_t)stream;
  int n = ctx->ntheta * ctx->nl;
  if (sed_out) {
    if (ctx->sed_tmp_cap < (size_t)n * 8) {
      ctx->sed_tmp_cap = 0;
      HIPCHK(dev_alloc((void **)&ctx->d_sed_tmp, (size_t)n * 8));
      ctx->sed_tmp_cap = (size_t)n * 8;
    }
    TabOff o = tab_offsets(ctx->nl, ctx->ns, ctx->nsrc, ctx->nrows);
    hipLaunchKernelGGL(k_sed_flux, dim3((n + 255) / 256), dim3(256), 0, st, ctx->d_sed,
                       ctx->d_tab + o.w, ctx->nl, ctx->ntheta, ctx->xi,
                       ctx->distance * ctx->distance, ctx->d_sed_tmp);
    HIPCHK(hipGetLastError());
    s = to_caller(ctx, sed_out, ctx->d_sed_tmp, (size_t)n * 8, mem, st);
    if (s) return s;
  }
  return to_caller(ctx, counts_out, ctx->d_sed, (size_t)n * 8, mem, st);
}

extern "C" mcrt_status mcrt_scattering(mcrt_ctx *ctx, double *ssca_out, int mem, void *stream) {
  mcrt_status s = ready(ctx);
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  uint64_t m = (uint64_t)ctx->nview * ctx->nimg * ctx->ncell;
  if (m == 0 || !ssca_out) return MCRT_OK;
  double *tmp = nullptr;
  HIPCHK(hipMalloc((void **)&tmp, m * 8));
  if (ctx->fp64)
    hipLaunchKernelGGL(k_ssca_out<double>, dim3(4096), dim3(256), 0, st,
                       (const double *)ctx->d_ssca, tmp, ctx->ssca_unit, ctx->nview, ctx->ncell,
                       ctx->nimg);
  else
    hipLaunchKernelGGL(k_ssca_out<float>, dim3(4096), dim3(256), 0, st,
                       (const float *)ctx->d_ssca, tmp, ctx->ssca_unit, ctx->nview, ctx->ncell,
                       ctx->nimg);
  HIPCHK(hipGetLastError());
  s = to_caller(ctx, ssca_out, tmp, m * 8, mem, st);
  HIPCHK(hipStreamSynchronize(st));
  (void)hipFree(tmp);
  return s;
}

extern "C" mcrt_status mcrt_packet_records(mcrt_ctx *ctx, mcrt_packet_record *out, uint64_t n, int mem) {
  if (!ctx) return MCRT_EINVAL;
  if (!out) return fail(ctx, MCRT_EINVAL, "out is NULL");
  if (!ctx->d_rec || ctx->rec_n == 0) return fail(ctx, MCRT_ESTATE, "no records (run with record = 1)");
  uint64_t m = n < ctx->rec_n ? n : ctx->rec_n;
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(out, ctx->d_rec, m * sizeof(mcrt_packet_record),
                   mem == MCRT_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
  return MCRT_OK;
}

// ------------------------------------------------------------- ray-tracer

static mcrt_status rt_check(mcrt_ctx *ctx, int npx, int npy) {
  mcrt_status s = ready(ctx);
  if (s) return s;
  if (ctx->nview < 1 || ctx->nimg < 1) return fail(ctx, MCRT_ESTATE, "set_views before ray-tracing");
  if (npx < 1 || npy < 1 || (uint64_t)npx * npy > (1ull << 28)) return fail(ctx, MCRT_EINVAL, "bad image size");
  return MCRT_OK;
}

// Ray-tracer arguments (frames of every view, extinction and point-source
// terms of the imaged wavelengths) with the source functions at S, staged
// to ctx->d_rt on stream st.
static mcrt_status rt_args(mcrt_ctx *ctx, int npx, int npy, const void *rho_rt, const void *S,
                           hipStream_t st, RtArgs &A) {
  const int nq = ctx->nimg;
  memset(&A, 0, sizeof A);
  A.nx = ctx->nx; A.ny = ctx->ny; A.nz = ctx->nz; A.nimg = nq; A.npx = npx; A.npy = npy;
  A.nview = ctx->nview; A.nsrc = ctx->nsrc;
  for (int k = 0; k < 3; ++k) A.origin[k] = ctx->origin[k];
  A.dcell = ctx->dcell;
  A.ncell = ctx->ncell;
  A.ncube = ctx->ncube;
  A.ref = ctx->nsub > 0 ? ctx->d_ref : nullptr;
  A.sub_off = ctx->nsub > 0 ? ctx->d_suboff : nullptr;
  A.rho = rho_rt ? rho_rt : ctx->d_rho;
  A.S = S;
  TabOff o = tab_offsets(ctx->nl, ctx->ns, ctx->nsrc, ctx->nrows);
  A.lit = ctx->rt_mode == MCRT_RT_ABS_LITERAL ? 1 : 0;
  for (int q = 0; q < nq; ++q) {
    int j = ctx->img_idx[q];
    if (A.lit) {
      // absorption of the whole mixture, summed in species order
      double k = 0.0;
      for (int s2 = 0; s2 < ctx->ns; ++s2)
        k += ctx->h_tab[o.frac + s2] * ctx->h_tab[o.kabs + s2 * ctx->nl + j];
      A.kext[q] = k;
    } else {
      A.kext[q] = ctx->h_tab[o.kext + j];
    }
    for (int s2 = 0; s2 < ctx->nsrc; ++s2) A.lnu[s2][q] = ctx->src_lnu[s2 * ctx->nl + j];
  }
  for (int s2 = 0; s2 < ctx->nsrc; ++s2)
    for (int k = 0; k < 3; ++k) A.srcpos[s2][k] = ctx->src_pos[3 * s2 + k];
  A.D2 = ctx->distance * ctx->distance;
  int n[3] = {ctx->nx, ctx->ny, ctx->nz};
  double L = 0.0, ctr[3];
  for (int k = 0; k < 3; ++k) {
    ctr[k] = ctx->origin[k] + 0.5 * (double)n[k] * ctx->dcell;
    if ((double)n[k] * ctx->dcell > L) L = (double)n[k] * ctx->dcell;
  }
  for (int v = 0; v < ctx->nview; ++v) {
    RtView &V = A.v[v];
    double th = ctx->views[2 * v] * PI_D / 180.0, ph = ctx->views[2 * v + 1] * PI_D / 180.0;
    V.k[0] = std::sin(th) * std::cos(ph); V.k[1] = std::sin(th) * std::sin(ph); V.k[2] = std::cos(th);
    V.ex[0] = std::cos(th) * std::cos(ph); V.ex[1] = std::cos(th) * std::sin(ph); V.ex[2] = -std::sin(th);
    V.ey[0] = -std::sin(ph); V.ey[1] = std::cos(ph); V.ey[2] = 0.0;
    for (int k = 0; k < 3; ++k) V.ctr[k] = ctr[k];
    V.fov = std::sqrt(3.0) * L;
    V.dpx = V.fov / (double)npx;
    V.dpy = V.fov / (double)npy;
    V.apix_d2 = V.dpx * V.dpy / A.D2;
  }
  HIPCHK(stage_copy(ctx, ctx->d_rt, &A, sizeof A, st));
  return MCRT_OK;
}

static mcrt_status rt_prepare(mcrt_ctx *ctx, int npx, int npy, const void *rho_rt, hipStream_t st,
                              RtArgs &A) {
  mcrt_status s = rt_check(ctx, npx, npy);
  if (s) return s;
  HIPCHK(hipSetDevice(ctx->device));
  s = ensure_state(ctx, st);
  if (s) return s;
  s = ensure_ssca(ctx);
  if (s) return s;
  if (!ctx->S_ok) {
    size_t need = (size_t)ctx->nview * ctx->ncell * ctx->nimg * rsize(ctx);
    if (need > ctx->S_cap) {
      ctx->S_cap = 0;
      HIPCHK(dev_alloc(&ctx->d_S, need));
      ctx->S_cap = need;
    }
    s = upload_model_only(ctx, st);
    if (s) return s;
    HIPCHK(hipEventRecord(ctx->evs0, st));
    HIPCHK(launch_build_S(ctx->d_model, ctx->fp64, rt_lit(ctx), sh_read(ctx) > 0, ctx->d_S, st));
    HIPCHK(hipEventRecord(ctx->evs1, st));
    ctx->have_s = true;
    ctx->S_ok = true;
  }
  return rt_args(ctx, npx, npy, rho_rt, ctx->d_S, st, A);
}

extern "C" mcrt_status mcrt_raytrace_image(mcrt_ctx *ctx, int npx, int npy, const void *rho_rt,
                                           void *img_out, double *sed_out, int mem, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  RtArgs A;
  mcrt_status s = rt_prepare(ctx, npx, npy, rho_rt, st, A);
  if (s) return s;
  size_t ib = (size_t)ctx->nview * ctx->nimg * npx * npy * rsize(ctx);
  void *img = img_out;
  if (!img_out || mem != MCRT_DEVICE) {
    if (ib > ctx->img_cap) {
      ctx->img_cap = 0;
      HIPCHK(dev_alloc(&ctx->d_img_tmp, ib));
      ctx->img_cap = ib;
    }
    img = ctx->d_img_tmp;
  }
  double *sed = nullptr;
  size_t sb = (size_t)ctx->nview * ctx->nimg * 8;
  if (sed_out) {
    if (ctx->sed_tmp_cap < sb) {
      ctx->sed_tmp_cap = 0;
      HIPCHK(dev_alloc((void **)&ctx->d_sed_tmp, sb));
      ctx->sed_tmp_cap = sb;
    }
    sed = (mem == MCRT_DEVICE) ? sed_out : ctx->d_sed_tmp;
  }
  HIPCHK(hipEventRecord(ctx->evf0, st));
  HIPCHK(launch_rt_fwd(ctx->d_rt, A, ctx->fp64, img, sed, ctx->evf1, st));
  ctx->have_f = true;
  if (mem != MCRT_DEVICE) {
    if (img_out) HIPCHK(hipMemcpyAsync(img_out, img, ib, hipMemcpyDeviceToHost, st));
    if (sed_out) HIPCHK(hipMemcpyAsync(sed_out, sed, sb, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  return MCRT_OK;
}

extern "C" mcrt_status mcrt_set_raytrace_mode(mcrt_ctx *ctx, int rt_mode) {
  if (!ctx) return MCRT_EINVAL;
  if (rt_mode != MCRT_RT_EXT && rt_mode != MCRT_RT_ABS_LITERAL)
    return fail(ctx, MCRT_EINVAL, "rt_mode must be MCRT_RT_EXT or MCRT_RT_ABS_LITERAL");
  if (rt_mode != ctx->rt_mode) ctx->S_ok = false;
  ctx->rt_mode = rt_mode;
  return MCRT_OK;
}

extern "C" mcrt_status mcrt_set_scattering_law(mcrt_ctx *ctx, int law) {
  if (!ctx) return MCRT_EINVAL;
  if (law != MCRT_SCAT_HG && law != MCRT_SCAT_GFACTOR)
    return fail(ctx, MCRT_EINVAL, "law must be MCRT_SCAT_HG or MCRT_SCAT_GFACTOR");
  if (law == ctx->scat_law) return MCRT_OK;
  ctx->scat_law = law;
  ctx->S_ok = false;
  if (ctx->tables_ok) {
    HIPCHK(hipSetDevice(ctx->device));
    mcrt_status s = build_tables(ctx);
    if (s) return s;
    HIPCHK(hipDeviceSynchronize());
  }
  return MCRT_OK;
}

extern "C" mcrt_status mcrt_set_scattered_light(mcrt_ctx *ctx, int source) {
  if (!ctx) return MCRT_EINVAL;
  if (source != MCRT_SSCA_PEELOFF && source != MCRT_SSCA_MOMENTS)
    return fail(ctx, MCRT_EINVAL, "source must be MCRT_SSCA_PEELOFF or MCRT_SSCA_MOMENTS");
  ctx->ssca_src = source;
  ctx->S_ok = false;
  return MCRT_OK;
}

// Moments (units of ssca_unit, [cell][img][lm]) to the API layout
// [img][lm][cell] in erg/s.
template <typename R>
__global__ void k_sh_out(const R *a, double *b, double unit, uint64_t ncell, int nq, int nlm) {
  const uint64_t n = ncell * (uint64_t)nq * nlm;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    const uint64_t c = i % ncell, r = i / ncell;
    const uint64_t lm = r % (uint64_t)nlm, q = r / (uint64_t)nlm;
    b[i] = (double)a[(c * nq + q) * (uint64_t)nlm + lm] * unit;
  }
}

extern "C" mcrt_status mcrt_scattering_moments(mcrt_ctx *ctx, double *out, int *order, int mem,
                                               void *stream) {
  if (!ctx) return MCRT_EINVAL;
  if (order) *order = ctx->sh_have;
  if (!out) return MCRT_OK;
  if (ctx->sh_have <= 0 || !ctx->d_sh)
    return fail(ctx, MCRT_ESTATE, "no moments (run with sh_order > 0 and imaged wavelengths)");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device));
  const int nlm = ctx->sh_have * ctx->sh_have;
  uint64_t m = ctx->ncell * (uint64_t)ctx->nimg * nlm;
  double *tmp = nullptr;
  HIPCHK(hipMalloc((void **)&tmp, m * 8));
  if (ctx->fp64)
    hipLaunchKernelGGL(k_sh_out<double>, dim3(4096), dim3(256), 0, st, (const double *)ctx->d_sh,
                       tmp, ctx->ssca_unit, ctx->ncell, ctx->nimg, nlm);
  else
    hipLaunchKernelGGL(k_sh_out<float>, dim3(4096), dim3(256), 0, st, (const float *)ctx->d_sh,
                       tmp, ctx->ssca_unit, ctx->ncell, ctx->nimg, nlm);
  HIPCHK(hipGetLastError());
  mcrt_status s = to_caller(ctx, out, tmp, m * 8, mem, st);
  HIPCHK(hipStreamSynchronize(st));
  (void)hipFree(tmp);
  return s;
}

// ------------------------------------------- ray-tracing without allocation
// For callers that cannot allocate device memory (code under graph capture,
// serving loops): the source functions live in this file-scope array, one
// copy per GPU, held until the process ends. Host code reaches it only
// through the address hipGetSymbolAddress returns for the current device
// (g_scratch); the array's own name is a host-side stand-in.
static constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
static constexpr int SCRATCH_MAX_DEV = 64;
static void *g_scratch[SCRATCH_MAX_DEV];
static std::mutex g_scratch_mu;

// Called by mcrt_create with `device` current: resolves this device's copy
// of the array once.
static hipError_t scratch_init(int device) {
  if (device < 0 || device >= SCRATCH_MAX_DEV) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return hipSuccess;
  void *p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e;
  }
  g_scratch[device] = p;
  return hipSuccess;
}

extern "C" mcrt_status mcrt_raytrace_image_noalloc(mcrt_ctx *ctx, int npx, int npy,
                                                   const void *rho_rt, void *img_out,
                                                   double *sed_out, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  mcrt_status s = rt_check(ctx, npx, npy);
  if (s) return s;
  if (!img_out) return fail(ctx, MCRT_EINVAL, "img_out is NULL");
  if (!ctx->d_k || ctx->state_cells != ctx->ncell || ctx->state_ns != ctx->ns)
    return fail(ctx, MCRT_ESTATE, "no temperatures yet (run, reset or set_temperatures first)");
  size_t nsum = (size_t)ctx->nview * ctx->nimg * ctx->ncell * rsize(ctx);
  if (!ctx->d_ssca || ctx->ssca_cap != nsum)
    return fail(ctx, MCRT_ESTATE, "no scattering sums for these views (reset or run first)");
  size_t need = (size_t)ctx->nview * ctx->ncell * ctx->nimg * rsize(ctx);
  if (need > SCRATCH_BYTES)
    return fail(ctx, MCRT_EINVAL,
                "source functions need %zu bytes; the no-allocation ray-tracer holds %zu",
                need, SCRATCH_BYTES);
  void *S = (ctx->device < SCRATCH_MAX_DEV) ? g_scratch[ctx->device] : nullptr;
  if (!S) return fail(ctx, MCRT_EDEVICE, "no scratch address for device %d", ctx->device);
  HIPCHK(hipSetDevice(ctx->device));
  s = upload_model_only(ctx, st);
  if (s) return s;
  // every (view, cell, wavelength) entry is written: nothing to clear
  HIPCHK(launch_build_S(ctx->d_model, ctx->fp64, rt_lit(ctx), sh_read(ctx) > 0, S, st));
  RtArgs A;
  s = rt_args(ctx, npx, npy, rho_rt, S, st, A);
  if (s) return s;
  HIPCHK(launch_rt_fwd(ctx->d_rt, A, ctx->fp64, img_out, sed_out, nullptr, st));
  return MCRT_OK;
}

extern "C" mcrt_status mcrt_raytrace_adjoint(mcrt_ctx *ctx, int npx, int npy, const void *rho_rt,
                                             const void *dL_dimg, const double *dL_dsed,
                                             void *dL_drho, int mem, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  if (ctx && !dL_drho) return fail(ctx, MCRT_EINVAL, "dL_drho is NULL");
  RtArgs A;
  mcrt_status s = rt_prepare(ctx, npx, npy, rho_rt, st, A);
  if (s) return s;
  size_t ib = (size_t)ctx->nview * ctx->nimg * npx * npy * rsize(ctx);
  size_t sb = (size_t)ctx->nview * ctx->nimg * 8;
  size_t gb = ctx->ncell * rsize(ctx);
  const void *wimg = dL_dimg;
  const double *wsed = dL_dsed;
  void *grad = dL_drho;
  void *tmp_img = nullptr, *tmp_g = nullptr;
  double *tmp_sed = nullptr;
  if (mem != MCRT_DEVICE) {
    if (dL_dimg) {
      HIPCHK(hipMalloc(&tmp_img, ib));
      HIPCHK(hipMemcpyAsync(tmp_img, dL_dimg, ib, hipMemcpyHostToDevice, st));
      wimg = tmp_img;
    }
    if (dL_dsed) {
      HIPCHK(hipMalloc((void **)&tmp_sed, sb));
      HIPCHK(hipMemcpyAsync(tmp_sed, dL_dsed, sb, hipMemcpyHostToDevice, st));
      wsed = tmp_sed;
    }
    HIPCHK(hipMalloc(&tmp_g, gb));
    grad = tmp_g;
  }
  if (ctx->fp64) HIPCHK(fill<double>((double *)grad, 0.0, ctx->ncell, st));
  else HIPCHK(fill<float>((float *)grad, 0.0f, ctx->ncell, st));
  HIPCHK(hipEventRecord(ctx->eva0, st));
  HIPCHK(launch_rt_adj(ctx->d_rt, A, ctx->fp64, wimg, wsed, grad, ctx->eva1, st));
  ctx->have_a = true;
  if (mem != MCRT_DEVICE) {
    HIPCHK(hipMemcpyAsync(dL_drho, grad, gb, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (tmp_img) (void)hipFree(tmp_img);
    if (tmp_sed) (void)hipFree(tmp_sed);
    (void)hipFree(tmp_g);
  }
  return MCRT_OK;
}

static double event_ms(hipEvent_t a, hipEvent_t b) {
  if (hipEventSynchronize(b) != hipSuccess) return -1.0;
  float ms = 0.0f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return -1.0;
  return ms;
}

extern "C" mcrt_status mcrt_last_timings(const mcrt_ctx *ctx, double *transport_ms, double *rt_fwd_ms,
                                         double *rt_adj_ms) {
  if (!ctx) return MCRT_EINVAL;
  if (transport_ms) *transport_ms = ctx->t_transport;
  if (rt_fwd_ms) *rt_fwd_ms = ctx->have_f ? event_ms(ctx->evf0, ctx->evf1) : 0.0;
  if (rt_adj_ms) *rt_adj_ms = ctx->have_a ? event_ms(ctx->eva0, ctx->eva1) : 0.0;
  return MCRT_OK;
}

extern "C" mcrt_status mcrt_last_source_build_ms(const mcrt_ctx *ctx, double *ms) {
  if (!ctx || !ms) return MCRT_EINVAL;
  *ms = ctx->have_s ? event_ms(ctx->evs0, ctx->evs1) : 0.0;
  return MCRT_OK;
}

extern "C" mcrt_status mcrt_sample_reemission(mcrt_ctx *ctx, int species, int mode, double T,
                                              uint64_t n, uint64_t seed, uint64_t *counts) {
  mcrt_status s = ready(ctx);
  if (s) return s;
  if (species < 0 || species >= ctx->ns || species == ctx->pah)
    return fail(ctx, MCRT_EINVAL, "species must be a thermal species");
  if (mode < MCRT_FROZEN || mode > MCRT_BW_TICKET) return fail(ctx, MCRT_EINVAL, "bad mode");
  if (!(T > 0.0) || !std::isfinite(T)) return fail(ctx, MCRT_EINVAL, "T must be > 0");
  if (!counts) return fail(ctx, MCRT_EINVAL, "counts is NULL");
  size_t lds = transport_lds_bytes(ctx->nl, ctx->ns, ctx->nsrc, ctx->nrows, ctx->ntheta, ctx->fp64);
  if (lds > ctx->lds_max) return fail(ctx, MCRT_EINVAL, "tables exceed LDS");
  HIPCHK(hipSetDevice(ctx->device));
  mcrt_run_opts o{};
  o.mode = mode;
  o.sed_theta_bins = ctx->ntheta > 0 ? ctx->ntheta : 1;
  ModelDev M;
  fill_model(ctx, M, &o, 0);
  M.ntheta = o.sed_theta_bins;
  unsigned long long *d_counts = nullptr;
  HIPCHK(hipMalloc((void **)&d_counts, (size_t)ctx->nl * 8));
  hipError_t e = hipMemset(d_counts, 0, (size_t)ctx->nl * 8);
  if (e == hipSuccess) e = hipMemcpy(ctx->d_model, &M, sizeof M, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_sample_reem(ctx->d_model, ctx->fp64, species, T, n, seed, d_counts, lds, 0);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(counts, d_counts, (size_t)ctx->nl * 8, hipMemcpyDeviceToHost);
  (void)hipFree(d_counts);
  if (e != hipSuccess) return fail(ctx, MCRT_EDEVICE, "re-emission sampling: %s", hipGetErrorString(e));
  return MCRT_OK;
}

extern "C" mcrt_status mcrt_phase_timings(const mcrt_ctx *ctx, double *emit_ms, double *walk_ms,
                                          double *interact_ms, uint64_t *rounds) {
  if (!ctx) return MCRT_EINVAL;
  if (emit_ms) *emit_ms = ctx->t_phase[0];
  if (walk_ms) *walk_ms = ctx->t_phase[1];
  if (interact_ms) *interact_ms = ctx->t_phase[2];
  if (rounds) *rounds = ctx->n_rounds;
  return MCRT_OK;
}

// ------------------------------------------------------------------ batch

// Queue counters of every model of a batch back to the start of a launch.
__global__ void k_wf_reset(const ModelDev *models, int nmodels) {
  wf_zero(models[blockIdx.x].ctl);
}

extern "C" mcrt_status mcrt_run_batch(mcrt_ctx *const *models, int n_models,
                                      const uint64_t *n_packets, const uint64_t *seeds,
                                      const mcrt_run_opts *opts, mcrt_run_stats *stats,
                                      void *stream) {
  if (!models || n_models < 1 || !models[0]) return MCRT_EINVAL;
  mcrt_ctx *ctx = models[0];
  if (!n_packets || !seeds) return fail(ctx, MCRT_EINVAL, "NULL n_packets/seeds");
  if (n_models > 1024) return fail(ctx, MCRT_EINVAL, "at most 1024 models per batch");
  mcrt_status s = check_opts(ctx, opts);
  if (s) return s;
  if (opts->mode == MCRT_BW_EPOCH || (opts->mode == MCRT_FROZEN && opts->n_iter != 1))
    return fail(ctx, MCRT_EINVAL, "batch supports BW_TICKET and single-pass FROZEN");
  if (opts->record) return fail(ctx, MCRT_EINVAL, "records are not kept in batch mode");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipSetDevice(ctx->device));
  std::vector<ModelDev> hm(n_models);
  size_t lds = 0, lds_w = 0, lds_f = 0;
  bool idx32 = true;
  for (int m = 0; m < n_models; ++m) {
    mcrt_ctx *c = models[m];
    if (c && !idx32_ok(c)) idx32 = false;
    if (!c || c->device != ctx->device || c->fp64 != ctx->fp64)
      return fail(ctx, MCRT_EINVAL, "model %d: same device and precision required", m);
    s = prepare_run(c, opts, n_packets[m], st);
    if (s) return fail(ctx, s, "model %d: %s", m, c->err.c_str());
    s = ensure_queues(c, opts, n_packets[m]);
    if (s) return fail(ctx, s, "model %d: %s", m, c->err.c_str());
    fill_model(c, hm[m], opts, 0);  // same streams as the model's own run_packets
    hm[m].seed = seeds[m];
    hm[m].first = 0;
    hm[m].n = n_packets[m];
    size_t b = transport_lds_bytes(c->nl, c->ns, c->nsrc, c->nrows, c->ntheta, c->fp64);
    if (b > lds) lds = b;
    b = walk_lds_bytes(c->nl, c->ns, c->nsrc, c->nrows, c->ntheta, c->ow, c->fp64);
    if (b > lds_w) lds_w = b;
    b = transport_lds_bytes(c->nl, c->ns, c->nsrc, c->nrows, c->ntheta, c->fp64) +
        (size_t)c->ow * 4;
    if (b > lds_f) lds_f = b;
  }
  if (lds > ctx->lds_max || lds_w > ctx->lds_max)
    return fail(ctx, MCRT_EINVAL, "batch tables need %zu bytes of LDS (limit %zu)", lds > lds_w ? lds : lds_w, ctx->lds_max);
  if (n_models > ctx->batch_cap) {
    ctx->batch_cap = 0;
    HIPCHK(dev_alloc((void **)&ctx->d_batch, sizeof(ModelDev) * n_models));
    ctx->batch_cap = n_models;
  }
  if (sizeof(ModelDev) * n_models > STAGE_BYTES) return fail(ctx, MCRT_EINVAL, "too many models");
  HIPCHK(stage_copy(ctx, ctx->d_batch, hm.data(), sizeof(ModelDev) * n_models, st));
  for (int m = 0; m < n_models; ++m) {
    s = zero_tallies(models[m], st);
    if (s) return s;
    models[m]->snap_stale = true;
  }
  hipLaunchKernelGGL(k_wf_reset, dim3(n_models), dim3(256), 0, st, ctx->d_batch, n_models);
  HIPCHK(hipGetLastError());
  const int fast = fast_mode(ctx, opts);
  if (fast == 2) HIPCHK(launch_mrw_cand(ctx->d_batch, n_models, ctx->num_cu, st));
  const int gfull = ctx->num_cu * (opts->blocks_per_cu > 0 ? opts->blocks_per_cu : default_bpc(fast));
  const int gwalk = ctx->num_cu * (opts->walk_blocks_per_cu > 0 ? opts->walk_blocks_per_cu : 4);
  const bool per_cell = opts->tau_mode == MCRT_TAU_PER_CELL;
  bool refined = false;
  for (int m = 0; m < n_models; ++m) refined |= models[m]->nsub > 0;
  // ROUNDS wavefront rounds over every model of the batch and the count of
  // models still busy, captured once on the library's own stream and
  // replayed on the caller's until no model has packets left
  constexpr int ROUNDS = 8;
  uint32_t *d_busy = &ctx->d_ctl->busy;  // address arithmetic only
  uint32_t *d_left = &ctx->d_ctl->left;
  static_assert(offsetof(WfCtl, inq) == offsetof(WfCtl, busy) + 4 &&
                    offsetof(WfCtl, left) == offsetof(WfCtl, busy) + 8,
                "busy, inq and left are read back as one 12-byte copy");
  const uint32_t fin_max = (uint32_t)ctx->num_cu * 2u * 256u;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cs_ = ctx->cap_stream;
  HIPCHK(hipStreamBeginCapture(cs_, hipStreamCaptureModeThreadLocal));
  hipError_t le = hipSuccess;
  for (int r = 0; r < ROUNDS && le == hipSuccess; ++r)
    le = launch_wf_round(ctx->d_batch, n_models, ctx->fp64, false, r & 1, gfull, gwalk, lds, lds_w,
                         idx32, per_cell, refined, fast_mode(ctx, opts), nullptr, cs_);
  if (le == hipSuccess)
    le = launch_wf_busy(ctx->d_batch, n_models, (ROUNDS - 1) & 1, d_busy, d_left, cs_);
  hipError_t ce = hipStreamEndCapture(cs_, &graph);
  if (le != hipSuccess || ce != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(ctx, MCRT_EDEVICE, "graph capture failed: %s",
                hipGetErrorString(le != hipSuccess ? le : ce));
  }
  HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  HIPCHK(hipEventRecord(ctx->ev0, st));
  mcrt_status rs = MCRT_OK;
  for (uint64_t rep = 0;; ++rep) {
    hipError_t e = hipGraphLaunch(exec, st);
    // busy, inq, left
    if (e == hipSuccess) e = hipMemcpyAsync(&ctx->h_ctl->busy, d_busy, 12, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      rs = fail(ctx, MCRT_EDEVICE, "batch round: %s", hipGetErrorString(e));
      break;
    }
    if (ctx->h_ctl->busy == 0u) break;
    if (ctx->h_ctl->left <= fin_max && lds_f <= ctx->lds_max) {
      // every packet started and few left: the finishing kernel ends them
      e = launch_wf_finish(ctx->d_batch, n_models, ctx->fp64, false, ROUNDS & 1, gfull, lds_f,
                           idx32, per_cell, refined, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) rs = fail(ctx, MCRT_EDEVICE, "batch finish: %s", hipGetErrorString(e));
      break;
    }
    if (rep > (1ull << 30)) {
      rs = fail(ctx, MCRT_EDEVICE, "batch did not finish");
      break;
    }
  }
  (void)hipGraphExecDestroy(exec);
  (void)hipGraphDestroy(graph);
  if (rs) return rs;
  for (int m = 0; m < n_models; ++m)
    HIPCHK(launch_finalize_T(ctx->d_batch + m, ctx->fp64, models[m]->d_T, nullptr, st));
  HIPCHK(hipEventRecord(ctx->ev1, st));
  HIPCHK(hipStreamSynchronize(st));
  float ms = 0.0f;
  HIPCHK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  ctx->t_transport = ms;
  for (int m = 0; m < n_models; ++m) {
    models[m]->S_ok = false;
    if (stats) {
      unsigned long long h[NSTAT];
      mcrt_ctx *c = models[m];
      HIPCHK(hipMemcpy(h, c->d_stats, sizeof h, hipMemcpyDeviceToHost));
      mcrt_run_stats &o = stats[m];
      o.packets = h[0]; o.escaped = h[1]; o.killed = h[2]; o.pah_stopped = h[3];
      o.crossings = h[4]; o.scatters = h[5]; o.absorptions = h[6]; o.mrw_steps = h[7];
      o.lucy_deposits = h[8]; o.clamped_T = h[9]; o.kernel_ms = ms;
    }
  }
  return MCRT_OK;
}
