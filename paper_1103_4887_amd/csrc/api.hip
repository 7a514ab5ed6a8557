// C ABI of libpimc: argument checking, workspace, launch-shape choice.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "hmc.hpp"
#include "kernels.hpp"
#include "pimc.h"

struct pimc_ctx {
  int device = 0;
  uint32_t* err = nullptr;        // device word of deferred error bits
  double* partial = nullptr;      // field-kernel workspace
  size_t partial_cap = 0;         // in doubles
  int64_t* offsets = nullptr;     // batch offsets (device copy)
  int32_t* order = nullptr;       // batch launch order (device)
  int8_t* blockK = nullptr;       // batch: sites per thread of each block (device)
  int blockK_NT = 0;              // workgroup size blockK was computed for (0: none)
  bool uniform_batch_K = false;   // every window of a batch with the launch's sites per thread
  size_t batch_cap = 0;           // in windows
  int tile_K = 0;                 // 0 = automatic choice of sites per thread
  int tiles = 0;                  // 0 = automatic number of time tiles per window
  bool no_graphs = false;         // launch HMC proposals one kernel at a time
  hipStream_t cap = nullptr;      // private stream that only records graphs (never runs work)
  // batch layout last copied to the device (the copy and its wait are
  // skipped when a call brings the same windows)
  std::vector<int64_t> last_offsets;
  // captured graph of the batched sweep launch, replayed with new arguments
  struct BatchGraph {
    bool valid = false;
    bool fp64 = false, dbg = false;
    int ext = 0;
    int K = 0, NT = 0, nblocks = 0, stage = 0;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    hipGraphNode_t node = nullptr;
  } bgraph;
  // cross-tile workspace: tile_cap tiles over group_cap windows (grow-only)
  size_t tile_cap = 0, group_cap = 0;
  void* halo = nullptr;
  double* wpart = nullptr;
  uint64_t* tsync = nullptr;
  uint64_t spin_ticks = 0;
  // exchange generations: a tiled call uses gen_next + 1 .. gen_next + n + 2
  // and moves gen_next past them, so words left by earlier calls are always
  // older than anything a later call waits for
  uint64_t gen_next = 0;
  // HMC workspace (grow-only)
  size_t hmc_sites = 0, hmc_blocks = 0, hmc_B = 0, hmc_tsize = 0;
  void* hQ1 = nullptr;
  void* hR0 = nullptr;
  void* hR1 = nullptr;
  void* hX0 = nullptr;
  double* hpart = nullptr;
  double* hp0 = nullptr;
  double* hpbuf = nullptr;
  double* hrpbuf = nullptr;
  double* hH0 = nullptr;
  double* hdH = nullptr;
  uint32_t* hout = nullptr;
  uint8_t* hacc = nullptr;
  int64_t* hoff = nullptr;
  int32_t* hbmap = nullptr;
  int32_t* hbfirst = nullptr;
  uint64_t* hk = nullptr;
};

namespace {

using pimc::ModelArgs;

int hip_ok(hipError_t e) { return e == hipSuccess ? PIMC_OK : PIMC_ERR_HIP; }

// STATES, PARAMS and/or KINETIC, and GIBBS only together with PARAMS
bool valid_flags(int32_t f) {
  if (f & ~(PIMC_STATES | PIMC_PARAMS | PIMC_GIBBS | PIMC_KINETIC)) return false;
  if (!(f & (PIMC_STATES | PIMC_PARAMS | PIMC_KINETIC))) return false;
  return !(f & PIMC_GIBBS) || (f & PIMC_PARAMS);
}

int model_args(const pimc_model* m, ModelArgs& a) {
  if (!m) return PIMC_ERR_ARG;
  if (!(m->dt > 0.0) || !(m->Ro >= 0.0) || !(m->beta >= 0.0)) return PIMC_ERR_ARG;
  for (int c = 0; c < 4; ++c)
    if (!(m->Rd[c] >= 0.0) || !(m->x_lo[c] <= m->x_hi[c])) return PIMC_ERR_ARG;
  for (int l = 0; l < 7; ++l)
    if (!(m->p_lo[l] <= m->p_hi[l])) return PIMC_ERR_ARG;
  for (int g = 0; g < 3; ++g)
    if (m->dVa[g] == 0.0 || !(m->tau0[g] > 0.0) || !(m->tau1[g] >= 0.0)) return PIMC_ERR_ARG;
  if (m->proposal != PIMC_PROP_GAUSS && m->proposal != PIMC_PROP_UNIFORM) return PIMC_ERR_ARG;
  if (m->p_mask & ~0x7Fu) return PIMC_ERR_ARG;
  if (m->k_mask & ~0xFFFu) return PIMC_ERR_ARG;
  for (int i = 0; i < 12; ++i)
    if (!(m->k_lo[i] <= m->k_hi[i])) return PIMC_ERR_ARG;
  std::memset(&a, 0, sizeof(a));
  a.dt = m->dt;
  a.Ro = m->Ro;
  a.beta = m->beta;
  for (int c = 0; c < 4; ++c) {
    a.Rd[c] = m->Rd[c];
    a.x_lo[c] = m->x_lo[c];
    a.x_hi[c] = m->x_hi[c];
  }
  for (int g = 0; g < 3; ++g) {
    a.Va[g] = m->Va[g];
    a.dVa[g] = m->dVa[g];
    a.tau0[g] = m->tau0[g];
    a.tau1[g] = m->tau1[g];
  }
  for (int l = 0; l < 7; ++l) {
    a.p_lo[l] = m->p_lo[l];
    a.p_hi[l] = m->p_hi[l];
  }
  a.p_mask = m->p_mask;
  a.proposal = m->proposal;
  for (int i = 0; i < 12; ++i) {
    a.k_lo[i] = m->k_lo[i];
    a.k_hi[i] = m->k_hi[i];
  }
  a.k_mask = m->k_mask;
  return PIMC_OK;
}

int ensure_partial(pimc_ctx* ctx, size_t n) {
  if (n <= ctx->partial_cap) return PIMC_OK;
  if (ctx->partial) {
    if (hipDeviceSynchronize() != hipSuccess) return PIMC_ERR_HIP;
    (void)hipFree(ctx->partial);
    ctx->partial = nullptr;
    ctx->partial_cap = 0;
  }
  if (hipMalloc(&ctx->partial, n * sizeof(double)) != hipSuccess) return PIMC_ERR_NOMEM;
  ctx->partial_cap = n;
  return PIMC_OK;
}

int ensure_batch(pimc_ctx* ctx, size_t B) {
  if (B <= ctx->batch_cap) return PIMC_OK;
  if (ctx->offsets) {
    if (hipDeviceSynchronize() != hipSuccess) return PIMC_ERR_HIP;
    (void)hipFree(ctx->offsets);
    (void)hipFree(ctx->order);
    (void)hipFree(ctx->blockK);
    ctx->offsets = nullptr;
    ctx->order = nullptr;
    ctx->blockK = nullptr;
    ctx->batch_cap = 0;
  }
  ctx->last_offsets.clear();   // new buffers: the layout must be copied again
  ctx->blockK_NT = 0;
  if (hipMalloc(&ctx->offsets, (B + 1) * sizeof(int64_t)) != hipSuccess) return PIMC_ERR_NOMEM;
  if (hipMalloc(&ctx->order, B * sizeof(int32_t)) != hipSuccess) return PIMC_ERR_NOMEM;
  if (hipMalloc(&ctx->blockK, B * sizeof(int8_t)) != hipSuccess) return PIMC_ERR_NOMEM;
  ctx->batch_cap = B;
  return PIMC_OK;
}

// Cross-tile workspace for `ntiles` tiles in total over `ngroups` windows:
// boundary sites (two slots of 16 generation words per tile), double-buffered
// parameter partials (70 generation words per tile), one entry word per tile.
// New words start at generation 0 (cleared once here, never per call).
int ensure_tilespace(pimc_ctx* c, size_t ntiles, size_t ngroups) {
  if (ntiles <= c->tile_cap && ngroups <= c->group_cap) return PIMC_OK;
  if (c->halo && hipDeviceSynchronize() != hipSuccess) return PIMC_ERR_HIP;
  ntiles = std::max(ntiles, c->tile_cap);
  ngroups = std::max(ngroups, c->group_cap);
  void** bufs[] = {&c->halo, (void**)&c->wpart, (void**)&c->tsync};
  for (void** q : bufs) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
  c->tile_cap = c->group_cap = 0;
  const size_t sz[] = {pimc::halo_words(ntiles) * sizeof(uint64_t), pimc::wpart_words(ntiles) * sizeof(uint64_t),
                       pimc::tsync_words(ntiles) * sizeof(uint64_t)};
  for (int i = 0; i < 3; ++i) {
    if (hipMalloc(bufs[i], sz[i]) != hipSuccess) return PIMC_ERR_NOMEM;
    if (hipMemset(*bufs[i], 0, sz[i]) != hipSuccess) return PIMC_ERR_HIP;
  }
  // the clears must be complete before any stream of the caller runs a tile
  if (hipDeviceSynchronize() != hipSuccess) return PIMC_ERR_HIP;
  c->tile_cap = ntiles;
  c->group_cap = ngroups;
  c->gen_next = 0;
  return PIMC_OK;
}

// Generation base of a tiled call of n sweeps on `stream`.  The 32-bit
// generations are cleared (in stream order) only when they would wrap.
int tile_generations(pimc_ctx* c, int64_t n, hipStream_t s, uint32_t& gen0, int per_sweep = 1) {
  const uint64_t need = (uint64_t)n * (uint64_t)per_sweep + 4;
  if (n > PIMC_MAX_TILED_SWEEPS) return PIMC_ERR_ARG;
  if (c->gen_next + need > 0xFFFFFFFFull) {
    // clear_words counts 32-bit words
    int r = pimc::clear_words(c->halo, pimc::halo_words(c->tile_cap) * 2, s);
    if (!r) r = pimc::clear_words(c->wpart, pimc::wpart_words(c->tile_cap) * 2, s);
    if (!r) r = pimc::clear_words(c->tsync, pimc::tsync_words(c->tile_cap) * 2, s);
    if (r) return r;
    c->gen_next = 0;
  }
  gen0 = (uint32_t)c->gen_next;
  c->gen_next += need;
  return PIMC_OK;
}

// Launch shape for windows of up to maxM steps under the context's tiling
// settings (choose_sweep_shape); returns K, 0 when no shape fits.
int choose_shape(const pimc_ctx* ctx, int64_t maxM, bool fp64, bool allow_tiles, int& NT, int& stage, int& T,
                 bool ext = false) {
  const pimc::SweepShape sh = pimc::choose_sweep_shape(maxM, fp64, allow_tiles, ctx->tile_K, ctx->tiles, ext);
  if (!sh.K) return 0;
  NT = sh.NT;
  stage = sh.stage;
  T = sh.T;
  return sh.K;
}

// Per-batch sums: the statistics samples one call takes (sweeps k0 .. k0+n-1
// with k >= burn and (k - burn) % stride == 0), their count and the sweep of
// the first; bslice elements per batch slice.
void fill_batch(pimc::SweepArgs& a, double* batch, int64_t nbatch, int64_t k0, int64_t n, int64_t bslice) {
  if (!batch) return;
  int64_t f = std::max(k0, a.burn);
  const int64_t r = (f - a.burn) % a.stride;
  if (r) f += a.stride - r;
  a.batch = batch;
  a.nbatch = nbatch;
  a.kfirst = f;
  a.nsamp = f < k0 + n ? (k0 + n - 1 - f) / a.stride + 1 : 0;
  a.bslice = bslice;
}

void fill_consts(pimc::SweepArgs& a) {
  a.cf.init(a.m);
  a.cd.init(a.m);
}

void fill_debug(pimc::SweepArgs& a, const pimc_debug* d) {
  if (!d) return;
  a.dbg_xprop = d->xprop;
  a.dbg_dA = d->dA;
  a.dbg_acc = d->accept;
  a.dbg_pprop = d->pprop;
  a.dbg_pdA = d->pdA;
  a.dbg_pacc = d->paccept;
}

}  // namespace

extern "C" {

int pimc_ctx_create(pimc_ctx** out, int device) {
  if (!out) return PIMC_ERR_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return PIMC_ERR_ARG;
  if (hipSetDevice(device) != hipSuccess) return PIMC_ERR_HIP;
  pimc_ctx* c = new (std::nothrow) pimc_ctx();
  if (!c) return PIMC_ERR_NOMEM;
  c->device = device;
  if (hipMalloc(&c->err, sizeof(uint32_t)) != hipSuccess) {
    delete c;
    return PIMC_ERR_NOMEM;
  }
  if (hipMemset(c->err, 0, sizeof(uint32_t)) != hipSuccess) {
    (void)hipFree(c->err);
    delete c;
    return PIMC_ERR_HIP;
  }
  if (const char* e = std::getenv("PIMC_TILE_K")) c->tile_K = std::atoi(e);
  if (const char* e = std::getenv("PIMC_NO_GRAPHS")) c->no_graphs = std::atoi(e) != 0;
  if (const char* e = std::getenv("PIMC_BATCH_UNIFORM_K")) c->uniform_batch_K = std::atoi(e) != 0;
  bool ok = ensure_tilespace(c, pimc::MAX_TILES, 4) == PIMC_OK;
  int khz = 0;
  ok = ok && hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0;
  if (!ok) {
    pimc_ctx_destroy(c);
    return PIMC_ERR_NOMEM;
  }
  c->spin_ticks = (uint64_t)khz * 1000ull * 4ull;   // a wait gives up after 4 s
  *out = c;
  return PIMC_OK;
}

void pimc_ctx_destroy(pimc_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->bgraph.ge) (void)hipGraphExecDestroy(ctx->bgraph.ge);
  if (ctx->bgraph.g) (void)hipGraphDestroy(ctx->bgraph.g);
  if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
  if (ctx->err) (void)hipFree(ctx->err);
  if (ctx->partial) (void)hipFree(ctx->partial);
  if (ctx->offsets) (void)hipFree(ctx->offsets);
  if (ctx->order) (void)hipFree(ctx->order);
  if (ctx->blockK) (void)hipFree(ctx->blockK);
  if (ctx->halo) (void)hipFree(ctx->halo);
  if (ctx->wpart) (void)hipFree(ctx->wpart);
  if (ctx->tsync) (void)hipFree(ctx->tsync);
  void* hbufs[] = {ctx->hQ1, ctx->hR0, ctx->hR1, ctx->hX0, ctx->hpart, ctx->hp0, ctx->hpbuf, ctx->hrpbuf,
                   ctx->hH0, ctx->hdH, ctx->hout, ctx->hacc, ctx->hoff, ctx->hbmap, ctx->hbfirst, ctx->hk};
  for (void* q : hbufs)
    if (q) (void)hipFree(q);
  delete ctx;
}

int pimc_set_sweep_tile(pimc_ctx* ctx, int K) {
  if (!ctx || !(K == 0 || K == 2 || K == 4 || K == 8 || K == 16)) return PIMC_ERR_ARG;
  ctx->tile_K = K;
  return PIMC_OK;
}

int pimc_set_sweep_tiles(pimc_ctx* ctx, int T) {
  if (!ctx || T < 0 || T > pimc::MAX_TILES) return PIMC_ERR_ARG;
  ctx->tiles = T;
  return PIMC_OK;
}

int pimc_sync(pimc_ctx* ctx, void* stream) {
  if (!ctx) return PIMC_ERR_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return PIMC_ERR_HIP;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return PIMC_ERR_HIP;
  uint32_t e = 0;
  if (hipMemcpy(&e, ctx->err, sizeof(e), hipMemcpyDeviceToHost) != hipSuccess) return PIMC_ERR_HIP;
  if (e) {
    if (hipMemset(ctx->err, 0, sizeof(uint32_t)) != hipSuccess) return PIMC_ERR_HIP;
    if (e & 4u) return PIMC_ERR_TIMEOUT;
    return (e & 2u) ? PIMC_ERR_BOX : PIMC_ERR_NONFINITE;
  }
  return PIMC_OK;
}

const char* pimc_strerror(int s) {
  switch (s) {
    case PIMC_OK: return "ok";
    case PIMC_ERR_ARG: return "invalid argument";
    case PIMC_ERR_HIP: return "HIP runtime error";
    case PIMC_ERR_NONFINITE: return "non-finite action change encountered";
    case PIMC_ERR_UNSUPPORTED: return "shape not supported by the built kernels";
    case PIMC_ERR_NOMEM: return "out of device memory";
    case PIMC_ERR_BOX: return "state or parameter outside its box at entry";
    case PIMC_ERR_TIMEOUT: return "a cross-tile wait timed out";
    default: return "unknown status";
  }
}

int pimc_action(pimc_ctx* ctx, const pimc_model* model, const pimc_path* path, double* out3, void* stream) {
  if (!ctx || !path || !out3 || !path->X || !path->p || !path->y || !path->I) return PIMC_ERR_ARG;
  if (path->M < 1 || (path->prec != PIMC_FP64 && path->prec != PIMC_FP32)) return PIMC_ERR_ARG;
  pimc::FieldArgs a;
  std::memset(&a, 0, sizeof(a));
  int r = model_args(model, a.m);
  if (r) return r;
  const int64_t nb = pimc::field_blocks(path->M);
  if ((r = ensure_partial(ctx, (size_t)nb * 8))) return r;
  a.M = path->M;
  a.X = path->X;
  a.p = path->p;
  a.y = path->y;
  a.I = path->I;
  a.kin = path->kin;
  a.partial = ctx->partial;
  a.out = out3;
  return pimc::launch_action(a, path->prec == PIMC_FP64, (hipStream_t)stream);
}

int pimc_model_errors(pimc_ctx* ctx, const pimc_model* model, const pimc_path* path, double* esum, double* esq,
                      void* stream) {
  if (!ctx || !path || !esum || !esq || !path->X || !path->p || !path->y || !path->I) return PIMC_ERR_ARG;
  if (path->M < 1 || (path->prec != PIMC_FP64 && path->prec != PIMC_FP32)) return PIMC_ERR_ARG;
  pimc::ErrArgs a;
  std::memset(&a, 0, sizeof(a));
  int r = model_args(model, a.m);
  if (r) return r;
  a.M = path->M;
  a.X = path->X;
  a.p = path->p;
  a.y = path->y;
  a.I = path->I;
  a.kin = path->kin;
  a.esum = esum;
  a.esq = esq;
  if (hipSetDevice(ctx->device) != hipSuccess) return PIMC_ERR_HIP;
  return pimc::launch_errors(a, path->prec == PIMC_FP64, (hipStream_t)stream);
}

int pimc_forecast(pimc_ctx* ctx, const pimc_model* model, int32_t B, const double* x0, const double* p,
                  const double* kin, const double* I, int64_t N, double noise, uint64_t seed, int64_t member0,
                  double* out, void* stream) {
  if (!ctx || B < 1 || N < 0 || !x0 || !p || !I || !out || !(noise >= 0.0) || member0 < 0) return PIMC_ERR_ARG;
  pimc::FcstArgs a;
  std::memset(&a, 0, sizeof(a));
  int r = model_args(model, a.m);
  if (r) return r;
  a.B = B;
  a.N = N;
  a.x0 = x0;
  a.p = p;
  a.I = I;
  a.kin = kin;
  a.noise = noise;
  a.seed = seed;
  a.member0 = member0;
  a.out = out;
  if (hipSetDevice(ctx->device) != hipSuccess) return PIMC_ERR_HIP;
  return pimc::launch_forecast(a, (hipStream_t)stream);
}

int pimc_action_noalloc(const pimc_model* model, const pimc_path* path, double* out3, void* stream) {
  if (!path || !out3 || !path->X || !path->p || !path->y || !path->I) return PIMC_ERR_ARG;
  if (path->M < 1 || (path->prec != PIMC_FP64 && path->prec != PIMC_FP32)) return PIMC_ERR_ARG;
  if (path->M + 1 > PIMC_NOALLOC_MAX_SITES) return PIMC_ERR_UNSUPPORTED;
  pimc::FieldArgs a;
  std::memset(&a, 0, sizeof(a));
  int r = model_args(model, a.m);
  if (r) return r;
  double* part = nullptr;
  if ((r = pimc::noalloc_scratch(&part))) return r;
  a.M = path->M;
  a.X = path->X;
  a.p = path->p;
  a.y = path->y;
  a.I = path->I;
  a.kin = path->kin;
  a.partial = part;
  a.out = out3;
  return pimc::launch_action(a, path->prec == PIMC_FP64, (hipStream_t)stream);
}

int pimc_grad(pimc_ctx* ctx, const pimc_model* model, const pimc_path* path, void* gX, double* gp, void* stream) {
  if (!ctx || !path || !gX || !gp || !path->X || !path->p || !path->y || !path->I) return PIMC_ERR_ARG;
  if (path->M < 1 || (path->prec != PIMC_FP64 && path->prec != PIMC_FP32)) return PIMC_ERR_ARG;
  pimc::FieldArgs a;
  std::memset(&a, 0, sizeof(a));
  int r = model_args(model, a.m);
  if (r) return r;
  const int64_t nb = pimc::field_blocks(path->M);
  if ((r = ensure_partial(ctx, (size_t)nb * 8))) return r;
  a.M = path->M;
  a.X = path->X;
  a.p = path->p;
  a.y = path->y;
  a.I = path->I;
  a.kin = path->kin;
  a.gX = gX;
  a.partial = ctx->partial;
  a.out = gp;
  return pimc::launch_grad(a, path->prec == PIMC_FP64, (hipStream_t)stream);
}

}  // extern "C"

namespace {

// Checks of an initialization-phase state; fills the kernel arguments.
int init_args(const pimc_init_phase* ip, pimc::SweepArgs& a) {
  if (!(ip->beta0 > 0.0 && ip->beta0 <= 1.0) || ip->n_cool < 1 || ip->n_skip < 1 || ip->n_init < 0) return PIMC_ERR_ARG;
  if (!(ip->alpha >= 0.0 && ip->alpha < 1e3) || !(ip->f_acc >= 0.0 && ip->f_acc <= 1.0)) return PIMC_ERR_ARG;
  if (!ip->beta || !ip->site_scale || !ip->w_param || !ip->cnt_site || !ip->cnt_param) return PIMC_ERR_ARG;
  a.ip_fbeta = std::pow(1.0 / ip->beta0, 1.0 / (double)ip->n_cool);   // eq. fbeta
  a.ip_ninit = ip->n_init;
  a.ip_nskip = ip->n_skip;
  a.ip_facc = ip->f_acc;
  a.ip_alpha = ip->alpha;
  a.ip_beta = ip->beta;
  a.ip_scale = ip->site_scale;
  a.ip_wpar = ip->w_param;
  a.ip_cnt = ip->cnt_site;
  a.ip_cntp = ip->cnt_param;
  return PIMC_OK;
}

int sweep_impl(pimc_ctx* ctx, const pimc_model* model, pimc_path* path, pimc_rng rng, const double* w,
               int64_t n_sweeps, int32_t flags, const pimc_init_phase* ip, const pimc_stats* stats,
               const pimc_debug* debug, void* stream) {
  if (!ctx || !path || !w || !path->X || !path->p || !path->y || !path->I) return PIMC_ERR_ARG;
  if (path->M < 1 || (path->prec != PIMC_FP64 && path->prec != PIMC_FP32)) return PIMC_ERR_ARG;
  if (n_sweeps < 0 || !valid_flags(flags)) return PIMC_ERR_ARG;
  if (stats && (stats->sum || stats->sumsq) && (!stats->xref || !stats->sum)) return PIMC_ERR_ARG;
  if (stats && stats->batch && (!stats->sum || stats->nbatch < 1)) return PIMC_ERR_ARG;
  if (n_sweeps == 0) return PIMC_OK;
  pimc::SweepArgs a;
  std::memset(&a, 0, sizeof(a));
  int r = model_args(model, a.m);
  if (r) return r;
  const bool fp64 = path->prec == PIMC_FP64;
  int NT = 0, stage = 0, T = 1;
  if (path->M >= (1ll << 30)) return PIMC_ERR_UNSUPPORTED;
  // the initialization phase and kinetic constants run in the extended
  // kernels (which draw exactly too), exact parameter draws alone in the
  // exact-draw kernels: shapes of at most 256 threads and 4 sites per thread
  const bool kinetic = (flags & PIMC_KINETIC) != 0;
  const int ext = (ip || kinetic) ? 1 : ((flags & PIMC_GIBBS) ? 2 : 0);
  const int K = choose_shape(ctx, path->M, fp64, true, NT, stage, T, ext != 0);
  if (!K) return PIMC_ERR_UNSUPPORTED;
  fill_consts(a);
  a.stage = stage;
  a.stride = 1;
  a.tiles = T;
  a.ngroups = 1;
  a.halo = ctx->halo;
  a.wpart = ctx->wpart;
  a.tsync = ctx->tsync;
  a.spin_ticks = ctx->spin_ticks;
  a.offsets = nullptr;
  a.M_single = path->M;
  a.X = path->X;
  a.p = path->p;
  a.y = path->y;
  a.I = path->I;
  a.chain_single = rng.chain;
  a.seed = rng.seed;
  a.sweep0 = rng.sweep0;
  a.n_sweeps = n_sweeps;
  a.flags = flags;
  a.w = w;
  if (stats) {
    a.sum = stats->sum;
    a.sumsq = stats->sumsq;
    a.xref = stats->xref;
    a.ptrace = stats->ptrace;
    a.acc = stats->acc;
    a.kacc = stats->kacc;
    a.burn = stats->burn;
    a.stride = stats->stride > 1 ? stats->stride : 1;
    fill_batch(a, stats->batch, stats->nbatch, (int64_t)rng.sweep0, n_sweeps, (path->M + 1) * 4);
  }
  fill_debug(a, debug);
  a.err = ctx->err;
  if (hipSetDevice(ctx->device) != hipSuccess) return PIMC_ERR_HIP;
  if (kinetic && !path->kin) return PIMC_ERR_ARG;
  a.kin = path->kin;
  if (debug) {
    a.dbg_kprop = debug->kprop;
    a.dbg_kdA = debug->kdA;
    a.dbg_kacc = debug->kaccept;
  }
  if (ext && NT > 256) return PIMC_ERR_UNSUPPORTED;
  if (ip && (r = init_args(ip, a))) return r;
  // all-reduces between the tiles per sweep: the parameter statistics and
  // one per sampled kinetic constant
  const int per_sweep = 1 + (kinetic ? __builtin_popcount(a.m.k_mask) : 0);
  if (T > 1 && (r = tile_generations(ctx, n_sweeps, (hipStream_t)stream, a.gen0, per_sweep))) return r;
  return pimc::launch_sweep(a, fp64, K, T, NT, (hipStream_t)stream, ext);
}

}  // namespace

extern "C" {

int pimc_sweep(pimc_ctx* ctx, const pimc_model* model, pimc_path* path, pimc_rng rng, const double* w,
               int64_t n_sweeps, int32_t flags, const pimc_stats* stats, const pimc_debug* debug, void* stream) {
  return sweep_impl(ctx, model, path, rng, w, n_sweeps, flags, nullptr, stats, debug, stream);
}

int pimc_sweep_init(pimc_ctx* ctx, const pimc_model* model, pimc_path* path, pimc_rng rng, const double* w,
                    int64_t n_sweeps, int32_t flags, const pimc_init_phase* init, const pimc_stats* stats,
                    void* stream) {
  if (!init) return PIMC_ERR_ARG;
  return sweep_impl(ctx, model, path, rng, w, n_sweeps, flags, init, stats, nullptr, stream);
}

int pimc_param_update(pimc_ctx* ctx, const pimc_model* model, pimc_path* path, pimc_rng rng, const double* w,
                      const pimc_debug* debug, void* stream) {
  return pimc_sweep(ctx, model, path, rng, w, 1, PIMC_PARAMS, nullptr, debug, stream);
}

// The batched sweep launch as a captured graph: recorded once per launch
// shape on the context's capture stream, then replayed on the caller's
// stream with this call's arguments written into its kernel node.  (Tiled
// batches are launched directly, not captured.)
static int launch_batch_graph(pimc_ctx* ctx, const pimc::SweepArgs& a, bool fp64, int K, int nblocks, int NT,
                              int stage, hipStream_t s, int ext) {
  auto& bg = ctx->bgraph;
  const bool dbg = a.dbg_xprop || a.dbg_dA || a.dbg_acc || a.dbg_pprop || a.dbg_pdA || a.dbg_pacc;
  int r = PIMC_OK;
  if (!(bg.valid && bg.fp64 == fp64 && bg.dbg == dbg && bg.ext == ext && bg.K == K && bg.NT == NT &&
        bg.nblocks == nblocks && bg.stage == stage)) {
    if (bg.ge) (void)hipGraphExecDestroy(bg.ge);
    if (bg.g) (void)hipGraphDestroy(bg.g);
    bg = pimc_ctx::BatchGraph{};
    if (!ctx->cap && (r = hip_ok(hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking)))) return r;
    if ((r = hip_ok(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal)))) return r;
    const int lr = pimc::launch_sweep(a, fp64, K, nblocks, NT, ctx->cap, ext);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(ctx->cap, &g);
    if (lr || ec != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return lr ? lr : PIMC_ERR_HIP;
    }
    size_t nn = 1;
    hipGraphNode_t node = nullptr;
    hipGraphExec_t ge = nullptr;
    if (hipGraphGetNodes(g, &node, &nn) != hipSuccess || nn != 1 ||
        hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      return PIMC_ERR_HIP;
    }
    bg.valid = true;
    bg.fp64 = fp64;
    bg.dbg = dbg;
    bg.ext = ext;
    bg.K = K;
    bg.NT = NT;
    bg.nblocks = nblocks;
    bg.stage = stage;
    bg.g = g;
    bg.ge = ge;
    bg.node = node;
  } else {
    hipKernelNodeParams kp;
    if ((r = hip_ok(hipGraphKernelNodeGetParams(bg.node, &kp)))) return r;
    pimc::SweepArgs copy = a;
    void* args[] = {&copy};
    kp.kernelParams = args;
    kp.extra = nullptr;
    if ((r = hip_ok(hipGraphExecKernelNodeSetParams(bg.ge, bg.node, &kp)))) return r;
  }
  return hip_ok(hipGraphLaunch(bg.ge, s));
}

int pimc_run_batch(pimc_ctx* ctx, const pimc_model* model, const pimc_batch* b, uint64_t seed, uint64_t sweep0,
                   const double* w, int64_t n_sweeps, int32_t flags, const pimc_batch_stats* stats, void* stream) {
  if (!ctx || !b || !w || !b->offsets || !b->X || !b->p || !b->y || !b->I || !b->chain) return PIMC_ERR_ARG;
  if (b->B < 1 || (b->prec != PIMC_FP64 && b->prec != PIMC_FP32)) return PIMC_ERR_ARG;
  if (n_sweeps < 0 || !valid_flags(flags) || (flags & PIMC_KINETIC)) return PIMC_ERR_ARG;   // no kin in a batch
  if (stats && (stats->sum || stats->sumsq) && (!stats->xref || !stats->sum)) return PIMC_ERR_ARG;
  if (stats && stats->batch && (!stats->sum || stats->nbatch < 1)) return PIMC_ERR_ARG;
  if (n_sweeps == 0) return PIMC_OK;
  const int B = b->B;
  if (b->offsets[0] != 0) return PIMC_ERR_ARG;
  std::vector<int64_t> Ms(B);
  for (int i = 0; i < B; ++i) {
    const int64_t Mi = b->offsets[i + 1] - b->offsets[i] - 1;
    if (Mi < 1 || Mi >= (1ll << 30)) return PIMC_ERR_ARG;
    Ms[i] = Mi;
  }
  pimc::SweepArgs a;
  std::memset(&a, 0, sizeof(a));
  int r = model_args(model, a.m);
  if (r) return r;
  const bool fp64 = b->prec == PIMC_FP64;
  // time tiles (set_sweep_tiles > 1) apply when every window of the batch
  // needs exactly that many tiles of the chosen shape; otherwise one
  // workgroup per window
  const pimc::SweepShape sh =
      pimc::choose_batch_shape(Ms.data(), B, fp64, ctx->tile_K, ctx->tiles, (flags & PIMC_GIBBS) != 0);
  const int K = sh.K, NT = sh.NT, stage = sh.stage, T = sh.T;
  if (!K) return PIMC_ERR_UNSUPPORTED;
  fill_consts(a);
  a.stage = stage;
  a.stride = 1;
  a.tiles = T;
  a.ngroups = B;
  if (hipSetDevice(ctx->device) != hipSuccess) return PIMC_ERR_HIP;
  if ((r = ensure_batch(ctx, (size_t)B))) return r;
  if (T > 1) {
    if ((r = ensure_tilespace(ctx, (size_t)B * T, (size_t)B))) return r;
    a.halo = ctx->halo;
    a.wpart = ctx->wpart;
    a.tsync = ctx->tsync;
    a.spin_ticks = ctx->spin_ticks;
  }
  // longest windows first, so the tail of the launch holds the short ones
  std::vector<int32_t> order(B);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return Ms[x] > Ms[y]; });
  hipStream_t s = (hipStream_t)stream;
  const bool same_layout = ctx->last_offsets.size() == (size_t)B + 1 &&
                           std::equal(ctx->last_offsets.begin(), ctx->last_offsets.end(), b->offsets);
  if (!same_layout) {
    ctx->last_offsets.clear();
    if ((r = hip_ok(hipMemcpyAsync(ctx->offsets, b->offsets, (B + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s))))
      return r;
    if ((r = hip_ok(hipMemcpyAsync(ctx->order, order.data(), B * sizeof(int32_t), hipMemcpyHostToDevice, s))))
      return r;
    // the host vectors die at return: make sure the copies have consumed them
    if ((r = hip_ok(hipStreamSynchronize(s)))) return r;
    ctx->last_offsets.assign(b->offsets, b->offsets + B + 1);
    ctx->blockK_NT = 0;
  }
  // a batch launched with 16 sites per thread runs each window with the
  // fewest of 4, 8, 12, 16 sites per thread that NT threads hold
  const bool perK = T == 1 && !fp64 && K == 16 && !ctx->uniform_batch_K;
  if (perK && ctx->blockK_NT != NT) {
    std::vector<int8_t> bk(B);
    for (int i = 0; i < B; ++i) bk[i] = (int8_t)pimc::batch_block_K(Ms[order[i]], NT);
    if ((r = hip_ok(hipMemcpyAsync(ctx->blockK, bk.data(), B * sizeof(int8_t), hipMemcpyHostToDevice, s))))
      return r;
    if ((r = hip_ok(hipStreamSynchronize(s)))) return r;
    ctx->blockK_NT = NT;
  }
  a.offsets = ctx->offsets;
  a.order = ctx->order;
  a.blockK = perK ? ctx->blockK : nullptr;
  a.X = b->X;
  a.p = b->p;
  a.y = b->y;
  a.I = b->I;
  a.chain_ids = b->chain;
  a.seed = seed;
  a.sweep0 = sweep0;
  a.n_sweeps = n_sweeps;
  a.flags = flags;
  a.w = w;
  if (stats) {
    a.sum = stats->sum;
    a.sumsq = stats->sumsq;
    a.xref = stats->xref;
    a.ptrace = stats->ptrace;
    a.acc = stats->acc;
    a.burn = stats->burn;
    a.stride = stats->stride > 1 ? stats->stride : 1;
    fill_batch(a, stats->batch, stats->nbatch, (int64_t)sweep0, n_sweeps, b->offsets[B] * 4);
  }
  a.err = ctx->err;
  const int ext = (flags & PIMC_GIBBS) ? 2 : 0;   // exact draws run in the exact-draw kernels
  if (ext && NT > 256) return PIMC_ERR_UNSUPPORTED;
  if (T > 1 && (r = tile_generations(ctx, n_sweeps, s, a.gen0))) return r;
  if (T == 1 && !ctx->no_graphs) return launch_batch_graph(ctx, a, fp64, K, B, NT, stage, s, ext);
  return pimc::launch_sweep(a, fp64, K, B * T, NT, s, ext);
}

}  // extern "C"

namespace {

int hmc_workspace(pimc_ctx* c, size_t S, size_t nb, size_t B, size_t ts) {
  if (S <= c->hmc_sites && nb <= c->hmc_blocks && B <= c->hmc_B && ts <= c->hmc_tsize && c->hk) return PIMC_OK;
  if (hipDeviceSynchronize() != hipSuccess) return PIMC_ERR_HIP;
  void** bufs[] = {&c->hQ1, &c->hR0, &c->hR1, &c->hX0, (void**)&c->hpart, (void**)&c->hp0, (void**)&c->hpbuf,
                   (void**)&c->hrpbuf, (void**)&c->hH0, (void**)&c->hdH, (void**)&c->hout, (void**)&c->hacc,
                   (void**)&c->hoff, (void**)&c->hbmap, (void**)&c->hbfirst, (void**)&c->hk};
  for (void** q : bufs) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
  S = std::max(S, c->hmc_sites);
  nb = std::max(nb, c->hmc_blocks);
  B = std::max(B, c->hmc_B);
  ts = std::max(ts, c->hmc_tsize);
  const size_t sz[] = {S * 4 * ts, S * 4 * ts, S * 4 * ts, S * 4 * ts, 2 * nb * 16 * 8, B * 7 * 8, 2 * B * 7 * 8,
                       2 * B * 7 * 8, B * 8, B * 8, B * 4, B, (B + 1) * 8, nb * 4, (B + 1) * 4, 8};
  for (size_t i = 0; i < sizeof(sz) / sizeof(sz[0]); ++i)
    if (hipMalloc(bufs[i], sz[i]) != hipSuccess) return PIMC_ERR_NOMEM;
  c->hmc_sites = S;
  c->hmc_blocks = nb;
  c->hmc_B = B;
  c->hmc_tsize = ts;
  return PIMC_OK;
}

}  // namespace

extern "C" int pimc_hmc(pimc_ctx* ctx, const pimc_model* model, const pimc_batch* b, uint64_t seed, uint64_t k0,
                        double eps, int32_t L, const double* minv, int64_t n_proposals, const pimc_hmc_stats* stats,
                        void* stream) {
  if (!ctx || !b || !minv || !b->offsets || !b->X || !b->p || !b->y || !b->I || !b->chain) return PIMC_ERR_ARG;
  if (b->B < 1 || (b->prec != PIMC_FP64 && b->prec != PIMC_FP32)) return PIMC_ERR_ARG;
  if (!(eps > 0.0) || L < 1 || n_proposals < 0) return PIMC_ERR_ARG;
  for (int i = 0; i < 11; ++i)
    if (!(minv[i] > 0.0)) return PIMC_ERR_ARG;
  if (n_proposals == 0) return PIMC_OK;
  const int B = b->B;
  if (b->offsets[0] != 0) return PIMC_ERR_ARG;
  std::vector<int32_t> bfirst(B + 1), bmap;
  for (int i = 0; i < B; ++i) {
    const int64_t Mi = b->offsets[i + 1] - b->offsets[i] - 1;
    if (Mi < 1 || Mi >= (1ll << 30)) return PIMC_ERR_ARG;
    bfirst[i] = (int32_t)bmap.size();
    const int64_t nbk = (Mi + 1 + pimc::HMC_BLOCK - 1) / pimc::HMC_BLOCK;
    for (int64_t q = 0; q < nbk; ++q) bmap.push_back(i);
  }
  bfirst[B] = (int32_t)bmap.size();
  pimc::HmcArgs a;
  std::memset(&a, 0, sizeof(a));
  int r = model_args(model, a.m);
  if (r) return r;
  const bool fp64 = b->prec == PIMC_FP64;
  const size_t S = (size_t)b->offsets[B];
  if (hipSetDevice(ctx->device) != hipSuccess) return PIMC_ERR_HIP;
  if ((r = hmc_workspace(ctx, S, bmap.size(), (size_t)B, fp64 ? 8 : 4))) return r;
  hipStream_t s = (hipStream_t)stream;
  if ((r = hip_ok(hipMemcpyAsync(ctx->hoff, b->offsets, (B + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s))))
    return r;
  if ((r = hip_ok(hipMemcpyAsync(ctx->hbmap, bmap.data(), bmap.size() * 4, hipMemcpyHostToDevice, s)))) return r;
  if ((r = hip_ok(hipMemcpyAsync(ctx->hbfirst, bfirst.data(), (B + 1) * 4, hipMemcpyHostToDevice, s)))) return r;
  if ((r = hip_ok(hipMemcpyAsync(ctx->hk, &k0, sizeof(k0), hipMemcpyHostToDevice, s)))) return r;
  if ((r = hip_ok(hipStreamSynchronize(s)))) return r;   // host vectors die at return
  a.cf.init(a.m);
  a.cd.init(a.m);
  a.B = B;
  a.nblocks = (int32_t)bmap.size();
  a.offsets = ctx->hoff;
  a.bmap = ctx->hbmap;
  a.bfirst = ctx->hbfirst;
  a.X = b->X;
  a.p = b->p;
  a.y = b->y;
  a.I = b->I;
  a.chain = b->chain;
  a.seed = seed;
  a.kptr = ctx->hk;
  a.k_first = k0;
  a.eps = eps;
  for (int i = 0; i < 11; ++i) a.minv[i] = minv[i];
  a.Q1 = ctx->hQ1;
  a.R0 = ctx->hR0;
  a.R1 = ctx->hR1;
  a.X0 = ctx->hX0;
  a.p0 = ctx->hp0;
  a.pbuf = ctx->hpbuf;
  a.rpbuf = ctx->hrpbuf;
  a.part = ctx->hpart;
  a.H0 = ctx->hH0;
  a.outside = ctx->hout;
  a.accepted = ctx->hacc;
  a.dH = ctx->hdH;
  if (stats) {
    a.acc = stats->acc;
    a.ptrace = stats->ptrace;
    a.dHtrace = stats->dH;
    const bool any = stats->traj_q || stats->traj_r || stats->traj_p || stats->traj_rp;
    const bool all = stats->traj_q && stats->traj_r && stats->traj_p && stats->traj_rp;
    if (any && !all) return PIMC_ERR_ARG;
    a.tq = stats->traj_q;
    a.tr = stats->traj_r;
    a.tp = stats->traj_p;
    a.trp = stats->traj_rp;
  }
  a.S = (int64_t)S;
  a.ntrace = n_proposals;
  if (n_proposals == 1 || ctx->no_graphs) {
    for (int64_t q = 0; q < n_proposals; ++q)
      if ((r = pimc::launch_hmc_proposal(a, fp64, L, s))) return r;
    return PIMC_OK;
  }
  // The L + 3 launches of one proposal take fixed arguments (the proposal
  // index is in device memory), so they are captured once and replayed on
  // the caller's stream.  Capture happens on a private stream because the
  // caller's may be the legacy default stream, which cannot be captured;
  // recording runs nothing, so that stream needs no ordering with `s`.
  if (!ctx->cap && (r = hip_ok(hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking)))) return r;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  if ((r = hip_ok(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal)))) return r;
  const int lr = pimc::launch_hmc_proposal(a, fp64, L, ctx->cap);
  const hipError_t ec = hipStreamEndCapture(ctx->cap, &g);
  if (lr || ec != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return lr ? lr : PIMC_ERR_HIP;
  }
  if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return PIMC_ERR_HIP;
  }
  for (int64_t q = 0; q < n_proposals && !r; ++q) r = hip_ok(hipGraphLaunch(ge, s));
  // the executable graph may be destroyed once its launches are enqueued
  const int r2 = hip_ok(hipStreamSynchronize(s));
  (void)hipGraphExecDestroy(ge);
  (void)hipGraphDestroy(g);
  return r ? r : r2;
}
