/*
 * libpimc -- path-integral Monte Carlo data assimilation on AMD MI355X (gfx950).
 *
 * The library samples the posterior exp(-A(X, p)) over the whole discretised
 * state history X = {x_0 .. x_M} of a Hodgkin-Huxley neuron and its
 * parameters p, following Quinn & Abarbanel, "Data Assimilation using a GPU
 * Accelerated Path Integral Monte Carlo Approach" (arXiv:1103.4887):
 *
 *   A = A_o + beta A_d                                   (Section 2.1)
 *   A_o = 1/2 sum_{n=1..M} Ro (y_n - V_n)^2              (observation error)
 *   A_d = 1/2 sum_{n=1..M} eps_n^T Rd eps_n              (model error)
 *   eps_n = x_n - x_{n-1} - dt/2 [F(x_n; p) + F(x_{n-1}; p)]   (trapezoid rule)
 *
 * with the HH vector field F of Section 5.1 (dV/dt and da/dt equations,
 * gating constants of Table 1) and a uniform box prior on states and
 * parameters (Section 2.1, Section 4.2).
 *
 * Conventions for every entry point:
 *  - all array pointers are caller-owned DEVICE memory unless stated; the
 *    library never frees or retains them;
 *  - `stream` is a hipStream_t (NULL = the default stream); every call is
 *    asynchronous on it;
 *  - argument errors are detected on the host before anything is enqueued and
 *    return a negative pimc_status; a problem found on the device (a state or
 *    parameter outside its box at entry, a non-finite action change) sets a
 *    flag in the context that the next pimc_sync() reports;
 *  - a path holds M+1 sites; X is [M+1][4] row-major in the order (V, m, h, n)
 *    in FP64 (PIMC_FP64) or FP32 (PIMC_FP32); y and I are [M+1] in the same
 *    precision, y[0] is never read (observations start at n = 1);
 *  - parameters p are FP64 [7] = (p1 .. p7) of the dV/dt equation.
 *
 * Random numbers are Philox4x32-10 (Salmon et al., SC'11) at fixed logical
 * addresses: key = (seed_lo32, seed_hi32 ^ chain), counter = (index,
 * sweep_lo32, tag << 24 | sweep_hi24, block).  Results therefore depend on
 * (seed, chain, sweep index) only, never on launch shape.
 */
#ifndef PIMC_H
#define PIMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PIMC_OK = 0,
  PIMC_ERR_ARG = -1,          /* invalid argument (null pointer, size, enum) */
  PIMC_ERR_HIP = -2,          /* a HIP runtime call failed */
  PIMC_ERR_NONFINITE = -3,    /* a non-finite action change was met (reported by pimc_sync) */
  PIMC_ERR_UNSUPPORTED = -4,  /* shape not supported by the built kernels */
  PIMC_ERR_NOMEM = -5,        /* workspace allocation failed */
  PIMC_ERR_BOX = -6,          /* state or parameter outside its box at entry (reported by pimc_sync) */
  PIMC_ERR_TIMEOUT = -7       /* a wait between the time tiles of a window gave up (reported by pimc_sync) */
} pimc_status;

enum { PIMC_FP64 = 0, PIMC_FP32 = 1 };          /* site arithmetic precision */
enum { PIMC_PROP_GAUSS = 0, PIMC_PROP_UNIFORM = 1 }; /* proposal law (Fig. 1 step 1a = uniform) */
/* pimc_sweep / pimc_run_batch flags.  PIMC_GIBBS (with PIMC_PARAMS): each
 * sampled parameter, in ascending order, is drawn from its exact conditional
 * given the path and the other parameters instead of a Metropolis step.
 * dV/dt is affine in each p_l (Section 5.1), so the action is quadratic in
 * p_l and the conditional is a Gaussian truncated to p_l's box, read from the
 * same path statistics the Metropolis moves use; the draw inverts its CDF
 * with word 0 of the parameter's Philox block.  It changes the chain, so it
 * is off unless asked for; acceptance counters then count finite draws.
 * Runs in the launch shapes of at most 256 threads per workgroup and at most
 * 4 sites per thread: the automatic choice cuts windows longer than 1024
 * steps into time tiles of such shapes, and a shape forced wider (see
 * pimc_set_sweep_tile, pimc_set_sweep_tiles) returns PIMC_ERR_UNSUPPORTED
 * before anything is launched. */
enum { PIMC_STATES = 1, PIMC_PARAMS = 2, PIMC_GIBBS = 4, PIMC_KINETIC = 8 };
/* PIMC_KINETIC (pimc_sweep / pimc_sweep_init on a path with `kin` set): after
 * the parameters, each Table 1 constant selected by model->k_mask, in the
 * order (m, h, n) x (V_a, dV_a, tau0, tau1), takes a Metropolis move
 * kin_i + w[11 + i] z (Philox KIN block of index i: z from words 0 and 1,
 * the accept uniform from word 2; rejected outside k_lo/k_hi).  The constants
 * enter the gate equations nonlinearly, so each move is a full pass over the
 * path with the change of A summed in FP64 over all links (the direct form of
 * Section 4.1; Section 5.1 notes all the model's constants can be estimated
 * this way).  Runs in the launch shapes of at most 256 threads and at most 4
 * sites per thread, as PIMC_GIBBS. */

/* Most sweeps one call may run when its windows are cut into time tiles
 * (longer runs are split into several calls by the caller). */
#define PIMC_MAX_TILED_SWEEPS (1ll << 30)

/* acceptance counters written to pimc_stats.acc */
enum { PIMC_ACC_EVEN = 0, PIMC_ACC_ODD = 1, PIMC_ACC_PARAM0 = 2, PIMC_ACC_NONFINITE = 9, PIMC_NACC = 10 };

typedef struct pimc_ctx pimc_ctx;

/* Model, noise precisions and box prior; host memory, copied at each call. */
typedef struct {
  double dt;          /* time step (ms) */
  double Ro;          /* observation precision (L = 1, observed component V) */
  double Rd[4];       /* diagonal model-error precision (V, m, h, n) */
  double beta;        /* multiplier of A_d (annealing factor, Section 4.2) */
  double Va[3], dVa[3], tau0[3], tau1[3];  /* Table 1, order (m, h, n) */
  double x_lo[4], x_hi[4];                 /* state box, every site */
  double p_lo[7], p_hi[7];                 /* parameter box */
  uint32_t p_mask;    /* bit l set => p_{l+1} is sampled */
  int32_t proposal;   /* PIMC_PROP_GAUSS or PIMC_PROP_UNIFORM */
  double k_lo[12], k_hi[12];  /* box of the Table 1 constants, order (m, h, n) x (V_a, dV_a, tau0, tau1) */
  uint32_t k_mask;    /* bit i set => Table 1 constant i is sampled (PIMC_KINETIC) */
} pimc_model;

/* One window.  X and p are read and written; y and I are read only. */
typedef struct {
  int64_t M;          /* number of steps; sites n = 0..M; M >= 1 */
  int32_t prec;       /* PIMC_FP64 or PIMC_FP32: type of X, y, I */
  void* X;            /* [M+1][4] */
  double* p;          /* [7] FP64 */
  const void* y;      /* [M+1], y[0] unused */
  const void* I;      /* [M+1], drive at t_n */
  double* kin;        /* [12] FP64 or NULL: the Table 1 constants of this window, order (m, h, n) x
                         (V_a, dV_a, tau0, tau1); when set they replace the model's Va/dVa/tau0/tau1
                         in every kernel of the call, and PIMC_KINETIC samples them (in/out) */
} pimc_path;

/* Random-number address: sweep k of a call is sweep0 + (0 .. n_sweeps-1). */
typedef struct {
  uint64_t seed;
  uint32_t chain;
  uint64_t sweep0;
} pimc_rng;

/* Statistics (every pointer nullable; device memory).
 *   sum, sumsq  [M+1][4] FP64, accumulated (+=) over sweeps k >= burn:
 *               sum (x - xref) and sum (x - xref)^2
 *   xref        [M+1][4] in path precision (required when sum/sumsq given)
 *   ptrace      [n_sweeps][7] FP64: p after every sweep of the call (written)
 *   acc         [PIMC_NACC] int64 acceptance counters (+=)
 *   stride      moments are accumulated at sweeps k >= burn with (k - burn) % stride == 0
 *               (the N_skip of Section 4.1; values <= 1 mean every sweep)
 *   batch       [nbatch][M+1][4] FP64 (nullable; requires sum): sum (x - xref) (+=) per run
 *               of consecutive samples: of the ns samples one call takes, the i-th
 *               (i = 0 .. ns-1) belongs to batch floor(i nbatch / ns), so batch b holds
 *               ceil((b+1) ns / nbatch) - ceil(b ns / nbatch) samples (batch means for
 *               the Monte Carlo error of the path means); nbatch >= 1 when batch is set */
typedef struct {
  double* sum;
  double* sumsq;
  const void* xref;
  double* ptrace;
  int64_t* acc;
  int64_t burn;
  int64_t stride;
  double* batch;
  int64_t nbatch;
  int64_t* kacc;      /* [12] int64 (+=), nullable: accepted moves of each Table 1 constant (PIMC_KINETIC) */
} pimc_stats;

/* What the LAST sweep of a call proposed and decided (every pointer nullable).
 *   xprop [M+1][4] path precision, dA [M+1] FP64 (NaN where the proposal left
 *   the box), accept [M+1] uint8; pprop/pdA [7] FP64, paccept [7] uint8
 *   (entries of unsampled parameters are left untouched); kprop/kdA [12]
 *   FP64, kaccept [12] uint8 for the Table 1 constants (PIMC_KINETIC).
 *   Calls with PIMC_KINETIC or PIMC_GIBBS record the parameter and k fields
 *   only: xprop, dA and accept must then be NULL (else
 *   PIMC_ERR_UNSUPPORTED).  A Gibbs draw records pdA = NaN. */
typedef struct {
  void* xprop;
  double* dA;
  uint8_t* accept;
  double* pprop;
  double* pdA;
  uint8_t* paccept;
  double* kprop;
  double* kdA;
  uint8_t* kaccept;
} pimc_debug;

/* Packed batch of independent windows for pimc_run_batch.
 *   offsets   HOST [B+1]: window w owns packed sites offsets[w] .. offsets[w+1]-1,
 *             so M_w = offsets[w+1] - offsets[w] - 1 >= 1
 *   X [S][4], y [S], I [S] packed in path precision (S = offsets[B])
 *   p [B][7] FP64, chain [B] uint32 (Philox chain id of each window) */
typedef struct {
  int32_t B;
  int32_t prec;
  const int64_t* offsets;
  void* X;
  double* p;
  const void* y;
  const void* I;
  const uint32_t* chain;
} pimc_batch;

/* Per-window statistics of a batch (every pointer nullable; device memory).
 *   sum, sumsq [S][4] FP64 packed like X; xref [S][4] path precision;
 *   ptrace [B][n_sweeps][7] FP64; acc [B][PIMC_NACC] int64; batch
 *   [nbatch][S][4] FP64 packed like X; burn, stride, nbatch as for pimc_stats. */
typedef struct {
  double* sum;
  double* sumsq;
  const void* xref;
  double* ptrace;
  int64_t* acc;
  int64_t burn;
  int64_t stride;
  double* batch;
  int64_t nbatch;
} pimc_batch_stats;

/* Create a context bound to HIP device `device` (it owns only its workspace:
 * error flags, reduction scratch, captured graphs).  Returns PIMC_OK. */
int pimc_ctx_create(pimc_ctx** out, int device);
void pimc_ctx_destroy(pimc_ctx* ctx);

/* Sites per thread of the sweep kernel: 2, 4, 8 or 16 (FP32) / 4 (FP64);
 * 0 restores the automatic choice (which never picks 2).  FP64 windows run
 * in one workgroup of at most 256 threads, so M <= 1024; longer FP64
 * windows are refused with PIMC_ERR_UNSUPPORTED.  The chain does not depend on it: random
 * numbers are addressed by (site, sweep), never by thread. */
int pimc_set_sweep_tile(pimc_ctx* ctx, int K);

/* Time tiles per window for pimc_sweep: T >= 2 cuts the window into T
 * workgroups of S sites each, (T-1) S < M <= T S, that exchange their
 * boundary sites and all-reduce the parameter statistics through global
 * memory (launched cooperatively so that all tiles are resident; every
 * wait is bounded).  0 restores the automatic choice (one workgroup of at
 * most 256 threads when the window fits, the fewest tiles otherwise); 1
 * forces one workgroup (up to 1024 threads); at most 256.  Only FP32 windows
 * are tiled: an FP64 window that does not fit one workgroup is refused with
 * PIMC_ERR_UNSUPPORTED.  The tiles of a launch must all be resident at once:
 * a launch larger than the device holds is refused (PIMC_ERR_UNSUPPORTED),
 * and if other work keeps a tile from being placed, the tiles' bounded waits
 * give up and pimc_sync reports PIMC_ERR_TIMEOUT.  A tiled call runs at most
 * PIMC_MAX_TILED_SWEEPS sweeps (PIMC_ERR_ARG beyond); calls on one context
 * share its exchange workspace, so they must not run concurrently.  pimc_run_batch uses T tiles per window when every
 * window of the batch needs exactly T tiles of the chosen shape, else one
 * workgroup per window. */
int pimc_set_sweep_tiles(pimc_ctx* ctx, int T);

/* Wait for `stream`, then return and clear any deferred device-side error
 * (PIMC_ERR_TIMEOUT first, then PIMC_ERR_BOX, then PIMC_ERR_NONFINITE). */
int pimc_sync(pimc_ctx* ctx, void* stream);

const char* pimc_strerror(int status);

/* Full action (Section 2.1): out3 (device, FP64 [3]) <- (A, A_o, A_d) with
 * A = A_o + beta A_d.  Terms are evaluated in FP64 for either path precision
 * and summed in a fixed order. */
int pimc_action(pimc_ctx* ctx, const pimc_model* model, const pimc_path* path,
                double* out3, void* stream);

/* Model checks of Section 6.  pimc_model_errors adds, for the current path,
 * the trapezoid model error eps_n (Section 2.1, components V, m, h, n) and
 * the observation error delta_n = y_n - V_n of every link n = 1..M to
 * esum[n-1][0..4] and their squares to esq[n-1][0..4] (device FP64 [M][5],
 * caller-owned, +=); called once per posterior sample, the sums give <eps_n>,
 * <delta_n> and their variances, which should be 0, 1/Rd and 1/Ro when the
 * model is right.  Terms in FP64 for either path precision. */
int pimc_model_errors(pimc_ctx* ctx, const pimc_model* model, const pimc_path* path, double* esum,
                      double* esq, void* stream);

/* Forecasts from the end of a window (Section 6): member b = 0..B-1 starts
 * at x0[b] (device FP64 [B][4]) with parameters p[b] (device FP64 [B][7])
 * and is integrated N steps of model->dt by Heun's method over the drive
 * I[0..N] (device FP64 [N+1], I[0] at the start time), adding per step the
 * model noise eps ~ N(0, 1/Rd) times `noise` (0: deterministic) from the
 * Philox block (index member0 + b, counter = step, tag 8, chain 0).  kin:
 * device [12] Table 1 constants or NULL (the model's).  out: device FP64
 * [B][N+1][4], the trajectory including the start.  FP64 throughout. */
int pimc_forecast(pimc_ctx* ctx, const pimc_model* model, int32_t B, const double* x0, const double* p,
                  const double* kin, const double* I, int64_t N, double noise, uint64_t seed, int64_t member0,
                  double* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * pimc_action without a context and without any allocation.  The FP64 block
 * partials of the reduction live in a fixed array inside the library
 * (256 KiB on each GPU it runs on, held until the process ends), so a window
 * may hold at most PIMC_NOALLOC_MAX_SITES sites (M + 1; PIMC_ERR_UNSUPPORTED
 * beyond).  Runs on the calling thread's current device; `stream` must belong
 * to it.  Every call on one GPU shares that array and it keeps the last
 * call's contents: calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller.  Result as pimc_action. */
#define PIMC_NOALLOC_MAX_SITES (4096 * 256)
int pimc_action_noalloc(const pimc_model* model, const pimc_path* path, double* out3, void* stream);

/* n_sweeps red-black Metropolis sweeps (Fig. 1; Sections 3.1, 4.1-4.2):
 * all even sites, then all odd sites (joint D-component proposal
 * x' = x + w z, box test, accept iff log u < -dA with dA in FP64 for the
 * decision), then -- if PIMC_PARAMS -- each sampled parameter in ascending
 * order.  w: device FP64 [11] = proposal widths of (V, m, h, n) then
 * (p1 .. p7), [23] with PIMC_KINETIC (then the 12 Table 1 constants).
 * stats and debug are nullable. */
int pimc_sweep(pimc_ctx* ctx, const pimc_model* model, pimc_path* path, pimc_rng rng,
               const double* w, int64_t n_sweeps, int32_t flags,
               const pimc_stats* stats, const pimc_debug* debug, void* stream);

/* State of the initialization phase (Section 4.2) for pimc_sweep_init.  The
 * scalars are host values read at each call; the five pointers are caller-
 * owned DEVICE memory that the call reads and updates, so consecutive calls
 * continue the phase (initialise beta = beta0, site_scale = 1, w_param = the
 * parameter widths, counts = 0 before the first call).
 *  - annealing: sweep k uses beta (in place of model->beta) as the
 *    multiplier of A_d; after every sweep beta <- min(1, beta f_beta) with
 *    f_beta = (1/beta0)^(1/n_cool) (eq. fbeta);
 *  - step sizes: after sweep k with k < n_init and (k + 1) % n_skip == 0,
 *    every step is scaled by 1 + alpha (N_acc / n_skip - f_acc) (the rule of
 *    Section 4.2; N_acc = accepted changes of that component since the last
 *    adjustment) and its count restarts.  The D components of a site move
 *    jointly with one decision, so they share N_acc: the step of component a
 *    at site n is w[a] * site_scale[n].  Parameter l uses w_param[l] (not
 *    w[4 + l]) and its own count.
 * Paper values (Section 5.1): beta0 = 0.01, n_cool = 1e5, n_init = 5e5,
 * n_skip = 400, f_acc = 0.23, alpha = 0.02. */
typedef struct {
  double beta0;        /* 0 < beta0 <= 1 */
  int64_t n_cool;      /* >= 1 */
  int64_t n_init;      /* >= 0 */
  int64_t n_skip;      /* >= 1 */
  double f_acc;        /* in [0, 1] */
  double alpha;        /* >= 0 */
  double* beta;        /* [1] FP64: beta of the next sweep */
  double* site_scale;  /* [M+1] FP64 */
  double* w_param;     /* [7] FP64 */
  int32_t* cnt_site;   /* [M+1] */
  int32_t* cnt_param;  /* [7] */
} pimc_init_phase;

/* pimc_sweep with the initialization phase of Section 4.2 (annealing of beta
 * and adjustment of the step sizes, see pimc_init_phase).  Runs in the launch
 * shapes of at most 256 threads per workgroup and at most 4 sites per thread
 * (the automatic choice, or time tiles); others return PIMC_ERR_UNSUPPORTED.
 * No debug record. */
int pimc_sweep_init(pimc_ctx* ctx, const pimc_model* model, pimc_path* path, pimc_rng rng,
                    const double* w, int64_t n_sweeps, int32_t flags, const pimc_init_phase* init,
                    const pimc_stats* stats, void* stream);

/* One round of sequential parameter moves (Fig. 1 step 3, Section 4.1) at
 * sweep index rng.sweep0, with the path held fixed; identical to pimc_sweep
 * with n_sweeps = 1 and flags = PIMC_PARAMS.  w as for pimc_sweep. */
int pimc_param_update(pimc_ctx* ctx, const pimc_model* model, pimc_path* path, pimc_rng rng,
                      const double* w, const pimc_debug* debug, void* stream);

/* Gradient of the action: gX [M+1][4] (path precision) <- dA/dX and
 * gp [7] FP64 <- dA/dp, from the local stencil of the trapezoid model error
 * (derivatives of A are what the force-bias / Hybrid Monte Carlo proposals
 * mentioned in Section 3.1 need). */
int pimc_grad(pimc_ctx* ctx, const pimc_model* model, const pimc_path* path,
              void* gX, double* gp, void* stream);

/* n_sweeps sweeps of every window of a packed batch in one persistent
 * launch (the batched workload).  All windows share model, seed and widths
 * w (device FP64 [11]); window w uses Philox chain id batch->chain[w] and
 * sweep indices sweep0 .. sweep0+n-1, so a window's chain equals its own
 * pimc_sweep run.  Windows run longest first, one workgroup each, or as
 * time tiles (see pimc_set_sweep_tiles).  When the launch gives 16 sites per
 * thread (FP32, untiled), each window runs with the fewest of 4, 8, 12, 16
 * sites per thread that the workgroup holds, so short windows finish early
 * (environment PIMC_BATCH_UNIFORM_K=1 keeps 16 for all).  The untiled launch is recorded
 * once per launch shape into a HIP graph and replayed with each call's
 * arguments; the batch layout (offsets) is copied to the device, with a
 * wait, only when it differs from the previous call's, so repeated calls on
 * the same windows are fully asynchronous (environment PIMC_NO_GRAPHS=1
 * launches directly).  Statistics as in pimc_batch_stats.  Errors: argument
 * errors and shapes the built kernels cannot run are returned before
 * anything is enqueued; device-side errors are reported by pimc_sync. */
int pimc_run_batch(pimc_ctx* ctx, const pimc_model* model, const pimc_batch* batch,
                   uint64_t seed, uint64_t sweep0, const double* w, int64_t n_sweeps,
                   int32_t flags, const pimc_batch_stats* stats, void* stream);

/* Statistics of pimc_hmc (every pointer nullable; device memory).
 *   acc     [B][PIMC_NACC] int64 (+=): [0] accepted proposals, [1] proposals
 *           whose trajectory was invalid (a coordinate outside its box after
 *           a reflection), [9] non-finite energy changes
 *   ptrace  [B][n_proposals][7] FP64: p after every proposal (written)
 *   dH      [B][n_proposals] FP64: H1 - H0 of every proposal (written)
 * Trajectory of the LAST proposal of the call, before its accept/reject
 * (for element-wise checks; nullable, all four or none):
 *   traj_q  [L+1][S][4] path precision: positions q(s) after drift s
 *           (q(0) = the start), S = offsets[B]
 *   traj_r  [L+1][S][4] path precision: momenta r(s+1/2) after kick s,
 *           r(L) for s = L
 *   traj_p  [L+1][B][7] FP64: parameters p(s)
 *   traj_rp [L+2][B][7] FP64: parameter momenta rp(0), rp(s-1/2) for
 *           s = 1..L, then rp(L) */
typedef struct {
  int64_t* acc;
  double* ptrace;
  double* dH;
  void* traj_q;
  void* traj_r;
  double* traj_p;
  double* traj_rp;
} pimc_hmc_stats;

/* n_proposals Hybrid Monte Carlo proposals (the Hybrid MC of Section 3, a
 * derivative-based proposal in the sense of Section 3.1) for every window of
 * a packed batch, on the coordinates (X, sampled p):
 *   momenta r ~ N(0, 1/minv) (Philox MOM / PMOM addresses of proposal k),
 *   L leapfrog steps of size eps driven by dA/d(X, p) (the local stencil of
 *   pimc_grad), H = A + 1/2 sum r^2 minv in FP64, accept iff log u < -dH
 *   (u at the HACC address) and the trajectory stayed valid.  A coordinate
 *   that a drift carries across a wall of its box is reflected back and its
 *   momentum component negated (Neal 2011, Section 5.1); one reflection per
 *   drift, and a coordinate still outside after it invalidates the
 *   trajectory.
 * Proposal indices are k0 .. k0 + n_proposals - 1.  minv: HOST FP64 [11],
 * inverse masses of (V, m, h, n) then p1..p7 (unsampled parameters never
 * move).  eps > 0, L >= 1.  Positions and parameters are updated in place.
 * With n_proposals > 1 the launches of one proposal are captured into a HIP
 * graph and replayed; the call then waits for the stream before returning
 * (environment PIMC_NO_GRAPHS=1 launches kernel by kernel instead). */
int pimc_hmc(pimc_ctx* ctx, const pimc_model* model, const pimc_batch* batch, uint64_t seed, uint64_t k0,
             double eps, int32_t L, const double* minv, int64_t n_proposals, const pimc_hmc_stats* stats,
             void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PIMC_H */
