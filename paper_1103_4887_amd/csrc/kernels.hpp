// Kernel argument blocks and launchers shared by the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"
#include "layout.hpp"

namespace pimc {

struct SweepArgs {
  ModelArgs m;
  Consts<float> cf;   // site constants, pre-converted on the host
  Consts<double> cd;
  // windows: offsets == nullptr means one window of M_single + 1 sites
  const int64_t* offsets;
  const int32_t* order;  // block -> window map (nullable: identity)
  const int8_t* blockK;  // block -> sites per thread, 4/8/12/16 (nullable: the launch's K; K = 16 launches only)
  int64_t M_single;
  void* X;
  double* p;
  const void* y;
  const void* I;
  const uint32_t* chain_ids;
  uint32_t chain_single;
  uint64_t seed;
  uint64_t sweep0;
  int64_t n_sweeps;
  int32_t flags;
  const double* w;  // [11]
  // statistics (nullable)
  double* sum;
  double* sumsq;
  const void* xref;
  double* ptrace;
  int64_t* acc;
  int64_t* kacc;      // [12] accepted moves of the Table 1 constants (nullable)
  int64_t burn;
  int64_t stride;     // statistics every stride-th sweep from burn on
  int32_t stage;      // sites per LDS staging chunk of the statistics pass
  double* batch;      // [nbatch][bslice] per-batch sums (nullable)
  int64_t nbatch;
  int64_t nsamp;      // statistics samples this call takes
  int64_t kfirst;     // sweep of the first of them
  int64_t bslice;     // elements of one batch slice (4 x sites)
  // last-sweep debug record (nullable)
  void* dbg_xprop;
  double* dbg_dA;
  uint8_t* dbg_acc;
  double* dbg_pprop;
  double* dbg_pdA;
  uint8_t* dbg_pacc;
  double* dbg_kprop;   // kinetic moves of the last sweep (extended kernels)
  double* dbg_kdA;
  uint8_t* dbg_kacc;
  double* kin;         // [12] Table 1 constants of the window (nullable: the model's), in/out
  uint32_t* err;  // bit 0: non-finite dA met, bit 1: entry state outside box, bit 2: wait timed out
  // time tiles (tiles == 1: a window is one workgroup, no global memory sync)
  int32_t tiles;
  int32_t ngroups;     // number of windows in the launch
  void* halo;          // [ngroups*tiles][2][SLOT_WORDS] generation words: first / last boundary site
  void* wpart;         // [2][ngroups][tiles][2 NRED] generation words: partial sums of the parameter statistics
  uint64_t* tsync;     // [ngroups*tiles] generation words: a tile's entry (payload: its entry check failed)
  uint32_t gen0;       // exchange generations of this call are gen0 + 1 .. gen0 + n_sweeps + 2
  uint64_t spin_ticks; // wall-clock ticks a wait may last
  // initialization phase (Section 4.2; used by the INIT kernels only)
  double ip_fbeta;     // beta grows by this factor after every sweep, capped at 1
  int64_t ip_ninit;    // steps are adjusted at sweeps k < ip_ninit ...
  int64_t ip_nskip;    // ... with (k + 1) % ip_nskip == 0
  double ip_facc, ip_alpha;
  double* ip_beta;     // [1] beta of the next sweep (in/out)
  double* ip_scale;    // [sites] per-site factor of the state steps (in/out)
  double* ip_wpar;     // [7] parameter steps (in/out)
  int32_t* ip_cnt;     // [sites] accepted site moves since the last adjustment (in/out)
  int32_t* ip_cntp;    // [7] accepted parameter moves since the last adjustment (in/out)
};

// ext: 0 the plain kernels; 1 the extended kernels (initialization phase,
// kinetic constants, exact draws); 2 the exact-draw kernels.  Extended
// kernels run in shapes of at most 256 threads and record the parameter and
// kinetic moves only.
int launch_sweep(const SweepArgs& a, bool fp64, int K, int nblocks, int NT, hipStream_t s, int ext = 0);
// Clear n 32-bit words of device memory in stream order (a kernel: the call
// may be recorded into a graph).
int clear_words(void* p, size_t n, hipStream_t s);

struct FieldArgs {  // action / gradient of one window
  ModelArgs m;
  int64_t M;
  const void* X;
  const double* p;
  const void* y;
  const void* I;
  const double* kin;  // [12] Table 1 constants (nullable: the model's)
  void* gX;         // gradient output (path precision), nullable
  double* partial;  // [nblocks][8] workspace
  double* out;      // action: [3]; gradient: gp [7]
};

constexpr int FIELD_BLOCK = 256;
int launch_action(const FieldArgs& a, bool fp64, hipStream_t s);
int launch_grad(const FieldArgs& a, bool fp64, hipStream_t s);
inline int64_t field_blocks(int64_t M) { return (M + 1 + FIELD_BLOCK - 1) / FIELD_BLOCK; }
// The fixed partials workspace of pimc_action_noalloc on the current device.
int noalloc_scratch(double** out);

struct ErrArgs {   // model and observation errors of one path, accumulated
  ModelArgs m;
  int64_t M;
  const void* X;
  const double* p;
  const void* y;
  const void* I;
  const double* kin;
  double* esum;     // [M][5]: eps (4 components), delta
  double* esq;      // [M][5]
};

struct FcstArgs {   // forecast ensemble (FP64)
  ModelArgs m;
  int32_t B;
  int64_t N;
  const double* x0;  // [B][4]
  const double* p;   // [B][7]
  const double* I;   // [N+1]
  const double* kin;
  double noise;
  uint64_t seed;
  int64_t member0;
  double* out;       // [B][N+1][4]
};

int launch_errors(const ErrArgs& a, bool fp64, hipStream_t s);
int launch_forecast(const FcstArgs& a, hipStream_t s);

}  // namespace pimc
