// Index arithmetic and launch shapes of the sweep kernel, in a form a host
// program can run too: which sites a thread of a time tile owns, where the
// kernel's LDS buffers lie, the word offsets of the cross-tile exchange
// buffers and their sizes, and the launch shape the C ABI picks for a
// window.  The kernel (sweep_body.inc) and the C-ABI layer (api.hip) use
// these functions; the host-side bounds check of the launch shapes
// (tests/layout_check.cpp) calls the same ones.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pimc {

constexpr int NRED = 35;          // parameter statistics: 7 (s) + 28 (upper triangle of G)
constexpr int SLOT_WORDS = 16;    // one published site: 7 values, two words each in FP64
constexpr int LDRAW = 40;         // doubles of the parameter-draw area
constexpr int LCNT = 16;          // ints of the counter area
constexpr size_t LDS_BYTES = 160 * 1024;     // LDS per CU on gfx950
constexpr size_t LDS_STATIC_RESERVE = 1024;  // kept free for the kernels' static LDS
constexpr int MAX_TILES = 256;    // time tiles per window

// The sites of thread t in a time tile.  A window of M + 1 sites is cut into
// `tiles` tiles of S = NT K sites; block_tile is the block's tile index in
// launch order (consecutive tiles are dealt to consecutive blocks of one XCD
// when the tile count allows).  Thread t owns sites n0 .. n0 + K - 1 (those
// <= M); the last tile's last thread also owns site M when the regular slots
// stop exactly at M (has_extra).
struct TileSites {
  int tb;          // tile of the window
  int S, tile0;    // sites per tile, first site of the tile
  bool last_tile;
  int NTneed;      // threads that own sites
  int n0;          // first site of the thread
  bool active, has_extra;
};

__host__ __device__ inline TileSites tile_sites(int M, int K, int NT, int tiles, int block_tile, int t) {
  TileSites s;
  int tb = block_tile;
  if (tiles % 8 == 0 && tiles > 8) tb = (tb % 8) * (tiles / 8) + tb / 8;
  s.tb = tb;
  s.S = NT * K;
  s.tile0 = tb * s.S;
  s.last_tile = tb == tiles - 1;
  s.NTneed = s.last_tile ? (M - s.tile0 + K - 1) / K : NT;
  s.active = t < s.NTneed;
  s.n0 = s.tile0 + t * K;
  s.has_extra = s.last_tile && (t == s.NTneed - 1) && (K * s.NTneed == M - s.tile0);
  return s;
}

// Byte offsets of the kernel's LDS buffers for NT threads, K sites per
// thread, site values of ts bytes and a statistics staging chunk of `stage`
// sites:
//   lfirst [NT][8], llast [NT][8]  the first and last site of each thread
//                                  (x, then the gates' F)
//   lyi    [NT K + 2][2]           (y_n, I_n) of the tile and its two halo sites
//   lred   [4 NW][NRED] FP64       block-reduction scratch (NW = NT / 64)
//   lstat  [NRED] FP64             the reduced statistics
//   ldraw  [LDRAW] FP64            parameter draws
//   lcnt   [LCNT] int              counters
//   lstage [stage][4]              statistics staging
struct SweepLds {
  uint32_t lfirst, llast, lyi, lred, lstat, ldraw, lcnt, lstage, end;
};

__host__ __device__ inline SweepLds sweep_lds(int NT, int K, int ts, int stage) {
  SweepLds l;
  const uint32_t NW = (uint32_t)NT / 64;
  l.lfirst = 0;
  l.llast = l.lfirst + (uint32_t)NT * 8 * ts;
  l.lyi = l.llast + (uint32_t)NT * 8 * ts;
  l.lred = l.lyi + 2 * ((uint32_t)NT * K + 2) * ts;
  l.lstat = l.lred + (uint32_t)NRED * 4 * NW * 8;
  l.ldraw = l.lstat + (uint32_t)NRED * 8;
  l.lcnt = l.ldraw + (uint32_t)LDRAW * 8;
  l.lstage = l.lcnt + (uint32_t)LCNT * 4;
  l.end = l.lstage + (uint32_t)stage * 4 * ts;
  return l;
}

inline size_t sweep_smem_bytes(int NT, int K, bool fp64, int stage) {
  return (size_t)sweep_lds(NT, K, fp64 ? 8 : 4, stage).end;
}

// ---- cross-tile exchange buffers (64-bit generation words) ----------------
// halo  [ntiles][2][SLOT_WORDS]  first / last boundary site of each tile
// wpart [2][ngroups][tiles][2 NRED]  partial sums, double-buffered by the
//                                    parity of the all-reduce count
// tsync [ntiles]                 a tile's entry word
// ntiles = ngroups tiles, the tiles of all windows of a launch.
__host__ __device__ inline size_t halo_words(size_t ntiles) { return ntiles * 2 * SLOT_WORDS; }
__host__ __device__ inline size_t wpart_words(size_t ntiles) { return 2 * ntiles * 2 * NRED; }
__host__ __device__ inline size_t tsync_words(size_t ntiles) { return ntiles; }

// first halo word of global tile gt (its first site; the last site follows
// SLOT_WORDS words later)
__host__ __device__ inline int64_t halo_slot(int64_t gt) { return gt * 2 * SLOT_WORDS; }

// first wpart word of window bi's tiles in the buffer half of the given
// parity; tile q's 2 NRED words follow at q 2 NRED
__host__ __device__ inline int64_t wpart_block(uint32_t parity, int64_t ngroups, int64_t tiles, int64_t bi) {
  return ((int64_t)parity * ngroups * tiles + bi * tiles) * (2 * NRED);
}

// ---- launch shapes (host) -------------------------------------------------
// Threads per workgroup each sites-per-thread instantiation is built for.
inline int sweep_max_threads(bool fp64, int K) {
  if (fp64) return K == 4 ? 256 : 0;
  if (K == 2) return 256;
  if (K == 4) return 1024;
  if (K == 8 || K == 16) return 512;
  return 0;
}

// Statistics staging chunk: the LDS left after the kernel's other buffers.
inline int64_t stage_room(int NT, int K, bool fp64) {
  const size_t base = sweep_smem_bytes(NT, K, fp64, 0) + LDS_STATIC_RESERVE;
  if (base >= LDS_BYTES) return 0;
  const int64_t ts = fp64 ? 8 : 4;
  const int64_t room = (int64_t)(LDS_BYTES - base) / (4 * ts);
  const int64_t want = (int64_t)NT * K + 1;
  return want < room ? want : room;
}

struct SweepShape {
  int K;       // sites per thread (0: no shape)
  int NT;      // threads per workgroup
  int stage;   // sites per statistics staging chunk
  int T;       // time tiles per window
};

// Launch shape of the sweep kernel for windows of up to maxM steps: sites per
// thread K, threads NT and time tiles T (workgroups per window, tiles of
// S = NT K sites with (T-1) S < M <= T S).  tile_K forces K (0: free);
// tiles: 0 automatic, 1 one workgroup per window, > 1 that many tiles.
// Automatic choice: one workgroup per window with the smallest K that keeps
// it within 256 threads (one wave per SIMD, no register spills), else (when
// tiles may not be used) any single-workgroup shape; windows too long for one
// 256-thread workgroup are cut into tiles of at most 256 threads.  ext: the
// shape of an extended kernel (exact draws, initialization phase, Table 1
// constants), at most 256 threads and at most 4 sites per thread.
inline SweepShape choose_sweep_shape(int64_t maxM, bool fp64, bool allow_tiles, int tile_K, int tiles,
                                     bool ext = false) {
  SweepShape sh{0, 0, 0, 1};
  // K = 2 (FP32 only) is never the automatic choice: it is a tuning option
  // for windows cut into many tiles, where it halves the sites per thread
  static const int cand32[] = {4, 8, 16, 2};
  // FP64 runs only in the spill-free shape (4 sites per thread, at most 256
  // threads): the wider FP64 shapes spill about 1 KB per thread to scratch,
  // and a GPU fault met with FP64 windows beyond one 256-thread workgroup
  // has no identified cause, so they are not launched
  static const int cand64[] = {4};
  const int* cand = fp64 ? cand64 : cand32;
  const int nc = fp64 ? 1 : (tile_K == 2 ? 4 : 3);
  const int want_T = allow_tiles ? tiles : 1;
  if (want_T <= 1) {
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = 0; i < nc; ++i) {
        const int K = cand[i];
        if ((tile_K && tile_K != K) || (ext && K > 4)) continue;
        const int64_t need = (maxM + K - 1) / K;
        const int64_t nt = need > 64 ? (need + 63) / 64 * 64 : 64;
        // wide single-workgroup shapes (more than 256 threads) spill to
        // scratch: FP64 never uses them, and an FP32 window that may be cut
        // into time tiles (automatic choice) is tiled instead
        if (pass == 1 && (fp64 || ext || (allow_tiles && want_T == 0))) continue;
        const int64_t lim = pass == 0 ? 256 : sweep_max_threads(fp64, K);
        if (nt > lim) continue;
        const int64_t st = stage_room((int)nt, K, fp64);
        if (st < 64) continue;
        sh.K = K;
        sh.NT = (int)nt;
        sh.stage = (int)st;
        sh.T = 1;
        return sh;
      }
    }
    if (want_T == 1 || !allow_tiles) return sh;
  }
  // FP64 windows are never cut into time tiles (the same unexplained fault)
  if (fp64) return sh;
  // tiled: the requested T, or the fewest tiles of at most 256 threads
  for (int Tt = want_T > 1 ? want_T : 2; Tt <= MAX_TILES; ++Tt) {
    for (int i = 0; i < nc; ++i) {
      const int K = cand[i];
      if ((tile_K && tile_K != K) || (ext && K > 4)) continue;
      for (int nt = 256; nt >= 64; nt -= 64) {
        const int64_t S = (int64_t)nt * K;
        if (!((Tt - 1) * S < maxM && maxM <= Tt * S)) continue;
        const int64_t st = stage_room(nt, K, fp64);
        if (st < 64) continue;
        sh.K = K;
        sh.NT = nt;
        sh.stage = (int)st;
        sh.T = Tt;
        return sh;
      }
    }
    if (want_T > 1) return sh;
  }
  return sh;
}

// Launch shape of a batch of B windows of Ms[i] steps: time tiles (tiles > 1,
// FP32) when every window needs exactly that many tiles of the shape chosen
// for the longest, else one workgroup per window.
inline SweepShape choose_batch_shape(const int64_t* Ms, int B, bool fp64, int tile_K, int tiles, bool ext = false) {
  int64_t maxM = 0;
  for (int i = 0; i < B; ++i) maxM = Ms[i] > maxM ? Ms[i] : maxM;
  SweepShape sh{0, 0, 0, 1};
  if (tiles > 1 && !fp64) {
    sh = choose_sweep_shape(maxM, fp64, true, tile_K, tiles, ext);
    const int64_t S = (int64_t)sh.NT * sh.K;
    for (int i = 0; sh.K && i < B; ++i)
      if (!((sh.T - 1) * S < Ms[i] && Ms[i] <= sh.T * S)) sh.K = 0;
  }
  if (!sh.K) sh = choose_sweep_shape(maxM, fp64, false, tile_K, tiles, ext);
  return sh;
}

// A batch launched with 16 sites per thread runs each window (M steps) with
// the fewest of 4, 8, 12, 16 sites per thread that NT threads hold.
inline int batch_block_K(int64_t M, int NT) {
  for (int c : {4, 8, 12})
    if ((int64_t)c * NT >= M) return c;
  return 16;
}

}  // namespace pimc
