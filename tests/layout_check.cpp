// Host-side bounds check of the sweep kernel's launch shapes (test
// infrastructure; built with the host compiler and run by
// tests/test_layout_check.py, no GPU involved).
//
// For each case it takes the launch shape the C ABI would pick
// (choose_sweep_shape / choose_batch_shape, or a shape forced on the command
// line), walks every block and thread of the launch through the same
// ownership and layout functions the kernel calls (tile_sites, sweep_lds,
// halo_slot, wpart_block; layout.hpp) and checks, for every site and thread:
//   * the sites of a window are owned exactly once, in the colour they are
//     updated in, and every neighbour a site update reads comes from where
//     the kernel fetches it (own registers, the neighbouring thread's LDS
//     slot, the neighbouring tile's halo slot, the extra site);
//   * every LDS index the kernel forms (boundary sites, (y, I) with the two
//     halo sites, the block-reduction scratch, statistics, draws, counters,
//     staging) lies inside its buffer, the buffers lie inside the launch's
//     dynamic LDS and that fits the CU;
//   * every global index (path, observations, drive, moments, batch sums,
//     initialization-phase state, debug records, acceptance counters, halo,
//     partial-sum and entry words) lies inside the buffer the C ABI sizes.
// The access expressions below restate the kernel's (sweep_body.inc) phase
// by phase: entry, even half-sweep, odd half-sweep, link statistics, block
// reduction, all-reduce over tiles, kinetic moves, statistics, write-back.
//
// Input (stdin), one case a line:
//   single <M> <fp64> <tile_K> <tiles> [ext]  one window, shape as pimc_sweep picks it
//                                             (ext 1: for an extended kernel)
//   batch <fp64> <tile_K> <tiles> <uniK> <M1> ...  a batch, shape as pimc_run_batch picks it
//                                             (uniK 1: every window with the launch's K)
//   forced <M> <fp64> <K> <NT> <T>            one window in the given shape, checked
//                                             also when the library refuses to launch it
// Output: one line a case ("ok ...", "refused ...") and "FAIL ..." lines;
// the exit status is 1 if any check failed.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <iostream>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "layout.hpp"
#include "pimc.h"

using namespace pimc;

namespace {

long long g_checks = 0;
int g_fail = 0;
std::string g_case;

void fail(const char* what, long long a, long long b, long long c = 0) {
  if (g_fail < 40) std::printf("FAIL [%s] %s (%lld, %lld, %lld)\n", g_case.c_str(), what, a, b, c);
  ++g_fail;
}

// index i inside [0, n)
inline void in_range(const char* what, long long i, long long n, long long ctx = 0) {
  ++g_checks;
  if (i < 0 || i >= n) fail(what, i, n, ctx);
}

inline void require(bool ok, const char* what, long long a = 0, long long b = 0, long long c = 0) {
  ++g_checks;
  if (!ok) fail(what, a, b, c);
}

struct Launch {
  bool fp64;
  int K, NT, T, stage;
  bool batch;
  bool perK;
  std::vector<int64_t> Ms;       // window lengths (steps)
  std::vector<int64_t> offsets;  // site offsets of the windows
  std::vector<int> order;        // block group -> window
};

// The checks a launch passes through before anything runs (launch_sweep).
bool launch_accepted(const Launch& L, int ext) {
  const size_t sm = sweep_smem_bytes(L.NT, L.K, L.fp64, L.stage);
  if (sm + LDS_STATIC_RESERVE > LDS_BYTES || L.NT > sweep_max_threads(L.fp64, L.K)) return false;
  if (L.fp64 && (L.K != 4 || L.NT > 256)) return false;
  if (!L.fp64 && L.K == 2 && L.NT > 256) return false;
  if (ext && (L.NT > 256 || L.K > 4)) return false;
  return true;
}

// sites a published boundary slot holds: 7 values of one or two words
inline int slot_words_used(bool fp64) { return 7 * (fp64 ? 2 : 1); }

void check_launch(const Launch& L) {
  const int ts = L.fp64 ? 8 : 4;
  const int B = (int)L.Ms.size();
  const int T = L.T, NT = L.NT, NW = NT / 64;
  const int64_t total_sites = L.offsets[B];
  const size_t sm = sweep_smem_bytes(NT, L.K, L.fp64, L.stage);
  require(sm + LDS_STATIC_RESERVE <= LDS_BYTES, "LDS of the launch exceeds the CU", (long long)sm);
  require(NT % 64 == 0 && NT >= 64, "threads not whole waves", NT);
  require(L.stage >= 1, "empty staging chunk", L.stage);
  if (L.stage < 1) return;
  // tile buffers: a single window runs in the context's standing workspace
  // of MAX_TILES tiles over 4 groups; a batch sizes it as B T tiles over B
  const size_t ntiles = L.batch ? (size_t)B * T : (size_t)MAX_TILES;
  const int64_t ngroups = L.batch ? B : 1;
  require(T <= MAX_TILES, "more tiles than the workspace holds", T);

  for (int bi = 0; bi < B; ++bi) {
    const int win = L.order[bi];
    const int64_t base = L.offsets[win];
    const int M = (int)L.Ms[win];
    const int Kb = L.perK ? batch_block_K(M, NT) : L.K;
    require(Kb <= L.K && (Kb == 2 || Kb % 4 == 0), "per-window K not instantiated", Kb, L.K);
    // the layout this block's body uses must sit inside the launch's LDS
    const SweepLds lay = sweep_lds(NT, Kb, ts, 0);
    const SweepLds lay_launch = sweep_lds(NT, L.K, ts, L.stage);
    require(lay.lstage + (size_t)L.stage * 4 * ts <= lay_launch.end, "staging beyond the launch's LDS",
            lay.lstage, lay_launch.end);
    require(lay.lred % 8 == 0 && lay.lstat % 8 == 0 && lay.ldraw % 8 == 0, "FP64 LDS buffer misaligned", lay.lred);
    require(lay.lcnt % 4 == 0 && lay.lstage % ts == 0 && lay.lyi % ts == 0, "LDS buffer misaligned", lay.lcnt);
    const long long n_lfirst = (long long)NT * 8, n_lyi = 2LL * ((long long)NT * Kb + 2);
    const long long n_lred = (long long)NRED * 4 * NW;
    require(lay.llast - lay.lfirst == (size_t)n_lfirst * ts && lay.lyi - lay.llast == (size_t)n_lfirst * ts &&
                lay.lred - lay.lyi == (size_t)n_lyi * ts && lay.lstat - lay.lred == (size_t)n_lred * 8 &&
                lay.ldraw - lay.lstat == (size_t)NRED * 8 && lay.lcnt - lay.ldraw == (size_t)LDRAW * 8 &&
                lay.lstage - lay.lcnt == (size_t)LCNT * 4,
            "LDS buffers overlap");

    std::vector<int> owner(M + 1, 0);
    std::vector<int> tile_seen(T, 0);
    // launch-order block of each tile (the XCD-aware deal is a permutation)
    std::vector<int> block_of(T, -1);
    for (int bt = 0; bt < T; ++bt) {
      const int tb = tile_sites(M, Kb, NT, T, bt, 0).tb;
      if (tb >= 0 && tb < T) block_of[tb] = bt;
    }
    for (int bt = 0; bt < T; ++bt) {
      const TileSites t0 = tile_sites(M, Kb, NT, T, bt, 0);
      const int tb = t0.tb;
      in_range("tile index", tb, T, bt);
      if (tb >= 0 && tb < T) tile_seen[tb]++;
      const int S = t0.S, tile0 = t0.tile0;
      const bool last_tile = t0.last_tile;
      const int64_t gt = (int64_t)bi * T + tb;
      if (last_tile) {
        require(t0.NTneed >= 1 && t0.NTneed <= NT, "last tile needs more threads than it has", t0.NTneed, NT, M);
      } else {
        // the tile's last thread fetches the next tile's first site
        require(tile0 + S <= M, "tile beyond the window that is not the last", tile0, S, M);
      }
      // (y, I) loaded for sites lo .. hi (global index n -> lyi 2 (n - tile0 + 1))
      const int lo = tile0 > 0 ? tile0 - 1 : 0;
      const int hi = std::min(M, tile0 + S);
      auto lyb = [&](int n, int comp, const char* what) {
        const long long e = 2LL * (n - tile0 + 1) + comp;
        in_range(what, e, n_lyi, n);
        require(n >= lo && n <= hi, "(y, I) read of a site not loaded", n, lo, hi);
      };
      for (int n = lo; n <= hi; ++n) {
        lyb(n, 0, "lyi store y");
        lyb(n, 1, "lyi store I");
        in_range("y/I global read", base + n, total_sites, n);
      }
      // halo and entry words of this tile and its neighbours
      if (T > 1) {
        const int64_t hf = halo_slot(gt);
        const int64_t hl = hf + SLOT_WORDS;
        const int64_t hprev = tb > 0 ? hf - SLOT_WORDS : hl;
        const int64_t hnext = !last_tile ? hf + 2 * SLOT_WORDS : hf;
        for (int64_t h : {hf, hl, hprev, hnext}) {
          in_range("halo slot start", h, (long long)halo_words(ntiles), gt);
          in_range("halo slot end", h + slot_words_used(L.fp64) - 1, (long long)halo_words(ntiles), gt);
        }
        // a neighbour's slot belongs to the same window
        if (tb > 0) require(hprev >= halo_slot((int64_t)bi * T), "previous halo of another window", gt);
        if (!last_tile) require(hnext < halo_slot((int64_t)bi * T + T), "next halo of another window", gt);
        in_range("tsync own", gt, (long long)tsync_words(ntiles));
        for (int q = 0; q < T; ++q) in_range("tsync wait", (int64_t)bi * T + q, (long long)tsync_words(ntiles));
        // partial sums: both parities, own words and every tile's words
        for (uint32_t par = 0; par < 2; ++par) {
          const int64_t wp = wpart_block(par, ngroups, T, bi);
          for (int i = 0; i < 2 * NRED; ++i) in_range("wpart store", wp + (int64_t)tb * 2 * NRED + i,
                                                      (long long)wpart_words(ntiles), gt);
          for (int q = 0; q < T; ++q) {
            in_range("wpart read", wp + (int64_t)q * 2 * NRED, (long long)wpart_words(ntiles), gt);
            in_range("wpart read", wp + (int64_t)q * 2 * NRED + 2 * NRED - 1, (long long)wpart_words(ntiles), gt);
          }
          // the other windows' blocks do not overlap this one
          require(wp + (int64_t)T * 2 * NRED <= wpart_block(par, ngroups, T, bi + 1) ||
                      bi + 1 == ngroups,
                  "partial-sum blocks of two windows overlap", bi);
        }
        const int NSEG = NT / NRED;
        require(NSEG >= 1, "fewer threads than partial sums", NT);
        for (int sg = 0; sg < NSEG; ++sg)
          for (int v = 0; v < NRED; ++v) in_range("lred segment sums", (long long)sg * NRED + v, n_lred);
      }

      for (int t = 0; t < NT; ++t) {
        const TileSites o = tile_sites(M, Kb, NT, T, bt, t);
        const int wv = t >> 6;
        const int n0 = o.n0;
        require(o.tb == tb && o.S == S && o.tile0 == tile0, "ownership differs between threads of a block", t);
        require(n0 % 2 == 0, "first site of a thread is odd", n0);
        in_range("lfirst/llast own", (long long)t * 8 + 7, n_lfirst, t);
        // block reduction: wave totals (slot sl < 4 of row j < 9), kinetic sums
        for (int j = 0; j < (NRED + 3) / 4; ++j)
          for (int sl = 0; sl < 4; ++sl)
            in_range("lred wave totals", (long long)wv * 4 * ((NRED + 3) / 4) + 4 * j + sl, n_lred, t);
        in_range("lred kinetic", (long long)wv * 4 + 3, n_lred, t);
        if (NT > 256) {
          // wide shapes: the two halves of the sums (values 0..17, 18..34)
          // are folded and stored separately, each below its own count
          for (int lo : {0, 18}) {
            const int n = lo == 0 ? 18 : NRED - 18;
            for (int j = 0; j < (n + 3) / 4; ++j)
              for (int sl = 0; sl < 4; ++sl)
                if (4 * j + sl < n) {
                  const long long pos = lo + 4 * j + sl;
                  require(pos < NRED, "half-sum slot beyond the wave's values", pos);
                  in_range("lred half-sum totals", (long long)wv * 4 * ((NRED + 3) / 4) + pos, n_lred, t);
                }
          }
        }
        if (t < NRED) in_range("lstat", t, NRED);
        if (t < 2 * NRED) in_range("lstat words", t >> 1, NRED);
        if (t < 16) in_range("lcnt clear", t, LCNT);
        if (wv == 0 && (t & 63) < 7) in_range("ldraw", 32 + (t & 63), LDRAW);
        if (!o.active) {
          require(!o.has_extra, "inactive thread owns the extra site", t);
          continue;
        }
        for (int j = 0; j < Kb; ++j) {
          const int n = n0 + j;
          if (n > M) continue;
          in_range("site index", n, M + 1, t);
          if (n >= 0 && n <= M) owner[n]++;
          for (int c = 0; c < 4; ++c) {
            in_range("X", (base + n) * 4 + c, total_sites * 4, n);
            in_range("moments", (base + n) * 4 + c, total_sites * 4, n);
          }
          in_range("initialization-phase state", base + n, total_sites, n);
          in_range("debug record", base + n0 + j, total_sites, n);
          lyb(n, 0, "lyi own y");
          lyb(n, 1, "lyi own I");
          // colour: slot j is updated in the half-sweep of parity j
          require((n & 1) == (j & 1), "site updated in the wrong colour", n, j);
          // left neighbour
          if (n >= 1) {
            lyb(n - 1, 1, "lyi left I");
            if (j == 0) {
              if (t == 0) {
                require(tb > 0, "first site of tile 0 has a left neighbour", n);
                if (tb > 0 && block_of[tb - 1] >= 0) {
                  // the previous tile's last thread holds site n - 1 as its slot K - 1
                  const TileSites p = tile_sites(M, Kb, NT, T, block_of[tb - 1], NT - 1);
                  require(p.tb == tb - 1 && p.active && p.n0 + Kb - 1 == n - 1,
                          "previous tile's last site is not the left neighbour", n, p.n0);
                }
              } else {
                in_range("llast left", (long long)(t - 1) * 8 + 7, n_lfirst, t);
                const TileSites q = tile_sites(M, Kb, NT, T, bt, t - 1);
                require(q.active && q.n0 + Kb - 1 == n - 1, "left thread does not hold the left neighbour", n, t);
              }
            }
          }
          // right neighbour
          if (n + 1 <= M) {
            lyb(n + 1, 1, "lyi right I");
            if (j == Kb - 1) {
              if (o.has_extra) {
                require(n + 1 == M, "extra site is not the right neighbour", n, M);
              } else if (t == NT - 1) {
                require(!last_tile, "last tile's last thread fetches a next tile", n);
                if (!last_tile && block_of[tb + 1] >= 0) {
                  const TileSites q = tile_sites(M, Kb, NT, T, block_of[tb + 1], 0);
                  require(q.tb == tb + 1 && q.active && q.n0 == n + 1,
                          "next tile's first site is not the right neighbour", n, q.n0);
                }
              } else {
                in_range("lfirst right", (long long)(t + 1) * 8 + 7, n_lfirst, t);
                const TileSites q = tile_sites(M, Kb, NT, T, bt, t + 1);
                require(q.active && q.n0 == n + 1, "right thread does not hold the right neighbour", n, t);
              }
            }
          }
        }
        if (o.has_extra) {
          require(o.last_tile && t == o.NTneed - 1, "extra site outside the last thread", t);
          require(n0 + Kb == M, "extra slot is not site M", n0 + Kb, M);
          require(M % 2 == 0, "extra site is odd", M);
          require(n0 + Kb - 1 <= M, "extra site's left neighbour not owned", n0);
          if (M >= 0 && M <= (int)owner.size() - 1) owner[M]++;
          lyb(M, 0, "lyi extra y");
          lyb(M, 1, "lyi extra I");
          for (int c = 0; c < 4; ++c) in_range("X extra", (base + n0 + Kb) * 4 + c, total_sites * 4, M);
          in_range("initialization-phase state extra", base + M, total_sites, M);
          in_range("debug record extra", base + n0 + Kb, total_sites, M);
        } else {
          lyb(tile0, 1, "lyi placeholder of the extra site");
        }
      }
      // statistics staging: chunks c0 .. c0 + stage - 1 of the tile's sites
      const int hi_site = last_tile ? M : tile0 + S - 1;
      for (int c0 = tile0; c0 <= hi_site; c0 += L.stage) {
        const int cnt = 4 * std::min(L.stage, hi_site + 1 - c0);
        in_range("staging count", cnt - 1, 4LL * L.stage, c0);
        in_range("moment chunk end", base * 4 + (int64_t)c0 * 4 + cnt - 1, total_sites * 4, c0);
      }
    }
    for (int tb = 0; tb < T; ++tb) require(tile_seen[tb] == 1, "tile not launched exactly once", tb, tile_seen[tb]);
    for (int n = 0; n <= M; ++n)
      if (owner[n] != 1) {
        fail("site not owned exactly once", n, owner[n], M);
        break;
      }
    // per-window records
    in_range("acceptance counters", (int64_t)win * PIMC_NACC + PIMC_NACC - 1, (int64_t)B * PIMC_NACC);
    in_range("parameters", (int64_t)win * 7 + 6, (int64_t)B * 7);
  }
}

std::vector<int64_t> offsets_of(const std::vector<int64_t>& Ms) {
  std::vector<int64_t> off(Ms.size() + 1, 0);
  for (size_t i = 0; i < Ms.size(); ++i) off[i + 1] = off[i] + Ms[i] + 1;
  return off;
}

}  // namespace

int main() {
  std::string line;
  int cases = 0, refused = 0;
  while (std::getline(std::cin, line)) {
    std::istringstream in(line);
    std::string kind;
    if (!(in >> kind) || kind[0] == '#') continue;
    Launch L{};
    int fp64 = 0, tile_K = 0, tiles = 0, uniK = 0, ext = 0;
    SweepShape sh{};
    if (kind == "single") {
      int64_t M;
      in >> M >> fp64 >> tile_K >> tiles;
      if (!(in >> ext)) ext = 0;
      L.Ms = {M};
      sh = choose_sweep_shape(M, fp64 != 0, true, tile_K, tiles, ext != 0);
      L.batch = false;
    } else if (kind == "batch") {
      in >> fp64 >> tile_K >> tiles >> uniK;
      int64_t M;
      while (in >> M) L.Ms.push_back(M);
      sh = choose_batch_shape(L.Ms.data(), (int)L.Ms.size(), fp64 != 0, tile_K, tiles);
      L.batch = true;
    } else if (kind == "forced") {
      int64_t M;
      in >> M >> fp64 >> sh.K >> sh.NT >> sh.T;
      L.Ms = {M};
      sh.stage = (int)stage_room(sh.NT, sh.K, fp64 != 0);
      L.batch = false;
    } else {
      std::printf("FAIL bad input line: %s\n", line.c_str());
      ++g_fail;
      continue;
    }
    g_case = line.substr(0, 60);
    ++cases;
    L.fp64 = fp64 != 0;
    L.K = sh.K;
    L.NT = sh.NT;
    L.T = sh.T;
    L.stage = sh.stage;
    const bool accepted = sh.K && launch_accepted(L, ext);
    if (!accepted) ++refused;
    if (!sh.K || (!accepted && kind != "forced")) {
      std::printf("refused %s\n", g_case.c_str());
      continue;
    }
    L.offsets = offsets_of(L.Ms);
    L.order.resize(L.Ms.size());
    std::iota(L.order.begin(), L.order.end(), 0);
    if (L.batch)
      std::stable_sort(L.order.begin(), L.order.end(), [&](int x, int y) { return L.Ms[x] > L.Ms[y]; });
    L.perK = L.batch && L.T == 1 && !L.fp64 && L.K == 16 && !uniK;
    const long long before = g_checks;
    const int fails = g_fail;
    check_launch(L);
    std::printf("%s %s K=%d NT=%d T=%d stage=%d LDS=%zu checks=%lld%s\n", g_fail == fails ? "ok" : "bad",
                g_case.c_str(), L.K, L.NT, L.T, L.stage, sweep_smem_bytes(L.NT, L.K, L.fp64, L.stage),
                g_checks - before, accepted ? "" : " (a shape launch_sweep refuses)");
  }
  std::printf("cases=%d refused=%d checks=%lld failures=%d\n", cases, refused, g_checks, g_fail);
  return g_fail ? 1 : 0;
}
