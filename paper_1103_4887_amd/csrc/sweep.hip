// Red-black Metropolis sweep of a whole window in one persistent launch.
//
// Method (Quinn & Abarbanel, Fig. 1 and Sections 3.1, 4.1-4.2): every even
// site, then every odd site, proposes x' = x + w z for all four components
// at once and accepts with probability min(1, exp(-dA)); then every sampled
// parameter is moved in turn against the change of the whole action.
//
// MI355X layout (differs from the paper's one-thread-per-site kernels):
//  * one workgroup owns a whole window; thread t owns the K consecutive sites
//    n = K t .. K t + K - 1 in registers (x, cached F(x), y, I), plus site M
//    when the regular slots end exactly at M;
//  * the only cross-thread data of a half-sweep is one neighbour site per
//    thread, exchanged through LDS; the colours are separated by workgroup
//    barriers instead of separate kernel launches;
//  * dA of a site is formed from the differences dx and dF directly
//    (d eps = +-dx - dt/2 dF, eps'^2 - eps^2 = d eps (2 eps + d eps)), which
//    keeps FP32 site arithmetic accurate; the decision log u < -dA is FP64;
//  * the parameters enter dV/dt linearly through theta = (p1, p2, p2 p3, p4,
//    p4 p5, p6, p6 p7), so the change of A under any parameter move follows
//    exactly from the FP64 sums s = sum phi_n eps_n,V and G = sum phi_n phi_n^T
//    (phi_n = dt/2 (psi_n + psi_{n-1})):  dA = beta Rd_V / 2 (dth^T G dth -
//    2 dth . s); after an accepted move s <- s - G dth.  The sums are
//    accumulated during the odd half-sweep, which replaces the paper's N_p
//    full passes and N_p global synchronisations with one block reduction.
#include "device.hpp"
#include "kernels.hpp"

namespace pimc {

namespace {

constexpr int NRED = 35;  // 7 (s) + 28 (upper triangle of G)

template <typename T>
struct Nb {  // a neighbour site: state and cached F
  T x[4];
  T F[4];
};

// Wave-uniform values that the site updates read on every iteration are
// held in vector registers: the kernel's uniform state (pointers, counters,
// model constants) exceeds the scalar register file, and values the compiler
// leaves in scalar registers are then spilled to vector lanes and read back
// with one v_readlane per use.  The copy goes through an opaque move, so the
// compiler cannot turn it back into a scalar.
__device__ __forceinline__ float in_vgpr(float x) {
  float r;
  asm("v_mov_b32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}
__device__ __forceinline__ double in_vgpr(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = __builtin_bit_cast(uint32_t, in_vgpr(__builtin_bit_cast(float, (uint32_t)b)));
  const uint32_t hi = __builtin_bit_cast(uint32_t, in_vgpr(__builtin_bit_cast(float, (uint32_t)(b >> 32))));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ void consts_in_vgprs(Consts<T>& C) {
  C.h = in_vgpr(C.h);
  C.half_Ro = in_vgpr(C.half_Ro);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    C.half_beta_Rd[a] = in_vgpr(C.half_beta_Rd[a]);
    C.lo[a] = in_vgpr(C.lo[a]);
    C.hi[a] = in_vgpr(C.hi[a]);
  }
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    C.Va[g] = in_vgpr(C.Va[g]);
    C.inv_dVa[g] = in_vgpr(C.inv_dVa[g]);
    C.tau0[g] = in_vgpr(C.tau0[g]);
    C.tau1[g] = in_vgpr(C.tau1[g]);
  }
#pragma unroll
  for (int l = 0; l < 7; ++l) C.p[l] = in_vgpr(C.p[l]);
}


// Accept iff log u < -dA, decided in FP64.  log u is first formed in FP32
// (hardware log2); only when -dA lies within a margin far wider than that
// estimate's error is the FP64 logarithm evaluated, so the decision is the
// FP64 one at a fraction of its cost.
__device__ __forceinline__ bool accept_u(uint32_t uword, double dA) {
  const float lu32 = __builtin_amdgcn_logf(u01_f(uword)) * 0.6931471805599453f;
  const double gap = -dA - (double)lu32;
  const double E = 1e-5 * (1.0 + (double)__builtin_fabsf(lu32));
  if (gap > E) return true;
  if (gap < -E) return false;
  return ::log(u01_d(uword)) < -dA;
}

// Spin until *p >= target (agent-scope acquire).  Every wait is bounded: past
// `ticks` of the constant wall clock the error flag gets bit 2 and the wait
// gives up, so a workgroup can never wait forever on a missing partner.
__device__ __forceinline__ void wait_ge(uint32_t* p, uint32_t target, uint32_t* err, uint64_t ticks) {
  if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target &&
      !(__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 4u)) {
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (wall_clock64() - t0 > ticks) {
        atomicOr(err, 4u);
        break;
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Barrier across the tiles of one window: a monotonic arrival counter.
__device__ __forceinline__ void tile_barrier(uint32_t* cnt, uint32_t target, uint32_t* err, uint64_t ticks) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    wait_ge(cnt, target, err, ticks);
  }
  __syncthreads();
}

// One Metropolis site update.  Returns true on accept (x, F replaced).
template <typename T>
__device__ __forceinline__ bool site_update(const Consts<T>& C, const T (&w)[4], bool uniform_prop,
                                            T (&x)[4], T (&F)[4], T y, T I, bool hasL, const Nb<T>& L,
                                            bool hasR, const Nb<T>& R, bool hasObs, const U4& blk,
                                            uint32_t uword, double& dA_out, T (&xp)[4], int& nonfinite) {
  T z[4];
  if (uniform_prop) {
    z[0] = Math<T>::uniform_pm1(blk.x);
    z[1] = Math<T>::uniform_pm1(blk.y);
    z[2] = Math<T>::uniform_pm1(blk.z);
    z[3] = Math<T>::uniform_pm1(blk.w);
  } else {
    Math<T>::box_muller(blk.x, blk.y, z[0], z[1]);
    Math<T>::box_muller(blk.z, blk.w, z[2], z[3]);
  }
  bool inbox = true;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    xp[a] = x[a] + w[a] * z[a];
    inbox = inbox && (xp[a] >= C.lo[a]) && (xp[a] <= C.hi[a]);
  }
  T Fp[4], dx[4], dF[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) dx[a] = xp[a] - x[a];
  if constexpr (sizeof(T) == 4) {
    hh_F_dF(C, x, xp, I, Fp, dF);
  } else {
    hh_F(C, xp, I, Fp);
#pragma unroll
    for (int a = 0; a < 4; ++a) dF[a] = Fp[a] - F[a];
  }
  T sdyn = (T)0;
  if (hasL) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const T e = (x[a] - L.x[a]) - C.h * (F[a] + L.F[a]);
      const T de = dx[a] - C.h * dF[a];
      sdyn += C.half_beta_Rd[a] * de * ((T)2 * e + de);
    }
  }
  if (hasR) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const T e = (R.x[a] - x[a]) - C.h * (R.F[a] + F[a]);
      const T de = -dx[a] - C.h * dF[a];
      sdyn += C.half_beta_Rd[a] * de * ((T)2 * e + de);
    }
  }
  T sobs = (T)0;
  if (hasObs) sobs = C.half_Ro * dx[0] * (dx[0] - (T)2 * (y - x[0]));
  double dA = (double)sdyn + (double)sobs;
  const bool fin = __builtin_isfinite(dA);
  const bool acc = inbox && fin && accept_u(uword, dA);
  if (inbox && !fin) ++nonfinite;
  dA_out = inbox ? dA : __builtin_nan("");
  if (acc) {
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      x[a] = xp[a];
      F[a] = Fp[a];
    }
  }
  return acc;
}

template <typename T>
__device__ __forceinline__ void lds_put(T* slot, const T (&x)[4], const T (&F)[4]) {
#pragma unroll
  for (int a = 0; a < 4; ++a) slot[a] = x[a];
  slot[4] = F[1];
  slot[5] = F[2];
  slot[6] = F[3];
}

// Neighbour from LDS: gates' F are cached, dV/dt is recomputed with the
// current parameters (so a parameter change never needs a re-publish).
template <typename T>
__device__ __forceinline__ void lds_get(const Consts<T>& C, const T* slot, T I, Nb<T>& nb) {
#pragma unroll
  for (int a = 0; a < 4; ++a) nb.x[a] = slot[a];
  nb.F[1] = slot[4];
  nb.F[2] = slot[5];
  nb.F[3] = slot[6];
  nb.F[0] = hh_FV(C, nb.x[0], nb.x[1], nb.x[2], nb.x[3], I);
}

// ---- exchange between the time tiles of a window -------------------------
// Every value crosses as "generation words": a 32-bit payload and the 32-bit
// generation it belongs to, written and read as one 64-bit relaxed atomic at
// agent scope.  A reader that sees the generation it waits for holds that
// generation's payload, so neither a separate flag nor a release/acquire
// fence (an L2 write-back and invalidate on this chip) is needed: one
// memory round trip per exchange.  The protocol guarantees that a slot is
// never overwritten by a later generation before its reader has consumed it
// (boundary sites: the writer needs the reader's progress first; partial
// sums: double-buffered by sweep parity).
constexpr int SLOT_WORDS = 16;   // one site: 7 values, two words each in FP64

__device__ __forceinline__ uint64_t gen_word(uint32_t gen, uint32_t payload) {
  return ((uint64_t)gen << 32) | payload;
}
__device__ __forceinline__ void gw_store(uint64_t* p, uint64_t w) {
  __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t gw_load(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Load n words (all in flight together) until each carries generation >= gen.
// A wait that outlasts `ticks` sets error bit 4 and returns what it has.
template <int N>
__device__ __forceinline__ void gw_wait(const uint64_t* const (&src)[N], uint64_t (&w)[N], uint32_t gen,
                                        uint32_t* err, uint64_t ticks) {
  bool ok = true;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    w[i] = gw_load(src[i]);
    ok = ok && (uint32_t)(w[i] >> 32) >= gen;
  }
  if (ok) return;
  const uint64_t t0 = wall_clock64();
  while (true) {
    __builtin_amdgcn_s_sleep(1);
    ok = true;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      w[i] = gw_load(src[i]);
      ok = ok && (uint32_t)(w[i] >> 32) >= gen;
    }
    if (ok) return;
    const uint64_t el = wall_clock64() - t0;
    // after one timed-out wait, every later wait gives up once it has
    // waited a small fraction of the limit, so a broken exchange ends the
    // launch quickly (with the error reported)
    if (el > (ticks >> 16) && (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 4u)) return;
    if (el > ticks) {
      atomicOr(err, 4u);
      return;
    }
  }
}

// Publish a boundary site (x and the gates' F) as generation `gen`.
template <typename T>
__device__ __forceinline__ void site_publish(uint64_t* slot, const T (&x)[4], const T (&F)[4], uint32_t gen) {
  const T v[7] = {x[0], x[1], x[2], x[3], F[1], F[2], F[3]};
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    if constexpr (sizeof(T) == 4) {
      gw_store(slot + i, gen_word(gen, __builtin_bit_cast(uint32_t, v[i])));
    } else {
      const uint64_t b = __builtin_bit_cast(uint64_t, v[i]);
      gw_store(slot + 2 * i, gen_word(gen, (uint32_t)b));
      gw_store(slot + 2 * i + 1, gen_word(gen, (uint32_t)(b >> 32)));
    }
  }
}

// Wait for generation `gen` of a published boundary site and read it (dV/dt
// recomputed with the current parameters, as for an LDS neighbour).
template <typename T>
__device__ __forceinline__ void site_fetch(const Consts<T>& C, const uint64_t* slot, uint32_t gen, T I, Nb<T>& nb,
                                           uint32_t* err, uint64_t ticks) {
  constexpr int N = sizeof(T) == 4 ? 7 : 14;
  const uint64_t* src[N];
#pragma unroll
  for (int i = 0; i < N; ++i) src[i] = slot + i;
  uint64_t w[N];
  gw_wait<N>(src, w, gen, err, ticks);
  T v[7];
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    if constexpr (sizeof(T) == 4)
      v[i] = __builtin_bit_cast(T, (uint32_t)w[i]);
    else
      v[i] = __builtin_bit_cast(T, ((uint64_t)(uint32_t)w[2 * i + 1] << 32) | (uint32_t)w[2 * i]);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) nb.x[a] = v[a];
  nb.F[1] = v[4];
  nb.F[2] = v[5];
  nb.F[3] = v[6];
  nb.F[0] = hh_FV(C, nb.x[0], nb.x[1], nb.x[2], nb.x[3], I);
}

// Hide a value from loop-invariant code motion.  Without it the compiler
// hoists the sweep-independent first Philox round of every owned site (and
// the data-only parts of the parameter statistics) out of the sweep loop and
// spills the result; recomputing them is cheaper than the spill traffic.
template <typename U>
__device__ __forceinline__ U opaque(U v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Per-site features needed by the parameter statistics: (I, V, m^3 h, n^4).
struct Feat {
  double I, V, m3h, n4;
};

template <typename T>
__device__ __forceinline__ Feat feat_of(const T (&x)[4], T I) {
  const double m = (double)x[1], n = (double)x[3];
  const double n2 = n * n;
  return Feat{(double)opaque(I), (double)x[0], m * m * m * (double)x[2], n2 * n2};
}

// Link (n-1 -> n) contribution to the parameter sufficient statistics:
// phi = dt/2 (psi_n + psi_{n-1}) with psi = (I, -m^3hV, m^3h, -n^4V, n^4, -V, 1),
// eps_V = (V_n - V_{n-1}) - theta . phi;  s += phi eps_V;  G += phi phi^T.
__device__ __forceinline__ void link_stats(const double (&th)[7], double h, const Feat& l, const Feat& r,
                                           double (&acc)[NRED]) {
  double phi[7];
  phi[0] = h * (r.I + l.I);
  phi[1] = -h * (r.m3h * r.V + l.m3h * l.V);
  phi[2] = h * (r.m3h + l.m3h);
  phi[3] = -h * (r.n4 * r.V + l.n4 * l.V);
  phi[4] = h * (r.n4 + l.n4);
  phi[5] = -h * (r.V + l.V);
  phi[6] = 2.0 * h;
  double thphi = 0.0;
#pragma unroll
  for (int q = 0; q < 7; ++q) thphi += th[q] * phi[q];
  const double e = (r.V - l.V) - thphi;
#pragma unroll
  for (int q = 0; q < 7; ++q) acc[q] += phi[q] * e;
#pragma unroll
  for (int a = 0; a < 7; ++a)
#pragma unroll
    for (int b = a; b < 7; ++b) acc[7 + sym7(a, b)] += phi[a] * phi[b];
}

// theta components moved by a change dp of parameter l (0-based), with the
// current parameters p:  theta = (p1, p2, p2 p3, p4, p4 p5, p6, p6 p7).
template <int L>
struct ThetaMove;
template <> struct ThetaMove<0> { static constexpr int ia = 0, ib = -1; };
template <> struct ThetaMove<1> { static constexpr int ia = 1, ib = 2; };
template <> struct ThetaMove<2> { static constexpr int ia = 2, ib = -1; };
template <> struct ThetaMove<3> { static constexpr int ia = 3, ib = 4; };
template <> struct ThetaMove<4> { static constexpr int ia = 4, ib = -1; };
template <> struct ThetaMove<5> { static constexpr int ia = 5, ib = 6; };
template <> struct ThetaMove<6> { static constexpr int ia = 6, ib = -1; };

__host__ __device__ constexpr int symi(int a, int b) { return a <= b ? sym7(a, b) : sym7(b, a); }

// One Metropolis move of parameter L against the sufficient statistics.
// pl: proposed value, drawn and box-tested beforehand (a move of p_l leaves
// every other p_j unchanged, so p_l before its own move is known when the
// sweep's parameter section starts); NaN when outside the box.  lu: FP64
// log u of the accept uniform, also formed beforehand (lane-parallel).
// cA = beta Rd_V / 2.  Written without branches, to keep the sequential
// chain of the seven moves short.
template <int L, bool DBG>
__device__ __forceinline__ void param_move(const SweepArgs& a, double pl, double lu, double cA, double (&pd)[7],
                                           double (&s)[7], const double (&G)[28], bool& changed, int& acc,
                                           int& nonfin, bool rec, int win) {
  if (!((a.m.p_mask >> L) & 1)) return;
  constexpr int ia = ThetaMove<L>::ia;
  constexpr int ib = ThetaMove<L>::ib;
  constexpr int ibb = ib >= 0 ? ib : 0;
  const bool inbox = pl == pl;
  const double dp = pl - pd[L];
  // p1, p2, p4, p6 move theta_L directly (p2, p4, p6 also p_L p_{L+1});
  // p3, p5, p7 move theta_L = p_{L-1} p_L
  const double da = (L == 2 || L == 4 || L == 6) ? pd[L == 0 ? 0 : L - 1] * dp : dp;
  const double db = ib >= 0 ? dp * pd[ibb] : 0.0;
  double quad = da * da * G[symi(ia, ia)];
  double lin = da * s[ia];
  if (ib >= 0) {
    quad += 2.0 * da * db * G[symi(ia, ibb)] + db * db * G[symi(ibb, ibb)];
    lin += db * s[ibb];
  }
  const double dA = cA * (quad - 2.0 * lin);
  const bool fin = __builtin_isfinite(dA);
  const bool ok = inbox && fin && lu < -dA;
  nonfin += (inbox && !fin) ? 1 : 0;
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    double gs = G[symi(j, ia)] * da;
    if (ib >= 0) gs += G[symi(j, ibb)] * db;
    s[j] = ok ? s[j] - gs : s[j];
  }
  pd[L] = ok ? pl : pd[L];
  changed = changed || ok;
  acc += ok ? 1 : 0;
  if (DBG && rec) {
    if (a.dbg_pprop) a.dbg_pprop[win * 7 + L] = pl;
    if (a.dbg_pdA) a.dbg_pdA[win * 7 + L] = inbox ? dA : __builtin_nan("");
    if (a.dbg_pacc) a.dbg_pacc[win * 7 + L] = ok;
  }
}

}  // namespace

template <typename T, int K, int MAXT, bool DBG>
__global__ void __launch_bounds__(MAXT) sweep_kernel(SweepArgs a) {
  static_assert(K == 2 || K % 4 == 0, "K must be 2 or a multiple of 4");
  extern __shared__ __align__(16) unsigned char smem[];
  const int NT = blockDim.x;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wv = t >> 6;
  const int NW = NT >> 6;

  // block -> (window, tile): a window is split into a.tiles time tiles of
  // S = NT K sites, one workgroup each
  const int tiles = a.tiles;
  const int bi = (int)blockIdx.x / tiles;
  int tb = (int)blockIdx.x - bi * tiles;
  // workgroups are dealt to the 8 XCDs round-robin (block b -> XCD b % 8);
  // when the tile count allows, consecutive tiles are given consecutive
  // blocks of one XCD, so most boundary exchanges stay inside one L2
  if (tiles % 8 == 0 && tiles > 8) tb = (tb % 8) * (tiles / 8) + tb / 8;
  const int win = a.order ? a.order[bi] : bi;
  const int S = NT * K;
  const int tile0 = tb * S;
  const bool last_tile = tb == tiles - 1;
  int64_t base = 0;
  int M = (int)a.M_single;
  if (a.offsets) {
    base = a.offsets[win];
    M = (int)(a.offsets[win + 1] - base - 1);
  }
  const uint32_t chain = a.chain_ids ? a.chain_ids[win] : a.chain_single;
  const Key key = make_key(a.seed, chain);
  double* P = a.p + (int64_t)win * 7;

  // ---- LDS ----------------------------------------------------------------
  T* lfirst = (T*)smem;                           // [NT][8] first site of each thread
  T* llast = lfirst + NT * 8;                     // [NT][8] last site of each thread
  T* lyi = llast + NT * 8;                        // [S+2][2] (y_n, I_n), n = tile0-1 .. tile0+S
  double* lred = (double*)(lyi + 2 * (NT * K + 2));  // [4*NW][NRED] row partials
  double* lstat = lred + NRED * 4 * NW;           // [NRED]
  double* ldraw = lstat + NRED;                   // [32]: p_l', accept word, FP32 log u_l, current p
  int* lcnt = (int*)(ldraw + 32);                 // [16]
  T* lstage = (T*)(lcnt + 16);                    // [stage][4] statistics staging

  Consts<T> C;
  if constexpr (sizeof(T) == 4)
    C = a.cf;
  else
    C = a.cd;
  double pd[7];
#pragma unroll
  for (int l = 0; l < 7; ++l) pd[l] = P[l];
  C.set_p(pd);
  // one wave per SIMD leaves room for the model constants in vector
  // registers; with two, register pressure decides otherwise
  constexpr bool VCONST = MAXT <= 256;
  if constexpr (VCONST) consts_in_vgprs(C);
  T ws[4];
  double wpar[7];
#pragma unroll
  for (int c = 0; c < 4; ++c) ws[c] = VCONST ? in_vgpr((T)a.w[c]) : (T)a.w[c];
#pragma unroll
  for (int l = 0; l < 7; ++l) wpar[l] = a.w[4 + l];
  const double cA = 0.5 * a.m.beta * a.m.Rd[0];
  const bool uniform_prop = a.m.proposal == PIMC_PROP_UNIFORM;
  const double hD = 0.5 * a.m.dt;

  // observations and drive of the tile and its two halo sites -> LDS;
  // lyb[2 n], lyb[2 n + 1] address (y_n, I_n) by global site index
  T* lyb = lyi + 2 * (1 - tile0);
  {
    const T* Yw = (const T*)a.y + base;
    const T* Iw = (const T*)a.I + base;
    const int lo = tile0 > 0 ? tile0 - 1 : 0;
    const int hi = min(M, tile0 + S);
    for (int n = lo + t; n <= hi; n += NT) {
      lyb[2 * n] = Yw[n];
      lyb[2 * n + 1] = Iw[n];
    }
  }

  // ---- own sites: n = n0 + j, j < K, plus site M on the last thread when
  //      the regular slots stop exactly at M ------------------------------
  const int NTneed = last_tile ? (M - tile0 + K - 1) / K : NT;
  const bool active = t < NTneed;
  const int n0 = tile0 + t * K;
  const bool has_extra = last_tile && (t == NTneed - 1) && (K * NTneed == M - tile0);
  // cross-tile halo: boundary sites of each tile in global memory, slot
  // [gt][0] the tile's first site, [gt][1] its last.  A single-tile window
  // never touches it; neighbours that do not exist alias this tile's own
  // slots, so every address formed is a valid one
  const int gt = bi * tiles + tb;                 // global tile index
  uint64_t* hfirst = (tiles > 1 && a.halo) ? (uint64_t*)a.halo + (int64_t)gt * 2 * SLOT_WORDS : (uint64_t*)lred;
  uint64_t* hlast = (tiles > 1 && a.halo) ? hfirst + SLOT_WORDS : hfirst;
  const uint64_t* hprev_last = tb > 0 ? hfirst - SLOT_WORDS : hlast;
  const uint64_t* hnext_first = !last_tile ? hfirst + 2 * SLOT_WORDS : hfirst;
  // LDS index of the extra site's (y, I): site M when this thread owns it,
  // else the tile's first site, so that no evaluation of the expression
  // (speculative or not) leaves the tile's LDS block
  const int me = has_extra ? M : tile0;
  T* Xt = (T*)a.X + (base + n0) * 4;
  __syncthreads();

  T x[K][4], F[K][4];
  T xe[4], Fe[4];
  bool bad = false;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const bool v = active && n0 + j <= M;
#pragma unroll
    for (int c = 0; c < 4; ++c) x[j][c] = v ? Xt[j * 4 + c] : C.lo[c];
    hh_F(C, x[j], v ? lyb[2 * (n0 + j) + 1] : (T)0, F[j]);
    if (v) {
#pragma unroll
      for (int c = 0; c < 4; ++c) bad = bad || !(x[j][c] >= C.lo[c] && x[j][c] <= C.hi[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) xe[c] = C.lo[c];
  if (has_extra) {
#pragma unroll
    for (int c = 0; c < 4; ++c) xe[c] = Xt[K * 4 + c];
  }
  hh_F(C, xe, has_extra ? lyb[2 * me + 1] : (T)0, Fe);
  if (has_extra) {
#pragma unroll
    for (int c = 0; c < 4; ++c) bad = bad || !(xe[c] >= C.lo[c] && xe[c] <= C.hi[c]);
  }
  if (t == 0) {
#pragma unroll
    for (int l = 0; l < 7; ++l) {
      bad = bad || !__builtin_isfinite(pd[l]);
      if ((a.m.p_mask >> l) & 1) bad = bad || !(pd[l] >= a.m.p_lo[l] && pd[l] <= a.m.p_hi[l]);
    }
  }
  if (tiles > 1) {
    // every tile learns whether any tile failed the entry check, and the
    // boundary sites are published before the first sweep
    if (__syncthreads_or(bad) && t == 0) atomicOr(&a.wsync[bi * 4 + 1], 1u);
    // generation 1: the entry state of both boundary sites; after the even
    // half-sweep of sweep it the first site is generation it + 2, after the
    // odd half-sweep the last site is generation it + 2
    if (t == 0) site_publish(hfirst, x[0], F[0], 1u);
    if (t == NT - 1 && !last_tile) site_publish(hlast, x[K - 1], F[K - 1], 1u);
    tile_barrier(&a.wsync[bi * 4], (uint32_t)tiles, a.err, a.spin_ticks);
    bad = __hip_atomic_load(&a.wsync[bi * 4 + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
  }
  if (__syncthreads_or(bad)) {
    if (t == 0) atomicOr(a.err, 2u);
    return;
  }
  if (active) {
    lds_put(lfirst + t * 8, x[0], F[0]);
    lds_put(llast + t * 8, x[K - 1], F[K - 1]);
  }
  if (t == 0) {
#pragma unroll
    for (int l = 0; l < 7; ++l) ldraw[24 + l] = pd[l];
  }
  __syncthreads();
  uint32_t nbar = 1;   // tile barriers passed so far (the entry barrier)

  int accE = 0, accO = 0, nonfin = 0;
  T xnx[4] = {0, 0, 0, 0};   // last thread of a tile: the next tile's first site
  int accP[7] = {0, 0, 0, 0, 0, 0, 0};
  T* dx_t = DBG && a.dbg_xprop ? (T*)a.dbg_xprop + (base + n0) * 4 : nullptr;
  double* ddA_t = DBG && a.dbg_dA ? a.dbg_dA + base + n0 : nullptr;
  uint8_t* dacc_t = DBG && a.dbg_acc ? a.dbg_acc + base + n0 : nullptr;

  for (int64_t it = 0; it < a.n_sweeps; ++it) {
    const uint64_t k = a.sweep0 + (uint64_t)it;
    const bool last = it == a.n_sweeps - 1;

    if (a.flags & PIMC_STATES) {
      // ---- even half-sweep ----------------------------------------------
      // accept words: block n >> 2 of the SACC stream holds word n & 3 for
      // sites n .. n + 3; with K = 2 two threads share a block (n0 is even)
      constexpr int KS = K < 4 ? K : 4;
      uint32_t uodd[K / 2];
#pragma unroll
      for (int q = 0; q < (K + 3) / 4; ++q) {
        const int j0 = 4 * q;
        U4 ub{0, 0, 0, 0};
        if (active && n0 + j0 <= M) ub = draw(key, opaque((uint32_t)((n0 + j0) >> 2)), k, TAG_SACC);
        uint32_t ueven[2];
        if constexpr (K >= 4) {
          ueven[0] = ub.x;
          ueven[1] = ub.z;
          uodd[2 * q] = ub.y;
          uodd[2 * q + 1] = ub.w;
        } else {
          const bool upper = (n0 & 2) != 0;
          ueven[0] = upper ? ub.z : ub.x;
          ueven[1] = 0u;
          uodd[0] = upper ? ub.w : ub.y;
        }
#pragma unroll
        for (int jj = 0; jj < KS; jj += 2) {
          const int j = j0 + jj;
          const int nn = n0 + j;
          if (active && nn <= M) {
            Nb<T> L, R;
            const bool hasL = nn >= 1;
            if (j == 0) {
              if (hasL) {
                if (t == 0) {   // last site of the previous tile, after its odd half-sweep
                  site_fetch(C, hprev_last, (uint32_t)it + 1, lyb[2 * nn - 1], L, a.err, a.spin_ticks);
                } else {
                  lds_get(C, llast + (t - 1) * 8, lyb[2 * nn - 1], L);
                }
              }
            } else {
#pragma unroll
              for (int c = 0; c < 4; ++c) {
                L.x[c] = x[j - 1][c];
                L.F[c] = F[j - 1][c];
              }
            }
            const bool hasR = nn + 1 <= M;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              R.x[c] = x[j + 1][c];
              R.F[c] = F[j + 1][c];
            }
            const U4 blk = draw(key, opaque((uint32_t)nn), k, TAG_SITE);
            double dA;
            T xp[4];
            const bool ok = site_update(C, ws, uniform_prop, x[j], F[j], lyb[2 * nn], lyb[2 * nn + 1], hasL, L,
                                        hasR, R, nn >= 1, blk, ueven[jj >> 1], dA, xp, nonfin);
            accE += ok;
            if (DBG && last) {
              if (dx_t)
#pragma unroll
                for (int c = 0; c < 4; ++c) dx_t[j * 4 + c] = xp[c];
              if (ddA_t) ddA_t[j] = dA;
              if (dacc_t) dacc_t[j] = ok;
            }
          }
        }
      }
      if (has_extra) {  // site M (even): left neighbour is own slot K-1, no right link
        Nb<T> L, R;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          L.x[c] = x[K - 1][c];
          L.F[c] = F[K - 1][c];
          R.x[c] = xe[c];
          R.F[c] = Fe[c];
        }
        const U4 blk = draw(key, opaque((uint32_t)M), k, TAG_SITE);
        const U4 ub = draw(key, opaque((uint32_t)(M >> 2)), k, TAG_SACC);
        const uint32_t uM = (M & 2) ? ub.z : ub.x;   // M is even
        double dA;
        T xp[4];
        const bool ok = site_update(C, ws, uniform_prop, xe, Fe, lyb[2 * me], lyb[2 * me + 1], true, L, false, R,
                                    true, blk, uM, dA, xp, nonfin);
        accE += ok;
        if (DBG && last) {
          if (dx_t)
#pragma unroll
            for (int c = 0; c < 4; ++c) dx_t[K * 4 + c] = xp[c];
          if (ddA_t) ddA_t[K] = dA;
          if (dacc_t) dacc_t[K] = ok;
        }
      }
      if (active) lds_put(lfirst + t * 8, x[0], F[0]);
      if (tiles > 1 && t == 0) site_publish(hfirst, x[0], F[0], (uint32_t)it + 2);
      __syncthreads();

      // ---- odd half-sweep -----------------------------------------------
#pragma unroll
      for (int j = 1; j < K; j += 2) {
        const int nn = n0 + j;
        if (active && nn <= M) {
          Nb<T> L, R;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            L.x[c] = x[j - 1][c];
            L.F[c] = F[j - 1][c];
          }
          const bool hasR = nn + 1 <= M;
          if (j == K - 1) {
            if (hasR) {
              if (has_extra) {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                  R.x[c] = xe[c];
                  R.F[c] = Fe[c];
                }
              } else if (t == NT - 1) {   // first site of the next tile, after its even half-sweep
                site_fetch(C, hnext_first, (uint32_t)it + 2, lyb[2 * nn + 3], R, a.err, a.spin_ticks);
#pragma unroll
                for (int c = 0; c < 4; ++c) xnx[c] = R.x[c];   // kept for the link statistics
              } else {
                lds_get(C, lfirst + (t + 1) * 8, lyb[2 * nn + 3], R);
              }
            }
          } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              R.x[c] = x[j + 1][c];
              R.F[c] = F[j + 1][c];
            }
          }
          const U4 blk = draw(key, opaque((uint32_t)nn), k, TAG_SITE);
          double dA;
          T xp[4];
          const bool ok = site_update(C, ws, uniform_prop, x[j], F[j], lyb[2 * nn], lyb[2 * nn + 1], true, L,
                                      hasR, R, true, blk, uodd[j >> 1], dA, xp, nonfin);
          accO += ok;
          if (DBG && last) {
            if (dx_t)
#pragma unroll
              for (int c = 0; c < 4; ++c) dx_t[j * 4 + c] = xp[c];
            if (ddA_t) ddA_t[j] = dA;
            if (dacc_t) dacc_t[j] = ok;
          }
        }
      }
      if (active) lds_put(llast + t * 8, x[K - 1], F[K - 1]);
      if (tiles > 1 && t == NT - 1 && !last_tile) site_publish(hlast, x[K - 1], F[K - 1], (uint32_t)it + 2);
    }

    if (a.flags & PIMC_PARAMS) {
      // ---- random numbers of the parameter moves (path independent), spread
      //      over the waves: wave w, lane i draws for parameter w + i NW;
      //      the proposed value and its box test are formed here too (a move
      //      of p_l changes no other p_j, so p_l before its move is the value
      //      at the start of the section).  With time tiles this work fills
      //      the wait for the other tiles' partial sums ----------------------
      auto param_draws = [&]() {
        const int l = wv + lane * NW;
        if (lane * NW < 7 && l < 7) {
          const U4 b = draw(key, opaque((uint32_t)l), k, TAG_PARAM);
          double z;
          if (uniform_prop) {
            z = Math<double>::uniform_pm1(b.x);
          } else if constexpr (sizeof(T) == 4) {
            float z0, z1;
            Math<float>::box_muller(b.x, b.y, z0, z1);
            z = (double)z0;
          } else {
            double z1;
            Math<double>::box_muller(b.x, b.y, z, z1);
          }
          // parameter-indexed values by selects (no dynamically indexed
          // register or argument arrays)
          double lo = 0.0, hi = 0.0;
#pragma unroll
          for (int q = 0; q < 7; ++q) {
            lo = q == l ? a.m.p_lo[q] : lo;
            hi = q == l ? a.m.p_hi[q] : hi;
          }
          const double pl = ldraw[24 + l] + a.w[4 + l] * z;
          const bool inbox = pl >= lo && pl <= hi;
          ldraw[l] = inbox ? pl : __builtin_nan("");
          ldraw[16 + l] = ::log(u01_d(b.z));
        }
      };
      if (tiles == 1) param_draws();
      // ---- sufficient statistics over the links of the odd sites ----------
      double th[7];
      theta_of(pd, th);
      double st[NRED];
#pragma unroll
      for (int i = 0; i < NRED; ++i) st[i] = 0.0;
      if (active) {
        Feat fl = feat_of(x[0], lyb[2 * n0 + 1]);
#pragma unroll
        for (int j = 1; j < K; j += 2) {
          const int nn = n0 + j;
          if (nn <= M) {
            const Feat fc = feat_of(x[j], lyb[2 * nn + 1]);
            link_stats(th, hD, fl, fc, st);
            if (nn + 1 <= M) {
              Feat fr;
              if (j == K - 1) {
                if (has_extra) {
                  fr = feat_of(xe, lyb[2 * me + 1]);
                } else {
                  // next thread's first site, or the next tile's: read during
                  // the odd half-sweep when sites moved, else the entry
                  // publication, which is then current
                  T xr[4];
                  if (t == NT - 1 && (a.flags & PIMC_STATES)) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) xr[c] = xnx[c];
                  } else if (t == NT - 1) {
                    Nb<T> nb;
                    site_fetch(C, hnext_first, 1u, lyb[2 * nn + 3], nb, a.err, a.spin_ticks);
#pragma unroll
                    for (int c = 0; c < 4; ++c) xr[c] = nb.x[c];
                  } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c) xr[c] = lfirst[(t + 1) * 8 + c];
                  }
                  fr = feat_of(xr, lyb[2 * nn + 3]);
                }
              } else {
                fr = feat_of(x[j + 1], lyb[2 * nn + 3]);
              }
              link_stats(th, hD, fc, fr, st);
              fl = fr;
            }
          }
        }
      }
      // ---- block reduction: rows of 16 lanes with DPP, then a fixed-order
      //      sum of the row partials through LDS --------------------------
#pragma unroll
      for (int i = 0; i < NRED; ++i) st[i] = row_sum(st[i]);
      if ((lane & 15) == 15) {
#pragma unroll
        for (int i = 0; i < NRED; ++i) lred[(wv * 4 + (lane >> 4)) * NRED + i] = st[i];
      }
      __syncthreads();
      if (t < NRED) {
        // row partials laid out [row][value]: consecutive threads read
        // consecutive words (no bank conflicts)
        const double* row = lred + t;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (int q = 0; q < 4 * NW; q += 4) {
          s0 += row[q * NRED];
          s1 += row[(q + 1) * NRED];
          s2 += row[(q + 2) * NRED];
          s3 += row[(q + 3) * NRED];
        }
        lstat[t] = (s0 + s1) + (s2 + s3);
      }
      __syncthreads();
      if (tiles > 1) {
        // all-reduce over the window's tiles: partials in a double buffer,
        // summed in tile order by every tile (identical results everywhere)
        // every partial value as two generation words, double-buffered by
        // the parity of the barrier count
        uint64_t* wp = (uint64_t*)a.wpart +
                       ((int64_t)(nbar & 1) * a.ngroups * tiles + (int64_t)bi * tiles) * (2 * NRED);
        ++nbar;
        for (int i = t; i < 2 * NRED; i += NT) {   // 70 words; a tile may have 64 threads
          const uint64_t b = __builtin_bit_cast(uint64_t, lstat[i >> 1]);
          gw_store(wp + tb * 2 * NRED + i, gen_word(nbar, (i & 1) ? (uint32_t)(b >> 32) : (uint32_t)b));
        }
        // the parameter proposals are drawn while the other tiles' partials
        // are on their way
        param_draws();
        // NRED x tiles partials: thread t sums tiles q = t / NRED, + NSEG, ...
        // for value t % NRED with all loads in flight, then NSEG segment sums
        // are combined in segment order (fixed for a given launch shape)
        {
          const int NSEG = NT / NRED;
          const int v = t % NRED, sg = t / NRED;
          if (sg < NSEG) {
            double acc = 0.0;
            for (int q0 = sg; q0 < tiles; q0 += 8 * NSEG) {
              const uint64_t* src[16];
#pragma unroll
              for (int u = 0; u < 8; ++u) {
                const int q = q0 + u * NSEG < tiles ? q0 + u * NSEG : tb;   // absent: own words, ignored
                src[2 * u] = wp + q * 2 * NRED + 2 * v;
                src[2 * u + 1] = src[2 * u] + 1;
              }
              uint64_t w[16];
              gw_wait<16>(src, w, nbar, a.err, a.spin_ticks);
              double vals[8];
#pragma unroll
              for (int u = 0; u < 8; ++u) {
                const uint64_t b = ((uint64_t)(uint32_t)w[2 * u + 1] << 32) | (uint32_t)w[2 * u];
                vals[u] = q0 + u * NSEG < tiles ? __builtin_bit_cast(double, b) : 0.0;
              }
#pragma unroll
              for (int u = 0; u < 8; ++u) acc += vals[u];
            }
            lred[sg * NRED + v] = acc;
          }
          __syncthreads();
          if (t < NRED) {
            double acc = 0.0;
            for (int q = 0; q < NSEG; ++q) acc += lred[q * NRED + t];
            lstat[t] = acc;
          }
        }
        __syncthreads();
      }
      // ---- sequential parameter moves, evaluated identically by every
      //      wave (no broadcast and no further barrier needed) ---------------
      {
        double s7[7], G[28], zz[7], lw[7];
#pragma unroll
        for (int l = 0; l < 7; ++l) {
          s7[l] = lstat[l];
          zz[l] = ldraw[l];
          lw[l] = ldraw[16 + l];
        }
#pragma unroll
        for (int i = 0; i < 28; ++i) G[i] = lstat[7 + i];
        bool changed = false;
        const bool rec = last && t == 0 && tb == 0;
        param_move<0, DBG>(a, zz[0], lw[0], cA, pd, s7, G, changed, accP[0], nonfin, rec, win);
        param_move<1, DBG>(a, zz[1], lw[1], cA, pd, s7, G, changed, accP[1], nonfin, rec, win);
        param_move<2, DBG>(a, zz[2], lw[2], cA, pd, s7, G, changed, accP[2], nonfin, rec, win);
        param_move<3, DBG>(a, zz[3], lw[3], cA, pd, s7, G, changed, accP[3], nonfin, rec, win);
        param_move<4, DBG>(a, zz[4], lw[4], cA, pd, s7, G, changed, accP[4], nonfin, rec, win);
        param_move<5, DBG>(a, zz[5], lw[5], cA, pd, s7, G, changed, accP[5], nonfin, rec, win);
        param_move<6, DBG>(a, zz[6], lw[6], cA, pd, s7, G, changed, accP[6], nonfin, rec, win);
        if (changed) {
          if (t == 0) {
#pragma unroll
            for (int l = 0; l < 7; ++l) ldraw[24 + l] = pd[l];
          }
          C.set_p(pd);
          if constexpr (VCONST) {
#pragma unroll
            for (int l = 0; l < 7; ++l) C.p[l] = in_vgpr(C.p[l]);
          }
#pragma unroll
          for (int j = 0; j < K; ++j) F[j][0] = hh_FV(C, x[j][0], x[j][1], x[j][2], x[j][3], lyb[2 * (n0 + j) + 1]);
          Fe[0] = hh_FV(C, xe[0], xe[1], xe[2], xe[3], has_extra ? lyb[2 * me + 1] : (T)0);
        }
      }
    } else {
      __syncthreads();
    }

    // ---- statistics ------------------------------------------------------
    if (a.ptrace && t == 0 && tb == 0) {
#pragma unroll
      for (int l = 0; l < 7; ++l) a.ptrace[(int64_t)win * a.n_sweeps * 7 + it * 7 + l] = pd[l];
    }
    if (a.sum && (int64_t)k >= a.burn && ((int64_t)k - a.burn) % a.stride == 0) {
      // stage the path through LDS so that the FP64 read-modify-write of the
      // moment sums is coalesced (consecutive lanes, consecutive addresses)
      const T* xr = (const T*)a.xref + base * 4;
      double* su = a.sum + base * 4;
      double* sq = a.sumsq ? a.sumsq + base * 4 : nullptr;
      // batch of this sample: the i-th of the call's nsamp samples belongs
      // to batch floor(i nbatch / nsamp)
      double* bt = nullptr;
      if (a.batch) {
        const int64_t si = ((int64_t)k - a.kfirst) / a.stride;
        bt = a.batch + (si * a.nbatch / a.nsamp) * a.bslice + base * 4;
      }
      const int Sst = a.stage;
      const int hi_site = last_tile ? M : tile0 + S - 1;   // this tile's sites only
      for (int c0 = tile0; c0 <= hi_site; c0 += Sst) {
        if (active) {
#pragma unroll
          for (int j = 0; j < K; ++j) {
            const int n = n0 + j;
            if (n <= M && n >= c0 && n < c0 + Sst) {
#pragma unroll
              for (int c = 0; c < 4; ++c) lstage[(n - c0) * 4 + c] = x[j][c];
            }
          }
          if (has_extra && M >= c0 && M < c0 + Sst) {
#pragma unroll
            for (int c = 0; c < 4; ++c) lstage[(M - c0) * 4 + c] = xe[c];
          }
        }
        __syncthreads();
        const int cnt = 4 * min(Sst, hi_site + 1 - c0);
        // eight independent elements per round: all loads are in flight
        // before the first add, so the loop is bandwidth- not latency-bound
        for (int e0 = t; e0 < cnt; e0 += 8 * NT) {
          double dv[8], s1[8], s2[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * NT;
            const int64_t g = (int64_t)c0 * 4 + e;
            dv[u] = e < cnt ? (double)lstage[e] - (double)xr[g] : 0.0;
            s1[u] = e < cnt ? su[g] : 0.0;
            s2[u] = (e < cnt && sq) ? sq[g] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * NT;
            const int64_t g = (int64_t)c0 * 4 + e;
            if (e < cnt) {
              su[g] = s1[u] + dv[u];
              if (sq) sq[g] = s2[u] + dv[u] * dv[u];
            }
          }
        }
        // the batch sums in a pass of their own, so that runs without them
        // keep the registers of the pass above
        if (bt) {
          for (int e0 = t; e0 < cnt; e0 += 8 * NT) {
            double dv[8], s3[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int e = e0 + u * NT;
              const int64_t g = (int64_t)c0 * 4 + e;
              dv[u] = e < cnt ? (double)lstage[e] - (double)xr[g] : 0.0;
              s3[u] = e < cnt ? bt[g] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int e = e0 + u * NT;
              if (e < cnt) bt[(int64_t)c0 * 4 + e] = s3[u] + dv[u];
            }
          }
        }
        __syncthreads();
      }
    }
  }

  // ---- write back ---------------------------------------------------------
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (active && n0 + j <= M) {
#pragma unroll
      for (int c = 0; c < 4; ++c) Xt[j * 4 + c] = x[j][c];
    }
  }
  if (has_extra) {
#pragma unroll
    for (int c = 0; c < 4; ++c) Xt[K * 4 + c] = xe[c];
  }
  if (t == 0 && tb == 0) {
#pragma unroll
    for (int l = 0; l < 7; ++l) P[l] = pd[l];
  }
  // ---- acceptance counters ----------------------------------------------
  __syncthreads();
  if (t < 16) lcnt[t] = 0;
  __syncthreads();
  if (accE) atomicAdd(&lcnt[0], accE);
  if (accO) atomicAdd(&lcnt[1], accO);
  if (nonfin && lane != 0) atomicAdd(&lcnt[9], nonfin);
  if (t == 0 && tb == 0) {
    // parameter counts (and their non-finite count) are identical in every
    // wave and every tile; lane 0 of wave 0 of tile 0 reports them once
#pragma unroll
    for (int l = 0; l < 7; ++l) lcnt[2 + l] += accP[l];
    if (nonfin) atomicAdd(&lcnt[9], nonfin);
  }
  __syncthreads();
  if (t == 0) {
    if (a.acc) {
      for (int i = 0; i < PIMC_NACC; ++i)
        if (lcnt[i]) atomicAdd((unsigned long long*)&a.acc[(int64_t)win * PIMC_NACC + i], (unsigned long long)lcnt[i]);
    }
    if (lcnt[9]) atomicOr(a.err, 1u);
  }
}

size_t sweep_smem_bytes(int NT, int K, bool fp64, int stage) {
  const size_t ts = fp64 ? 8 : 4;
  const size_t NW = (size_t)NT / 64;
  return (size_t)NT * 8 * ts * 2 + (size_t)2 * (NT * K + 2) * ts + (NRED * 4 * NW + NRED + 32) * sizeof(double) +
         16 * sizeof(int) + (size_t)stage * 4 * ts;
}

__global__ void zero_u32_kernel(uint32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// The launch is refused on the host (never enqueued) when the kernel's static
// LDS plus the requested dynamic LDS exceeds what a workgroup may allocate.
template <typename Kern>
static int launch_checked(Kern k, int nblocks, int NT, size_t sm, hipStream_t s, const SweepArgs& a) {
  hipFuncAttributes at;
  if (hipFuncGetAttributes(&at, (const void*)k) != hipSuccess) return PIMC_ERR_HIP;
  int dev = 0, lim = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PIMC_ERR_HIP;
  if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return PIMC_ERR_HIP;
  if (sm + at.sharedSizeBytes > (size_t)lim || NT > at.maxThreadsPerBlock) return PIMC_ERR_UNSUPPORTED;
  if (a.tiles > 1) {
    // tiles wait on each other, so all of them must be resident: a shape
    // the device cannot hold at once is refused before anything is enqueued
    int per_cu = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k, NT, sm) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return PIMC_ERR_HIP;
    if ((int64_t)per_cu * ncu < nblocks) return PIMC_ERR_UNSUPPORTED;
    // reset the exchange words (generation 0) and the entry counters in
    // stream order, then launch cooperatively
    const int nh = nblocks * 2 * SLOT_WORDS * 2, np = 2 * nblocks * 2 * NRED * 2, nw = a.ngroups * 4;
    hipLaunchKernelGGL(zero_u32_kernel, dim3((nh + 255) / 256), dim3(256), 0, s, (uint32_t*)a.halo, nh);
    hipLaunchKernelGGL(zero_u32_kernel, dim3((np + 255) / 256), dim3(256), 0, s, (uint32_t*)a.wpart, np);
    hipLaunchKernelGGL(zero_u32_kernel, dim3((nw + 255) / 256), dim3(256), 0, s, a.wsync, nw);
    SweepArgs copy = a;
    void* args[] = {&copy};
    const hipError_t e = hipLaunchCooperativeKernel((const void*)k, dim3(nblocks), dim3(NT), args, (unsigned)sm, s);
    if (e == hipErrorCooperativeLaunchTooLarge) {
      (void)hipGetLastError();   // leave no stale error for the caller's next runtime call
      return PIMC_ERR_UNSUPPORTED;
    }
    return e == hipSuccess ? PIMC_OK : PIMC_ERR_HIP;
  }
  hipLaunchKernelGGL(k, dim3(nblocks), dim3(NT), sm, s, a);
  return hipGetLastError() == hipSuccess ? PIMC_OK : PIMC_ERR_HIP;
}

#define PIMC_SWEEP_LAUNCH(T, K, MAXT)                                                \
  do {                                                                               \
    if (dbg)                                                                         \
      return launch_checked(sweep_kernel<T, K, MAXT, true>, nblocks, NT, sm, s, a);  \
    else                                                                             \
      return launch_checked(sweep_kernel<T, K, MAXT, false>, nblocks, NT, sm, s, a); \
  } while (0)

// Launch bounds follow the thread count: up to 256 threads (one wave per
// SIMD) a wave may hold 512 registers (architectural + accumulation), so the
// register-resident path never spills to scratch.
#define PIMC_SWEEP_PICK(T, K, BIG)          \
  do {                                      \
    if (NT <= 256)                          \
      PIMC_SWEEP_LAUNCH(T, K, 256);         \
    else                                    \
      PIMC_SWEEP_LAUNCH(T, K, BIG);         \
  } while (0)

int launch_sweep(const SweepArgs& a, bool fp64, int K, int nblocks, int NT, hipStream_t s) {
  const size_t sm = sweep_smem_bytes(NT, K, fp64, a.stage);
  if (sm + LDS_STATIC_RESERVE > LDS_BYTES || NT > sweep_max_threads(fp64, K)) return PIMC_ERR_UNSUPPORTED;
  const bool dbg = a.dbg_xprop || a.dbg_dA || a.dbg_acc || a.dbg_pprop || a.dbg_pdA || a.dbg_pacc;
  if (fp64) {
    switch (K) {
      case 4:
        if (NT > 256) return PIMC_ERR_UNSUPPORTED;   // wide FP64 shapes are not launched
        PIMC_SWEEP_LAUNCH(double, 4, 256);
      default: return PIMC_ERR_UNSUPPORTED;
    }
  } else {
    switch (K) {
      case 2:
        if (NT > 256) return PIMC_ERR_UNSUPPORTED;   // a tiling option: one wave per SIMD only
        PIMC_SWEEP_LAUNCH(float, 2, 256);
      case 4: PIMC_SWEEP_PICK(float, 4, 1024); break;
      case 8: PIMC_SWEEP_PICK(float, 8, 512); break;
      case 16: PIMC_SWEEP_PICK(float, 16, 512); break;
      default: return PIMC_ERR_UNSUPPORTED;
    }
  }
  return PIMC_ERR_UNSUPPORTED;
}

int sweep_max_threads(bool fp64, int K) {
  if (fp64) return K == 4 ? 256 : 0;
  if (K == 2) return 256;
  if (K == 4) return 1024;
  if (K == 8 || (!fp64 && K == 16)) return 512;
  return 0;
}

}  // namespace pimc
