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
#include <map>
#include <mutex>
#include <tuple>

#include "device.hpp"
#include "kernels.hpp"

namespace pimc {

namespace {

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
// recomputed with the current parameters, as for an LDS neighbour; the
// gates' fields too when `gates`, i.e. when the Table 1 constants may have
// moved since the site was published).
template <typename T>
__device__ __forceinline__ void site_fetch(const Consts<T>& C, const uint64_t* slot, uint32_t gen, T I, Nb<T>& nb,
                                           uint32_t* err, uint64_t ticks, bool gates) {
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
  if (gates) {
#pragma unroll
    for (int g = 0; g < 3; ++g) nb.F[1 + g] = hh_Fgate(C, g, nb.x[0], nb.x[1 + g]);
  }
}

// Gate equation of Section 5.1 in FP64 with the constants (V_a, dV_a, tau0,
// tau1) of one gate: (a_inf(V) - a) / tau(V).
__device__ __forceinline__ double gate_field64(double V, double a, const double (&gk)[4]) {
  const double t = ::tanh((V - gk[0]) / gk[1]);
  return (0.5 + 0.5 * t - a) / (gk[2] + gk[3] * (1.0 - t * t));
}

// Component 1 + g (the gate g) of a site state, by selects.
template <typename T>
__device__ __forceinline__ T sel_gate(const T (&x)[4], int g) {
  return g == 0 ? x[1] : (g == 1 ? x[2] : x[3]);
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

// The values LO .. LO + N - 1 of link_stats (the same sums, term for term),
// for shapes whose registers cannot hold all 35 sums beside the path.
template <int LO, int N>
__device__ __forceinline__ void link_stats_part(const double (&th)[7], double h, const Feat& l, const Feat& r,
                                                double (&acc)[N]) {
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
  for (int q = 0; q < 7; ++q)
    if (q >= LO && q < LO + N) acc[q - LO] += phi[q] * e;
#pragma unroll
  for (int a = 0; a < 7; ++a)
#pragma unroll
    for (int b = a; b < 7; ++b) {
      const int i = 7 + sym7(a, b);
      if (i >= LO && i < LO + N) acc[i - LO] += phi[a] * phi[b];
    }
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

// The value a lane holds in lane `src` of its wave (a wave-uniform result).
__device__ __forceinline__ double lane_value(double v, int src) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), src);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// One Metropolis move of parameter L against the sufficient statistics,
// spread over the lanes of a wave: lane j < 7 holds s_j and row j of G
// (Grow[c] = G_jc; lanes past 6 repeat row 6), so the update of s after an
// accepted move is one step per lane, and the move reads s_ia, s_ib from
// their lanes.  Gd: the three entries of G the move needs (G_aa, G_ab,
// G_bb).  pl: proposed value, drawn and box-tested beforehand (a move of
// p_l leaves every other p_j unchanged, so p_l before its own move is known
// when the sweep's parameter section starts); NaN when outside the box.
// lu: FP64 log u of the accept uniform, also formed beforehand.
// cA = beta Rd_V / 2.  Written without branches, to keep the sequential
// chain of the seven moves short.
template <int L, bool DBG>
__device__ __forceinline__ void param_move(const SweepArgs& a, double pl, double lu, double cA, double (&pd)[7],
                                           double& sj, const double (&Grow)[7], const double (&Gd)[3],
                                           bool& changed, int& acc, int& nonfin, bool rec, int win) {
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
  double quad = da * da * Gd[0];
  double lin = da * lane_value(sj, ia);
  if (ib >= 0) {
    quad += 2.0 * da * db * Gd[1] + db * db * Gd[2];
    lin += db * lane_value(sj, ibb);
  }
  const double dA = cA * (quad - 2.0 * lin);
  const bool fin = __builtin_isfinite(dA);
  const bool ok = inbox && fin && lu < -dA;
  nonfin += (inbox && !fin) ? 1 : 0;
  double gs = Grow[ia] * da;
  if (ib >= 0) gs += Grow[ibb] * db;
  sj = ok ? sj - gs : sj;
  pd[L] = ok ? pl : pd[L];
  changed = changed || ok;
  acc += ok ? 1 : 0;
  if (DBG && rec) {
    if (a.dbg_pprop) a.dbg_pprop[win * 7 + L] = pl;
    if (a.dbg_pdA) a.dbg_pdA[win * 7 + L] = inbox ? dA : __builtin_nan("");
    if (a.dbg_pacc) a.dbg_pacc[win * 7 + L] = ok;
  }
}

// G entries (G_aa, G_ab, G_bb) of the move of parameter L.
template <int L>
__device__ __forceinline__ void move_gram(const double* lG, double (&Gd)[3]) {
  constexpr int ia = ThetaMove<L>::ia;
  constexpr int ib = ThetaMove<L>::ib;
  constexpr int ibb = ib >= 0 ? ib : 0;
  Gd[0] = lG[symi(ia, ia)];
  Gd[1] = ib >= 0 ? lG[symi(ia, ibb)] : 0.0;
  Gd[2] = ib >= 0 ? lG[symi(ibb, ibb)] : 0.0;
}

// Standard normal quantile of x in (0, 1): a single-precision estimate
// (relative error near 1e-7) refined by one Halley step for Phi(z) = x in
// FP64, which converges cubically, so the step leaves an error far below
// FP64 rounding.  The lower tail is solved directly and the upper tail by
// symmetry from 1 - x (exact for x >= 1/2), so Phi(z) - x never cancels
// against a value near 1.  About 2.4 times faster here than the FP64 library
// quantile, whose result it matches to rounding.
__device__ __forceinline__ double normal_quantile(double x) {
  const bool up = x > 0.5;
  const double q = up ? 1.0 - x : x;
  double z = (double)normcdfinvf((float)q);
  const double e = 0.5 * erfc(-z * 0.70710678118654752440) - q;    // Phi(z) - q
  const double d = exp(-0.5 * z * z) * 0.39894228040143267794;     // phi(z)
  const double r = e / d;
  z -= r / (1.0 + 0.5 * z * r);
  return up ? -z : z;
}

// log P(Z > z) of a standard normal, z >= 0, through the scaled
// complementary error function (no underflow however far out z lies).
__device__ __forceinline__ double log_upper_tail(double z) {
  return ::log(0.5 * erfcx(z * 0.70710678118654752440)) - 0.5 * z * z;
}

// The u-quantile of Z given a <= Z <= b, 0 <= a < b <= inf: solves
// log P(Z > z) = log P(Z > a) + log(1 - u (1 - P(Z > b) / P(Z > a))) by
// Newton steps from z = a.  log P(Z > z) is concave and decreasing, so the
// first step lands right of the root and the rest descend onto it
// (quadratically); twelve steps reach full precision from any start.
__device__ __forceinline__ double upper_tail_quantile(double a, double b, double u) {
  const double la = log_upper_tail(a);
  const double r = b < 1e300 ? ::exp(log_upper_tail(b) - la) : 0.0;
  const double T = la + (u < 0.5 ? ::log1p(-u * (1.0 - r)) : ::log((1.0 - u) + u * r));
  double z = a;
  for (int it = 0; it < 12; ++it)
    z += (log_upper_tail(z) - T) * erfcx(z * 0.70710678118654752440) * 1.25331413731550025121;  // sqrt(pi/2)
  return z;
}

// The u-quantile of N(mu, sg^2) truncated to [lo, hi].  A box that holds
// the mean inverts the normal CDF directly; a box entirely on one side of
// it goes through the upper-tail quantile above (mirrored for a box below
// the mean), which stays exact when the box lies many standard deviations
// out, where the CDF itself underflows.  Not inlined: the seven calls of a
// sweep share one copy.
__device__ __attribute__((noinline)) double trunc_normal_inv(double mu, double sg, double lo, double hi, double u) {
  const double za = (lo - mu) / sg, zb = (hi - mu) / sg;
  if (za >= 0.0) return mu + sg * upper_tail_quantile(za, zb, u);
  if (zb <= 0.0) return mu - sg * upper_tail_quantile(-zb, -za, 1.0 - u);
  const double pa = normcdf(za), pb = normcdf(zb);
  return mu + sg * normal_quantile(pa + u * (pb - pa));
}

// Exact conditional draw of parameter L given the path and the other
// parameters.  The action is quadratic in p_L: with q = d theta / d p_L,
// A(p_L + d) - A(p_L) = cA (d^2 q^T G q - 2 d q . s), so p_L given the rest
// is N(p_L + q.s / q^T G q, 1 / (2 cA q^T G q)) truncated to its box (drawn
// uniformly on the box when the curvature is not positive).  ug: the
// uniform of the draw, zq its standard normal quantile (formed beforehand).
// When both box edges lie more than 10 standard deviations from the mean,
// the normal mass the box cuts off is below 1e-23, and mean + sd zq is the
// truncated quantile to within 1e-13 standard deviations for any ug of the
// generator's (0, 1) grid; other boxes go through the full inversion.  The
// statistics follow the move as for an accepted Metropolis step.  Only the
// extended kernels draw, and they record the draw (rec) whenever the
// parameter records are asked for.
template <int L>
__device__ __forceinline__ void param_gibbs(const SweepArgs& a, double ug, double zq, double cA, double (&pd)[7],
                                            double (&s)[7], const double (&G)[28], bool& changed, int& acc,
                                            int& nonfin, bool rec, int win) {
  if (!((a.m.p_mask >> L) & 1)) return;
  constexpr int ia = ThetaMove<L>::ia;
  constexpr int ib = ThetaMove<L>::ib;
  constexpr int ibb = ib >= 0 ? ib : 0;
  constexpr bool prod = L == 2 || L == 4 || L == 6;   // theta_L = p_{L-1} p_L
  const double qa = prod ? pd[prod ? L - 1 : 0] : 1.0;
  const double qb = ib >= 0 ? pd[ibb] : 0.0;
  double qGq = qa * qa * G[symi(ia, ia)];
  double qs = qa * s[ia];
  if (ib >= 0) {
    qGq += 2.0 * qa * qb * G[symi(ia, ibb)] + qb * qb * G[symi(ibb, ibb)];
    qs += qb * s[ibb];
  }
  const double lo = a.m.p_lo[L], hi = a.m.p_hi[L];
  const double curv = cA * qGq;
  double v;
  if (curv > 0.0 && __builtin_isfinite(curv)) {
    const double mu = pd[L] + qs / qGq, sg = 1.0 / sqrt(2.0 * curv);
    if ((lo - mu) < -10.0 * sg && (hi - mu) > 10.0 * sg)
      v = mu + sg * zq;
    else
      v = trunc_normal_inv(mu, sg, lo, hi, ug);
  } else {
    v = lo + ug * (hi - lo);
  }
  const bool ok = __builtin_isfinite(v);
  nonfin += ok ? 0 : 1;
  v = ok ? fmin(fmax(v, lo), hi) : pd[L];
  const double dp = v - pd[L];
  const double da = qa * dp, db = qb * dp;
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    double gs = G[symi(j, ia)] * da;
    if (ib >= 0) gs += G[symi(j, ibb)] * db;
    s[j] -= gs;
  }
  pd[L] = v;
  changed = changed || dp != 0.0;
  acc += ok ? 1 : 0;
  if (rec) {
    if (a.dbg_pprop) a.dbg_pprop[win * 7 + L] = v;
    if (a.dbg_pdA) a.dbg_pdA[win * 7 + L] = __builtin_nan("");
    if (a.dbg_pacc) a.dbg_pacc[win * 7 + L] = ok;
  }
}

}  // namespace

// The sweep of one workgroup (a window, or one time tile of it) with K
// sites per thread.  The statements live in sweep_body.inc, which forms the
// kernel for the launch's K and, for launches of 16 sites per thread, a
// device function for each smaller K that a window of a batch may use; the
// kernels of every other shape are the statements alone.
template <typename T, int K, int MAXT, bool DBG, int EXT>
__device__ __forceinline__ void sweep_body(SweepArgs a) {
#include "sweep_body.inc"
}

// In a batch of windows of different lengths, block b runs its window with
// blockK[b] sites per thread (4, 8, 12 or the launch's 16: the fewest that
// its workgroup holds), so a short window's workgroup is done in proportion
// to its length rather than as late as the longest window's.
template <typename T, int K, int MAXT, bool DBG, int EXT>
__global__ void __launch_bounds__(MAXT) sweep_kernel(SweepArgs a) {
  if constexpr (K == 16 && sizeof(T) == 4 && EXT == 0) {
    const int kb = a.blockK ? (int)a.blockK[blockIdx.x] : K;
    if (kb == 4) {
      sweep_body<T, 4, MAXT, DBG, EXT>(a);
      return;
    }
    if (kb == 8) {
      sweep_body<T, 8, MAXT, DBG, EXT>(a);
      return;
    }
    if (kb == 12) {
      sweep_body<T, 12, MAXT, DBG, EXT>(a);
      return;
    }
  }
#include "sweep_body.inc"
}

__global__ void zero_u32_kernel(uint32_t* p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

int clear_words(void* p, size_t n, hipStream_t s) {
  if (!n) return PIMC_OK;
  hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (uint32_t*)p, n);
  return hipGetLastError() == hipSuccess ? PIMC_OK : PIMC_ERR_HIP;
}

// Launch limits of one kernel at one launch shape on one device: whether
// its static plus dynamic LDS and its thread count fit a workgroup, and how
// many of its workgroups the device holds at once.  Queried from the runtime
// once per (kernel, device, threads, LDS) and kept for the process, so that
// a call's host cost is the launch itself.
struct LaunchLimits {
  bool fits;
  int64_t resident;
};

static int launch_limits(const void* k, int dev, int NT, size_t sm, LaunchLimits& out) {
  struct Key {
    const void* k;
    int dev, NT;
    size_t sm;
    bool operator<(const Key& o) const {
      return std::tie(k, dev, NT, sm) < std::tie(o.k, o.dev, o.NT, o.sm);
    }
  };
  static std::mutex mu;
  static std::map<Key, LaunchLimits> cache;
  const Key key{k, dev, NT, sm};
  {
    std::lock_guard<std::mutex> lock(mu);
    const auto it = cache.find(key);
    if (it != cache.end()) {
      out = it->second;
      return PIMC_OK;
    }
  }
  hipFuncAttributes at;
  int lim = 0, per_cu = 0, ncu = 0;
  if (hipFuncGetAttributes(&at, k) != hipSuccess ||
      hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return PIMC_ERR_HIP;
  LaunchLimits l;
  l.fits = sm + at.sharedSizeBytes <= (size_t)lim && NT <= at.maxThreadsPerBlock;
  l.resident = 0;
  if (l.fits) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, NT, sm) != hipSuccess) return PIMC_ERR_HIP;
    l.resident = (int64_t)per_cu * ncu;
  }
  std::lock_guard<std::mutex> lock(mu);
  cache[key] = l;
  out = l;
  return PIMC_OK;
}

// The launch is refused on the host (never enqueued) when the kernel's static
// LDS plus the requested dynamic LDS exceeds what a workgroup may allocate.
template <typename Kern>
static int launch_checked(Kern k, int nblocks, int NT, size_t sm, hipStream_t s, const SweepArgs& a) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PIMC_ERR_HIP;
  LaunchLimits l;
  const int r = launch_limits((const void*)k, dev, NT, sm, l);
  if (r) return r;
  if (!l.fits) return PIMC_ERR_UNSUPPORTED;
  // tiles wait on each other, so all of them must be resident at once: a
  // shape the device cannot hold is refused before anything is enqueued.
  // Every tile is then resident once launched: the waits between tiles are
  // bounded, so a tile that cannot be placed (other work holding the CUs)
  // ends the launch with a timeout, never a hang
  if (a.tiles > 1 && l.resident < nblocks) return PIMC_ERR_UNSUPPORTED;
  hipLaunchKernelGGL(k, dim3(nblocks), dim3(NT), sm, s, a);
  return hipGetLastError() == hipSuccess ? PIMC_OK : PIMC_ERR_HIP;
}

// One launch shape: an extended kernel when asked for (ext 1: the
// initialization phase, kinetic constants and exact draws; ext 2: exact
// draws only; one wave per SIMD and at most 4 sites per thread), the debug
// kernel when a debug record is, else the plain kernel.
template <typename T, int K, int MAXT>
static int launch_shape(const SweepArgs& a, bool dbg, int ext, int nblocks, int NT, size_t sm, hipStream_t s) {
  if (ext) {
    if constexpr (MAXT <= 256 && K <= 4) {
      if (ext == 2) return launch_checked(sweep_kernel<T, K, MAXT, false, 2>, nblocks, NT, sm, s, a);
      return launch_checked(sweep_kernel<T, K, MAXT, false, 1>, nblocks, NT, sm, s, a);
    } else {
      return PIMC_ERR_UNSUPPORTED;
    }
  }
  if (dbg) return launch_checked(sweep_kernel<T, K, MAXT, true, 0>, nblocks, NT, sm, s, a);
  return launch_checked(sweep_kernel<T, K, MAXT, false, 0>, nblocks, NT, sm, s, a);
}

// Launch bounds follow the thread count: up to 256 threads (one wave per
// SIMD) a wave may hold 512 registers (architectural + accumulation), so the
// register-resident path never spills to scratch.
template <typename T, int K, int BIG>
static int launch_pick(const SweepArgs& a, bool dbg, int ext, int nblocks, int NT, size_t sm, hipStream_t s) {
  if (NT <= 256) return launch_shape<T, K, 256>(a, dbg, ext, nblocks, NT, sm, s);
  return launch_shape<T, K, BIG>(a, dbg, ext, nblocks, NT, sm, s);
}

int launch_sweep(const SweepArgs& a, bool fp64, int K, int nblocks, int NT, hipStream_t s, int ext) {
  const size_t sm = sweep_smem_bytes(NT, K, fp64, a.stage);
  if (sm + LDS_STATIC_RESERVE > LDS_BYTES || NT > sweep_max_threads(fp64, K)) return PIMC_ERR_UNSUPPORTED;
  const bool dbg = a.dbg_xprop || a.dbg_dA || a.dbg_acc || a.dbg_pprop || a.dbg_pdA || a.dbg_pacc;
  // the extended kernels record the parameter and kinetic moves, not sites
  if (ext && (a.dbg_xprop || a.dbg_dA || a.dbg_acc)) return PIMC_ERR_UNSUPPORTED;
  // the extended kernels run with at most 4 sites per thread: two test runs
  // that launched them with 16 (exact draws, then the initialization phase,
  // each a single workgroup of 256 threads on a 4096-step window) were
  // followed by GPU faults whose cause is not identified, and the shapes of
  // 2 and 4 sites per thread are the ones their tests have run throughout
  if (ext && K > 4) return PIMC_ERR_UNSUPPORTED;
  if (fp64) {
    if (K != 4 || NT > 256) return PIMC_ERR_UNSUPPORTED;   // wide FP64 shapes are not launched
    return launch_shape<double, 4, 256>(a, dbg, ext, nblocks, NT, sm, s);
  }
  switch (K) {
    case 2:
      if (NT > 256) return PIMC_ERR_UNSUPPORTED;   // a tiling option: one wave per SIMD only
      return launch_shape<float, 2, 256>(a, dbg, ext, nblocks, NT, sm, s);
    case 4: return launch_pick<float, 4, 1024>(a, dbg, ext, nblocks, NT, sm, s);
    case 8: return launch_pick<float, 8, 512>(a, dbg, ext, nblocks, NT, sm, s);
    case 16: return launch_pick<float, 16, 512>(a, dbg, ext, nblocks, NT, sm, s);
    default: return PIMC_ERR_UNSUPPORTED;
  }
}

}  // namespace pimc
