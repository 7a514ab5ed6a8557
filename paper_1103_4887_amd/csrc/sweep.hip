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
  const double lu = ::log(u01_d(uword));
  const bool fin = __builtin_isfinite(dA);
  const bool acc = inbox && fin && (lu < -dA);
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
template <int L>
__device__ __forceinline__ void param_move(const SweepArgs& a, Key key, uint64_t k, bool uniform_prop,
                                           const double (&wpar)[7], double (&pd)[7], double (&s)[7],
                                           const double (&G)[28], bool& changed, int& acc, int& nonfin,
                                           bool last, int win) {
  if (!((a.m.p_mask >> L) & 1)) return;
  const U4 b = draw(key, (uint32_t)L, k, TAG_PARAM);
  double z, z1;
  if (uniform_prop)
    z = Math<double>::uniform_pm1(b.x);
  else
    Math<double>::box_muller(b.x, b.y, z, z1);
  const double u = u01_d(b.z);
  const double pl = pd[L] + wpar[L] * z;
  double dA = __builtin_nan("");
  bool ok = false;
  if (pl >= a.m.p_lo[L] && pl <= a.m.p_hi[L]) {
    constexpr int ia = ThetaMove<L>::ia, ib = ThetaMove<L>::ib;
    const double dp = pl - pd[L];
    // p2, p4, p6 move theta_l and theta_{l+1} = p_l p_{l+1}; p3, p5, p7 move p_{l-1} p_l
    const double da = (L == 2 || L == 4 || L == 6) ? pd[L - 1 < 0 ? 0 : L - 1] * dp : dp;
    const double db = ib >= 0 ? dp * pd[ib >= 0 ? ib : 0] : 0.0;
    double quad = da * da * G[symi(ia, ia)];
    double lin = da * s[ia];
    if (ib >= 0) {
      quad += 2.0 * da * db * G[symi(ia, ib >= 0 ? ib : 0)] + db * db * G[symi(ib >= 0 ? ib : 0, ib >= 0 ? ib : 0)];
      lin += db * s[ib >= 0 ? ib : 0];
    }
    dA = 0.5 * a.m.beta * a.m.Rd[0] * (quad - 2.0 * lin);
    const bool fin = __builtin_isfinite(dA);
    ok = fin && (::log(u) < -dA);
    if (!fin) ++nonfin;
    if (ok) {
#pragma unroll
      for (int j = 0; j < 7; ++j) {
        double gs = G[symi(j, ia)] * da;
        if (ib >= 0) gs += G[symi(j, ib >= 0 ? ib : 0)] * db;
        s[j] -= gs;
      }
      pd[L] = pl;
      changed = true;
      ++acc;
    }
  }
  if (last) {
    if (a.dbg_pprop) a.dbg_pprop[win * 7 + L] = pl;
    if (a.dbg_pdA) a.dbg_pdA[win * 7 + L] = dA;
    if (a.dbg_pacc) a.dbg_pacc[win * 7 + L] = ok;
  }
}

}  // namespace

template <typename T, int K, int MAXT, bool DBG>
__global__ void __launch_bounds__(MAXT) sweep_kernel(SweepArgs a) {
  static_assert(K % 4 == 0, "K must be a multiple of 4");
  extern __shared__ __align__(16) unsigned char smem[];
  const int NT = blockDim.x;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wv = t >> 6;
  const int NW = NT >> 6;

  const int win = a.order ? a.order[blockIdx.x] : (int)blockIdx.x;
  int64_t base = 0;
  int M = (int)a.M_single;
  if (a.offsets) {
    base = a.offsets[win];
    M = (int)(a.offsets[win + 1] - base - 1);
  }
  const uint32_t chain = a.chain_ids ? a.chain_ids[win] : a.chain_single;
  const Key key = make_key(a.seed, chain);
  double* P = a.p + (int64_t)win * 7;

  T* lfirst = (T*)smem;          // [NT][8]
  T* llast = lfirst + NT * 8;    // [NT][8]
  double* lred = (double*)(llast + NT * 8);  // [16][NRED]
  double* lstat = lred + 16 * NRED;          // [NRED]
  double* lpar = lstat + NRED;               // [8]: p, changed flag
  int* lcnt = (int*)(lpar + 8);              // [16] counters

  Consts<T> C;
  C.init(a.m);
  double pd[7];
#pragma unroll
  for (int l = 0; l < 7; ++l) pd[l] = P[l];
  C.set_p(pd);
  T ws[4];
  double wpar[7];
#pragma unroll
  for (int c = 0; c < 4; ++c) ws[c] = (T)a.w[c];
#pragma unroll
  for (int l = 0; l < 7; ++l) wpar[l] = a.w[4 + l];
  const bool uniform_prop = a.m.proposal == PIMC_PROP_UNIFORM;
  const double hD = 0.5 * a.m.dt;

  // ---- own sites: n = n0 + j, j < K, plus site M on the last thread when
  //      the regular slots stop exactly at M ------------------------------
  const int NTneed = (M + K - 1) / K;
  const bool active = t < NTneed;
  const int n0 = t * K;
  const bool has_extra = (t == NTneed - 1) && (K * NTneed == M);
  // per-thread base pointers: every slot access below is a constant offset
  T* Xt = (T*)a.X + (base + n0) * 4;
  const T* Yt = (const T*)a.y + base + n0;
  const T* It = (const T*)a.I + base + n0;

  T x[K][4], F[K][4], yv[K], Iv[K];
  T xe[4], Fe[4], ye = 0, Ie = 0;
  bool bad = false;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const bool v = active && n0 + j <= M;
#pragma unroll
    for (int c = 0; c < 4; ++c) x[j][c] = v ? Xt[j * 4 + c] : C.lo[c];
    yv[j] = v ? Yt[j] : (T)0;
    Iv[j] = v ? It[j] : (T)0;
    hh_F(C, x[j], Iv[j], F[j]);
    if (v) {
#pragma unroll
      for (int c = 0; c < 4; ++c) bad = bad || !(x[j][c] >= C.lo[c] && x[j][c] <= C.hi[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) xe[c] = has_extra ? Xt[K * 4 + c] : C.lo[c];
  if (has_extra) {
    ye = Yt[K];
    Ie = It[K];
#pragma unroll
    for (int c = 0; c < 4; ++c) bad = bad || !(xe[c] >= C.lo[c] && xe[c] <= C.hi[c]);
  }
  hh_F(C, xe, Ie, Fe);
  if (t == 0) {
#pragma unroll
    for (int l = 0; l < 7; ++l) {
      bad = bad || !__builtin_isfinite(pd[l]);
      if ((a.m.p_mask >> l) & 1) bad = bad || !(pd[l] >= a.m.p_lo[l] && pd[l] <= a.m.p_hi[l]);
    }
  }
  if (__syncthreads_or(bad)) {
    if (t == 0) atomicOr(a.err, 2u);
    return;
  }
  if (active) {
    lds_put(lfirst + t * 8, x[0], F[0]);
    lds_put(llast + t * 8, x[K - 1], F[K - 1]);
  }
  __syncthreads();

  int accE = 0, accO = 0, nonfin = 0;
  int accP[7] = {0, 0, 0, 0, 0, 0, 0};
  T* dx_t = DBG && a.dbg_xprop ? (T*)a.dbg_xprop + (base + n0) * 4 : nullptr;
  double* ddA_t = DBG && a.dbg_dA ? a.dbg_dA + base + n0 : nullptr;
  uint8_t* dacc_t = DBG && a.dbg_acc ? a.dbg_acc + base + n0 : nullptr;

  for (int64_t it = 0; it < a.n_sweeps; ++it) {
    const uint64_t k = a.sweep0 + (uint64_t)it;
    const bool last = it == a.n_sweeps - 1;

    if (a.flags & PIMC_STATES) {
      // ---- even half-sweep ----------------------------------------------
      uint32_t uodd[K / 2];
#pragma unroll
      for (int q = 0; q < K / 4; ++q) {
        const int j0 = 4 * q;
        U4 ub{0, 0, 0, 0};
        if (active && n0 + j0 <= M) ub = draw(key, opaque((uint32_t)((n0 + j0) >> 2)), k, TAG_SACC);
        uodd[2 * q] = ub.y;
        uodd[2 * q + 1] = ub.w;
#pragma unroll
        for (int jj = 0; jj < 4; jj += 2) {
          const int j = j0 + jj;
          const int nn = n0 + j;
          if (active && nn <= M) {
            Nb<T> L, R;
            const bool hasL = nn >= 1;
            if (j == 0) {
              if (hasL) lds_get(C, llast + (t - 1) * 8, It[-1], L);
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
            const bool ok = site_update(C, ws, uniform_prop, x[j], F[j], yv[j], Iv[j], hasL, L, hasR, R,
                                        nn >= 1, blk, jj == 0 ? ub.x : ub.z, dA, xp, nonfin);
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
        double dA;
        T xp[4];
        const bool ok = site_update(C, ws, uniform_prop, xe, Fe, ye, Ie, true, L, false, R, true, blk, ub.x,
                                    dA, xp, nonfin);
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
              } else {
                lds_get(C, lfirst + (t + 1) * 8, It[K], R);
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
          const bool ok = site_update(C, ws, uniform_prop, x[j], F[j], yv[j], Iv[j], true, L, hasR, R, true, blk,
                                      uodd[j >> 1], dA, xp, nonfin);
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
    }

    if (a.flags & PIMC_PARAMS) {
      // ---- sufficient statistics over the links of the odd sites ----------
      double th[7];
      theta_of(pd, th);
      double st[NRED];
#pragma unroll
      for (int i = 0; i < NRED; ++i) st[i] = 0.0;
      if (active) {
        Feat fl = feat_of(x[0], Iv[0]);
#pragma unroll
        for (int j = 1; j < K; j += 2) {
          const int nn = n0 + j;
          if (nn <= M) {
            const Feat fc = feat_of(x[j], Iv[j]);
            link_stats(th, hD, fl, fc, st);
            if (nn + 1 <= M) {
              Feat fr;
              if (j == K - 1) {
                if (has_extra) {
                  fr = feat_of(xe, Ie);
                } else {
                  T xr[4];
#pragma unroll
                  for (int c = 0; c < 4; ++c) xr[c] = lfirst[(t + 1) * 8 + c];
                  fr = feat_of(xr, It[K]);
                }
              } else {
                fr = feat_of(x[j + 1], Iv[j + 1]);
              }
              link_stats(th, hD, fc, fr, st);
              fl = fr;
            }
          }
        }
      }
      // ---- block reduction (fixed order for a given launch shape) ---------
#pragma unroll
      for (int i = 0; i < NRED; ++i) {
        double v = st[i];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
        st[i] = v;
      }
      if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NRED; ++i) lred[wv * NRED + i] = st[i];
      }
      __syncthreads();
      if (t < NRED) {
        double s = 0.0;
        for (int q = 0; q < NW; ++q) s += lred[q * NRED + t];
        lstat[t] = s;
      }
      __syncthreads();
      // ---- sequential parameter moves (one lane) --------------------------
      if (t == 0) {
        double s7[7], G[28];
#pragma unroll
        for (int l = 0; l < 7; ++l) s7[l] = lstat[l];
#pragma unroll
        for (int i = 0; i < 28; ++i) G[i] = lstat[7 + i];
        bool changed = false;
        param_move<0>(a, key, k, uniform_prop, wpar, pd, s7, G, changed, accP[0], nonfin, last, win);
        param_move<1>(a, key, k, uniform_prop, wpar, pd, s7, G, changed, accP[1], nonfin, last, win);
        param_move<2>(a, key, k, uniform_prop, wpar, pd, s7, G, changed, accP[2], nonfin, last, win);
        param_move<3>(a, key, k, uniform_prop, wpar, pd, s7, G, changed, accP[3], nonfin, last, win);
        param_move<4>(a, key, k, uniform_prop, wpar, pd, s7, G, changed, accP[4], nonfin, last, win);
        param_move<5>(a, key, k, uniform_prop, wpar, pd, s7, G, changed, accP[5], nonfin, last, win);
        param_move<6>(a, key, k, uniform_prop, wpar, pd, s7, G, changed, accP[6], nonfin, last, win);
#pragma unroll
        for (int l = 0; l < 7; ++l) lpar[l] = pd[l];
        lpar[7] = changed ? 1.0 : 0.0;
      }
      __syncthreads();
      if (lpar[7] != 0.0) {
#pragma unroll
        for (int l = 0; l < 7; ++l) pd[l] = lpar[l];
        C.set_p(pd);
#pragma unroll
        for (int j = 0; j < K; ++j) F[j][0] = hh_FV(C, x[j][0], x[j][1], x[j][2], x[j][3], Iv[j]);
        Fe[0] = hh_FV(C, xe[0], xe[1], xe[2], xe[3], Ie);
      }
    } else {
      __syncthreads();
    }

    // ---- statistics ------------------------------------------------------
    if (a.ptrace && t == 0) {
#pragma unroll
      for (int l = 0; l < 7; ++l) a.ptrace[(int64_t)win * a.n_sweeps * 7 + it * 7 + l] = pd[l];
    }
    if (a.sum && (int64_t)k >= a.burn && active) {
      const T* xr = (const T*)a.xref + (base + n0) * 4;
      double* su = a.sum + (base + n0) * 4;
      double* sq = a.sumsq ? a.sumsq + (base + n0) * 4 : nullptr;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        if (n0 + j <= M) {
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const double d = (double)x[j][c] - (double)xr[j * 4 + c];
            su[j * 4 + c] += d;
            if (sq) sq[j * 4 + c] += d * d;
          }
        }
      }
      if (has_extra) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double d = (double)xe[c] - (double)xr[K * 4 + c];
          su[K * 4 + c] += d;
          if (sq) sq[K * 4 + c] += d * d;
        }
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
  if (t == 0) {
#pragma unroll
    for (int l = 0; l < 7; ++l) P[l] = pd[l];
  }
  // ---- acceptance counters ----------------------------------------------
  if (t < 16) lcnt[t] = 0;
  __syncthreads();
  if (accE) atomicAdd(&lcnt[0], accE);
  if (accO) atomicAdd(&lcnt[1], accO);
  if (nonfin) atomicAdd(&lcnt[9], nonfin);
  if (t == 0) {
#pragma unroll
    for (int l = 0; l < 7; ++l) lcnt[2 + l] += accP[l];
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

size_t sweep_smem_bytes(int NT, bool fp64) {
  const size_t ts = fp64 ? 8 : 4;
  return (size_t)NT * 8 * ts * 2 + (16 * NRED + NRED + 8) * sizeof(double) + 16 * sizeof(int);
}

#define PIMC_SWEEP_LAUNCH(T, K, MAXT)                                                          \
  do {                                                                                         \
    if (dbg)                                                                                   \
      hipLaunchKernelGGL((sweep_kernel<T, K, MAXT, true>), dim3(nblocks), dim3(NT), sm, s, a);  \
    else                                                                                       \
      hipLaunchKernelGGL((sweep_kernel<T, K, MAXT, false>), dim3(nblocks), dim3(NT), sm, s, a); \
  } while (0)

int launch_sweep(const SweepArgs& a, bool fp64, int K, int nblocks, int NT, hipStream_t s) {
  const size_t sm = sweep_smem_bytes(NT, fp64);
  const bool dbg = a.dbg_xprop || a.dbg_dA || a.dbg_acc || a.dbg_pprop || a.dbg_pdA || a.dbg_pacc;
  if (fp64) {
    switch (K) {
      case 4: PIMC_SWEEP_LAUNCH(double, 4, 1024); break;
      case 8: PIMC_SWEEP_LAUNCH(double, 8, 512); break;
      default: return PIMC_ERR_UNSUPPORTED;
    }
  } else {
    switch (K) {
      case 4: PIMC_SWEEP_LAUNCH(float, 4, 1024); break;
      case 8: PIMC_SWEEP_LAUNCH(float, 8, 512); break;
      case 16: PIMC_SWEEP_LAUNCH(float, 16, 512); break;
      default: return PIMC_ERR_UNSUPPORTED;
    }
  }
  return hipGetLastError() == hipSuccess ? PIMC_OK : PIMC_ERR_HIP;
}

int sweep_max_threads(bool fp64, int K) {
  if (K == 4) return 1024;
  if (K == 8 || (!fp64 && K == 16)) return 512;
  return 0;
}

}  // namespace pimc
