// Hybrid Monte Carlo proposals on the path action, for many chains at once.
//
// The paper names Hybrid Monte Carlo among the samplers of exp(-A) (Section 3)
// and derivative-based proposals as a way to converge in fewer iterations
// (Section 3.1).  One proposal for every chain of a packed batch:
//
//   r ~ N(0, 1/minv) per site component and sampled parameter
//   H0 = A(q0) + 1/2 sum r^2 minv                          (FP64)
//   r(1/2) = r0 - e/2 g(q0)
//   for s = 1..L:  q(s) = q(s-1) + e minv r(s-1/2);  g(s) = dA/dq at q(s)
//                  r(s+1/2) = r(s-1/2) - e g(s)  (the last step kicks e/2)
//   H1 = A(qL) + 1/2 sum rL^2 minv;  accept iff log u < -(H1 - H0)
//   and every drift ended inside the box.
//
// A coordinate that a drift carries across a wall of its box is reflected
// back and its momentum negated (constraint handling by reflection, Neal,
// "MCMC using Hamiltonian dynamics", 2011, Section 5.1: reversible and volume
// preserving, so the target exp(-A) on the box is unchanged).  One reflection
// per drift; a coordinate still outside afterwards invalidates the trajectory.
//
// One kernel per leapfrog step over all chains' sites (blocks of 256 sites
// of one chain, plus one halo site on each side whose drift is recomputed
// locally), positions and momenta double-buffered by step parity, FP64
// partials per block.  Every kernel of the parameter part reduces the
// previous kernel's partials of its chain in block order, so all blocks of a
// chain hold identical parameter values without any inter-block wait.  The
// proposal index is read from device memory, so the launch sequence of one
// proposal is fixed and can be captured and replayed.
#include "device.hpp"
#include "hmc.hpp"

namespace pimc {

namespace {

constexpr int HB = HMC_BLOCK;  // sites per block = threads per block
constexpr int NPART = 10;      // gp[7], A_o, A_d, K

// Sum over the blocks b0..b1-1 of one chain of the per-block partials
// part[b][off + v], v < N, in a fixed order that every block of the chain
// reproduces: thread (v, g) = (t % N, t / N) adds blocks b0 + g, b0 + g + G,
// ... (G = 256 / N segments, all loads of a segment independent), then the
// segment sums are added in segment order.  lds: [256] doubles; out: [N] in
// LDS, valid for every thread after the call.
template <int N>
__device__ __forceinline__ void chain_sum(const double* part, int b0, int b1, int off, double* lds, double* out,
                                          int t) {
  constexpr int G = HB / N;
  const int v = t % N, g = t / N;
  if (g < G) {
    double acc = 0.0;
    for (int b = b0 + g; b < b1; b += G) acc += part[(int64_t)b * 16 + off + v];
    lds[g * N + v] = acc;
  }
  __syncthreads();
  if (t < N) {
    // segments past the chain's block count hold nothing
    const int gmax = b1 - b0 < G ? b1 - b0 : G;
    double acc = 0.0;
    for (int q = 0; q < gmax; ++q) acc += lds[q * N + t];
    out[t] = acc;
  }
  __syncthreads();
}

template <typename T>
struct HmcJ {  // Jacobian rows of the HH field
  T VV, Vg[3], gV[3], gg[3];
};


// F and its Jacobian at one site, sharing the gates' tanh and 1/tau.
template <typename T>
__device__ __forceinline__ void hh_F_J(const Consts<T>& C, const T (&x)[4], T I, T (&F)[4], HmcJ<T>& J) {
  const T V = x[0], m = x[1], hh = x[2], n = x[3];
  const T m2 = m * m, m3 = m2 * m, n2 = n * n, n3 = n2 * n, n4 = n2 * n2;
  F[0] = hh_FV(C, V, m, hh, n, I);
  J.VV = -(C.p[1] * m3 * hh + C.p[3] * n4 + C.p[5]);
  J.Vg[0] = (T)3 * C.p[1] * m2 * hh * (C.p[2] - V);
  J.Vg[1] = C.p[1] * m3 * (C.p[2] - V);
  J.Vg[2] = (T)4 * C.p[3] * n3 * (C.p[4] - V);
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    const T t = Math<T>::tanh((V - C.Va[g]) * C.inv_dVa[g]);
    const T sech2 = (T)1 - t * t;
    const T ainf = (T)0.5 + (T)0.5 * t;
    const T tau = C.tau0[g] + C.tau1[g] * sech2;
    const T itau = Math<T>::rcp(tau);
    F[1 + g] = (ainf - x[1 + g]) * itau;
    const T dt_dV = sech2 * C.inv_dVa[g];
    J.gV[g] = (T)0.5 * dt_dV * itau - (ainf - x[1 + g]) * ((T)-2 * C.tau1[g] * t * dt_dV) * itau * itau;
    J.gg[g] = -itau;
  }
}

// Sum N values over the HB threads of a block: DPP sums over rows of 16
// lanes, then the HB / 16 row partials added in row order by thread i < N,
// which writes sum i to out[i].  lds: [HB / 16][N] doubles.
template <int N>
__device__ __forceinline__ void block_sum_rows(const double (&v)[N], double* lds, double* out, int t) {
  double r[N];
#pragma unroll
  for (int i = 0; i < N; ++i) r[i] = row_sum(v[i]);
  if ((t & 15) == 15) {
#pragma unroll
    for (int i = 0; i < N; ++i) lds[(t >> 4) * N + i] = r[i];
  }
  __syncthreads();
  if (t < N) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < HB / 16; ++q) acc += lds[q * N + t];
    out[t] = acc;
  }
}

// dF_V/dp at a site in the site precision (parameters from C)
template <typename T>
__device__ __forceinline__ void dFVdp_T(const Consts<T>& C, T V, T m, T h, T n, T I, T (&d)[7]) {
  const T m3h = m * m * m * h, n2 = n * n, n4 = n2 * n2;
  d[0] = I;
  d[1] = m3h * (C.p[2] - V);
  d[2] = C.p[1] * m3h;
  d[3] = n4 * (C.p[4] - V);
  d[4] = C.p[3] * n4;
  d[5] = C.p[6] - V;
  d[6] = C.p[5];
}


// Parameter part of a leapfrog step for one chain: the momentum
// rp(s-1/2) = rp_in - c e gp (c = 1/2 on the first step), then the drift
// p(s) = p_in + e minv rp(s-1/2), reflected once at the box walls with the
// momentum negated.
__device__ __forceinline__ void param_drift(const HmcArgs& a, double c, const double (&gp)[7],
                                            const double (&rp_in)[7], const double (&p_in)[7], double (&ps)[7],
                                            double (&rps)[7]) {
#pragma unroll
  for (int l = 0; l < 7; ++l) {
    const bool on = (a.m.p_mask >> l) & 1;
    rps[l] = on ? rp_in[l] - c * a.eps * gp[l] : 0.0;
    double q = on ? p_in[l] + a.eps * a.minv[4 + l] * rps[l] : p_in[l];
    if (on && q < a.m.p_lo[l]) {
      q = 2.0 * a.m.p_lo[l] - q;
      rps[l] = -rps[l];
    } else if (on && q > a.m.p_hi[l]) {
      q = 2.0 * a.m.p_hi[l] - q;
      rps[l] = -rps[l];
    }
    ps[l] = q;
  }
}

// Parameter state of chain `ch` at leapfrog kernel s (identical in every
// block of the chain): p(s), and the momentum rp(s-1/2) that moved it there.
__device__ __forceinline__ void chain_params(const HmcArgs& a, int ch, int s, double (&ps)[7], double (&rps)[7],
                                             double* red) {
  const int b0 = a.bfirst[ch], b1 = a.bfirst[ch + 1];
  const double* part = a.part + (int64_t)((s - 1) & 1) * a.nblocks * 16;
  // fixed-order reduction of the previous kernel's partials of this chain
  chain_sum<7>(part, b0, b1, 0, red + 16, red, (int)threadIdx.x);
  double gp[7], rp_in[7], p_in[7];
  const double* rpi = a.rpbuf + (int64_t)((s - 1) & 1) * a.B * 7 + (int64_t)ch * 7;
  const double* pi = s == 1 ? a.p + (int64_t)ch * 7 : a.pbuf + (int64_t)((s - 1) & 1) * a.B * 7 + (int64_t)ch * 7;
#pragma unroll
  for (int l = 0; l < 7; ++l) {
    gp[l] = red[l];
    rp_in[l] = rpi[l];
    p_in[l] = pi[l];
  }
  param_drift(a, s == 1 ? 0.5 : 1.0, gp, rp_in, p_in, ps, rps);
}

// One drift of a site, q + e minv r, reflected once at the walls of the
// state box; bit c of the result marks a reflected component (its momentum
// is negated at the kick).
template <typename T>
__device__ __forceinline__ uint32_t drift_site(const Consts<T>& C, const T (&minv)[4], T e, T (&q)[4],
                                               const T (&r)[4]) {
  uint32_t flip = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    q[c] = q[c] + e * minv[c] * r[c];
    if (q[c] < C.lo[c]) {
      q[c] = (T)2 * C.lo[c] - q[c];
      flip |= 1u << c;
    } else if (q[c] > C.hi[c]) {
      q[c] = (T)2 * C.hi[c] - q[c];
      flip |= 1u << c;
    }
  }
  return flip;
}

// dA/dx at site n (LDS index j) from the stencil of positions lq and fields
// lF with the site's Jacobian J; w0 = beta Rd_V (eps_V of link n + eps_V of
// link n + 1), the links that exist.
template <typename T>
__device__ __forceinline__ void site_grad(const HmcArgs& a, const Consts<T>& C, const HmcJ<T>& J,
                                          const T (*lq)[4], const T (*lF)[4], int j, int n, int M, T y_own,
                                          const T (&x)[4], T (&g)[4], T& w0) {
  const T h = C.h;
  const T beta = (T)a.m.beta;
  T vl[4] = {0, 0, 0, 0}, vr[4] = {0, 0, 0, 0};
  if (n >= 1) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const T el = (x[c] - lq[j - 1][c]) - h * (lF[j][c] + lF[j - 1][c]);
      vl[c] = beta * (T)a.m.Rd[c] * el;
    }
  }
  if (n + 1 <= M) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
      vr[c] = beta * (T)a.m.Rd[c] * ((lq[j + 1][c] - x[c]) - h * (lF[j + 1][c] + lF[j][c]));
  }
  T u[4], w[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    u[c] = vl[c] - vr[c];
    w[c] = vl[c] + vr[c];
  }
  g[0] = u[0] - h * (J.VV * w[0] + J.gV[0] * w[1] + J.gV[1] * w[2] + J.gV[2] * w[3]);
#pragma unroll
  for (int q = 0; q < 3; ++q) g[1 + q] = u[1 + q] - h * (J.Vg[q] * w[0] + J.gg[q] * w[1 + q]);
  if (n >= 1) g[0] -= (T)a.m.Ro * (y_own - x[0]);
  w0 = w[0];
}

// dA/dp contribution of site n: dF_V/dp at the site enters the errors of
// its two links, so the link sum of the action's derivative regroups into
// -(dt/2) w0 dF_V/dp(x_n) per site (w0 from site_grad); per-site terms in
// the site precision, written as FP64 partials part[0..6].
template <typename T, int N>
__device__ __forceinline__ void site_dadp(const HmcArgs& a, const Consts<T>& C, const T* lI, int j, const T (&x)[4],
                                          T w0, double (&part)[N]) {
  T d[7];
  dFVdp_T(C, x[0], x[1], x[2], x[3], lI[j], d);
  const T f = (T)(-0.5 * a.m.dt) * w0;
#pragma unroll
  for (int l = 0; l < 7; ++l) part[l] = (double)(f * d[l]);
}

}  // namespace

// MODE 0: initial kernel (momenta, g(q0), H0 partials);
// MODE 1: interior leapfrog step; MODE 2: last step (half kick, H1 partials).
template <typename T, int MODE>
__global__ void __launch_bounds__(HB) hmc_step_kernel(HmcArgs a, int s) {
  __shared__ T lq[HB + 2][4];
  __shared__ T lF[HB + 2][4];
  __shared__ T lI[HB + 2];
  __shared__ double red[16 + HB];   // [0..15] results, then chain_sum scratch
  __shared__ double lsum[HB / 16 * NPART];
  __shared__ uint8_t lflip[HB + 2];   // bit c: component c reflected in this drift
  // FP64 fields for the Hamiltonian (first and last kernels, FP32 sites):
  // each site's once, shared by its two links
  constexpr bool F64 = MODE != 1 && sizeof(T) == 4;
  __shared__ double lF64[F64 ? HB + 2 : 1][4];
  const int t = threadIdx.x;
  const int b = blockIdx.x;
  const int ch = a.bmap[b];
  const int64_t base = a.offsets[ch];
  const int M = (int)(a.offsets[ch + 1] - base - 1);
  const int site0 = (b - a.bfirst[ch]) * HB;
  const uint64_t k = *a.kptr;
  const Key key = make_key(a.seed, a.chain[ch]);

  Consts<T> C;
  if constexpr (sizeof(T) == 4)
    C = a.cf;
  else
    C = a.cd;

  // ---- positions of the block's sites and the two halo sites: loaded,
  //      drifted and reflected before the parameter section, so that these
  //      loads and the parameter partials' loads share one memory round trip
  // lq[j] holds site n = site0 - 1 + j
  const T* Qin = (const T*)(MODE == 0 ? a.X : (((s - 1) & 1) ? a.Q1 : a.X)) + base * 4;
  const T* Rin = (const T*)(((s - 1) & 1) ? a.R1 : a.R0) + base * 4;   // r(s-1/2)
  const T* Ip = (const T*)a.I + base;
  const T* Yp = (const T*)a.y + base;
  const T e = (T)a.eps;
  {
    T minv_s[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) minv_s[c] = (T)a.minv[c];
    for (int j = t; j < HB + 2; j += HB) {
      const int n = site0 - 1 + j;
      if (n >= 0 && n <= M) {
        T q[4];
        uint32_t flip = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) q[c] = Qin[(int64_t)n * 4 + c];
        if (MODE != 0) {
          T rr[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) rr[c] = Rin[(int64_t)n * 4 + c];
          flip = drift_site(C, minv_s, e, q, rr);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) lq[j][c] = q[c];
        lflip[j] = (uint8_t)flip;
        lI[j] = Ip[n];
      }
    }
  }
  // the own site's momentum and observation, also loaded now
  const int n_own = site0 + t;
  T r_own[4] = {0, 0, 0, 0};
  T y_own = (T)0;
  if (n_own <= M) {
    if (MODE != 0) {
#pragma unroll
      for (int c = 0; c < 4; ++c) r_own[c] = Rin[(int64_t)n_own * 4 + c];
    }
    if (n_own >= 1) y_own = Yp[n_own];
  }

  // ---- parameters at this step -------------------------------------------
  double ps[7], rps[7];
  if (MODE == 0) {
#pragma unroll
    for (int l = 0; l < 7; ++l) ps[l] = a.p[(int64_t)ch * 7 + l];
  } else {
    chain_params(a, ch, s, ps, rps, red);
    bool out = false;
#pragma unroll
    for (int l = 0; l < 7; ++l)
      if ((a.m.p_mask >> l) & 1) out = out || !(ps[l] >= a.m.p_lo[l] && ps[l] <= a.m.p_hi[l]);
    if (b == a.bfirst[ch] && t == 0) {
      double* rp_out = a.rpbuf + (int64_t)(s & 1) * a.B * 7 + (int64_t)ch * 7;
      double* p_out = a.pbuf + (int64_t)(s & 1) * a.B * 7 + (int64_t)ch * 7;
#pragma unroll
      for (int l = 0; l < 7; ++l) {
        rp_out[l] = rps[l];
        p_out[l] = ps[l];
      }
      if (a.tp) {
#pragma unroll
        for (int l = 0; l < 7; ++l) {
          a.tp[((int64_t)s * a.B + ch) * 7 + l] = ps[l];
          a.trp[((int64_t)s * a.B + ch) * 7 + l] = rps[l];
        }
      }
      if (out) atomicOr(&a.outside[ch], 1u);
    }
    if (s == 1 && b == a.bfirst[ch]) {
      // H0 from the initial kernel's partials: A(q0) + K(r0) + K(rp0)
      chain_sum<3>(a.part /* parity 0 */, a.bfirst[ch], a.bfirst[ch + 1], 7, red + 16, red + 8, t);
      if (t == 0) {
        const double* rp0 = a.rpbuf + (int64_t)ch * 7;  // parity 0 holds rp0
        double Kp = 0.0;
#pragma unroll
        for (int l = 0; l < 7; ++l) Kp += 0.5 * rp0[l] * rp0[l] * a.minv[4 + l];
        a.H0[ch] = red[8] + a.m.beta * red[9] + red[10] + Kp;
      }
    }
  }
  C.set_p(ps);

  // ---- F at the block's sites with this step's parameters: thread t its
  //      own site (with the Jacobian, kept in registers), threads 0 and 1
  //      also the two halo sites -------------------------------------------
  __syncthreads();
  HmcJ<T> J;
  if (n_own <= M) {
    T q[4], F[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) q[c] = lq[t + 1][c];
    hh_F_J(C, q, lI[t + 1], F, J);
#pragma unroll
    for (int c = 0; c < 4; ++c) lF[t + 1][c] = F[c];
  }
  if (t < 2) {
    const int j = t == 0 ? 0 : HB + 1;
    const int n = site0 - 1 + j;
    if (n >= 0 && n <= M) {
      T q[4], F[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) q[c] = lq[j][c];
      hh_F(C, q, lI[j], F);
#pragma unroll
      for (int c = 0; c < 4; ++c) lF[j][c] = F[c];
    }
  }
  if constexpr (F64) {
    // own site and the left halo site (the links n - 1 -> n of the block)
    Consts<double> CD = a.cd;
    CD.set_p(ps);
    for (int j = t + 1; j >= t; --j) {
      const int n = site0 - 1 + j;
      if ((j == t + 1 || t == 0) && n >= 0 && n <= M) {
        double xd[4], Fd[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) xd[c] = (double)lq[j][c];
        hh_F(CD, xd, (double)lI[j], Fd);
#pragma unroll
        for (int c = 0; c < 4; ++c) lF64[j][c] = Fd[c];
      }
    }
  }
  __syncthreads();

  // ---- own site: gradient, kick, partials ---------------------------------
  const int n = site0 + t;
  const int j = t + 1;
  double part[NPART];
#pragma unroll
  for (int i = 0; i < NPART; ++i) part[i] = 0.0;
  if (n <= M) {
    T x[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) x[c] = lq[j][c];
    bool out = false;
    if (MODE != 0) {
#pragma unroll
      for (int c = 0; c < 4; ++c) out = out || !(x[c] >= C.lo[c] && x[c] <= C.hi[c]);
      if (out) atomicOr(&a.outside[ch], 1u);
    }
    T g[4], w0;
    site_grad(a, C, J, lq, lF, j, n, M, y_own, x, g, w0);

    // momenta: drawn (MODE 0) or r(s-1/2); kick; kinetic energy partial
    T r[4];
    if (MODE == 0) {
      const U4 blk = draw(key, (uint32_t)n, k, TAG_MOM);
      T z[4];
      Math<T>::box_muller(blk.x, blk.y, z[0], z[1]);
      Math<T>::box_muller(blk.z, blk.w, z[2], z[3]);
      double kin = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        r[c] = z[c] / (T)sqrt(a.minv[c]);
        kin += 0.5 * (double)r[c] * (double)r[c] * a.minv[c];
      }
      part[9] = kin;
    } else {
      const uint32_t flip = lflip[j];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        r[c] = r_own[c];
        if ((flip >> c) & 1u) r[c] = -r[c];
      }
    }
    const T kick = MODE == 1 ? e : e * (T)0.5;
    T rn[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) rn[c] = r[c] - kick * g[c];
    T* Rout = (T*)((s & 1) ? a.R1 : a.R0) + base * 4;
#pragma unroll
    for (int c = 0; c < 4; ++c) Rout[(int64_t)n * 4 + c] = rn[c];
    if (a.tq) {
      T* tq = (T*)a.tq + ((int64_t)s * a.S + base + n) * 4;
      T* tr = (T*)a.tr + ((int64_t)s * a.S + base + n) * 4;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        tq[c] = x[c];
        tr[c] = rn[c];
      }
    }
    if (MODE != 0) {
      T* Qout = (T*)((s & 1) ? a.Q1 : a.X) + base * 4;
#pragma unroll
      for (int c = 0; c < 4; ++c) Qout[(int64_t)n * 4 + c] = x[c];
    } else {
      T* X0 = (T*)a.X0 + base * 4;
#pragma unroll
      for (int c = 0; c < 4; ++c) X0[(int64_t)n * 4 + c] = x[c];
    }
    if (MODE == 2) {
      double kin = 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) kin += 0.5 * (double)rn[c] * (double)rn[c] * a.minv[c];
      part[9] = kin;
    }
    // action terms of link n (initial and last kernels), then dA/dp of site n
    if (n >= 1) {
      if (MODE != 1) {
        const double d = (double)y_own - (double)x[0];
        part[7] = 0.5 * a.m.Ro * d * d;
        double s2 = 0.0;
        // FP64 model error of link n for the Hamiltonian
        const double hd = a.cd.h;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double x1 = (double)x[c], x0 = (double)lq[j - 1][c];
          double F1, F0;
          if constexpr (F64) {
            F1 = lF64[j][c];
            F0 = lF64[j - 1][c];
          } else {   // FP64 sites: the fields of the step itself
            F1 = (double)lF[j][c];
            F0 = (double)lF[j - 1][c];
          }
          const double ee = (x1 - x0) - hd * (F1 + F0);
          s2 += a.m.Rd[c] * ee * ee;
        }
        part[8] = 0.5 * s2;
      }
    }
    site_dadp(a, C, lI, j, x, w0, part);
  }
  // ---- block partials (interior steps carry only dA/dp) --------------------
  double* pout = a.part + (int64_t)(s & 1) * a.nblocks * 16 + (int64_t)b * 16;
  if (MODE == 1) {
    double v[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) v[i] = part[i];
    block_sum_rows<7>(v, lsum, pout, t);
  } else {
    block_sum_rows<NPART>(part, lsum, pout, t);
  }
  if (MODE == 0 && b == a.bfirst[ch] && t == 0) {
    // parameter momenta and backups, chain-level (one block per chain)
    const U4 q0 = draw(key, 0u, k, TAG_PMOM, 0);
    const U4 q1 = draw(key, 0u, k, TAG_PMOM, 1);
    double z[8];
    Math<double>::box_muller(q0.x, q0.y, z[0], z[1]);
    Math<double>::box_muller(q0.z, q0.w, z[2], z[3]);
    Math<double>::box_muller(q1.x, q1.y, z[4], z[5]);
    Math<double>::box_muller(q1.z, q1.w, z[6], z[7]);
    double* rp0 = a.rpbuf + (int64_t)ch * 7;   // parity 0
#pragma unroll
    for (int l = 0; l < 7; ++l) {
      const bool on = (a.m.p_mask >> l) & 1;
      rp0[l] = on ? z[l] / sqrt(a.minv[4 + l]) : 0.0;
      a.p0[(int64_t)ch * 7 + l] = ps[l];
      if (a.tp) {
        a.tp[(int64_t)ch * 7 + l] = ps[l];
        a.trp[(int64_t)ch * 7 + l] = rp0[l];
      }
    }
    a.outside[ch] = 0u;
  }
}

// One block per chain: H1, decision, parameters, counters.
__global__ void __launch_bounds__(HB) hmc_finish_kernel(HmcArgs a, int L) {
  __shared__ double red[16 + HB];
  const int ch = blockIdx.x;
  const double* part = a.part + (int64_t)(L & 1) * a.nblocks * 16;
  chain_sum<NPART>(part, a.bfirst[ch], a.bfirst[ch + 1], 0, red + 16, red, (int)threadIdx.x);
  if (threadIdx.x != 0) return;
  const uint64_t k = *a.kptr;
  const Key key = make_key(a.seed, a.chain[ch]);
  double gp[7];
#pragma unroll
  for (int l = 0; l < 7; ++l) gp[l] = red[l];
  const double Ao = red[7], Ad = red[8], Ks = red[9];
  const double* rpL = a.rpbuf + (int64_t)(L & 1) * a.B * 7 + (int64_t)ch * 7;   // rp(L-1/2)
  const double* pL = a.pbuf + (int64_t)(L & 1) * a.B * 7 + (int64_t)ch * 7;
  double Kp = 0.0;
#pragma unroll
  for (int l = 0; l < 7; ++l) {
    const bool on = (a.m.p_mask >> l) & 1;
    const double r = on ? rpL[l] - 0.5 * a.eps * gp[l] : 0.0;
    Kp += 0.5 * r * r * a.minv[4 + l];
    if (a.trp) a.trp[((int64_t)(L + 1) * a.B + ch) * 7 + l] = r;
  }
  const double H1 = Ao + a.m.beta * Ad + Ks + Kp;
  const double dH = H1 - a.H0[ch];
  const double u = u01_d(draw(key, 0u, k, TAG_HACC).x);
  const bool ok = a.outside[ch] == 0u && __builtin_isfinite(dH) && ::log(u) < -dH;
  a.accepted[ch] = ok ? 1 : 0;
  a.dH[ch] = dH;
#pragma unroll
  for (int l = 0; l < 7; ++l) a.p[(int64_t)ch * 7 + l] = ok ? pL[l] : a.p0[(int64_t)ch * 7 + l];
  if (a.acc) {
    a.acc[(int64_t)ch * PIMC_NACC + 0] += ok ? 1 : 0;
    if (!__builtin_isfinite(dH)) a.acc[(int64_t)ch * PIMC_NACC + PIMC_ACC_NONFINITE] += 1;
    if (a.outside[ch]) a.acc[(int64_t)ch * PIMC_NACC + 1] += 1;
  }
  if (a.ptrace) {
    const int64_t it = (int64_t)(k - a.k_first);
#pragma unroll
    for (int l = 0; l < 7; ++l) a.ptrace[((int64_t)ch * a.ntrace + it) * 7 + l] = a.p[(int64_t)ch * 7 + l];
  }
  if (a.dHtrace) a.dHtrace[(int64_t)ch * a.ntrace + (int64_t)(k - a.k_first)] = dH;
}

// Final positions: the end of the trajectory if accepted, else the start.
template <typename T>
__global__ void hmc_restore_kernel(HmcArgs a, int L) {
  const int b = blockIdx.x;
  const int ch = a.bmap[b];
  const int64_t base = a.offsets[ch];
  const int M = (int)(a.offsets[ch + 1] - base - 1);
  const int n = (b - a.bfirst[ch]) * HB + threadIdx.x;
  // the next proposal's index (no kernel of this proposal reads it any more)
  if (b == 0 && threadIdx.x == 0) *a.kptr += 1;
  if (n > M) return;
  const bool ok = a.accepted[ch] != 0;
  const T* src = (const T*)(ok ? ((L & 1) ? a.Q1 : a.X) : a.X0) + (base + n) * 4;
  T* X = (T*)a.X + (base + n) * 4;
  if (src != X) {
#pragma unroll
    for (int c = 0; c < 4; ++c) X[c] = src[c];
  }
}

int launch_hmc_proposal(const HmcArgs& a, bool fp64, int L, hipStream_t s) {
  const dim3 gb(a.nblocks), tb(HB);
  if (fp64) {
    hipLaunchKernelGGL((hmc_step_kernel<double, 0>), gb, tb, 0, s, a, 0);
    for (int st = 1; st < L; ++st) hipLaunchKernelGGL((hmc_step_kernel<double, 1>), gb, tb, 0, s, a, st);
    hipLaunchKernelGGL((hmc_step_kernel<double, 2>), gb, tb, 0, s, a, L);
  } else {
    hipLaunchKernelGGL((hmc_step_kernel<float, 0>), gb, tb, 0, s, a, 0);
    for (int st = 1; st < L; ++st) hipLaunchKernelGGL((hmc_step_kernel<float, 1>), gb, tb, 0, s, a, st);
    hipLaunchKernelGGL((hmc_step_kernel<float, 2>), gb, tb, 0, s, a, L);
  }
  hipLaunchKernelGGL(hmc_finish_kernel, dim3(a.B), dim3(HB), 0, s, a, L);
  if (fp64)
    hipLaunchKernelGGL(hmc_restore_kernel<double>, gb, tb, 0, s, a, L);
  else
    hipLaunchKernelGGL(hmc_restore_kernel<float>, gb, tb, 0, s, a, L);
  return hipGetLastError() == hipSuccess ? PIMC_OK : PIMC_ERR_HIP;
}

}  // namespace pimc
