// Device-side building blocks of libpimc (gfx950): Philox4x32-10, uniform and
// normal mappings, the Hodgkin-Huxley vector field and its per-site features.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pimc.h"

namespace pimc {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The key schedule only
// depends on (seed, chain), which are uniform over a workgroup, so the Weyl
// additions land on the scalar unit; each round costs two 32x32->64 products.
// ---------------------------------------------------------------------------
enum : uint32_t { TAG_SITE = 1, TAG_SACC = 2, TAG_PARAM = 3, TAG_MOM = 4, TAG_PMOM = 5, TAG_HACC = 6, TAG_KIN = 7 };

struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

struct Key {
  uint32_t k0, k1;
};

__device__ __forceinline__ Key make_key(uint64_t seed, uint32_t chain) {
  return Key{(uint32_t)seed, (uint32_t)(seed >> 32) ^ chain};
}

// counter = (idx, sweep_lo, tag << 24 | sweep_hi24, blk)
__device__ __forceinline__ U4 draw(Key k, uint32_t idx, uint64_t sweep, uint32_t tag, uint32_t blk = 0) {
  U4 c{idx, (uint32_t)sweep, (tag << 24) | ((uint32_t)(sweep >> 32) & 0xFFFFFFu), blk};
  return philox10(c, k.k0, k.k1);
}

// u = (c + 0.5) 2^-32 in (0, 1); exact in FP64.
__device__ __forceinline__ double u01_d(uint32_t c) { return ((double)c + 0.5) * 0x1p-32; }
__device__ __forceinline__ float u01_f(uint32_t c) { return ((float)c + 0.5f) * 0x1p-32f; }

// ---------------------------------------------------------------------------
// Precision-dependent math.  FP32: hardware exp2/log2/rcp/sin/cos (quarter
// rate transcendental unit), errors far below the FP32 parity budget.  FP64:
// correctly rounded library calls.
// ---------------------------------------------------------------------------
template <typename T>
struct Math;

template <>
struct Math<float> {
  static __device__ __forceinline__ float tanh(float s) {
    // 1 - 2 / (1 + e^{2s}); saturates cleanly at +-1, absolute error ~1e-7
    const float e = __builtin_amdgcn_exp2f(s * 2.8853900817779268f);  // 2 log2(e)
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + e);
  }
  static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  // two standard normals from a word pair (Box-Muller); sin/cos take turns
  static __device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float& z0, float& z1) {
    const float ua = u01_f(a);
    const float ub = (float)b * 0x1p-32f;
    const float r = __builtin_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(ua));  // -2 ln 2 log2
    z0 = r * __builtin_amdgcn_cosf(ub);
    z1 = r * __builtin_amdgcn_sinf(ub);
  }
  static __device__ __forceinline__ float uniform_pm1(uint32_t c) { return 2.0f * u01_f(c) - 1.0f; }
};

template <>
struct Math<double> {
  static __device__ __forceinline__ double tanh(double s) { return ::tanh(s); }
  static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
  static __device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double& z0, double& z1) {
    const double ua = u01_d(a);
    const double ub = (double)b * 0x1p-32;
    const double r = ::sqrt(-2.0 * ::log(ua));
    double s, c;
    ::sincospi(2.0 * ub, &s, &c);
    z0 = r * c;
    z1 = r * s;
  }
  static __device__ __forceinline__ double uniform_pm1(uint32_t c) { return 2.0 * u01_d(c) - 1.0; }
};

// ---------------------------------------------------------------------------
// Model constants as passed to kernels (FP64, converted per kernel).
// ---------------------------------------------------------------------------
struct ModelArgs {
  double dt, Ro, Rd[4], beta;
  double Va[3], dVa[3], tau0[3], tau1[3];
  double x_lo[4], x_hi[4], p_lo[7], p_hi[7];
  uint32_t p_mask;
  int32_t proposal;
  double k_lo[12], k_hi[12];
  uint32_t k_mask;
};

template <typename T>
struct Consts {
  T h;            // dt / 2
  T half_beta_Rd[4];
  T half_Ro;
  T Va[3], inv_dVa[3], tau0[3], tau1[3];
  T lo[4], hi[4];
  // current parameters (site precision)
  T p[7];

  __host__ __device__ void init(const ModelArgs& m) {
    h = (T)(0.5 * m.dt);
    for (int a = 0; a < 4; ++a) {
      half_beta_Rd[a] = (T)(0.5 * m.beta * m.Rd[a]);
      lo[a] = (T)m.x_lo[a];
      hi[a] = (T)m.x_hi[a];
    }
    half_Ro = (T)(0.5 * m.Ro);
    for (int g = 0; g < 3; ++g) {
      Va[g] = (T)m.Va[g];
      inv_dVa[g] = (T)(1.0 / m.dVa[g]);
      tau0[g] = (T)m.tau0[g];
      tau1[g] = (T)m.tau1[g];
    }
  }
  __device__ __forceinline__ void set_p(const double* pd) {
    for (int l = 0; l < 7; ++l) p[l] = (T)pd[l];
  }
  // Table 1 constants from kin [12], order (m, h, n) x (V_a, dV_a, tau0, tau1)
  __host__ __device__ void set_gates(const double* kin) {
    for (int g = 0; g < 3; ++g) {
      Va[g] = (T)kin[4 * g];
      inv_dVa[g] = (T)(1.0 / kin[4 * g + 1]);
      tau0[g] = (T)kin[4 * g + 2];
      tau1[g] = (T)kin[4 * g + 3];
    }
  }
};

// Move a double across lanes with one DPP control (two 32-bit moves).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  // every lane reads a lane of its own row, so no lane keeps an old value
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over each row of 16 lanes with DPP (quad_perm xor 1, xor 2, then
// row_ror 4 and 8); the row total lands in lanes 12..15 of the row.
__device__ __forceinline__ double row_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x124>(v);  // row_ror:4
  v += dpp_d<0x128>(v);  // row_ror:8
  return v;
}

// One folding step of a wave sum of two values x, y: with the lane swap
// across the two 32-lane halves (HALF) or across neighbouring 16-lane rows,
// returns x summed over each lane and its partner where the lane keeps x
// (lower half, or even rows), y likewise where it keeps y.
template <bool HALF>
__device__ __forceinline__ double fold_pair(double x, double y) {
  const uint64_t bx = __builtin_bit_cast(uint64_t, x), by = __builtin_bit_cast(uint64_t, y);
  const uint32_t xl = (uint32_t)bx, xh = (uint32_t)(bx >> 32), yl = (uint32_t)by, yh = (uint32_t)(by >> 32);
  uint32_t al, ah, bl, bh;
  if constexpr (HALF) {
    const auto lo = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
    al = lo[0], bl = lo[1], ah = hi[0], bh = hi[1];
  } else {
    const auto lo = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
    al = lo[0], bl = lo[1], ah = hi[0], bh = hi[1];
  }
  return __builtin_bit_cast(double, ((uint64_t)ah << 32) | al) + __builtin_bit_cast(double, ((uint64_t)bh << 32) | bl);
}

// Wave totals of N <= 36 values: the halves of the wave, then its rows,
// are folded pairwise (N -> N/2 -> N/4 registers), and each of the
// remaining registers is summed over its row of 16 lanes.  On return every
// lane of row r (lanes 16 r .. 16 r + 15) holds in w[j] the total of value
// 4 j + fold_slot(r) (values past N are zero).
__host__ __device__ constexpr int fold_slot(int row) { return row == 1 ? 2 : (row == 2 ? 1 : row); }
template <int N>
__device__ __forceinline__ void wave_fold(const double (&v)[N], double (&w)[(N + 3) / 4]) {
  constexpr int NH = (N + 1) / 2, NQ = (N + 3) / 4;
  double h[2 * NQ];
#pragma unroll
  for (int i = 0; i < NH; ++i) h[i] = fold_pair<true>(v[2 * i], 2 * i + 1 < N ? v[2 * i + 1] : 0.0);
#pragma unroll
  for (int i = NH; i < 2 * NQ; ++i) h[i] = 0.0;
#pragma unroll
  for (int j = 0; j < NQ; ++j) w[j] = row_sum(fold_pair<false>(h[2 * j], h[2 * j + 1]));
}

// Values that every lane of a wave holds identically (the parameters after
// a move) are moved to scalar registers, which frees vector registers.
__device__ __forceinline__ double wave_uniform(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// dV/dt of Section 5.1: p1 I + p2 m^3 h (p3 - V) + p4 n^4 (p5 - V) + p6 (p7 - V)
template <typename T>
__device__ __forceinline__ T hh_FV(const Consts<T>& C, T V, T m, T h, T n, T I) {
  const T m3h = m * m * m * h;
  const T n2 = n * n;
  const T n4 = n2 * n2;
  return C.p[0] * I + C.p[1] * m3h * (C.p[2] - V) + C.p[3] * n4 * (C.p[4] - V) + C.p[5] * (C.p[6] - V);
}

// da/dt = (a_inf(V) - a) / tau_a(V) for gate g (0 = m, 1 = h, 2 = n)
template <typename T>
__device__ __forceinline__ T hh_Fgate(const Consts<T>& C, int g, T V, T a) {
  const T t = Math<T>::tanh((V - C.Va[g]) * C.inv_dVa[g]);
  const T ainf = (T)0.5 + (T)0.5 * t;
  const T tau = C.tau0[g] + C.tau1[g] * ((T)1 - t * t);
  return (ainf - a) * Math<T>::rcp(tau);
}

template <typename T>
__device__ __forceinline__ void hh_F(const Consts<T>& C, const T (&x)[4], T I, T (&F)[4]) {
  F[0] = hh_FV(C, x[0], x[1], x[2], x[3], I);
  F[1] = hh_Fgate(C, 0, x[0], x[1]);
  F[2] = hh_Fgate(C, 1, x[0], x[2]);
  F[3] = hh_Fgate(C, 2, x[0], x[3]);
}

// tanh of a small argument with full relative accuracy in FP32 (odd series
// to s^7 for |s| < 1/8, error < 1e-9 relative; the general form beyond).
__device__ __forceinline__ float tanh_small(float s) {
  const float s2 = s * s;
  if (__builtin_fabsf(s) < 0.125f)
    return s + s * s2 * (-0.333333333f + s2 * (0.133333333f + s2 * -0.0539682540f));
  return Math<float>::tanh(s);
}

// F(x') and F(x') - F(x) in FP32 without cancellation: the difference is
// built from the differences of the inputs,
//   tanh(s') - tanh(s) = tanh(s' - s) (1 - tanh(s) tanh(s')),
//   1/tau' - 1/tau = tau1 (t' - t)(t' + t) / (tau tau'),
//   m'^3 h' - m^3 h = (m' - m)(m'^2 + m' m + m^2) h' + m^3 (h' - h),
//   n'^4 - n^4 = (n' - n)(n' + n)(n'^2 + n^2),
// so dF carries a relative (not an absolute) FP32 error.
__device__ __forceinline__ void hh_F_dF(const Consts<float>& C, const float (&x)[4], const float (&xp)[4], float I,
                                        float (&Fp)[4], float (&dF)[4]) {
  const float V = x[0], m = x[1], h = x[2], n = x[3];
  const float Vp = xp[0], mp = xp[1], hp = xp[2], np_ = xp[3];
  const float dV = Vp - V, dm = mp - m, dh = hp - h, dn = np_ - n;
  Fp[0] = hh_FV(C, Vp, mp, hp, np_, I);
  const float m3 = m * m * m;
  const float A = m3 * h;
  const float n2 = n * n;
  const float N4 = n2 * n2;
  const float dA = dm * (mp * mp + mp * m + m * m) * hp + m3 * dh;
  const float dN4 = dn * (np_ + n) * (np_ * np_ + n2);
  dF[0] = C.p[1] * (dA * (C.p[2] - Vp) - A * dV) + C.p[3] * (dN4 * (C.p[4] - Vp) - N4 * dV) - C.p[5] * dV;
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    const float t = Math<float>::tanh((V - C.Va[g]) * C.inv_dVa[g]);
    const float tp = Math<float>::tanh((Vp - C.Va[g]) * C.inv_dVa[g]);
    const float r = Math<float>::rcp(C.tau0[g] + C.tau1[g] * (1.0f - t * t));
    const float rp = Math<float>::rcp(C.tau0[g] + C.tau1[g] * (1.0f - tp * tp));
    const float a = x[1 + g], ap = xp[1 + g];
    Fp[1 + g] = (0.5f + 0.5f * tp - ap) * rp;
    const float dt_ = tanh_small(dV * C.inv_dVa[g]) * (1.0f - t * tp);
    dF[1 + g] = (0.5f * dt_ - (ap - a)) * rp + (0.5f + 0.5f * t - a) * C.tau1[g] * dt_ * (tp + t) * r * rp;
  }
}

// p-linear features of dV/dt: F_V = theta . psi with
// theta = (p1, p2, p2 p3, p4, p4 p5, p6, p6 p7), psi = (I, -m^3hV, m^3h, -n^4V, n^4, -V, 1)
__device__ __forceinline__ void hh_psi(double V, double m, double h, double n, double I, double (&psi)[7]) {
  const double m3h = m * m * m * h;
  const double n2 = n * n;
  const double n4 = n2 * n2;
  psi[0] = I;
  psi[1] = -m3h * V;
  psi[2] = m3h;
  psi[3] = -n4 * V;
  psi[4] = n4;
  psi[5] = -V;
  psi[6] = 1.0;
}

__device__ __forceinline__ void theta_of(const double* p, double (&th)[7]) {
  th[0] = p[0];
  th[1] = p[1];
  th[2] = p[1] * p[2];
  th[3] = p[3];
  th[4] = p[3] * p[4];
  th[5] = p[5];
  th[6] = p[5] * p[6];
}

// Upper-triangle index of (a, b), a <= b, in a packed 7x7 symmetric matrix.
__host__ __device__ constexpr int sym7(int a, int b) { return a * 7 - a * (a - 1) / 2 + (b - a); }

}  // namespace pimc
