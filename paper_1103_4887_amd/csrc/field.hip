// Full action A(X, p) and its gradient for one window (Section 2.1).
//
//   A   = 1/2 sum_{n>=1} Ro (y_n - V_n)^2 + beta/2 sum_{n>=1} eps_n^T Rd eps_n
//   dA/dx_n = beta (1 - h J_n)^T Rd eps_n [n>=1] + beta (-1 - h J_n)^T Rd eps_{n+1} [n<=M-1]
//             - Ro (y_n - V_n) e_V [n>=1]
//   dA/dp   = -beta h sum_{n>=1} eps_n^T Rd [dF/dp(x_n) + dF/dp(x_{n-1})]
//
// with h = dt/2 and J = dF/dx.  A is a sum of site- and link-local terms, so
// both are one pass of independent threads plus a deterministic two-level
// FP64 reduction (fixed 256-site chunks, fixed tree order, then a single
// block summing the chunk partials in index order).
#include <mutex>

#include "device.hpp"
#include "kernels.hpp"

namespace pimc {

// Fixed device workspace of pimc_action_noalloc: the FP64 block partials of
// the action reduction for up to NOALLOC_BLOCKS blocks (256 KiB per GPU,
// held until the process ends).  Every block writes its whole partial
// record before the final kernel reads it, so nothing needs clearing.
constexpr int64_t NOALLOC_BLOCKS = PIMC_NOALLOC_MAX_SITES / FIELD_BLOCK;
static __device__ __align__(256) double scratch[NOALLOC_BLOCKS * 8];

// Device address of `scratch` on the current device, looked up once per
// device (the host-side name is only a stand-in for the symbol).
int noalloc_scratch(double** out) {
  constexpr int MAXDEV = 64;
  static std::mutex mu;
  static double* ptrs[MAXDEV] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAXDEV) return PIMC_ERR_HIP;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptrs[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PIMC_ERR_HIP;
    ptrs[dev] = (double*)p;
  }
  *out = ptrs[dev];
  return PIMC_OK;
}

namespace {

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds, int t, double* out) {
  // blockDim == FIELD_BLOCK (4 waves)
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = v[i];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    v[i] = s;
  }
  if ((t & 63) == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) lds[(t >> 6) * NV + i] = v[i];
  }
  __syncthreads();
  if (t < NV) out[t] = ((lds[t] + lds[NV + t]) + (lds[2 * NV + t] + lds[3 * NV + t]));
}

template <typename T>
__device__ __forceinline__ void load_site(const T* X, int64_t n, T (&x)[4]) {
#pragma unroll
  for (int c = 0; c < 4; ++c) x[c] = X[n * 4 + c];
}

// Jacobian rows of the HH field at x (row V full; gate rows only dV and self).
template <typename T>
struct Jac {
  T VV, Vg[3];  // dF_V/dV, dF_V/d(m,h,n)
  T gV[3], gg[3];
};

template <typename T>
__device__ __forceinline__ void hh_J(const Consts<T>& C, const T (&x)[4], Jac<T>& J) {
  const T V = x[0], m = x[1], hh = x[2], n = x[3];
  const T m2 = m * m, m3 = m2 * m, n2 = n * n, n3 = n2 * n, n4 = n2 * n2;
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
    const T dt_dV = sech2 * C.inv_dVa[g];
    const T dainf = (T)0.5 * dt_dV;
    const T dtau = (T)-2 * C.tau1[g] * t * dt_dV;
    J.gV[g] = dainf * itau - (ainf - x[1 + g]) * dtau * itau * itau;
    J.gg[g] = -itau;
  }
}

}  // namespace

// One thread per link n = 1..M (thread index n-1 ... ), terms in FP64.
template <typename T>
__global__ void __launch_bounds__(FIELD_BLOCK) action_partial_kernel(FieldArgs a) {
  __shared__ double lds[4 * 2];
  const int t = threadIdx.x;
  const int64_t n = (int64_t)blockIdx.x * FIELD_BLOCK + t;  // site index
  Consts<double> C;
  C.init(a.m);
  C.set_p(a.p);
  if (a.kin) C.set_gates(a.kin);
  double v[2] = {0.0, 0.0};
  if (n >= 1 && n <= a.M) {
    const T* X = (const T*)a.X;
    const T* Y = (const T*)a.y;
    const T* I = (const T*)a.I;
    double x1[4], x0[4], F1[4], F0[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      x1[c] = (double)X[n * 4 + c];
      x0[c] = (double)X[(n - 1) * 4 + c];
    }
    hh_F(C, x1, (double)I[n], F1);
    hh_F(C, x0, (double)I[n - 1], F0);
    const double d = (double)Y[n] - x1[0];
    v[0] = 0.5 * a.m.Ro * d * d;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double e = (x1[c] - x0[c]) - C.h * (F1[c] + F0[c]);
      s += a.m.Rd[c] * e * e;
    }
    v[1] = 0.5 * s;
  }
  block_sum<2>(v, lds, t, a.partial + (int64_t)blockIdx.x * 8);
}

__global__ void __launch_bounds__(FIELD_BLOCK) action_final_kernel(const double* partial, int64_t nb, double beta,
                                                                   double* out) {
  __shared__ double lds[4 * 2];
  const int t = threadIdx.x;
  double v[2] = {0.0, 0.0};
  for (int64_t b = t; b < nb; b += FIELD_BLOCK) {
    v[0] += partial[b * 8 + 0];
    v[1] += partial[b * 8 + 1];
  }
  __shared__ double res[2];
  block_sum<2>(v, lds, t, res);
  __syncthreads();
  if (t == 0) {
    out[0] = res[0] + beta * res[1];
    out[1] = res[0];
    out[2] = res[1];
  }
}

// One thread per site n = 0..M: gX[n] and the link-n share of dA/dp.
template <typename T>
__global__ void __launch_bounds__(FIELD_BLOCK) grad_partial_kernel(FieldArgs a) {
  __shared__ double lds[4 * 7];
  const int t = threadIdx.x;
  const int64_t n = (int64_t)blockIdx.x * FIELD_BLOCK + t;
  const int64_t M = a.M;
  Consts<T> C;
  C.init(a.m);
  C.set_p(a.p);
  if (a.kin) C.set_gates(a.kin);
  double gp[7] = {0, 0, 0, 0, 0, 0, 0};
  if (n <= M) {
    const T* X = (const T*)a.X;
    const T* Y = (const T*)a.y;
    const T* I = (const T*)a.I;
    const T h = C.h;
    const T beta = (T)a.m.beta;
    T x[4], F[4];
    load_site(X, n, x);
    hh_F(C, x, I[n], F);
    T vl[4] = {0, 0, 0, 0}, vr[4] = {0, 0, 0, 0};
    T xl[4];
    if (n >= 1) {
      T Fl[4];
      load_site(X, n - 1, xl);
      hh_F(C, xl, I[n - 1], Fl);
#pragma unroll
      for (int c = 0; c < 4; ++c) vl[c] = beta * (T)a.m.Rd[c] * ((x[c] - xl[c]) - h * (F[c] + Fl[c]));
    }
    if (n + 1 <= M) {
      T xr[4], Fr[4];
      load_site(X, n + 1, xr);
      hh_F(C, xr, I[n + 1], Fr);
#pragma unroll
      for (int c = 0; c < 4; ++c) vr[c] = beta * (T)a.m.Rd[c] * ((xr[c] - x[c]) - h * (Fr[c] + F[c]));
    }
    Jac<T> J;
    hh_J(C, x, J);
    T u[4], w[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      u[c] = vl[c] - vr[c];
      w[c] = vl[c] + vr[c];
    }
    T g[4];
    g[0] = u[0] - h * (J.VV * w[0] + J.gV[0] * w[1] + J.gV[1] * w[2] + J.gV[2] * w[3]);
#pragma unroll
    for (int q = 0; q < 3; ++q) g[1 + q] = u[1 + q] - h * (J.Vg[q] * w[0] + J.gg[q] * w[1 + q]);
    if (n >= 1) g[0] -= (T)a.m.Ro * (Y[n] - x[0]);
    if (a.gX) {
      T* G = (T*)a.gX;
#pragma unroll
      for (int c = 0; c < 4; ++c) G[n * 4 + c] = g[c];
    }
    if (n >= 1) {
      // link n: -h v_V [dF_V/dp(x_n) + dF_V/dp(x_{n-1})], in FP64
      const double pd1 = a.p[1], pd2 = a.p[2], pd3 = a.p[3], pd4 = a.p[4], pd5 = a.p[5], pd6 = a.p[6];
      double s[7] = {0, 0, 0, 0, 0, 0, 0};
      for (int side = 0; side < 2; ++side) {
        const double V = side ? (double)xl[0] : (double)x[0];
        const double m = side ? (double)xl[1] : (double)x[1];
        const double hh = side ? (double)xl[2] : (double)x[2];
        const double nn = side ? (double)xl[3] : (double)x[3];
        const double Iv = side ? (double)I[n - 1] : (double)I[n];
        const double m3h = m * m * m * hh;
        const double n4 = nn * nn * nn * nn;
        s[0] += Iv;
        s[1] += m3h * (pd2 - V);
        s[2] += pd1 * m3h;
        s[3] += n4 * (pd4 - V);
        s[4] += pd3 * n4;
        s[5] += pd6 - V;
        s[6] += pd5;
      }
      const double f = -0.5 * a.m.dt * (double)vl[0];
#pragma unroll
      for (int l = 0; l < 7; ++l) gp[l] = f * s[l];
    }
  }
  block_sum<7>(gp, lds, t, a.partial + (int64_t)blockIdx.x * 8);
}

__global__ void __launch_bounds__(FIELD_BLOCK) grad_final_kernel(const double* partial, int64_t nb, double* gp) {
  __shared__ double lds[4 * 7];
  const int t = threadIdx.x;
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int64_t b = t; b < nb; b += FIELD_BLOCK) {
#pragma unroll
    for (int l = 0; l < 7; ++l) v[l] += partial[b * 8 + l];
  }
  block_sum<7>(v, lds, t, gp);
}

int launch_action(const FieldArgs& a, bool fp64, hipStream_t s) {
  const int64_t nb = field_blocks(a.M);
  if (fp64)
    hipLaunchKernelGGL(action_partial_kernel<double>, dim3(nb), dim3(FIELD_BLOCK), 0, s, a);
  else
    hipLaunchKernelGGL(action_partial_kernel<float>, dim3(nb), dim3(FIELD_BLOCK), 0, s, a);
  hipLaunchKernelGGL(action_final_kernel, dim3(1), dim3(FIELD_BLOCK), 0, s, a.partial, nb, a.m.beta, a.out);
  return hipGetLastError() == hipSuccess ? PIMC_OK : PIMC_ERR_HIP;
}

int launch_grad(const FieldArgs& a, bool fp64, hipStream_t s) {
  const int64_t nb = field_blocks(a.M);
  if (fp64)
    hipLaunchKernelGGL(grad_partial_kernel<double>, dim3(nb), dim3(FIELD_BLOCK), 0, s, a);
  else
    hipLaunchKernelGGL(grad_partial_kernel<float>, dim3(nb), dim3(FIELD_BLOCK), 0, s, a);
  hipLaunchKernelGGL(grad_final_kernel, dim3(1), dim3(FIELD_BLOCK), 0, s, a.partial, nb, a.out);
  return hipGetLastError() == hipSuccess ? PIMC_OK : PIMC_ERR_HIP;
}

}  // namespace pimc
