// Model checks of Section 6: the model and observation errors of a path,
// accumulated over posterior samples, and forecasts of the model from the
// end of the window.
//
//  * errors: one thread per link n = 1..M adds eps_n (the trapezoid model
//    error of Section 2.1, all D components) and delta_n = y_n - V_n to
//    running sums and sums of squares (FP64).  Their means should vanish and
//    their variances equal 1/Rd and 1/Ro when the model is right; the
//    discretisation shows as <eps_n> away from zero at spikes.
//  * forecast: one thread per ensemble member integrates the model with
//    Heun's method (the explicit form of the trapezoid rule) from its own
//    final state and parameters over a given drive, adding model noise
//    eps ~ N(0, 1/Rd) times `noise` per step (Philox FCST block of
//    (member, step)); FP64.
#include "device.hpp"
#include "kernels.hpp"

namespace pimc {

namespace {

constexpr uint32_t TAG_FCST = 8;

template <typename T>
__global__ void __launch_bounds__(256) errors_kernel(ErrArgs a) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x + 1;   // link n - 1 -> n
  if (n > a.M) return;
  Consts<double> C;
  C.init(a.m);
  C.set_p(a.p);
  if (a.kin) C.set_gates(a.kin);
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
  double* s = a.esum + (n - 1) * 5;
  double* q = a.esq + (n - 1) * 5;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double e = (x1[c] - x0[c]) - C.h * (F1[c] + F0[c]);
    s[c] += e;
    q[c] += e * e;
  }
  const double d = (double)Y[n] - x1[0];
  s[4] += d;
  q[4] += d * d;
}

__global__ void __launch_bounds__(64) forecast_kernel(FcstArgs a) {
  const int b = blockIdx.x * 64 + threadIdx.x;
  if (b >= a.B) return;
  Consts<double> C;
  C.init(a.m);
  C.set_p(a.p + (int64_t)b * 7);
  if (a.kin) C.set_gates(a.kin);
  const Key key = make_key(a.seed, 0u);
  double sd[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) sd[c] = a.noise / sqrt(a.m.Rd[c]);
  double x[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) x[c] = a.x0[(int64_t)b * 4 + c];
  double* out = a.out + (int64_t)b * (a.N + 1) * 4;
#pragma unroll
  for (int c = 0; c < 4; ++c) out[c] = x[c];
  const double dt = a.m.dt;
  for (int64_t k = 0; k < a.N; ++k) {
    double k1[4], xt[4], k2[4];
    hh_F(C, x, a.I[k], k1);
#pragma unroll
    for (int c = 0; c < 4; ++c) xt[c] = x[c] + dt * k1[c];
    hh_F(C, xt, a.I[k + 1], k2);
#pragma unroll
    for (int c = 0; c < 4; ++c) x[c] = x[c] + 0.5 * dt * (k1[c] + k2[c]);
    if (a.noise != 0.0) {
      const U4 blk = draw(key, (uint32_t)(a.member0 + b), (uint64_t)k, TAG_FCST);
      double z[4];
      Math<double>::box_muller(blk.x, blk.y, z[0], z[1]);
      Math<double>::box_muller(blk.z, blk.w, z[2], z[3]);
#pragma unroll
      for (int c = 0; c < 4; ++c) x[c] += sd[c] * z[c];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) out[(k + 1) * 4 + c] = x[c];
  }
}

}  // namespace

int launch_errors(const ErrArgs& a, bool fp64, hipStream_t s) {
  const dim3 g((unsigned)((a.M + 255) / 256)), b(256);
  if (fp64)
    hipLaunchKernelGGL(errors_kernel<double>, g, b, 0, s, a);
  else
    hipLaunchKernelGGL(errors_kernel<float>, g, b, 0, s, a);
  return hipGetLastError() == hipSuccess ? PIMC_OK : PIMC_ERR_HIP;
}

int launch_forecast(const FcstArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(forecast_kernel, dim3((unsigned)((a.B + 63) / 64)), dim3(64), 0, s, a);
  return hipGetLastError() == hipSuccess ? PIMC_OK : PIMC_ERR_HIP;
}

}  // namespace pimc
