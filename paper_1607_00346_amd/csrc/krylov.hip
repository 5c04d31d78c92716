// Accuracy diagnostics of a factor (paper, Section 4, result metrics): the
// relative solve error e_s and a power-method estimate of ||I - F^{-1}A||_2.
#include <cmath>

#include "hif_impl.hpp"

namespace hif {
namespace {

constexpr int NT = 256;

unsigned grid_of(int64_t N) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(N, NT), 8192));
}

// y = x - y
__global__ __launch_bounds__(NT) void k_sub_from(const double* __restrict__ x, double* y,
                                                 int64_t N) {
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < N; i += (int64_t)gridDim.x * NT)
    y[i] = x[i] - y[i];
}

// y = x / sqrt(*nrm2)
__global__ __launch_bounds__(NT) void k_normalize(const double* __restrict__ x, double* y,
                                                  const double* __restrict__ nrm2, int64_t N) {
  const double inv = 1.0 / sqrt(*nrm2);
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < N; i += (int64_t)gridDim.x * NT)
    y[i] = x[i] * inv;
}

double fetch(const double* d, hipStream_t s) {
  double h = 0.0;
  HIF_HIP(hipMemcpyAsync(&h, d, sizeof(double), hipMemcpyDeviceToHost, s));
  HIF_HIP(hipStreamSynchronize(s));
  return h;
}

}  // namespace

void factor_error(const hif_problem_s* A, hif_factor_s* F, const double* x, int power_iters,
                  double* e_s, double* err_norm, hipStream_t s) {
  const int64_t N = A->N;
  const Stencil st = A->stencil();
  FactorBase& Fi = *F->impl;
  DevBuf<double> t(N), w(N), v(N), sc(4);
  const unsigned g = grid_of(N);
  // e_s: w = x - F^{-1} A x
  stencil_matvec(st, x, t.get(), s);
  Fi.apply(t.get(), w.get(), s);
  hipLaunchKernelGGL(k_sub_from, dim3(g), dim3(NT), 0, s, x, w.get(), N);
  HIF_LAUNCH_CHECK();
  device_dot(w.get(), w.get(), nullptr, N, sc.get() + 0, s);
  device_dot(x, x, nullptr, N, sc.get() + 1, s);
  const double xx = fetch(sc.get() + 1, s);
  HIF_REQUIRE(xx > 0.0 && std::isfinite(xx), HIF_EINVAL, "x must be nonzero and finite");
  *e_s = std::sqrt(fetch(sc.get(), s) / xx);
  *err_norm = std::nan("");
  if (power_iters <= 0) return;
  // power method on B^T B with B = I - F^{-1} A and B^T = I - A F^{-1}
  hipLaunchKernelGGL(k_normalize, dim3(g), dim3(NT), 0, s, x, v.get(),
                     (const double*)(sc.get() + 1), N);
  HIF_LAUNCH_CHECK();
  double est = 0.0;
  for (int it = 0; it < power_iters; ++it) {
    // w = B v
    stencil_matvec(st, v.get(), t.get(), s);
    Fi.apply(t.get(), w.get(), s);
    hipLaunchKernelGGL(k_sub_from, dim3(g), dim3(NT), 0, s, (const double*)v.get(), w.get(), N);
    // v = B^T w = w - A F^{-1} w
    Fi.apply(w.get(), t.get(), s);
    stencil_matvec(st, t.get(), v.get(), s);
    hipLaunchKernelGGL(k_sub_from, dim3(g), dim3(NT), 0, s, (const double*)w.get(), v.get(), N);
    HIF_LAUNCH_CHECK();
    device_dot(v.get(), v.get(), nullptr, N, sc.get() + 2, s);
    const double vv = fetch(sc.get() + 2, s);
    if (!(vv > 0.0) || !std::isfinite(vv)) {
      est = std::sqrt(std::sqrt(std::max(vv, 0.0)));
      break;
    }
    est = std::sqrt(std::sqrt(vv));  // ||B^T B v|| -> sigma_max^2 for unit v
    hipLaunchKernelGGL(k_normalize, dim3(g), dim3(NT), 0, s, (const double*)v.get(), v.get(),
                       (const double*)(sc.get() + 2), N);
    HIF_LAUNCH_CHECK();
  }
  *err_norm = est;
}

}  // namespace hif
