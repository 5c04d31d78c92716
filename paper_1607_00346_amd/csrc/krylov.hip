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

// ---- GMRES with F^{-1} as a right preconditioner (paper, Section 4) ------
//
// Restarted flexible GMRES: z_j = F^{-1} v_j is kept beside the Arnoldi
// basis v_j, so that the update u += Z y needs no further application (and
// the FP32 factor's application, linear only up to rounding, is handled as a
// varying preconditioner).  Arnoldi orthogonalization is classical
// Gram-Schmidt run twice (each pass one batched inner-product launch and one
// update launch over all basis vectors), with fixed-order reductions.  The
// small Hessenberg least-squares problem is updated by Givens rotations on
// the host, which reads back one column of H per step.

namespace hif {
namespace {

constexpr int kMdotBlocks = 512;

// part[c * gridDim.x + b] = sum over a strided slice of V_c . w
__global__ __launch_bounds__(NT) void k_mdot_partial(const double* __restrict__ V, int64_t ldv,
                                                     const double* __restrict__ w, int64_t N,
                                                     double* part) {
  __shared__ double red[NT / 64];
  const int c = blockIdx.y;
  const double* v = V + ldv * c;
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < N; i += (int64_t)gridDim.x * NT)
    s += v[i] * w[i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < NT / 64; ++k) t += red[k];
    part[(int64_t)c * gridDim.x + blockIdx.x] = t;
  }
}

// out[c] = sum_b part[c * nb + b] (and acc[c] += out[c] if acc is not null),
// one workgroup per column
__global__ __launch_bounds__(NT) void k_mdot_final(const double* __restrict__ part, int nb,
                                                   double* out, double* acc) {
  __shared__ double red[NT / 64];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += NT) s += part[(int64_t)c * nb + i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < NT / 64; ++k) t += red[k];
    out[c] = t;
    if (acc) acc[c] += t;
  }
}

// w -= sum_c coef[c] V_c
__global__ __launch_bounds__(NT) void k_sub_combination(const double* __restrict__ V, int64_t ldv,
                                                        int ncol, const double* __restrict__ coef,
                                                        double* w, int64_t N) {
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < N; i += (int64_t)gridDim.x * NT) {
    double s = 0.0;
    for (int c = 0; c < ncol; ++c) s += coef[c] * V[ldv * c + i];
    w[i] -= s;
  }
}

// u += sum_c coef[c] Z_c
__global__ __launch_bounds__(NT) void k_add_combination(const double* __restrict__ Z, int64_t ldz,
                                                        int ncol, const double* __restrict__ coef,
                                                        double* u, int64_t N) {
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < N; i += (int64_t)gridDim.x * NT) {
    double s = 0.0;
    for (int c = 0; c < ncol; ++c) s += coef[c] * Z[ldz * c + i];
    u[i] += s;
  }
}

// y = x * (1 / *den)
__global__ __launch_bounds__(NT) void k_scale_by(const double* __restrict__ x, double* y,
                                                 const double* __restrict__ den, int64_t N) {
  const double inv = 1.0 / *den;
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < N; i += (int64_t)gridDim.x * NT)
    y[i] = x[i] * inv;
}

__global__ void k_sqrt_scalar(double* x) { *x = sqrt(*x); }

}  // namespace

void gmres_solve(const hif_problem_s* A, hif_factor_s* F, const double* f, double* u, double tol,
                 int restart, int maxit, hif_pcg_info* info, hipStream_t s) {
  const int64_t N = A->N;
  const Stencil st = A->stencil();
  FactorBase& Fi = *F->impl;
  const int m = restart;
  const unsigned g = grid_of(N);
  const unsigned nb = (unsigned)std::min<int64_t>(kMdotBlocks, ceil_div(N, NT));
  DevBuf<double> V((size_t)N * (m + 1)), Z((size_t)N * m), w(N);
  DevBuf<double> part((size_t)nb * (m + 1)), hcol(m + 2), sc(2), ydev(m);
  std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), gv(m + 1), y(m);
  auto vcol = [&](int j) { return V.get() + (int64_t)N * j; };
  auto zcol = [&](int j) { return Z.get() + (int64_t)N * j; };
  auto fetch_n = [&](double* h, const double* d, int cnt) {
    HIF_HIP(hipMemcpyAsync(h, d, sizeof(double) * cnt, hipMemcpyDeviceToHost, s));
    HIF_HIP(hipStreamSynchronize(s));
  };
  // true residual r = f - A u into V_0; returns ||r||
  auto residual = [&]() {
    stencil_matvec(st, u, vcol(0), s);
    hipLaunchKernelGGL(k_sub_from, dim3(g), dim3(NT), 0, s, f, vcol(0), N);
    HIF_LAUNCH_CHECK();
    device_dot(vcol(0), vcol(0), nullptr, N, sc.get(), s);
    double h = 0.0;
    fetch_n(&h, sc.get(), 1);
    return std::sqrt(h);
  };
  HIF_HIP(hipMemsetAsync(u, 0, sizeof(double) * N, s));
  device_dot(f, f, nullptr, N, sc.get() + 1, s);
  double ff = 0.0;
  fetch_n(&ff, sc.get() + 1, 1);
  const double fn = std::sqrt(ff);
  info->iters = 0;
  info->converged = 0;
  info->relres = fn == 0.0 ? 0.0 : 1.0;
  if (fn == 0.0) {
    info->converged = 1;
    return;
  }
  HIF_REQUIRE(std::isfinite(fn), HIF_EINVAL, "f must be finite");
  int its = 0;
  while (true) {
    const double beta = residual();
    info->relres = beta / fn;
    if (beta <= tol * fn) {
      info->converged = 1;
      break;
    }
    if (its >= maxit || !std::isfinite(beta)) break;
    // v_0 = r / beta (sc[0] holds ||r||^2)
    hipLaunchKernelGGL(k_normalize, dim3(g), dim3(NT), 0, s, (const double*)vcol(0), vcol(0),
                       (const double*)sc.get(), N);
    HIF_LAUNCH_CHECK();
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    int k = 0;  // Arnoldi steps of this cycle
    for (int j = 0; j < m; ++j) {
      Fi.apply(vcol(j), zcol(j), s);
      stencil_matvec(st, zcol(j), w.get(), s);
      // classical Gram-Schmidt, twice: d = V^T w; w -= V d; h += d
      for (int pass = 0; pass < 2; ++pass) {
        double* d = pass == 0 ? hcol.get() : ydev.get();
        hipLaunchKernelGGL(k_mdot_partial, dim3(nb, (unsigned)(j + 1)), dim3(NT), 0, s,
                           (const double*)V.get(), N, (const double*)w.get(), N, part.get());
        hipLaunchKernelGGL(k_mdot_final, dim3((unsigned)(j + 1)), dim3(NT), 0, s,
                           (const double*)part.get(), (int)nb, d,
                           pass == 0 ? (double*)nullptr : hcol.get());
        hipLaunchKernelGGL(k_sub_combination, dim3(g), dim3(NT), 0, s, (const double*)V.get(), N,
                           j + 1, (const double*)d, w.get(), N);
        HIF_LAUNCH_CHECK();
      }
      device_dot(w.get(), w.get(), nullptr, N, hcol.get() + j + 1, s);
      hipLaunchKernelGGL(k_sqrt_scalar, dim3(1), dim3(1), 0, s, hcol.get() + j + 1);
      HIF_LAUNCH_CHECK();
      std::vector<double> hc(j + 2);
      fetch_n(hc.data(), hcol.get(), j + 2);
      ++its;
      k = j + 1;
      // apply the previous rotations to the new column, then make its own
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * hc[i] + sn[i] * hc[i + 1];
        hc[i + 1] = -sn[i] * hc[i] + cs[i] * hc[i + 1];
        hc[i] = t;
      }
      const double hjj = hc[j], hj1 = hc[j + 1];
      const double rr = std::hypot(hjj, hj1);
      cs[j] = rr == 0.0 ? 1.0 : hjj / rr;
      sn[j] = rr == 0.0 ? 0.0 : hj1 / rr;
      hc[j] = rr;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      for (int i = 0; i <= j; ++i) H[(size_t)i + (size_t)(m + 1) * j] = hc[i];
      const bool done = std::fabs(gv[j + 1]) <= tol * fn || !(hj1 > 0.0) || its >= maxit ||
                        !std::isfinite(hj1);
      if (done || j + 1 == m) break;
      // v_{j+1} = w / h_{j+1,j}
      hipLaunchKernelGGL(k_scale_by, dim3(g), dim3(NT), 0, s, (const double*)w.get(),
                         vcol(j + 1), (const double*)(hcol.get() + j + 1), N);
      HIF_LAUNCH_CHECK();
    }
    // y = R^{-1} g (upper triangular, k x k), u += Z y
    for (int i = k - 1; i >= 0; --i) {
      double t = gv[i];
      for (int c = i + 1; c < k; ++c) t -= H[(size_t)i + (size_t)(m + 1) * c] * y[c];
      const double d = H[(size_t)i + (size_t)(m + 1) * i];
      y[i] = d != 0.0 ? t / d : 0.0;
    }
    upload_bytes(ydev.get(), y.data(), sizeof(double) * k, s);
    hipLaunchKernelGGL(k_add_combination, dim3(g), dim3(NT), 0, s, (const double*)Z.get(), N, k,
                       (const double*)ydev.get(), u, N);
    HIF_LAUNCH_CHECK();
    info->iters = its;
  }
  info->iters = its;
}

}  // namespace hif
