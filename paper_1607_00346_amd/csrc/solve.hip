// Operator assembly and matvec (paper, Section 2.4, seven-point stencil),
// application of F^{-1} by level-wise sweeps (Section 2.4, product form of
// F^{-1}), and the FP64 preconditioned CG driver.
#include <cmath>
#include <cstring>

#include "hif_impl.hpp"
#include "prof.hpp"

namespace hif {
namespace {

constexpr int NT = 256;

__device__ __forceinline__ double harmonic(double u, double v) { return 2.0 * u * v / (u + v); }

__global__ __launch_bounds__(NT) void k_assemble(int n, double h2inv, const double* __restrict__ a,
                                                 const double* __restrict__ b, double* diag,
                                                 double* cx, double* cy, double* cz, int* bad) {
  const int64_t N = (int64_t)n * n * n;
  const int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x;
  if (p >= N) return;
  const int x = (int)(p % n), y = (int)((p / n) % n), z = (int)(p / ((int64_t)n * n));
  const double ap = a[p], bp = b[p];
  if (!(ap > 0.0) || !isfinite(ap) || !isfinite(bp)) atomicOr(bad, 1);
  const int64_t sx = 1, sy = n, sz = (int64_t)n * n;
  double d = bp;
  double c;
  c = x < n - 1 ? harmonic(ap, a[p + sx]) * h2inv : 0.0;
  cx[p] = c;
  d += x < n - 1 ? c : ap * h2inv;
  d += x > 0 ? harmonic(ap, a[p - sx]) * h2inv : ap * h2inv;
  c = y < n - 1 ? harmonic(ap, a[p + sy]) * h2inv : 0.0;
  cy[p] = c;
  d += y < n - 1 ? c : ap * h2inv;
  d += y > 0 ? harmonic(ap, a[p - sy]) * h2inv : ap * h2inv;
  c = z < n - 1 ? harmonic(ap, a[p + sz]) * h2inv : 0.0;
  cz[p] = c;
  d += z < n - 1 ? c : ap * h2inv;
  d += z > 0 ? harmonic(ap, a[p - sz]) * h2inv : ap * h2inv;
  diag[p] = d;
}

__global__ __launch_bounds__(NT) void k_matvec(Stencil st, const double* __restrict__ x,
                                               double* __restrict__ y) {
  const int n = st.n;
  const int64_t N = (int64_t)n * n * n;
  const int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x;
  if (p >= N) return;
  const int64_t sy = n, sz = (int64_t)n * n;
  const int xx = (int)(p % n), yy = (int)((p / n) % n), zz = (int)(p / sz);
  double v = st.diag[p] * x[p];
  if (xx < n - 1) v -= st.cx[p] * x[p + 1];
  if (xx > 0) v -= st.cx[p - 1] * x[p - 1];
  if (yy < n - 1) v -= st.cy[p] * x[p + sy];
  if (yy > 0) v -= st.cy[p - sy] * x[p - sy];
  if (zz < n - 1) v -= st.cz[p] * x[p + sz];
  if (zz > 0) v -= st.cz[p - sz] * x[p - sz];
  y[p] = v;
}

// ---- apply sweeps ------------------------------------------------------

__global__ __launch_bounds__(NT) void k_gather_cell(const double* __restrict__ x,
                                                    const int* __restrict__ rows,
                                                    const int64_t* __restrict__ crow_off,
                                                    const FrontDesc* __restrict__ fd,
                                                    const int64_t* __restrict__ yoff,
                                                    const int64_t* __restrict__ zoff, double* xi,
                                                    double* xs, int with_s) {
  const int c = blockIdx.y;
  const FrontDesc f = fd[c];
  const int i = blockIdx.x * NT + threadIdx.x;
  const int* r = rows + crow_off[c];
  if (i < f.nI) xi[yoff[c] + i] = x[r[i]];
  else if (with_s && i < f.nR) xs[zoff[c] + i - f.nI] = x[r[i]];
}

// y = L_I^{-1} x_I  (thread per row of the stored lower-triangular inverse)
template <typename T>
__global__ __launch_bounds__(NT) void k_up_L(const T* __restrict__ arena,
                                             const FrontDesc* __restrict__ fd,
                                             const int64_t* __restrict__ yoff,
                                             const double* __restrict__ xi, double* y) {
  const int c = blockIdx.y;
  const FrontDesc f = fd[c];
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= f.nI) return;
  const T* row = arena + f.off + i;
  const double* xv = xi + yoff[c];
  double s = 0.0;
  for (int t = 0; t <= i; ++t) s += (double)row[(int64_t)f.ld * t] * xv[t];
  y[yoff[c] + i] = s;
}

// z = L_SI y  (rows of S)
template <typename T>
__global__ __launch_bounds__(NT) void k_up_S(const T* __restrict__ arena,
                                             const FrontDesc* __restrict__ fd,
                                             const int64_t* __restrict__ yoff,
                                             const int64_t* __restrict__ zoff,
                                             const double* __restrict__ y, double* z) {
  const int c = blockIdx.y;
  const FrontDesc f = fd[c];
  const int sidx = blockIdx.x * NT + threadIdx.x;
  const int nS = f.nR - f.nI;
  if (sidx >= nS) return;
  const T* row = arena + f.off + f.nI + sidx;
  const double* yv = y + yoff[c];
  double s = 0.0;
  for (int t = 0; t < f.nI; ++t) s += (double)row[(int64_t)f.ld * t] * yv[t];
  z[zoff[c] + sidx] = s;
}

__global__ __launch_bounds__(NT) void k_scatter_I(double* x, const int* __restrict__ rows,
                                                  const int64_t* __restrict__ crow_off,
                                                  const FrontDesc* __restrict__ fd,
                                                  const int64_t* __restrict__ yoff,
                                                  const double* __restrict__ y) {
  const int c = blockIdx.y;
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= fd[c].nI) return;
  x[rows[crow_off[c] + i]] = y[yoff[c] + i];
}

// x_F -= (L_SI y) of the two neighbouring cells, in a fixed order.
__global__ __launch_bounds__(NT) void k_face_sub(double* x, const int* __restrict__ fpts,
                                                 const int64_t* __restrict__ fpt_off,
                                                 const int* __restrict__ fN,
                                                 const int* __restrict__ fcellA,
                                                 const int* __restrict__ fcellB,
                                                 const int* __restrict__ rb_sa,
                                                 const int* __restrict__ rb_sb,
                                                 const int64_t* __restrict__ zoff,
                                                 const double* __restrict__ z) {
  const int f = blockIdx.y;
  const int j = blockIdx.x * NT + threadIdx.x;
  if (j >= fN[f]) return;
  const double za = z[zoff[fcellA[f]] + rb_sa[(size_t)f * kRowBlocks] + j];
  const double zb = z[zoff[fcellB[f]] + rb_sb[(size_t)f * kRowBlocks] + j];
  x[fpts[fpt_off[f] + j]] -= za + zb;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// S_F̌^T Q_F^T: x_F̌ -= T^T x_F̂; x_F̌ <- L_F̌^{-1} x_F̌; x_F̂ -= Y^T x_F̌.
template <typename T>
__global__ __launch_bounds__(NT) void k_skel_up(double* x, const int* __restrict__ skpts,
                                                const SkelDesc* __restrict__ sk,
                                                const T* __restrict__ skel) {
  extern __shared__ double sm[];
  const SkelDesc d = sk[blockIdx.x];
  const int k = d.k, r = d.r;
  double* xh = sm;
  double* xc = sm + k;
  double* xt = xc + r;
  const int* pts = skpts + d.pts_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < k; i += NT) xh[i] = x[pts[i]];
  for (int b = tid; b < r; b += NT) xc[b] = x[pts[k + b]];
  __syncthreads();
  const T* Tm = skel + d.offT;
  for (int b = wave; b < r; b += NT / 64) {
    double s = 0.0;
    for (int i = lane; i < k; i += 64) s += (double)Tm[i + (int64_t)k * b] * xh[i];
    s = wave_sum(s);
    if (lane == 0) xc[b] -= s;
  }
  __syncthreads();
  const T* Lc = skel + d.offL;
  for (int a = tid; a < r; a += NT) {
    double s = 0.0;
    for (int t = 0; t <= a; ++t) s += (double)Lc[a + (int64_t)r * t] * xc[t];
    xt[a] = s;
  }
  __syncthreads();
  const T* Y = skel + d.offY;
  for (int i = wave; i < k; i += NT / 64) {
    double s = 0.0;
    for (int b = lane; b < r; b += 64) s += (double)Y[b + (int64_t)r * i] * xt[b];
    s = wave_sum(s);
    if (lane == 0) xh[i] -= s;
  }
  __syncthreads();
  for (int i = tid; i < k; i += NT) x[pts[i]] = xh[i];
  for (int b = tid; b < r; b += NT) x[pts[k + b]] = xt[b];
}

// Q_F S_F̌: x_F̌ <- L_F̌^{-T}(x_F̌ - Y x_F̂); x_F̂ -= T x_F̌.
template <typename T>
__global__ __launch_bounds__(NT) void k_skel_down(double* x, const int* __restrict__ skpts,
                                                  const SkelDesc* __restrict__ sk,
                                                  const T* __restrict__ skel) {
  extern __shared__ double sm[];
  const SkelDesc d = sk[blockIdx.x];
  const int k = d.k, r = d.r;
  double* xh = sm;
  double* xc = sm + k;
  double* xt = xc + r;
  const int* pts = skpts + d.pts_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < k; i += NT) xh[i] = x[pts[i]];
  for (int b = tid; b < r; b += NT) xc[b] = x[pts[k + b]];
  __syncthreads();
  const T* Y = skel + d.offY;
  for (int b = tid; b < r; b += NT) {
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += (double)Y[b + (int64_t)r * i] * xh[i];
    xt[b] = xc[b] - s;
  }
  __syncthreads();
  const T* Lc = skel + d.offL;
  for (int b = wave; b < r; b += NT / 64) {
    double s = 0.0;
    for (int t = b + lane; t < r; t += 64) s += (double)Lc[t + (int64_t)r * b] * xt[t];
    s = wave_sum(s);
    if (lane == 0) xc[b] = s;
  }
  __syncthreads();
  const T* Tm = skel + d.offT;
  for (int i = tid; i < k; i += NT) {
    double s = 0.0;
    for (int b = 0; b < r; ++b) s += (double)Tm[i + (int64_t)k * b] * xc[b];
    xh[i] -= s;
  }
  __syncthreads();
  for (int i = tid; i < k; i += NT) x[pts[i]] = xh[i];
  for (int b = tid; b < r; b += NT) x[pts[k + b]] = xc[b];
}

// t = x_I - L_SI^T x_S  (wave per column)
template <typename T>
__global__ __launch_bounds__(NT) void k_down_S(const T* __restrict__ arena,
                                               const FrontDesc* __restrict__ fd,
                                               const int64_t* __restrict__ yoff,
                                               const int64_t* __restrict__ zoff,
                                               const double* __restrict__ xi,
                                               const double* __restrict__ xs, double* t) {
  const int c = blockIdx.y;
  const FrontDesc f = fd[c];
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  if (i >= f.nI) return;
  const int nS = f.nR - f.nI;
  const T* col = arena + f.off + f.nI + (int64_t)f.ld * i;
  const double* xv = xs + zoff[c];
  double s = 0.0;
  for (int q = lane; q < nS; q += 64) s += (double)col[q] * xv[q];
  s = wave_sum(s);
  if (lane == 0) t[yoff[c] + i] = xi[yoff[c] + i] - s;
}

// x_I = L_I^{-T} t  (wave per column of the stored inverse)
template <typename T>
__global__ __launch_bounds__(NT) void k_down_L(const T* __restrict__ arena,
                                               const FrontDesc* __restrict__ fd,
                                               const int64_t* __restrict__ yoff,
                                               const double* __restrict__ t, double* x,
                                               const int* __restrict__ rows,
                                               const int64_t* __restrict__ crow_off) {
  const int c = blockIdx.y;
  const FrontDesc f = fd[c];
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  if (i >= f.nI) return;
  const T* col = arena + f.off + (int64_t)f.ld * i;
  const double* tv = t + yoff[c];
  double s = 0.0;
  for (int q = i + lane; q < f.nI; q += 64) s += (double)col[q] * tv[q];
  s = wave_sum(s);
  if (lane == 0) x[rows[crow_off[c] + i]] = s;
}

// ---- PCG vector kernels --------------------------------------------------

constexpr int kDotBlocks = 1024;

// part[b] = sum over a strided slice of a .* (b - c) (c may be null)
__global__ __launch_bounds__(NT) void k_dot_partial(const double* __restrict__ a,
                                                    const double* __restrict__ b,
                                                    const double* __restrict__ c, int64_t N,
                                                    double* part) {
  __shared__ double red[NT / 64];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < N; i += (int64_t)gridDim.x * NT)
    s += a[i] * (c ? b[i] - c[i] : b[i]);
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NT / 64; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(NT) void k_dot_final(const double* __restrict__ part, int nb,
                                                  double* out) {
  __shared__ double red[NT / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += NT) s += part[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NT / 64; ++w) t += red[w];
    *out = t;
  }
}

// alpha = sc[0] / sc[1]; r_old = r; r -= alpha q; u += alpha p
__global__ __launch_bounds__(NT) void k_cg_step(double* u, double* r, double* rold,
                                                const double* __restrict__ p,
                                                const double* __restrict__ q,
                                                const double* __restrict__ sc, int64_t N) {
  const double alpha = sc[0] / sc[1];
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < N; i += (int64_t)gridDim.x * NT) {
    const double ri = r[i];
    rold[i] = ri;
    r[i] = ri - alpha * q[i];
    u[i] += alpha * p[i];
  }
}

// beta = sc[2] / sc[0]; p = z + beta p
__global__ __launch_bounds__(NT) void k_cg_dir(double* p, const double* __restrict__ z,
                                               const double* __restrict__ sc, int64_t N) {
  const double beta = sc[2] / sc[0];
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < N; i += (int64_t)gridDim.x * NT)
    p[i] = z[i] + beta * p[i];
}

__global__ void k_copy_scalar(double* sc, int dst, int src) { sc[dst] = sc[src]; }

// y = f - y
__global__ __launch_bounds__(NT) void k_residual(const double* __restrict__ f, double* y, int64_t N) {
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < N; i += (int64_t)gridDim.x * NT)
    y[i] = f[i] - y[i];
}

unsigned grid_for(int64_t N) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(N, NT), 8192)); }

}  // namespace

void problem_assemble(hif_problem_s* A, const double* a, const double* b, hipStream_t s) {
  const int n = A->n;
  const int64_t N = A->N;
  A->diag.alloc(N);
  A->cx.alloc(N);
  A->cy.alloc(N);
  A->cz.alloc(N);
  DevBuf<int> bad(1);
  HIF_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int), s));
  const double h2inv = (double)(n + 1) * (double)(n + 1);
  hipLaunchKernelGGL(k_assemble, dim3((unsigned)ceil_div(N, NT)), dim3(NT), 0, s, n, h2inv, a, b,
                     A->diag.get(), A->cx.get(), A->cy.get(), A->cz.get(), bad.get());
  HIF_LAUNCH_CHECK();
  int h = 0;
  HIF_HIP(hipMemcpyAsync(&h, bad.get(), sizeof(int), hipMemcpyDeviceToHost, s));
  HIF_HIP(hipStreamSynchronize(s));
  HIF_REQUIRE(h == 0, HIF_EINVAL, "a must be positive and finite, b finite");
}

void stencil_matvec(const Stencil& st, const double* x, double* y, hipStream_t s) {
  const int64_t N = (int64_t)st.n * st.n * st.n;
  ProfScope ps("matvec", s, 13.0 * N, 48.0 * N);
  hipLaunchKernelGGL(k_matvec, dim3((unsigned)ceil_div(N, NT)), dim3(NT), 0, s, st, x, y);
  HIF_LAUNCH_CHECK();
}

template <typename T>
void FactorImpl<T>::apply(const double* f, double* u, hipStream_t s) {
  if (u != f) HIF_HIP(hipMemcpyAsync(u, f, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
  int64_t ymax = 1, zmax = 1;
  for (auto& l : levels) { ymax = std::max(ymax, l.ysum); zmax = std::max(zmax, l.zsum); }
  if ((int64_t)ybuf.size() < 2 * ymax) ybuf.alloc(2 * ymax);
  if ((int64_t)zbuf.size() < 2 * zmax) zbuf.alloc(2 * zmax);
  double* xi = ybuf.get();
  double* yv = ybuf.get() + ymax;
  double* zv = zbuf.get();
  double* xsv = zbuf.get() + zmax;
  const int nlev = (int)levels.size();
  for (auto& lv : levels) {
    if (lv.bytes_L > 0.0 || lv.P.ncell == 0) continue;
    for (const FrontDesc& d : lv.hfd) {
      lv.bytes_L += sizeof(T) * 0.5 * d.nI * (d.nI + 1.0) + 24.0 * d.nI;
      lv.bytes_S += sizeof(T) * (double)(d.nR - d.nI) * d.nI + 16.0 * (d.nR - d.nI) + 8.0 * d.nI;
    }
    for (const SkelDesc& d : lv.hsk)
      lv.bytes_skel += sizeof(T) * (2.0 * d.k * d.r + 0.5 * d.r * (d.r + 1.0)) +
                       32.0 * (d.k + d.r);
  }
  // W^l^T for l = 0..L (level L: L_Sigma^{-1})
  for (int l = 0; l < nlev; ++l) {
    Level<T>& lv = levels[l];
    profiler().level = l;
    const int nc = lv.P.ncell;
    if (nc > 0) {
      dim3 gI((unsigned)ceil_div(std::max(1, lv.maxI), NT), (unsigned)nc);
      {
        ProfScope ps("apply_up_L", s, 0.0, lv.bytes_L);
        hipLaunchKernelGGL(k_gather_cell, gI, dim3(NT), 0, s, u, lv.rows.get(), lv.crow_off.get(),
                           lv.fd.get(), lv.yoff.get(), lv.zoff.get(), xi, xsv, 0);
        hipLaunchKernelGGL((k_up_L<T>), gI, dim3(NT), 0, s, lv.front.get(), lv.fd.get(),
                           lv.yoff.get(), xi, yv);
      }
      if (lv.maxS > 0) {
        ProfScope ps("apply_up_S", s, 0.0, lv.bytes_S);
        dim3 gS((unsigned)ceil_div(lv.maxS, NT), (unsigned)nc);
        hipLaunchKernelGGL((k_up_S<T>), gS, dim3(NT), 0, s, lv.front.get(), lv.fd.get(),
                           lv.yoff.get(), lv.zoff.get(), yv, zv);
      }
      {
        ProfScope ps("apply_scatter", s);
        hipLaunchKernelGGL(k_scatter_I, gI, dim3(NT), 0, s, u, lv.rows.get(), lv.crow_off.get(),
                           lv.fd.get(), lv.yoff.get(), yv);
      }
      HIF_LAUNCH_CHECK();
    }
    if (!lv.P.root && lv.P.nface > 0) {
      {
        ProfScope ps("apply_scatter", s);
        dim3 gF((unsigned)ceil_div(std::max(1, lv.maxF), NT), (unsigned)lv.P.nface);
        hipLaunchKernelGGL(k_face_sub, gF, dim3(NT), 0, s, u, lv.fpts.get(), lv.fpt_off.get(),
                           lv.fN.get(), lv.fcellA.get(), lv.fcellB.get(), lv.rb_sa.get(),
                           lv.rb_sb.get(), lv.zoff.get(), zv);
        HIF_LAUNCH_CHECK();
      }
      if (!lv.hsk.empty()) {
        ProfScope ps("apply_skel", s, 0.0, lv.bytes_skel);
        const size_t shm = sizeof(double) * (lv.maxk + 2 * (size_t)lv.maxr);
        hipLaunchKernelGGL((k_skel_up<T>), dim3((unsigned)lv.hsk.size()), dim3(NT), shm, s, u,
                           lv.skpts.get(), lv.sk.get(), lv.skel.get());
        HIF_LAUNCH_CHECK();
      }
    }
  }
  // W^l for l = L..0
  for (int l = nlev - 1; l >= 0; --l) {
    Level<T>& lv = levels[l];
    profiler().level = l;
    if (!lv.P.root && !lv.hsk.empty()) {
      ProfScope ps("apply_skel", s, 0.0, lv.bytes_skel);
      const size_t shm = sizeof(double) * (lv.maxk + 2 * (size_t)lv.maxr);
      hipLaunchKernelGGL((k_skel_down<T>), dim3((unsigned)lv.hsk.size()), dim3(NT), shm, s, u,
                         lv.skpts.get(), lv.sk.get(), lv.skel.get());
      HIF_LAUNCH_CHECK();
    }
    const int nc = lv.P.ncell;
    if (nc == 0) continue;
    const int gmax = std::max(lv.maxI, lv.maxI + lv.maxS);
    dim3 gG((unsigned)ceil_div(std::max(1, gmax), NT), (unsigned)nc);
    dim3 gW((unsigned)ceil_div(std::max(1, lv.maxI), NT / 64), (unsigned)nc);
    {
      ProfScope ps("apply_down_S", s, 0.0, lv.bytes_S);
      hipLaunchKernelGGL(k_gather_cell, gG, dim3(NT), 0, s, u, lv.rows.get(), lv.crow_off.get(),
                         lv.fd.get(), lv.yoff.get(), lv.zoff.get(), xi, xsv, 1);
      hipLaunchKernelGGL((k_down_S<T>), gW, dim3(NT), 0, s, lv.front.get(), lv.fd.get(),
                         lv.yoff.get(), lv.zoff.get(), xi, xsv, yv);
    }
    {
      ProfScope ps("apply_down_L", s, 0.0, lv.bytes_L);
      hipLaunchKernelGGL((k_down_L<T>), gW, dim3(NT), 0, s, lv.front.get(), lv.fd.get(),
                         lv.yoff.get(), yv, u, lv.rows.get(), lv.crow_off.get());
    }
    HIF_LAUNCH_CHECK();
  }
  profiler().level = -1;
}

template void FactorImpl<double>::apply(const double*, double*, hipStream_t);
template void FactorImpl<float>::apply(const double*, double*, hipStream_t);

namespace {

struct Dot {
  DevBuf<double> part{kDotBlocks};
  void run(const double* a, const double* b, const double* c, int64_t N, double* out,
           hipStream_t s) {
    const unsigned nb = (unsigned)std::min<int64_t>(kDotBlocks, std::max<int64_t>(1, ceil_div(N, NT)));
    ProfScope ps("pcg_dot", s, 2.0 * N, (c ? 24.0 : 16.0) * N);
    hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(NT), 0, s, a, b, c, N, part.get());
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(NT), 0, s, (const double*)part.get(), (int)nb, out);
    HIF_LAUNCH_CHECK();
  }
};

}  // namespace

void pcg_solve(const hif_problem_s* A, hif_factor_s* F, const double* f, double* u, double tol,
               int maxit, hif_pcg_info* info, hipStream_t s) {
  const int64_t N = A->N;
  const Stencil st = A->stencil();
  DevBuf<double> r(N), rold(N), z(N), p(N), q(N), sc(8);
  Dot dot;
  double h[8];
  auto fetch = [&]() {
    HIF_HIP(hipMemcpyAsync(h, sc.get(), sizeof(h), hipMemcpyDeviceToHost, s));
    HIF_HIP(hipStreamSynchronize(s));
  };
  HIF_HIP(hipMemsetAsync(u, 0, sizeof(double) * N, s));
  HIF_HIP(hipMemcpyAsync(r.get(), f, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
  dot.run(f, f, nullptr, N, sc.get() + 5, s);
  fetch();
  const double fn = std::sqrt(h[5]);
  info->iters = 0;
  info->converged = 0;
  info->relres = fn == 0.0 ? 0.0 : 1.0;
  if (fn == 0.0) {
    info->converged = 1;
    return;
  }
  F->impl->apply(r.get(), z.get(), s);
  HIF_HIP(hipMemcpyAsync(p.get(), z.get(), sizeof(double) * N, hipMemcpyDeviceToDevice, s));
  dot.run(r.get(), z.get(), nullptr, N, sc.get() + 0, s);
  const unsigned g = grid_for(N);
  for (int it = 1; it <= maxit; ++it) {
    stencil_matvec(st, p.get(), q.get(), s);
    dot.run(p.get(), q.get(), nullptr, N, sc.get() + 1, s);
    hipLaunchKernelGGL(k_cg_step, dim3(g), dim3(NT), 0, s, u, r.get(), rold.get(), p.get(), q.get(),
                       (const double*)sc.get(), N);
    dot.run(r.get(), r.get(), nullptr, N, sc.get() + 4, s);
    fetch();
    info->iters = it;
    if (!(h[1] > 0.0) || !std::isfinite(h[4])) break;  // breakdown
    if (std::sqrt(h[4]) <= tol * fn) {
      stencil_matvec(st, u, q.get(), s);
      hipLaunchKernelGGL(k_residual, dim3(g), dim3(NT), 0, s, f, q.get(), N);
      dot.run(q.get(), q.get(), nullptr, N, sc.get() + 6, s);
      fetch();
      info->relres = std::sqrt(h[6]) / fn;
      if (info->relres <= tol) {
        info->converged = 1;
        return;
      }
      HIF_HIP(hipMemcpyAsync(r.get(), q.get(), sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    }
    F->impl->apply(r.get(), z.get(), s);
    dot.run(z.get(), r.get(), rold.get(), N, sc.get() + 2, s);
    dot.run(r.get(), z.get(), nullptr, N, sc.get() + 3, s);
    hipLaunchKernelGGL(k_cg_dir, dim3(g), dim3(NT), 0, s, p.get(), (const double*)z.get(),
                       (const double*)sc.get(), N);
    hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, s, sc.get(), 0, 3);
    HIF_LAUNCH_CHECK();
  }
  stencil_matvec(st, u, q.get(), s);
  hipLaunchKernelGGL(k_residual, dim3(g), dim3(NT), 0, s, f, q.get(), N);
  dot.run(q.get(), q.get(), nullptr, N, sc.get() + 6, s);
  fetch();
  info->relres = std::sqrt(h[6]) / fn;
  info->converged = info->relres <= tol;
}

}  // namespace hif
