// Operator assembly and matvec (paper, Section 2.4, seven-point stencil),
// application of F^{-1} by level-wise sweeps (Section 2.4, product form of
// F^{-1}), and the FP64 preconditioned CG driver.
#include <cmath>
#include <thread>
#include <mutex>
#include <exception>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <string>

#include "hif_impl.hpp"
#include "prof.hpp"

namespace hif {
namespace {

constexpr int NT = 256;

__device__ __forceinline__ double harmonic(double u, double v) { return 2.0 * u * v / (u + v); }

// Periodic variant of k_assemble: every point has six neighbours, indices wrap.
__global__ __launch_bounds__(NT) void k_assemble_periodic(int n, double h2inv,
                                                          const double* __restrict__ a,
                                                          const double* __restrict__ b,
                                                          double* diag, double* cx, double* cy,
                                                          double* cz, int* bad) {
  const int64_t N = (int64_t)n * n * n;
  const int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x;
  if (p >= N) return;
  const int x = (int)(p % n), y = (int)((p / n) % n), z = (int)(p / ((int64_t)n * n));
  const double ap = a[p], bp = b[p];
  if (!(ap > 0.0) || !isfinite(ap) || !isfinite(bp)) atomicOr(bad, 1);
  const int64_t sy = n, sz = (int64_t)n * n;
  const int64_t xp = x < n - 1 ? p + 1 : p - (n - 1), xm = x > 0 ? p - 1 : p + (n - 1);
  const int64_t yp = y < n - 1 ? p + sy : p - (n - 1) * sy, ym = y > 0 ? p - sy : p + (n - 1) * sy;
  const int64_t zp = z < n - 1 ? p + sz : p - (n - 1) * sz, zm = z > 0 ? p - sz : p + (n - 1) * sz;
  double d = bp;
  double c = harmonic(ap, a[xp]) * h2inv;
  cx[p] = c;
  d += c + harmonic(ap, a[xm]) * h2inv;
  c = harmonic(ap, a[yp]) * h2inv;
  cy[p] = c;
  d += c + harmonic(ap, a[ym]) * h2inv;
  c = harmonic(ap, a[zp]) * h2inv;
  cz[p] = c;
  d += c + harmonic(ap, a[zm]) * h2inv;
  diag[p] = d;
}

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
  if (!st.periodic) {
    if (xx < n - 1) v -= st.cx[p] * x[p + 1];
    if (xx > 0) v -= st.cx[p - 1] * x[p - 1];
    if (yy < n - 1) v -= st.cy[p] * x[p + sy];
    if (yy > 0) v -= st.cy[p - sy] * x[p - sy];
    if (zz < n - 1) v -= st.cz[p] * x[p + sz];
    if (zz > 0) v -= st.cz[p - sz] * x[p - sz];
  } else {
    const int64_t xp = xx < n - 1 ? p + 1 : p - (n - 1), xm = xx > 0 ? p - 1 : p + (n - 1);
    const int64_t yp = yy < n - 1 ? p + sy : p - (n - 1) * sy;
    const int64_t ym = yy > 0 ? p - sy : p + (n - 1) * sy;
    const int64_t zp = zz < n - 1 ? p + sz : p - (n - 1) * sz;
    const int64_t zm = zz > 0 ? p - sz : p + (n - 1) * sz;
    v -= st.cx[p] * x[xp] + st.cx[xm] * x[xm];
    v -= st.cy[p] * x[yp] + st.cy[ym] * x[ym];
    v -= st.cz[p] * x[zp] + st.cz[zm] * x[zm];
  }
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

// y[roff + i] (+)= alpha sum_t A(i, t) x[coff + t] (tri: t <= i only): 64
// rows per workgroup, the columns split over the NW waves in groups of 8
// (independent loads in flight), partial sums reduced through LDS in wave
// order.  Groups that straddle the diagonal load all 8 columns (the stored
// upper triangle is in bounds) and drop the entries above it by selects.
// Launches of few row blocks take NW = 16, so that each workgroup keeps
// enough loads in flight to stream its long rows.
template <typename T, int NW>
__global__ __launch_bounds__(64 * NW) void k_gemv_n(const GemvDesc* __restrict__ dd,
                                                    const double* __restrict__ x, double* y,
                                                    double alpha, int accumulate) {
  __shared__ double part[NW][64];
  const GemvDesc d = dd[blockIdx.y];
  const int r0 = blockIdx.x * 64;
  if (r0 >= d.m) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = r0 + lane;
  const bool row_ok = i < d.m;
  const int tend = d.tri ? min(d.n, r0 + 64) : d.n;
  const auto A = as_global((const T*)d.A + (row_ok ? i : 0));
  const auto xv = as_global(x + d.coff);
  double s0 = 0.0, s1 = 0.0;
  for (int t0 = wave * 8; t0 < tend; t0 += 8 * NW) {
    if (t0 + 8 <= tend) {
      double a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = (double)A[(int64_t)d.lda * (t0 + u)];
      if (!d.tri || t0 + 8 <= r0) {
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
          s0 += a[u] * xv[t0 + u];
          s1 += a[u + 1] * xv[t0 + u + 1];
        }
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) s0 += t0 + u <= i ? a[u] * xv[t0 + u] : 0.0;
      }
    } else {
      for (int t = t0; t < tend; ++t)
        if (!d.tri || t <= i) s0 += (double)A[(int64_t)d.lda * t] * xv[t];
    }
  }
  part[wave][lane] = row_ok ? s0 + s1 : 0.0;
  __syncthreads();
  if (wave == 0 && row_ok) {
    double sum = part[0][lane];
#pragma unroll
    for (int w = 1; w < NW; ++w) sum += part[w][lane];
    const double v = alpha * sum;
    const auto yo = as_global(y + d.roff + i);
    *yo = accumulate ? *yo + v : v;
  }
}

// Sixteen bytes of matrix elements, and the matching entries of x.
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  static constexpr int N = 4;
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct Vec16<double> {
  static constexpr int N = 2;
  typedef double type __attribute__((ext_vector_type(2)));
};

// y[coff + j] (+)= alpha sum_i A(i, j) x[roff + i] (tri: i >= j only): 16
// lanes per column, NG columns at a time, 64 columns per workgroup.  Each
// column is read as 16-byte vectors (two full cache lines per load across its
// 16 lanes) after a scalar head up to the first aligned row, then a scalar
// tail.  Launches of few column blocks over long columns take NG = 64 (all 64
// columns at once); a column's sum is the same either way.
constexpr int kGemvTCols = 64;
template <typename T, int NG>
__global__ __launch_bounds__(16 * NG) void k_gemv_t(const GemvDesc* __restrict__ dd,
                                                    const double* __restrict__ x, double* y,
                                                    double alpha, int accumulate) {
  using V = typename Vec16<T>::type;
  constexpr int VN = Vec16<T>::N;
  const GemvDesc d = dd[blockIdx.y];
  const int g = threadIdx.x >> 4, l = threadIdx.x & 15;
  const auto xv = as_global(x + d.roff);
  const int jend = min(d.n, (int)(blockIdx.x + 1) * kGemvTCols);
  for (int jb = blockIdx.x * kGemvTCols; jb < jend; jb += NG) {
    const int j = jb + g;
    double s0 = 0.0, s1 = 0.0;
    if (j < jend) {
      const T* col = (const T*)d.A + (int64_t)d.lda * j;
      const int i0 = d.tri ? j : 0;
      const int head = min(d.m - i0, (int)(((16 - ((uintptr_t)(col + i0) & 15)) & 15) / sizeof(T)));
      if (l < head) s0 += (double)as_global(col)[i0 + l] * xv[i0 + l];
      const int ib = i0 + head;
      const int nv = (d.m - ib) / VN;
      const auto cv = as_global((const V*)(col + ib));
      auto madd = [&](const V a, int v) {
        const int i = ib + VN * v;
#pragma unroll
        for (int e = 0; e < VN; e += 2) {
          s0 += (double)a[e] * xv[i + e];
          s1 += (double)a[e + 1] * xv[i + e + 1];
        }
      };
      int v = l;
      // four loads in flight per lane before their products
      for (; v + 48 < nv; v += 64) {
        const V a0 = cv[v], a1 = cv[v + 16], a2 = cv[v + 32], a3 = cv[v + 48];
        madd(a0, v);
        madd(a1, v + 16);
        madd(a2, v + 32);
        madd(a3, v + 48);
      }
      for (; v < nv; v += 16) {
        const V a = cv[v];
        madd(a, v);
      }
      const int it = ib + VN * nv + l;
      if (it < d.m) s0 += (double)as_global(col)[it] * xv[it];
    }
    double v = s0 + s1;
    v += __shfl_xor(v, 8, 16);
    v += __shfl_xor(v, 4, 16);
    v += __shfl_xor(v, 2, 16);
    v += __shfl_xor(v, 1, 16);
    if (j < jend && l == 0) {
      const auto yo = as_global(y + d.coff + j);
      *yo = accumulate ? *yo + alpha * v : alpha * v;
    }
  }
}

// y[roff + i] (+)= alpha sum_t A(i, t) x[coff + t] (tri: t <= i only) for
// matrices whose columns start 16-byte aligned: lane l of group g reads VN
// consecutive rows as one 16-byte vector, the NG groups take every NG-th
// column, partial sums are reduced through LDS in group order.  Rows past m
// are read only by the lanes that hold both valid and invalid rows, element
// by element.  Launches of few row blocks (the top levels' few large
// triangles, where one workgroup streams a whole row block of up to several
// thousand columns) take NG = 64.
template <typename T, int NG>
__global__ __launch_bounds__(16 * NG) void k_gemv_nv(const GemvDesc* __restrict__ dd,
                                                     const double* __restrict__ x, double* y,
                                                     double alpha, int accumulate) {
  using V = typename Vec16<T>::type;
  constexpr int VN = Vec16<T>::N;
  constexpr int R = 16 * VN;  // rows per workgroup
  __shared__ double part[NG][R + 1];
  const GemvDesc d = dd[blockIdx.y];
  const int r0 = blockIdx.x * R;
  if (r0 >= d.m) return;
  const int g = threadIdx.x >> 4, l = threadIdx.x & 15;
  const int i = r0 + VN * l;
  const int tend = d.tri ? min(d.n, r0 + R) : d.n;
  const auto xv = as_global(x + d.coff);
  const bool full = i + VN <= d.m;
  double acc[VN];
#pragma unroll
  for (int e = 0; e < VN; ++e) acc[e] = 0.0;
#pragma unroll 4
  for (int t = g; t < tend; t += NG) {
    const double xt = xv[t];
    const T* col = (const T*)d.A + (int64_t)d.lda * t;
    T a[VN];
    if (full) {
      const V v = *as_global((const V*)(col + i));
#pragma unroll
      for (int e = 0; e < VN; ++e) a[e] = v[e];
    } else {
#pragma unroll
      for (int e = 0; e < VN; ++e) a[e] = i + e < d.m ? as_global(col)[i + e] : T(0);
    }
#pragma unroll
    for (int e = 0; e < VN; ++e) acc[e] += (!d.tri || t <= i + e) ? (double)a[e] * xt : 0.0;
  }
#pragma unroll
  for (int e = 0; e < VN; ++e) part[g][VN * l + e] = acc[e];
  __syncthreads();
  if (threadIdx.x < R) {
    const int row = r0 + threadIdx.x;
    if (row < d.m) {
      double sum = 0.0;
#pragma unroll
      for (int q = 0; q < NG; ++q) sum += part[q][threadIdx.x];
      const double v = alpha * sum;
      const auto yo = as_global(y + d.roff + row);
      *yo = accumulate ? *yo + v : v;
    }
  }
}

// Skeleton vectors: xh[kofs + i] = u[F̂_i], xc[rofs + b] = u[F̌_b] (gather) or
// the reverse (scatter).
__global__ __launch_bounds__(NT) void k_skel_move(double* u, const int* __restrict__ skpts,
                                                  const SkelDesc* __restrict__ sk, double* xh,
                                                  double* xc, int to_u) {
  const SkelDesc d = sk[blockIdx.y];
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= d.k + d.r) return;
  const int p = skpts[d.pts_off + i];
  double* s = i < d.k ? xh + d.kofs + i : xc + d.rofs + (i - d.k);
  if (to_u) u[p] = *s;
  else *s = u[p];
}

// ---- fused per-front sweeps (levels of many small fronts) -------------------
// One workgroup per cell gathers the cell's vector entries into LDS, applies
// its factor blocks reading each stored word once, and scatters the result:
// one launch per level and sweep instead of a gather, two matrix-vector
// launches and a scatter.  Factor columns are read as 16-byte vectors from
// quads of rows aligned to the column start (the front base is 16-byte
// aligned and ld a multiple of the quad), so a quad may reach past the rows
// wanted: those entries lie inside the column's padded ld rows and are
// dropped.

// out[r - r0] = sum_t A(r, t) x[t] for r in [r0, r1), t < ncol (tri: only
// t < the end of r's quad; the stored upper triangle is zero).
template <typename T>
__device__ __forceinline__ void fused_gemv_n(const T* A, int ld, int r0, int r1, int ncol,
                                             bool tri, const double* x, double* out,
                                             double* part) {
  using V = typename Vec16<T>::type;
  constexpr int VN = Vec16<T>::N;
  const int q0 = r0 / VN, q1 = (r1 + VN - 1) / VN, nq = q1 - q0;
  if (nq <= 0) return;  // uniform over the workgroup
  const int tid = threadIdx.x;
  const int G = nq >= NT ? 1 : NT / nq;  // column groups
  const int busy = nq >= NT ? NT : nq * G;
  const int g = tid / (nq >= NT ? NT : nq);
  for (int qq = tid % (nq >= NT ? NT : nq); qq < nq && tid < busy; qq += (nq >= NT ? NT : nq)) {
    const int q = q0 + qq;
    const int tend = tri ? min(ncol, VN * q + VN) : ncol;
    double acc[VN];
#pragma unroll
    for (int e = 0; e < VN; ++e) acc[e] = 0.0;
    const auto col = as_global((const V*)(A + VN * q));
    const int64_t ldv = ld / VN;
    int t = g;
    for (; t + 3 * G < tend; t += 4 * G) {
      const V a0 = col[ldv * t], a1 = col[ldv * (t + G)], a2 = col[ldv * (t + 2 * G)],
              a3 = col[ldv * (t + 3 * G)];
#pragma unroll
      for (int e = 0; e < VN; ++e)
        acc[e] += (double)a0[e] * x[t] + (double)a1[e] * x[t + G] + (double)a2[e] * x[t + 2 * G] +
                  (double)a3[e] * x[t + 3 * G];
    }
    for (; t < tend; t += G) {
      const V a = col[ldv * t];
#pragma unroll
      for (int e = 0; e < VN; ++e) acc[e] += (double)a[e] * x[t];
    }
    if (G == 1) {
#pragma unroll
      for (int e = 0; e < VN; ++e) {
        const int r = VN * q + e;
        if (r >= r0 && r < r1) out[r - r0] = acc[e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < VN; ++e) part[g * (nq * VN) + qq * VN + e] = acc[e];
    }
  }
  if (G > 1) {
    __syncthreads();
    for (int i = tid; i < nq * VN; i += NT) {
      const int r = VN * q0 + i;
      if (r < r0 || r >= r1) continue;
      double v = 0.0;
      for (int k = 0; k < G; ++k) v += part[k * (nq * VN) + i];
      out[r - r0] = v;
    }
  }
  __syncthreads();
}

// out[t] = sum_{r in [r0, r1)} A(r, t) x[r - r0] for t < ncol (tri: r >= t):
// 16 lanes per column, the columns dealt to the 16 groups of the workgroup.
template <typename T>
__device__ __forceinline__ void fused_gemv_t(const T* A, int ld, int r0, int r1, int ncol,
                                             bool tri, const double* x, double* out) {
  using V = typename Vec16<T>::type;
  constexpr int VN = Vec16<T>::N;
  const int g = threadIdx.x >> 4, l = threadIdx.x & 15;
  for (int tb = 0; tb < ncol; tb += NT / 16) {
    const int t = tb + g;
    double s = 0.0;
    if (t < ncol) {
      const int rs = tri ? max(r0, t) : r0;
      const int qb = rs / VN, qe = (r1 + VN - 1) / VN;
      const auto col = as_global((const V*)(A + (int64_t)ld * t));
      int q = qb + l;
      for (; q + 16 < qe; q += 32) {
        const V a0 = col[q], a1 = col[q + 16];
#pragma unroll
        for (int e = 0; e < VN; ++e) {
          const int r = VN * q + e, r2 = r + 16 * VN;
          s += (r >= rs && r < r1) ? (double)a0[e] * x[r - r0] : 0.0;
          s += (r2 >= rs && r2 < r1) ? (double)a1[e] * x[r2 - r0] : 0.0;
        }
      }
      for (; q < qe; q += 16) {
        const V a = col[q];
#pragma unroll
        for (int e = 0; e < VN; ++e) {
          const int r = VN * q + e;
          s += (r >= rs && r < r1) ? (double)a[e] * x[r - r0] : 0.0;
        }
      }
    }
    s += __shfl_xor(s, 8, 16);
    s += __shfl_xor(s, 4, 16);
    s += __shfl_xor(s, 2, 16);
    s += __shfl_xor(s, 1, 16);
    if (t < ncol && l == 0) out[t] = s;
  }
  __syncthreads();
}

// Up sweep of one level: x_I <- L_I^{-1} x_I (scattered into u) and
// z = L_SI x_I for the face update.  Dynamic LDS: 2 maxI + 4 NT doubles.
template <typename T>
__global__ __launch_bounds__(NT) void k_up_fused(double* u, const int* __restrict__ rows,
                                                 const int64_t* __restrict__ crow_off,
                                                 const FrontDesc* __restrict__ fd, int maxI,
                                                 const int64_t* __restrict__ zoff, double* zv) {
  extern __shared__ double lds[];
  double* xs = lds;
  double* ys = lds + maxI;
  double* part = lds + 2 * maxI;
  const FrontDesc f = fd[blockIdx.x];
  const int* r = rows + crow_off[blockIdx.x];
  const T* L = static_cast<const T*>(f.ptr);
  for (int i = threadIdx.x; i < f.nI; i += NT) xs[i] = u[r[i]];
  __syncthreads();
  fused_gemv_n<T>(L, f.ld, 0, f.nI, f.nI, true, xs, ys, part);
  for (int i = threadIdx.x; i < f.nI; i += NT) u[r[i]] = ys[i];
  if (f.nR > f.nI) fused_gemv_n<T>(L, f.ld, f.nI, f.nR, f.nI, false, ys, zv + zoff[blockIdx.x], part);
}

// Down sweep of one level: x_I <- L_I^{-T} (x_I - L_SI^T x_S), scattered into
// u.  Dynamic LDS: 2 maxI + maxS doubles.
template <typename T>
__global__ __launch_bounds__(NT) void k_down_fused(double* u, const int* __restrict__ rows,
                                                   const int64_t* __restrict__ crow_off,
                                                   const FrontDesc* __restrict__ fd, int maxI) {
  extern __shared__ double lds[];
  double* xi = lds;
  double* ys = lds + maxI;
  double* xsv = lds + 2 * maxI;
  const FrontDesc f = fd[blockIdx.x];
  const int* r = rows + crow_off[blockIdx.x];
  const T* L = static_cast<const T*>(f.ptr);
  for (int i = threadIdx.x; i < f.nR; i += NT) {
    const double v = u[r[i]];
    if (i < f.nI) xi[i] = v;
    else xsv[i - f.nI] = v;
  }
  __syncthreads();
  if (f.nR > f.nI) {
    fused_gemv_t<T>(L, f.ld, f.nI, f.nR, f.nI, false, xsv, ys);
    for (int i = threadIdx.x; i < f.nI; i += NT) xi[i] -= ys[i];
    __syncthreads();
  }
  fused_gemv_t<T>(L, f.ld, 0, f.nI, f.nI, true, xi, ys);
  for (int i = threadIdx.x; i < f.nI; i += NT) u[r[i]] = ys[i];
}

// Skeleton step of one face in one wave (levels of many small faces): the
// face's x_F̂ (k) and x_F̌ (r) are gathered into LDS and the three small
// products run there.  Up: x_F̌ -= T^T x_F̂, x_F̌ <- L_F̌^{-1} x_F̌,
// x_F̂ -= Y^T x_F̌.  Down: x_F̌ -= Y x_F̂, x_F̌ <- L_F̌^{-T} x_F̌, x_F̂ -= T x_F̌.
// L_F̌^{-1}'s stored upper triangle is not zero, so its loops stop at the
// diagonal.  Dynamic LDS: maxF + maxr doubles.
template <typename T>
__global__ __launch_bounds__(64) void k_skel_fused(double* u, const int* __restrict__ skpts,
                                                   const SkelDesc* __restrict__ sk,
                                                   const T* __restrict__ skel, int maxF, int down) {
  extern __shared__ double lds[];
  const SkelDesc d = sk[blockIdx.x];
  const int k = d.k, r = d.r, lane = threadIdx.x;
  double* xh = lds;
  double* xc = lds + k;
  double* yc = lds + maxF;
  const int* pts = skpts + d.pts_off;
  const auto Tm = as_global(skel + d.offT);
  const auto Lc = as_global(skel + d.offL);
  const auto Y = as_global(skel + d.offY);
  for (int i = lane; i < k + r; i += 64) lds[i] = u[pts[i]];
  __syncthreads();
  if (!down) {
    for (int b = lane; b < r; b += 64) {
      double s = 0.0;
      for (int i = 0; i < k; ++i) s += (double)Tm[i + (int64_t)k * b] * xh[i];
      xc[b] -= s;
    }
    __syncthreads();
    for (int b = lane; b < r; b += 64) {
      double s = 0.0;
      for (int t = 0; t <= b; ++t) s += (double)Lc[b + (int64_t)r * t] * xc[t];
      yc[b] = s;
    }
    __syncthreads();
    for (int i = lane; i < k; i += 64) {
      double s = 0.0;
      for (int b = 0; b < r; ++b) s += (double)Y[b + (int64_t)r * i] * yc[b];
      xh[i] -= s;
    }
  } else {
    for (int b = lane; b < r; b += 64) {
      double s = 0.0;
      for (int i = 0; i < k; ++i) s += (double)Y[b + (int64_t)r * i] * xh[i];
      xc[b] -= s;
    }
    __syncthreads();
    for (int b = lane; b < r; b += 64) {
      double s = 0.0;
      for (int t = b; t < r; ++t) s += (double)Lc[t + (int64_t)r * b] * xc[t];
      yc[b] = s;
    }
    __syncthreads();
    for (int i = lane; i < k; i += 64) {
      double s = 0.0;
      for (int b = 0; b < r; ++b) s += (double)Tm[i + (int64_t)k * b] * yc[b];
      xh[i] -= s;
    }
  }
  __syncthreads();
  for (int i = lane; i < k; i += 64) u[pts[i]] = xh[i];
  for (int b = lane; b < r; b += 64) u[pts[k + b]] = yc[b];
}

// The same three products for faces of more than 64 points, one workgroup
// per face.  Products with a transposed factor (a dot product per column)
// give each column 16 lanes reading along it; the others give each row a
// lane and deal the columns to the four waves in turn, partial sums through
// LDS in wave order.  Every word of T, L_F̌^{-1} and Y is then read in
// contiguous runs, where the one-wave kernel walks them with a stride of a
// column per lane.  Dynamic LDS: maxF + maxr + NT doubles.

// out[c] (-)= sum_{i in [lo, n)} A(i, c) x[i] for c < ncols, lo = c if tri
// else 0; ends with a barrier.
template <typename T>
__device__ __forceinline__ void wg_col_dots(const T* __restrict__ A, int ld, int n, int ncols,
                                            bool tri, const double* x, double* out, bool sub) {
  const int g = threadIdx.x >> 4, l = threadIdx.x & 15;
  for (int c0 = 0; c0 < ncols; c0 += NT / 16) {
    const int c = c0 + g;
    double s0 = 0.0, s1 = 0.0;
    if (c < ncols) {
      const auto col = as_global(A + (int64_t)ld * c);
      int i = (tri ? c : 0) + l;
      for (; i + 16 < n; i += 32) {
        const double a0 = (double)col[i], a1 = (double)col[i + 16];
        s0 += a0 * x[i];
        s1 += a1 * x[i + 16];
      }
      if (i < n) s0 += (double)col[i] * x[i];
    }
    double v = s0 + s1;
    v += __shfl_xor(v, 8, 16);
    v += __shfl_xor(v, 4, 16);
    v += __shfl_xor(v, 2, 16);
    v += __shfl_xor(v, 1, 16);
    if (c < ncols && l == 0) out[c] = sub ? out[c] - v : v;
  }
  __syncthreads();
}

// out[r] (-)= sum_{c < cend} A(r, c) x[c] for r < nrows, cend = r + 1 if tri
// (the stored upper triangle is in bounds and dropped by selects) else
// ncols; part holds NT doubles; ends with a barrier.
template <typename T>
__device__ __forceinline__ void wg_row_dots(const T* __restrict__ A, int ld, int nrows, int ncols,
                                            bool tri, const double* x, double* out, bool sub,
                                            double* part) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int r0 = 0; r0 < nrows; r0 += 64) {
    const int r = r0 + lane;
    const bool ok = r < nrows;
    const int cend = tri ? min(ncols, r0 + 64) : ncols;
    const auto a = as_global(A + (ok ? r : 0));
    double s0 = 0.0, s1 = 0.0;
    int c = w;
    for (; c + 4 < cend; c += 8) {
      const double a0 = (double)a[(int64_t)ld * c], a1 = (double)a[(int64_t)ld * (c + 4)];
      s0 += (!tri || c <= r) ? a0 * x[c] : 0.0;
      s1 += (!tri || c + 4 <= r) ? a1 * x[c + 4] : 0.0;
    }
    if (c < cend && (!tri || c <= r)) s0 += (double)a[(int64_t)ld * c] * x[c];
    part[threadIdx.x] = s0 + s1;
    __syncthreads();
    if (w == 0 && ok) {
      const double v = part[lane] + part[64 + lane] + part[128 + lane] + part[192 + lane];
      out[r] = sub ? out[r] - v : v;
    }
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_skel_fused_wg(double* u, const int* __restrict__ skpts,
                                                      const SkelDesc* __restrict__ sk,
                                                      const T* __restrict__ skel, int maxF,
                                                      int maxr, int down) {
  extern __shared__ double lds[];
  const SkelDesc d = sk[blockIdx.x];
  const int k = d.k, r = d.r;
  double* xh = lds;
  double* xc = lds + k;
  double* yc = lds + maxF;
  double* part = lds + maxF + maxr;
  const int* pts = skpts + d.pts_off;
  const T* Tm = skel + d.offT;
  const T* Lc = skel + d.offL;
  const T* Y = skel + d.offY;
  for (int i = threadIdx.x; i < k + r; i += NT) lds[i] = u[pts[i]];
  __syncthreads();
  if (!down) {
    wg_col_dots<T>(Tm, k, k, r, false, xh, xc, true);        // x_F̌ -= T^T x_F̂
    wg_row_dots<T>(Lc, r, r, r, true, xc, yc, false, part);  // y = L_F̌^{-1} x_F̌
    wg_col_dots<T>(Y, r, r, k, false, yc, xh, true);         // x_F̂ -= Y^T y
  } else {
    wg_row_dots<T>(Y, r, r, k, false, xh, xc, true, part);   // x_F̌ -= Y x_F̂
    wg_col_dots<T>(Lc, r, r, r, true, xc, yc, false);        // y = L_F̌^{-T} x_F̌
    wg_row_dots<T>(Tm, k, k, r, false, yc, xh, true, part);  // x_F̂ -= T y
  }
  for (int i = threadIdx.x; i < k; i += NT) u[pts[i]] = xh[i];
  for (int b = threadIdx.x; b < r; b += NT) u[pts[k + b]] = yc[b];
}

// ---- block apply (several right-hand sides) --------------------------------
// Vector blocks: column z of u at u + z * N; column z of a scratch segment of
// length ld at base + z * ld (scratch in the factor's precision T).

template <typename T>
__global__ __launch_bounds__(NT) void k_gather_cell_b(const double* __restrict__ u, int64_t N,
                                                      const int* __restrict__ rows,
                                                      const int64_t* __restrict__ crow_off,
                                                      const FrontDesc* __restrict__ fd,
                                                      const int64_t* __restrict__ yoff,
                                                      const int64_t* __restrict__ zoff, T* xi,
                                                      int64_t ldy, T* xs, int64_t ldz,
                                                      int with_s) {
  const int c = blockIdx.y;
  const FrontDesc f = fd[c];
  const int i = blockIdx.x * NT + threadIdx.x;
  const int64_t z = blockIdx.z;
  const int* r = rows + crow_off[c];
  if (i < f.nI) xi[z * ldy + yoff[c] + i] = (T)u[z * N + r[i]];
  else if (with_s && i < f.nR) xs[z * ldz + zoff[c] + i - f.nI] = (T)u[z * N + r[i]];
}

template <typename T>
__global__ __launch_bounds__(NT) void k_scatter_I_b(double* u, int64_t N,
                                                    const int* __restrict__ rows,
                                                    const int64_t* __restrict__ crow_off,
                                                    const FrontDesc* __restrict__ fd,
                                                    const int64_t* __restrict__ yoff,
                                                    const T* __restrict__ y, int64_t ldy) {
  const int c = blockIdx.y;
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= fd[c].nI) return;
  const int64_t z = blockIdx.z;
  u[z * N + rows[crow_off[c] + i]] = (double)y[z * ldy + yoff[c] + i];
}

template <typename T>
__global__ __launch_bounds__(NT) void k_face_sub_b(
    double* u, int64_t N, const int* __restrict__ fpts, const int64_t* __restrict__ fpt_off,
    const int* __restrict__ fN, const int* __restrict__ fcellA, const int* __restrict__ fcellB,
    const int* __restrict__ rb_sa, const int* __restrict__ rb_sb,
    const int64_t* __restrict__ zoff, const T* __restrict__ zv, int64_t ldz) {
  const int f = blockIdx.y;
  const int j = blockIdx.x * NT + threadIdx.x;
  if (j >= fN[f]) return;
  const int64_t z = blockIdx.z;
  const T* zc = zv + z * ldz;
  const double za = (double)zc[zoff[fcellA[f]] + rb_sa[(size_t)f * kRowBlocks] + j];
  const double zb = (double)zc[zoff[fcellB[f]] + rb_sb[(size_t)f * kRowBlocks] + j];
  u[z * N + fpts[fpt_off[f] + j]] -= za + zb;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_skel_move_b(double* u, int64_t N,
                                                    const int* __restrict__ skpts,
                                                    const SkelDesc* __restrict__ sk, T* xh,
                                                    int64_t ldk, T* xc, int64_t ldr, int to_u) {
  const SkelDesc d = sk[blockIdx.y];
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= d.k + d.r) return;
  const int64_t z = blockIdx.z;
  const int64_t p = z * N + skpts[d.pts_off + i];
  T* s = i < d.k ? xh + z * ldk + d.kofs + i : xc + z * ldr + d.rofs + (i - d.k);
  if (to_u) u[p] = (double)*s;
  else *s = (T)u[p];
}

// u[rows[i]] *= sign[i] for every column of u (leading dimension ldu): the
// S = diag(+-1) between the two triangular sweeps of a periodic root.
template <typename T>
__global__ __launch_bounds__(NT) void k_root_sign(double* u, int64_t ldu, int ncol,
                                                  const int* __restrict__ rows,
                                                  const T* __restrict__ sign, int n) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const double sg = (double)sign[i];
  for (int c = 0; c < ncol; ++c) u[(int64_t)c * ldu + rows[i]] *= sg;
}

// ---- forward apply: products with L and L^T from the stored L^{-1} -------
//
// One workgroup per block; thread t owns the rows i = t (mod NT) of the
// block's vector segment, so every entry is read and written by its owner
// only, and the solved entry of each step reaches the others through LDS.

// v <- M^{-1} v = L v (M = L^{-1} lower triangular): forward substitution.
template <typename T>
__global__ __launch_bounds__(NT) void k_trsv_lower(const TrsvDesc* __restrict__ dd, double* v) {
  __shared__ double yj;
  const TrsvDesc d = dd[blockIdx.x];
  const T* M = static_cast<const T*>(d.M);
  double* x = v + d.off;
  const int tid = threadIdx.x;
  for (int j = 0; j < d.n; ++j) {
    if (tid == j % NT) {
      const double t = x[j] / (double)M[j + (int64_t)d.ld * j];
      x[j] = t;
      yj = t;
    }
    __syncthreads();
    const double y = yj;
    const T* col = M + (int64_t)d.ld * j;
    const int i0 = j + 1 + (((tid - (j + 1)) % NT) + NT) % NT;
    for (int i = i0; i < d.n; i += NT) x[i] -= (double)col[i] * y;
    __syncthreads();
  }
}

// v <- M^{-T} v = L^T v: back substitution with the upper triangular M^T.
template <typename T>
__global__ __launch_bounds__(NT) void k_trsv_upper_t(const TrsvDesc* __restrict__ dd, double* v) {
  __shared__ double yj;
  const TrsvDesc d = dd[blockIdx.x];
  const T* M = static_cast<const T*>(d.M);
  double* x = v + d.off;
  const int tid = threadIdx.x;
  for (int j = d.n - 1; j >= 0; --j) {
    if (tid == j % NT) {
      const double t = x[j] / (double)M[j + (int64_t)d.ld * j];
      x[j] = t;
      yj = t;
    }
    __syncthreads();
    const double y = yj;
    for (int i = tid; i < j; i += NT) x[i] -= (double)M[j + (int64_t)d.ld * i] * y;
    __syncthreads();
  }
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

__global__ __launch_bounds__(NT) void k_copy(const double* __restrict__ src, double* dst,
                                             int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    dst[i] = src[i];
}

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
  if (A->opts.bc == HIF_PERIODIC) {  // h = 1/n
    const double h2inv = (double)n * (double)n;
    hipLaunchKernelGGL(k_assemble_periodic, dim3((unsigned)ceil_div(N, NT)), dim3(NT), 0, s, n,
                       h2inv, a, b, A->diag.get(), A->cx.get(), A->cy.get(), A->cz.get(),
                       bad.get());
  } else {  // h = 1/(n+1)
    const double h2inv = (double)(n + 1) * (double)(n + 1);
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)ceil_div(N, NT)), dim3(NT), 0, s, n, h2inv, a,
                       b, A->diag.get(), A->cx.get(), A->cy.get(), A->cz.get(), bad.get());
  }
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
void gemv_launch(bool trans, const GemvDesc* d, int batch, int maxm, int maxn, const double* x,
                 double* y, double alpha, int acc, hipStream_t s, bool aligned = false) {
  if (batch <= 0 || maxm <= 0 || maxn <= 0) return;
  // few row (column) blocks over long rows (columns): the last row block of a
  // large triangle streams the whole matrix width: wide workgroups
  auto wide = [&](int64_t blocks, int len) { return blocks < 2048 && len >= 256; };
  if (!trans && aligned) {
    dim3 g((unsigned)ceil_div(maxm, 16 * Vec16<T>::N), (unsigned)batch);
    if (wide((int64_t)g.x * batch, maxn))
      hipLaunchKernelGGL((k_gemv_nv<T, 64>), g, dim3(1024), 0, s, d, x, y, alpha, acc);
    else
      hipLaunchKernelGGL((k_gemv_nv<T, 16>), g, dim3(NT), 0, s, d, x, y, alpha, acc);
  } else if (trans) {
    dim3 g((unsigned)ceil_div(maxn, kGemvTCols), (unsigned)batch);
    if (wide((int64_t)g.x * batch, maxm))
      hipLaunchKernelGGL((k_gemv_t<T, 64>), g, dim3(1024), 0, s, d, x, y, alpha, acc);
    else
      hipLaunchKernelGGL((k_gemv_t<T, 16>), g, dim3(NT), 0, s, d, x, y, alpha, acc);
  } else {
    dim3 g((unsigned)ceil_div(maxm, 64), (unsigned)batch);
    if (wide((int64_t)g.x * batch, maxn))
      hipLaunchKernelGGL((k_gemv_n<T, 16>), g, dim3(1024), 0, s, d, x, y, alpha, acc);
    else
      hipLaunchKernelGGL((k_gemv_n<T, 4>), g, dim3(NT), 0, s, d, x, y, alpha, acc);
  }
  HIF_LAUNCH_CHECK();
}

template <typename T>
void FactorImpl<T>::prepare(hipStream_t s) {
  if (prepared) return;
  for (auto& l : levels) {
    ymax = std::max(ymax, l.ysum);
    zmax = std::max(zmax, l.zsum);
    kmax = std::max(kmax, l.ksum);
    rmax = std::max(rmax, l.rsum);
  }
  if ((int64_t)ybuf.size() < 2 * ymax) ybuf.alloc(2 * ymax);
  if ((int64_t)zbuf.size() < 2 * zmax) zbuf.alloc(2 * zmax);
  if ((int64_t)sbuf.size() < kmax + 2 * rmax) sbuf.alloc(kmax + 2 * rmax);
  for (auto& lv : levels) {
    if (lv.gv_ready) continue;
    std::vector<GemvDesc> gl, gs, gt, gc, gy;
    for (const FrontDesc& d : lv.hfd) {
      lv.bytes_L += sizeof(T) * 0.5 * d.nI * (d.nI + 1.0) + 24.0 * d.nI;
      lv.bytes_S += sizeof(T) * (double)(d.nR - d.nI) * d.nI + 16.0 * (d.nR - d.nI) + 8.0 * d.nI;
    }
    std::vector<int64_t> yoff(lv.plan->ncell), zoff(lv.plan->ncell);
    int64_t ya = 0, za = 0;
    for (int c = 0; c < lv.plan->ncell; ++c) {
      yoff[c] = ya;
      zoff[c] = za;
      ya += lv.hfd[c].nI;
      za += lv.hfd[c].nR - lv.hfd[c].nI;
    }
    for (int c = 0; c < lv.plan->ncell; ++c) {
      const FrontDesc& d = lv.hfd[c];
      const T* base = static_cast<const T*>(d.ptr);
      gl.push_back({base, d.nI, d.nI, d.ld, 1, yoff[c], yoff[c]});
      if (((uintptr_t)base % 16) != 0 || d.ld % Vec16<T>::N != 0) lv.gv_L_vec = false;
      if (d.nR > d.nI) gs.push_back({base + d.nI, d.nR - d.nI, d.nI, d.ld, 0, zoff[c], yoff[c]});
    }
    for (const SkelDesc& d : lv.hsk) {
      HIF_REQUIRE(d.k >= 0 && d.r > 0 && d.kofs >= 0 && d.rofs >= 0 && d.kofs + d.k <= lv.ksum &&
                      d.rofs + d.r <= lv.rsum && d.k + d.r <= lv.maxF,
                  HIF_EDEVICE, "inconsistent skeleton descriptor");
      const T* sk = lv.skel.get();
      gt.push_back({sk + d.offT, d.k, d.r, std::max(1, d.k), 0, d.kofs, d.rofs});
      gc.push_back({sk + d.offL, d.r, d.r, d.r, 1, d.rofs, d.rofs});
      gy.push_back({sk + d.offY, d.r, d.k, d.r, 0, d.rofs, d.kofs});
      lv.bytes_skel += sizeof(T) * (2.0 * d.k * d.r + 0.5 * d.r * (d.r + 1.0)) + 32.0 * (d.k + d.r);
    }
    lv.gv_L.upload(gl, s);
    lv.gv_S.upload(gs, s);
    lv.gv_T.upload(gt, s);
    lv.gv_Lc.upload(gc, s);
    lv.gv_Y.upload(gy, s);
    lv.gv_nS = (int)gs.size();
    lv.gv_ready = true;
  }
  prepared = true;
}

// Levels of many small fronts take the fused per-front sweeps (one workgroup
// per cell; their vectors must fit in LDS and the factor columns must start
// 16-byte aligned).  HIF_APPLY_FUSED=0 in the environment turns them off.
constexpr int kFuseMinCells = 1024, kFuseMaxI = 2048, kFuseMaxS = 4096;

template <typename T>
bool fused_level(const Level<T>& lv) {
  const char* e = std::getenv("HIF_APPLY_FUSED");
  const bool off = e && e[0] == '0';
  return !off && lv.plan->ncell >= kFuseMinCells && lv.maxI <= kFuseMaxI &&
         lv.maxS <= kFuseMaxS && lv.gv_L_vec;
}

// Skeleton step of a level (same switch).  Levels of many faces take a fused
// kernel: 1 = one wave per face (faces of at most 64 points), 2 = one
// workgroup per face (up to 1024 points).  0 = gather, three batched
// matrix-vector launches, scatter: for levels of few faces, whose
// workgroups would leave most of the chip idle.
constexpr int kSkelFuseMinFaces = 1024, kSkelWaveMaxF = 64, kSkelFuseMaxF = 1024;

template <typename T>
int fused_skel(const Level<T>& lv) {
  const char* e = std::getenv("HIF_APPLY_FUSED");
  if ((e && e[0] == '0') || lv.hsk.size() < (size_t)kSkelFuseMinFaces) return 0;
  if (lv.maxF <= kSkelWaveMaxF) return 1;
  return lv.maxF <= kSkelFuseMaxF ? 2 : 0;
}

template <typename T>
void launch_skel_fused(const Level<T>& lv, int mode, double* u, int down, hipStream_t s) {
  const unsigned ns = (unsigned)lv.hsk.size();
  if (mode == 1) {
    hipLaunchKernelGGL((k_skel_fused<T>), dim3(ns), dim3(64),
                       sizeof(double) * (size_t)(lv.maxF + lv.maxr), s, u, lv.skpts.get(),
                       lv.sk.get(), (const T*)lv.skel.get(), lv.maxF, down);
  } else {
    hipLaunchKernelGGL((k_skel_fused_wg<T>), dim3(ns), dim3(NT),
                       sizeof(double) * (size_t)(lv.maxF + lv.maxr + NT), s, u, lv.skpts.get(),
                       lv.sk.get(), (const T*)lv.skel.get(), lv.maxF, lv.maxr, down);
  }
  HIF_LAUNCH_CHECK();
}

template <typename T>
void FactorImpl<T>::root_sign(double* u, int64_t ldu, int ncol, hipStream_t s) {
  const Level<T>& lv = levels.back();
  if (lv.sign.size() == 0 || lv.plan->ncell == 0) return;
  const int n = lv.hfd[0].nI;
  hipLaunchKernelGGL((k_root_sign<T>), dim3((unsigned)ceil_div(std::max(1, n), NT)), dim3(NT), 0,
                     s, u, ldu, ncol, lv.rows.get(), (const T*)lv.sign.get(), n);
  HIF_LAUNCH_CHECK();
}

template <typename T>
void FactorImpl<T>::apply(const double* f, double* u, hipStream_t s) {
  prepare(s);
  double* sc = sbuf.get() + kmax;
  sweep(f, u, ybuf.get(), ybuf.get() + ymax, zbuf.get(), zbuf.get() + zmax, sbuf.get(), sc,
        sc + rmax, s);
}

// Scratch segments of apply_scratch, each starting on a 256-byte boundary.
inline int64_t seg_round(int64_t n) { return (n + 31) / 32 * 32; }

template <typename T>
int64_t FactorImpl<T>::scratch_doubles() const {
  return 2 * seg_round(ymax) + 2 * seg_round(zmax) + seg_round(kmax) + 2 * seg_round(rmax);
}

template <typename T>
void FactorImpl<T>::apply_scratch(const double* f, double* u, double* scratch, int64_t cap,
                                  hipStream_t s) {
  HIF_REQUIRE(prepared, HIF_EINVAL, "factor has no sweep descriptors");
  const int64_t need = scratch_doubles();
  HIF_REQUIRE(need <= cap, HIF_EINVAL,
              "this factor's apply needs " + std::to_string((need * 8 + (1 << 20) - 1) >> 20) +
                  " MiB of scratch, more than the " + std::to_string((cap * 8) >> 20) +
                  " MiB available without allocation");
  double* p = scratch;
  auto take = [&](int64_t n) {
    double* q = p;
    p += seg_round(n);
    return q;
  };
  double* xi = take(ymax);
  double* yv = take(ymax);
  double* zv = take(zmax);
  double* xsv = take(zmax);
  double* sh = take(kmax);
  double* sc = take(rmax);
  double* sc2 = take(rmax);
  sweep(f, u, xi, yv, zv, xsv, sh, sc, sc2, s);
}

template <typename T>
void FactorImpl<T>::sweep(const double* f, double* u, double* xi, double* yv, double* zv,
                          double* xsv, double* sh, double* sc, double* sc2, hipStream_t s) {
  if (u != f) {  // a kernel, not a copy node, so that the sweep can be captured in a graph
    hipLaunchKernelGGL(k_copy, dim3(grid_for(N)), dim3(NT), 0, s, f, u, N);
    HIF_LAUNCH_CHECK();
  }
  const int nlev = (int)levels.size();
  // W^l^T for l = 0..L (level L: L_Sigma^{-1})
  for (int l = 0; l < nlev; ++l) {
    Level<T>& lv = levels[l];
    prof_level() = l;
    const int nc = lv.plan->ncell;
    if (nc > 0 && fused_level(lv)) {
      ProfScope ps("apply_up_fused", s, 0.0, lv.bytes_L + lv.bytes_S);
      const size_t lds = sizeof(double) * (2 * (size_t)lv.maxI + 4 * NT);
      hipLaunchKernelGGL((k_up_fused<T>), dim3((unsigned)nc), dim3(NT), lds, s, u, lv.rows.get(),
                         lv.crow_off.get(), lv.fd.get(), lv.maxI, lv.zoff.get(), zv);
      HIF_LAUNCH_CHECK();
    } else if (nc > 0) {
      dim3 gI((unsigned)ceil_div(std::max(1, lv.maxI), NT), (unsigned)nc);
      {
        ProfScope ps("apply_up_L", s, 0.0, lv.bytes_L);
        hipLaunchKernelGGL(k_gather_cell, gI, dim3(NT), 0, s, u, lv.rows.get(), lv.crow_off.get(),
                           lv.fd.get(), lv.yoff.get(), lv.zoff.get(), xi, xsv, 0);
        gemv_launch<T>(false, lv.gv_L.get(), nc, lv.maxI, lv.maxI, xi, yv, 1.0, 0, s,
                       lv.gv_L_vec);
      }
      if (lv.gv_nS > 0) {
        ProfScope ps("apply_up_S", s, 0.0, lv.bytes_S);
        gemv_launch<T>(false, lv.gv_S.get(), lv.gv_nS, lv.maxS, lv.maxI, yv, zv, 1.0, 0, s);
      }
      {
        ProfScope ps("apply_scatter", s);
        hipLaunchKernelGGL(k_scatter_I, gI, dim3(NT), 0, s, u, lv.rows.get(), lv.crow_off.get(),
                           lv.fd.get(), lv.yoff.get(), yv);
      }
      HIF_LAUNCH_CHECK();
    }
    if (!lv.plan->root && lv.plan->nface > 0) {
      {
        ProfScope ps("apply_scatter", s);
        dim3 gF((unsigned)ceil_div(std::max(1, lv.maxF), NT), (unsigned)lv.plan->nface);
        hipLaunchKernelGGL(k_face_sub, gF, dim3(NT), 0, s, u, lv.fpts.get(), lv.fpt_off.get(),
                           lv.fN.get(), lv.fcellA.get(), lv.fcellB.get(), lv.rb_sa.get(),
                           lv.rb_sb.get(), lv.zoff.get(), zv);
        HIF_LAUNCH_CHECK();
      }
      const int ns = (int)lv.hsk.size();
      const int fm = ns > 0 ? fused_skel(lv) : 0;
      if (fm) {
        ProfScope ps("apply_skel_fused", s, 0.0, lv.bytes_skel);
        launch_skel_fused(lv, fm, u, 0, s);
      } else if (ns > 0) {
        ProfScope ps("apply_skel", s, 0.0, lv.bytes_skel);
        dim3 gM((unsigned)ceil_div(std::max(1, lv.maxF), NT), (unsigned)ns);
        hipLaunchKernelGGL(k_skel_move, gM, dim3(NT), 0, s, u, lv.skpts.get(), lv.sk.get(), sh, sc,
                           0);
        // x_F̌ -= T^T x_F̂ ; x_F̌ <- L_F̌^{-1} x_F̌ ; x_F̂ -= Y^T x_F̌
        gemv_launch<T>(true, lv.gv_T.get(), ns, lv.maxk, lv.maxr, sh, sc, -1.0, 1, s);
        gemv_launch<T>(false, lv.gv_Lc.get(), ns, lv.maxr, lv.maxr, sc, sc2, 1.0, 0, s);
        gemv_launch<T>(true, lv.gv_Y.get(), ns, lv.maxr, lv.maxk, sc2, sh, -1.0, 1, s);
        hipLaunchKernelGGL(k_skel_move, gM, dim3(NT), 0, s, u, lv.skpts.get(), lv.sk.get(), sh,
                           sc2, 1);
        HIF_LAUNCH_CHECK();
      }
    }
  }
  root_sign(u, N, 1, s);
  // W^l for l = L..0
  for (int l = nlev - 1; l >= 0; --l) {
    Level<T>& lv = levels[l];
    prof_level() = l;
    const int ns = (int)lv.hsk.size();
    const int fm = !lv.plan->root && ns > 0 ? fused_skel(lv) : 0;
    if (fm) {
      ProfScope ps("apply_skel_fused", s, 0.0, lv.bytes_skel);
      launch_skel_fused(lv, fm, u, 1, s);
    } else if (!lv.plan->root && ns > 0) {
      ProfScope ps("apply_skel", s, 0.0, lv.bytes_skel);
      dim3 gM((unsigned)ceil_div(std::max(1, lv.maxF), NT), (unsigned)ns);
      hipLaunchKernelGGL(k_skel_move, gM, dim3(NT), 0, s, u, lv.skpts.get(), lv.sk.get(), sh, sc, 0);
      // x_F̌ -= Y x_F̂ ; x_F̌ <- L_F̌^{-T} x_F̌ ; x_F̂ -= T x_F̌
      gemv_launch<T>(false, lv.gv_Y.get(), ns, lv.maxr, lv.maxk, sh, sc, -1.0, 1, s);
      gemv_launch<T>(true, lv.gv_Lc.get(), ns, lv.maxr, lv.maxr, sc, sc2, 1.0, 0, s);
      gemv_launch<T>(false, lv.gv_T.get(), ns, lv.maxk, lv.maxr, sc2, sh, -1.0, 1, s);
      hipLaunchKernelGGL(k_skel_move, gM, dim3(NT), 0, s, u, lv.skpts.get(), lv.sk.get(), sh, sc2,
                         1);
      HIF_LAUNCH_CHECK();
    }
    const int nc = lv.plan->ncell;
    if (nc == 0) continue;
    if (fused_level(lv)) {
      ProfScope ps("apply_down_fused", s, 0.0, lv.bytes_L + lv.bytes_S);
      const size_t lds = sizeof(double) * (2 * (size_t)lv.maxI + lv.maxS);
      hipLaunchKernelGGL((k_down_fused<T>), dim3((unsigned)nc), dim3(NT), lds, s, u,
                         lv.rows.get(), lv.crow_off.get(), lv.fd.get(), lv.maxI);
      HIF_LAUNCH_CHECK();
      continue;
    }
    const int gmax = std::max(lv.maxI, lv.maxI + lv.maxS);
    dim3 gG((unsigned)ceil_div(std::max(1, gmax), NT), (unsigned)nc);
    dim3 gI((unsigned)ceil_div(std::max(1, lv.maxI), NT), (unsigned)nc);
    {
      ProfScope ps("apply_down_S", s, 0.0, lv.bytes_S);
      hipLaunchKernelGGL(k_gather_cell, gG, dim3(NT), 0, s, u, lv.rows.get(), lv.crow_off.get(),
                         lv.fd.get(), lv.yoff.get(), lv.zoff.get(), xi, xsv, 1);
      // x_I -= L_SI^T x_S
      gemv_launch<T>(true, lv.gv_S.get(), lv.gv_nS, lv.maxS, lv.maxI, xsv, xi, -1.0, 1, s);
    }
    {
      ProfScope ps("apply_down_L", s, 0.0, lv.bytes_L);
      gemv_launch<T>(true, lv.gv_L.get(), nc, lv.maxI, lv.maxI, xi, yv, 1.0, 0, s);
      hipLaunchKernelGGL(k_scatter_I, gI, dim3(NT), 0, s, u, lv.rows.get(), lv.crow_off.get(),
                         lv.fd.get(), lv.yoff.get(), yv);
    }
    HIF_LAUNCH_CHECK();
  }
  prof_level() = -1;
}

// u = F f, F = W^0^{-T} ... W^L^{-T} W^L^{-1} ... W^0^{-1}: every elementary
// step of apply() inverted, in the reverse order.  The inverses multiply by
// L_I, L_F̌ and L_Sigma (and their transposes), which the factor holds as
// explicit inverses: those products are triangular solves with the stored
// blocks (k_trsv_*), the rest are the sweeps' batched matrix-vector products
// with the opposite sign.  One workgroup per triangular block and one step
// per row, so this costs far more than apply(); it is not on the solve path.
template <typename T>
void FactorImpl<T>::apply_forward(const double* f, double* u, hipStream_t s) {
  prepare(s);
  for (auto& lv : levels) {
    if (lv.tr_ready) continue;
    std::vector<TrsvDesc> tc, tf;
    for (int c = 0; c < lv.plan->ncell; ++c)
      if (lv.hfd[c].nI > 0) tc.push_back({lv.hfd[c].ptr, lv.hfd[c].nI, lv.hfd[c].ld, lv.hyoff[c]});
    for (const SkelDesc& d : lv.hsk)
      tf.push_back({(const T*)lv.skel.get() + d.offL, d.r, d.r, d.rofs});
    lv.tr_cells.upload(tc, s);
    lv.tr_faces.upload(tf, s);
    lv.tr_ready = true;
  }
  if (u != f) {
    hipLaunchKernelGGL(k_copy, dim3(grid_for(N)), dim3(NT), 0, s, f, u, N);
    HIF_LAUNCH_CHECK();
  }
  double* xi = ybuf.get();
  double* zv = zbuf.get();
  double* xsv = zbuf.get() + zmax;
  double* sh = sbuf.get();
  double* sc = sbuf.get() + kmax;
  const int nlev = (int)levels.size();
  auto trsv = [&](const Level<T>& lv, bool faces, bool lower, double* v) {
    const size_t cnt = faces ? lv.tr_faces.size() : lv.tr_cells.size();
    if (cnt == 0) return;
    ProfScope ps("forward_trsv", s);
    const TrsvDesc* d = faces ? lv.tr_faces.get() : lv.tr_cells.get();
    if (lower) hipLaunchKernelGGL((k_trsv_lower<T>), dim3((unsigned)cnt), dim3(NT), 0, s, d, v);
    else hipLaunchKernelGGL((k_trsv_upper_t<T>), dim3((unsigned)cnt), dim3(NT), 0, s, d, v);
    HIF_LAUNCH_CHECK();
  };
  auto gather = [&](const Level<T>& lv, int with_s) {
    const int gmax = with_s ? lv.maxI + lv.maxS : lv.maxI;
    dim3 g((unsigned)ceil_div(std::max(1, gmax), NT), (unsigned)lv.plan->ncell);
    hipLaunchKernelGGL(k_gather_cell, g, dim3(NT), 0, s, (const double*)u, lv.rows.get(),
                       lv.crow_off.get(), lv.fd.get(), lv.yoff.get(), lv.zoff.get(), xi, xsv,
                       with_s);
    HIF_LAUNCH_CHECK();
  };
  auto scatter = [&](const Level<T>& lv) {
    dim3 g((unsigned)ceil_div(std::max(1, lv.maxI), NT), (unsigned)lv.plan->ncell);
    hipLaunchKernelGGL(k_scatter_I, g, dim3(NT), 0, s, u, lv.rows.get(), lv.crow_off.get(),
                       lv.fd.get(), lv.yoff.get(), (const double*)xi);
    HIF_LAUNCH_CHECK();
  };
  auto skel_move = [&](const Level<T>& lv, int to_u) {
    dim3 g((unsigned)ceil_div(std::max(1, lv.maxF), NT), (unsigned)lv.hsk.size());
    hipLaunchKernelGGL(k_skel_move, g, dim3(NT), 0, s, u, lv.skpts.get(), lv.sk.get(), sh, sc,
                       to_u);
    HIF_LAUNCH_CHECK();
  };
  // W^l^{-1}, l = 0..L-1: cells (x_I <- L_I^T x_I + L_SI^T x_S), then faces
  // (x_F̂ += T x_F̌; x_F̌ <- L_F̌^T x_F̌ + Y x_F̂)
  for (int l = 0; l + 1 < nlev; ++l) {
    Level<T>& lv = levels[l];
    prof_level() = l;
    const int nc = lv.plan->ncell;
    if (nc > 0) {
      gather(lv, 1);
      trsv(lv, false, false, xi);
      if (lv.gv_nS > 0)
        gemv_launch<T>(true, lv.gv_S.get(), lv.gv_nS, lv.maxS, lv.maxI, xsv, xi, 1.0, 1, s);
      scatter(lv);
    }
    const int ns = (int)lv.hsk.size();
    if (ns > 0) {
      skel_move(lv, 0);
      gemv_launch<T>(false, lv.gv_T.get(), ns, lv.maxk, lv.maxr, sc, sh, 1.0, 1, s);
      trsv(lv, true, false, sc);
      gemv_launch<T>(false, lv.gv_Y.get(), ns, lv.maxr, lv.maxk, sh, sc, 1.0, 1, s);
      skel_move(lv, 1);
    }
  }
  // the root: x <- L_Sigma^T x, then x <- S x (periodic roots), then x <- L_Sigma x
  {
    Level<T>& lv = levels[nlev - 1];
    prof_level() = nlev - 1;
    if (lv.plan->ncell > 0) {
      gather(lv, 0);
      trsv(lv, false, false, xi);
      scatter(lv);
      root_sign(u, N, 1, s);
      gather(lv, 0);
      trsv(lv, false, true, xi);
      scatter(lv);
    }
  }
  // W^l^{-T}, l = L-1..0: faces (x_F̂ += Y^T x_F̌; x_F̌ <- L_F̌ x_F̌ + T^T x_F̂),
  // then cells (x_S += L_SI x_I; x_I <- L_I x_I)
  for (int l = nlev - 2; l >= 0; --l) {
    Level<T>& lv = levels[l];
    prof_level() = l;
    const int ns = (int)lv.hsk.size();
    if (ns > 0) {
      skel_move(lv, 0);
      gemv_launch<T>(true, lv.gv_Y.get(), ns, lv.maxr, lv.maxk, sc, sh, 1.0, 1, s);
      trsv(lv, true, true, sc);
      gemv_launch<T>(true, lv.gv_T.get(), ns, lv.maxk, lv.maxr, sh, sc, 1.0, 1, s);
      skel_move(lv, 1);
    }
    const int nc = lv.plan->ncell;
    if (nc == 0) continue;
    gather(lv, 0);
    if (lv.gv_nS > 0 && lv.plan->nface > 0) {
      gemv_launch<T>(false, lv.gv_S.get(), lv.gv_nS, lv.maxS, lv.maxI, xi, zv, -1.0, 0, s);
      dim3 gF((unsigned)ceil_div(std::max(1, lv.maxF), NT), (unsigned)lv.plan->nface);
      hipLaunchKernelGGL(k_face_sub, gF, dim3(NT), 0, s, u, lv.fpts.get(), lv.fpt_off.get(),
                         lv.fN.get(), lv.fcellA.get(), lv.fcellB.get(), lv.rb_sa.get(),
                         lv.rb_sb.get(), lv.zoff.get(), (const double*)zv);
      HIF_LAUNCH_CHECK();
    }
    trsv(lv, false, true, xi);
    scatter(lv);
  }
  prof_level() = -1;
}

// The sweeps of apply() on a block of nb vectors: every matrix-vector product
// of a level becomes one batched GEMM (MFMA) whose N dimension is the block,
// so each stored factor word is read once per sweep for the whole block.
// Scratch blocks are in the factor's precision T (FP32 for the mixed factor:
// the block apply of that factor rounds like the factor itself).
template <typename T>
double FactorImpl<T>::apply_bytes() const {
  double b = 0.0;
  for (const auto& lv : levels) b += 2.0 * (lv.bytes_L + lv.bytes_S + lv.bytes_skel);
  return b;
}

template <typename T>
void FactorImpl<T>::apply_block(const double* f, double* u, int nrhs, hipStream_t s) {
  prepare(s);
  constexpr int kCols = 32;  // right-hand sides per pass
  if (u != f) {
    hipLaunchKernelGGL(k_copy, dim3(grid_for(N * nrhs)), dim3(NT), 0, s, f, u, N * nrhs);
    HIF_LAUNCH_CHECK();
  }
  const int nb = std::min(nrhs, kCols);
  // segment layout of the scratch: XI, YV (ymax), ZV, XS (zmax), SH (kmax), SC, SC2 (rmax)
  const int64_t seg = 2 * ymax + 2 * zmax + kmax + 2 * rmax;
  if (mbuf_cols < nb) {
    mbuf.alloc(seg * nb);
    mbuf_cols = nb;
  }
  T* XI = mbuf.get();
  T* YV = XI + ymax * nb;
  T* ZV = YV + ymax * nb;
  T* XS = ZV + zmax * nb;
  T* SH = XS + zmax * nb;
  T* SC = SH + kmax * nb;
  T* SC2 = SC + rmax * nb;
  if (bsteps_cols != nb) {
    bsteps.clear();
    bsteps.resize(levels.size());
    for (size_t l = 0; l < levels.size(); ++l) {
      Level<T>& lv = levels[l];
      std::vector<std::vector<GemmDesc>> g(kSteps);
      for (int c = 0; c < lv.plan->ncell; ++c) {
        const FrontDesc& d = lv.hfd[c];
        if (d.nI == 0) continue;
        T* L = static_cast<T*>(d.ptr);
        const int nS = d.nR - d.nI;
        const int64_t yo = lv.hyoff[c], zo = lv.hzoff[c];
        g[kStepL].push_back({L, XI + yo, YV + yo, d.nI, nb, d.nI, d.ld, (int)ymax, (int)ymax});
        g[kStepL2].push_back({L, XI + yo, YV + yo, d.nI, nb, d.nI, d.ld, (int)ymax, (int)ymax});
        if (nS > 0) {
          g[kStepS].push_back({L + d.nI, YV + yo, ZV + zo, nS, nb, d.nI, d.ld, (int)ymax,
                               (int)zmax});
          g[kStepS2].push_back({L + d.nI, XS + zo, XI + yo, d.nI, nb, nS, d.ld, (int)zmax,
                                (int)ymax});
        }
      }
      T* sk = lv.skel.get();
      for (const SkelDesc& d : lv.hsk) {
        T* Tm = sk + d.offT;
        T* Lc = sk + d.offL;
        T* Y = sk + d.offY;
        const int k = d.k, r = d.r, ldt = std::max(1, k);
        const int ldk = (int)kmax, ldr = (int)rmax;
        g[kStepLc1].push_back({Lc, SC + d.rofs, SC2 + d.rofs, r, nb, r, r, ldr, ldr});
        g[kStepLc2].push_back({Lc, SC + d.rofs, SC2 + d.rofs, r, nb, r, r, ldr, ldr});
        if (k == 0) continue;
        g[kStepT1].push_back({Tm, SH + d.kofs, SC + d.rofs, r, nb, k, ldt, ldk, ldr});
        g[kStepY1].push_back({Y, SC2 + d.rofs, SH + d.kofs, k, nb, r, r, ldr, ldk});
        g[kStepY2].push_back({Y, SH + d.kofs, SC + d.rofs, r, nb, k, r, ldk, ldr});
        g[kStepT2].push_back({Tm, SC2 + d.rofs, SH + d.kofs, k, nb, r, ldt, ldr, ldk});
      }
      bsteps[l].resize(kSteps);
      for (int q = 0; q < kSteps; ++q) {
        BlockStep& b = bsteps[l][q];
        b.count = (int)g[q].size();
        for (const GemmDesc& d : g[q]) {
          b.max_m = std::max(b.max_m, d.m);
          b.max_n = std::max(b.max_n, d.n);
          b.flops += 2.0 * d.m * d.n * (double)d.k;
        }
        if (b.count > 0) b.d.upload(g[q], s);
      }
    }
    bsteps_cols = nb;
  }
  // op(A), triangular structure and (alpha, beta) of each step
  struct StepKind {
    int opa, flags;
    T alpha, beta;
  };
  const StepKind kind[kSteps] = {
      {OP_N, GF_A_LOWER | GF_TRI_ZEROS, T(1), T(0)},  // YV = L_I^{-1} XI
      {OP_N, 0, T(1), T(0)},                          // ZV = L_SI YV
      {OP_T, 0, T(-1), T(1)},                         // SC -= T^T SH
      {OP_N, GF_A_LOWER, T(1), T(0)},                 // SC2 = L_F̌^{-1} SC
      {OP_T, 0, T(-1), T(1)},                         // SH -= Y^T SC2
      {OP_N, 0, T(-1), T(1)},                         // SC -= Y SH
      {OP_T, GF_A_UPPER, T(1), T(0)},                 // SC2 = L_F̌^{-T} SC
      {OP_N, 0, T(-1), T(1)},                         // SH -= T SC2
      {OP_T, 0, T(-1), T(1)},                         // XI -= L_SI^T XS
      {OP_T, GF_A_UPPER | GF_TRI_ZEROS, T(1), T(0)},  // YV = L_I^{-T} XI
  };
  auto gemm = [&](size_t l, int q, int nc) {
    const BlockStep& b = bsteps[l][q];
    if (b.count == 0) return;
    gemm_batched<T, T>(kind[q].opa, OP_N, kind[q].flags, b.d.get(), b.count, b.max_m, b.max_n,
                       kind[q].alpha, kind[q].beta, s, "apply_block",
                       b.flops * nc / (double)nb);
  };
  const int nlev = (int)levels.size();
  for (int c0 = 0; c0 < nrhs; c0 += nb) {
    const int nc = std::min(nb, nrhs - c0);
    double* U = u + (int64_t)c0 * N;
    // a short last pass still runs nb columns of GEMM work on scratch; only its
    // nc columns are gathered from and scattered to u
    for (int l = 0; l < nlev; ++l) {
      Level<T>& lv = levels[l];
      prof_level() = l;
      const int ncell = lv.plan->ncell;
      if (ncell > 0) {
        dim3 gI((unsigned)ceil_div(std::max(1, lv.maxI), NT), (unsigned)ncell, (unsigned)nc);
        hipLaunchKernelGGL((k_gather_cell_b<T>), gI, dim3(NT), 0, s, U, N, lv.rows.get(),
                           lv.crow_off.get(), lv.fd.get(), lv.yoff.get(), lv.zoff.get(), XI,
                           ymax, XS, zmax, 0);
        HIF_LAUNCH_CHECK();
        gemm(l, kStepL, nc);
        gemm(l, kStepS, nc);
        hipLaunchKernelGGL((k_scatter_I_b<T>), gI, dim3(NT), 0, s, U, N, lv.rows.get(),
                           lv.crow_off.get(), lv.fd.get(), lv.yoff.get(), (const T*)YV, ymax);
        HIF_LAUNCH_CHECK();
      }
      if (!lv.plan->root && lv.plan->nface > 0) {
        dim3 gF((unsigned)ceil_div(std::max(1, lv.maxF), NT), (unsigned)lv.plan->nface,
                (unsigned)nc);
        hipLaunchKernelGGL((k_face_sub_b<T>), gF, dim3(NT), 0, s, U, N, lv.fpts.get(),
                           lv.fpt_off.get(), lv.fN.get(), lv.fcellA.get(), lv.fcellB.get(),
                           lv.rb_sa.get(), lv.rb_sb.get(), lv.zoff.get(), (const T*)ZV, zmax);
        HIF_LAUNCH_CHECK();
        const int ns = (int)lv.hsk.size();
        if (ns > 0) {
          dim3 gM((unsigned)ceil_div(std::max(1, lv.maxF), NT), (unsigned)ns, (unsigned)nc);
          hipLaunchKernelGGL((k_skel_move_b<T>), gM, dim3(NT), 0, s, U, N, lv.skpts.get(),
                             lv.sk.get(), SH, kmax, SC, rmax, 0);
          HIF_LAUNCH_CHECK();
          gemm(l, kStepT1, nc);
          gemm(l, kStepLc1, nc);
          gemm(l, kStepY1, nc);
          hipLaunchKernelGGL((k_skel_move_b<T>), gM, dim3(NT), 0, s, U, N, lv.skpts.get(),
                             lv.sk.get(), SH, kmax, SC2, rmax, 1);
          HIF_LAUNCH_CHECK();
        }
      }
    }
    root_sign(U, N, nc, s);
    for (int l = nlev - 1; l >= 0; --l) {
      Level<T>& lv = levels[l];
      prof_level() = l;
      const int ns = (int)lv.hsk.size();
      if (!lv.plan->root && ns > 0) {
        dim3 gM((unsigned)ceil_div(std::max(1, lv.maxF), NT), (unsigned)ns, (unsigned)nc);
        hipLaunchKernelGGL((k_skel_move_b<T>), gM, dim3(NT), 0, s, U, N, lv.skpts.get(),
                           lv.sk.get(), SH, kmax, SC, rmax, 0);
        HIF_LAUNCH_CHECK();
        gemm(l, kStepY2, nc);
        gemm(l, kStepLc2, nc);
        gemm(l, kStepT2, nc);
        hipLaunchKernelGGL((k_skel_move_b<T>), gM, dim3(NT), 0, s, U, N, lv.skpts.get(),
                           lv.sk.get(), SH, kmax, SC2, rmax, 1);
        HIF_LAUNCH_CHECK();
      }
      const int ncell = lv.plan->ncell;
      if (ncell == 0) continue;
      const int gmax = std::max(lv.maxI, lv.maxI + lv.maxS);
      dim3 gG((unsigned)ceil_div(std::max(1, gmax), NT), (unsigned)ncell, (unsigned)nc);
      dim3 gI((unsigned)ceil_div(std::max(1, lv.maxI), NT), (unsigned)ncell, (unsigned)nc);
      hipLaunchKernelGGL((k_gather_cell_b<T>), gG, dim3(NT), 0, s, U, N, lv.rows.get(),
                         lv.crow_off.get(), lv.fd.get(), lv.yoff.get(), lv.zoff.get(), XI, ymax,
                         XS, zmax, 1);
      HIF_LAUNCH_CHECK();
      gemm(l, kStepS2, nc);
      gemm(l, kStepL2, nc);
      hipLaunchKernelGGL((k_scatter_I_b<T>), gI, dim3(NT), 0, s, U, N, lv.rows.get(),
                         lv.crow_off.get(), lv.fd.get(), lv.yoff.get(), (const T*)YV, ymax);
      HIF_LAUNCH_CHECK();
    }
  }
  prof_level() = -1;
}

template void FactorImpl<double>::prepare(hipStream_t);
template void FactorImpl<float>::prepare(hipStream_t);
template void FactorImpl<double>::apply(const double*, double*, hipStream_t);
template void FactorImpl<float>::apply(const double*, double*, hipStream_t);
template void FactorImpl<double>::apply_forward(const double*, double*, hipStream_t);
template void FactorImpl<float>::apply_forward(const double*, double*, hipStream_t);
template void FactorImpl<double>::apply_scratch(const double*, double*, double*, int64_t,
                                                hipStream_t);
template void FactorImpl<float>::apply_scratch(const double*, double*, double*, int64_t,
                                               hipStream_t);
template int64_t FactorImpl<double>::scratch_doubles() const;
template int64_t FactorImpl<float>::scratch_doubles() const;

// Scratch of apply_noalloc: every GPU the library runs on holds its own copy
// of this array until the process ends.  Host code never passes the array's
// name to a kernel (on the host it is a stand-in, not a device address): the
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

namespace {

double* scratch_on_current_device() {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double* ptr[kMaxDevices] = {};
  int dev = 0;
  HIF_HIP(hipGetDevice(&dev));
  HIF_REQUIRE(dev >= 0 && dev < kMaxDevices, HIF_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    HIF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    HIF_REQUIRE(p != nullptr, HIF_EDEVICE, "no device address for the scratch array");
    ptr[dev] = static_cast<double*>(p);
  }
  return ptr[dev];
}

}  // namespace

void apply_noalloc(hif_factor_s* F, const double* f, double* u, hipStream_t s) {
  double* p = scratch_on_current_device();
  F->impl->apply_scratch(f, u, p, kNoAllocScratchBytes / (int64_t)sizeof(double), s);
}
template void FactorImpl<double>::apply_block(const double*, double*, int, hipStream_t);
template double FactorImpl<double>::apply_bytes() const;
template double FactorImpl<float>::apply_bytes() const;
template void FactorImpl<float>::apply_block(const double*, double*, int, hipStream_t);

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

void device_dot(const double* a, const double* b, const double* c, int64_t N, double* out,
                hipStream_t s) {
  Dot d;
  d.run(a, b, c, N, out, s);
}

// A preconditioner application captured once into a HIP graph (on a private
// stream: the caller's may be the legacy stream, which cannot be captured) and
// replayed on the caller's stream, which replaces its ~10 launches per level by
// one graph launch.  The captured work is kernels only (no memset or copy
// nodes).  HIF_APPLY_GRAPH=0 in the environment (read at every use) launches
// the sweeps directly instead; a capture the runtime refuses falls back to the
// same direct launches.
struct ApplyGraph {
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
  hipStream_t cs = nullptr;
  bool failed = false;
  double bytes = 0.0;  // algorithmic bytes of one application (profiler)

  explicit ApplyGraph(double b) : bytes(b) {}
  ~ApplyGraph() {
    if (x) (void)hipGraphExecDestroy(x);
    if (g) (void)hipGraphDestroy(g);
    if (cs) (void)hipStreamDestroy(cs);
  }
  ApplyGraph(const ApplyGraph&) = delete;
  ApplyGraph& operator=(const ApplyGraph&) = delete;
  static bool env_off() {
    const char* e = std::getenv("HIF_APPLY_GRAPH");
    return e && e[0] == '0';
  }
  template <typename Fn>
  void run(Fn&& fn, hipStream_t s) {
    if (env_off() || failed) {
      fn(s);
      return;
    }
    if (!x) capture(fn);
    if (!x) {
      fn(s);
      return;
    }
    ProfScope ps("apply_graph", s, 0.0, bytes);
    HIF_HIP(hipGraphLaunch(x, s));
  }

 private:
  template <typename Fn>
  void capture(Fn& fn) {
    if (!cs) HIF_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    Profiler& P = profiler();
    const bool was = P.on;
    if (was) P.on = false;  // no event records inside the graph
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      try {
        fn(cs);
      } catch (...) {
        hipGraph_t t = nullptr;
        (void)hipStreamEndCapture(cs, &t);
        if (t) (void)hipGraphDestroy(t);
        if (was) P.on = true;
        throw;
      }
      e = hipStreamEndCapture(cs, &g);
      if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    }
    if (was) P.on = true;
    if (e != hipSuccess) {
      (void)hipGetLastError();
      if (x) (void)hipGraphExecDestroy(x);
      if (g) (void)hipGraphDestroy(g);
      x = nullptr;
      g = nullptr;
      failed = true;
    }
  }
};

// Workspace of the single-vector PCG kept with the factor: its residual and
// preconditioned residual vectors and the graph of F^{-1} applied from one to
// the other.  The first solve with a factor launches the sweeps directly (a
// capture costs about as much as it saves over one solve); the second captures
// the graph, and it and every later solve replay it.
struct PcgCache {
  DevBuf<double> r, z;
  std::unique_ptr<ApplyGraph> graph;
  int solves = 0;
};

void pcg_solve(const hif_problem_s* A, hif_factor_s* F, const double* f, double* u, double tol,
               int maxit, hif_pcg_info* info, hipStream_t s) {
  const int64_t N = A->N;
  const Stencil st = A->stencil();
  if (!F->impl->pcg) F->impl->pcg = std::make_shared<PcgCache>();
  PcgCache& C = *F->impl->pcg;
  if ((int64_t)C.r.size() != N) {
    C.r.alloc(N);
    C.z.alloc(N);
    C.graph.reset();
  }
  if (!C.graph) C.graph = std::make_unique<ApplyGraph>(F->impl->apply_bytes());
  DevBuf<double>& r = C.r;
  DevBuf<double>& z = C.z;
  DevBuf<double> rold(N), p(N), q(N), sc(8);
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
  ApplyGraph& ag = *C.graph;
  const bool replay = ++C.solves >= 2;
  auto precondition = [&](hipStream_t q) { F->impl->apply(r.get(), z.get(), q); };
  auto apply_z = [&]() {
    if (replay) ag.run(precondition, s);
    else precondition(s);
  };
  apply_z();
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
    apply_z();
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

// nrhs > 1: independent PCG runs, one per column, sharing each preconditioner
// application (apply_block).  Vector operations and inner products run per
// live column; a column leaves when its true residual reaches tol or on
// breakdown, and the others go on.
void pcg_solve_block(const hif_problem_s* A, hif_factor_s* F, const double* f, double* u, int nrhs,
                     double tol, int maxit, hif_pcg_info* info, hipStream_t s) {
  const int64_t N = A->N;
  const int64_t NB = N * nrhs;
  const Stencil st = A->stencil();
  DevBuf<double> r(NB), rold(NB), z(NB), p(NB), q(NB), sc(8 * (size_t)nrhs);
  Dot dot;
  std::vector<double> h(8 * (size_t)nrhs);
  auto fetch = [&]() {
    HIF_HIP(hipMemcpyAsync(h.data(), sc.get(), sizeof(double) * h.size(), hipMemcpyDeviceToHost,
                           s));
    HIF_HIP(hipStreamSynchronize(s));
  };
  auto at = [&](double* b, int j) { return b + (int64_t)j * N; };
  auto cat = [&](const double* b, int j) { return b + (int64_t)j * N; };
  const unsigned g = grid_for(N);
  HIF_HIP(hipMemsetAsync(u, 0, sizeof(double) * NB, s));
  HIF_HIP(hipMemcpyAsync(r.get(), f, sizeof(double) * NB, hipMemcpyDeviceToDevice, s));
  for (int j = 0; j < nrhs; ++j) dot.run(cat(f, j), cat(f, j), nullptr, N, sc.get() + 8 * j + 5, s);
  fetch();
  std::vector<double> fn(nrhs);
  std::vector<char> live(nrhs, 0);
  int nlive = 0;
  for (int j = 0; j < nrhs; ++j) {
    fn[j] = std::sqrt(h[8 * j + 5]);
    info[j].iters = 0;
    info[j].converged = fn[j] == 0.0;
    info[j].relres = fn[j] == 0.0 ? 0.0 : 1.0;
    live[j] = fn[j] > 0.0;
    nlive += live[j];
  }
  if (nlive == 0) return;
  F->impl->apply_block(r.get(), z.get(), nrhs, s);
  HIF_HIP(hipMemcpyAsync(p.get(), z.get(), sizeof(double) * NB, hipMemcpyDeviceToDevice, s));
  for (int j = 0; j < nrhs; ++j)
    if (live[j]) dot.run(at(r.get(), j), at(z.get(), j), nullptr, N, sc.get() + 8 * j, s);
  for (int it = 1; it <= maxit && nlive > 0; ++it) {
    for (int j = 0; j < nrhs; ++j) {
      if (!live[j]) continue;
      double* scj = sc.get() + 8 * j;
      stencil_matvec(st, at(p.get(), j), at(q.get(), j), s);
      dot.run(at(p.get(), j), at(q.get(), j), nullptr, N, scj + 1, s);
      hipLaunchKernelGGL(k_cg_step, dim3(g), dim3(NT), 0, s, at(u, j), at(r.get(), j),
                         at(rold.get(), j), (const double*)at(p.get(), j),
                         (const double*)at(q.get(), j), (const double*)scj, N);
      dot.run(at(r.get(), j), at(r.get(), j), nullptr, N, scj + 4, s);
    }
    fetch();
    std::vector<int> check;
    for (int j = 0; j < nrhs; ++j) {
      if (!live[j]) continue;
      info[j].iters = it;
      if (!(h[8 * j + 1] > 0.0) || !std::isfinite(h[8 * j + 4])) {  // breakdown
        live[j] = 0;
        --nlive;
        continue;
      }
      if (std::sqrt(h[8 * j + 4]) <= tol * fn[j]) check.push_back(j);
    }
    if (!check.empty()) {
      for (int j : check) {
        stencil_matvec(st, at(u, j), at(q.get(), j), s);
        hipLaunchKernelGGL(k_residual, dim3(g), dim3(NT), 0, s, cat(f, j), at(q.get(), j), N);
        dot.run(at(q.get(), j), at(q.get(), j), nullptr, N, sc.get() + 8 * j + 6, s);
      }
      fetch();
      for (int j : check) {
        info[j].relres = std::sqrt(h[8 * j + 6]) / fn[j];
        if (info[j].relres <= tol) {
          info[j].converged = 1;
          live[j] = 0;
          --nlive;
        } else {
          HIF_HIP(hipMemcpyAsync(at(r.get(), j), at(q.get(), j), sizeof(double) * N,
                                 hipMemcpyDeviceToDevice, s));
        }
      }
    }
    if (nlive == 0) break;
    F->impl->apply_block(r.get(), z.get(), nrhs, s);
    for (int j = 0; j < nrhs; ++j) {
      if (!live[j]) continue;
      double* scj = sc.get() + 8 * j;
      dot.run(at(z.get(), j), at(r.get(), j), at(rold.get(), j), N, scj + 2, s);
      dot.run(at(r.get(), j), at(z.get(), j), nullptr, N, scj + 3, s);
      hipLaunchKernelGGL(k_cg_dir, dim3(g), dim3(NT), 0, s, at(p.get(), j),
                         (const double*)at(z.get(), j), (const double*)scj, N);
      hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, s, scj, 0, 3);
      HIF_LAUNCH_CHECK();
    }
  }
  std::vector<int> rest;
  for (int j = 0; j < nrhs; ++j)
    if (!info[j].converged && fn[j] > 0.0) rest.push_back(j);
  if (rest.empty()) return;
  for (int j : rest) {
    stencil_matvec(st, at(u, j), at(q.get(), j), s);
    hipLaunchKernelGGL(k_residual, dim3(g), dim3(NT), 0, s, cat(f, j), at(q.get(), j), N);
    dot.run(at(q.get(), j), at(q.get(), j), nullptr, N, sc.get() + 8 * j + 6, s);
  }
  fetch();
  for (int j : rest) {
    info[j].relres = std::sqrt(h[8 * j + 6]) / fn[j];
    info[j].converged = info[j].relres <= tol;
  }
}

void pcg_solve_batched(int count, hif_problem_s* const* A, hif_factor_s* const* F,
                       const double* const* f, double* const* u, double tol, int maxit,
                       hif_pcg_info* info, hipStream_t s) {
  // Each solve is latency-bound on small problems (a host round trip per
  // iteration); a few solves in flight on separate streams keep the GPU busy
  // (8 measured best for the 48-problem workload; 4 and 16 were slower).
  constexpr int kWorkers = 8;
  // profiling records are not thread safe: a profiled run solves in turn
  const int workers = profiler().on ? 1 : std::min(count, kWorkers);
  if (workers <= 1) {
    for (int i = 0; i < count; ++i) pcg_solve(A[i], F[i], f[i], u[i], tol, maxit, &info[i], s);
    return;
  }
  struct Streams {
    std::vector<hipStream_t> st;
    std::vector<hipEvent_t> ev;
    ~Streams() {
      for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
      for (hipStream_t q : st)
        if (q) (void)hipStreamDestroy(q);
    }
  } R;
  R.st.assign(workers, nullptr);
  R.ev.assign(workers + 1, nullptr);
  for (auto& e : R.ev) HIF_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  HIF_HIP(hipEventRecord(R.ev[workers], s));  // the inputs are ready on s
  for (int w = 0; w < workers; ++w) {
    HIF_HIP(hipStreamCreateWithFlags(&R.st[w], hipStreamNonBlocking));
    HIF_HIP(hipStreamWaitEvent(R.st[w], R.ev[workers], 0));
  }
  std::atomic<int> next{0};
  std::mutex emu;
  std::exception_ptr first;
  auto work = [&](int w) {
    try {
      StreamScope scope(R.st[w]);
      for (;;) {
        const int i = next.fetch_add(1);
        if (i >= count) break;
        pcg_solve(A[i], F[i], f[i], u[i], tol, maxit, &info[i], R.st[w]);
      }
    } catch (...) {
      std::lock_guard<std::mutex> lock(emu);
      if (!first) first = std::current_exception();
      next.store(count);
    }
  };
  std::vector<std::thread> th;
  for (int w = 0; w < workers; ++w) th.emplace_back(work, w);
  for (auto& t : th) t.join();
  for (int w = 0; w < workers; ++w) {  // s waits for every worker stream
    HIF_HIP(hipEventRecord(R.ev[w], R.st[w]));
    HIF_HIP(hipStreamWaitEvent(s, R.ev[w], 0));
  }
  if (first) std::rethrow_exception(first);
}

}  // namespace hif
