// Level executor of the HIF factorization (paper, Section 2.4 level loop,
// Section 3.2 face snapshot).  One level = gather fronts, factor them,
// form the Schur updates, assemble face panels, interpolative decomposition
// of every face, skeleton update; a host round trip reads the ranks back.
#include <chrono>
#include <cmath>
#include <climits>
#include <cstring>

#include "hif_impl.hpp"
#include "prof.hpp"

namespace hif {
namespace {

constexpr int NT = 256;

// A^l entry lookup.  At level 0, A^0 is the stencil.  At level l >= 1 the
// entry between two points of level-(l-1) faces lives in the panel of the
// column point's face (row block of the row point's face), and every entry
// that involves an edge or corner point is still the stencil value.
template <typename T>
struct Src {
  Stencil st;
  int has_prev;
  const int2* pmap;  // per grid point: (level-(l-1) face, index in it) or (-1, 0)
  const T* panels;
  const int64_t* poff;
  const int* pld;
  const int* prb_face;
  const int* prb_off;
};

// The part of an A^l lookup that depends only on the column point q, hoisted
// out of the loops over rows: q's previous-level face, the column of that
// face's panel, and the panel's row-block faces with their row offsets.
template <typename T>
struct ColLookup {
  int q, fq;
  int qx, qy, qz;  // grid coordinates of q (periodic stencil lookups)
  const T* pcol;
  int gface[kRowBlocks], goff[kRowBlocks];
};

template <typename T>
__device__ __forceinline__ ColLookup<T> col_lookup(const Src<T>& s, int q) {
  ColLookup<T> c;
  c.q = q;
  const int2 mq = s.has_prev ? s.pmap[q] : make_int2(-1, 0);
  c.fq = mq.x;
  const int n = s.st.n;
  c.qx = q % n;
  c.qy = (q / n) % n;
  c.qz = q / (n * n);
  c.pcol = nullptr;
#pragma unroll
  for (int t = 0; t < kRowBlocks; ++t) {
    c.gface[t] = -1;
    c.goff[t] = 0;
  }
  if (c.fq >= 0) {
    c.pcol = s.panels + s.poff[c.fq] + (int64_t)s.pld[c.fq] * mq.y;
#pragma unroll
    for (int t = 0; t < kRowBlocks; ++t) {
      c.gface[t] = s.prb_face[kRowBlocks * c.fq + t];
      c.goff[t] = s.prb_off[kRowBlocks * c.fq + t];
    }
  }
  return c;
}

// A^l(p, q).  At level 0, A^0 is the stencil.  At level l >= 1 the entry
// between two points of level-(l-1) faces lives in the panel of the column
// point's face (zero if the row point's face is not one of its row blocks),
// and every entry that involves an edge or corner point is still the stencil
// value.  mp is p's entry of the lookup map, read by the caller from an
// array laid out like its rows (contiguous, not a gather by p).
template <typename T>
__device__ __forceinline__ T row_lookup(const Src<T>& s, const ColLookup<T>& c, int p, int2 mp) {
  if (c.fq >= 0) {
    const int fp = mp.x;
    if (fp >= 0) {
      int off = -1;
#pragma unroll
      for (int t = 0; t < kRowBlocks; ++t)
        if (c.gface[t] == fp) off = c.goff[t];
      return off >= 0 ? c.pcol[off + mp.y] : T(0);
    }
  }
  const int q = c.q;
  if (p == q) return (T)s.st.diag[p];
  const int n = s.st.n;
  if (s.st.periodic) {
    // neighbours along one dimension, the index wrapping around (n >= 4)
    const int dx = c.qx - p % n, dy = c.qy - (p / n) % n, dz = c.qz - p / (n * n);
    const double* cd = dy == 0 && dz == 0 ? s.st.cx
                       : (dx == 0 && dz == 0 ? s.st.cy : (dx == 0 && dy == 0 ? s.st.cz : nullptr));
    const int dd = cd == s.st.cx ? dx : (cd == s.st.cy ? dy : dz);
    if (cd == nullptr) return T(0);
    if (dd == 1 || dd == -(n - 1)) return (T)(-cd[p]);  // q is p's + neighbour
    if (dd == -1 || dd == n - 1) return (T)(-cd[q]);    // p is q's + neighbour
    return T(0);
  }
  const int dl = q - p;
  const int lo = p < q ? p : q;
  if (dl == 1 || dl == -1) return (T)(-s.st.cx[lo]);
  if (dl == n || dl == -n) return (T)(-s.st.cy[lo]);
  if (dl == n * n || dl == -n * n) return (T)(-s.st.cz[lo]);
  return T(0);
}

// The gathers give each wave one column (four columns per workgroup): the
// column's lookup state is then wave-uniform (scalar registers) and columns
// of a few dozen rows still keep most lanes busy.
constexpr int kGatherCols = NT / 64;
constexpr int kGatherUnroll = 4;  // rows per lane whose loads are issued together

__device__ __forceinline__ int wave_column(int block) {
  return block * kGatherCols + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// Front of cell c, column j: A_II(i, j) for i >= j into Phi, and zeros above
// the diagonal (the factorization keeps them, so the inverse's products need
// no triangular masks).
// Lookup-map entry i of an array laid out like the rows (none at level 0).
__device__ __forceinline__ int2 map_at(int has_prev, const int2* __restrict__ m, int64_t i) {
  return has_prev ? m[i] : make_int2(-1, 0);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_gather_front(Src<T> s, const int* __restrict__ rows,
                                                     const int2* __restrict__ rmap,
                                                     const int64_t* __restrict__ crow_off,
                                                     const FrontDesc* __restrict__ fd) {
  const int c = blockIdx.y;
  const FrontDesc f = fd[c];
  const int j = wave_column(blockIdx.x);
  if (j >= f.nI) return;
  const int lane = threadIdx.x & 63;
  const int64_t o = crow_off[c];
  const int* r = rows + o;
  const ColLookup<T> cl = col_lookup(s, r[j]);
  T* col = static_cast<T*>(f.ptr) + (int64_t)f.ld * j;
  for (int i = lane; i < j; i += 64) col[i] = T(0);
  // kGatherUnroll rows per lane at a time: all lookups' loads before any store
  for (int i0 = j + lane; i0 < f.nI; i0 += 64 * kGatherUnroll) {
    int p[kGatherUnroll];
    int2 mp[kGatherUnroll];
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u) {
      const int i = min(i0 + 64 * u, f.nI - 1);
      p[u] = r[i];
      mp[u] = map_at(s.has_prev, rmap, o + i);
    }
    T v[kGatherUnroll];
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u) v[u] = row_lookup(s, cl, p[u], mp[u]);
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u)
      if (i0 + 64 * u < f.nI) col[i0 + 64 * u] = v[u];
  }
}

// A_SI of cell c, column j (the j-th interior point): nS x nI, leading dimension nS.
template <typename T>
__global__ __launch_bounds__(NT) void k_gather_front_SI(Src<T> s, const int* __restrict__ rows,
                                                        const int2* __restrict__ rmap,
                                                        const int64_t* __restrict__ crow_off,
                                                        const FrontDesc* __restrict__ fd, T* asi,
                                                        const int64_t* __restrict__ aoff) {
  const int c = blockIdx.y;
  const FrontDesc f = fd[c];
  const int j = wave_column(blockIdx.x);
  if (j >= f.nI) return;
  const int nS = f.nR - f.nI;
  const int lane = threadIdx.x & 63;
  const int64_t o = crow_off[c];
  const int* r = rows + o;
  const ColLookup<T> cl = col_lookup(s, r[j]);
  T* col = asi + aoff[c] + (int64_t)((nS + 3) / 4 * 4) * j;  // leading dimension pad_ld(nS)
  for (int i0 = lane; i0 < nS; i0 += 64 * kGatherUnroll) {
    int p[kGatherUnroll];
    int2 mp[kGatherUnroll];
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u) {
      const int i = min(i0 + 64 * u, nS - 1);
      p[u] = r[f.nI + i];
      mp[u] = map_at(s.has_prev, rmap, o + f.nI + i);
    }
    T v[kGatherUnroll];
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u) v[u] = row_lookup(s, cl, p[u], mp[u]);
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u)
      if (i0 + 64 * u < nS) col[i0 + 64 * u] = v[u];
  }
}

// L_SI = A_SI L_I^{-T} at the leaf level, where A_SI is the stencil itself: a
// shell point couples to at most its six grid neighbours, so row i of L_SI is
// the sum, over the neighbours j of shell point i inside the cell, of
// A(p_i, q_j) times column j of L_I^{-1} (as a row): the nonzero terms of the
// dense product (a single one for every shell point of a face), summed in
// direction order.  Two kernels: the neighbour lists of the shell points,
// then L_SI by 64 x 64 tiles through LDS (columns of L_I^{-1} read
// contiguously, columns of L_SI written contiguously).
constexpr int kLeafIntMax = 1024;
constexpr int kMaxGridZ = 65535;  // largest z dimension of a launch grid

// Neighbour lists, one workgroup per cell: the cell's interior points
// (sorted) are staged in LDS and each (shell point, direction) finds its
// neighbour there by binary search.  Shell row i of cell c (global row
// zoff[c] + i) gets nb_c = the count and, in direction order, nb_j (interior
// index) and nb_a (coefficient) in its six slots; a row with no neighbour
// keeps column 0 with a zero coefficient, so that its first term is always
// a plain load.
template <typename T>
__global__ __launch_bounds__(NT) void k_leaf_nbr(Src<T> s, const int* __restrict__ rows,
                                                 const int64_t* __restrict__ crow_off,
                                                 const FrontDesc* __restrict__ fd,
                                                 const int64_t* __restrict__ zoff, int* nb_c,
                                                 int* nb_j, T* nb_a) {
  __shared__ int ri[kLeafIntMax];
  const FrontDesc f = fd[blockIdx.x];
  const int nI = f.nI, nS = f.nR - f.nI;
  if (nS <= 0 || nI <= 0) return;
  const int* r = rows + crow_off[blockIdx.x];
  const int64_t z0 = zoff[blockIdx.x];
  const int n = s.st.n;
  for (int t = threadIdx.x; t < nI; t += NT) ri[t] = r[t];
  __syncthreads();
  for (int i = threadIdx.x; i < nS; i += NT) {
    const int p = r[nI + i];
    const int pc[3] = {p % n, (p / n) % n, p / (n * n)};
    int c = 0;
    int* jj = nb_j + 6 * (z0 + i);
    T* aa = nb_a + 6 * (z0 + i);
    for (int d = 0; d < 6; ++d) {
      int qc[3] = {pc[0], pc[1], pc[2]};
      qc[d >> 1] += (d & 1) ? 1 : -1;
      if (!s.st.periodic && (qc[d >> 1] < 0 || qc[d >> 1] >= n)) continue;
      qc[d >> 1] = (qc[d >> 1] + n) % n;
      const int q = (qc[2] * n + qc[1]) * n + qc[0];
      int lo = 0, hi = nI;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ri[mid] < q) lo = mid + 1;
        else hi = mid;
      }
      if (lo < nI && ri[lo] == q) {
        jj[c] = lo;
        aa[c] = row_lookup(s, col_lookup(s, q), p, make_int2(-1, 0));
        ++c;
      }
    }
    if (c == 0) {
      jj[0] = 0;
      aa[0] = T(0);
    }
    nb_c[z0 + i] = c;
  }
}

// One 64 x 64 tile (shell rows i0.., interior columns t0..) of one cell's
// L_SI: lanes read a column of L_I^{-1} along t, the tile is turned in LDS,
// and lanes write a column of L_SI along i.
template <typename T>
__global__ __launch_bounds__(NT) void k_lsi_leaf(const FrontDesc* __restrict__ fd,
                                                 const int64_t* __restrict__ zoff,
                                                 const int* __restrict__ nb_c,
                                                 const int* __restrict__ nb_j,
                                                 const T* __restrict__ nb_a) {
  __shared__ T tile[64][65];  // [i][t]
  const FrontDesc f = fd[blockIdx.z];
  const int nI = f.nI, nS = f.nR - f.nI;
  const int t0 = blockIdx.x * 64, i0 = blockIdx.y * 64;
  if (t0 >= nI || i0 >= nS) return;
  const int64_t z0 = zoff[blockIdx.z];
  const T* Linv = static_cast<const T*>(f.ptr);
  T* C = static_cast<T*>(f.ptr) + nI;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int t = min(t0 + tx, nI - 1);
  // all list loads, then all column loads, so that their latencies overlap
  int64_t g[16];
  int jn[16], cn[16];
  T a[16], v[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int i = min(i0 + ty + 4 * k, nS - 1);
    g[k] = 6 * (z0 + i);
    jn[k] = nb_j[g[k]];
    a[k] = nb_a[g[k]];
    cn[k] = nb_c[z0 + i];
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = a[k] * Linv[t + (int64_t)f.ld * jn[k]];
#pragma unroll
  for (int k = 0; k < 16; ++k)  // shell points with more than one neighbour (edges)
    for (int e = 1; e < cn[k]; ++e) v[k] += nb_a[g[k] + e] * Linv[t + (int64_t)f.ld * nb_j[g[k] + e]];
#pragma unroll
  for (int k = 0; k < 16; ++k) tile[ty + 4 * k][tx] = v[k];
  __syncthreads();
  const int i = i0 + tx;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int tt = t0 + ty + 4 * k;
    if (i < nS && tt < nI) C[i + (int64_t)f.ld * tt] = tile[tx][ty + 4 * k];
  }
}

// Panel of face f, column j: Ã^l(rows, F_j) = A^l(rows, F_j) + U_A + U_B, the
// Schur updates of the two neighbouring cells added in a fixed order.  The
// panel's row blocks (the face and the other faces of both cells) are
// contiguous in the column, so the rows run as one range: lane t < 11 reads
// the descriptors of block t, which every lane then holds in scalar
// registers, and each lane takes kGatherUnroll rows at a time, finding a
// row's block by comparison, with all their loads issued before any store.
template <typename T>
__global__ __launch_bounds__(NT) void k_gather_panel(
    Src<T> s, const int* __restrict__ fpts, const int2* __restrict__ fmap,
    const int64_t* __restrict__ fpt_off,
    const int* __restrict__ fN, const int* __restrict__ rb_face, const int* __restrict__ rb_off,
    const int* __restrict__ rb_sa, const int* __restrict__ rb_sb, const int* __restrict__ fcellA,
    const int* __restrict__ fcellB, const T* __restrict__ U, const int64_t* __restrict__ uoff,
    const int* __restrict__ uld, T* panels, const int64_t* __restrict__ poff,
    const int* __restrict__ pld) {
  const int f = blockIdx.y;
  const int j = wave_column(blockIdx.x);
  if (j >= fN[f]) return;
  const int lane = threadIdx.x & 63;
  const ColLookup<T> cl = col_lookup(s, fpts[fpt_off[f] + j]);
  const int A = fcellA[f], B = fcellB[f];
  const size_t base = (size_t)f * kRowBlocks;
  const int colA = rb_sa[base] + j, colB = rb_sb[base] + j;
  const T* UA = U + uoff[A];
  const T* UB = U + uoff[B];
  const int ldA = uld[A], ldB = uld[B];
  T* col = panels + poff[f] + (int64_t)pld[f] * j;
  // block descriptors: lane t holds block t (used blocks form a prefix)
  int lg = -1, lro = 0, lsa = -1, lsb = -1, lgo = 0, lng = 0;
  if (lane < kRowBlocks) {
    lg = rb_face[base + lane];
    if (lg >= 0) {
      lro = rb_off[base + lane];
      lsa = rb_sa[base + lane];
      lsb = rb_sb[base + lane];
      lgo = (int)fpt_off[lg];
      lng = fN[lg];
    }
  }
  int ro[kRowBlocks], go[kRowBlocks], sa[kRowBlocks], sb[kRowBlocks];
  int nb = 0;
#pragma unroll
  for (int t = 0; t < kRowBlocks; ++t) {
    ro[t] = __builtin_amdgcn_readlane(lro, t);
    go[t] = __builtin_amdgcn_readlane(lgo, t);
    sa[t] = __builtin_amdgcn_readlane(lsa, t);
    sb[t] = __builtin_amdgcn_readlane(lsb, t);
    nb += __builtin_amdgcn_readlane(lg, t) >= 0 ? 1 : 0;
  }
  if (nb == 0) return;
  int nrow = 0;  // rows of the panel: the end of the last block
#pragma unroll
  for (int t = 0; t < kRowBlocks; ++t)
    if (t == nb - 1) nrow = ro[t] + __builtin_amdgcn_readlane(lng, t);
  for (int r0 = lane; r0 < nrow; r0 += 64 * kGatherUnroll) {
    int p[kGatherUnroll];
    int2 mp[kGatherUnroll];
    T ua[kGatherUnroll], ub[kGatherUnroll];
    bool ha[kGatherUnroll], hb[kGatherUnroll];
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u) {
      const int r = min(r0 + 64 * u, nrow - 1);
      int bro = ro[0], bgo = go[0], bsa = sa[0], bsb = sb[0];
#pragma unroll
      for (int t = 1; t < kRowBlocks; ++t)
        if (t < nb && r >= ro[t]) {
          bro = ro[t];
          bgo = go[t];
          bsa = sa[t];
          bsb = sb[t];
        }
      const int i = r - bro;
      p[u] = fpts[bgo + i];
      mp[u] = map_at(s.has_prev, fmap, (int64_t)bgo + i);
      ha[u] = bsa >= 0;
      hb[u] = bsb >= 0;
      ua[u] = ha[u] ? UA[(bsa + i) + (int64_t)ldA * colA] : T(0);
      ub[u] = hb[u] ? UB[(bsb + i) + (int64_t)ldB * colB] : T(0);
    }
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u) {
      T v = row_lookup(s, cl, p[u], mp[u]);
      if (ha[u]) v += ua[u];
      if (hb[u]) v += ub[u];
      if (r0 + 64 * u < nrow) col[r0 + 64 * u] = v;
    }
  }
}

__device__ __forceinline__ int nsep(int x, int y, int z, int w, int periodic) {
  return (x % w == 0 && (periodic || x != 0)) + (y % w == 0 && (periodic || y != 0)) +
         (z % w == 0 && (periodic || z != 0));
}

// Rows of edge points in Ã^l(R, F) hold one stencil coupling each, so they add
// only squares to the Gram diagonal.
__global__ __launch_bounds__(NT) void k_gram_edges(Stencil st, int w, const int* __restrict__ fpts,
                                                   const int64_t* __restrict__ fpt_off,
                                                   const int* __restrict__ fN, double* G,
                                                   const int64_t* __restrict__ goff,
                                                   const int* __restrict__ gld) {
  const int f = blockIdx.y;
  const int j = blockIdx.x * NT + threadIdx.x;
  if (j >= fN[f]) return;
  const int n = st.n, per = st.periodic;
  const int q = fpts[fpt_off[f] + j];
  const int c3[3] = {q % n, (q / n) % n, q / (n * n)};
  const double* cd[3] = {st.cx, st.cy, st.cz};
  double add = 0.0;
  for (int d = 0; d < 3; ++d) {
    for (int dir = -1; dir <= 1; dir += 2) {
      int nb[3] = {c3[0], c3[1], c3[2]};
      nb[d] += dir;
      if (nb[d] < 0 || nb[d] >= n) {
        if (!per) continue;  // the Dirichlet ghost
        nb[d] = (nb[d] + n) % n;
      }
      if (nsep(nb[0], nb[1], nb[2], w, per) != 2) continue;
      const int r = nb[0] + n * nb[1] + n * n * nb[2];
      const double v = dir > 0 ? cd[d][q] : cd[d][r];  // the coupling lives at the lower point
      add += v * v;
    }
  }
  G[goff[f] + j + (int64_t)gld[f] * j] += add;
}

// Split the pivoted Cholesky factor into L11 (k x k, pivot order) and L21
// (r x k) for T = L11^{-T} L21^T.
__global__ __launch_bounds__(NT) void k_split_L(const double* __restrict__ Lp,
                                                const int64_t* __restrict__ goff,
                                                const int* __restrict__ gld,
                                                const int* __restrict__ perm,
                                                const int64_t* __restrict__ poff,
                                                const SkelDesc* __restrict__ sk, double* L11,
                                                const int64_t* __restrict__ o11, double* L21,
                                                const int64_t* __restrict__ o21,
                                                const int* __restrict__ fN) {
  const SkelDesc d = sk[blockIdx.y];
  const int t = blockIdx.x;
  if (t >= d.k) return;
  const int f = d.face;
  const double* L = Lp + goff[f] + (int64_t)gld[f] * t;
  const int* pm = perm + poff[f];
  const int nF = fN[f];
  for (int i = threadIdx.x; i < nF; i += NT) {
    const double v = L[pm[i]];
    if (i < d.k) L11[o11[blockIdx.y] + i + (int64_t)d.k * t] = v;
    else L21[o21[blockIdx.y] + (i - d.k) + (int64_t)d.r * t] = v;
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_convert(const double* __restrict__ src, T* dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    dst[i] = (T)src[i];
}

// A_F̂F̂, A_F̂F̌, A_F̌F̌ from the face's own block of its panel, in pivot order.
template <typename T>
__global__ __launch_bounds__(NT) void k_skel_gather(const T* __restrict__ panels,
                                                    const int64_t* __restrict__ poff,
                                                    const int* __restrict__ pld,
                                                    const int* __restrict__ perm,
                                                    const int64_t* __restrict__ permoff,
                                                    const SkelDesc* __restrict__ sk, T* Ahh,
                                                    const int64_t* __restrict__ ohh, T* Ahc,
                                                    const int64_t* __restrict__ ohc, T* skel) {
  const SkelDesc d = sk[blockIdx.y];
  const int j = blockIdx.x;
  const int nF = d.k + d.r;
  if (j >= nF) return;
  const int f = d.face;
  const int* pm = perm + permoff[f];
  const T* P = panels + poff[f] + (int64_t)pld[f] * pm[j];
  for (int i = threadIdx.x; i < nF; i += NT) {
    const T v = P[pm[i]];
    if (j < d.k) {
      if (i < d.k) Ahh[ohh[blockIdx.y] + i + (int64_t)d.k * j] = v;
    } else if (i < d.k) {
      Ahc[ohc[blockIdx.y] + i + (int64_t)d.k * (j - d.k)] = v;
    } else {
      skel[d.offL + (i - d.k) + (int64_t)d.r * (j - d.k)] = v;
    }
  }
}

// B_F̂F̂ back into the face's own panel block at the skeleton positions.
template <typename T>
__global__ __launch_bounds__(NT) void k_skel_writeback(T* panels, const int64_t* __restrict__ poff,
                                                       const int* __restrict__ pld,
                                                       const int* __restrict__ perm,
                                                       const int64_t* __restrict__ permoff,
                                                       const SkelDesc* __restrict__ sk,
                                                       const T* __restrict__ Ahh,
                                                       const int64_t* __restrict__ ohh) {
  const SkelDesc d = sk[blockIdx.y];
  const int j = blockIdx.x;
  if (j >= d.k) return;
  const int f = d.face;
  const int* pm = perm + permoff[f];
  T* P = panels + poff[f] + (int64_t)pld[f] * pm[j];
  for (int i = threadIdx.x; i < d.k; i += NT) P[pm[i]] = Ahh[ohh[blockIdx.y] + i + (int64_t)d.k * j];
}

__global__ __launch_bounds__(NT) void k_perm_points(const int* __restrict__ fpts,
                                                    const int* __restrict__ perm,
                                                    const int64_t* __restrict__ fpt_off,
                                                    const int* __restrict__ fN, int* skpts) {
  const int f = blockIdx.y;
  const int j = blockIdx.x * NT + threadIdx.x;
  if (j >= fN[f]) return;
  const int64_t o = fpt_off[f];
  skpts[o + j] = fpts[o + perm[o + j]];
}

// Lookup map for the next level: (face, index within the face) of every face
// point, (-1, 0) for every other point (the fill runs first).
__global__ __launch_bounds__(NT) void k_fill_map(int2* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    p[i] = make_int2(-1, 0);
}

__global__ __launch_bounds__(NT) void k_face_map(const int* __restrict__ fpts,
                                                 const int64_t* __restrict__ fpt_off,
                                                 const int* __restrict__ fN, int2* pmap) {
  const int f = blockIdx.y;
  const int j = blockIdx.x * NT + threadIdx.x;
  if (j >= fN[f]) return;
  const int p = fpts[fpt_off[f] + j];
  pmap[p] = make_int2(f, j);
}

// out[t] = pmap[idx[t]]: the map entries of a row list, laid out like it, so
// that the gathers read them contiguously instead of gathering by point.
__global__ __launch_bounds__(NT) void k_map_rows(const int* __restrict__ idx, int64_t n,
                                                 const int2* __restrict__ pmap, int2* out) {
  for (int64_t t = blockIdx.x * (int64_t)NT + threadIdx.x; t < n; t += (int64_t)gridDim.x * NT)
    out[t] = pmap[idx[t]];
}

template <typename T>
Src<T> make_src(const hif_problem_s* A, const Level<T>* prev, const int2* pmap) {
  Src<T> s;
  s.st = A->stencil();
  s.has_prev = prev != nullptr;
  s.pmap = pmap;
  s.panels = prev ? prev->panel.get() : nullptr;
  s.poff = prev ? prev->panel_off.get() : nullptr;
  s.pld = prev ? prev->panel_ld.get() : nullptr;
  s.prb_face = prev ? prev->rb_face.get() : nullptr;
  s.prb_off = prev ? prev->rb_off.get() : nullptr;
  return s;
}

template <typename V>
DevBuf<V> to_dev(const std::vector<V>& h, hipStream_t s) {
  DevBuf<V> d;
  d.upload(h, s);
  return d;
}

template <typename TIn, typename TC>
void run_gemms(const char* name, int opa, int opb, int flags, const std::vector<GemmDesc>& h0,
               TC alpha, TC beta, hipStream_t s, int cls = GC_GENERIC) {
  if (h0.empty()) return;
  // only the large products of the cell fronts are reordered (reordering the
  // many small products of the face steps measured slower)
  const std::vector<GemmDesc> h =
      cls == GC_SYRK || cls == GC_LSI ? balance_xcds(h0, flags) : h0;
  int mm = 0, mn = 0;
  double fl = 0.0;
  for (auto& d : h) {
    mm = std::max(mm, d.m);
    mn = std::max(mn, d.n);
    fl += gemm_flops(d, flags);
  }
  // leading dimensions on the 16-byte grid let the batch take the DMA-fed tile
  constexpr int V = 16 / (int)sizeof(TIn);
  bool ld16 = true;
  for (auto& d : h)  // (A^T B: the two operands also share their 16-byte offset)
    ld16 = ld16 && d.lda % V == 0 && d.ldb % V == 0 &&
           (opa != OP_T || (uintptr_t)d.A % 16 == (uintptr_t)d.B % 16);
  DevBuf<GemmDesc> d;
  d.upload(h, s);
  gemm_batched<TIn, TC>(opa, opb, flags, d.get(), (int)h.size(), mm, mn, alpha, beta, s, name, fl,
                        cls, ld16);
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

namespace {

// One problem of a batch while the batch is factored level by level.
template <typename T>
struct Job {
  const hif_problem_s* A = nullptr;
  hif_options o{};
  hif_factor_s* F = nullptr;
  std::unique_ptr<FactorImpl<T>> impl;
  int L = 0;
  int64_t N = 0;
  double flops = 0.0;
  // 0 for points the ID has left out so far (the candidates of a level are
  // separator points of the level below, so interior points never need it)
  std::vector<uint8_t> active;
  // (face, index in it) of every level-(l-1) face point, for the A^l lookup,
  // and that map laid out like the level's front rows and face points
  DevBuf<int2> d_pmap, rmap, fmap;
  // temporaries of the current level
  DevBuf<T> ASI, U, Ahh, Ahc;
  DevBuf<int64_t> d_xoff, d_o11, d_o21, d_ohh, d_ohc;
  DevBuf<double> L11, L21, Td;
  std::vector<int64_t> uoff, poff, o11, o21, ohh, ohc;
  std::vector<int> uld, pld, hperm;
  int64_t face0 = 0;  // first face of this problem in the level's joint ID arrays
  int64_t pt0 = 0;    // first face point of this problem in the joint pivot order
  int64_t ssz = 0;    // skeleton arena size of the level
  std::vector<double> flops_mark;  // flops counted before each level
};

// The problem and the cell (or skeleton) that a front id of a joint launch names.
struct Owner {
  int job, index;
};

}  // namespace

// Factors a batch of problems together: level l of every problem (counted from
// the leaves) is one set of launches, so fronts and faces of all problems share
// each batched kernel, and the host waits once per level for all of them.
template <typename T>
void build_factors(const std::vector<BuildRequest>& req, hipStream_t s) {
  const int nj = (int)req.size();
  HIF_REQUIRE(nj >= 1, HIF_EINVAL, "no problems to factor");
  const double t_begin = now_s();
  const int64_t mem0 = mem_stats().live;
  mem_stats().peak = mem0;
  const double eps = req[0].o.eps;
  for (int j = 0; j < nj; ++j) {
    HIF_REQUIRE(req[j].o.eps == eps, HIF_EINVAL, "the problems of a batch must share eps");
    for (int i = 0; i < j; ++i)
      HIF_REQUIRE(req[i].A != req[j].A || req[i].o.leaf == req[j].o.leaf, HIF_EINVAL,
                  "a problem listed twice in a batch needs the same leaf size");
  }
  std::vector<Job<T>> jobs(nj);
  int maxL = 0;
  for (int j = 0; j < nj; ++j) {
    Job<T>& J = jobs[j];
    J.A = req[j].A;
    J.o = req[j].o;
    J.F = req[j].F;
    const int n = J.A->n;
    J.L = levels_for(n, J.o.leaf);
    HIF_REQUIRE(J.L >= 0 && J.L <= HIF_MAX_LEVELS - 1, HIF_EINVAL, "n must be leaf * 2^L");
    J.N = J.A->N;
    J.impl = std::make_unique<FactorImpl<T>>();
    J.impl->n = n;
    J.impl->L = J.L;
    J.impl->N = J.N;
    J.impl->levels.resize(J.L + 1);
    hif_stats& st = J.F->stats;
    std::memset(&st, 0, sizeof(st));
    st.levels = J.L;
    st.precision = J.o.precision;
    st.n_dof = J.N;
    const hif_problem_s* A = J.A;
    if (A->geom_leaf != J.o.leaf) {
      A->geom = plan_geometry(n, J.o.leaf, A->opts.bc == HIF_PERIODIC);
      A->plan0 = std::make_shared<const LevelPlan>(
          plan_level(A->geom[0], std::vector<uint8_t>((size_t)J.N, 1)));
      A->dev0 = {};
      A->geom_leaf = J.o.leaf;
    }
    J.active.assign((size_t)J.N, 1);
    if (J.L > 0) {
      J.d_pmap.alloc(J.N);
    }
    maxL = std::max(maxL, J.L);
  }
  auto of_problem = [&](int j) {
    return nj > 1 ? " of problem " + std::to_string(j) : std::string();
  };
  // failure flags: per level, the interior Cholesky (front id) and the Cholesky
  // of B_F̌F̌ (skeleton id); checked whenever the host synchronizes anyway
  const int kNoErr = INT_MAX;
  std::vector<int> h_err(2 * (maxL + 1), kNoErr);
  DevBuf<int> d_err = to_dev(h_err, s);
  std::vector<std::vector<Owner>> own_front(maxL + 1), own_skel(maxL + 1);
  auto check_errors = [&]() {
    HIF_HIP(hipMemcpyAsync(h_err.data(), d_err.get(), sizeof(int) * h_err.size(),
                           hipMemcpyDeviceToHost, s));
    HIF_HIP(hipStreamSynchronize(s));
    for (int l = 0; l <= maxL; ++l) {
      if (h_err[2 * l] != kNoErr) {
        const Owner w = own_front[l].at(h_err[2 * l]);
        const bool ldl = l == jobs[w.job].L && jobs[w.job].A->opts.bc == HIF_PERIODIC;
        throw Error(HIF_ENOTSPD, (ldl ? std::string("zero pivot in the LDL^T of the root")
                                      : "non-positive pivot in the interior Cholesky at level " +
                                            std::to_string(l) + ", cell " +
                                            std::to_string(w.index)) +
                                     of_problem(w.job));
      }
      if (h_err[2 * l + 1] != kNoErr) {
        const Owner w = own_skel[l].at(h_err[2 * l + 1]);
        throw Error(HIF_ENOTSPD,
                    "non-positive pivot in B_F̌F̌ at level " + std::to_string(l) + ", face " +
                        std::to_string(jobs[w.job].impl->levels[l].hsk[w.index].face) +
                        of_problem(w.job));
      }
    }
  };
  // device-side level timing
  struct Events {
    std::vector<hipEvent_t> e;
    ~Events() {
      for (hipEvent_t x : e) (void)hipEventDestroy(x);
    }
  } ev;
  ev.e.resize(maxL + 2, nullptr);
  for (auto& x : ev.e) HIF_HIP(hipEventCreate(&x));

  for (int level = 0; level <= maxL; ++level) {
    HIF_HIP(hipEventRecord(ev.e[level], s));
    prof_level() = level;
    for (auto& J : jobs) J.flops_mark.push_back(J.flops);
    std::vector<int> here, below;  // problems with this level; those for which it is not the root
    for (int j = 0; j < nj; ++j) {
      if (level <= jobs[j].L) here.push_back(j);
      if (level < jobs[j].L) below.push_back(j);
    }

    // ---- fronts: gather, partial Cholesky + inverse (Section 2.2) -------
    std::vector<FrontDesc> tops;
    std::vector<std::pair<int, FrontDesc>> ldl_roots;  // periodic roots: signed LDL^T
    std::vector<GemmDesc> g_lsi;
    std::vector<int> leaf_jobs;  // problems whose leaf L_SI comes from the stencil
    // Lower bandwidth of the leaf fronts: a leaf interior is a box of the grid
    // in lexicographic order, whose largest neighbour offset (and so the band
    // of A_II and of its Cholesky factor) is the size of one z-plane of it.
    int leaf_band = 0;
    for (int j : here) {
      Job<T>& J = jobs[j];
      const hif_problem_s* A = J.A;
      hif_stats& st = J.F->stats;
      Level<T>& lev = J.impl->levels[level];
      Level<T>* prev = level > 0 ? &J.impl->levels[level - 1] : nullptr;
      lev.plan = level == 0 ? A->plan0
                            : std::make_shared<const LevelPlan>(plan_level(A->geom[level], J.active));
      const LevelPlan& P = *lev.plan;
      const Src<T> src = make_src<T>(A, prev, J.d_pmap.get());
      // index arrays of the plan; level 0's are uploaded once per problem
      auto arr = [&](auto& cached, const auto& host) {
        if (level > 0) return dev_arr(host, s);
        if (!cached.buf) cached = dev_arr(host, s);
        return cached;
      };
      lev.rows = arr(A->dev0.rows, P.rows);
      lev.crow_off = arr(A->dev0.crow_off, P.crow_off);
      lev.hfd.resize(P.ncell);
      int64_t off = 0;
      std::vector<int64_t> foff(P.ncell), yoff(P.ncell), zoff(P.ncell);
      for (int c = 0; c < P.ncell; ++c) {
        FrontDesc& d = lev.hfd[c];
        foff[c] = off;
        d.nI = P.cI[c];
        d.nR = P.cI[c] + P.cS[c];
        d.ld = pad_ld(d.nR);
        d.id = c;
        off += (int64_t)d.ld * d.nI;
        yoff[c] = lev.ysum;
        zoff[c] = lev.zsum;
        lev.ysum += d.nI;
        lev.zsum += P.cS[c];
        lev.maxI = std::max(lev.maxI, d.nI);
        lev.maxS = std::max(lev.maxS, P.cS[c]);
        const double nI = d.nI, nS = P.cS[c];
        J.flops += nI * nI * nI / 3.0 + nS * nI * nI + nI * nI * nI / 3.0 + nS * nS * nI;
        st.max_front[level] = std::max<int64_t>(st.max_front[level], d.nR);
      }
      lev.front.alloc(off);
      for (int c = 0; c < P.ncell; ++c) lev.hfd[c].ptr = lev.front.get() + foff[c];
      lev.fd = to_dev(lev.hfd, s);
      lev.yoff = to_dev(yoff, s);
      lev.zoff = to_dev(zoff, s);
      lev.hyoff = std::move(yoff);
      lev.hzoff = std::move(zoff);
      st.cells[level] = P.ncell;
      st.eliminated[level] = lev.ysum;
      if (P.ncell == 0) continue;
      // A_SI (nS x nI per cell) until L_SI = A_SI L_I^{-T} is formed; at the
      // leaf level L_SI comes from the stencil directly (k_lsi_leaf)
      const bool leaf_lsi = level == 0 && lev.maxS > 0 && lev.maxI <= kLeafIntMax;
      if (leaf_lsi) leaf_jobs.push_back(j);
      std::vector<int64_t> xoff(P.ncell);
      int64_t xsz = 0;
      for (int c = 0; c < P.ncell && !leaf_lsi; ++c) {
        xoff[c] = xsz;
        xsz += (int64_t)P.cI[c] * pad_ld(P.cS[c]);
      }
      if (!leaf_lsi) {
        J.ASI.alloc(std::max<int64_t>(xsz, 1));
        J.d_xoff = to_dev(xoff, s);
      }
      {
        // algorithmic bytes: the blocks written, and above the leaf level one
        // source entry (a previous panel's) read per entry
        double gbytes = 0.0;
        for (int c = 0; c < P.ncell; ++c)
          gbytes += (double)P.cI[c] * (P.cI[c] + (leaf_lsi ? 0 : P.cS[c])) * sizeof(T);
        ProfScope ps("gather_front", s, 0.0, prev ? 2.0 * gbytes : gbytes);
        if (prev) {
          const int64_t nr = (int64_t)P.rows.size();
          J.rmap.alloc(std::max<int64_t>(nr, 1));
          hipLaunchKernelGGL(k_map_rows, dim3((unsigned)std::min<int64_t>(ceil_div(nr, NT), 8192)),
                             dim3(NT), 0, s, lev.rows.get(), nr, (const int2*)J.d_pmap.get(),
                             J.rmap.get());
          HIF_LAUNCH_CHECK();
        }
        dim3 g((unsigned)ceil_div(std::max(1, lev.maxI), kGatherCols), (unsigned)P.ncell);
        hipLaunchKernelGGL((k_gather_front<T>), g, dim3(NT), 0, s, src, lev.rows.get(),
                           (const int2*)J.rmap.get(), lev.crow_off.get(), lev.fd.get());
        HIF_LAUNCH_CHECK();
        if (lev.maxS > 0 && !leaf_lsi) {
          hipLaunchKernelGGL((k_gather_front_SI<T>), g, dim3(NT), 0, s, src, lev.rows.get(),
                             (const int2*)J.rmap.get(), lev.crow_off.get(), lev.fd.get(),
                             J.ASI.get(), J.d_xoff.get());
          HIF_LAUNCH_CHECK();
        }
        J.rmap.release();
      }
      // interior Cholesky and in-place inverse on the top nI x nI block; the
      // root of a periodic problem keeps the LDL^T of the paper (Section 2.2):
      // compression can leave it indefinite along the near-constant mode
      const bool signed_root = level == J.L && A->opts.bc == HIF_PERIODIC;
      if (level == 0) {
        const int64_t n2 = (int64_t)A->opts.n * A->opts.n;
        for (int c = 0; c < P.ncell; ++c) {
          const int* r = P.rows.data() + P.crow_off[c];
          int w = 0;
          while (w < P.cI[c] && r[w] / n2 == r[0] / n2) ++w;
          leaf_band = std::max(leaf_band, w);
        }
      }
      for (int c = 0; c < P.ncell; ++c) {
        FrontDesc t = lev.hfd[c];
        t.nR = t.nI;
        t.id = (int)own_front[level].size();
        own_front[level].push_back({j, c});
        if (signed_root && t.nI > 0) ldl_roots.push_back({j, t});
        else tops.push_back(t);
      }
      // L_SI = A_SI L_I^{-T} into the front below L_I^{-1} (L_I^{-T} is upper)
      for (int c = 0; c < P.ncell && !leaf_lsi; ++c) {
        if (P.cS[c] == 0) continue;
        const FrontDesc& d = lev.hfd[c];
        T* base = static_cast<T*>(d.ptr);
        g_lsi.push_back({J.ASI.get() + xoff[c], base, base + d.nI, P.cS[c], d.nI, d.nI,
                         pad_ld(P.cS[c]), d.ld, d.ld});
      }
    }
    if (!tops.empty()) {
      DevBuf<FrontDesc> d_top = to_dev(tops, s);
      front_factor<T>(d_top.get(), tops, d_err.get() + 2 * level, s, true,
                      level == 0 ? kSmallFrontLeaf : kSmallFrontUpper, level == 0 ? leaf_band : 0);
    }
    for (auto& jr : ldl_roots) {
      Level<T>& lev = jobs[jr.first].impl->levels[level];
      lev.sign.alloc(jr.second.nI);
      DevBuf<FrontDesc> d_root = to_dev(std::vector<FrontDesc>{jr.second}, s);
      root_ldl<T>(jr.second, d_root.get(), lev.sign.get(), d_err.get() + 2 * level, s);
    }
    for (int j : leaf_jobs) {
      Job<T>& J = jobs[j];
      const Level<T>& lev = J.impl->levels[level];
      const int nc = lev.plan->ncell;
      ProfScope ps("lsi_leaf", s);
      DevBuf<int> nb_c(std::max<int64_t>(lev.zsum, 1)), nb_j(6 * std::max<int64_t>(lev.zsum, 1));
      DevBuf<T> nb_a(6 * std::max<int64_t>(lev.zsum, 1));
      hipLaunchKernelGGL((k_leaf_nbr<T>), dim3((unsigned)nc), dim3(NT), 0, s,
                         make_src<T>(J.A, nullptr, nullptr), lev.rows.get(), lev.crow_off.get(),
                         lev.fd.get(), lev.zoff.get(), nb_c.get(), nb_j.get(), nb_a.get());
      HIF_LAUNCH_CHECK();
      for (int c0 = 0; c0 < nc; c0 += kMaxGridZ) {
        dim3 g((unsigned)ceil_div(lev.maxI, 64), (unsigned)ceil_div(lev.maxS, 64),
               (unsigned)std::min(kMaxGridZ, nc - c0));
        hipLaunchKernelGGL((k_lsi_leaf<T>), g, dim3(NT), 0, s, lev.fd.get() + c0,
                           lev.zoff.get() + c0, nb_c.get(), nb_j.get(), nb_a.get());
        HIF_LAUNCH_CHECK();
      }
    }
    run_gemms<T, T>("gemm_lsi", OP_N, OP_T, GF_B_UPPER | GF_TRI_ZEROS, g_lsi, T(1), T(0), s,
                    GC_LSI);
    for (int j : here) {
      jobs[j].ASI.release();
      jobs[j].d_xoff.release();
      if (level == jobs[j].L) {  // the root: a dense factor, no faces
        Level<T>& lev = jobs[j].impl->levels[level];
        jobs[j].F->stats.root_size = lev.ysum;
        if (level > 0) jobs[j].impl->levels[level - 1].panel.release();
      }
    }
    if (below.empty()) continue;

    // ---- Schur updates U_c = -L_SI L_SI^T (both triangles) ---------------
    {
      std::vector<GemmDesc> gd;
      for (int j : below) {
        Job<T>& J = jobs[j];
        Level<T>& lev = J.impl->levels[level];
        const LevelPlan& P = *lev.plan;
        J.uoff.assign(P.ncell, 0);
        J.uld.assign(P.ncell, 1);
        int64_t usz = 0;
        for (int c = 0; c < P.ncell; ++c) {
          J.uoff[c] = usz;
          J.uld[c] = std::max(1, P.cS[c]);
          usz += (int64_t)J.uld[c] * P.cS[c];
        }
        J.U.alloc(std::max<int64_t>(usz, 1));
        for (int c = 0; c < P.ncell; ++c) {
          if (P.cS[c] == 0) continue;
          const FrontDesc& d = lev.hfd[c];
          const T* LSI = static_cast<const T*>(d.ptr) + d.nI;
          gd.push_back(
              {LSI, LSI, J.U.get() + J.uoff[c], P.cS[c], P.cS[c], d.nI, d.ld, d.ld, J.uld[c]});
        }
      }
      // both triangles of U, so that the panel gather reads columns only
      run_gemms<T, T>("gemm_syrk", OP_N, OP_T, GF_C_LOWER | GF_C_MIRROR, gd, T(-1), T(0), s,
                      GC_SYRK);
    }

    // ---- face panels Ã^l([F; R-faces], F) --------------------------------
    int64_t nface_all = 0, npt_all = 0;
    for (int j : below) {
      Job<T>& J = jobs[j];
      const hif_problem_s* A = J.A;
      hif_stats& st = J.F->stats;
      Level<T>& lev = J.impl->levels[level];
      Level<T>* prev = level > 0 ? &J.impl->levels[level - 1] : nullptr;
      const LevelPlan& P = *lev.plan;
      const Src<T> src = make_src<T>(A, prev, J.d_pmap.get());
      auto arr = [&](auto& cached, const auto& host) {
        if (level > 0) return dev_arr(host, s);
        if (!cached.buf) cached = dev_arr(host, s);
        return cached;
      };
      J.poff.assign(P.nface, 0);
      J.pld.assign(P.nface, 1);
      int64_t psz = 0;
      for (int f = 0; f < P.nface; ++f) {
        J.poff[f] = psz;
        J.pld[f] = pad_ld(P.prow[f]);
        psz += (int64_t)J.pld[f] * P.fN[f];
        lev.maxF = std::max(lev.maxF, P.fN[f]);
      }
      lev.fpts = arr(A->dev0.fpts, P.fpts);
      lev.fpt_off = arr(A->dev0.fpt_off, P.fpt_off);
      lev.fN = arr(A->dev0.fN, P.fN);
      lev.fcellA = arr(A->dev0.fcellA, P.fcellA);
      lev.fcellB = arr(A->dev0.fcellB, P.fcellB);
      lev.rb_face = arr(A->dev0.rb_face, P.rb_face);
      lev.rb_off = arr(A->dev0.rb_off, P.rb_off);
      lev.rb_sa = arr(A->dev0.rb_sa, P.rb_sa);
      lev.rb_sb = arr(A->dev0.rb_sb, P.rb_sb);
      lev.panel_off = to_dev(J.poff, s);
      lev.panel_ld = to_dev(J.pld, s);
      lev.panel.alloc(std::max<int64_t>(psz, 1));
      st.faces[level] = P.nface;
      if (P.nface > 0) {
        DevBuf<int64_t> d_uoff = to_dev(J.uoff, s);
        DevBuf<int> d_uld = to_dev(J.uld, s);
        // algorithmic bytes: the panels written, the Schur blocks U read once,
        // and above the leaf level one previous-panel entry per panel entry
        double ubytes = 0.0;
        for (int c = 0; c < P.ncell; ++c) ubytes += (double)J.uld[c] * P.cS[c] * sizeof(T);
        const double pbytes = (double)psz * sizeof(T);
        ProfScope ps("gather_panel", s, 0.0, pbytes + ubytes + (prev ? pbytes : 0.0));
        if (prev) {
          const int64_t nf = (int64_t)P.fpts.size();
          J.fmap.alloc(std::max<int64_t>(nf, 1));
          hipLaunchKernelGGL(k_map_rows, dim3((unsigned)std::min<int64_t>(ceil_div(nf, NT), 8192)),
                             dim3(NT), 0, s, lev.fpts.get(), nf, (const int2*)J.d_pmap.get(),
                             J.fmap.get());
          HIF_LAUNCH_CHECK();
        }
        dim3 g((unsigned)ceil_div(std::max(1, lev.maxF), kGatherCols), (unsigned)P.nface);
        hipLaunchKernelGGL((k_gather_panel<T>), g, dim3(NT), 0, s, src, lev.fpts.get(),
                           (const int2*)J.fmap.get(), lev.fpt_off.get(), lev.fN.get(),
                           lev.rb_face.get(), lev.rb_off.get(), lev.rb_sa.get(), lev.rb_sb.get(), lev.fcellA.get(), lev.fcellB.get(),
                           J.U.get(), d_uoff.get(), d_uld.get(), lev.panel.get(),
                           lev.panel_off.get(), lev.panel_ld.get());
        HIF_LAUNCH_CHECK();
      }
      J.U.release();
      J.fmap.release();
      if (prev) prev->panel.release();  // A^l has been read for the last time
      for (int f = 0; f < P.nface; ++f) st.face_dofs[level] += P.fN[f];
      lev.hk.assign(P.nface, 0);
      J.hperm.assign(P.fpts.size(), 0);
      J.face0 = nface_all;
      J.pt0 = npt_all;
      nface_all += P.nface;
      npt_all += (int64_t)P.fpts.size();
    }

    // ---- interpolative decomposition of every face (Section 2.3) ---------
    // one joint pivot order, rank list and Gram arena for the faces of all problems
    DevBuf<int> d_perm(std::max<int64_t>(npt_all, 1));
    DevBuf<double> Lp;
    DevBuf<int64_t> d_goff;
    DevBuf<int> d_gld;
    if (eps > 0.0 && nface_all > 0) {
      std::vector<int64_t> goff(nface_all), ppoff(nface_all);
      std::vector<int> gld(nface_all), nF(nface_all);
      int64_t gsz = 0;
      for (int j : below) {
        Job<T>& J = jobs[j];
        const Level<T>& lev = J.impl->levels[level];
        const LevelPlan& P = *lev.plan;
        HIF_REQUIRE(lev.maxF <= kPcholMax, HIF_EINVAL, "face larger than the ID kernel supports");
        for (int f = 0; f < P.nface; ++f) {
          const int64_t i = J.face0 + f;
          goff[i] = gsz;
          gld[i] = std::max(1, P.fN[f]);
          nF[i] = P.fN[f];
          ppoff[i] = J.pt0 + P.fpt_off[f];
          gsz += (int64_t)gld[i] * P.fN[f];
        }
      }
      DevBuf<double> G(std::max<int64_t>(gsz, 1));
      Lp.alloc(std::max<int64_t>(gsz, 1));
      // G = M^T M with M = the panel rows outside F (K x |F| per face), read in
      // place; the lower part is computed and both triangles are written
      std::vector<GemmDesc> gd;
      for (int j : below) {
        Job<T>& J = jobs[j];
        const Level<T>& lev = J.impl->levels[level];
        const LevelPlan& P = *lev.plan;
        for (int f = 0; f < P.nface; ++f) {
          const T* PR = lev.panel.get() + J.poff[f] + P.fN[f];
          const int K = P.prow[f] - P.fN[f];
          const int64_t i = J.face0 + f;
          gd.push_back(
              {PR, PR, G.get() + goff[i], P.fN[f], P.fN[f], K, J.pld[f], J.pld[f], gld[i]});
          J.flops += 2.0 * K * P.fN[f] * (double)P.fN[f];
        }
      }
      run_gemms<T, double>("gemm_gram", OP_T, OP_N, GF_C_LOWER | GF_C_MIRROR, gd, 1.0, 0.0, s,
                           GC_GRAM);
      d_goff = to_dev(goff, s);
      d_gld = to_dev(gld, s);
      DevBuf<int> d_nF = to_dev(nF, s);
      DevBuf<int64_t> d_ppoff = to_dev(ppoff, s);
      for (int j : below) {
        Job<T>& J = jobs[j];
        const Level<T>& lev = J.impl->levels[level];
        const LevelPlan& P = *lev.plan;
        if (P.nface == 0) continue;
        dim3 g((unsigned)ceil_div(std::max(1, lev.maxF), NT), (unsigned)P.nface);
        hipLaunchKernelGGL(k_gram_edges, g, dim3(NT), 0, s, J.A->stencil(), P.w, lev.fpts.get(),
                           lev.fpt_off.get(), lev.fN.get(), G.get(), d_goff.get() + J.face0,
                           d_gld.get() + J.face0);
        HIF_LAUNCH_CHECK();
      }
      DevBuf<int> d_k(nface_all);
      pivoted_cholesky(G.get(), Lp.get(), d_goff.get(), d_nF.get(), d_gld.get(), d_ppoff.get(),
                       d_perm.get(), d_k.get(), (int)nface_all, eps, nF, goff, gld, ppoff, s);
      std::vector<int> k_all(nface_all), perm_all(npt_all);
      HIF_HIP(hipMemcpyAsync(k_all.data(), d_k.get(), sizeof(int) * nface_all,
                             hipMemcpyDeviceToHost, s));
      HIF_HIP(hipMemcpyAsync(perm_all.data(), d_perm.get(), sizeof(int) * npt_all,
                             hipMemcpyDeviceToHost, s));
      check_errors();  // synchronizes: ranks, pivots and flags are on the host
      staging_synced(s);
      G.release();
      for (int j : below) {
        Job<T>& J = jobs[j];
        Level<T>& lev = J.impl->levels[level];
        std::copy(k_all.begin() + J.face0, k_all.begin() + J.face0 + lev.plan->nface,
                  lev.hk.begin());
        std::copy(perm_all.begin() + J.pt0, perm_all.begin() + J.pt0 + J.hperm.size(),
                  J.hperm.begin());
      }

      // skeleton descriptors and arenas; T = R11^{-1} R12 = L11^{-T} L21^T (FP64)
      std::vector<FrontDesc> tri;
      for (int j : below) {
        Job<T>& J = jobs[j];
        Level<T>& lev = J.impl->levels[level];
        const LevelPlan& P = *lev.plan;
        int64_t ssz = 0, s11 = 0, s21 = 0, shh = 0, shc = 0;
        J.o11.clear();
        J.o21.clear();
        J.ohh.clear();
        J.ohc.clear();
        for (int f = 0; f < P.nface; ++f) {
          const int k = lev.hk[f], r = P.fN[f] - k;
          J.flops += (double)P.fN[f] * k * k;
          if (r == 0) continue;
          SkelDesc d{};
          d.face = f;
          d.k = k;
          d.r = r;
          d.pad_ = 0;
          d.pts_off = P.fpt_off[f];
          d.offT = ssz;
          ssz += (int64_t)k * r;
          d.offL = ssz;
          ssz += (int64_t)r * r;
          d.offY = ssz;
          ssz += (int64_t)r * k;
          d.kofs = lev.ksum;
          d.rofs = lev.rsum;
          lev.ksum += k;
          lev.rsum += r;
          lev.hsk.push_back(d);
          J.o11.push_back(s11);
          s11 += (int64_t)k * k;
          J.o21.push_back(s21);
          s21 += (int64_t)r * k;
          J.ohh.push_back(shh);
          shh += (int64_t)k * k;
          J.ohc.push_back(shc);
          shc += (int64_t)k * r;
          lev.maxk = std::max(lev.maxk, k);
          lev.maxr = std::max(lev.maxr, r);
          lev.redundant += r;
          const double kk = k, rr = r;
          J.flops += 2 * kk * kk * kk / 3 + kk * kk * rr + 2 * rr * rr * kk + 2 * kk * kk * rr +
                     2 * rr * rr * kk + 2 * rr * rr * rr / 3 + rr * rr * kk + 2 * kk * kk * rr;
        }
        const int nsk = (int)lev.hsk.size();
        // every block and vector range a descriptor names lies inside the arena
        // it indexes (the skeleton kernels and the apply sweeps trust them)
        for (const SkelDesc& d : lev.hsk)
          HIF_REQUIRE(d.face >= 0 && d.face < P.nface && d.k >= 0 && d.r > 0 &&
                          d.k + d.r == P.fN[d.face] && d.pts_off == P.fpt_off[d.face] &&
                          d.offT >= 0 && d.offL == d.offT + (int64_t)d.k * d.r &&
                          d.offY == d.offL + (int64_t)d.r * d.r &&
                          d.offY + (int64_t)d.r * d.k <= ssz && d.kofs >= 0 &&
                          d.kofs + d.k <= lev.ksum && d.rofs >= 0 && d.rofs + d.r <= lev.rsum,
                      HIF_EDEVICE, "internal error: a skeleton descriptor leaves its arenas");
        J.ssz = ssz;
        lev.sk = to_dev(lev.hsk, s);
        lev.skel.alloc(std::max<int64_t>(ssz, 1));
        if (nsk == 0) continue;
        J.L11.alloc(std::max<int64_t>(s11, 1));
        J.L21.alloc(std::max<int64_t>(s21, 1));
        J.Ahh.alloc(std::max<int64_t>(shh, 1));
        J.Ahc.alloc(std::max<int64_t>(shc, 1));
        J.d_o11 = to_dev(J.o11, s);
        J.d_o21 = to_dev(J.o21, s);
        J.d_ohh = to_dev(J.ohh, s);
        J.d_ohc = to_dev(J.ohc, s);
        {
          dim3 g((unsigned)std::max(1, lev.maxk), (unsigned)nsk);
          hipLaunchKernelGGL(k_split_L, g, dim3(NT), 0, s, Lp.get(), d_goff.get() + J.face0,
                             d_gld.get() + J.face0, d_perm.get() + J.pt0, lev.fpt_off.get(),
                             lev.sk.get(), J.L11.get(), J.d_o11.get(), J.L21.get(),
                             J.d_o21.get(), lev.fN.get());
          HIF_LAUNCH_CHECK();
        }
        for (int i = 0; i < nsk; ++i) {
          const int k = lev.hsk[i].k;
          if (k > 0) tri.push_back({J.L11.get() + J.o11[i], k, k, k, 0});
        }
      }
      if (!tri.empty()) {
        DevBuf<FrontDesc> d_tri = to_dev(tri, s);
        // L11 holds zeros above the diagonal (rows pivoted earlier)
        front_invert<double>(d_tri.get(), tri, s, true);
      }
      std::vector<GemmDesc> tg;
      for (int j : below) {
        Job<T>& J = jobs[j];
        Level<T>& lev = J.impl->levels[level];
        if (lev.hsk.empty()) continue;
        double* Tdst = (double*)lev.skel.get();
        if (!std::is_same<T, double>::value) {
          J.Td.alloc(std::max<int64_t>(J.ssz, 1));
          Tdst = J.Td.get();
        }
        for (size_t i = 0; i < lev.hsk.size(); ++i) {
          const SkelDesc& d = lev.hsk[i];
          if (d.k == 0) continue;
          tg.push_back({J.L11.get() + J.o11[i], J.L21.get() + J.o21[i], Tdst + d.offT, d.k, d.r,
                        d.k, d.k, d.r, d.k});
        }
      }
      run_gemms<double, double>("gemm_interp", OP_T, OP_T, GF_A_UPPER, tg, 1.0, 0.0, s);
      for (int j : below) {
        Job<T>& J = jobs[j];
        Level<T>& lev = J.impl->levels[level];
        if (!std::is_same<T, double>::value && !lev.hsk.empty() && J.ssz > 0) {
          ProfScope ps("convert_T", s);
          hipLaunchKernelGGL((k_convert<T>),
                             dim3((unsigned)std::min<int64_t>(ceil_div(J.ssz, NT), 8192)),
                             dim3(NT), 0, s, J.Td.get(), lev.skel.get(), J.ssz);
          HIF_LAUNCH_CHECK();
        }
        J.L11.release();
        J.L21.release();
        J.Td.release();
      }
      Lp.release();

      // ---- skeleton update (Section 2.3, B blocks) -----------------------
      std::vector<GemmDesc> g1, g2, g3, g4, g5;
      std::vector<FrontDesc> cfd;
      for (int j : below) {
        Job<T>& J = jobs[j];
        Level<T>& lev = J.impl->levels[level];
        const int nsk = (int)lev.hsk.size();
        if (nsk == 0) continue;
        {
          dim3 g((unsigned)std::max(1, lev.maxF), (unsigned)nsk);
          hipLaunchKernelGGL((k_skel_gather<T>), g, dim3(NT), 0, s, lev.panel.get(),
                             lev.panel_off.get(), lev.panel_ld.get(), d_perm.get() + J.pt0,
                             lev.fpt_off.get(), lev.sk.get(), J.Ahh.get(), J.d_ohh.get(),
                             J.Ahc.get(), J.d_ohc.get(), lev.skel.get());
          HIF_LAUNCH_CHECK();
        }
        T* SK = lev.skel.get();
        for (int i = 0; i < nsk; ++i) {
          const SkelDesc& d = lev.hsk[i];
          T* Tm = SK + d.offT;
          T* Acc = SK + d.offL;
          T* Hh = J.Ahh.get() + J.ohh[i];
          T* Hc = J.Ahc.get() + J.ohc[i];
          const int k = std::max(d.k, 1), r = d.r;
          g1.push_back({Tm, Hc, Acc, d.r, d.r, d.k, k, k, r});        // Acc -= T^T A_hc
          g2.push_back({Hh, Tm, Hc, d.k, d.r, d.k, k, k, k});         // A_hc -= A_hh T  (= B_hc)
          g3.push_back({Hc, Tm, Acc, d.r, d.r, d.k, k, k, r});        // Acc -= B_hc^T T (= B_cc)
          g4.push_back({Acc, Hc, SK + d.offY, d.r, d.k, d.r, r, k, r});  // Y = Lc^{-1} B_hc^T
          g5.push_back({SK + d.offY, SK + d.offY, Hh, d.k, d.k, d.r, r, r, k});  // A_hh -= Y^T Y
          cfd.push_back({Acc, d.r, d.r, d.r, (int)own_skel[level].size()});
          own_skel[level].push_back({j, i});
        }
      }
      run_gemms<T, T>("gemm_skel", OP_T, OP_N, 0, g1, T(-1), T(1), s);
      run_gemms<T, T>("gemm_skel", OP_N, OP_N, 0, g2, T(-1), T(1), s);
      run_gemms<T, T>("gemm_skel", OP_T, OP_N, 0, g3, T(-1), T(1), s);
      if (!cfd.empty()) {
        DevBuf<FrontDesc> d_cfd = to_dev(cfd, s);
        front_factor<T>(d_cfd.get(), cfd, d_err.get() + 2 * level + 1, s, false, kSmallFrontLeaf);
      }
      run_gemms<T, T>("gemm_skel", OP_N, OP_T, GF_A_LOWER, g4, T(1), T(0), s);
      run_gemms<T, T>("gemm_skel", OP_T, OP_N, 0, g5, T(-1), T(1), s);
      for (int j : below) {
        Job<T>& J = jobs[j];
        Level<T>& lev = J.impl->levels[level];
        const int nsk = (int)lev.hsk.size();
        if (nsk > 0) {
          dim3 g((unsigned)std::max(1, lev.maxk), (unsigned)nsk);
          hipLaunchKernelGGL((k_skel_writeback<T>), g, dim3(NT), 0, s, lev.panel.get(),
                             lev.panel_off.get(), lev.panel_ld.get(), d_perm.get() + J.pt0,
                             lev.fpt_off.get(), lev.sk.get(), J.Ahh.get(), J.d_ohh.get());
          HIF_LAUNCH_CHECK();
        }
        J.Ahh.release();
        J.Ahc.release();
      }
    } else {
      // eps = 0: no ID, every face point is a skeleton point
      std::vector<int> perm_all((size_t)std::max<int64_t>(npt_all, 1), 0);
      for (int j : below) {
        Job<T>& J = jobs[j];
        Level<T>& lev = J.impl->levels[level];
        const LevelPlan& P = *lev.plan;
        for (int f = 0; f < P.nface; ++f) {
          lev.hk[f] = P.fN[f];
          for (int q = 0; q < P.fN[f]; ++q) {
            J.hperm[P.fpt_off[f] + q] = q;
            perm_all[J.pt0 + P.fpt_off[f] + q] = q;
          }
        }
      }
      d_perm.upload(perm_all, s);
    }

    for (int j : below) {
      Job<T>& J = jobs[j];
      hif_stats& st = J.F->stats;
      Level<T>& lev = J.impl->levels[level];
      const LevelPlan& P = *lev.plan;
      // face points in pivot order for the apply
      lev.skpts.alloc(std::max<size_t>(P.fpts.size(), 1));
      if (P.nface > 0) {
        dim3 g((unsigned)ceil_div(std::max(1, lev.maxF), NT), (unsigned)P.nface);
        hipLaunchKernelGGL(k_perm_points, g, dim3(NT), 0, s, lev.fpts.get(), d_perm.get() + J.pt0,
                           lev.fpt_off.get(), lev.fN.get(), lev.skpts.get());
        HIF_LAUNCH_CHECK();
      }
      st.redundant[level] = lev.redundant;

      // ---- next level's active set and lookup maps ------------------------
      hipLaunchKernelGGL(k_fill_map, dim3((unsigned)std::min<int64_t>(ceil_div(J.N, NT), 8192)),
                         dim3(NT), 0, s, J.d_pmap.get(), J.N);
      HIF_LAUNCH_CHECK();
      if (P.nface > 0) {
        dim3 g((unsigned)ceil_div(std::max(1, lev.maxF), NT), (unsigned)P.nface);
        hipLaunchKernelGGL(k_face_map, g, dim3(NT), 0, s, lev.fpts.get(), lev.fpt_off.get(),
                           lev.fN.get(), J.d_pmap.get());
        HIF_LAUNCH_CHECK();
      }
      std::vector<int> red;
      red.reserve(lev.redundant);
      for (int f = 0; f < P.nface; ++f) {
        const int64_t o0 = P.fpt_off[f];
        for (int q = lev.hk[f]; q < P.fN[f]; ++q) {
          const int p = P.fpts[o0 + J.hperm[o0 + q]];
          J.active[p] = 0;
          red.push_back(p);
        }
      }
      J.F->redundant_pts.push_back(std::move(red));
      J.F->ranks.push_back(lev.hk);
      J.F->sizes.push_back(P.fN);
    }
  }
  HIF_HIP(hipEventRecord(ev.e[maxL + 1], s));
  for (auto& J : jobs) J.impl->prepare(s);
  check_errors();
  staging_synced(s);
  std::vector<double> level_s(maxL + 1);
  for (int level = 0; level <= maxL; ++level) {
    float ms = 0.f;
    HIF_HIP(hipEventElapsedTime(&ms, ev.e[level], ev.e[level + 1]));
    level_s[level] = 1e-3 * ms;
  }
  prof_level() = -1;
  const double t_end = now_s();
  for (auto& J : jobs) {
    hif_stats& st = J.F->stats;
    J.flops_mark.push_back(J.flops);
    for (int level = 0; level <= J.L; ++level) {
      st.level_seconds[level] = level_s[level];
      st.level_flops[level] = J.flops_mark[level + 1] - J.flops_mark[level];
      st.level_bytes[level] = (int64_t)(J.impl->levels[level].front.bytes() +
                                        J.impl->levels[level].skel.bytes());
    }
    st.e_s = std::nan("");
    st.err_norm = std::nan("");
    st.factor_flops = J.flops;
    st.build_seconds = t_end - t_begin;
    st.peak_bytes = mem_stats().peak - mem0;
    J.F->impl = std::move(J.impl);
    st.factor_bytes = J.F->impl->stored_bytes();
  }
}

template <typename T>
void build_factor(const hif_problem_s* A, const hif_options& o, hipStream_t s, hif_factor_s* F) {
  build_factors<T>({BuildRequest{A, o, F}}, s);
}

template <typename T>
int64_t FactorImpl<T>::stored_bytes() const {
  int64_t b = 0;
  for (auto& l : levels) b += (int64_t)(l.front.bytes() + l.skel.bytes());
  return b;
}

template void build_factors<double>(const std::vector<BuildRequest>&, hipStream_t);
template void build_factors<float>(const std::vector<BuildRequest>&, hipStream_t);
template void build_factor<double>(const hif_problem_s*, const hif_options&, hipStream_t,
                                   hif_factor_s*);
template void build_factor<float>(const hif_problem_s*, const hif_options&, hipStream_t,
                                  hif_factor_s*);
template int64_t FactorImpl<double>::stored_bytes() const;
template int64_t FactorImpl<float>::stored_bytes() const;

}  // namespace hif
