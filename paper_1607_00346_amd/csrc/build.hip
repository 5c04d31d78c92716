// Level executor of the HIF factorization (paper, Section 2.4 level loop,
// Section 3.2 face snapshot).  One level = gather fronts, factor them,
// form the Schur updates, assemble face panels, interpolative decomposition
// of every face, skeleton update; a host round trip reads the ranks back.
#include <chrono>
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
  const int* pface;
  const int* ploc;
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
  const T* pcol;
  int gface[kRowBlocks], goff[kRowBlocks];
};

template <typename T>
__device__ __forceinline__ ColLookup<T> col_lookup(const Src<T>& s, int q) {
  ColLookup<T> c;
  c.q = q;
  c.fq = s.has_prev ? s.pface[q] : -1;
  c.pcol = nullptr;
#pragma unroll
  for (int t = 0; t < kRowBlocks; ++t) {
    c.gface[t] = -1;
    c.goff[t] = 0;
  }
  if (c.fq >= 0) {
    c.pcol = s.panels + s.poff[c.fq] + (int64_t)s.pld[c.fq] * s.ploc[q];
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
// value.
template <typename T>
__device__ __forceinline__ T row_lookup(const Src<T>& s, const ColLookup<T>& c, int p) {
  if (c.fq >= 0) {
    const int fp = s.pface[p];
    if (fp >= 0) {
      int off = -1;
#pragma unroll
      for (int t = 0; t < kRowBlocks; ++t)
        if (c.gface[t] == fp) off = c.goff[t];
      return off >= 0 ? c.pcol[off + s.ploc[p]] : T(0);
    }
  }
  const int q = c.q;
  if (p == q) return (T)s.st.diag[p];
  const int dl = q - p;
  const int lo = p < q ? p : q;
  const int n = s.st.n;
  if (dl == 1 || dl == -1) return (T)(-s.st.cx[lo]);
  if (dl == n || dl == -n) return (T)(-s.st.cy[lo]);
  if (dl == n * n || dl == -n * n) return (T)(-s.st.cz[lo]);
  return T(0);
}

// The gathers give each wave one column (four columns per workgroup): the
// column's lookup state is then wave-uniform (scalar registers) and columns
// of a few dozen rows still keep most lanes busy.
constexpr int kGatherCols = NT / 64;

__device__ __forceinline__ int wave_column(int block) {
  return block * kGatherCols + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// Front of cell c, column j: A_II(i, j) for i >= j into Phi, and zeros above
// the diagonal (the factorization keeps them, so the inverse's products need
// no triangular masks).
template <typename T>
__global__ __launch_bounds__(NT) void k_gather_front(Src<T> s, const int* __restrict__ rows,
                                                     const int64_t* __restrict__ crow_off,
                                                     const FrontDesc* __restrict__ fd, T* arena) {
  const int c = blockIdx.y;
  const FrontDesc f = fd[c];
  const int j = wave_column(blockIdx.x);
  if (j >= f.nI) return;
  const int lane = threadIdx.x & 63;
  const int* r = rows + crow_off[c];
  const ColLookup<T> cl = col_lookup(s, r[j]);
  T* col = arena + f.off + (int64_t)f.ld * j;
  for (int i = lane; i < j; i += 64) col[i] = T(0);
  for (int i = j + lane; i < f.nI; i += 64) col[i] = row_lookup(s, cl, r[i]);
}

// A_SI of cell c, column j (the j-th interior point): nS x nI, leading dimension nS.
template <typename T>
__global__ __launch_bounds__(NT) void k_gather_front_SI(Src<T> s, const int* __restrict__ rows,
                                                        const int64_t* __restrict__ crow_off,
                                                        const FrontDesc* __restrict__ fd, T* asi,
                                                        const int64_t* __restrict__ aoff) {
  const int c = blockIdx.y;
  const FrontDesc f = fd[c];
  const int j = wave_column(blockIdx.x);
  if (j >= f.nI) return;
  const int nS = f.nR - f.nI;
  const int lane = threadIdx.x & 63;
  const int* r = rows + crow_off[c];
  const ColLookup<T> cl = col_lookup(s, r[j]);
  T* col = asi + aoff[c] + (int64_t)nS * j;
  for (int i = lane; i < nS; i += 64) col[i] = row_lookup(s, cl, r[f.nI + i]);
}

// Panel of face f, column j: Ã^l(rows, F_j) = A^l(rows, F_j) + U_A + U_B, the
// Schur updates of the two neighbouring cells added in a fixed order.
template <typename T>
__global__ __launch_bounds__(NT) void k_gather_panel(
    Src<T> s, const int* __restrict__ fpts, const int64_t* __restrict__ fpt_off,
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
  for (int t = 0; t < kRowBlocks; ++t) {
    const int g = rb_face[base + t];
    if (g < 0) break;
    const int ro = rb_off[base + t], sa = rb_sa[base + t], sb = rb_sb[base + t];
    const int ng = fN[g];
    const int* G = fpts + fpt_off[g];
    for (int i = lane; i < ng; i += 64) {
      T v = row_lookup(s, cl, G[i]);
      if (sa >= 0) v += UA[(sa + i) + (int64_t)ldA * colA];
      if (sb >= 0) v += UB[(sb + i) + (int64_t)ldB * colB];
      col[ro + i] = v;
    }
  }
}

__device__ __forceinline__ int nsep(int x, int y, int z, int w) {
  return (x % w == 0 && x != 0) + (y % w == 0 && y != 0) + (z % w == 0 && z != 0);
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
  const int n = st.n;
  const int q = fpts[fpt_off[f] + j];
  const int x = q % n, y = (q / n) % n, z = q / (n * n);
  double add = 0.0;
  if (x > 0 && nsep(x - 1, y, z, w) == 2) add += st.cx[q - 1] * st.cx[q - 1];
  if (x < n - 1 && nsep(x + 1, y, z, w) == 2) add += st.cx[q] * st.cx[q];
  if (y > 0 && nsep(x, y - 1, z, w) == 2) add += st.cy[q - n] * st.cy[q - n];
  if (y < n - 1 && nsep(x, y + 1, z, w) == 2) add += st.cy[q] * st.cy[q];
  if (z > 0 && nsep(x, y, z - 1, w) == 2) add += st.cz[q - n * n] * st.cz[q - n * n];
  if (z < n - 1 && nsep(x, y, z + 1, w) == 2) add += st.cz[q] * st.cz[q];
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

// Lookup maps for the next level: the face of every face point and its index
// within the face (-1 for every other point; the fill runs first).
__global__ __launch_bounds__(NT) void k_fill_int(int* p, int64_t n, int v) {
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    p[i] = v;
}

__global__ __launch_bounds__(NT) void k_face_map(const int* __restrict__ fpts,
                                                 const int64_t* __restrict__ fpt_off,
                                                 const int* __restrict__ fN, int* pface, int* ploc) {
  const int f = blockIdx.y;
  const int j = blockIdx.x * NT + threadIdx.x;
  if (j >= fN[f]) return;
  const int p = fpts[fpt_off[f] + j];
  pface[p] = f;
  ploc[p] = j;
}

template <typename T>
Src<T> make_src(const hif_problem_s* A, const Level<T>* prev, const int* pface, const int* ploc) {
  Src<T> s;
  s.st = A->stencil();
  s.has_prev = prev != nullptr;
  s.pface = pface;
  s.ploc = ploc;
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
void run_gemms(const char* name, int opa, int opb, int flags, const std::vector<GemmDesc>& h,
               TC alpha, TC beta, hipStream_t s, int cls = GC_GENERIC) {
  if (h.empty()) return;
  int mm = 0, mn = 0;
  double fl = 0.0;
  for (auto& d : h) {
    mm = std::max(mm, d.m);
    mn = std::max(mn, d.n);
    fl += gemm_flops(d, flags);
  }
  DevBuf<GemmDesc> d;
  d.upload(h, s);
  gemm_batched<TIn, TC>(opa, opb, flags, d.get(), (int)h.size(), mm, mn, alpha, beta, s, name, fl,
                        cls);
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

template <typename T>
void build_factor(const hif_problem_s* A, const hif_options& o, hipStream_t s, hif_factor_s* F) {
  const int n = A->n;
  const int leaf = o.leaf;
  const int L = levels_for(n, leaf);
  HIF_REQUIRE(L >= 0 && L <= HIF_MAX_LEVELS - 1, HIF_EINVAL, "n must be leaf * 2^L");
  const int64_t N = A->N;
  auto impl = std::make_unique<FactorImpl<T>>();
  FactorImpl<T>& Fi = *impl;
  Fi.n = n;
  Fi.L = L;
  Fi.N = N;
  Fi.levels.resize(L + 1);
  hif_stats& st = F->stats;
  std::memset(&st, 0, sizeof(st));
  st.levels = L;
  st.precision = o.precision;
  st.n_dof = N;
  const double t_begin = now_s();
  const int64_t mem0 = mem_stats().live;
  mem_stats().peak = mem0;

  if (A->geom_leaf != leaf) {
    A->geom = plan_geometry(n, leaf);
    A->plan0 = std::make_shared<const LevelPlan>(
        plan_level(A->geom[0], std::vector<uint8_t>((size_t)N, 1)));
    A->dev0 = {};
    A->geom_leaf = leaf;
  }
  // 0 for points the ID has left out so far (the candidates of a level are
  // separator points of the level below, so interior points never need it)
  std::vector<uint8_t> active(N, 1);
  // face / local index of every level-(l-1) face point, for the A^l lookup
  DevBuf<int> d_pface(L > 0 ? N : 0), d_ploc(L > 0 ? N : 0);
  // failure flags: per level, the interior Cholesky (cell) and the Cholesky of
  // B_F̌F̌ (skeleton index); checked whenever the host synchronizes anyway
  const int kNoErr = INT_MAX;
  std::vector<int> h_err(2 * (L + 1), kNoErr);
  DevBuf<int> d_err = to_dev(h_err, s);
  auto check_errors = [&]() {
    HIF_HIP(hipMemcpyAsync(h_err.data(), d_err.get(), sizeof(int) * h_err.size(),
                           hipMemcpyDeviceToHost, s));
    HIF_HIP(hipStreamSynchronize(s));
    for (int l = 0; l <= L; ++l) {
      if (h_err[2 * l] != kNoErr)
        throw Error(HIF_ENOTSPD, "non-positive pivot in the interior Cholesky at level " +
                                     std::to_string(l) + ", cell " + std::to_string(h_err[2 * l]));
      if (h_err[2 * l + 1] != kNoErr)
        throw Error(HIF_ENOTSPD, "non-positive pivot in B_F̌F̌ at level " + std::to_string(l) +
                                     ", face " +
                                     std::to_string(Fi.levels[l].hsk[h_err[2 * l + 1]].face));
    }
  };
  // device-side level timing
  struct Events {
    std::vector<hipEvent_t> e;
    ~Events() {
      for (hipEvent_t x : e) (void)hipEventDestroy(x);
    }
  } ev;
  ev.e.resize(L + 2, nullptr);
  for (auto& x : ev.e) HIF_HIP(hipEventCreate(&x));
  double flops = 0.0;

  for (int level = 0; level <= L; ++level) {
    HIF_HIP(hipEventRecord(ev.e[level], s));
    profiler().level = level;
    Level<T>& lev = Fi.levels[level];
    Level<T>* prev = level > 0 ? &Fi.levels[level - 1] : nullptr;
    lev.plan = level == 0 ? A->plan0
                          : std::make_shared<const LevelPlan>(plan_level(A->geom[level], active));
    const LevelPlan& P = *lev.plan;
    const Src<T> src = make_src<T>(A, prev, d_pface.get(), d_ploc.get());
    // index arrays of the plan; level 0's are uploaded once per problem
    auto arr = [&](auto& cached, const auto& host) {
      if (level > 0) return dev_arr(host, s);
      if (!cached.buf) cached = dev_arr(host, s);
      return cached;
    };

    // ---- fronts: gather, partial Cholesky + inverse (Section 2.2) -------
    lev.rows = arr(A->dev0.rows, P.rows);
    lev.crow_off = arr(A->dev0.crow_off, P.crow_off);
    lev.hfd.resize(P.ncell);
    int64_t off = 0;
    std::vector<int64_t> yoff(P.ncell), zoff(P.ncell);
    for (int c = 0; c < P.ncell; ++c) {
      FrontDesc& d = lev.hfd[c];
      d.off = off;
      d.nI = P.cI[c];
      d.nR = P.cI[c] + P.cS[c];
      d.ld = pad_ld(d.nR);
      d.pad_ = 0;
      off += (int64_t)d.ld * d.nI;
      yoff[c] = lev.ysum;
      zoff[c] = lev.zsum;
      lev.ysum += d.nI;
      lev.zsum += P.cS[c];
      lev.maxI = std::max(lev.maxI, d.nI);
      lev.maxS = std::max(lev.maxS, P.cS[c]);
      const double nI = d.nI, nS = P.cS[c];
      flops += nI * nI * nI / 3.0 + nS * nI * nI + nI * nI * nI / 3.0 + nS * nS * nI;
      st.max_front[level] = std::max<int64_t>(st.max_front[level], d.nR);
    }
    lev.fd = to_dev(lev.hfd, s);
    lev.yoff = to_dev(yoff, s);
    lev.zoff = to_dev(zoff, s);
    lev.front.alloc(off);
    st.cells[level] = P.ncell;
    st.eliminated[level] = lev.ysum;
    // A_SI (nS x nI per cell) until L_SI = A_SI L_I^{-T} is formed
    std::vector<int64_t> xoff(P.ncell);
    int64_t xsz = 0;
    for (int c = 0; c < P.ncell; ++c) {
      xoff[c] = xsz;
      xsz += (int64_t)P.cI[c] * P.cS[c];
    }
    if (P.ncell > 0) {
      DevBuf<T> ASI(std::max<int64_t>(xsz, 1));
      DevBuf<int64_t> d_xoff = to_dev(xoff, s);
      {
        ProfScope ps("gather_front", s);
        dim3 g((unsigned)ceil_div(std::max(1, lev.maxI), kGatherCols), (unsigned)P.ncell);
        hipLaunchKernelGGL((k_gather_front<T>), g, dim3(NT), 0, s, src, lev.rows.get(),
                           lev.crow_off.get(), lev.fd.get(), lev.front.get());
        HIF_LAUNCH_CHECK();
        if (lev.maxS > 0) {
          dim3 g2((unsigned)ceil_div(std::max(1, lev.maxI), kGatherCols), (unsigned)P.ncell);
          hipLaunchKernelGGL((k_gather_front_SI<T>), g2, dim3(NT), 0, s, src, lev.rows.get(),
                             lev.crow_off.get(), lev.fd.get(), ASI.get(), d_xoff.get());
          HIF_LAUNCH_CHECK();
        }
      }
      // interior Cholesky and in-place inverse on the top nI x nI block
      std::vector<FrontDesc> top = lev.hfd;
      for (auto& d : top) d.nR = d.nI;
      DevBuf<FrontDesc> d_top = to_dev(top, s);
      front_factor<T>(lev.front.get(), d_top.get(), top, d_err.get() + 2 * level, s, true);
      // L_SI = A_SI L_I^{-T} into the front below L_I^{-1} (L_I^{-T} is upper)
      std::vector<GemmDesc> gd;
      for (int c = 0; c < P.ncell; ++c) {
        if (P.cS[c] == 0) continue;
        const FrontDesc& d = lev.hfd[c];
        T* base = lev.front.get() + d.off;
        gd.push_back({ASI.get() + xoff[c], base, base + d.nI, P.cS[c], d.nI, d.nI, P.cS[c], d.ld,
                      d.ld});
      }
      run_gemms<T, T>("gemm_lsi", OP_N, OP_T, GF_B_UPPER | GF_TRI_ZEROS, gd, T(1), T(0), s,
                      GC_LSI);
    }

    if (!P.root) {
      // ---- Schur updates U_c = -L_SI L_SI^T (both triangles) -----------
      std::vector<int64_t> uoff(P.ncell);
      std::vector<int> uld(P.ncell);
      int64_t usz = 0;
      for (int c = 0; c < P.ncell; ++c) {
        uoff[c] = usz;
        uld[c] = std::max(1, P.cS[c]);
        usz += (int64_t)uld[c] * P.cS[c];
      }
      DevBuf<T> U(std::max<int64_t>(usz, 1));
      {
        std::vector<GemmDesc> gd;
        for (int c = 0; c < P.ncell; ++c) {
          if (P.cS[c] == 0) continue;
          const FrontDesc& d = lev.hfd[c];
          const T* LSI = lev.front.get() + d.off + d.nI;
          gd.push_back({LSI, LSI, U.get() + uoff[c], P.cS[c], P.cS[c], d.nI, d.ld, d.ld, uld[c]});
        }
        // both triangles of U, so that the panel gather reads columns only
        run_gemms<T, T>("gemm_syrk", OP_N, OP_T, GF_C_LOWER | GF_C_MIRROR, gd, T(-1), T(0), s,
                        GC_SYRK);
      }
      // ---- face panels Ã^l([F; R-faces], F) ------------------------------
      std::vector<int64_t> poff(P.nface);
      std::vector<int> pld(P.nface);
      int64_t psz = 0;
      for (int f = 0; f < P.nface; ++f) {
        poff[f] = psz;
        pld[f] = pad_ld(P.prow[f]);
        psz += (int64_t)pld[f] * P.fN[f];
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
      lev.panel_off = to_dev(poff, s);
      lev.panel_ld = to_dev(pld, s);
      lev.panel.alloc(std::max<int64_t>(psz, 1));
      st.faces[level] = P.nface;
      if (P.nface > 0) {
        DevBuf<int64_t> d_uoff = to_dev(uoff, s);
        DevBuf<int> d_uld = to_dev(uld, s);
        ProfScope ps("gather_panel", s);
        dim3 g((unsigned)ceil_div(std::max(1, lev.maxF), kGatherCols), (unsigned)P.nface);
        hipLaunchKernelGGL((k_gather_panel<T>), g, dim3(NT), 0, s, src, lev.fpts.get(),
                           lev.fpt_off.get(), lev.fN.get(), lev.rb_face.get(), lev.rb_off.get(),
                           lev.rb_sa.get(), lev.rb_sb.get(), lev.fcellA.get(), lev.fcellB.get(),
                           U.get(), d_uoff.get(), d_uld.get(), lev.panel.get(),
                           lev.panel_off.get(), lev.panel_ld.get());
        HIF_LAUNCH_CHECK();
      }
      U.release();
      if (prev) {  // A^l has been read for the last time
        prev->panel.release();
      }

      // ---- interpolative decomposition of every face (Section 2.3) -------
      std::vector<int> hperm(P.fpts.size());
      lev.hk.assign(P.nface, 0);
      DevBuf<int> d_perm(std::max<size_t>(P.fpts.size(), 1));
      for (int f = 0; f < P.nface; ++f) st.face_dofs[level] += P.fN[f];
      if (o.eps > 0.0 && P.nface > 0) {
        HIF_REQUIRE(lev.maxF <= kPcholMax, HIF_EINVAL, "face larger than the ID kernel supports");
        std::vector<int64_t> goff(P.nface);
        std::vector<int> gld(P.nface);
        int64_t gsz = 0;
        std::vector<GemmDesc> gd;
        for (int f = 0; f < P.nface; ++f) {
          goff[f] = gsz;
          gld[f] = std::max(1, P.fN[f]);
          gsz += (int64_t)gld[f] * P.fN[f];
        }
        DevBuf<double> G(std::max<int64_t>(gsz, 1)), Lp(std::max<int64_t>(gsz, 1));
        // G = M^T M with M = the panel rows outside F (K x |F| per face), read in
        // place; the lower part is computed and both triangles are written
        for (int f = 0; f < P.nface; ++f) {
          const T* PR = lev.panel.get() + poff[f] + P.fN[f];
          const int K = P.prow[f] - P.fN[f];
          gd.push_back({PR, PR, G.get() + goff[f], P.fN[f], P.fN[f], K, pld[f], pld[f], gld[f]});
          flops += 2.0 * K * P.fN[f] * (double)P.fN[f];
        }
        run_gemms<T, double>("gemm_gram", OP_T, OP_N, GF_C_LOWER | GF_C_MIRROR, gd, 1.0, 0.0, s,
                             GC_GRAM);
        DevBuf<int64_t> d_goff = to_dev(goff, s);
        DevBuf<int> d_gld = to_dev(gld, s);
        {
          dim3 g((unsigned)ceil_div(std::max(1, lev.maxF), NT), (unsigned)P.nface);
          hipLaunchKernelGGL(k_gram_edges, g, dim3(NT), 0, s, A->stencil(), P.w, lev.fpts.get(),
                             lev.fpt_off.get(), lev.fN.get(), G.get(), d_goff.get(), d_gld.get());
          HIF_LAUNCH_CHECK();
        }
        DevBuf<int> d_k(P.nface);
        std::vector<int64_t> hpoff(P.fpt_off.begin(), P.fpt_off.end() - 1);
        pivoted_cholesky(G.get(), Lp.get(), d_goff.get(), lev.fN.get(), d_gld.get(),
                         lev.fpt_off.get(), d_perm.get(), d_k.get(), P.nface, o.eps, P.fN, goff,
                         gld, hpoff, s);
        HIF_HIP(hipMemcpyAsync(lev.hk.data(), d_k.get(), sizeof(int) * P.nface,
                               hipMemcpyDeviceToHost, s));
        HIF_HIP(hipMemcpyAsync(hperm.data(), d_perm.get(), sizeof(int) * hperm.size(),
                               hipMemcpyDeviceToHost, s));
        check_errors();  // synchronizes: ranks, pivots and flags are on the host
        staging_synced(s);
        G.release();

        // skeleton descriptors and arena
        int64_t ssz = 0, s11 = 0, s21 = 0, shh = 0, shc = 0;
        std::vector<int64_t> o11, o21, ohh, ohc;
        for (int f = 0; f < P.nface; ++f) {
          const int k = lev.hk[f], r = P.fN[f] - k;
          flops += (double)P.fN[f] * k * k;
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
          o11.push_back(s11);
          s11 += (int64_t)k * k;
          o21.push_back(s21);
          s21 += (int64_t)r * k;
          ohh.push_back(shh);
          shh += (int64_t)k * k;
          ohc.push_back(shc);
          shc += (int64_t)k * r;
          lev.maxk = std::max(lev.maxk, k);
          lev.maxr = std::max(lev.maxr, r);
          lev.redundant += r;
          const double kk = k, rr = r;
          flops += 2 * kk * kk * kk / 3 + kk * kk * rr + 2 * rr * rr * kk + 2 * kk * kk * rr +
                   2 * rr * rr * kk + 2 * rr * rr * rr / 3 + rr * rr * kk + 2 * kk * kk * rr;
        }
        const int nsk = (int)lev.hsk.size();
        lev.sk = to_dev(lev.hsk, s);
        lev.skel.alloc(std::max<int64_t>(ssz, 1));
        if (nsk > 0) {
          // T = R11^{-1} R12 = L11^{-T} L21^T (FP64)
          DevBuf<double> L11(std::max<int64_t>(s11, 1)), L21(std::max<int64_t>(s21, 1));
          DevBuf<int64_t> d_o11 = to_dev(o11, s), d_o21 = to_dev(o21, s);
          {
            dim3 g((unsigned)std::max(1, lev.maxk), (unsigned)nsk);
            hipLaunchKernelGGL(k_split_L, g, dim3(NT), 0, s, Lp.get(), d_goff.get(), d_gld.get(),
                               d_perm.get(), lev.fpt_off.get(), lev.sk.get(), L11.get(),
                               d_o11.get(), L21.get(), d_o21.get(), lev.fN.get());
            HIF_LAUNCH_CHECK();
          }
          std::vector<FrontDesc> tri;
          for (int i = 0; i < nsk; ++i)
            if (lev.hsk[i].k > 0) tri.push_back({o11[i], lev.hsk[i].k, lev.hsk[i].k, lev.hsk[i].k, 0});
          if (!tri.empty()) {
            DevBuf<FrontDesc> d_tri = to_dev(tri, s);
            // L11 holds zeros above the diagonal (rows pivoted earlier)
            front_invert<double>(L11.get(), d_tri.get(), tri, s, true);
          }
          DevBuf<double> Td;
          if (!std::is_same<T, double>::value) Td.alloc(std::max<int64_t>(ssz, 1));
          double* Tdst = std::is_same<T, double>::value ? (double*)lev.skel.get() : Td.get();
          std::vector<GemmDesc> tg;
          for (int i = 0; i < nsk; ++i) {
            const SkelDesc& d = lev.hsk[i];
            if (d.k == 0) continue;
            tg.push_back({L11.get() + o11[i], L21.get() + o21[i], Tdst + d.offT, d.k, d.r, d.k,
                          d.k, d.r, d.k});
          }
          run_gemms<double, double>("gemm_interp", OP_T, OP_T, GF_A_UPPER, tg, 1.0, 0.0, s);
          if (!std::is_same<T, double>::value && ssz > 0) {
            ProfScope ps("convert_T", s);
            hipLaunchKernelGGL((k_convert<T>),
                               dim3((unsigned)std::min<int64_t>(ceil_div(ssz, NT), 8192)),
                               dim3(NT), 0, s, Td.get(), lev.skel.get(), ssz);
            HIF_LAUNCH_CHECK();
          }
          L11.release();
          L21.release();
          Lp.release();

          // ---- skeleton update (Section 2.3, B blocks) -----------------
          DevBuf<T> Ahh(std::max<int64_t>(shh, 1)), Ahc(std::max<int64_t>(shc, 1));
          DevBuf<int64_t> d_ohh = to_dev(ohh, s), d_ohc = to_dev(ohc, s);
          {
            dim3 g((unsigned)std::max(1, lev.maxF), (unsigned)nsk);
            hipLaunchKernelGGL((k_skel_gather<T>), g, dim3(NT), 0, s, lev.panel.get(),
                               lev.panel_off.get(), lev.panel_ld.get(), d_perm.get(),
                               lev.fpt_off.get(), lev.sk.get(), Ahh.get(), d_ohh.get(), Ahc.get(),
                               d_ohc.get(), lev.skel.get());
            HIF_LAUNCH_CHECK();
          }
          T* SK = lev.skel.get();
          std::vector<GemmDesc> g1, g2, g3, g4, g5;
          for (int i = 0; i < nsk; ++i) {
            const SkelDesc& d = lev.hsk[i];
            T* Tm = SK + d.offT;
            T* Acc = SK + d.offL;
            T* Hh = Ahh.get() + ohh[i];
            T* Hc = Ahc.get() + ohc[i];
            const int k = std::max(d.k, 1), r = d.r;
            g1.push_back({Tm, Hc, Acc, d.r, d.r, d.k, k, k, r});        // Acc -= T^T A_hc
            g2.push_back({Hh, Tm, Hc, d.k, d.r, d.k, k, k, k});         // A_hc -= A_hh T  (= B_hc)
            g3.push_back({Hc, Tm, Acc, d.r, d.r, d.k, k, k, r});        // Acc -= B_hc^T T (= B_cc)
            g4.push_back({Acc, Hc, SK + d.offY, d.r, d.k, d.r, r, k, r});  // Y = Lc^{-1} B_hc^T
            g5.push_back({SK + d.offY, SK + d.offY, Hh, d.k, d.k, d.r, r, r, k});  // A_hh -= Y^T Y
          }
          run_gemms<T, T>("gemm_skel", OP_T, OP_N, 0, g1, T(-1), T(1), s);
          run_gemms<T, T>("gemm_skel", OP_N, OP_N, 0, g2, T(-1), T(1), s);
          run_gemms<T, T>("gemm_skel", OP_T, OP_N, 0, g3, T(-1), T(1), s);
          std::vector<FrontDesc> cfd;
          for (int i = 0; i < nsk; ++i)
            cfd.push_back({lev.hsk[i].offL, lev.hsk[i].r, lev.hsk[i].r, lev.hsk[i].r, 0});
          {
            DevBuf<FrontDesc> d_cfd = to_dev(cfd, s);
            front_factor<T>(SK, d_cfd.get(), cfd, d_err.get() + 2 * level + 1, s, false);
          }
          run_gemms<T, T>("gemm_skel", OP_N, OP_T, GF_A_LOWER, g4, T(1), T(0), s);
          run_gemms<T, T>("gemm_skel", OP_T, OP_N, 0, g5, T(-1), T(1), s);
          {
            dim3 g((unsigned)std::max(1, lev.maxk), (unsigned)nsk);
            hipLaunchKernelGGL((k_skel_writeback<T>), g, dim3(NT), 0, s, lev.panel.get(),
                               lev.panel_off.get(), lev.panel_ld.get(), d_perm.get(),
                               lev.fpt_off.get(), lev.sk.get(), Ahh.get(), d_ohh.get());
            HIF_LAUNCH_CHECK();
          }
        }
      } else {
        for (int f = 0; f < P.nface; ++f) {
          lev.hk[f] = P.fN[f];
          for (int j = 0; j < P.fN[f]; ++j) hperm[P.fpt_off[f] + j] = j;
        }
        d_perm.upload(hperm, s);
      }
      // face points in pivot order for the apply
      lev.skpts.alloc(std::max<size_t>(P.fpts.size(), 1));
      if (P.nface > 0) {
        dim3 g((unsigned)ceil_div(std::max(1, lev.maxF), NT), (unsigned)P.nface);
        hipLaunchKernelGGL(k_perm_points, g, dim3(NT), 0, s, lev.fpts.get(), d_perm.get(),
                           lev.fpt_off.get(), lev.fN.get(), lev.skpts.get());
        HIF_LAUNCH_CHECK();
      }
      st.redundant[level] = lev.redundant;

      // ---- next level's active set and lookup maps --------------------
      {
        hipLaunchKernelGGL(k_fill_int, dim3((unsigned)std::min<int64_t>(ceil_div(N, NT), 8192)),
                           dim3(NT), 0, s, d_pface.get(), N, -1);
        HIF_LAUNCH_CHECK();
        if (P.nface > 0) {
          dim3 g((unsigned)ceil_div(std::max(1, lev.maxF), NT), (unsigned)P.nface);
          hipLaunchKernelGGL(k_face_map, g, dim3(NT), 0, s, lev.fpts.get(), lev.fpt_off.get(),
                             lev.fN.get(), d_pface.get(), d_ploc.get());
          HIF_LAUNCH_CHECK();
        }
      }
      std::vector<int> red;
      red.reserve(lev.redundant);
      for (int f = 0; f < P.nface; ++f) {
        const int64_t o0 = P.fpt_off[f];
        for (int j = lev.hk[f]; j < P.fN[f]; ++j) {
          const int p = P.fpts[o0 + hperm[o0 + j]];
          active[p] = 0;
          red.push_back(p);
        }
      }
      F->redundant_pts.push_back(std::move(red));
      F->ranks.push_back(lev.hk);
      F->sizes.push_back(P.fN);
    } else {
      st.root_size = lev.ysum;
      if (prev) prev->panel.release();
    }
  }
  HIF_HIP(hipEventRecord(ev.e[L + 1], s));
  Fi.prepare(s);
  check_errors();
  staging_synced(s);
  for (int level = 0; level <= L; ++level) {
    float ms = 0.f;
    HIF_HIP(hipEventElapsedTime(&ms, ev.e[level], ev.e[level + 1]));
    st.level_seconds[level] = 1e-3 * ms;
  }
  profiler().level = -1;
  st.factor_flops = flops;
  st.build_seconds = now_s() - t_begin;
  st.peak_bytes = mem_stats().peak - mem0;
  F->impl = std::move(impl);
  st.factor_bytes = F->impl->stored_bytes();
}

template <typename T>
int64_t FactorImpl<T>::stored_bytes() const {
  int64_t b = 0;
  for (auto& l : levels) b += (int64_t)(l.front.bytes() + l.skel.bytes());
  return b;
}

template void build_factor<double>(const hif_problem_s*, const hif_options&, hipStream_t,
                                   hif_factor_s*);
template void build_factor<float>(const hif_problem_s*, const hif_options&, hipStream_t,
                                  hif_factor_s*);
template int64_t FactorImpl<double>::stored_bytes() const;
template int64_t FactorImpl<float>::stored_bytes() const;

}  // namespace hif
