// Internal data structures of the HIF library: the operator, the per-level
// factor store and the entry points of the build / apply / solve modules.
#pragma once

#include <memory>
#include <vector>

#include "common.hpp"
#include "dense.hpp"
#include "plan.hpp"

namespace hif {

// 7-point operator: A(p,p) = diag[p]; A(p, p+e_d) = -c_d[p].  Dirichlet:
// c_d = 0 past the last grid line, so the coupling across a wrapped index is
// always zero.  Periodic (n >= 4): at x_d = n-1, c_d[p] couples p to the
// point with x_d = 0 on the same line.
struct Stencil {
  int n;
  int periodic;
  const double* diag;
  const double* cx;
  const double* cy;
  const double* cz;
};

// Face skeleton of one face with r = |F̌| > 0 (k = |F̂| may be 0).  Offsets are
// element offsets into the level's skeleton arena (T: k x r, Lc^{-1}: r x r,
// Y: r x k, all column-major with ld = rows) and into the level's skeleton
// point list (the face's points in pivot order: F̂ then F̌).
struct SkelDesc {
  int face, k, r, pad_;
  int64_t pts_off;
  int64_t offT, offL, offY;
  int64_t kofs, rofs;  // offsets of x_F̂ / x_F̌ in the apply scratch vectors
};

// One triangular block of the forward apply: M (n x n, column-major, ld) is a
// stored inverse L^{-1}; its vector segment starts at off in a scratch array.
struct TrsvDesc {
  const void* M;
  int n, ld;
  int64_t off;
};

// One matrix of a batched matrix-vector product in the sweeps: A (m x n,
// column-major, lower triangular if tri), its row-space vector at roff and
// column-space vector at coff in the scratch arrays.
struct GemvDesc {
  const void* A;
  int m, n, lda, tri;
  int64_t roff, coff;
};

template <typename T>
struct Level {
  std::shared_ptr<const LevelPlan> plan;  // shared: the level-0 plan is cached per problem
  // cells
  DevArr<int> rows;
  DevArr<int64_t> crow_off;
  std::vector<FrontDesc> hfd;
  DevBuf<FrontDesc> fd;
  DevBuf<T> front;  // per cell [L_I^{-1}; L_SI], (nI+nS) x nI column-major
  DevBuf<T> sign;   // root of a periodic problem: S of its L S L^T (+-1 per row)
  DevBuf<int64_t> yoff, zoff;  // per cell offsets into the apply scratch vectors
  std::vector<int64_t> hyoff, hzoff;
  int64_t ysum = 0, zsum = 0;
  int maxI = 0, maxS = 0;
  // faces
  DevArr<int> fpts, fN, fcellA, fcellB, rb_face, rb_off, rb_sa, rb_sb;
  DevArr<int64_t> fpt_off;
  DevBuf<T> panel;  // per face Ã^l([F; other faces of both cells], F)
  DevBuf<int64_t> panel_off;
  DevBuf<int> panel_ld;
  int maxF = 0;
  // skeletons
  std::vector<int> hk;      // rank per face
  DevBuf<int> skpts;        // face points in pivot order (offsets = fpt_off)
  std::vector<SkelDesc> hsk;
  DevBuf<SkelDesc> sk;
  DevBuf<T> skel;
  int maxk = 0, maxr = 0;
  int64_t redundant = 0;
  // algorithmic bytes of one sweep over this level (factor words read once,
  // 8-byte vector entries read and written), for the profiler
  double bytes_L = 0.0, bytes_S = 0.0, bytes_skel = 0.0;
  // sweep descriptors (built at the end of the build)
  bool gv_ready = false;
  bool gv_L_vec = true;  // every L_I^{-1} starts 16-byte aligned (vector row GEMV)
  DevBuf<GemvDesc> gv_L, gv_S, gv_T, gv_Lc, gv_Y;
  int gv_nS = 0;  // cells with nS > 0 (gv_S entries)
  // triangular blocks of the forward apply (built on its first use)
  bool tr_ready = false;
  DevBuf<TrsvDesc> tr_cells, tr_faces;
  int64_t ksum = 0, rsum = 0;
};

struct PcgCache;  // the single-vector PCG's workspace and captured apply graph

// Calls on one factor must not overlap (they share its scratch vectors).
struct FactorBase {
  virtual ~FactorBase() = default;
  std::shared_ptr<PcgCache> pcg;
  virtual void apply(const double* f, double* u, hipStream_t s) = 0;
  // u = F f (the product form of F itself), one vector, FP64 in and out.
  virtual void apply_forward(const double* f, double* u, hipStream_t s) = 0;
  // apply() with its scratch vectors carved out of `scratch` (cap doubles,
  // 256-byte aligned) instead of the factor's own; allocates nothing.
  virtual void apply_scratch(const double* f, double* u, double* scratch, int64_t cap,
                             hipStream_t s) = 0;
  // doubles of scratch apply_scratch needs
  virtual int64_t scratch_doubles() const = 0;
  // u = F^{-1} f for nrhs column-major vectors (leading dimension N) at once.
  virtual void apply_block(const double* f, double* u, int nrhs, hipStream_t s) = 0;
  // algorithmic HBM bytes of one single-vector apply (profiler)
  virtual double apply_bytes() const = 0;
  virtual int64_t stored_bytes() const = 0;
  virtual const LevelPlan& level_plan(int level) const = 0;
};

template <typename T>
struct FactorImpl : FactorBase {
  int n = 0, L = 0;
  int64_t N = 0;
  std::vector<Level<T>> levels;
  DevBuf<double> ybuf, zbuf, xs;  // apply scratch
  DevBuf<double> sbuf;            // skeleton scratch (x_F̂, x_F̌, L_F̌^{-1} x_F̌)
  int64_t ymax = 1, zmax = 1, kmax = 1, rmax = 1;  // scratch segment sizes
  bool prepared = false;
  // Block apply: scratch blocks in the factor's precision (segment sizes as
  // above, one column per right-hand side) and the GEMM descriptors of every
  // sweep step, built once per block width.
  DevBuf<T> mbuf;
  int mbuf_cols = 0;
  struct BlockStep {
    DevBuf<GemmDesc> d;
    int count = 0, max_m = 0, max_n = 0;
    double flops = 0.0;
  };
  enum { kStepL, kStepS, kStepT1, kStepLc1, kStepY1, kStepY2, kStepLc2, kStepT2, kStepS2,
         kStepL2, kSteps };
  std::vector<std::vector<BlockStep>> bsteps;  // [level][step], for bsteps_cols columns
  int bsteps_cols = 0;
  // Sweep descriptors and scratch of the apply (idempotent).
  void prepare(hipStream_t s);
  void apply(const double* f, double* u, hipStream_t s) override;
  void apply_forward(const double* f, double* u, hipStream_t s) override;
  void apply_scratch(const double* f, double* u, double* scratch, int64_t cap,
                     hipStream_t s) override;
  int64_t scratch_doubles() const override;
  // Multiply the root's rows of ncol vectors (leading dimension ldu) by the
  // signs of its L S L^T (a no-op unless the root is a periodic problem's).
  void root_sign(double* u, int64_t ldu, int ncol, hipStream_t s);
  // The single-vector sweeps on the given scratch segments: xi, yv (ymax
  // each), zv, xsv (zmax each), sh (kmax), sc, sc2 (rmax each).
  void sweep(const double* f, double* u, double* xi, double* yv, double* zv, double* xsv,
             double* sh, double* sc, double* sc2, hipStream_t s);
  void apply_block(const double* f, double* u, int nrhs, hipStream_t s) override;
  double apply_bytes() const override;
  int64_t stored_bytes() const override;
  const LevelPlan& level_plan(int level) const override { return *levels[level].plan; }
};

}  // namespace hif

struct hif_problem_s {
  hif_options opts;
  int n = 0;
  int64_t N = 0;
  hif::DevBuf<double> diag, cx, cy, cz;
  // cell/face geometry of every level, computed on the first build with a leaf
  mutable int geom_leaf = -1;
  mutable std::vector<hif::LevelGeom> geom;
  mutable std::shared_ptr<const hif::LevelPlan> plan0;  // level 0: every point active
  // device copies of plan0's index arrays
  struct Level0Arrays {
    hif::DevArr<int> rows, fpts, fN, fcellA, fcellB, rb_face, rb_off, rb_sa, rb_sb;
    hif::DevArr<int64_t> crow_off, fpt_off;
  };
  mutable Level0Arrays dev0;
  hif::Stencil stencil() const {
    return {n, opts.bc == HIF_PERIODIC ? 1 : 0, diag.get(), cx.get(), cy.get(), cz.get()};
  }
};

struct hif_factor_s {
  hif_options opts;
  std::unique_ptr<hif::FactorBase> impl;
  hif_stats stats;
  std::vector<std::vector<int>> redundant_pts;  // per level l < L: points left out by the ID
  std::vector<std::vector<int>> ranks, sizes;  // per level l < L
};

namespace hif {

void problem_assemble(hif_problem_s* A, const double* a, const double* b, hipStream_t s);
void stencil_matvec(const Stencil& st, const double* x, double* y, hipStream_t s);

template <typename T>
void build_factor(const hif_problem_s* A, const hif_options& o, hipStream_t s, hif_factor_s* F);

// One problem of a batched build: its operator, options and the factor to fill.
struct BuildRequest {
  const hif_problem_s* A;
  hif_options o;
  hif_factor_s* F;
};

// Factors every request (same precision T and eps; grids and leaf sizes may
// differ) with joint launches per level.
template <typename T>
void build_factors(const std::vector<BuildRequest>& req, hipStream_t s);

// Factor files: save F (blocks copied to the host, then written), or fill
// an empty F from a file (plans and layouts rebuilt, blocks uploaded).
void factor_save(const hif_factor_s* F, const char* path, hipStream_t s);
void factor_load(const char* path, hipStream_t s, hif_factor_s* F);

// e_s = ||x - F^{-1}A x|| / ||x|| and, for power_iters > 0, the power-method
// estimate of ||I - F^{-1}A||_2 started at x (NaN for power_iters = 0).
void factor_error(const hif_problem_s* A, hif_factor_s* F, const double* x, int power_iters,
                  double* e_s, double* err_norm, hipStream_t s);

// Device inner product a.(b - c) (c may be null) into *out (device), FP64,
// in a fixed reduction order.
void device_dot(const double* a, const double* b, const double* c, int64_t N, double* out,
                hipStream_t s);

// u = F^{-1} f with every scratch vector in the library's static device
// array (one per GPU, kNoAllocScratchBytes); allocates nothing.
void apply_noalloc(hif_factor_s* F, const double* f, double* u, hipStream_t s);
constexpr int64_t kNoAllocScratchBytes = int64_t(64) << 20;

// Restarted flexible GMRES(restart) with F^{-1} as a right preconditioner,
// from u = 0, to a true relative residual <= tol (info->iters counts Arnoldi
// steps over all cycles).
void gmres_solve(const hif_problem_s* A, hif_factor_s* F, const double* f, double* u, double tol,
                 int restart, int maxit, hif_pcg_info* info, hipStream_t s);

void pcg_solve(const hif_problem_s* A, hif_factor_s* F, const double* f, double* u, double tol,
               int maxit, hif_pcg_info* info, hipStream_t s);
void pcg_solve_block(const hif_problem_s* A, hif_factor_s* F, const double* f, double* u, int nrhs,
                     double tol, int maxit, hif_pcg_info* info, hipStream_t s);
// One single-vector PCG per problem, run concurrently by host worker threads,
// each on a stream of its own ordered after s; s waits for all of them.
void pcg_solve_batched(int count, hif_problem_s* const* A, hif_factor_s* const* F,
                       const double* const* f, double* const* u, double tol, int maxit,
                       hif_pcg_info* info, hipStream_t s);

}  // namespace hif
