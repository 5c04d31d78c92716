// Batched dense kernels for the HIF fronts (gfx950).
//
//   * gemm_batched: C_b = alpha op(A_b) op(B_b) + beta C_b over a batch of
//     independently sized problems, 64x64 tiles on MFMA (FP64 16x16x4 or FP32
//     16x16x4), optional triangular masks on the operands and on C.
//   * front_factor: per front [A_II; A_SI] ((nI+nS) x nI, column-major), a
//     blocked right-looking Cholesky of the first nI columns (L_I and
//     L_SI = A_SI L_I^{-T}), then an in-place blocked inverse of L_I.
//   * pivoted_cholesky: greedy diagonal-pivoted Cholesky of a Gram matrix in
//     FP64, stopped at relative precision eps (rank-revealing, equivalent to
//     column-pivoted QR of the Gram's factor).
#pragma once

#include "common.hpp"

namespace hif {

enum : int { OP_N = 0, OP_T = 1 };

// Triangular structure of the logical operands op(A) (m x k), op(B) (k x n)
// and of the written part of C.  Masked operand entries read as zero, so the
// unreferenced triangle of a stored factor may hold anything.
enum : int {
  GF_A_LOWER = 1,   // op(A)(i,t) = 0 for t > i
  GF_A_UPPER = 2,   // op(A)(i,t) = 0 for t < i
  GF_B_LOWER = 4,   // op(B)(t,j) = 0 for t < j
  GF_B_UPPER = 8,   // op(B)(t,j) = 0 for t > j
  GF_C_LOWER = 16,  // only C(i,j) with i >= j is computed and written
  GF_C_MIRROR = 32, // with GF_C_LOWER (square C): C(j,i) is written too
  GF_TRI_ZEROS = 64, // the entries that GF_A_* / GF_B_* mask are stored as zeros, so the
                     // masks only shorten the K range of a tile
};

struct GemmDesc {
  const void* A;
  const void* B;
  void* C;
  int m, n, k;
  int lda, ldb, ldc;
};

// TIn: element type of A and B; TC: accumulation and C type.
enum : int { GC_GENERIC = 0, GC_SYRK = 1, GC_LSI = 2, GC_GRAM = 3 };  // kernel symbol per use

template <typename TIn, typename TC>
void gemm_batched(int opa, int opb, int flags, const GemmDesc* d_desc, int batch, int max_m,
                  int max_n, TC alpha, TC beta, hipStream_t s, const char* name = "gemm",
                  double flops = 0.0, int cls = GC_GENERIC, bool ld16 = false);

// Algorithmic flops of one descriptor under the triangular flags (one flag class).
double gemm_flops(const GemmDesc& d, int flags);

// The batch reordered (and padded with empty products) so that the eighths
// of it that the batched GEMM gives the eight XCDs cost the same; only the
// order of independent products changes.
std::vector<GemmDesc> balance_xcds(const std::vector<GemmDesc>& h, int flags);

// Tile autotuning on a real workload: between tune_begin() and tune_end(),
// every batched GEMM that overwrites its output is run and timed with each
// candidate tile; tune_end() picks the fastest tile per key (summed device
// time), writes the table to `path` (if not empty), makes it the table in use
// and returns the number of keys.
void tune_begin();
int tune_end(const char* path);

// Batched out-of-place transpose: dst (cols x rows, leading dimension ldd) =
// src (rows x cols, leading dimension lds)^T, column-major.
struct TransDesc {
  const void* src;
  void* dst;
  int rows, cols, lds, ldd;
};
template <typename T>
void transpose_batched(const TransDesc* d_desc, int batch, int max_rows, int max_cols,
                       hipStream_t s, const char* name = "transpose");

// One front: device address of its column-major block, interior count nI,
// total rows nR = nI + nS, leading dimension ld >= nR, and the id that a
// failed factorization reports.  Fronts of one batch may live in different
// allocations (for instance, of different problems).
struct FrontDesc {
  void* ptr;
  int nI, nR, ld;
  int id;
};

constexpr int kPanel = 64;  // block width of the blocked factorizations

// Partial Cholesky of the first nI columns of every front (rows nI..nR-1 get
// A_SI L_I^{-T}), then L_I <- L_I^{-1} in place.  err[0] receives the smallest
// id of a front with a non-positive pivot (untouched otherwise).  upper_zero:
// the strict upper triangle of every nI x nI block is stored as zeros (the
// factorization keeps it so, and the inverse can then skip its masks).
// small_limit: fronts of at most this many interior columns are factored one
// per workgroup (one launch), larger ones by blocked steps batched over the
// fronts.  One workgroup per front pays off for the thousands of cell fronts
// of the leaf level and for the redundant blocks of faces; the few hundred
// cell fronts of 300-800 columns one level up leave most of the chip idle
// that way.  The limit depends on the level and the kind of front only, so a
// front takes the same kernels in a single and in a batched build.  band > 0
// (with upper_zero): every L_I is known to be zero more than band rows below
// its diagonal (the leaf fronts), which the inverse uses to shorten its
// products.
constexpr int kSmallFrontLeaf = 512, kSmallFrontUpper = 256;

template <typename T>
void front_factor(const FrontDesc* d_fronts, const std::vector<FrontDesc>& h_fronts,
                  int* err, hipStream_t s, bool upper_zero, int small_limit, int band = 0);

// Signed LDL^T of one dense front f (nI x nI, no shell rows, strict upper
// triangle stored as zeros; d_front is f on the device): f <- L^{-1} in place
// and sgn[0..nI) <- S, where A = L S L^T with S = diag(+-1) and L lower
// triangular with a positive diagonal (unpivoted; the paper's LDL^T stored as
// L_unit |D|^{1/2} and sign(D)).  A zero pivot sets *err to f.id.
template <typename T>
void root_ldl(const FrontDesc& f, const FrontDesc* d_front, T* sgn, int* err, hipStream_t s);

// Only the in-place inverse of an already factored lower-triangular L_I
// (band as for front_factor; diag_done: its 64 x 64 diagonal blocks already
// hold their inverses).
template <typename T>
void front_invert(const FrontDesc* d_fronts, const std::vector<FrontDesc>& h_fronts,
                  hipStream_t s, bool upper_zero, int band = 0, bool diag_done = false);

// Pivoted Cholesky of each symmetric G_b (nF x nF, FP64, offset goff[b], ld
// ldg[b]), blocked: G is overwritten by its trailing updates.  Writes the
// pivot columns L (same layout as G; column j = j-th pivot, rows in original
// order, zero on rows pivoted earlier), perm (nF entries at poff[b]: pivots,
// then the unpivoted indices ascending) and the rank k[b].  eps > 0.
constexpr int kPcholMax = 4096;
void pivoted_cholesky(double* G, double* L, const int64_t* goff, const int* nF, const int* ldg,
                      const int64_t* poff, int* perm, int* k, int batch, double eps,
                      const std::vector<int>& h_nF, const std::vector<int64_t>& h_goff,
                      const std::vector<int>& h_ldg, const std::vector<int64_t>& h_poff,
                      hipStream_t s);

}  // namespace hif
