// Batched dense kernels for the HIF fronts on gfx950 (CDNA4, wave64).
#include <algorithm>
#include <climits>
#include <cfloat>

#include "dense.hpp"

#include <dlfcn.h>

#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <type_traits>
#include "prof.hpp"

namespace hif {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// 16x16x4 MFMA.  Lane l supplies A(l%16, l/16) and B(l/16, l%16).  Result
// element v of lane l is C(row(l, v), l%16): row = l/16 + 4v for FP64 and
// 4(l/16) + v for FP32 (measured on gfx950).
template <typename TC>
struct Mfma;
template <>
struct Mfma<double> {
  typedef d4 acc_t;
  static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct Mfma<float> {
  typedef f4 acc_t;
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

constexpr int BM = 64, BN = 64, KC = 16, NTHR = 256;
constexpr int kMaxGridY = 65535;  // largest y or z dimension of a launch grid

// LDS staging of one K chunk: As[k][m], Bs[k][n], rows padded by one element
// so that stores along k (transposed operands) do not collide in banks.
template <typename TC, int TM, int TN>
struct TileSmem {
  static constexpr int NBUF = sizeof(TC) * (TM + TN + 2) * KC * 2 <= 36 * 1024 ? 2 : 1;
  TC As[NBUF][KC][TM + 1];
  TC Bs[NBUF][KC][TN + 1];
};

// One TM x TN tile of C = alpha op(A) op(B) + beta C by 256 threads: four
// waves in a 2 x 2 arrangement, each owning (TM/2) x (TN/2) as 16 x 16 MFMA
// blocks.  K is staged through LDS in chunks of 16 with a register prefetch of
// the next chunk.  Masked operand entries (triangular flags, out of range)
// read as zero.
template <typename TIn, typename TC, int OPA, int OPB, int TM, int TN>
__device__ __forceinline__ void gemm_tile_t(int flags, const TIn* A, int lda, const TIn* __restrict__ B, int ldb,
                            TC* C, int ldc, int m, int n, int k, int m0, int n0, TC alpha, TC beta,
                            TileSmem<TIn, TM, TN>& sm) {
  const auto gA = as_global(A);
  const auto gB = as_global(B);
  const auto gC = as_global(C);
  constexpr int FM = TM / 32, FN = TN / 32;        // 16x16 blocks per wave
  constexpr int LA = TM * KC / NTHR, LB = TN * KC / NTHR;  // loads per thread
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  int kb = 0, ke = k;
  if (flags & GF_A_LOWER) ke = min(ke, m0 + TM);
  if (flags & GF_A_UPPER) kb = max(kb, m0);
  if (flags & GF_B_LOWER) kb = max(kb, n0);
  if (flags & GF_B_UPPER) ke = min(ke, n0 + TN);
  const int nchunk = ke > kb ? (ke - kb + KC - 1) / KC : 0;

  typename Mfma<TC>::acc_t acc[FM][FN];
#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int y = 0; y < FN; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[x][y][v] = TC(0);

  // Element coordinates of this thread's loads inside a chunk (fixed for the
  // tile): along the operand's contiguous dimension, consecutive threads.
  static_assert(NTHR % TM == 0 && NTHR % TN == 0 && NTHR % KC == 0, "load mapping");
  int ai[LA], at[LA], bj[LB], bt[LB];
#pragma unroll
  for (int r = 0; r < LA; ++r) {
    if (OPA == OP_N) { ai[r] = tid % TM; at[r] = tid / TM + (NTHR / TM) * r; }
    else { at[r] = tid % KC; ai[r] = tid / KC + (NTHR / KC) * r; }
  }
#pragma unroll
  for (int r = 0; r < LB; ++r) {
    if (OPB == OP_N) { bt[r] = tid % KC; bj[r] = tid / KC + (NTHR / KC) * r; }
    else { bj[r] = tid % TN; bt[r] = tid / TN + (NTHR / TN) * r; }
  }
  // Byte offsets of those elements from the chunk's corner: a chunk that needs
  // no masking is then one load instruction per element off a uniform base.
  // Rows past m (columns past n) are clamped onto the last one: they only
  // feed entries of C that are never written.
  uint32_t oa[LA], ob[LB];
#pragma unroll
  for (int r = 0; r < LA; ++r) {
    const int i = min(ai[r], m - 1 - m0);
    oa[r] = (uint32_t)((OPA == OP_N ? i + lda * at[r] : at[r] + lda * i) * sizeof(TIn));
  }
#pragma unroll
  for (int r = 0; r < LB; ++r) {
    const int j = min(bj[r], n - 1 - n0);
    ob[r] = (uint32_t)((OPB == OP_N ? bt[r] + ldb * j : j + ldb * bt[r]) * sizeof(TIn));
  }
  auto clean = [&](int t0) {
    bool c = t0 + KC <= ke;
    if (flags & GF_TRI_ZEROS) return c;
    if (flags & GF_A_LOWER) c = c && t0 + KC - 1 <= m0;
    if (flags & GF_A_UPPER) c = c && t0 >= m0 + TM - 1;
    if (flags & GF_B_LOWER) c = c && t0 >= n0 + TN - 1;
    if (flags & GF_B_UPPER) c = c && t0 + KC - 1 <= n0;
    return c;
  };

  TIn ra[LA], rb[LB];  // operands stay in their own type until the MFMA reads them
  auto load = [&](int c) {
    const int t0 = kb + c * KC;
    if (clean(t0)) {
      const TIn* ca = OPA == OP_N ? A + m0 + (int64_t)lda * t0 : A + t0 + (int64_t)lda * m0;
      const TIn* cb = OPB == OP_N ? B + t0 + (int64_t)ldb * n0 : B + n0 + (int64_t)ldb * t0;
#pragma unroll
      for (int r = 0; r < LA; ++r) ra[r] = load_global(ca, oa[r]);
#pragma unroll
      for (int r = 0; r < LB; ++r) rb[r] = load_global(cb, ob[r]);
      return;
    }
#pragma unroll
    for (int r = 0; r < LA; ++r) {
      const int gi = m0 + ai[r], gt = t0 + at[r];
      bool ok = gi < m && gt < ke;
      if (flags & GF_A_LOWER) ok = ok && gt <= gi;
      if (flags & GF_A_UPPER) ok = ok && gt >= gi;
      TIn v = TIn(0);
      if (ok) v = OPA == OP_N ? gA[gi + (int64_t)lda * gt] : gA[gt + (int64_t)lda * gi];
      ra[r] = v;
    }
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      const int gj = n0 + bj[r], gt = t0 + bt[r];
      bool ok = gj < n && gt < ke;
      if (flags & GF_B_LOWER) ok = ok && gt >= gj;
      if (flags & GF_B_UPPER) ok = ok && gt <= gj;
      TIn v = TIn(0);
      if (ok) v = OPB == OP_N ? gB[gt + (int64_t)ldb * gj] : gB[gj + (int64_t)ldb * gt];
      rb[r] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int r = 0; r < LA; ++r) sm.As[buf][at[r]][ai[r]] = ra[r];
#pragma unroll
    for (int r = 0; r < LB; ++r) sm.Bs[buf][bt[r]][bj[r]] = rb[r];
  };
  auto compute = [&](int buf) {
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const int kk = 4 * s + (lane >> 4);
      TC av[FM], bv[FN];
#pragma unroll
      for (int x = 0; x < FM; ++x) av[x] = (TC)sm.As[buf][kk][wm * (TM / 2) + 16 * x + (lane & 15)];
#pragma unroll
      for (int y = 0; y < FN; ++y) bv[y] = (TC)sm.Bs[buf][kk][wn * (TN / 2) + 16 * y + (lane & 15)];
#pragma unroll
      for (int x = 0; x < FM; ++x)
#pragma unroll
        for (int y = 0; y < FN; ++y) acc[x][y] = Mfma<TC>::run(av[x], bv[y], acc[x][y]);
    }
  };

  if (nchunk > 0) {
    if constexpr (TileSmem<TIn, TM, TN>::NBUF == 2) {
      load(0);
      store(0);
      __syncthreads();
      for (int c = 0; c < nchunk; ++c) {
        const int buf = c & 1;
        if (c + 1 < nchunk) load(c + 1);
        // keep the next chunk's global loads issued ahead of this chunk's MFMAs,
        // and let this wave's MFMA phase take issue priority over the other
        // waves' load and store phases
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_setprio(1);
        compute(buf);
        __builtin_amdgcn_s_setprio(0);
        __builtin_amdgcn_sched_barrier(0);
        if (c + 1 < nchunk) store(buf ^ 1);
        __syncthreads();
      }
    } else {
      load(0);
      for (int c = 0; c < nchunk; ++c) {
        store(0);
        __syncthreads();
        if (c + 1 < nchunk) load(c + 1);
        __builtin_amdgcn_sched_barrier(0);
        compute(0);
        __syncthreads();
      }
    }
  }

#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int y = 0; y < FN; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = m0 + wm * (TM / 2) + x * 16 + Mfma<TC>::row(lane, v);
        const int gj = n0 + wn * (TN / 2) + y * 16 + (lane & 15);
        if (gi < m && gj < n && (!(flags & GF_C_LOWER) || gi >= gj)) {
          const int64_t idx = gi + (int64_t)ldc * gj;
          TC val = alpha * acc[x][y][v];
          if (beta != TC(0)) val += beta * gC[idx];
          gC[idx] = val;
          if ((flags & GF_C_MIRROR) && gi > gj) gC[gj + (int64_t)ldc * gi] = val;
        }
      }
}

// CLS only gives each use (generic, Schur SYRK, L_SI, Gram) its own kernel
// symbol for profilers.
// Workgroups are dealt to the 8 XCDs round-robin; remap the linear block id
// so that each XCD runs a contiguous range of tiles (neighbouring tiles share
// A and B panels in that XCD's L2).  A batch whose count is a multiple of 8
// thus gives XCD x its x-th eighth of the products, which the host orders to
// balance the eighths' costs.
__device__ __forceinline__ void xcd_remap(unsigned& bx, unsigned& by, unsigned& bz) {
  const unsigned gx = gridDim.x, gy = gridDim.y;
  const unsigned T = gx * gy * gridDim.z;
  unsigned L = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const unsigned per = T / 8;
  if (L < 8 * per) L = (L % 8) * per + L / 8;
  bx = L % gx;
  by = (L / gx) % gy;
  bz = L / (gx * gy);
}

template <typename TIn, typename TC, int OPA, int OPB, int TM, int TN, int CLS>
__global__ __launch_bounds__(NTHR) void k_gemm_desc(int flags, const GemmDesc* __restrict__ desc,
                                                    TC alpha, TC beta) {
  __shared__ TileSmem<TIn, TM, TN> sm;
  unsigned bx, by, bz;
  xcd_remap(bx, by, bz);
  const GemmDesc d = desc[bz];
  const int m0 = by * TM, n0 = bx * TN;
  if (m0 >= d.m || n0 >= d.n) return;
  if ((flags & GF_C_LOWER) && m0 + TM - 1 < n0) return;
  gemm_tile_t<TIn, TC, OPA, OPB, TM, TN>(flags, (const TIn*)d.A, d.lda, (const TIn*)d.B, d.ldb,
                                         (TC*)d.C, d.ldc, d.m, d.n, d.k, m0, n0, alpha, beta, sm);
}

// ---- GEMM tile fed by 16-byte direct-to-LDS loads ------------------------
//
// C = alpha A B^T + beta C for an A (m x k) and a B (n x k) whose columns are
// contiguous (op(A) = A, op(B) = B^T: the Schur SYRK and the L_SI product).
// Square TS x TS tiles (TS = 128 or 64 for FP32, 64 for FP64) on four waves in
// a 2 x 2 arrangement, each wave FM = TS / 32 blocks of 16 rows by FM blocks of
// 16 columns.  K runs in chunks of kDmaK through kDmaStages LDS stages that
// global_load_lds_dwordx4 fills without passing through registers: the next
// chunk is in flight while one is multiplied, with one barrier per chunk.
// A stage holds each operand as [k][TS] rows.  Block x of a wave's FM row
// blocks takes rows FM i + x (i = lane % 16), so a lane reads the operands of
// all FM blocks with one LDS read of FM consecutive values, and output row r
// of block x is row FM r + x of the wave's sub-tile (columns likewise).
// Leading dimensions must be multiples of V = 16 / sizeof(T).  A pointer off
// the 16-byte grid shifts the tile grid by its offset: the rows before it
// belong to the same 16-byte block, are read and never written; rows past m
// are clamped to the last 16-byte block that holds a valid row, and k past
// the chunk range to the last valid column (masked to zero before the MFMA).
constexpr int kDmaK = 16, kDmaStages = 2;

template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// One 16-byte global -> LDS copy per lane: lane l writes bytes [16 l, 16 l + 16)
// after the wave-uniform LDS address lds.  (A plain device function: inside a
// kernel template the target builtin would keep the host stub from being
// emitted.)
__device__ __forceinline__ void dma16(const void* g, void* lds) {
  __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}

template <typename T, int TS>
struct DmaSmem {
  static constexpr int V = 16 / (int)sizeof(T);         // values per 16 bytes
  static constexpr int FM = TS / 32;                    // row blocks per wave
  static constexpr int LPR = TS * (int)sizeof(T) / 16;  // DMA lanes per k row
  static constexpr int KPI = 64 / LPR;                  // k rows per DMA instruction
  static constexpr int IPW = kDmaK / KPI / 2;           // DMA instructions per chunk and wave
  static constexpr int SW = TS / 2;  // rows (and columns) of a wave's sub-tile
  static constexpr int EC = 32;      // sub-tile columns per epilogue pass
  union __align__(16) {
    T op[kDmaStages][2][kDmaK][TS];  // [stage][A, B][k][row]
    T epi[4][EC][SW + 1];            // [wave][column][row], staged outputs
  };
};

// Four workgroups per CU (at most 128 VGPRs): four waves per SIMD keep the
// matrix pipe fed across the per-chunk barriers.
template <typename T, int TS, int CLS>
__global__ __launch_bounds__(NTHR, 4) void k_gemm_nt(int flags, const GemmDesc* __restrict__ desc,
                                                     T alpha, T beta) {
  using S = DmaSmem<T, TS>;
  constexpr int V = S::V, FM = S::FM, LPR = S::LPR, KPI = S::KPI, IPW = S::IPW;
  typedef T vec_t __attribute__((ext_vector_type(FM)));
  __shared__ S sm;
  unsigned bx, by, bz;
  xcd_remap(bx, by, bz);
  const GemmDesc d = desc[bz];
  const int offA = (int)(((uintptr_t)d.A / sizeof(T)) % V);
  const int offB = (int)(((uintptr_t)d.B / sizeof(T)) % V);
  const int ms = d.m + offA, ns = d.n + offB;  // extents in the shifted grid
  const int m0s = by * TS, n0s = bx * TS;
  if (m0s >= ms || n0s >= ns) return;
  const int m0 = m0s - offA, n0 = n0s - offB;  // C coordinates of the tile corner
  if ((flags & GF_C_LOWER) && m0 + TS - 1 < n0) return;
  // triangular operands arrive with their zeros stored: only the K range shrinks
  int kb = 0, ke = d.k;
  if (flags & GF_A_LOWER) ke = min(ke, m0 + TS);
  if (flags & GF_A_UPPER) kb = max(kb, m0);
  if (flags & GF_B_LOWER) kb = max(kb, n0);
  if (flags & GF_B_UPPER) ke = min(ke, n0 + TS);
  const int nchunk = ke > kb ? (ke - kb + kDmaK - 1) / kDmaK : 0;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;

  // This wave's IPW DMA instructions per chunk: operand (wave >> 1) (A for
  // waves 0-1, B for 2-3), the half (wave & 1) of the chunk's k rows, KPI k
  // rows an instruction, 16-byte block lane % LPR of the row.
  const int opnd = wave >> 1;
  const T* base = opnd == 0 ? static_cast<const T*>(d.A) - offA : static_cast<const T*>(d.B) - offB;
  const int ld = opnd == 0 ? d.lda : d.ldb;
  const int qmax = ((opnd == 0 ? ms : ns) - 1) / V;
  const int q = min((opnd == 0 ? m0s : n0s) / V + lane % LPR, qmax);
  const T* src = base + (int64_t)V * q;
  const int krow0 = (kDmaK / 2) * (wave & 1) + lane / LPR;
  auto issue = [&](int c) {
    const int st = c % kDmaStages;
    const int t0 = kb + c * kDmaK;
#pragma unroll
    for (int j = 0; j < IPW; ++j) {
      const int kr = krow0 + KPI * j;
      const int kk = min(t0 + kr, ke - 1);
      dma16(src + (int64_t)ld * kk, &sm.op[st][opnd][(kDmaK / 2) * (wave & 1) + KPI * j][0]);
    }
  };

  typename Mfma<T>::acc_t acc[FM][FM];
#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int y = 0; y < FM; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[x][y][v] = T(0);

  const int ra = wm * (TS / 2) + FM * (lane & 15);
  const int rb = wn * (TS / 2) + FM * (lane & 15);
#pragma unroll
  for (int c = 0; c < kDmaStages - 1; ++c)
    if (c < nchunk) issue(c);
  for (int c = 0; c < nchunk; ++c) {
    // chunk c landed; the later chunks already issued may still fly
    if (c + kDmaStages - 2 < nchunk)
      wait_vmcnt<(kDmaStages - 2) * IPW>();
    else
      wait_vmcnt<0>();
    asm volatile("s_barrier" ::: "memory");  // every wave's part of chunk c is in LDS
    // into the stage freed by chunk c - 1
    if (c + kDmaStages - 1 < nchunk) issue(c + kDmaStages - 1);
    const int st = c % kDmaStages;
    const int kvalid = ke - (kb + c * kDmaK);  // k rows of this chunk inside [kb, ke)
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int s4 = 0; s4 < kDmaK / 4; ++s4) {
      const int kr = 4 * s4 + (lane >> 4);
      vec_t a = *reinterpret_cast<const vec_t*>(&sm.op[st][0][kr][ra]);
      vec_t b = *reinterpret_cast<const vec_t*>(&sm.op[st][1][kr][rb]);
      if (kr >= kvalid) {
        a = vec_t(T(0));
        b = vec_t(T(0));
      }
#pragma unroll
      for (int x = 0; x < FM; ++x)
#pragma unroll
        for (int y = 0; y < FM; ++y) acc[x][y] = Mfma<T>::run(a[x], b[y], acc[x][y]);
    }
    __builtin_amdgcn_s_setprio(0);
  }

  // Epilogue through LDS, EC sub-tile columns at a time: each column goes out
  // with consecutive rows on consecutive lanes, and (GF_C_MIRROR) each
  // mirrored row with consecutive columns on consecutive lanes, so that the
  // stores fill whole cache lines.
  constexpr int SW = S::SW, EC = S::EC;
  asm volatile("s_barrier" ::: "memory");  // every wave is done with the stages
  T(*E)[SW + 1] = sm.epi[wave];
  T* C = static_cast<T*>(d.C);
  const int rbase = m0 + wm * SW, cbase = n0 + wn * SW;
  const bool lower = (flags & GF_C_LOWER) != 0, mirror = (flags & GF_C_MIRROR) != 0;
#pragma unroll
  for (int p = 0; p < SW / EC; ++p) {
#pragma unroll
    for (int x = 0; x < FM; ++x)
#pragma unroll
      for (int y = 0; y < FM; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int cl = FM * (lane & 15) + y - EC * p;
          if (cl >= 0 && cl < EC) E[cl][FM * Mfma<T>::row(lane, v) + x] = acc[x][y][v];
        }
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    constexpr int CPI = 64 / SW;  // columns per store (1 or 2)
    {
      const int rl = lane % SW;
      const int gi = rbase + rl;
      for (int j = lane / SW; j < EC; j += CPI) {
        const int gj = cbase + EC * p + j;
        if (gi >= 0 && gj >= 0 && gi < d.m && gj < d.n && (!lower || gi >= gj)) {
          const int64_t idx = gi + (int64_t)d.ldc * gj;
          T val = alpha * E[j][rl];
          if (beta != T(0)) val += beta * C[idx];
          C[idx] = val;
        }
      }
    }
    if (mirror) {  // (only with beta = 0: the lower entries are already overwritten)
      constexpr int RPI = 64 / EC;  // rows per store
      const int jl = lane % EC;
      const int gj = cbase + EC * p + jl;
      for (int r = lane / EC; r < SW; r += RPI) {
        const int gi = rbase + r;
        if (gi >= 0 && gj >= 0 && gi < d.m && gj < d.n && gi > gj)
          C[gj + (int64_t)d.ldc * gi] = alpha * E[jl][r];
      }
    }
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");  // E is rewritten next
  }
}

// LDS of the DMA-fed A B tile (both column-major, B's columns contiguous in
// k): A as in the A B^T tile, [k][row]; B by 16-byte blocks of k, block kb of
// column n at slot BPC n + (kb ^ swz(n)), so that the 16 lanes that read one k
// of columns n = i + 16 y (i = 0 .. 15) meet distinct banks.
template <typename T, int TS>
struct NnSmem {
  static constexpr int V = 16 / (int)sizeof(T);         // values per 16 bytes
  static constexpr int FM = TS / 32;                    // row (column) blocks per wave
  static constexpr int LPR = TS * (int)sizeof(T) / 16;  // A: DMA lanes per k row
  static constexpr int KPI = 64 / LPR;                  // A: k rows per DMA instruction
  static constexpr int IPW = kDmaK / KPI / 2;           // A: DMA instructions per chunk and wave
  static constexpr int BPC = kDmaK / V;                 // B: 16-byte blocks per column and chunk
  static constexpr int BIW = TS * BPC / 64 / 2;         // B: DMA instructions per chunk and wave
  static constexpr int SWS = BPC == 4 ? 2 : 1;          // B: log2 columns per 256 bytes of banks
  static constexpr int SW = TS / 2;
  static constexpr int EC = 32;
  struct Ops {
    T a[kDmaStages][kDmaK][TS];
    T b[kDmaStages][TS * kDmaK];
  };
  union __align__(16) {
    Ops op;
    T epi[4][EC][SW + 1];
  };
  static __device__ __forceinline__ int swz(int n) { return (n >> SWS) & (BPC - 1); }
};

// C = alpha A B + beta C on DMA-fed TS x TS tiles: the A B^T tile's pipeline
// (K in 16-wide chunks through two LDS stages, one barrier per chunk, A rows
// on the shifted grid), with B taken by 16-byte k blocks of its columns (B on
// the 16-byte grid).  Lane i of a 16-lane group multiplies rows FM i + x of A
// by columns i + 16 y of B; the K order is that of the other tiles.
template <typename T, int TS>
__global__ __launch_bounds__(NTHR, 4) void k_gemm_nn(int flags, const GemmDesc* __restrict__ desc,
                                                     T alpha, T beta) {
  using S = NnSmem<T, TS>;
  constexpr int V = S::V, FM = S::FM, LPR = S::LPR, KPI = S::KPI, IPW = S::IPW;
  constexpr int BPC = S::BPC, BIW = S::BIW;
  static_assert(IPW == BIW, "both operand halves take the same DMA count");
  typedef T vec_t __attribute__((ext_vector_type(FM)));
  __shared__ S sm;
  unsigned bx, by, bz;
  xcd_remap(bx, by, bz);
  const GemmDesc d = desc[bz];
  const int offA = (int)(((uintptr_t)d.A / sizeof(T)) % V);
  const int ms = d.m + offA;  // rows in the shifted grid
  const int m0s = by * TS, n0 = bx * TS;
  if (m0s >= ms || n0 >= d.n) return;
  const int m0 = m0s - offA;
  if ((flags & GF_C_LOWER) && m0 + TS - 1 < n0) return;
  int kb = 0, ke = d.k;  // (kb stays on the 16-byte grid: no A-upper mask here)
  if (flags & GF_A_LOWER) ke = min(ke, m0 + TS);
  if (flags & GF_B_LOWER) kb = max(kb, n0);
  if (flags & GF_B_UPPER) ke = min(ke, n0 + TS);
  const int nchunk = ke > kb ? (ke - kb + kDmaK - 1) / kDmaK : 0;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const int half = wave & 1;

  // waves 0-1: A, as in the A B^T tile; waves 2-3: B, slots 64 I + lane of
  // instruction I = BIW half + j
  const bool opa = wave < 2;
  const T* baseA = static_cast<const T*>(d.A) - offA;
  const int qa = min(m0s / V + lane % LPR, (ms - 1) / V);
  const T* srcA = baseA + (int64_t)V * qa;
  const int krow0 = (kDmaK / 2) * half + lane / LPR;
  const T* B = static_cast<const T*>(d.B);
  const int kqmax = ((ke - 1) / V) * V;  // start of the last 16-byte k block holding a value
  auto issue = [&](int c) {
    const int st = c % kDmaStages;
    const int t0 = kb + c * kDmaK;
    if (opa) {
#pragma unroll
      for (int j = 0; j < IPW; ++j) {
        const int kr = krow0 + KPI * j;
        const int kk = min(t0 + kr, ke - 1);
        dma16(srcA + (int64_t)d.lda * kk, &sm.op.a[st][(kDmaK / 2) * half + KPI * j][0]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < BIW; ++j) {
        const int I = BIW * half + j;
        const int slot = 64 * I + lane;
        const int n = slot / BPC;
        const int blk = (slot % BPC) ^ S::swz(n);
        const int gn = min(n0 + n, d.n - 1);
        const int gk = min(t0 + V * blk, kqmax);
        dma16(B + (int64_t)d.ldb * gn + gk, &sm.op.b[st][64 * V * I]);
      }
    }
  };

  typename Mfma<T>::acc_t acc[FM][FM];
#pragma unroll
  for (int x = 0; x < FM; ++x)
#pragma unroll
    for (int y = 0; y < FM; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[x][y][v] = T(0);

  const int ra = wm * (TS / 2) + FM * (lane & 15);
  const int cb = wn * (TS / 2) + (lane & 15);  // columns cb + 16 y
#pragma unroll
  for (int c = 0; c < kDmaStages - 1; ++c)
    if (c < nchunk) issue(c);
  for (int c = 0; c < nchunk; ++c) {
    if (c + kDmaStages - 2 < nchunk)
      wait_vmcnt<(kDmaStages - 2) * IPW>();
    else
      wait_vmcnt<0>();
    asm volatile("s_barrier" ::: "memory");  // every wave's part of chunk c is in LDS
    if (c + kDmaStages - 1 < nchunk) issue(c + kDmaStages - 1);
    const int st = c % kDmaStages;
    const int kvalid = ke - (kb + c * kDmaK);
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int s4 = 0; s4 < kDmaK / 4; ++s4) {
      const int kr = 4 * s4 + (lane >> 4);
      vec_t a = *reinterpret_cast<const vec_t*>(&sm.op.a[st][kr][ra]);
      T b[FM];
#pragma unroll
      for (int y = 0; y < FM; ++y) {
        const int n = cb + 16 * y;
        b[y] = sm.op.b[st][V * (BPC * n + ((kr / V) ^ S::swz(n))) + kr % V];
      }
      if (kr >= kvalid) {
        a = vec_t(T(0));
#pragma unroll
        for (int y = 0; y < FM; ++y) b[y] = T(0);
      }
#pragma unroll
      for (int x = 0; x < FM; ++x)
#pragma unroll
        for (int y = 0; y < FM; ++y) acc[x][y] = Mfma<T>::run(a[x], b[y], acc[x][y]);
    }
    __builtin_amdgcn_s_setprio(0);
  }

  // epilogue through LDS as in the A B^T tile (columns cb + 16 y here)
  constexpr int SW = S::SW, EC = S::EC;
  asm volatile("s_barrier" ::: "memory");
  T(*E)[SW + 1] = sm.epi[wave];
  T* C = static_cast<T*>(d.C);
  const int rbase = m0 + wm * SW, cbase = n0 + wn * SW;
  const bool lower = (flags & GF_C_LOWER) != 0;
#pragma unroll
  for (int p = 0; p < SW / EC; ++p) {
#pragma unroll
    for (int x = 0; x < FM; ++x)
#pragma unroll
      for (int y = 0; y < FM; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int cl = (lane & 15) + 16 * y - EC * p;
          if (cl >= 0 && cl < EC) E[cl][FM * Mfma<T>::row(lane, v) + x] = acc[x][y][v];
        }
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    constexpr int CPI = 64 / SW;
    {
      const int rl = lane % SW;
      const int gi = rbase + rl;
      for (int j = lane / SW; j < EC; j += CPI) {
        const int gj = cbase + EC * p + j;
        if (gi >= 0 && gi < d.m && gj < d.n && (!lower || gi >= gj)) {
          const int64_t idx = gi + (int64_t)d.ldc * gj;
          T val = alpha * E[j][rl];
          if (beta != T(0)) val += beta * C[idx];
          C[idx] = val;
        }
      }
    }
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
  }
}

// ---- A^T B tile fed by 16-byte DMA loads (the ID's Gram) -----------------
//
// C = alpha A^T B + beta C accumulated in FP64, for an A (k x m) and a B
// (k x n) whose columns are contiguous (op(A) = A^T, op(B) = B: the Gram of a
// face's panel), with FP32 or FP64 values.  64 x 64 tiles on four waves
// (2 x 2, 32 x 32 each, FP64 MFMA 16x16x4).  K runs in chunks of 128 bytes
// per column (KC = 32 FP32 or 16 FP64 values) through two LDS stages filled
// by global_load_lds_dwordx4.  A stage holds each operand as 64 columns of
// eight 16-byte blocks, their order XOR-swizzled by column so that the 16
// lanes reading one block of 16 columns hit distinct banks.  A lane's 16-byte
// read gives E = 16 / sizeof(TIn) consecutive k of its column, used by E MFMA
// steps: in a chunk, lane group g (lane / 16) supplies k-blocks g and g + 4,
// the same for both operands, so the MFMA steps run over the chunk's k in a
// fixed permuted order.  The k grid starts on the 16-byte boundary below the
// operands (A and B must share their offset from it); values outside [0, k)
// are masked to zero.
template <typename TIn>
struct TnSmem {
  static constexpr int E = 16 / (int)sizeof(TIn);  // values per 16 bytes
  static constexpr int KC = 8 * E;                  // k per chunk
  union __align__(16) {
    TIn op[2][2][64][KC];   // [stage][A, B][column][k, 16-byte blocks swizzled]
    double epi[4][32][33];  // [wave][column][row], staged outputs
  };
};

template <typename TIn, int CLS>
__global__ __launch_bounds__(NTHR, 4) void k_gemm_tn(int flags, const GemmDesc* __restrict__ desc,
                                                     double alpha, double beta) {
  constexpr int E = TnSmem<TIn>::E, KC = TnSmem<TIn>::KC;
  typedef TIn vin_t __attribute__((ext_vector_type(E)));
  __shared__ TnSmem<TIn> sm;
  unsigned bx, by, bz;
  xcd_remap(bx, by, bz);
  const GemmDesc d = desc[bz];
  const int m0 = by * 64, n0 = bx * 64;
  if (m0 >= d.m || n0 >= d.n) return;
  if ((flags & GF_C_LOWER) && m0 + 63 < n0) return;
  const int off = (int)(((uintptr_t)d.A / sizeof(TIn)) % E);  // (the same for B)
  const int ks = d.k + off;                                     // k extent, shifted grid
  const int nchunk = ks > off ? (ks + KC - 1) / KC : 0;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;

  // DMA: wave w loads operand w >> 1, columns 32 (w & 1) + 8 j + lane / 8 of
  // the tile (j = 0..3); lane % 8 is the block's place in the stage row, which
  // holds k-block (lane % 8) ^ swz(column)
  const int opnd = wave >> 1;
  const TIn* base = static_cast<const TIn*>(opnd == 0 ? d.A : d.B) - off;
  const int ld = opnd == 0 ? d.lda : d.ldb;
  const int ncol = opnd == 0 ? d.m : d.n;
  const int cbeg = opnd == 0 ? m0 : n0;
  const int qmax = (ks - 1) / E;  // last 16-byte block of a column that holds a value
  auto swz = [](int col) { return (col >> 1) & 7; };
  auto issue = [&](int c) {
    const int st = c & 1;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = 32 * (wave & 1) + 8 * j + (lane >> 3);
      const int gcol = min(cbeg + col, ncol - 1);
      const int q = min(8 * c + ((lane & 7) ^ swz(col)), qmax);
      dma16(base + (int64_t)ld * gcol + (int64_t)E * q,
            &sm.op[st][opnd][32 * (wave & 1) + 8 * j][0]);
    }
  };

  Mfma<double>::acc_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[x][y][v] = 0.0;

  const int g = lane >> 4;
  int ca[2], cb[2];  // this lane's columns in the stage rows
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    ca[x] = wm * 32 + 16 * x + (lane & 15);
    cb[x] = wn * 32 + 16 * x + (lane & 15);
  }
  // The 16 x 16 output blocks of this wave that hold a stored entry: inside
  // C and, for a lower C, not wholly above the diagonal.  The others take no
  // MFMA (a face whose width lies just past a multiple of 64 leaves most of
  // its last tile row empty); a live block's sums are formed in the same
  // order either way.  (Wave-uniform: the branches are scalar.)
  bool live[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const int r0 = m0 + wm * 32 + 16 * x, c0 = n0 + wn * 32 + 16 * y;
      live[x][y] = r0 < d.m && c0 < d.n && (!(flags & GF_C_LOWER) || r0 + 15 >= c0);
    }
  // (FP64 operands keep every block: measured slower with the skips)
  const bool all_live =
      sizeof(TIn) == 8 || (live[0][0] && live[0][1] && live[1][0] && live[1][1]);
  if (nchunk > 0) issue(0);
  for (int c = 0; c < nchunk; ++c) {
    wait_vmcnt<0>();                         // chunk c landed
    asm volatile("s_barrier" ::: "memory");  // ... for every wave; chunk c - 1 is done
    if (c + 1 < nchunk) issue(c + 1);        // into the stage chunk c - 1 used
    const int st = c & 1;
    const bool edge = (c == 0 && off > 0) || KC * (c + 1) > ks;
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int blk = g + 4 * r;
      vin_t a[2], b[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        a[x] = *reinterpret_cast<const vin_t*>(&sm.op[st][0][ca[x]][E * (blk ^ swz(ca[x]))]);
        b[x] = *reinterpret_cast<const vin_t*>(&sm.op[st][1][cb[x]][E * (blk ^ swz(cb[x]))]);
      }
      if (edge) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int k = KC * c + E * blk + e;
          if (k < off || k >= ks) {
#pragma unroll
            for (int x = 0; x < 2; ++x) {
              a[x][e] = TIn(0);
              b[x][e] = TIn(0);
            }
          }
        }
      }
      if (all_live) {
#pragma unroll
        for (int e = 0; e < E; ++e)
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
              acc[x][y] = Mfma<double>::run((double)a[x][e], (double)b[y][e], acc[x][y]);
      } else {
        double da[2][E], db[2][E];  // widened first: no VALU result feeds an MFMA directly
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int e = 0; e < E; ++e) {
            da[x][e] = (double)a[x][e];
            db[x][e] = (double)b[x][e];
          }
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            if (live[x][y]) {
#pragma unroll
              for (int e = 0; e < E; ++e) acc[x][y] = Mfma<double>::run(da[x][e], db[y][e], acc[x][y]);
            }
      }
    }
    __builtin_amdgcn_s_setprio(0);
  }

  // epilogue through LDS, as in the A B^T tile: columns out with consecutive
  // rows on consecutive lanes, mirrored rows with consecutive columns
  asm volatile("s_barrier" ::: "memory");  // every wave is done with the stages
  double(*Ep)[33] = sm.epi[wave];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        Ep[16 * y + (lane & 15)][16 * x + Mfma<double>::row(lane, v)] = acc[x][y][v];
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
  double* C = static_cast<double*>(d.C);
  const int rbase = m0 + wm * 32, cbase = n0 + wn * 32;
  const bool lower = (flags & GF_C_LOWER) != 0;
  {
    const int rl = lane & 31;
    const int gi = rbase + rl;
    for (int j = lane >> 5; j < 32; j += 2) {
      const int gj = cbase + j;
      if (gi < d.m && gj < d.n && (!lower || gi >= gj)) {
        const int64_t idx = gi + (int64_t)d.ldc * gj;
        double val = alpha * Ep[j][rl];
        if (beta != 0.0) val += beta * C[idx];
        C[idx] = val;
      }
    }
  }
  if (flags & GF_C_MIRROR) {  // (only with beta = 0)
    const int jl = lane & 31;
    const int gj = cbase + jl;
    for (int r = lane >> 5; r < 32; r += 2) {
      const int gi = rbase + r;
      if (gi < d.m && gj < d.n && gi > gj) C[gj + (int64_t)d.ldc * gi] = alpha * Ep[jl][r];
    }
  }
}

// Value of v in lane l of the wave (l uniform).
template <typename T>
__device__ __forceinline__ T read_lane(T v, int l) {
  if constexpr (sizeof(T) == 4) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
  } else {
    const long long x = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(x & 0xffffffffll), l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(x >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
  }
}

// LDS of one diagonal-block step: Lcol[t][i] = L_jj(i, t); the same columns
// shifted to start at their diagonal, Lsh[t][u] = L_jj(t + u, t) (zero past
// the block); rd[t] = 1 / L_jj(t, t).
template <typename T>
struct DiagSmem {
  __align__(16) T Lcol[kPanel][kPanel];
  T rd[kPanel];
};
template <typename T>
struct StepSmem : DiagSmem<T> {
  __align__(16) T Lsh[kPanel][kPanel];
};
// ... with the inverse staged row by row, X[i][c] = L_jj^{-1}(i, c) (rows
// padded so that a column read down the lanes meets distinct banks)
template <typename T>
struct DiagInvSmem : DiagSmem<T> {
  T X[kPanel][kPanel + 1];
};

// Cholesky of the diagonal block A(j0:j0+nb, j0:j0+nb) held in the column
// block col0 (leading dimension ld) into LDS, by the four waves of the
// workgroup: lane = row, wave q holds columns 16q .. 16q + 15; at step t the
// wave owning column t forms L(:, t) and publishes it through LDS, then every
// wave updates its later columns.  One barrier per column, but few registers:
// the form for the leaf fronts, whose many workgroups per CU hide the
// barriers.  Ends with a barrier.  Returns, per thread,
// whether its wave met a non-positive pivot (replaced by 1 to continue).
template <typename T, typename S>
__device__ __forceinline__ bool diag_factor_col(const T* col0, int64_t ld, int j0, int nb, S& ss) {
  constexpr bool kShift = std::is_same<S, StepSmem<T>>::value;  // also fill Lsh
  const int tid = threadIdx.x;
  if constexpr (kShift)
    for (int e = tid; e < kPanel * kPanel; e += NTHR) (&ss.Lsh[0][0])[e] = T(0);
  const int lane = tid & 63;
  const int q = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index, uniform
  const int rl = min(lane, nb - 1);
  T w[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int c = 16 * q + v;
    const T g = col0[ld * min(c, nb - 1) + j0 + rl];
    w[v] = (lane < nb && c < nb && c <= lane) ? g : T(0);
  }
  __syncthreads();
  bool bad = false;
  for (int qt = 0; 16 * qt < nb; ++qt) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int t = 16 * qt + v;
      if (t < nb) {  // uniform; a break here would keep the loop rolled
        if (q == qt) {
          T d = read_lane(w[v], t);
          bad = bad || !(d > T(0));
          d = d > T(0) ? d : T(1);
          T ltt, r;
          if constexpr (sizeof(T) == 4) {
            r = __builtin_amdgcn_rsqf(d);  // 1 ulp; shortens the serial chain
            ltt = d * r;
          } else {
            ltt = sqrt(d);
            r = T(1) / ltt;
          }
          const T lit = lane > t ? w[v] * r : (lane == t ? ltt : T(0));
          w[v] = lit;
          ss.Lcol[t][lane] = lit;
          if constexpr (kShift)
            if (lane >= t) ss.Lsh[t][lane - t] = lit;
        }
        __syncthreads();
        if (q >= qt) {
          const T li = ss.Lcol[t][lane];
          T lc[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) lc[u] = ss.Lcol[t][16 * q + u];
          if (q > qt) {
#pragma unroll
            for (int u = 0; u < 16; ++u) w[u] -= li * lc[u];
          } else {
#pragma unroll
            for (int u = v + 1; u < 16; ++u) w[u] -= li * lc[u];
          }
        }
      }
    }
  }
  if (tid < nb) ss.rd[tid] = T(1) / ss.Lcol[tid][tid];
  __syncthreads();
  return bad;
}

// The same Cholesky with four barriers instead of 64, for the latency-bound
// diagonal steps of the large fronts (one workgroup per front).  Blocked by
// wave: the wave owning columns 16k .. 16k + 15 factors them in its registers
// (the entries L(16k + u, t) that a column update needs are read across lanes,
// no barrier), publishes them through LDS, and every later wave then takes
// their rank-16 update: one barrier per 16 columns instead of one per column.
// A block narrower than 64 is padded with the identity: its own entries then
// receive only the same fused multiply-adds, in the same order, as in the
// column-by-column right-looking form (the padding contributes exact zeros of
// negative sign, which change no value).  Ends with a barrier; returns as
// diag_factor_col.
template <typename T>
__device__ __forceinline__ bool diag_factor_blk(const T* col0, int64_t ld, int j0, int nb,
                                                DiagSmem<T>& ss) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int q = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index, uniform
  const int rl = min(lane, nb - 1);
  T w[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int c = 16 * q + v;
    const T g = col0[ld * min(c, nb - 1) + j0 + rl];
    w[v] = (lane < nb && c < nb) ? (c <= lane ? g : T(0)) : (c == lane ? T(1) : T(0));
  }
  bool bad = false;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (q == k) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int t = 16 * k + v;
        T d = read_lane(w[v], t);
        bad = bad || !(d > T(0));
        d = d > T(0) ? d : T(1);
        T ltt, r;
        if constexpr (sizeof(T) == 4) {
          r = __builtin_amdgcn_rsqf(d);  // 1 ulp; shortens the serial chain
          ltt = d * r;
        } else {
          ltt = sqrt(d);
          r = T(1) / ltt;
        }
        const T lit = lane > t ? w[v] * r : (lane == t ? ltt : T(0));
        w[v] = lit;
#pragma unroll
        for (int u = v + 1; u < 16; ++u) w[u] -= lit * read_lane(lit, 16 * k + u);
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int t = 16 * k + v;
        ss.Lcol[t][lane] = w[v];
      }
    }
    __syncthreads();
    if (q > k) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int t = 16 * k + v;
        const T li = ss.Lcol[t][lane];
#pragma unroll
        for (int u = 0; u < 16; ++u) w[u] -= li * ss.Lcol[t][16 * q + u];
      }
    }
  }
  if (tid < kPanel) ss.rd[tid] = T(1) / ss.Lcol[tid][tid];
  __syncthreads();
  return bad;
}

// One panel row below the factored diagonal block: x L_jj^T = p in place (row
// points at column j0 of the row, leading dimension ld), by forward
// substitution.  A row that is zero stays zero and is left as it is; returns
// whether the row was nonzero.
template <typename T>
__device__ __forceinline__ bool panel_row_light(T* row, int64_t ld, int nb,
                                                const StepSmem<T>& ss) {
  T w[kPanel];
  bool nz = false;
#pragma unroll
  for (int u = 0; u < kPanel; ++u) {
    const T g = row[ld * min(u, nb - 1)];
    w[u] = u < nb ? g : T(0);
    nz = nz || w[u] != T(0);
  }
  if (!nz) return false;
  for (int t = 0; t < nb; ++t) {
    T l[kPanel];
#pragma unroll
    for (int u = 0; u < kPanel; ++u) l[u] = ss.Lsh[t][u];
    const T x = w[0] * ss.rd[t];
    row[ld * t] = x;
#pragma unroll
    for (int u = 1; u < kPanel; ++u) w[u - 1] = w[u] - l[u] * x;
    w[kPanel - 1] = T(0);
  }
  return true;
}

// Diagonal block of the blocked right-looking Cholesky at block column j0,
// by one workgroup: L_jj by diag_factor_blk, then its inverse X by the four waves,
// lane = column of X and wave p = its rows 16p .. 16p + 15.  Row block p takes
// the contributions of the row blocks above it as they are published, then
// solves its own 16 rows (the same operations, in the same order, as the
// column-by-column forward substitution).  The inverse is written over the
// block (strict upper part zero) from LDS, with rows on lanes.  The panel
// kernel then forms the rows below as P L_jj^{-T}, and the inverse of L_I
// starts from these inverted diagonal blocks.  (Past nb the block is the
// identity, as diag_factor_blk pads it.)
template <typename T>
__device__ __forceinline__ void diag_step(T* col0, int64_t ld, int j0, int nb,
                                          DiagInvSmem<T>& ss, int* err, int id) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int p = __builtin_amdgcn_readfirstlane(tid >> 6);
  const bool bad = diag_factor_blk<T>(col0, ld, j0, nb, ss);
  if (bad && lane == 0) atomicMin(err, id);
  T x[16];  // rows 16p .. 16p + 15 of column `lane`, from the identity
#pragma unroll
  for (int i = 0; i < 16; ++i) x[i] = 16 * p + i == lane ? T(1) : T(0);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (p == k) {
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const int t = 16 * k + s;
        x[s] *= ss.rd[t];
#pragma unroll
        for (int i = s + 1; i < 16; ++i) x[i] -= ss.Lcol[t][16 * k + i] * x[s];
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) ss.X[16 * k + i][lane] = x[i];
    }
    __syncthreads();
    if (p > k) {
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const int t = 16 * k + s;
        const T xt = ss.X[t][lane];
#pragma unroll
        for (int i = 0; i < 16; ++i) x[i] -= ss.Lcol[t][16 * p + i] * xt;
      }
    }
  }
  if (lane < nb) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int c = 16 * p + v;
      if (c < nb) col0[j0 + lane + ld * c] = lane >= c ? ss.X[lane][c] : T(0);
    }
  }
}

// The diagonal step of every front, one workgroup each.
template <typename T>
__global__ __launch_bounds__(NTHR) void k_front_diag(const FrontDesc* __restrict__ fd, int j0,
                                                     int* err) {
  __shared__ DiagInvSmem<T> ss;
  const FrontDesc f = fd[blockIdx.x];
  if (j0 >= f.nI) return;
  const int nb = min(kPanel, f.nI - j0);
  T* col0 = static_cast<T*>(f.ptr) + (int64_t)f.ld * j0;
  diag_step<T>(col0, f.ld, j0, nb, ss, err, f.id);
}

// Trailing update of the blocked front Cholesky with the factored panel
// columns [p0, p0 + pw): Phi[c0:nR, c0:c0 + cw] -= P[c0:nR] P[c0:c0 + cw]^T
// (lower part), P = Phi[:, p0:p0 + pw], all ranges clipped to the front, with
// the panel read in place as both operands.
template <typename T, int TS>
__global__ __launch_bounds__(NTHR) void k_front_trailing(const FrontDesc* __restrict__ fd,
                                                         int p0, int pw, int c0, int cw) {
  __shared__ TileSmem<T, TS, TS> sm;
  unsigned bx, by, bz;
  xcd_remap(bx, by, bz);
  const FrontDesc f = fd[bz];
  T* base = static_cast<T*>(f.ptr);
  const int k = min(p0 + pw, f.nI) - p0;
  const int m = f.nR - c0, n = min(c0 + cw, f.nI) - c0;
  const int m0 = by * TS, n0 = bx * TS;
  if (k <= 0 || m0 >= m || n0 >= n) return;
  if (m0 + TS - 1 < n0) return;
  const T* P = base + c0 + (int64_t)f.ld * p0;
  gemm_tile_t<T, T, OP_N, OP_T, TS, TS>(GF_C_LOWER, P, f.ld, P, f.ld,
                                        base + c0 + (int64_t)f.ld * c0, f.ld, m, n, k, m0, n0,
                                        T(-1), T(1), sm);
}

// Panel rows below the diagonal block at j0, TM rows per workgroup: P <- P
// L_jj^{-T} in place, one TM x 64 GEMM tile over all of the block's columns
// (the rows are read in full before any is written; the diagonal block holds
// L_jj^{-1}).
template <typename T, int TM>
__global__ __launch_bounds__(NTHR) void k_front_panel(const FrontDesc* __restrict__ fd, int j0) {
  __shared__ TileSmem<T, TM, 64> sm;
  unsigned bx, by, bz;
  xcd_remap(bx, by, bz);
  const FrontDesc f = fd[by];
  if (j0 >= f.nI) return;
  const int nb = min(kPanel, f.nI - j0);
  const int j1 = j0 + nb;
  const int m = f.nR - j1;
  const int m0 = bx * TM;
  if (m0 >= m) return;
  T* col0 = static_cast<T*>(f.ptr) + (int64_t)f.ld * j0;
  gemm_tile_t<T, T, OP_N, OP_T, TM, 64>(GF_B_UPPER | GF_TRI_ZEROS, col0 + j1, f.ld, col0 + j0,
                                        f.ld, col0 + j1, f.ld, m, nb, nb, m0, 0, T(1), T(0), sm);
}

// The whole blocked Cholesky of one small front per workgroup (every step's
// diagonal block, panel rows and trailing update in one launch), for the many
// small fronts of the lowest level, where per-step launches would leave the
// chip waiting on latency.  The step buffers and the GEMM tile share LDS.
// Zero blocks are skipped exactly: a panel row that is zero stays zero, and a
// trailing tile whose two panel blocks (64 rows) hold no nonzero is left as
// it is.  The leaf fronts, the stencil on a box in lexicographic order, have
// a band of at most 64, so each step updates one trailing tile.
template <typename T>
__global__ __launch_bounds__(NTHR, 16 / sizeof(T)) void k_front_small(
                                                         const FrontDesc* __restrict__ fd,
                                                         int* err) {
  constexpr size_t kBytes = sizeof(StepSmem<T>) > sizeof(TileSmem<T, 64, 64>)
                                ? sizeof(StepSmem<T>)
                                : sizeof(TileSmem<T, 64, 64>);
  __shared__ __align__(16) char smem[kBytes];
  StepSmem<T>& ss = *reinterpret_cast<StepSmem<T>*>(smem);
  TileSmem<T, 64, 64>& ts = *reinterpret_cast<TileSmem<T, 64, 64>*>(smem);
  constexpr int kMaxBlk = 16;     // panel blocks tracked (fronts of up to 1024 rows)
  __shared__ int nzb[kMaxBlk];  // panel block b (rows 64 b ..) holds a nonzero
  const FrontDesc f = fd[blockIdx.x];
  T* base = static_cast<T*>(f.ptr);
  const int tid = threadIdx.x;
  bool bad_any = false;
  for (int j0 = 0; j0 < f.nI; j0 += kPanel) {
    const int nb = min(kPanel, f.nI - j0);
    const int j1 = j0 + nb;
    const int m = f.nR - j1, n = f.nI - j1;
    const bool dense = m > kMaxBlk * 64;
    T* col0 = base + (int64_t)f.ld * j0;
    if (tid < kMaxBlk) nzb[tid] = 0;  // visible after diag_factor_col's barriers
    bad_any = diag_factor_col<T>(col0, f.ld, j0, nb, ss) || bad_any;
    for (int e = tid; e < kPanel * kPanel; e += NTHR) {
      const int c = e >> 6, r = e & 63;
      if (r < nb && c < nb && c <= r) col0[j0 + r + (int64_t)f.ld * c] = ss.Lcol[c][r];
    }
    for (int i = tid; i < m; i += NTHR)
      if (panel_row_light<T>(col0 + j1 + i, f.ld, nb, ss) && !dense) nzb[i >> 6] = 1;
    __syncthreads();  // panel rows and block flags visible to the workgroup; LDS free
    const T* P = col0 + j1;
    for (int n0 = 0; n0 < n; n0 += 64) {
      if (!dense && !nzb[n0 >> 6]) continue;  // uniform over the workgroup
      for (int m0 = n0; m0 < m; m0 += 64) {
        if (!dense && !nzb[m0 >> 6]) continue;
        gemm_tile_t<T, T, OP_N, OP_T, 64, 64>(GF_C_LOWER, P, f.ld, P, f.ld,
                                              base + j1 + (int64_t)f.ld * j1, f.ld, m, n, nb, m0,
                                              n0, T(-1), T(1), ts);
      }
    }
    __syncthreads();
  }
  if (bad_any && (tid & 63) == 0) atomicMin(err, f.id);
}

// In-place inverse of every 64 x 64 diagonal block of the factored L_I, one
// wave per block: lane c forms column c of the inverse, right-looking (after
// x_t is final it is eliminated from every later row at once, so the updates
// of one step are independent), with the columns of L read as LDS
// broadcasts.  Rows and columns past nb are padded with the identity.
template <typename T>
__global__ __launch_bounds__(64) void k_diag_inv(const FrontDesc* __restrict__ fd) {
  // Lc[t][i] = L(i, t) while the inverse is formed, then Xs[c][i] = L^{-1}(i, c)
  // in the same storage (one wave: its LDS accesses complete in issue order),
  // which doubles the waves per CU of this latency-bound kernel
  __shared__ __align__(16) T buf[kPanel * (kPanel + 1)];
  T(*Lc)[kPanel] = reinterpret_cast<T(*)[kPanel]>(buf);
  T(*Xs)[kPanel + 1] = reinterpret_cast<T(*)[kPanel + 1]>(buf);
  __shared__ T rd[kPanel];
  const FrontDesc f = fd[blockIdx.y];
  const int j0 = blockIdx.x * kPanel;
  if (j0 >= f.nI) return;
  const int nb = min(kPanel, f.nI - j0);
  const int lane = threadIdx.x;
  T* base = static_cast<T*>(f.ptr) + j0 + (int64_t)f.ld * j0;
  // one wave: its LDS accesses complete in issue order, no barriers needed.
  // Lane r reads row r of every column, all 64 loads issued before the first
  // is used (clamped to the block; entries outside it are replaced below):
  // the block comes from HBM, and batches of a few loads each waited out the
  // memory latency in turn.
  T g[kPanel];
  const int rl = min(lane, nb - 1);
#pragma unroll
  for (int c = 0; c < kPanel; ++c) g[c] = base[(int64_t)f.ld * min(c, nb - 1) + rl];
#pragma unroll
  for (int c = 0; c < kPanel; ++c) {
    const int r = lane;
    T v = r == c ? T(1) : T(0);
    if (r < nb && c < nb && c <= r) v = g[c];
    Lc[c][r] = v;
    if (r == c) rd[c] = T(1) / v;
  }
  T x[kPanel];  // column `lane` of the inverse, from e_lane
#pragma unroll
  for (int i = 0; i < kPanel; ++i) x[i] = i == lane ? T(1) : T(0);
#pragma unroll
  for (int t = 0; t < kPanel; ++t) {
    x[t] *= rd[t];
#pragma unroll
    for (int u = t + 1; u < kPanel; ++u) x[u] -= Lc[t][u] * x[t];
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int i = 0; i < kPanel; ++i) Xs[lane][i] = x[i];
#pragma unroll 4
  for (int e = lane; e < kPanel * kPanel; e += 64) {
    const int c = e >> 6, r = e & 63;
    if (r < nb && c < nb && c <= r) base[(int64_t)f.ld * c + r] = Xs[c][r];
  }
}

// One panel (up to kPivPanel pivots) of the diagonal-pivoted Cholesky of a
// Gram matrix, one workgroup per face.  G is up to date for all columns
// before j0 (the trailing updates of earlier panels were applied by GEMM);
// within the panel each new column subtracts the panel's earlier columns.
// The Schur diagonal d, the pivot flags and the stop state persist in global
// memory between launches.  Pivot: largest remaining diagonal, ties to the
// lowest index; stop when it is <= eps^2 times the first pivot.
constexpr int kPivPanel = 64;

// NTP threads per face: 1024 for large faces (few faces, each pivot's column
// spread over more lanes), 64 for faces of at most 64 points, 256 otherwise.
template <int NTP, int MAXF>
__global__ __launch_bounds__(NTP) void k_pchol_panel(
    const double* __restrict__ G, double* __restrict__ L, const int64_t* __restrict__ goff,
    const int* __restrict__ nFa, const int* __restrict__ ldga, const int64_t* __restrict__ poff,
    int* __restrict__ perm, double* __restrict__ dbuf, int* __restrict__ pivbuf,
    int* __restrict__ kst, double* __restrict__ r11, double eps, int j0) {
  // sized for the largest face of the launch, so that small faces keep many
  // workgroups resident per CU
  __shared__ double d[MAXF];
  __shared__ unsigned char piv[MAXF];
  __shared__ double lp[kPivPanel];
  __shared__ double rv[NTP / 64];
  __shared__ int ri[NTP / 64];
  __shared__ int s_p, s_stop;
  __shared__ double s_dp, s_r11;
  const int b = blockIdx.x;
  const int nF = nFa[b];
  if (kst[b] >= 0 || j0 >= nF) return;
  const int ld = ldga[b];
  const double* Gb = G + goff[b];
  double* Lb = L + goff[b];
  int* pb = perm + poff[b];
  double* db = dbuf + poff[b];
  int* pvb = pivbuf + poff[b];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int a = tid; a < nF; a += NTP) {
    d[a] = j0 == 0 ? Gb[a + (int64_t)ld * a] : db[a];
    piv[a] = j0 == 0 ? 0 : (unsigned char)pvb[a];
  }
  if (tid == 0) s_r11 = j0 == 0 ? 0.0 : r11[b];
  __syncthreads();
  const int jend = min(j0 + kPivPanel, nF);
  int stopped = 0;
  for (int j = j0; j < jend; ++j) {
    double bv = -DBL_MAX;
    int bi = INT_MAX;
    for (int a = tid; a < nF; a += NTP) {
      if (!piv[a]) {
        const double v = d[a];
        if (v > bv || (v == bv && a < bi)) { bv = v; bi = a; }
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(bv, off);
      const int oi = __shfl_xor(bi, off);
      if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
    }
    if (lane == 0) { rv[wave] = bv; ri[wave] = bi; }
    __syncthreads();
    if (wave == 0) {  // the waves' candidates, reduced across lanes (a total order: any tree)
      if (NTP > 64) {
        bv = lane < NTP / 64 ? rv[lane] : -DBL_MAX;
        bi = lane < NTP / 64 ? ri[lane] : INT_MAX;
#pragma unroll
        for (int off = NTP / 128; off > 0; off >>= 1) {
          const double ov = __shfl_xor(bv, off);
          const int oi = __shfl_xor(bi, off);
          if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
      }
    }
    if (tid == 0) {
      if (j == 0) s_r11 = bv;
      const int stop = (j == 0) ? !(bv > 0.0) : !(bv > eps * eps * s_r11);
      s_stop = stop;
      if (stop) {
        kst[b] = j;
      } else {
        s_p = bi;
        s_dp = bv;
        piv[bi] = 1;
        pb[j] = bi;
      }
    }
    __syncthreads();
    if (s_stop) { stopped = 1; break; }
    const int p = s_p;
    const double ljj = sqrt(s_dp);
    const int np = j - j0;
    // this thread's first entry of column p, in flight with the pivot row's load
    const double g0 = tid < nF ? Gb[tid + (int64_t)ld * p] : 0.0;
    if (tid < np) lp[tid] = Lb[p + (int64_t)ld * (j0 + tid)];
    __syncthreads();
    for (int a = tid; a < nF; a += NTP) {
      double v;
      if (a == p) v = ljj;
      else if (piv[a]) v = 0.0;
      else {
        const double* la = Lb + a + (int64_t)ld * j0;
        double s0 = a == tid ? g0 : Gb[a + (int64_t)ld * p], s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int t = 0;
        for (; t + 4 <= np; t += 4) {
          s0 -= la[(int64_t)ld * t] * lp[t];
          s1 -= la[(int64_t)ld * (t + 1)] * lp[t + 1];
          s2 -= la[(int64_t)ld * (t + 2)] * lp[t + 2];
          s3 -= la[(int64_t)ld * (t + 3)] * lp[t + 3];
        }
        for (; t < np; ++t) s0 -= la[(int64_t)ld * t] * lp[t];
        v = ((s0 + s1) + (s2 + s3)) / ljj;
        d[a] -= v * v;
      }
      Lb[a + (int64_t)ld * j] = v;
    }
    __threadfence_block();
    __syncthreads();
  }
  if (tid == 0) {
    if (!stopped && jend == nF) kst[b] = nF;
    r11[b] = s_r11;
  }
  for (int a = tid; a < nF; a += NTP) {
    db[a] = d[a];
    pvb[a] = piv[a];
  }
}

// 32 x 32 tiles through LDS; reads and writes are both along columns.
template <typename T>
__global__ __launch_bounds__(NTHR) void k_transpose(const TransDesc* __restrict__ dd) {
  __shared__ T tile[32][33];
  const TransDesc d = dd[blockIdx.z];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  if (r0 >= d.rows || c0 >= d.cols) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const auto src = as_global((const T*)d.src);
  const auto dst = as_global((T*)d.dst);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = r0 + tx, c = c0 + ty + 8 * k;
    if (r < d.rows && c < d.cols) tile[ty + 8 * k][tx] = src[r + (int64_t)d.lds * c];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int c = c0 + tx, r = r0 + ty + 8 * k;
    if (r < d.rows && c < d.cols) dst[c + (int64_t)d.ldd * r] = tile[tx][ty + 8 * k];
  }
}

// Faces whose rank is already settled (kst >= 0) need no further update of
// their Gram: their descriptors of the coming update get m = n = k = 0, so
// that every tile of the batched product returns at once.  (What the update
// would write there is never read: the ID takes only the first k pivot
// columns of L, and the panel kernel returns for a finished face.)
__global__ __launch_bounds__(NTHR) void k_pchol_drop_done(GemmDesc* __restrict__ desc,
                                                          const int* __restrict__ bidx,
                                                          const int* __restrict__ kst, int cnt) {
  const int i = blockIdx.x * NTHR + threadIdx.x;
  if (i < cnt && kst[bidx[i]] >= 0) {
    desc[i].m = 0;
    desc[i].n = 0;
    desc[i].k = 0;
  }
}

// Rank and the tail of the permutation: unpivoted indices ascending.
__global__ __launch_bounds__(64) void k_pchol_tail(const int* __restrict__ nFa,
                                                   const int64_t* __restrict__ poff,
                                                   int* __restrict__ perm,
                                                   const int* __restrict__ pivbuf,
                                                   const int* __restrict__ kst,
                                                   int* __restrict__ kout) {
  const int b = blockIdx.x;
  if (threadIdx.x != 0) return;
  const int nF = nFa[b];
  int k = kst[b];
  if (k < 0) k = nF;
  kout[b] = k;
  int* pb = perm + poff[b];
  const int* pvb = pivbuf + poff[b];
  int pos = k;
  for (int a = 0; a < nF; ++a)
    if (!pvb[a]) pb[pos++] = a;
}

}  // namespace

template <typename TIn, typename TC, int OPA, int OPB, int TS, int CLS>
void launch_gemm(int flags, const GemmDesc* d_desc, int batch, int max_m, int max_n, TC alpha,
                 TC beta, hipStream_t s) {
  for (int b0 = 0; b0 < batch; b0 += kMaxGridY) {
    const int nb = std::min(batch - b0, kMaxGridY);
    dim3 grid((unsigned)ceil_div(max_n, TS), (unsigned)ceil_div(max_m, TS), (unsigned)nb);
    hipLaunchKernelGGL((k_gemm_desc<TIn, TC, OPA, OPB, TS, TS, CLS>), grid, dim3(NTHR), 0, s,
                       flags, d_desc + b0, alpha, beta);
    HIF_LAUNCH_CHECK();
  }
}

template <typename TIn, int CLS>
void launch_gemm_tn(int flags, const GemmDesc* d_desc, int batch, int max_m, int max_n,
                    double alpha, double beta, hipStream_t s) {
  for (int b0 = 0; b0 < batch; b0 += kMaxGridY) {
    const int nb = std::min(batch - b0, kMaxGridY);
    dim3 grid((unsigned)ceil_div(max_n, 64), (unsigned)ceil_div(max_m, 64), (unsigned)nb);
    hipLaunchKernelGGL((k_gemm_tn<TIn, CLS>), grid, dim3(NTHR), 0, s, flags, d_desc + b0, alpha,
                       beta);
    HIF_LAUNCH_CHECK();
  }
}

template <typename T, int TS, int CLS>
void launch_gemm_nt(int flags, const GemmDesc* d_desc, int batch, int max_m, int max_n, T alpha,
                    T beta, hipStream_t s) {
  constexpr int V = DmaSmem<T, TS>::V;
  for (int b0 = 0; b0 < batch; b0 += kMaxGridY) {
    const int nb = std::min(batch - b0, kMaxGridY);
    // the shifted grid is up to V - 1 rows (columns) longer
    dim3 grid((unsigned)ceil_div(max_n + V - 1, TS), (unsigned)ceil_div(max_m + V - 1, TS),
              (unsigned)nb);
    hipLaunchKernelGGL((k_gemm_nt<T, TS, CLS>), grid, dim3(NTHR), 0, s, flags, d_desc + b0, alpha,
                       beta);
    HIF_LAUNCH_CHECK();
  }
}

template <typename T, int TS>
void launch_gemm_nn(int flags, const GemmDesc* d_desc, int batch, int max_m, int max_n, T alpha,
                    T beta, hipStream_t s) {
  constexpr int V = NnSmem<T, TS>::V;
  for (int b0 = 0; b0 < batch; b0 += kMaxGridY) {
    const int nb = std::min(batch - b0, kMaxGridY);
    dim3 grid((unsigned)ceil_div(max_n, TS), (unsigned)ceil_div(max_m + V - 1, TS), (unsigned)nb);
    hipLaunchKernelGGL((k_gemm_nn<T, TS>), grid, dim3(NTHR), 0, s, flags, d_desc + b0, alpha, beta);
    HIF_LAUNCH_CHECK();
  }
}

template <typename TIn, typename TC, int TS>
void dispatch_gemm(int opa, int opb, int flags, int cls, const GemmDesc* d_desc, int batch,
                   int max_m, int max_n, TC alpha, TC beta, hipStream_t s) {
  if (cls == GC_SYRK && opa == OP_N && opb == OP_T)
    launch_gemm<TIn, TC, OP_N, OP_T, TS, GC_SYRK>(flags, d_desc, batch, max_m, max_n, alpha, beta, s);
  else if (cls == GC_LSI && opa == OP_N && opb == OP_T)
    launch_gemm<TIn, TC, OP_N, OP_T, TS, GC_LSI>(flags, d_desc, batch, max_m, max_n, alpha, beta, s);
  else if (cls == GC_GRAM && opa == OP_T && opb == OP_N)
    launch_gemm<TIn, TC, OP_T, OP_N, TS, GC_GRAM>(flags, d_desc, batch, max_m, max_n, alpha, beta, s);
  else if (opa == OP_N && opb == OP_N)
    launch_gemm<TIn, TC, OP_N, OP_N, TS, 0>(flags, d_desc, batch, max_m, max_n, alpha, beta, s);
  else if (opa == OP_N)
    launch_gemm<TIn, TC, OP_N, OP_T, TS, 0>(flags, d_desc, batch, max_m, max_n, alpha, beta, s);
  else if (opb == OP_N)
    launch_gemm<TIn, TC, OP_T, OP_N, TS, 0>(flags, d_desc, batch, max_m, max_n, alpha, beta, s);
  else
    launch_gemm<TIn, TC, OP_T, OP_T, TS, 0>(flags, d_desc, batch, max_m, max_n, alpha, beta, s);
}

// ---- tile shapes --------------------------------------------------------
// A batched GEMM runs square TS x TS tiles, TS in {32, 64, 128} (128 only for
// FP32 accumulation, whose tile fits the register file).  The shape comes from
// a table keyed by the operand and accumulator types, the two transposes, the
// triangular flags and the size bucket (the smallest power of two >= the
// largest m or n of the batch), written by the autotuner (tune_tiles.py) into
// tiles.tsv beside the library.  Keys it does not hold fall back to the
// built-in rule: 128 for FP32 outputs of at least 1024 x 1024, else 64.

namespace {

struct TileKey {
  int in_bytes, acc_bytes, opa, opb, flags, bucket;
  bool operator<(const TileKey& o) const {
    return std::tie(in_bytes, acc_bytes, opa, opb, flags, bucket) <
           std::tie(o.in_bytes, o.acc_bytes, o.opa, o.opb, o.flags, o.bucket);
  }
};

constexpr int kTileFlags = GF_A_LOWER | GF_A_UPPER | GF_B_LOWER | GF_B_UPPER | GF_C_LOWER |
                           GF_C_MIRROR | GF_TRI_ZEROS;

int size_bucket(int max_m, int max_n) {
  const int v = std::max(max_m, max_n);
  int b = 32;
  while (b < v && b < 8192) b *= 2;
  return b;
}

struct TileTable {
  std::mutex mu;
  bool loaded = false;
  std::map<TileKey, int> tiles;
  // tuning mode: device time per key and candidate tile, summed over launches
  bool tuning = false;
  std::map<TileKey, std::map<int, double>> timed;
};

TileTable& tile_table() {
  static TileTable t;
  return t;
}

std::string library_dir() {
  Dl_info info;
  if (dladdr((const void*)&library_dir, &info) && info.dli_fname) {
    std::string p(info.dli_fname);
    const size_t k = p.rfind('/');
    return k == std::string::npos ? std::string(".") : p.substr(0, k);
  }
  return ".";
}

void load_tiles_locked(TileTable& T) {
  T.loaded = true;
  std::ifstream in(library_dir() + "/tiles.tsv");
  std::string line;
  while (std::getline(in, line)) {
    const size_t hash = line.find('#');
    if (hash != std::string::npos) line.resize(hash);
    std::istringstream ss(line);
    TileKey k{};
    int tile = 0;
    if (!(ss >> k.in_bytes >> k.acc_bytes >> k.opa >> k.opb >> k.flags >> k.bucket >> tile))
      continue;
    if (tile == 32 || tile == 64 || (tile == 128 && k.acc_bytes == 4)) T.tiles[k] = tile;
  }
}

template <typename TIn, typename TC>
TileKey tile_key(int opa, int opb, int flags, int max_m, int max_n) {
  return {(int)sizeof(TIn), (int)sizeof(TC), opa, opb, flags & kTileFlags,
          size_bucket(max_m, max_n)};
}

template <typename TIn, typename TC>
int pick_tile(const TileKey& k, int max_m, int max_n) {
  TileTable& T = tile_table();
  std::lock_guard<std::mutex> lock(T.mu);
  if (!T.loaded) load_tiles_locked(T);
  auto it = T.tiles.find(k);
  if (it != T.tiles.end()) return it->second;
  return (sizeof(TC) == 4 && max_m >= 1024 && max_n >= 1024) ? 128 : 64;
}

// The DMA tile serves A B^T products whose leading dimensions are multiples of
// 16 bytes, in one precision, with triangular operands only when their zeros
// are stored and a mirrored output only when it overwrites C, at the tile size
// the table picks for it.
// ... and A B products (no mirror, no A-upper mask), B on the 16-byte grid.
template <typename TIn, typename TC>
bool use_dma_nn(int ts, int opa, int opb, int flags, bool ld16) {
  if (!std::is_same<TIn, TC>::value || !ld16 || opa != OP_N || opb != OP_N) return false;
  if (flags & (GF_C_MIRROR | GF_A_UPPER)) return false;
  if ((flags & (GF_A_LOWER | GF_B_LOWER | GF_B_UPPER)) && !(flags & GF_TRI_ZEROS)) return false;
  return ts == 64 || (sizeof(TC) == 4 && ts == 128);
}

template <typename TIn, typename TC>
bool use_dma_tile(int ts, int opa, int opb, int flags, bool ld16, bool beta0) {
  if (!std::is_same<TIn, TC>::value || !ld16 || opa != OP_N || opb != OP_T) return false;
  if ((flags & GF_C_MIRROR) && !beta0) return false;
  if ((flags & (GF_A_LOWER | GF_A_UPPER | GF_B_LOWER | GF_B_UPPER)) && !(flags & GF_TRI_ZEROS))
    return false;
  return ts == 64 || (sizeof(TC) == 4 && ts == 128);
}

template <typename TIn, typename TC>
void launch_tile(int ts, int opa, int opb, int flags, int cls, const GemmDesc* d_desc, int batch,
                 int max_m, int max_n, TC alpha, TC beta, hipStream_t s, bool ld16 = false) {
  // the Gram: A^T B in FP64 from columns on the 16-byte grid, no operand masks
  if constexpr (std::is_same<TC, double>::value) {
    if (cls == GC_GRAM && ld16 && opa == OP_T && opb == OP_N &&
        !(flags & (GF_A_LOWER | GF_A_UPPER | GF_B_LOWER | GF_B_UPPER)) &&
        (!(flags & GF_C_MIRROR) || beta == TC(0))) {
      launch_gemm_tn<TIn, GC_GRAM>(flags, d_desc, batch, max_m, max_n, alpha, beta, s);
      return;
    }
  }
  if constexpr (std::is_same<TIn, TC>::value) {
    if (use_dma_tile<TIn, TC>(ts, opa, opb, flags, ld16, beta == TC(0))) {
      auto go = [&](auto tsc) {
        constexpr int TSC = decltype(tsc)::value;
        if (cls == GC_SYRK)
          launch_gemm_nt<TC, TSC, GC_SYRK>(flags, d_desc, batch, max_m, max_n, alpha, beta, s);
        else if (cls == GC_LSI)
          launch_gemm_nt<TC, TSC, GC_LSI>(flags, d_desc, batch, max_m, max_n, alpha, beta, s);
        else
          launch_gemm_nt<TC, TSC, GC_GENERIC>(flags, d_desc, batch, max_m, max_n, alpha, beta, s);
      };
      if constexpr (sizeof(TC) == 4) {
        if (ts == 128) go(std::integral_constant<int, 128>());
        else go(std::integral_constant<int, 64>());
      } else {
        go(std::integral_constant<int, 64>());
      }
      return;
    }
    if (use_dma_nn<TIn, TC>(ts, opa, opb, flags, ld16)) {
      if constexpr (sizeof(TC) == 4) {
        if (ts == 128)
          launch_gemm_nn<TC, 128>(flags, d_desc, batch, max_m, max_n, alpha, beta, s);
        else
          launch_gemm_nn<TC, 64>(flags, d_desc, batch, max_m, max_n, alpha, beta, s);
      } else {
        launch_gemm_nn<TC, 64>(flags, d_desc, batch, max_m, max_n, alpha, beta, s);
      }
      return;
    }
  }
  if (sizeof(TC) == 4 && ts == 128)
    dispatch_gemm<TIn, TC, 128>(opa, opb, flags, cls, d_desc, batch, max_m, max_n, alpha, beta, s);
  else if (ts == 32)
    dispatch_gemm<TIn, TC, 32>(opa, opb, flags, cls, d_desc, batch, max_m, max_n, alpha, beta, s);
  else
    dispatch_gemm<TIn, TC, 64>(opa, opb, flags, cls, d_desc, batch, max_m, max_n, alpha, beta, s);
}

}  // namespace

template <typename TIn, typename TC>
void gemm_batched(int opa, int opb, int flags, const GemmDesc* d_desc, int batch, int max_m,
                  int max_n, TC alpha, TC beta, hipStream_t s, const char* name, double flops,
                  int cls, bool ld16) {
  if (batch <= 0 || max_m <= 0 || max_n <= 0) return;
  const TileKey key = tile_key<TIn, TC>(opa, opb, flags, max_m, max_n);
  bool tuning;
  {
    TileTable& T = tile_table();
    std::lock_guard<std::mutex> lock(T.mu);
    tuning = T.tuning;
  }
  // Tuning: a product that overwrites C (beta = 0; no library GEMM with
  // beta = 0 reads C or lets it overlap A or B) is run with every candidate
  // tile and each run timed.  All tile sizes take K in the same chunk order,
  // so every run writes the same C (the Gram's DMA tile, whose K order is its
  // own, runs at every candidate size, as outside tuning).
  if (tuning && beta == TC(0)) {
    std::vector<int> cands = {32, 64};
    if (sizeof(TC) == 4) cands.push_back(128);
    hipEvent_t e0, e1;
    HIF_HIP(hipEventCreate(&e0));
    HIF_HIP(hipEventCreate(&e1));
    std::vector<float> ms(cands.size(), 0.f);
    for (size_t c = 0; c < cands.size(); ++c) {
      HIF_HIP(hipEventRecord(e0, s));
      launch_tile<TIn, TC>(cands[c], opa, opb, flags, cls, d_desc, batch, max_m, max_n, alpha,
                           beta, s, ld16);
      HIF_HIP(hipEventRecord(e1, s));
      HIF_HIP(hipEventSynchronize(e1));
      HIF_HIP(hipEventElapsedTime(&ms[c], e0, e1));
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    TileTable& T = tile_table();
    std::lock_guard<std::mutex> lock(T.mu);
    for (size_t c = 0; c < cands.size(); ++c) T.timed[key][cands[c]] += ms[c];
    return;
  }
  ProfScope ps(name, s, flops);
  launch_tile<TIn, TC>(pick_tile<TIn, TC>(key, max_m, max_n), opa, opb, flags, cls, d_desc,
                       batch, max_m, max_n, alpha, beta, s, ld16);
}

void tune_begin() {
  TileTable& T = tile_table();
  std::lock_guard<std::mutex> lock(T.mu);
  T.timed.clear();
  T.tuning = true;
}

int tune_end(const char* path) {
  TileTable& T = tile_table();
  std::lock_guard<std::mutex> lock(T.mu);
  T.tuning = false;
  std::map<TileKey, int> best;
  for (auto& kv : T.timed) {
    int bt = 0;
    double bm = 0.0;
    for (auto& tm : kv.second)
      if (bt == 0 || tm.second < bm) {
        bt = tm.first;
        bm = tm.second;
      }
    best[kv.first] = bt;
  }
  if (path && *path) {
    std::ofstream out(path);
    HIF_REQUIRE(out.good(), HIF_EINVAL, std::string("cannot write ") + path);
    out << "# in_bytes acc_bytes opa opb flags bucket tile   device ms per candidate tile "
           "(summed over the tuning run)\n";
    for (auto& kv : best) {
      const TileKey& k = kv.first;
      out << k.in_bytes << ' ' << k.acc_bytes << ' ' << k.opa << ' ' << k.opb << ' ' << k.flags
          << ' ' << k.bucket << ' ' << kv.second << "   #";
      for (auto& tm : T.timed[k]) out << ' ' << tm.first << ':' << tm.second;
      out << '\n';
    }
  }
  T.tiles = best;
  T.loaded = true;
  T.timed.clear();
  return (int)best.size();
}

// The batched GEMM kernels give XCD x the x-th eighth of a launch's products
// (the tiles of one product share its operands in that XCD's L2).  Order a
// batch so that the eighths cost the same: products
// are dealt, largest first, onto the least loaded eighth among those not yet
// full, and each eighth runs its largest first; the batch is padded with
// empty products to a multiple of eight.  Only the order changes, never a
// result.
std::vector<GemmDesc> balance_xcds(const std::vector<GemmDesc>& h, int flags) {
  constexpr int kXcd = 8;
  const size_t per = (h.size() + kXcd - 1) / kXcd;
  if (h.size() < 2 * kXcd || per * kXcd > 65535) return h;  // one launch only
  std::vector<double> cost(per * kXcd, 0.0);
  for (size_t i = 0; i < h.size(); ++i) cost[i] = gemm_flops(h[i], flags);
  std::vector<size_t> idx(cost.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
  std::vector<std::vector<size_t>> grp(kXcd);
  std::vector<double> load(kXcd, 0.0);
  for (size_t i : idx) {
    int best = -1;
    for (int g = 0; g < kXcd; ++g)
      if (grp[g].size() < per && (best < 0 || load[g] < load[best])) best = g;
    grp[best].push_back(i);
    load[best] += cost[i];
  }
  const GemmDesc empty{nullptr, nullptr, nullptr, 0, 0, 0, 1, 1, 1};
  std::vector<GemmDesc> out;
  out.reserve(cost.size());
  for (auto& g : grp)
    for (size_t i : g) out.push_back(i < h.size() ? h[i] : empty);
  return out;
}

template <typename T>
void transpose_batched(const TransDesc* d_desc, int batch, int max_rows, int max_cols,
                       hipStream_t s, const char* name) {
  if (batch <= 0 || max_rows <= 0 || max_cols <= 0) return;
  ProfScope ps(name, s);
  for (int b0 = 0; b0 < batch; b0 += kMaxGridY) {
    const int nb = std::min(batch - b0, kMaxGridY);
    dim3 g((unsigned)ceil_div(max_cols, 32), (unsigned)ceil_div(max_rows, 32), (unsigned)nb);
    hipLaunchKernelGGL((k_transpose<T>), g, dim3(NTHR), 0, s, d_desc + b0);
    HIF_LAUNCH_CHECK();
  }
}
template void transpose_batched<double>(const TransDesc*, int, int, int, hipStream_t, const char*);
template void transpose_batched<float>(const TransDesc*, int, int, int, hipStream_t, const char*);

double gemm_flops(const GemmDesc& d, int flags) {
  const double m = d.m, n = d.n, k = d.k;
  if (d.m <= 0 || d.n <= 0 || d.k <= 0) return 0.0;
  // sum over r < rows of min(r + 1, k) and of max(0, k - r), in closed form
  auto tri_lo = [&](double rows) {
    const double p = std::min(rows, k);
    return p * (p + 1) / 2 + (rows - p) * k;
  };
  auto tri_up = [&](double rows) {
    const double p = std::min(rows, k);
    return p * k - p * (p - 1) / 2;
  };
  if (flags & GF_C_LOWER) {  // computed outputs: i >= j
    const double nn = std::min(n, m);
    return 2.0 * k * (nn * m - nn * (nn - 1) / 2);
  }
  if (flags & GF_A_LOWER) return 2.0 * n * tri_lo(m);  // row i uses t < min(i+1, k)
  if (flags & GF_A_UPPER) return 2.0 * n * tri_up(m);  // row i uses t in [i, k)
  if (flags & GF_B_UPPER) return 2.0 * m * tri_lo(n);  // column j uses t < min(j+1, k)
  if (flags & GF_B_LOWER) return 2.0 * m * tri_up(n);  // column j uses t in [j, k)
  return 2.0 * m * n * k;
}

// Below this many 64-wide tiles a step's panel and trailing launches take
// 32-wide tiles (every tile size sums K in the same order: same results).
constexpr int64_t kFewTiles = 1024;

template <typename T>
void front_factor(const FrontDesc* d_fronts, const std::vector<FrontDesc>& h_fronts,
                  int* err, hipStream_t s, bool upper_zero, int small_limit, int band) {
  const int batch = (int)h_fronts.size();
  if (batch == 0) return;
  if (batch > kMaxGridY) {  // the per-front grid dimension is limited
    for (int b0 = 0; b0 < batch; b0 += kMaxGridY) {
      const int nb = std::min(kMaxGridY, batch - b0);
      std::vector<FrontDesc> sub(h_fronts.begin() + b0, h_fronts.begin() + b0 + nb);
      front_factor<T>(d_fronts + b0, sub, err, s, upper_zero, small_limit, band);
    }
    return;
  }
  int nsmall = 0;
  for (auto& f : h_fronts) nsmall += f.nI <= small_limit;
  if (nsmall > 0 && nsmall < batch) {
    // two size buckets (fronts of several problems or levels): one workgroup
    // per small front, blocked steps only for the large ones
    std::vector<FrontDesc> small, large;
    for (auto& f : h_fronts) (f.nI <= small_limit ? small : large).push_back(f);
    DevBuf<FrontDesc> ds, dl;
    ds.upload(small, s);
    dl.upload(large, s);
    front_factor<T>(ds.get(), small, err, s, upper_zero, small_limit, band);
    front_factor<T>(dl.get(), large, err, s, upper_zero, small_limit, band);
    return;
  }
  int maxI = 0;
  for (auto& f : h_fronts) maxI = std::max(maxI, f.nI);
  if (maxI <= small_limit) {
    double fl = 0.0;
    for (auto& f : h_fronts) {
      const double nI = f.nI, nS = f.nR - f.nI;
      fl += nI * nI * nI / 3.0 + nS * nI * nI;
    }
    {
      ProfScope ps("potrf_small", s, fl);
      hipLaunchKernelGGL((k_front_small<T>), dim3((unsigned)batch), dim3(NTHR), 0, s,
                         d_fronts, err);
      HIF_LAUNCH_CHECK();
    }
    front_invert<T>(d_fronts, h_fronts, s, upper_zero, band, false);
    return;
  }
  // Trailing update of panel columns [p0, p0 + pw) into [c0, c0 + cw).
  auto trailing = [&](int p0, int pw, int c0, int cw) {
    int max_m = 0, max_n = 0;
    double fl = 0.0;
    for (auto& f : h_fronts) {
      const double k = std::min(p0 + pw, f.nI) - p0;
      const int m = f.nR - c0, n = std::min(c0 + cw, f.nI) - c0;
      if (k <= 0 || m <= 0 || n <= 0) continue;
      max_m = std::max(max_m, m);
      max_n = std::max(max_n, n);
      fl += 2.0 * k * ((double)n * m - (double)n * (n - 1) / 2);
    }
    if (max_n == 0) return;
    ProfScope ps("potrf_trailing", s, fl);
    const int64_t nwg64 = ceil_div(max_n, 64) * ceil_div(max_m, 64) * (int64_t)batch;
    if (sizeof(T) == 4 && max_n >= 1024) {
      dim3 gt((unsigned)ceil_div(max_n, 128), (unsigned)ceil_div(max_m, 128), (unsigned)batch);
      hipLaunchKernelGGL((k_front_trailing<T, 128>), gt, dim3(NTHR), 0, s, d_fronts, p0, pw, c0,
                         cw);
    } else if (nwg64 < kFewTiles) {  // few fronts (the root): 32-wide tiles, four times the workgroups
      dim3 gt((unsigned)ceil_div(max_n, 32), (unsigned)ceil_div(max_m, 32), (unsigned)batch);
      hipLaunchKernelGGL((k_front_trailing<T, 32>), gt, dim3(NTHR), 0, s, d_fronts, p0, pw, c0,
                         cw);
    } else {
      dim3 gt((unsigned)std::max<int64_t>(1, ceil_div(max_n, 64)),
              (unsigned)std::max<int64_t>(1, ceil_div(max_m, 64)), (unsigned)batch);
      hipLaunchKernelGGL((k_front_trailing<T, 64>), gt, dim3(NTHR), 0, s, d_fronts, p0, pw, c0,
                         cw);
    }
    HIF_LAUNCH_CHECK();
  };
  // Super-panels of kSuper columns: inside one, each step updates only the
  // columns up to the super-panel's end; the rest of the trailing matrix is
  // updated once per super-panel with all of its columns (rank kSuper), which
  // reads and writes the trailing matrix kSuper / kPanel times less often.
  // A step: the diagonal block factored and inverted once per front, the
  // panel rows below formed as P L_jj^{-T} (a product, 64 rows a workgroup),
  // then the trailing update inside the super-panel.
  constexpr int kSuper = 4 * kPanel;
  for (int J = 0; J < maxI; J += kSuper) {
    const int Je = std::min(J + kSuper, maxI);
    for (int j0 = J; j0 < Je; j0 += kPanel) {
      int max_m = 0;
      double fl_diag = 0.0, fl_panel = 0.0;
      for (auto& f : h_fronts) {
        if (f.nI <= j0) continue;
        const int nb = std::min(kPanel, f.nI - j0);
        const double m = f.nR - j0 - nb;
        max_m = std::max(max_m, (int)m);
        fl_diag += 2.0 * nb * (double)nb * nb / 3.0;  // L_jj and its inverse
        fl_panel += m * nb * (double)(nb + 1);
      }
      {
        ProfScope ps("potrf_diag", s, fl_diag);
        hipLaunchKernelGGL((k_front_diag<T>), dim3((unsigned)batch), dim3(NTHR), 0, s, d_fronts,
                           j0, err);
        HIF_LAUNCH_CHECK();
      }
      if (max_m > 0) {
        ProfScope ps("potrf_panel", s, fl_panel);
        if (ceil_div(max_m, 64) * batch < kFewTiles) {
          dim3 g((unsigned)ceil_div(max_m, 32), (unsigned)batch);
          hipLaunchKernelGGL((k_front_panel<T, 32>), g, dim3(NTHR), 0, s, d_fronts, j0);
        } else {
          dim3 g((unsigned)ceil_div(max_m, 64), (unsigned)batch);
          hipLaunchKernelGGL((k_front_panel<T, 64>), g, dim3(NTHR), 0, s, d_fronts, j0);
        }
        HIF_LAUNCH_CHECK();
      }
      trailing(j0, kPanel, j0 + kPanel, J + kSuper - (j0 + kPanel));
    }
    if (J + kSuper < maxI) {
      // the rest of every front: one batched product (rank kSuper)
      std::vector<GemmDesc> gd;
      double fl = 0.0;
      int max_m = 0, max_n = 0;
      for (auto& f : h_fronts) {
        const int k = std::min(J + kSuper, f.nI) - J;
        const int c0 = J + kSuper;
        const int m = f.nR - c0, n = f.nI - c0;
        if (k <= 0 || m <= 0 || n <= 0) continue;
        T* base = static_cast<T*>(f.ptr);
        const T* P = base + c0 + (int64_t)f.ld * J;
        gd.push_back({P, P, base + c0 + (int64_t)f.ld * c0, m, n, k, f.ld, f.ld, f.ld});
        fl += gemm_flops(gd.back(), GF_C_LOWER);
        max_m = std::max(max_m, m);
        max_n = std::max(max_n, n);
      }
      if (!gd.empty()) {
        gd = balance_xcds(gd, GF_C_LOWER);
        DevBuf<GemmDesc> dd;
        dd.upload(gd, s);
        gemm_batched<T, T>(OP_N, OP_T, GF_C_LOWER, dd.get(), (int)gd.size(), max_m, max_n, T(-1),
                           T(1), s, "potrf_trailing", fl, GC_GENERIC,
                           std::all_of(h_fronts.begin(), h_fronts.end(),
                                       [](const FrontDesc& f) { return f.ld % (16 / (int)sizeof(T)) == 0; }));
      }
    }
  }
  front_invert<T>(d_fronts, h_fronts, s, upper_zero, band, true);
}

// ---- signed LDL^T of one dense front (the root of a periodic problem) -----
//
// A = L S L^T with S = diag(+-1) and L lower triangular with a positive
// diagonal (the paper's LDL^T with L = L_unit |D|^{1/2}), unpivoted, blocked
// right-looking in kPanel-column steps: the diagonal block in one workgroup,
// the panel rows below one per thread, the trailing matrix by the batched GEMM
// with the sign-scaled panel as one operand.

// Diagonal block A(j0:j0+nb, j0:j0+nb) -> L_jj and its signs, in LDS by one
// workgroup, column by column.  A zero (or non-finite) pivot sets *err to id
// and continues with a unit pivot.
template <typename T>
__global__ __launch_bounds__(NTHR) void k_ldl_diag(T* A, int ld, int j0, int nb, T* sgn,
                                                   int* err, int id) {
  __shared__ T a[kPanel][kPanel + 1];  // a[c][r] = A(j0 + r, j0 + c)
  __shared__ T piv, sg;
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += NTHR) {
    const int c = e / nb, r = e % nb;
    a[c][r] = r >= c ? A[(j0 + r) + (int64_t)ld * (j0 + c)] : T(0);
  }
  __syncthreads();
  bool bad = false;
  for (int t = 0; t < nb; ++t) {
    if (tid == 0) {
      T d = a[t][t];
      const bool ok = d != T(0) && isfinite((double)d);
      bad = bad || !ok;
      if (!ok) d = T(1);
      sg = d > T(0) ? T(1) : T(-1);
      piv = sqrt(d > T(0) ? d : -d);
      a[t][t] = piv;
    }
    __syncthreads();
    const T den = sg * piv;
    for (int r = t + 1 + tid; r < nb; r += NTHR) a[t][r] /= den;
    __syncthreads();
    // a(r, c) -= L(r, t) s_t L(c, t) for t < c <= r
    const T st = sg;
    for (int e = tid; e < nb * nb; e += NTHR) {
      const int c = e / nb, r = e % nb;
      if (c > t && r >= c) a[c][r] -= a[t][r] * st * a[t][c];
    }
    if (tid == 0) sgn[j0 + t] = st;
    __syncthreads();
  }
  for (int e = tid; e < nb * nb; e += NTHR) {
    const int c = e / nb, r = e % nb;
    if (r >= c) A[(j0 + r) + (int64_t)ld * (j0 + c)] = a[c][r];
  }
  if (bad) atomicMin(err, id);
}

// Panel rows below the diagonal block: L(i, j0:j1) = A(i, j0:j1) L_jj^{-T} S_j,
// one row per thread; W(i - j1, :) = L(i, j0:j1) S_j, the trailing update's
// left operand (leading dimension ldw).
template <typename T>
__global__ __launch_bounds__(NTHR) void k_ldl_rows(T* A, int ld, int n, int j0, int nb,
                                                   const T* __restrict__ sgn, T* W, int ldw) {
  __shared__ T l[kPanel][kPanel + 1];  // l[c][r] = L_jj(r, c)
  __shared__ T sj[kPanel];
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += NTHR) {
    const int c = e / nb, r = e % nb;
    l[c][r] = r >= c ? A[(j0 + r) + (int64_t)ld * (j0 + c)] : T(0);
  }
  if (tid < nb) sj[tid] = sgn[j0 + tid];
  __syncthreads();
  const int j1 = j0 + nb;
  const int i = j1 + blockIdx.x * NTHR + tid;
  if (i >= n) return;
  T y[kPanel];
#pragma unroll
  for (int t = 0; t < kPanel; ++t) y[t] = t < nb ? A[i + (int64_t)ld * (j0 + t)] : T(0);
  // y L_jj^T = a_i: forward substitution
#pragma unroll
  for (int t = 0; t < kPanel; ++t) {
    if (t < nb) {
      T v = y[t];
#pragma unroll
      for (int u = 0; u < t; ++u) v -= y[u] * l[u][t];
      y[t] = v / l[t][t];
    }
  }
#pragma unroll
  for (int t = 0; t < kPanel; ++t) {
    if (t < nb) {
      const T v = y[t] * sj[t];
      A[i + (int64_t)ld * (j0 + t)] = v;
      W[(i - j1) + (int64_t)ldw * t] = v * sj[t];
    }
  }
}

// In-place inverse of the lower-triangular L_I of every front, bottom-up over
// doubling block sizes: with the two diagonal halves already inverted,
// inv([[A, 0], [B, C]]) = [[A^-1, 0], [-C^-1 B A^-1, C^-1]].
template <typename T>
void front_invert(const FrontDesc* d_fronts, const std::vector<FrontDesc>& h_fronts,
                  hipStream_t s, bool upper_zero, int band, bool diag_done) {
  const int zf = upper_zero ? GF_TRI_ZEROS : 0;
  if (!upper_zero) band = 0;  // (the band shortcut reads stored zeros)
  const int batch = (int)h_fronts.size();
  if (batch == 0) return;
  if (batch > kMaxGridY) {
    for (int b0 = 0; b0 < batch; b0 += kMaxGridY) {
      const int nb = std::min(kMaxGridY, batch - b0);
      std::vector<FrontDesc> sub(h_fronts.begin() + b0, h_fronts.begin() + b0 + nb);
      front_invert<T>(d_fronts + b0, sub, s, upper_zero, band, diag_done);
    }
    return;
  }
  int maxI = 0;
  for (auto& f : h_fronts) maxI = std::max(maxI, f.nI);
  if (!diag_done) {
    ProfScope ps("trtri_diag", s);
    dim3 g((unsigned)ceil_div(maxI, kPanel), (unsigned)batch);
    hipLaunchKernelGGL((k_diag_inv<T>), g, dim3(64), 0, s, d_fronts);
    HIF_LAUNCH_CHECK();
  }
  // W blocks with their leading dimension on the 16-byte grid (a DMA-fed B)
  auto wld = [](int nc) { return (nc + 3) & ~3; };
  int64_t wmax = 0;
  for (int sz = kPanel; sz < maxI; sz *= 2) {
    int64_t w = 0;
    for (auto& f : h_fronts)
      for (int o = 0; o + sz < f.nI; o += 2 * sz) w += (int64_t)wld(std::min(sz, f.nI - o - sz)) * sz;
    wmax = std::max(wmax, w);
  }
  if (wmax == 0) return;
  DevBuf<T> W(wmax);
  std::vector<GemmDesc> g1, g2;
  DevBuf<GemmDesc> d1, d2;
  for (int sz = kPanel; sz < maxI; sz *= 2) {
    g1.clear();
    g2.clear();
    int64_t w = 0;
    int mm = 0, mk = 0;
    double f1 = 0.0, f2 = 0.0;
    // With a band bw < sz, the block B = L(o+sz.., o..o+sz) is nonzero only in
    // its first rb = min(nc, bw) rows and its last bw columns: W = B A^{-1}
    // needs those rows and the matching rows k0.. of A^{-1}, and
    // -C^{-1} W needs the first rb columns of C^{-1}.
    const bool banded = band > 0 && band < sz;
    const int k0 = banded ? sz - band : 0;
    int m1 = 0;
    for (auto& f : h_fronts) {
      T* base = static_cast<T*>(f.ptr);
      for (int o = 0; o + sz < f.nI; o += 2 * sz) {
        const int nc = std::min(sz, f.nI - o - sz);
        const int rb = banded ? std::min(nc, band) : nc;
        T* Bp = base + (o + sz) + (int64_t)f.ld * o;
        T* Ai = base + o + (int64_t)f.ld * o;
        T* Ci = base + (o + sz) + (int64_t)f.ld * (o + sz);
        const int lw = wld(nc);
        g1.push_back({Bp + (int64_t)f.ld * k0, Ai + k0, W.get() + w, rb, sz, sz - k0, f.ld, f.ld,
                      lw});
        g2.push_back({Ci, W.get() + w, Bp, nc, sz, rb, f.ld, lw, f.ld});
        f1 += gemm_flops(g1.back(), banded ? 0 : GF_B_LOWER);
        f2 += gemm_flops(g2.back(), GF_A_LOWER);
        w += (int64_t)lw * sz;
        mm = std::max(mm, nc);
        m1 = std::max(m1, rb);
      }
    }
    (void)mk;
    if (g1.empty()) continue;
    d1.upload(g1, s);
    d2.upload(g2, s);
    // (A^{-1} from row k0 on is no longer aligned with its triangle: the band
    // product drops the mask and multiplies the stored zeros)
    // a DMA-fed B needs its columns on the 16-byte grid (A's rows may be shifted)
    constexpr int V = 16 / (int)sizeof(T);
    auto grid16 = [&](const std::vector<GemmDesc>& g) {
      for (const GemmDesc& e : g)
        if (e.lda % V || e.ldb % V || ((uintptr_t)e.B % 16)) return false;
      return true;
    };
    gemm_batched<T, T>(OP_N, OP_N, (banded ? 0 : GF_B_LOWER) | zf, d1.get(), (int)g1.size(), m1,
                       sz, T(1), T(0), s, "trtri_gemm", f1, GC_GENERIC, grid16(g1));
    gemm_batched<T, T>(OP_N, OP_N, GF_A_LOWER | zf, d2.get(), (int)g2.size(), mm, sz, T(-1), T(0), s,
                       "trtri_gemm", f2, GC_GENERIC, grid16(g2));
  }
}

void pivoted_cholesky(double* G, double* L, const int64_t* goff, const int* nF, const int* ldg,
                      const int64_t* poff, int* perm, int* k, int batch, double eps,
                      const std::vector<int>& h_nF, const std::vector<int64_t>& h_goff,
                      const std::vector<int>& h_ldg, const std::vector<int64_t>& h_poff,
                      hipStream_t s) {
  if (batch <= 0) return;
  int maxF = 0;
  for (int v : h_nF) maxF = std::max(maxF, v);
  const int64_t tot = h_poff.back() + h_nF.back();
  DevBuf<double> dbuf(std::max<int64_t>(tot, 1)), r11(batch);
  DevBuf<int> pivbuf(std::max<int64_t>(tot, 1)), kst(batch);
  HIF_HIP(hipMemsetAsync(kst.get(), 0xff, sizeof(int) * batch, s));  // -1: running
  std::vector<GemmDesc> gd;
  std::vector<int> gb;  // face of each update descriptor
  DevBuf<GemmDesc> dd;
  DevBuf<int> db;
  for (int j0 = 0; j0 < maxF; j0 += kPivPanel) {
    {
      ProfScope ps("pivoted_cholesky", s);
      if (maxF > 1024)
        hipLaunchKernelGGL((k_pchol_panel<1024, kPcholMax>), dim3((unsigned)batch), dim3(1024),
                           0, s, G, L, goff, nF, ldg, poff, perm, dbuf.get(), pivbuf.get(),
                           kst.get(), r11.get(), eps, j0);
      else if (maxF > 256)
        hipLaunchKernelGGL((k_pchol_panel<1024, 1024>), dim3((unsigned)batch), dim3(1024), 0, s,
                           G, L, goff, nF, ldg, poff, perm, dbuf.get(), pivbuf.get(), kst.get(),
                           r11.get(), eps, j0);
      else if (maxF <= 64)
        hipLaunchKernelGGL((k_pchol_panel<64, 64>), dim3((unsigned)batch), dim3(64), 0, s, G, L,
                           goff, nF, ldg, poff, perm, dbuf.get(), pivbuf.get(), kst.get(),
                           r11.get(), eps, j0);
      else
        hipLaunchKernelGGL((k_pchol_panel<NTHR, 256>), dim3((unsigned)batch), dim3(NTHR), 0, s,
                           G, L, goff, nF, ldg, poff, perm, dbuf.get(), pivbuf.get(), kst.get(),
                           r11.get(), eps, j0);
      HIF_LAUNCH_CHECK();
    }
    if (j0 + kPivPanel >= maxF) break;
    // G -= L_p L_p^T with the panel's columns L_p (lower part computed, both written)
    gd.clear();
    gb.clear();
    int mm = 0;
    double fl = 0.0;
    for (int b = 0; b < batch; ++b) {
      if (h_nF[b] <= j0 + kPivPanel) continue;
      const int kk = std::min(kPivPanel, h_nF[b] - j0);
      double* Lp = L + h_goff[b] + (int64_t)h_ldg[b] * j0;
      gd.push_back({Lp, Lp, G + h_goff[b], h_nF[b], h_nF[b], kk, h_ldg[b], h_ldg[b], h_ldg[b]});
      gb.push_back(b);
      mm = std::max(mm, h_nF[b]);
      fl += gemm_flops(gd.back(), GF_C_LOWER);
    }
    if (gd.empty()) continue;
    dd.upload(gd, s);
    db.upload(gb, s);
    hipLaunchKernelGGL(k_pchol_drop_done, dim3((unsigned)ceil_div((int)gd.size(), NTHR)),
                       dim3(NTHR), 0, s, dd.get(), (const int*)db.get(), (const int*)kst.get(),
                       (int)gd.size());
    HIF_LAUNCH_CHECK();
    gemm_batched<double, double>(OP_N, OP_T, GF_C_LOWER | GF_C_MIRROR, dd.get(), (int)gd.size(),
                                 mm, mm, -1.0, 1.0, s, "pivchol_update", fl);
  }
  hipLaunchKernelGGL(k_pchol_tail, dim3((unsigned)batch), dim3(64), 0, s, nF, poff, perm,
                     (const int*)pivbuf.get(), (const int*)kst.get(), k);
  HIF_LAUNCH_CHECK();
}

template void gemm_batched<double, double>(int, int, int, const GemmDesc*, int, int, int, double,
                                           double, hipStream_t, const char*, double, int, bool);
template void gemm_batched<float, float>(int, int, int, const GemmDesc*, int, int, int, float,
                                         float, hipStream_t, const char*, double, int, bool);
template void gemm_batched<float, double>(int, int, int, const GemmDesc*, int, int, int, double,
                                          double, hipStream_t, const char*, double, int, bool);
template <typename T>
void root_ldl(const FrontDesc& f, const FrontDesc* d_front, T* sgn, int* err, hipStream_t s) {
  const int n = f.nI, ld = f.ld;
  T* A = static_cast<T*>(f.ptr);
  DevBuf<T> W((size_t)std::max(1, n) * kPanel);
  DevBuf<GemmDesc> dd;
  for (int j0 = 0; j0 < n; j0 += kPanel) {
    const int nb = std::min(kPanel, n - j0);
    const int j1 = j0 + nb, m = n - j1;
    const double fl = nb * (double)nb * nb / 3.0 + m * (double)nb * nb;
    {
      ProfScope ps("ldl_step", s, fl);
      hipLaunchKernelGGL((k_ldl_diag<T>), dim3(1), dim3(NTHR), 0, s, A, ld, j0, nb, sgn, err,
                         f.id);
      if (m > 0)
        hipLaunchKernelGGL((k_ldl_rows<T>), dim3((unsigned)ceil_div(m, NTHR)), dim3(NTHR), 0, s,
                           A, ld, n, j0, nb, (const T*)sgn, W.get(), std::max(1, m));
      HIF_LAUNCH_CHECK();
    }
    if (m == 0) break;
    // A(j1:n, j1:n) -= (L_21 S) L_21^T, lower triangle
    const std::vector<GemmDesc> g = {{W.get(), A + j1 + (int64_t)ld * j0, A + j1 + (int64_t)ld * j1,
                                      m, m, nb, std::max(1, m), ld, ld}};
    dd.upload(g, s);
    gemm_batched<T, T>(OP_N, OP_T, GF_C_LOWER, dd.get(), 1, m, m, T(-1), T(1), s, "ldl_trailing",
                       gemm_flops(g[0], GF_C_LOWER));
  }
  std::vector<FrontDesc> hf = {f};
  front_invert<T>(d_front, hf, s, true);
}

template void root_ldl<double>(const FrontDesc&, const FrontDesc*, double*, int*, hipStream_t);
template void root_ldl<float>(const FrontDesc&, const FrontDesc*, float*, int*, hipStream_t);

template void front_factor<double>(const FrontDesc*, const std::vector<FrontDesc>&, int*,
                                   hipStream_t, bool, int, int);
template void front_factor<float>(const FrontDesc*, const std::vector<FrontDesc>&, int*,
                                  hipStream_t, bool, int, int);
template void front_invert<double>(const FrontDesc*, const std::vector<FrontDesc>&, hipStream_t,
                                   bool, int, bool);
template void front_invert<float>(const FrontDesc*, const std::vector<FrontDesc>&, hipStream_t,
                                  bool, int, bool);

}  // namespace hif
