/*
 * hif.h — C ABI of the MI355X hierarchical interpolative factorization (HIF)
 * of the 3-D variable-coefficient elliptic operator
 *
 *     -div(a(x) grad u(x)) + b(x) u(x) = f(x)          (paper, eq. 1.1)
 *
 * discretized by the 7-point stencil (paper, Section 2.4, "seven-point
 * stencil") with harmonic-mean edge coefficients on an n x n x n grid,
 * either with zero Dirichlet values outside an interior grid (h = 1/(n+1))
 * or periodic on [0,1)^3 as in the paper (Section 2.1: h = 1/n, indices
 * wrap around).
 *
 * The factorization follows the paper's sequential HIF (Section 2.4) with
 * the distributed version's face snapshot (Section 3.2): for each level
 * l = 0..L-1 of the cell tree (cells of width leaf*2^l, Section 2.1) every
 * cell interior is eliminated (Section 2.2) and every face is skeletonized
 * by an interpolative decomposition to relative precision eps (Section
 * 2.3); level L is a dense factorization.  A ~= F and
 * F^{-1} = W^0 ... W^L D^{-1} W^L^T ... W^0^T (Section 2.4).
 *
 * Conventions shared by every call:
 *   - Grid vectors are in natural order: index x1 + n*x2 + n^2*x3 (x1
 *     fastest).  A block of nrhs vectors is column-major N x nrhs, N = n^3.
 *   - Array arguments named a, b, f, u, x, y are DEVICE pointers to doubles
 *     owned by the caller; the library copies what it keeps.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   - Calls that use the same factor must not overlap in time, from several
 *     threads or on several streams: they share its scratch vectors.  The
 *     single-vector preconditioner application inside hif_pcg is captured
 *     into a HIP graph at the second solve with a factor and replayed from
 *     then on (HIF_APPLY_GRAPH=0 in the environment launches it directly).
 *   - Levels of many fronts or faces apply their factor blocks with fused
 *     per-front and per-face kernels; HIF_APPLY_FUSED=0 in the environment
 *     selects the gather / batched matrix-vector / scatter sweeps instead.
 *     Both give the same result up to the order of the FP64 sums.  The
 *     variable is read at every direct application (hif_apply, and the first
 *     PCG solve with a factor); the HIP graph that later hif_pcg solves
 *     replay keeps the choice made when it was captured.
 *   - Every call returns a status; nothing throws or aborts across the ABI.
 *     On error an output handle is set to NULL and nothing leaks;
 *     hif_last_error() gives a thread-local description.
 */
#ifndef HIF_H
#define HIF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hif_problem_s* hif_problem_t; /* operator A (library-owned)          */
typedef struct hif_factor_s* hif_factor_t;   /* factorization F (device arenas)     */

typedef enum {
  HIF_OK = 0,
  HIF_EINVAL = -1,   /* bad sizes/options, non-positive or non-finite a, non-finite b */
  HIF_ENOMEM = -2,   /* device allocation failed                                   */
  HIF_ENOTSPD = -3,  /* a Cholesky pivot was not positive (level/front in message) */
  HIF_ENOCONV = -4,  /* PCG reached maxit; u holds the last iterate                */
  HIF_EDEVICE = -5   /* any other HIP runtime error, or a failed internal check    */
} hif_status;

enum { HIF_FP64 = 0, HIF_MIXED = 1 };  /* factor precision                        */
enum { HIF_DIRICHLET = 0, HIF_PERIODIC = 1 };  /* boundary condition           */

#define HIF_MAX_LEVELS 16

typedef struct {
  int32_t n;         /* grid points per dimension; n = leaf * 2^L, L >= 0         */
  int32_t leaf;      /* leaf cell width m >= 2 (paper: m, Section 2.1)             */
  double eps;        /* ID relative precision; 0 = no ID (exact nested dissection).
                        Otherwise 1e-7 <= eps < 1 (HIF_EINVAL outside): the ID's
                        rank test compares the FP64 Gram matrix's downdated
                        diagonal with eps^2 times its largest entry, which
                        resolves only while eps^2 is far above the FP64 unit
                        roundoff (1.1e-16).                                      */
  int32_t precision; /* HIF_FP64: all front work in FP64.  HIF_MIXED: fronts,
                        Schur updates and skeleton algebra in FP32; ID pivot
                        decisions (Gram + pivoted Cholesky) in FP64.             */
  int32_t bc;        /* HIF_DIRICHLET: zero values outside the grid; separators of
                        level l are the planes x_d = w j, j >= 1 (w = leaf 2^l).
                        HIF_PERIODIC (n >= 4): the paper's setting; every plane
                        x_d = w j, j >= 0, below the root is a separator, the
                        faces on x_d = 0 joining the last and the first cell;
                        the root is factored as L S L^T (the paper's LDL^T, S =
                        sign(D), unpivoted), since compression can make it
                        indefinite along the constant mode.  Cell interiors
                        and the other factored blocks must be definite.      */
} hif_options;

typedef struct {      /* result of hif_pcg, hif_pcg_batched and hif_gmres        */
  int32_t iters;     /* Krylov iterations taken                                   */
  int32_t converged; /* 1 if the true relative residual reached tol               */
  double relres;     /* ||f - A u||_2 / ||f||_2 recomputed in FP64 at exit         */
} hif_pcg_info;

typedef struct {
  int32_t levels;                          /* L                                    */
  int32_t precision;
  int64_t n_dof;                           /* N = n^3                              */
  int64_t root_size;                       /* |Sigma_L|, active DOFs at level L    */
  int64_t cells[HIF_MAX_LEVELS + 1];       /* cells per level (level L: 1 root)    */
  int64_t faces[HIF_MAX_LEVELS];           /* faces per level                      */
  int64_t eliminated[HIF_MAX_LEVELS + 1];  /* interior DOFs eliminated per level   */
  int64_t face_dofs[HIF_MAX_LEVELS];       /* active face DOFs entering the ID     */
  int64_t redundant[HIF_MAX_LEVELS];       /* face DOFs removed as redundant       */
  int64_t max_front[HIF_MAX_LEVELS + 1];   /* largest |I| + |S| per level          */
  double level_seconds[HIF_MAX_LEVELS + 1];/* wall time per level of hif_build     */
  double factor_flops;                     /* algorithmic flops counted per front  */
  int64_t factor_bytes;                    /* bytes of stored factor blocks        */
  int64_t peak_bytes;                      /* device high-water mark of the library */
  double build_seconds;                    /* wall time of hif_build               */
  /* Appended after the fields above (their layout is unchanged): */
  double level_flops[HIF_MAX_LEVELS + 1];  /* algorithmic flops counted per level  */
  int64_t level_bytes[HIF_MAX_LEVELS + 1]; /* stored factor bytes per level        */
  double e_s;       /* relative solve error ||x - F^{-1}A x|| / ||x|| of the last
                       hif_factor_error call (paper, Section 4, result metrics);
                       NaN until then                                          */
  double err_norm;  /* ||I - F^{-1}A||_2 estimated by power iteration in the last
                       hif_factor_error call with power_iters > 0; NaN until then */
} hif_stats;

/* Create the operator A from coefficient fields a (> 0, finite) and b
 * (finite), both device arrays of N doubles.  Builds the 7-point stencil
 * (paper, Section 2.4).  Returns HIF_EINVAL for bad options or values. */
hif_status hif_problem_create(const hif_options* opts, const double* a, const double* b,
                              void* stream, hif_problem_t* out);

/* Factor A ~= F (paper, Sections 2.2-2.4 and 3.2).  Blocks the calling
 * thread: ranks of each level are read back before the next level is
 * planned.  The factor keeps no reference to caller memory.  The ID of a
 * face runs on at most 4096 active points: a level with a larger face
 * (e.g. n = 512, or 256^3 with eps <= 1e-6) returns HIF_EINVAL. */
hif_status hif_build(hif_problem_t A, const hif_options* opts, void* stream,
                     hif_factor_t* out);

/* Factor `count` problems together (paper, Sections 2.2-2.4 and 3.2, as in
 * hif_build): level l of every problem, counted from the leaves, runs as one
 * set of batched launches over the fronts and faces of all problems, and the
 * host waits once per level for all of them.  A, opts and out are host
 * arrays of `count` entries; opts[i] describes A[i] (grids and leaf sizes may
 * differ; precision and eps must be the same for all).  A problem listed
 * twice needs the same leaf both times.  On success out[i] receives the
 * factor of A[i], which is used and destroyed like one from hif_build; its
 * level_seconds and build_seconds are those of the joint build.  On error
 * every out[i] is NULL and nothing leaks.  Blocks the calling thread. */
hif_status hif_build_batched(int32_t count, const hif_problem_t* A, const hif_options* opts,
                             void* stream, hif_factor_t* out);

/* u = F^{-1} f for nrhs column-major vectors (paper, Section 2.4: the
 * product W^0..W^L D^{-1} W^L^T..W^0^T).  FP64 in and out.  One vector: the
 * sweeps are batched matrix-vector products, and the mixed factor is read in
 * FP32 and accumulated in FP64.  Several vectors: the sweeps are batched GEMMs
 * over up to 32 vectors at a time, computed in the factor's precision (the
 * mixed factor's block apply rounds to about 1e-7 relative).  u may alias f
 * (exactly, not partly).  Asynchronous on `stream`.  nrhs = 0 is a no-op. */
hif_status hif_apply(hif_factor_t F, const double* f, double* u, int32_t nrhs, void* stream);

/* y = F x for one vector: the factorization itself, F = W^0^{-T} ... W^L^{-T}
 * D W^L^{-1} ... W^0^{-1} (paper, Section 2.4, the product form of F), which
 * approximates A (F = A up to rounding at eps = 0).  Every elementary step
 * of hif_apply is inverted, in the reverse order; the products with the
 * triangular factors L_I, L_F̌ and L_Sigma, which the factor stores as
 * explicit inverses, are triangular solves with those blocks (one
 * workgroup per block, one step per row: far slower than hif_apply, and
 * meant for checks such as ||(A - F) x|| and F F^{-1} x = x).  FP64 in and
 * out; the mixed factor's blocks are read in FP32.  y may alias x
 * (exactly).  The first call on a factor builds and keeps its block lists.
 * Asynchronous on `stream`. */
hif_status hif_apply_forward(hif_factor_t F, const double* x, double* y, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): u = F^{-1} f
 * for one vector, exactly as hif_apply with nrhs = 1 (same kernels, same
 * result bit for bit), but with every scratch vector of the sweeps in a
 * static device array of the library (64 MiB per GPU, held from the first
 * call on a GPU until the process ends) instead of the factor's own buffers.
 * No device memory is allocated or freed.  The scratch needed is at most
 * about 26 bytes per unknown (the 128^3 problem with 8^3 leaves needs at
 * most 53 MiB); a factor that needs more than 64 MiB returns HIF_EINVAL,
 * with the size it needs in hif_last_error(), and nothing is launched.  Every
 * call on a GPU shares that GPU's array: calls that overlap in time on one
 * GPU (several streams or threads) race and give wrong results.  The array
 * keeps the last call's contents; the sweeps write every entry before they
 * read it.  u may alias f (exactly).  Asynchronous on `stream`. */
hif_status hif_apply_noalloc(hif_factor_t F, const double* f, double* u, void* stream);

/* y = A x for nrhs column-major vectors, FP64: the 7-point operator of
 * hif_problem_create (paper, Section 2.4, seven-point stencil), one thread
 * per grid point.  x and y must not alias.  Asynchronous. */
hif_status hif_matvec(hif_problem_t A, const double* x, double* y, int32_t nrhs, void* stream);

/* Solve A u = f by preconditioned CG with F^{-1} as the preconditioner,
 * FP64 residuals, matvecs and inner products, from u = 0; stops when the
 * true relative residual is <= tol.  The paper (Section 4) uses the HIF as
 * the preconditioner of GMRES; A and F^{-1} are symmetric positive definite
 * here, so CG is the Krylov method used for the timed solve (with the
 * Polak-Ribiere form of beta, which tolerates the slightly non-symmetric
 * FP32 preconditioner).  nrhs > 1: one CG per column, all
 * columns sharing each block application of F^{-1} (see hif_apply); a
 * column stops on its own.  info has nrhs entries (host memory).  f and u
 * must not alias.  Returns HIF_ENOCONV if any column hit maxit.  Blocks the
 * calling thread. */
hif_status hif_pcg(hif_problem_t A, hif_factor_t F, const double* f, double* u, int32_t nrhs,
                   double tol, int32_t maxit, hif_pcg_info* info, void* stream);

/* Solve A u = f by GMRES with F^{-1} as the preconditioner, the Krylov
 * method of the paper's experiments (Section 4: GMRES to a relative
 * tolerance of 1e-12, n_iter in its tables).  Restarted GMRES(restart) from
 * u = 0 with right preconditioning in its flexible form (z_j = F^{-1} v_j
 * kept beside the Arnoldi basis v_j, so the mixed factor's FP32 application
 * is allowed to vary by rounding); Arnoldi orthogonalization by classical
 * Gram-Schmidt applied twice, all vectors and inner products FP64.  A cycle
 * ends when the least-squares residual estimate reaches tol * ||f|| (or
 * after `restart` steps); the true residual ||f - A u|| then decides between
 * stopping and another cycle.  info (one entry, host memory): iters =
 * Arnoldi steps over all cycles, relres = the final true relative residual,
 * converged = relres <= tol.  Needs 1 <= restart <= 1024 and device memory
 * for 2 * restart + 2 vectors of N doubles.  f and u must not alias.
 * Returns HIF_ENOCONV when maxit steps do not reach tol (u holds the last
 * iterate).  Blocks the calling thread. */
hif_status hif_gmres(hif_problem_t A, hif_factor_t F, const double* f, double* u, double tol,
                     int32_t restart, int32_t maxit, hif_pcg_info* info, void* stream);

/* hif_pcg for several problems at once: for each i, one single-vector PCG
 * solve of A[i] u[i] = f[i] with F[i] (as hif_pcg with nrhs = 1).  The solves
 * run concurrently on library-owned streams (ordered after `stream`, which
 * then waits for all of them), so that the latency-bound iterations of small
 * problems overlap.  A, F, f, u and info are host arrays of `count` entries;
 * f[i] and u[i] are device pointers; no factor may appear twice.  Returns
 * HIF_ENOCONV if any solve hit maxit.  Blocks the calling thread. */
hif_status hif_pcg_batched(int32_t count, const hif_problem_t* A, const hif_factor_t* F,
                           const double* const* f, double* const* u, double tol, int32_t maxit,
                           hif_pcg_info* info, void* stream);

/* Sizes, ranks, flops, bytes and times of a factor (host struct): the
 * result metrics of the paper's Section 4 (|Sigma_L| = root_size, factor
 * time t_f = build_seconds, memory m_f = peak_bytes / factor_bytes, e_s and
 * ||I - F^{-1}A|| after hif_factor_error) plus per-level counts. */
hif_status hif_factor_stats(hif_factor_t F, hif_stats* out);

/* Rank k of every face of `level` in face order (faces enumerated by
 * (normal d, plane j_d (>= 1 Dirichlet, >= 0 periodic), then the other two
 * cell indices, slowest first)), and the face sizes |F| (host arrays of `cap` entries; either
 * may be NULL).  *count receives the number of faces. */
hif_status hif_factor_ranks(hif_factor_t F, int32_t level, int32_t* ranks, int32_t* sizes,
                            int32_t cap, int32_t* count);

/* Active-DOF mask after `level` (0..L-1): mask[p] = 1 if grid point p is
 * still active in A^{level+1} (host array of N bytes). */
hif_status hif_factor_active(hif_factor_t F, int32_t level, uint8_t* mask);

/* Write the factorization to the file `path` (created or truncated): the
 * stored blocks of F (paper, Section 2.4: the factors of every S_I, Q_F,
 * S_F̌ and of the root, in the factor's precision) with the options,
 * statistics, ranks and skeleton choices, so that hif_factor_load can
 * rebuild it without the problem.  A 128^3 mixed factor takes about 8 GB.
 * Blocks the calling thread (device blocks are copied to the host first).
 * HIF_EINVAL if the file cannot be written. */
hif_status hif_factor_save(hif_factor_t F, const char* path, void* stream);

/* Read a file written by hif_factor_save into a new factor on the current
 * device (used and destroyed like one from hif_build; hif_pcg and
 * hif_gmres need a problem of the same grid and boundary condition).
 * Applications of the loaded factor equal those of the saved one bit for
 * bit.  HIF_EINVAL for a missing, truncated or foreign file (*out = NULL,
 * nothing leaks).  Blocks the calling thread. */
hif_status hif_factor_load(const char* path, void* stream, hif_factor_t* out);

/* Accuracy of F as an approximation of A (paper, Section 4, result
 * metrics): *e_s = ||x - F^{-1} A x||_2 / ||x||_2 for the caller's device
 * vector x (N doubles, e.g. i.i.d. Gaussian), and, if power_iters > 0,
 * *err_norm = an estimate of ||I - F^{-1} A||_2 from power_iters steps of
 * the power method on B^T B, B = I - F^{-1} A, B^T = I - A F^{-1}, started
 * at x (either output pointer may be NULL; *err_norm is NaN when
 * power_iters = 0).  Both are also stored in the factor's hif_stats.  FP64
 * vectors; single-vector applies of F^{-1}.  Blocks the calling thread. */
hif_status hif_factor_error(hif_problem_t A, hif_factor_t F, const double* x, int32_t power_iters,
                            double* e_s, double* err_norm, void* stream);

/* Per-kernel-class device timing.  hif_profile_begin() clears and starts
 * recording: every library kernel launch made afterwards (on any stream)
 * is bracketed by a pair of HIP events recorded on that launch's stream,
 * together with the launch's algorithmic flops and bytes.  hif_profile_end()
 * waits for the recorded events, stops recording and returns one entry per
 * kernel class (host array of `cap` entries; *count = number of classes).
 * Process-wide and not thread safe; it exists for benchmarks and
 * roofline measurements. */
typedef struct {
  char name[40];     /* kernel class, e.g. "gemm_syrk", "apply_up_L"           */
  int64_t launches;  /* timed launches                                        */
  double seconds;    /* summed event-to-event device time                     */
  double flops;      /* algorithmic flops of those launches (0: not counted)  */
  double bytes;      /* algorithmic HBM bytes of those launches (0: not counted) */
} hif_kernel_stat;

hif_status hif_profile_begin(void);
hif_status hif_profile_end(hif_kernel_stat* out, int32_t cap, int32_t* count);

/* Restrict the recording of hif_profile_begin to the kernel classes named in
 * `classes`, a comma-separated list of class names without the "@level"
 * suffix (e.g. "gemm_syrk"), so that a timed region carries event pairs
 * around those launches only.  NULL or "" records every class again.  Takes
 * effect for launches made after the call; process-wide, not thread safe. */
hif_status hif_profile_select(const char* classes);

/* Device memory the library released is kept in a process-wide cache for
 * reuse by later calls (up to three quarters of the device's memory; an
 * allocation that finds the device full empties the cache and retries).
 * This returns all of it to the device after a device synchronization, e.g.
 * between workloads of very different sizes.  Memory held by live problems
 * and factors is not touched. */
hif_status hif_release_cached_memory(void);

/* Tile autotuning (tune_tiles.py drives it; not needed to factor or solve).
 * The batched GEMMs of the library run square tiles of 32, 64 or (FP32
 * accumulation only) 128, chosen per key (operand bytes, accumulator bytes,
 * transposes, triangular flags, size bucket = smallest power of two >= the
 * batch's largest m or n) from the table file tiles.tsv beside the library,
 * else by a built-in rule (128 for FP32 outputs of at least 1024 x 1024, else
 * 64).
 * hif_tune_begin: from now on every batched GEMM that overwrites its output
 * is run and timed with each candidate tile (results are unchanged: all tiles
 * take K in the same order).  Run the builds and solves to tune on.
 * hif_tune_end: pick the fastest tile per key, write the table to `path`
 * (NULL or "": do not write), use it from now on, and return the number of
 * keys in *keys (may be NULL).  Process-wide; not thread safe. */
hif_status hif_tune_begin(void);
hif_status hif_tune_end(const char* path, int32_t* keys);

void hif_factor_destroy(hif_factor_t F);
void hif_problem_destroy(hif_problem_t A);

const char* hif_status_string(hif_status s);
const char* hif_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HIF_H */
