"""Plain dense kernels of the CPU oracle, written out from their definitions.

TEST INFRASTRUCTURE ONLY: this package is the independent FP64 reference the
HIP path is checked against.  Only tests, the smoke check and the benchmark's
CPU-baseline leg may import it; the product path never does.

Every routine is a direct transcription of a textbook definition, one column
(or row, or Householder step) at a time; numpy supplies only vector and
matrix-vector products.  No blocking, no reordering.
"""
from __future__ import annotations

import numpy as np


class NotSPD(ArithmeticError):
    """A Cholesky pivot was not strictly positive."""

    def __init__(self, column: int, value: float):
        super().__init__(f"non-positive pivot {value!r} at column {column}")
        self.column = column
        self.value = value


def cholesky(A: np.ndarray) -> np.ndarray:
    """Lower-triangular L with A = L L^T (symmetric positive definite A).

    Column j follows the definition
        L[j,j]^2 = A[j,j] - sum_{t<j} L[j,t]^2
        L[i,j]   = (A[i,j] - sum_{t<j} L[i,t] L[j,t]) / L[j,j],   i > j.
    Only the lower triangle of A is read.  This is the Cholesky (D = I) form
    of the LDL^T factorization the paper uses for A_II and B_{F̌F̌}
    (Section 2.2, sparse elimination; Section 2.3, skeletonization).
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    L = np.zeros((n, n))
    for j in range(n):
        d = A[j, j] - L[j, :j] @ L[j, :j]
        if not d > 0.0:
            raise NotSPD(j, float(d))
        L[j, j] = np.sqrt(d)
        if j + 1 < n:
            L[j + 1:, j] = (A[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    return L


def ldl_signed(A: np.ndarray):
    """Unpivoted symmetric factorization A = L S L^T of a symmetric A whose
    leading principal minors are nonzero: S = diag(+-1), L lower triangular
    with a positive diagonal.  This is the LDL^T factorization the paper
    uses (unit-diagonal factor times D, Section 2.2), stored as
    L = L_unit |D|^{1/2} and S = sign(D).  Column j from the definition:
        d_j    = A[j,j] - sum_{t<j} L[j,t]^2 S[t]
        S[j]   = sign(d_j),  L[j,j] = sqrt(|d_j|)
        L[i,j] = (A[i,j] - sum_{t<j} L[i,t] S[t] L[j,t]) / (S[j] L[j,j]),  i > j.
    Only the lower triangle of A is read.  Raises NotSPD (naming the column)
    on a zero pivot.  For a positive definite A it is the Cholesky factor
    (every S[j] = +1)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    L = np.zeros((n, n))
    S = np.zeros(n)
    for j in range(n):
        d = A[j, j] - (L[j, :j] * S[:j]) @ L[j, :j]
        if d == 0.0 or not np.isfinite(d):
            raise NotSPD(j, float(d))
        S[j] = 1.0 if d > 0.0 else -1.0
        L[j, j] = np.sqrt(abs(d))
        if j + 1 < n:
            L[j + 1:, j] = (A[j + 1:, j] - L[j + 1:, :j] @ (S[:j] * L[j, :j])) / (S[j] * L[j, j])
    return L, S


def _as2d(B):
    B = np.asarray(B, dtype=np.float64)
    return (B[:, None], True) if B.ndim == 1 else (B, False)


def solve_lower(L: np.ndarray, B: np.ndarray) -> np.ndarray:
    """X with L X = B, L lower triangular: forward substitution row by row."""
    B2, vec = _as2d(B)
    n = L.shape[0]
    X = np.zeros_like(B2)
    for i in range(n):
        X[i] = (B2[i] - L[i, :i] @ X[:i]) / L[i, i]
    return X[:, 0] if vec else X


def solve_lower_t(L: np.ndarray, B: np.ndarray) -> np.ndarray:
    """X with L^T X = B, L lower triangular: back substitution row by row."""
    B2, vec = _as2d(B)
    n = L.shape[0]
    X = np.zeros_like(B2)
    for i in range(n - 1, -1, -1):
        X[i] = (B2[i] - L[i + 1:, i] @ X[i + 1:]) / L[i, i]
    return X[:, 0] if vec else X


def solve_upper(U: np.ndarray, B: np.ndarray) -> np.ndarray:
    """X with U X = B, U upper triangular: back substitution row by row."""
    B2, vec = _as2d(B)
    n = U.shape[0]
    X = np.zeros_like(B2)
    for i in range(n - 1, -1, -1):
        X[i] = (B2[i] - U[i, i + 1:] @ X[i + 1:]) / U[i, i]
    return X[:, 0] if vec else X


def cpqr(M: np.ndarray, eps: float):
    """Householder QR with column pivoting, stopped at relative precision eps.

    At step i the remaining column with the largest Euclidean norm over rows
    i.. of the current (partially reduced) matrix is swapped to position i;
    norms are recomputed from the trailing block at every step (no
    downdating); equal norms go to the column with the lowest original index.
    The step records |R_ii| = that largest norm.  The factorization stops at
    the first step whose |R_ii| <= eps * |R_11| (or when rows or columns run
    out), so k = #{i : |R_ii| > eps |R_11|}; k = 0 when M is zero.

    Returns (perm, R, k): perm[j] is the original column at position j, and
    R (k x ncols) is the leading block row of the triangular factor in
    permuted column order, so that M[:, perm] = Q [R; R22-part] with the
    trailing block discarded.  This is the pivoted QR the paper names for the
    interpolative decomposition (Section 2.3; Section 3.3, computation).
    """
    W = np.array(M, dtype=np.float64, copy=True)
    m, ncol = W.shape
    perm = np.arange(ncol)
    r11 = None
    k = 0
    for i in range(min(m, ncol)):
        norms = np.sqrt(np.sum(W[i:, i:] ** 2, axis=0))
        best = norms.max()
        cands = np.nonzero(norms == best)[0] + i
        p = cands[np.argmin(perm[cands])]
        if i == 0:
            r11 = best
            if r11 == 0.0:
                break
        if not best > eps * r11:
            break
        if p != i:
            W[:, [i, p]] = W[:, [p, i]]
            perm[[i, p]] = perm[[p, i]]
        v = W[i:, i].copy()
        alpha = -np.copysign(np.linalg.norm(v), v[0])
        v[0] -= alpha
        vn = np.linalg.norm(v)
        if vn > 0.0:
            v /= vn
            W[i:, i:] -= 2.0 * np.outer(v, v @ W[i:, i:])
        W[i, i] = alpha
        W[i + 1:, i] = 0.0
        k = i + 1
    return perm, W[:k, :].copy(), k


def interp_decomp(M: np.ndarray, eps: float):
    """Interpolative decomposition M[:, F̌] ~= M[:, F̂] T from `cpqr`.

    Returns (skel, redund, T): skel = original columns of the k skeleton
    points, redund = the remaining columns, T = R11^{-1} R12 (k x r).
    """
    perm, R, k = cpqr(M, eps)
    skel = perm[:k]
    redund = perm[k:]
    if k == 0:
        return skel, redund, np.zeros((0, len(redund)))
    T = solve_upper(R[:, :k], R[:, k:])
    return skel, redund, T
