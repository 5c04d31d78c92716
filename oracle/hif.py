"""Plain FP64 CPU hierarchical interpolative factorization (HIF).

TEST INFRASTRUCTURE ONLY.  This is the independent reference the HIP path is
checked against; it shares no code with it.  Only tests, the smoke check and
the benchmark's CPU-baseline leg may import it.

It follows the paper's sequential HIF (Section 2.4) step by step, with the
DHIF reading of skeletonization (Section 3.2: every face of a level is
skeletonized from the same matrix after all sparse eliminations):

  * the operator A is the 7-point discretization of -div(a grad u) + b u
    (eq. "seven-point stencil") with harmonic-mean edge coefficients, either
    with zero Dirichlet values outside an n^3 interior grid (h = 1/(n+1)) or
    periodic on [0,1)^3 as in the paper (Section 2.1: h = 1/n, indices
    wrap around);
  * level l = 0..L-1: sparse elimination of every cell interior I (Section
    2.2), giving Ã^l; then skeletonization of every face F by an
    interpolative decomposition of Ã^l(R, F) (Section 2.3);
  * level L: dense factorization of the remaining active block (Section 2.4).

A^l is kept as a global-index scipy.sparse matrix whose rows and columns of
inactive points are empty; the shells S of interiors and the row sets R of
faces are read off its sparsity structure rather than from geometry.

Readings where the paper is silent (all listed in the design notes):
  - LDL^T is replaced by Cholesky (D = I); F^{-1} is unchanged.  The one
    exception is the root of a periodic problem: there the compressed
    matrix can lose definiteness along the near-null (constant) mode, and
    the root keeps the paper's LDL^T, stored as L S L^T with S = sign(D).
  - Dirichlet layout: the plane x_d = 0 is not a separator; separators of
    level l are the coordinates x_d = w j with j >= 1, w = leaf * 2^l.
    Periodic layout (the paper's, Section 2.1): every x_d = w j, j >= 0, is
    a separator, and the face on x_d = 0 lies between the last and the
    first cell along d.
  - "relative precision eps" of the ID: k = #{i : |R_ii| > eps |R_11|} from
    column-pivoted QR; eps = 0 skips the ID (exact nested dissection).
  - W^l = (prod_I S_I)(prod_F Q_F S_F̌), F^{-1} = W^0 ... W^L W^L^T ... W^0^T.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from .dense import cholesky, interp_decomp, ldl_signed, solve_lower, solve_lower_t


# ---------------------------------------------------------------------------
# Operator (Section 2.4, seven-point stencil)
# ---------------------------------------------------------------------------

def assemble(n: int, a: np.ndarray, b: np.ndarray, bc: str = "dirichlet") -> sp.csr_matrix:
    """7-point operator on the n^3 grid, natural order x1 fastest.

    Row j: (1/h^2) sum_e a_e (u_j - u_k) + b_j u_j over the six neighbours k,
    where a_e is the harmonic mean 2 a_j a_k / (a_j + a_k).
    bc = "dirichlet": h = 1/(n+1); an edge to the zero ghost outside the grid
    uses a_j.  bc = "periodic": h = 1/n and neighbour indices wrap around
    (x = n-1 couples to x = 0).
    """
    if bc == "periodic":
        return _assemble_periodic(n, a, b)
    if bc != "dirichlet":
        raise ValueError(f"unknown boundary condition {bc!r}")
    N = n ** 3
    a = np.asarray(a, dtype=np.float64).reshape(n, n, n)  # axes (x3, x2, x1)
    b = np.asarray(b, dtype=np.float64).reshape(n, n, n)
    h2 = 1.0 / (n + 1) ** 2
    idx = np.arange(N).reshape(n, n, n)
    diag = b.copy()
    rows, cols, vals = [], [], []
    for axis in (2, 1, 0):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, n - 1)
        hi[axis] = slice(1, n)
        lo, hi = tuple(lo), tuple(hi)
        aj, ak = a[lo], a[hi]
        ae = 2.0 * aj * ak / (aj + ak) / h2
        diag[lo] += ae
        diag[hi] += ae
        rows += [idx[lo].ravel(), idx[hi].ravel()]
        cols += [idx[hi].ravel(), idx[lo].ravel()]
        vals += [-ae.ravel(), -ae.ravel()]
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[axis] = 0
        last[axis] = n - 1
        diag[tuple(first)] += a[tuple(first)] / h2
        diag[tuple(last)] += a[tuple(last)] / h2
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    return A.tocsr()


def _assemble_periodic(n: int, a: np.ndarray, b: np.ndarray) -> sp.csr_matrix:
    """The periodic operator: every grid point has six neighbours, the edge
    between j and its wrapped neighbour k carrying 2 a_j a_k / (a_j + a_k) / h^2
    with h = 1/n.  Duplicate entries (n = 2: both neighbours along a
    dimension are the same point) are summed."""
    N = n ** 3
    a = np.asarray(a, dtype=np.float64).reshape(n, n, n)
    b = np.asarray(b, dtype=np.float64).reshape(n, n, n)
    h2 = 1.0 / n ** 2
    idx = np.arange(N).reshape(n, n, n)
    diag = b.copy()
    rows, cols, vals = [], [], []
    for axis in (2, 1, 0):
        ak = np.roll(a, -1, axis=axis)        # the +1 neighbour along axis, wrapped
        kk = np.roll(idx, -1, axis=axis)
        ae = 2.0 * a * ak / (a + ak) / h2
        diag += ae
        diag += np.roll(ae, 1, axis=axis)     # the edge to the -1 neighbour
        rows += [idx.ravel(), kk.ravel()]
        cols += [kk.ravel(), idx.ravel()]
        vals += [-ae.ravel(), -ae.ravel()]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    return A.tocsr()


def energy(n: int, a: np.ndarray, b: np.ndarray, x: np.ndarray) -> float:
    """x^T A x written as a sum over grid edges (used as an independent check)."""
    a = np.asarray(a, dtype=np.float64).reshape(n, n, n)
    x3 = np.asarray(x, dtype=np.float64).reshape(n, n, n)
    h2 = 1.0 / (n + 1) ** 2
    e = float(np.sum(np.asarray(b).reshape(n, n, n) * x3 * x3))
    for axis in range(3):
        d = np.diff(x3, axis=axis)
        aj = np.take(a, range(n - 1), axis=axis)
        ak = np.take(a, range(1, n), axis=axis)
        e += float(np.sum(2 * aj * ak / (aj + ak) * d * d)) / h2
        for end in (0, n - 1):
            xe = np.take(x3, end, axis=axis)
            e += float(np.sum(np.take(a, end, axis=axis) * xe * xe)) / h2
    return e


# ---------------------------------------------------------------------------
# Cell hierarchy (Section 2.1)
# ---------------------------------------------------------------------------

class Geometry:
    """n = leaf * 2^L grid with level-l cells of width w = leaf * 2^l.

    Dirichlet: the separators of level l are x_d = w j with j >= 1.
    Periodic: every x_d = w j (j >= 0) is a separator, and the face on the
    plane j lies between cell j - 1 (mod n / w) and cell j."""

    def __init__(self, n: int, leaf: int, bc: str = "dirichlet"):
        if bc not in ("dirichlet", "periodic"):
            raise ValueError(f"unknown boundary condition {bc!r}")
        self.periodic = bc == "periodic"
        if leaf < 2 or n < leaf:
            raise ValueError("need leaf >= 2 and n >= leaf")
        L = 0
        while leaf << L < n:
            L += 1
        if leaf << L != n:
            raise ValueError(f"n={n} is not leaf*2^L for leaf={leaf}")
        self.n, self.leaf, self.L = n, leaf, L
        idx = np.arange(n ** 3)
        self.coords = (idx % n, (idx // n) % n, idx // (n * n))

    def width(self, level: int) -> int:
        return self.leaf << level

    def classify(self, level: int):
        """Per point: c = number of level-l separator coordinates (0 interior,
        1 face, 2 edge, 3 corner), the lexicographic id of the cell holding an
        interior point, and the id of the face holding a face point."""
        w = self.width(level)
        nc = self.n // w
        if self.periodic:
            sep = [(x % w == 0) for x in self.coords]
            planes, first = nc, 0
        else:
            sep = [(x % w == 0) & (x != 0) for x in self.coords]
            planes, first = nc - 1, 1
        c = sep[0].astype(np.int64) + sep[1] + sep[2]
        cidx = [x // w for x in self.coords]
        cell = (cidx[2] * nc + cidx[1]) * nc + cidx[0]
        face = np.full(self.n ** 3, -1, dtype=np.int64)
        for d in range(3):
            o1, o2 = [e for e in range(3) if e != d]
            on = sep[d] & (c == 1)
            fid = ((d * planes + (cidx[d] - first)) * nc + cidx[o2]) * nc + cidx[o1]
            face[on] = fid[on]
        return c, cell, face


def count_levels(n: int, leaf: int, bc: str = "dirichlet"):
    """Points that first become interior at each level, and the points left
    for the root, read off the classification (eps = 0 elimination counts)."""
    g = Geometry(n, leaf, bc)
    seen = np.zeros(n ** 3, dtype=bool)
    out = []
    for level in range(g.L):
        c, _, _ = g.classify(level)
        new = (c == 0) & ~seen
        out.append(int(new.sum()))
        seen |= new
    return out, int((~seen).sum())


# ---------------------------------------------------------------------------
# Factorization
# ---------------------------------------------------------------------------

@dataclass
class CellFactor:
    """S_I of one cell: interior I, shell S, L_I (A_II = L_I L_I^T), X = L_I^{-1} A_IS."""
    I: np.ndarray
    S: np.ndarray
    L: np.ndarray
    X: np.ndarray


@dataclass
class FaceFactor:
    """Q_F and S_F̌ of one face: skeleton F̂, redundant F̌, interpolation T,
    L_F̌ (B_F̌F̌ = L_F̌ L_F̌^T) and Y = L_F̌^{-1} B_F̂F̌^T."""
    hat: np.ndarray
    chk: np.ndarray
    T: np.ndarray
    Lc: np.ndarray
    Y: np.ndarray
    size: int = 0


@dataclass
class Level:
    cells: list = field(default_factory=list)
    faces: list = field(default_factory=list)
    face_sizes: list = field(default_factory=list)
    face_ranks: list = field(default_factory=list)


@dataclass
class Factor:
    n: int
    leaf: int
    eps: float
    levels: list
    root: np.ndarray
    Lroot: np.ndarray
    bc: str = "dirichlet"
    Sroot: np.ndarray = None   # signs of the root's LDL^T (None: Cholesky, all +1)

    @property
    def root_size(self) -> int:
        return len(self.root)

    def stored_words(self) -> int:
        w = self.Lroot.size
        for lev in self.levels:
            for c in lev.cells:
                w += c.L.size + c.X.size
            for f in lev.faces:
                w += f.T.size + f.Lc.size + f.Y.size
        return int(w)


def _restrict(A: sp.spmatrix, keep: np.ndarray) -> sp.csr_matrix:
    """A with the rows and columns of points outside `keep` removed (left empty)."""
    A = A.tocoo()
    m = keep[A.row] & keep[A.col]
    return sp.csr_matrix((A.data[m], (A.row[m], A.col[m])), shape=A.shape)


def _blocks_to_csr(N, blocks) -> sp.csr_matrix:
    """Sum of dense blocks (rows, cols, values) as one sparse matrix."""
    if not blocks:
        return sp.csr_matrix((N, N))
    r = np.concatenate([np.repeat(rr, len(cc)) for rr, cc, _ in blocks])
    c = np.concatenate([np.tile(cc, len(rr)) for rr, cc, _ in blocks])
    v = np.concatenate([vv.ravel() for _, _, vv in blocks])
    return sp.coo_matrix((v, (r, c)), shape=(N, N)).tocsr()


def _groups(ids: np.ndarray, mask: np.ndarray):
    """Sorted point lists of each id among the masked points, ids ascending."""
    pts = np.nonzero(mask)[0]
    keys = ids[pts]
    order = np.argsort(keys, kind="stable")
    pts, keys = pts[order], keys[order]
    bounds = np.nonzero(np.diff(keys))[0] + 1
    return [(int(g[0]), p) for g, p in zip(np.split(keys, bounds), np.split(pts, bounds))
            if len(p)]


def build(n: int, leaf: int, a: np.ndarray, b: np.ndarray, eps: float,
          bc: str = "dirichlet") -> Factor:
    """Factor A ~= F level by level (Section 2.4 with the Section 3.2 face snapshot)."""
    geo = Geometry(n, leaf, bc)
    N = n ** 3
    A = assemble(n, a, b, bc)
    active = np.ones(N, dtype=bool)
    levels = []
    for level in range(geo.L):
        c, cell, face = geo.classify(level)
        lev = Level()
        # -- sparse elimination of every cell interior (Section 2.2) --------
        Acsr = A.tocsr()
        Acsc = A.tocsc()
        updates = []
        for _, I in _groups(cell, active & (c == 0)):
            rows = np.unique(Acsc[:, I].indices)
            S = np.setdiff1d(rows, I)
            A_II = Acsr[I][:, I].toarray()
            A_SI = Acsr[S][:, I].toarray()
            L = cholesky(A_II)
            X = solve_lower(L, A_SI.T)                      # L_I^{-1} A_IS
            updates.append((S, S, -(X.T @ X)))              # -A_SI A_II^{-1} A_IS
            lev.cells.append(CellFactor(I, S, L, X))
            active[I] = False
        At = (_restrict(A, active) + _blocks_to_csr(N, updates)).tocsc()
        # -- skeletonization of every face from the same Ã^l (Section 2.3) --
        replace = []
        redundant = []
        for _, F in _groups(face, active & (c == 1)):
            sub = At[:, F]
            lev.face_sizes.append(len(F))
            if eps == 0.0:
                lev.face_ranks.append(len(F))
                continue
            R = np.setdiff1d(np.unique(sub.indices), F)
            sub_r = sub.tocsr()
            M = sub_r[R].toarray()
            skel, red, T = interp_decomp(M, eps)
            lev.face_ranks.append(len(skel))
            if len(red) == 0:
                continue
            AFF = sub_r[F].toarray()
            Ahh = AFF[np.ix_(skel, skel)]
            Ahc = AFF[np.ix_(skel, red)]
            Acc = AFF[np.ix_(red, red)]
            Bcc = Acc - T.T @ Ahc - Ahc.T @ T + T.T @ Ahh @ T
            Bhc = Ahc - Ahh @ T
            Lc = cholesky(Bcc)
            Y = solve_lower(Lc, Bhc.T)                     # L_F̌^{-1} B_F̂F̌^T
            Bhh = Ahh - Y.T @ Y                             # B_F̂F̂
            hat, chk = F[skel], F[red]
            lev.faces.append(FaceFactor(hat, chk, T, Lc, Y, len(F)))
            replace.append((hat, hat, Bhh - Ahh))
            redundant.append(chk)
        for chk in redundant:
            active[chk] = False
        A = (_restrict(At, active) + _blocks_to_csr(N, replace)).tocsr()
        levels.append(lev)
    root = np.nonzero(active)[0]
    Aroot = A.tocsr()[root][:, root].toarray()
    if bc == "periodic":
        Lroot, Sroot = ldl_signed(Aroot)
    else:
        Lroot, Sroot = cholesky(Aroot), None
    return Factor(n, leaf, eps, levels, root, Lroot, bc, Sroot)


# ---------------------------------------------------------------------------
# Application of F^{-1} = W^0 ... W^L W^L^T ... W^0^T (Section 2.4)
# ---------------------------------------------------------------------------

def apply_inverse(fac: Factor, f: np.ndarray) -> np.ndarray:
    x = np.array(f, dtype=np.float64, copy=True)
    for lev in fac.levels:                                  # W^l^T, l = 0..L-1
        for cf in lev.cells:                                # S_I^T
            x[cf.I] = solve_lower(cf.L, x[cf.I])
            x[cf.S] -= cf.X.T @ x[cf.I]
        for ff in lev.faces:                                # S_F̌^T Q_F^T
            x[ff.chk] -= ff.T.T @ x[ff.hat]
            x[ff.chk] = solve_lower(ff.Lc, x[ff.chk])
            x[ff.hat] -= ff.Y.T @ x[ff.chk]
    y = solve_lower(fac.Lroot, x[fac.root])                # W^L^T (then D^{-1} = S)
    if fac.Sroot is not None:
        y = fac.Sroot * y
    x[fac.root] = solve_lower_t(fac.Lroot, y)
    for lev in reversed(fac.levels):                        # W^l, l = L-1..0
        for ff in lev.faces:                                # Q_F S_F̌
            x[ff.chk] = solve_lower_t(ff.Lc, x[ff.chk] - ff.Y @ x[ff.hat])
            x[ff.hat] -= ff.T @ x[ff.chk]
        for cf in lev.cells:                                # S_I
            x[cf.I] = solve_lower_t(cf.L, x[cf.I] - cf.X @ x[cf.S])
    return x


def apply_forward(fac: Factor, x: np.ndarray) -> np.ndarray:
    """F x with F = W^0^{-T} ... W^L^{-T} D W^L^{-1} ... W^0^{-1} (Section 2.4,
    the product form of F): the inverse of every elementary step of
    apply_inverse, in the reverse order.  The inverses need the triangular
    factors themselves (products with L and L^T) where apply_inverse solves
    with them."""
    y = np.array(x, dtype=np.float64, copy=True)
    for lev in fac.levels:                                  # W^l^{-1}, l = 0..L-1
        for cf in lev.cells:                                # S_I^{-1}
            y[cf.I] = cf.L.T @ y[cf.I] + cf.X @ y[cf.S]
        for ff in lev.faces:                                # (Q_F S_F̌)^{-1}
            y[ff.hat] += ff.T @ y[ff.chk]
            y[ff.chk] = ff.Lc.T @ y[ff.chk] + ff.Y @ y[ff.hat]
    z = fac.Lroot.T @ y[fac.root]                           # W^L^{-1}, then D
    if fac.Sroot is not None:
        z = fac.Sroot * z
    y[fac.root] = fac.Lroot @ z                             # W^L^{-T}
    for lev in reversed(fac.levels):                        # W^l^{-T}, l = L-1..0
        for ff in reversed(lev.faces):                      # (S_F̌^T Q_F^T)^{-1}
            y[ff.hat] += ff.Y.T @ y[ff.chk]
            y[ff.chk] = ff.Lc @ y[ff.chk] + ff.T.T @ y[ff.hat]
        for cf in reversed(lev.cells):                      # S_I^{-T}
            y[cf.S] += cf.X.T @ y[cf.I]
            y[cf.I] = cf.L @ y[cf.I]
    return y


# ---------------------------------------------------------------------------
# Diagnostics (Section 4, result metrics) and the Krylov driver
# ---------------------------------------------------------------------------

def active_after(fac: Factor, level: int) -> np.ndarray:
    """Mask of the points still active in A^{level+1}: every interior
    eliminated and every redundant face point left out at levels 0..level
    is inactive (Section 2.4, the sets Sigma^l)."""
    N = fac.n ** 3
    active = np.ones(N, dtype=bool)
    for lev in fac.levels[:level + 1]:
        for cf in lev.cells:
            active[cf.I] = False
        for ff in lev.faces:
            active[ff.chk] = False
    return active


def relative_solve_error(fac: Factor, A, x: np.ndarray) -> float:
    """e_s = ||(I - F^{-1} A) x|| / ||x||."""
    return float(np.linalg.norm(x - apply_inverse(fac, A @ x)) / np.linalg.norm(x))


def power_norm_error(fac: Factor, A, iters: int = 30, seed: int = 7, start=None) -> float:
    """||I - F^{-1} A||_2 by power iteration on B^T B, B = I - F^{-1} A,
    B^T = I - A F^{-1} (A and F^{-1} symmetric), from the vector `start`
    (default: a Gaussian vector drawn with `seed`)."""
    if start is None:
        v = np.random.Generator(np.random.PCG64(seed)).standard_normal(A.shape[0])
    else:
        v = np.array(start, dtype=np.float64, copy=True)
    v /= np.linalg.norm(v)
    s = 0.0
    for _ in range(iters):
        Bv = v - apply_inverse(fac, A @ v)
        BtBv = Bv - A @ apply_inverse(fac, Bv)
        s = np.sqrt(np.linalg.norm(BtBv))
        v = BtBv / np.linalg.norm(BtBv)
    return float(s)


def pcg(A, apply, f: np.ndarray, tol: float, maxit: int = 500):
    """Preconditioned CG from u = 0 with the flexible (Polak-Ribiere) beta.

    Stops when the recursive residual reaches tol*||f|| and the true residual
    ||f - A u|| confirms it (else the residual is replaced and CG goes on).
    Returns (u, iterations, true relative residual, converged).
    """
    f = np.asarray(f, dtype=np.float64)
    fn = np.linalg.norm(f)
    u = np.zeros_like(f)
    if fn == 0.0:
        return u, 0, 0.0, True
    r = f.copy()
    z = apply(r)
    p = z.copy()
    rz = r @ z
    for it in range(1, maxit + 1):
        q = A @ p
        alpha = rz / (p @ q)
        u += alpha * p
        r_old = r
        r = r - alpha * q
        if np.linalg.norm(r) <= tol * fn:
            true = np.linalg.norm(f - A @ u)
            if true <= tol * fn:
                return u, it, float(true / fn), True
            r = f - A @ u
        z_new = apply(r)
        beta = (z_new @ (r - r_old)) / rz
        rz = r @ z_new
        p = z_new + beta * p
    return u, maxit, float(np.linalg.norm(f - A @ u) / fn), False


def gmres(A, apply, f: np.ndarray, tol: float, restart: int = 50, maxit: int = 500):
    """Restarted GMRES(restart) with right preconditioning, from u = 0.

    The paper solves A u = f by GMRES with F^{-1} as the preconditioner to a
    relative tolerance of 1e-12 (Section 4).  Each cycle builds the Arnoldi
    basis V of the Krylov space of A F^{-1} started at the residual r
    (modified Gram-Schmidt), and after every step takes y minimising
    || ||r|| e_1 - H y || over the current Hessenberg matrix H (a plain
    least-squares solve, no Givens updating).  When that minimum falls to
    tol * ||f|| (or the cycle ends, or H has a zero subdiagonal), the iterate
    becomes u + F^{-1} V y, and the true residual ||f - A u|| decides between
    stopping and another cycle.  Returns (u, iterations, true relative
    residual, converged); iterations count Arnoldi steps over all cycles.
    """
    f = np.asarray(f, dtype=np.float64)
    fn = np.linalg.norm(f)
    u = np.zeros_like(f)
    if fn == 0.0:
        return u, 0, 0.0, True
    its = 0
    while True:
        r = f - A @ u
        beta = np.linalg.norm(r)
        if beta <= tol * fn:
            return u, its, float(beta / fn), True
        if its >= maxit:
            return u, its, float(beta / fn), False
        V = [r / beta]
        H = np.zeros((restart + 1, restart))
        y = np.zeros(0)
        for j in range(restart):
            w = A @ apply(V[j])
            for i in range(j + 1):
                H[i, j] = V[i] @ w
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            its += 1
            e1 = np.zeros(j + 2)
            e1[0] = beta
            y = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)[0]
            res = np.linalg.norm(e1 - H[:j + 2, :j + 1] @ y)
            if res <= tol * fn or H[j + 1, j] == 0.0 or its >= maxit:
                break
            V.append(w / H[j + 1, j])
        u = u + apply(np.stack(V[:len(y)], axis=1) @ y)
