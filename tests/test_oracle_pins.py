"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test ties one part of the oracle to a closed form, an invariant, a
library routine on inputs where it is the same mathematical object, or the
paper's own matrix definitions written out in full.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import oracle as O
from workloads import const_field, log_uniform_field, uniform_field


# --- operator (Section 2.4, seven-point stencil) ----------------------------

def test_assembly_sine_eigenpairs():
    """a = 1, b = 0: v = prod_d sin(pi k_d (j_d+1) h) is an eigenvector with
    lambda = (4/h^2) sum_d sin^2(pi k_d h / 2), h = 1/(n+1)."""
    n = 7
    A = O.assemble(n, const_field(n, 1.0), const_field(n, 0.0))
    h = 1.0 / (n + 1)
    j = np.arange(n)
    for k in [(1, 1, 1), (2, 5, 3), (7, 1, 4)]:
        s = [np.sin(np.pi * kd * (j + 1) * h) for kd in k]
        v = np.einsum("k,j,i->kji", s[2], s[1], s[0]).ravel()
        lam = 4.0 / h ** 2 * sum(np.sin(np.pi * kd * h / 2) ** 2 for kd in k)
        assert np.linalg.norm(A @ v - lam * v) <= 1e-12 * lam * np.linalg.norm(v)


def test_assembly_energy_and_symmetry():
    """x^T A x equals the edge-by-edge energy sum; A is exactly symmetric."""
    n = 6
    a = log_uniform_field(n, -2, 2, 11)
    b = uniform_field(n, 0, 1, 12)
    A = O.assemble(n, a, b)
    assert abs(A - A.T).max() == 0.0
    g = np.random.default_rng(3)
    for _ in range(3):
        x = g.standard_normal(n ** 3)
        e = O.energy(n, a, b, x)
        assert abs(x @ (A @ x) - e) <= 1e-12 * e


def test_assembly_rejects_arithmetic_mean():
    """The energy pin separates harmonic from arithmetic edge averages."""
    n = 5
    a = log_uniform_field(n, -2, 2, 13)
    b = const_field(n, 0.0)
    A = O.assemble(n, a, b)
    x = np.random.default_rng(4).standard_normal(n ** 3)
    a3 = a.reshape(n, n, n)
    h2 = 1.0 / (n + 1) ** 2
    e_arith = 0.0
    x3 = x.reshape(n, n, n)
    for ax in range(3):
        d = np.diff(x3, axis=ax)
        am = 0.5 * (np.take(a3, range(n - 1), axis=ax) + np.take(a3, range(1, n), axis=ax))
        e_arith += np.sum(am * d * d) / h2
        for end in (0, n - 1):
            e_arith += np.sum(np.take(a3, end, axis=ax) * np.take(x3, end, axis=ax) ** 2) / h2
    assert abs(x @ (A @ x) - e_arith) > 1e-6 * e_arith


# --- dense kernels vs LAPACK -------------------------------------------------

def _spd(n, seed):
    g = np.random.default_rng(seed)
    B = g.standard_normal((n, n))
    return B @ B.T + n * np.eye(n)


@pytest.mark.parametrize("n", [1, 5, 37])
def test_cholesky_vs_lapack(n):
    A = _spd(n, n)
    assert np.allclose(O.cholesky(A), sla.cholesky(A, lower=True), rtol=1e-13, atol=1e-13)


def test_cholesky_rejects_indefinite():
    A = _spd(6, 1)
    A[3, 3] = -1.0
    with pytest.raises(O.NotSPD):
        O.cholesky(A)


def test_triangular_solves_vs_lapack():
    g = np.random.default_rng(5)
    L = np.tril(g.standard_normal((23, 23))) + 23 * np.eye(23)
    B = g.standard_normal((23, 4))
    assert np.allclose(O.solve_lower(L, B), sla.solve_triangular(L, B, lower=True), rtol=1e-13)
    assert np.allclose(O.solve_lower_t(L, B), sla.solve_triangular(L.T, B, lower=False),
                       rtol=1e-13)
    assert np.allclose(O.solve_upper(L.T, B[:, 0]), sla.solve_triangular(L.T, B[:, 0]),
                       rtol=1e-13)


@pytest.mark.parametrize("shape", [(40, 12), (12, 12), (9, 15)])
def test_cpqr_vs_lapack(shape):
    """Same pivots and |R| as LAPACK's geqp3 on a tie-free random matrix (eps = 0
    runs to full rank)."""
    M = np.random.default_rng(sum(shape)).standard_normal(shape)
    perm, R, k = O.cpqr(M, 0.0)
    _, R2, p2 = sla.qr(M, pivoting=True, mode="economic")
    assert k == min(shape)
    assert np.array_equal(perm[:k], p2[:k])
    assert np.allclose(np.abs(R), np.abs(R2[:k]), rtol=1e-12, atol=1e-12)


def test_id_exact_rank_and_bound():
    """An exact rank-6 matrix gives k = 6; the ID residual obeys
    ||M_F̌ - M_F̂ T||_F <= sqrt(r) eps |R_11| for any eps."""
    g = np.random.default_rng(9)
    M = g.standard_normal((50, 6)) @ g.standard_normal((6, 20))
    skel, red, T = O.interp_decomp(M, 1e-12)
    assert len(skel) == 6
    assert np.linalg.norm(M[:, red] - M[:, skel] @ T) <= 1e-10 * np.linalg.norm(M)
    W = g.standard_normal((60, 30)) * np.logspace(0, -9, 30)
    for eps in (1e-2, 1e-5, 1e-8):
        perm, R, k = O.cpqr(W, eps)
        skel, red, T = O.interp_decomp(W, eps)
        r11 = np.linalg.norm(W, axis=0).max()
        res = np.linalg.norm(W[:, red] - W[:, skel] @ T)
        assert res <= np.sqrt(len(red)) * eps * r11 * (1 + 1e-8)
        assert 0 < k < 30


def test_id_zero_matrix():
    skel, red, T = O.interp_decomp(np.zeros((5, 4)), 1e-6)
    assert len(skel) == 0 and len(red) == 4 and T.shape == (0, 4)


# --- hierarchy (Section 2.1) ------------------------------------------------

@pytest.mark.parametrize("n,m", [(4, 2), (8, 2), (16, 4), (12, 3), (48, 6), (64, 8), (128, 8)])
def test_level_counts_closed_form(n, m):
    """With the Dirichlet layout, s_l = n / w_l - 1 separator coordinates per
    dimension at level l, so (n - s_l)^3 points are interior at or before
    level l; the root keeps n^3 - (n - 1)^3."""
    counts, root = O.count_levels(n, m)
    L = len(counts)
    cum = [(n - (n // (m << l) - 1)) ** 3 for l in range(L)]
    assert counts == [cum[0]] + [cum[l] - cum[l - 1] for l in range(1, L)]
    assert root == n ** 3 - (n - 1) ** 3
    assert sum(counts) + root == n ** 3


# --- whole factorization -----------------------------------------------------

@pytest.mark.parametrize("n,m", [(8, 2), (12, 3), (16, 4), (16, 8), (4, 4)])
def test_eps0_is_exact_solve(n, m):
    """eps = 0 skips every ID: the HIF is exact nested dissection, F^{-1} = A^{-1}."""
    a = log_uniform_field(n, -2, 2, 21)
    b = uniform_field(n, 0, 1, 22)
    A = O.assemble(n, a, b)
    fac = O.build(n, m, a, b, 0.0)
    f = np.random.default_rng(23).standard_normal(n ** 3)
    x = O.apply_inverse(fac, f)
    xd = spla.spsolve(A.tocsc(), f)
    assert np.linalg.norm(x - xd) <= 1e-12 * np.linalg.norm(xd)
    counts, root = O.count_levels(n, m)
    assert [sum(len(c.I) for c in lev.cells) for lev in fac.levels] == counts
    assert fac.root_size == root


def _explicit_W(fac, N):
    """W^l written out as dense N x N products of the paper's S_I, Q_F, S_F̌."""
    Ws = []
    for lev in fac.levels:
        W = np.eye(N)
        for cf in lev.cells:
            S = np.eye(N)
            Linv_t = np.linalg.inv(cf.L).T
            S[np.ix_(cf.I, cf.I)] = Linv_t                   # L_I^{-T}
            S[np.ix_(cf.I, cf.S)] = -Linv_t @ cf.X          # -A_II^{-1} A_IS
            W = W @ S
        for ff in lev.faces:
            Q = np.eye(N)
            Q[np.ix_(ff.hat, ff.chk)] = -ff.T               # [[I,0],[-T,I]] on (F̌, F̂)
            S = np.eye(N)
            Lc_inv_t = np.linalg.inv(ff.Lc).T
            S[np.ix_(ff.chk, ff.chk)] = Lc_inv_t            # L_F̌^{-T}
            S[np.ix_(ff.chk, ff.hat)] = -Lc_inv_t @ ff.Y    # -B_F̌F̌^{-1} B_F̂F̌^T
            W = W @ Q @ S
        Ws.append(W)
    WL = np.eye(N)
    WL[np.ix_(fac.root, fac.root)] = np.linalg.inv(fac.Lroot).T
    Ws.append(WL)
    return Ws


@pytest.mark.parametrize("eps", [0.0, 1e-3])
def test_sweeps_equal_explicit_product(eps):
    """The sweeps in apply_inverse equal W^0...W^L W^L^T...W^0^T built from the
    paper's matrices; at eps = 0 the congruence W^T A W is the identity."""
    n, m = 8, 2
    N = n ** 3
    a = log_uniform_field(n, -1, 1, 31)
    b = const_field(n, 0.0)
    A = O.assemble(n, a, b).toarray()
    fac = O.build(n, m, a, b, eps)
    if eps > 0:
        assert sum(len(f.chk) for lev in fac.levels for f in lev.faces) > 0
    Ws = _explicit_W(fac, N)
    W = np.eye(N)
    for Wl in Ws:
        W = W @ Wl
    Finv = W @ W.T
    cols = np.random.default_rng(5).choice(N, 40, replace=False)
    E = np.eye(N)[:, cols]
    got = np.stack([O.apply_inverse(fac, E[:, i]) for i in range(len(cols))], axis=1)
    assert np.abs(got - Finv[:, cols]).max() <= 1e-12 * np.abs(Finv).max()
    if eps == 0.0:
        assert np.abs(W.T @ A @ W - np.eye(N)).max() <= 1e-10


def test_inverse_is_symmetric_positive():
    n, m = 16, 4
    a = log_uniform_field(n, -2, 2, 41)
    b = const_field(n, 0.0)
    fac = O.build(n, m, a, b, 1e-3)
    g = np.random.default_rng(42)
    x, y = g.standard_normal(n ** 3), g.standard_normal(n ** 3)
    fx, fy = O.apply_inverse(fac, x), O.apply_inverse(fac, y)
    assert abs(y @ fx - x @ fy) <= 1e-12 * np.linalg.norm(fx) * np.linalg.norm(y)
    assert x @ fx > 0 and y @ fy > 0


def test_error_scales_with_eps():
    """e_s and ||I - F^{-1}A||_2 fall roughly like eps (log-log slope in [0.5, 1.5])."""
    n, m = 16, 4
    a = log_uniform_field(n, -1, 1, 51)
    b = const_field(n, 0.0)
    A = O.assemble(n, a, b)
    x = np.random.default_rng(52).standard_normal(n ** 3)
    epss = [1e-2, 1e-4, 1e-6, 1e-8]
    es, pn = [], []
    for eps in epss:
        fac = O.build(n, m, a, b, eps)
        es.append(O.relative_solve_error(fac, A, x))
        pn.append(O.power_norm_error(fac, A, iters=15))
    for vals in (es, pn):
        slope = np.polyfit(np.log10(epss), np.log10(vals), 1)[0]
        assert 0.5 <= slope <= 1.5, (vals, slope)
    assert all(e < 10 * eps for e, eps in zip(es, epss))


def test_pcg_matches_direct_solve():
    n, m = 16, 4
    a = log_uniform_field(n, -2, 2, 61)
    b = const_field(n, 0.0)
    A = O.assemble(n, a, b)
    f = np.random.default_rng(62).standard_normal(n ** 3)
    fac = O.build(n, m, a, b, 1e-2)
    u, its, rel, ok = O.pcg(A, lambda r: O.apply_inverse(fac, r), f, 1e-12, 200)
    assert ok and rel <= 1e-12
    ud = spla.spsolve(A.tocsc(), f)
    assert np.linalg.norm(u - ud) <= 1e-9 * np.linalg.norm(ud)


@pytest.mark.slow
def test_pcg_iterations_bounded_in_n():
    """Iteration counts at fixed eps stay flat as n doubles (paper: Section 4, Example 1)."""
    its = []
    for n, m in [(8, 4), (16, 4), (32, 4)]:
        a = const_field(n, 1.0)
        b = const_field(n, 0.0)
        A = O.assemble(n, a, b)
        f = np.random.default_rng(71).standard_normal(n ** 3)
        fac = O.build(n, m, a, b, 1e-3)
        _, it, rel, ok = O.pcg(A, lambda r: O.apply_inverse(fac, r), f, 1e-10, 200)
        assert ok
        its.append(it)
    assert max(its) - min(its) <= 3, its


@pytest.mark.parametrize("n,leaf", [(16, 4), (24, 6)])
def test_edge_columns_are_orthogonal(n, leaf):
    """Why edges are not skeletonized: the couplings of the points of one
    level-l edge to everything outside the edge have disjoint supports (each
    outside neighbour touches one edge point), so an ID of an edge could only
    drop columns by norm.  At eps = 1e-4 on the high-contrast field none
    qualifies.  Edge points never receive fill, so the same holds for the
    matrix seen after any level's eliminations."""
    a = log_uniform_field(n, -2, 2, 191)
    A = O.assemble(n, a, np.zeros(n ** 3)).tocsc()
    geo = O.Geometry(n, leaf)
    checked = 0
    for level in range(geo.L):
        c, _, _ = geo.classify(level)
        w = geo.width(level)
        xs = geo.coords
        edge = np.flatnonzero(c == 2)
        # group edge points into edges: the free coordinate varies, the two
        # separator coordinates and the segment index along the free one fix it
        keys = {}
        for p in edge:
            co = [int(xs[d][p]) for d in range(3)]
            free = [d for d in range(3) if not (co[d] % w == 0 and co[d] != 0)][0]
            k = tuple(co[d] if d != free else -1 - co[d] // w for d in range(3))
            keys.setdefault(k, []).append(p)
        for pts in keys.values():
            E = np.array(sorted(pts))
            outside = np.ones(n ** 3, bool)
            outside[E] = False
            M = A[:, E][outside, :].toarray()
            G = M.T @ M
            off = G - np.diag(np.diag(G))
            assert np.all(off == 0.0)
            norms = np.sqrt(np.diag(G))
            assert np.all(norms > 1e-4 * norms.max())
            checked += 1
    assert checked > 0


@pytest.mark.parametrize("n,m", [(8, 2), (12, 3), (16, 4), (32, 8)])
def test_face_sizes_closed_form(n, m):
    """At eps = 0 every face point stays active, so level l has 3 (nc-1) nc^2
    faces (nc = n / w cells per dimension, w = m 2^l) and a face spans, along
    each of its two in-plane dimensions, the w points of a first cell (the
    plane x = 0 is no separator) or the w - 1 points of any other cell.  The
    sizes are listed in the face order of the C ABI: normal d, plane j >= 1,
    then the slower and the faster in-plane cell index."""
    fac = O.build(n, m, log_uniform_field(n, -1, 1, 5), const_field(n, 0.0), 0.0)
    for level, lev in enumerate(fac.levels):
        w = m << level
        nc = n // w

        def width(i):
            return w if i == 0 else w - 1
        expect = [width(i_lo) * width(i_hi) for d in range(3) for j in range(1, nc)
                  for i_hi in range(nc) for i_lo in range(nc)]
        assert len(expect) == 3 * (nc - 1) * nc * nc
        assert lev.face_sizes == expect
        assert lev.face_ranks == expect


@pytest.mark.parametrize("n,m,eps", [(6, 3, 1e-3), (8, 2, 1e-3), (8, 4, 1e-2)])
def test_power_norm_error_vs_dense(n, m, eps):
    """The power-method estimate of ||I - F^{-1}A||_2 equals the largest
    singular value of the dense matrix I - F^{-1}A, formed column by column
    from the sweeps, and never exceeds it (the method converges from below)."""
    a = log_uniform_field(n, -1, 1, 9)
    b = const_field(n, 0.0)
    fac = O.build(n, m, a, b, eps)
    A = O.assemble(n, a, b)
    N = n ** 3
    Finv = np.stack([O.apply_inverse(fac, e) for e in np.eye(N)], axis=1)
    sigma = np.linalg.norm(np.eye(N) - Finv @ A.toarray(), 2)
    est = O.power_norm_error(fac, A, iters=40)
    assert est <= sigma * (1 + 1e-10)
    assert est >= sigma * (1 - 1e-6), (est, sigma)


def test_active_after_counts():
    """The active set after level l keeps exactly the points not eliminated
    as interiors and not left out as redundant face points up to l; at the
    last level it is the root."""
    n, m = 16, 4
    fac = O.build(n, m, log_uniform_field(n, -2, 2, 17), const_field(n, 0.0), 1e-3)
    left = n ** 3
    for level, lev in enumerate(fac.levels):
        left -= sum(len(c.I) for c in lev.cells) + sum(len(f.chk) for f in lev.faces)
        assert int(O.active_after(fac, level).sum()) == left
    assert np.array_equal(np.flatnonzero(O.active_after(fac, len(fac.levels) - 1)), fac.root)


# --- GMRES (Section 4: the paper's Krylov solver) ---------------------------

def test_gmres_distinct_eigenvalues():
    """Unpreconditioned GMRES on a diagonal matrix with k distinct eigenvalues
    reaches the exact solution in exactly k steps (the minimal polynomial of
    A has degree k); one step fewer leaves a residual far above tol."""
    import scipy.sparse as sp
    vals = np.repeat([1.0, 2.0, 3.5, 7.0, 11.0], 20)
    A = sp.diags(vals).tocsr()
    f = np.random.default_rng(81).standard_normal(len(vals))
    u, its, rel, ok = O.gmres(A, lambda r: r, f, 1e-12, restart=50, maxit=50)
    assert ok and its == 5 and rel <= 1e-12
    assert np.allclose(u, f / vals, rtol=1e-12, atol=0)
    _, its4, rel4, ok4 = O.gmres(A, lambda r: r, f, 1e-12, restart=50, maxit=4)
    assert not ok4 and its4 == 4 and rel4 > 1e-6


def test_gmres_exact_preconditioner_one_step():
    """At eps = 0 F^{-1} = A^{-1}: GMRES with it converges in one step."""
    n, m = 8, 2
    a = log_uniform_field(n, -2, 2, 83)
    b = const_field(n, 0.0)
    A = O.assemble(n, a, b)
    fac = O.build(n, m, a, b, 0.0)
    f = np.random.default_rng(84).standard_normal(n ** 3)
    u, its, rel, ok = O.gmres(A, lambda r: O.apply_inverse(fac, r), f, 1e-12)
    assert ok and its == 1 and rel <= 1e-12


@pytest.mark.parametrize("restart", [50, 2])
def test_gmres_matches_direct_solve(restart):
    """With the eps = 1e-2 HIF as preconditioner GMRES (also restarted every
    two steps) reaches 1e-12 and the direct solution."""
    n, m = 16, 4
    a = log_uniform_field(n, -2, 2, 85)
    b = const_field(n, 0.0)
    A = O.assemble(n, a, b)
    fac = O.build(n, m, a, b, 1e-2)
    f = np.random.default_rng(86).standard_normal(n ** 3)
    u, its, rel, ok = O.gmres(A, lambda r: O.apply_inverse(fac, r), f, 1e-12, restart, 300)
    assert ok and rel <= 1e-12
    assert np.linalg.norm(f - A @ u) <= 1e-12 * np.linalg.norm(f)
    ud = spla.spsolve(A.tocsc(), f)
    assert np.linalg.norm(u - ud) <= 1e-9 * np.linalg.norm(ud)


# --- forward operator F (Section 2.4, product form) ---------------------------

@pytest.mark.parametrize("bc,bval", [("dirichlet", 0.0), ("periodic", 0.1)])
@pytest.mark.parametrize("eps", [0.0, 1e-3])
def test_forward_apply_inverts_and_reduces_to_A(bc, bval, eps):
    """F (F^{-1} x) = x to rounding; at eps = 0 F is A itself; at eps > 0
    ||(A - F) x|| stays of the order of eps ||A x||."""
    n, m = 8, 2
    a = log_uniform_field(n, -1, 1, 31)
    b = const_field(n, bval)
    A = O.assemble(n, a, b, bc)
    fac = O.build(n, m, a, b, eps, bc)
    x = np.random.default_rng(32).standard_normal(n ** 3)
    fx = O.apply_forward(fac, x)
    assert np.linalg.norm(O.apply_inverse(fac, fx) - x) <= 1e-12 * np.linalg.norm(x)
    assert np.linalg.norm(O.apply_forward(fac, O.apply_inverse(fac, x)) - x) <= \
        1e-12 * np.linalg.norm(x)
    rel = np.linalg.norm(fx - A @ x) / np.linalg.norm(A @ x)
    assert rel <= (1e-14 if eps == 0.0 else 10 * eps), rel


def test_forward_apply_equals_explicit_product():
    """F x equals (W W^T)^{-1} x with W = W^0 ... W^L written out from the
    paper's S_I, Q_F, S_F̌ matrices."""
    n, m, eps = 8, 2, 1e-3
    N = n ** 3
    a = log_uniform_field(n, -1, 1, 33)
    b = const_field(n, 0.0)
    fac = O.build(n, m, a, b, eps)
    W = np.eye(N)
    for Wl in _explicit_W(fac, N):
        W = W @ Wl
    Fd = np.linalg.inv(W @ W.T)
    x = np.random.default_rng(34).standard_normal(N)
    ref = Fd @ x
    assert np.linalg.norm(O.apply_forward(fac, x) - ref) <= 1e-9 * np.linalg.norm(ref)
