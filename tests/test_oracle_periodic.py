"""Pins of the oracle's periodic variant (the paper's setting, Section 2.1:
[0,1)^3, h = 1/n, indices wrap around) and of its root LDL^T."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import oracle as O
from workloads import WORKLOADS, const_field, log_uniform_field, normal_rhs, uniform_field


def test_periodic_assembly_fourier_eigenpairs():
    """a = 1, b = beta: v = prod_d cos(2 pi k_d j_d / n) is an eigenvector with
    lambda = beta + (4/h^2) sum_d sin^2(pi k_d / n), h = 1/n; A is exactly
    symmetric."""
    n, beta = 6, 0.3
    A = O.assemble(n, const_field(n, 1.0), const_field(n, beta), "periodic")
    assert abs(A - A.T).max() == 0.0
    h = 1.0 / n
    j = np.arange(n)
    for k in [(0, 0, 0), (1, 2, 3), (3, 1, 0)]:
        c = [np.cos(2 * np.pi * kd * j / n) for kd in k]
        v = np.einsum("k,j,i->kji", c[2], c[1], c[0]).ravel()
        lam = beta + 4.0 / h ** 2 * sum(np.sin(np.pi * kd / n) ** 2 for kd in k)
        assert np.linalg.norm(A @ v - lam * v) <= 1e-12 * (4 / h ** 2) * np.linalg.norm(v)


def test_periodic_row_sums_are_b():
    """Every row of the periodic operator sums to b_j (A 1 = b): the wrapped
    couplings are present with the same harmonic-mean weights."""
    n = 5
    a = log_uniform_field(n, -2, 2, 3)
    b = uniform_field(n, 0, 1, 4)
    A = O.assemble(n, a, b, "periodic")
    assert np.allclose(A @ np.ones(n ** 3), b, rtol=0, atol=1e-9 * np.abs(A).max())
    assert A.nnz == 7 * n ** 3


@pytest.mark.parametrize("n,m", [(8, 2), (12, 3), (16, 4), (32, 8)])
def test_periodic_counts_and_face_sizes_closed_form(n, m):
    """Every plane x_d = w j (j >= 0) is a separator: (n - n/w)^3 points are
    interior at or before level l, the root keeps n^3 - (n-2)^3, and level l
    has 3 nc^3 faces of (w-1)^2 points each (nc = n / w)."""
    counts, root = O.count_levels(n, m, "periodic")
    L = len(counts)
    cum = [(n - n // (m << l)) ** 3 for l in range(L)]
    assert counts == [cum[0]] + [cum[l] - cum[l - 1] for l in range(1, L)]
    assert root == n ** 3 - (n - 2) ** 3
    fac = O.build(n, m, log_uniform_field(n, -1, 1, 5), const_field(n, 1.0), 0.0, "periodic")
    for level, lev in enumerate(fac.levels):
        w = m << level
        nc = n // w
        assert lev.face_sizes == [(w - 1) ** 2] * (3 * nc ** 3)


@pytest.mark.parametrize("n,m", [(8, 2), (12, 3), (16, 4), (8, 4)])
def test_periodic_eps0_is_exact_solve(n, m):
    a = log_uniform_field(n, -2, 2, 21)
    b = uniform_field(n, 0.5, 1, 22)
    A = O.assemble(n, a, b, "periodic")
    fac = O.build(n, m, a, b, 0.0, "periodic")
    f = np.random.default_rng(23).standard_normal(n ** 3)
    x = O.apply_inverse(fac, f)
    xd = spla.spsolve(A.tocsc(), f)
    assert np.linalg.norm(x - xd) <= 1e-11 * np.linalg.norm(xd)


def test_ldl_signed_reconstructs_and_keeps_inertia():
    """L S L^T = A for a symmetric indefinite A with nonzero leading minors;
    the number of negative signs is the number of negative eigenvalues
    (Sylvester's law of inertia); on an SPD matrix it is LAPACK's Cholesky."""
    g = np.random.default_rng(7)
    Q = np.linalg.qr(g.standard_normal((30, 30)))[0]
    ev = np.concatenate([-np.linspace(1, 3, 4), np.linspace(0.5, 9, 26)])
    A = (Q * ev) @ Q.T
    L, S = O.ldl_signed(A)
    assert np.allclose(np.tril(L), L) and np.all(np.diag(L) > 0)
    assert np.abs((L * S) @ L.T - A).max() <= 1e-12 * np.abs(A).max()
    assert int(np.sum(S < 0)) == 4 == int(np.sum(np.linalg.eigvalsh(A) < 0))
    B = g.standard_normal((12, 12))
    B = B @ B.T + 12 * np.eye(12)
    L2, S2 = O.ldl_signed(B)
    assert np.all(S2 == 1.0)
    assert np.allclose(L2, sla.cholesky(B, lower=True), rtol=1e-13, atol=1e-13)


def test_periodic_indefinite_root_keeps_ldl():
    """With b = 0.1 on the 1/h^2 stencil the constant mode's eigenvalue (0.1)
    is far below the compression error: at 32^3, leaf 8, eps = 1e-3 the
    compressed root is indefinite (Cholesky fails on it, the LDL^T keeps at
    least one negative sign), and GMRES with the LDL^T-rooted F^{-1} still
    reaches 1e-12."""
    n, m = 32, 8
    a, b = const_field(n, 1.0), const_field(n, 0.1)
    A = O.assemble(n, a, b, "periodic")
    fac = O.build(n, m, a, b, 1e-3, "periodic")
    assert int(np.sum(fac.Sroot < 0)) >= 1
    Lm = fac.Lroot * fac.Sroot
    with pytest.raises(O.NotSPD):
        O.cholesky(Lm @ fac.Lroot.T)
    f = normal_rhs(n, 24)
    u, its, rel, ok = O.gmres(A, lambda r: O.apply_inverse(fac, r), f, 1e-12, 50, 200)
    assert ok and rel <= 1e-12
    assert np.linalg.norm(f - A @ u) <= 1e-12 * np.linalg.norm(f)


def test_paper_example1_32():
    """The paper's Example 1 at 32^3 (Section 4, first row of its Table for
    Example 1: periodic, a = 1, b = 0.1 on the unscaled stencil, leaf 4^3,
    eps = 1e-3): |Sigma_L| = 3440 and 6 GMRES steps to 1e-12, as printed; e_s
    (the paper prints 3.8e-4 to 7.3e-4 over its process counts) within 3x of
    4.84e-4."""
    wl = WORKLOADS["ex1_32"]
    a, b, f = wl.a(), wl.b(), wl.f()
    fac = O.build(wl.n, wl.leaf, a, b, wl.eps, wl.bc)
    assert fac.root_size == 3440
    A = O.assemble(wl.n, a, b, wl.bc)
    es = O.relative_solve_error(fac, A, normal_rhs(wl.n, 9))
    assert 4.84e-4 / 3 <= es <= 4.84e-4 * 3, es
    _, its, rel, ok = O.gmres(A, lambda r: O.apply_inverse(fac, r), f, 1e-12, 50, 100)
    assert ok and its == 6


@pytest.mark.parametrize("n,m", [(8, 8), (16, 4)])
def test_periodic_negative_b_exact_with_ldl_root(n, m):
    """b = -10: the periodic operator has one negative eigenvalue (the
    constant mode's), the cell interiors stay definite, and at eps = 0 the
    LDL^T root (one negative sign, by Sylvester's law) gives A^{-1} exactly."""
    a, b = log_uniform_field(n, -1, 1, 5), const_field(n, -10.0)
    A = O.assemble(n, a, b, "periodic")
    assert int(np.sum(np.linalg.eigvalsh(A.toarray()) < 0)) == 1
    fac = O.build(n, m, a, b, 0.0, "periodic")
    assert int(np.sum(fac.Sroot < 0)) == 1
    f = normal_rhs(n, 64)
    x = O.apply_inverse(fac, f)
    xd = spla.spsolve(A.tocsc(), f)
    assert np.linalg.norm(x - xd) <= 1e-11 * np.linalg.norm(xd)
    assert np.linalg.norm(O.apply_forward(fac, x) - f) <= 1e-11 * np.linalg.norm(f)
