"""GPU path vs the CPU oracle, through the C ABI.

Tolerances:
  * FP64 at eps = 0 the HIF is exact nested dissection, so F^{-1} f equals
    A^{-1} f up to rounding: relative error <= 1e-11 (kappa(A) u with
    kappa <= 1e5 on these grids, u = 1.1e-16).
  * Mixed precision at eps = 0: the factor is an FP32 Cholesky, error ~
    kappa(A) * u32 * growth; bound 2e-3 on the small grids used here.
  * eps > 0: skeleton sets could differ on near ties (several answers are
    correct), so every face whose rank differs from the oracle's is counted
    and at least 98% must match exactly (on these tie-free inputs all do);
    where the skeletons coincide the applies agree element by element (FP64:
    1e-11 relative to max |F^{-1} f|), and PCG solutions driven to 1e-13
    agree to 1e-10.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from workloads import const_field, log_uniform_field, normal_rhs, uniform_field

pytestmark = pytest.mark.gpu


def _t(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


class GpuHif:
    def __init__(self, H, n, leaf, eps, a, b, precision=0):
        import torch
        self.H = H
        self.n = n
        self.opts = H.make_options(n, leaf, eps, precision)
        self.ta, self.tb = _t(a), _t(b)
        self.A = H.hif_problem_create(self.opts, self.ta, self.tb)
        self.F = H.hif_build(self.A, self.opts)
        torch.cuda.synchronize()

    def apply(self, f):
        import torch
        tf = _t(f)
        tu = torch.empty_like(tf)
        self.H.hif_apply(self.F, tf, tu)
        torch.cuda.synchronize()
        return tu.cpu().numpy()

    def matvec(self, x):
        import torch
        tx = _t(x)
        ty = torch.empty_like(tx)
        self.H.hif_matvec(self.A, tx, ty)
        torch.cuda.synchronize()
        return ty.cpu().numpy()

    def pcg(self, f, tol, maxit=300):
        import torch
        tf = _t(f)
        tu = torch.empty_like(tf)
        st, info = self.H.hif_pcg(self.A, self.F, tf, tu, tol=tol, maxit=maxit)
        torch.cuda.synchronize()
        return st, info[0], tu.cpu().numpy()

    def stats(self):
        return self.H.hif_factor_stats(self.F).as_dict()

    def close(self):
        self.H.hif_factor_destroy(self.F)
        self.H.hif_problem_destroy(self.A)


@pytest.mark.parametrize("n", [5, 12])
def test_matvec_matches_oracle(gpu_lib, n):
    a = log_uniform_field(n, -2, 2, 81)
    b = uniform_field(n, 0, 1, 82)
    x = normal_rhs(n, 83)
    A = O.assemble(n, a, b)
    g = GpuHif(gpu_lib, n, n, 0.0, a, b)
    y = g.matvec(x)
    ref = A @ x
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    g.close()


@pytest.mark.parametrize("n,leaf", [(4, 4), (8, 2), (12, 3), (16, 4), (16, 8), (24, 6), (32, 8)])
def test_eps0_apply_is_exact(gpu_lib, n, leaf):
    """eps = 0: GPU F^{-1} f = A^{-1} f (sparse direct solve) and = oracle apply."""
    a = log_uniform_field(n, -2, 2, 91 + n)
    b = const_field(n, 0.0)
    f = normal_rhs(n, 92 + n)
    A = O.assemble(n, a, b)
    ref = spla.spsolve(A.tocsc(), f)
    g = GpuHif(gpu_lib, n, leaf, 0.0, a, b)
    u = g.apply(f)
    err = np.linalg.norm(u - ref) / np.linalg.norm(ref)
    assert err <= 1e-11, err
    st = g.stats()
    counts, root = O.count_levels(n, leaf)
    assert st["eliminated"][:len(counts)] == counts
    assert st["root_size"] == root
    g.close()


@pytest.mark.parametrize("n,leaf", [(16, 4), (32, 8)])
def test_eps0_mixed_precision(gpu_lib, n, leaf):
    a = log_uniform_field(n, -1, 1, 101)
    b = const_field(n, 0.0)
    f = normal_rhs(n, 102)
    A = O.assemble(n, a, b)
    ref = spla.spsolve(A.tocsc(), f)
    g = GpuHif(gpu_lib, n, leaf, 0.0, a, b, precision=1)
    u = g.apply(f)
    err = np.linalg.norm(u - ref) / np.linalg.norm(ref)
    assert err <= 2e-3, err
    st, info, u2 = g.pcg(f, 1e-10)
    assert st == 0 and info.converged and info.relres <= 1e-10
    assert np.linalg.norm(u2 - ref) / np.linalg.norm(ref) <= 1e-8
    g.close()


@pytest.mark.parametrize("n,leaf,eps", [(16, 4, 1e-6), (16, 4, 1e-3), (32, 8, 1e-6)])
def test_eps_ranks_match_oracle(gpu_lib, n, leaf, eps):
    a = log_uniform_field(n, -1, 1, 111)
    b = const_field(n, 0.0)
    fac = O.build(n, leaf, a, b, eps)
    g = GpuHif(gpu_lib, n, leaf, eps, a, b)
    total, bad = 0, 0
    for level, lev in enumerate(fac.levels):
        ranks, sizes = gpu_lib.hif_factor_ranks(g.F, level)
        assert list(sizes) == lev.face_sizes
        total += len(ranks)
        bad += int(np.sum(np.array(ranks) != np.array(lev.face_ranks)))
    assert bad <= total // 50, (bad, total)
    st = g.stats()
    assert abs(st["root_size"] - fac.root_size) <= fac.root_size // 50
    g.close()


@pytest.mark.parametrize("n,leaf,eps", [(16, 4, 1e-6), (32, 8, 1e-4)])
def test_apply_close_to_oracle(gpu_lib, n, leaf, eps):
    """eps > 0: both F^{-1} approximate A^{-1} to O(eps); with the same
    skeletons they agree element by element to rounding (1e-11 relative to
    max |F^{-1} f|), and the GPU's e_s is the oracle's."""
    a = log_uniform_field(n, -1, 1, 121)
    b = const_field(n, 0.0)
    f = normal_rhs(n, 122)
    fac = O.build(n, leaf, a, b, eps)
    g = GpuHif(gpu_lib, n, leaf, eps, a, b)
    u = g.apply(f)
    uo = O.apply_inverse(fac, f)
    d = np.abs(u - uo).max() / np.abs(uo).max()
    A = O.assemble(n, a, b)
    x = normal_rhs(n, 123)
    es_gpu = np.linalg.norm(x - g.apply(A @ x)) / np.linalg.norm(x)
    es_or = O.relative_solve_error(fac, A, x)
    assert d <= 1e-11, d
    assert abs(es_gpu - es_or) <= 1e-6 * es_or, (es_gpu, es_or)
    g.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_pcg_matches_oracle_solution(gpu_lib, prec):
    n, leaf, eps = 32, 8, 1e-4
    a = log_uniform_field(n, -2, 2, 131)
    b = const_field(n, 0.0)
    f = normal_rhs(n, 132)
    A = O.assemble(n, a, b)
    fac = O.build(n, leaf, a, b, eps)
    uo, _, rel_o, ok = O.pcg(A, lambda r: O.apply_inverse(fac, r), f, 1e-13, 300)
    assert ok
    g = GpuHif(gpu_lib, n, leaf, eps, a, b, precision=prec)
    st, info, u = g.pcg(f, 1e-13)
    assert st == 0 and info.converged
    res = np.linalg.norm(f - A @ u) / np.linalg.norm(f)
    assert res <= 1e-12
    assert np.linalg.norm(u - uo) / np.linalg.norm(uo) <= 1e-10
    g.close()


def test_indefinite_reports_not_spd(gpu_lib):
    n = 8
    a = const_field(n, 1.0)
    b = const_field(n, -1e6)   # far below -lambda_min: A is indefinite
    H = gpu_lib
    opts = H.make_options(n, 2, 0.0)
    A = H.hif_problem_create(opts, _t(a), _t(b))
    with pytest.raises(H.HifError) as ei:
        H.hif_build(A, opts)
    assert ei.value.status == H.HIF_ENOTSPD
    H.hif_problem_destroy(A)


def test_bad_coefficients_rejected(gpu_lib):
    n = 8
    H = gpu_lib
    opts = H.make_options(n, 2, 0.0)
    a = const_field(n, 1.0)
    a[17] = -1.0
    with pytest.raises(H.HifError) as ei:
        H.hif_problem_create(opts, _t(a), _t(const_field(n, 0.0)))
    assert ei.value.status == H.HIF_EINVAL
    a[17] = np.nan
    with pytest.raises(H.HifError):
        H.hif_problem_create(opts, _t(a), _t(const_field(n, 0.0)))


def test_pcg_maxit_reports_noconv(gpu_lib):
    n, leaf = 16, 4
    a = log_uniform_field(n, -2, 2, 141)
    b = const_field(n, 0.0)
    g = GpuHif(gpu_lib, n, leaf, 1e-2, a, b)
    st, info, _ = g.pcg(normal_rhs(n, 142), 1e-14, maxit=1)
    assert st == gpu_lib.HIF_ENOCONV and not info.converged and info.iters == 1
    g.close()


def test_empty_rhs_and_zero_rhs(gpu_lib):
    import torch
    n, leaf = 8, 2
    g = GpuHif(gpu_lib, n, leaf, 1e-6, const_field(n, 1.0), const_field(n, 0.0))
    tf = torch.zeros(n ** 3, dtype=torch.float64, device="cuda:0")
    tu = torch.empty_like(tf)
    gpu_lib.hif_apply(g.F, tf, tu, nrhs=0)
    st, info, u = g.pcg(np.zeros(n ** 3), 1e-10)
    assert st == 0 and info.converged and np.all(u == 0)
    g.close()


@pytest.mark.parametrize("prec,nrhs", [(0, 3), (0, 40), (1, 5)])
def test_multi_rhs_apply(gpu_lib, prec, nrhs):
    """Block apply (batched GEMM sweeps, 32 columns per pass) = one apply per
    column.  FP64 factor: the same products summed in another order (1e-12
    relative).  Mixed factor: the block path computes in FP32, the column path
    accumulates in FP64 (1e-5 relative, far below eps)."""
    import torch
    n, leaf = 16, 4
    a = log_uniform_field(n, -1, 1, 151)
    g = GpuHif(gpu_lib, n, leaf, 1e-4, a, const_field(n, 0.0), precision=prec)
    F = normal_rhs(n, 152, nrhs=nrhs)
    tf = _t(F)
    tu = torch.empty_like(tf)
    gpu_lib.hif_apply(g.F, tf, tu, nrhs=nrhs)
    torch.cuda.synchronize()
    U = tu.cpu().numpy()
    tol = 1e-12 if prec == 0 else 1e-5
    for i in range(nrhs):
        ref = g.apply(F[i])
        assert np.linalg.norm(U[i] - ref) <= tol * np.linalg.norm(ref), i
    # in place (u = f)
    gpu_lib.hif_apply(g.F, tf, tf, nrhs=nrhs)
    torch.cuda.synchronize()
    assert np.array_equal(tf.cpu().numpy(), U)
    g.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_multi_rhs_pcg(gpu_lib, prec):
    """Block PCG (one shared block apply per iteration): every column reaches a
    true residual of 1e-10 (oracle operator) and matches its single-RHS solve;
    a zero column stays zero."""
    import torch
    n, leaf, nrhs = 24, 6, 4
    a = log_uniform_field(n, -2, 2, 171)
    b = const_field(n, 0.0)
    g = GpuHif(gpu_lib, n, leaf, 1e-4, a, b, precision=prec)
    A = O.assemble(n, a, b)
    F = normal_rhs(n, 172, nrhs=nrhs)
    F[2] = 0.0
    tf = _t(F)
    tu = torch.empty_like(tf)
    st, info = gpu_lib.hif_pcg(g.A, g.F, tf, tu, nrhs=nrhs, tol=1e-10, maxit=100)
    torch.cuda.synchronize()
    U = tu.cpu().numpy()
    assert st == 0
    for i in range(nrhs):
        assert info[i].converged
        if i == 2:
            assert np.all(U[i] == 0) and info[i].iters == 0
            continue
        assert np.linalg.norm(F[i] - A @ U[i]) <= 1e-10 * np.linalg.norm(F[i])
        st1, info1, u1 = g.pcg(F[i], 1e-10)
        assert st1 == 0 and info1.converged
        assert np.linalg.norm(U[i] - u1) <= 1e-8 * np.linalg.norm(u1)
    g.close()


def test_deterministic_factor(gpu_lib):
    n, leaf = 16, 4
    a = log_uniform_field(n, -2, 2, 161)
    b = const_field(n, 0.0)
    f = normal_rhs(n, 162)
    g1 = GpuHif(gpu_lib, n, leaf, 1e-5, a, b)
    g2 = GpuHif(gpu_lib, n, leaf, 1e-5, a, b)
    assert np.array_equal(g1.apply(f), g2.apply(f))
    g1.close()
    g2.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_coarse_eps_degenerate_skeletons(gpu_lib, prec):
    """eps = 0.5: almost every face point is redundant (ranks 1-4 of up to
    49 points at level 0: skeleton blocks far narrower than the redundant
    ones).  Ranks match the oracle face by face and the weak preconditioner
    still drives PCG to 1e-10."""
    n, leaf, eps = 16, 4, 0.5
    a = log_uniform_field(n, -1, 1, 211)
    b = uniform_field(n, 0, 1, 212)
    fac = O.build(n, leaf, a, b, eps)
    g = GpuHif(gpu_lib, n, leaf, eps, a, b, precision=prec)
    total, bad = 0, 0
    for level, lev in enumerate(fac.levels):
        ranks, sizes = gpu_lib.hif_factor_ranks(g.F, level)
        r_gpu, r_orc = np.array(ranks), np.array(lev.face_ranks)
        total += len(ranks)
        bad += int(np.sum(r_gpu != r_orc))
    assert bad <= total // 50, (bad, total)
    f = normal_rhs(n, 213)
    st, info, u = g.pcg(f, 1e-10, maxit=300)
    assert st == 0 and info.converged
    A = O.assemble(n, a, b)
    assert np.linalg.norm(f - A @ u) <= 1e-10 * np.linalg.norm(f)
    g.close()


def test_fused_sweeps_exact_at_eps0(gpu_lib):
    """32^3 with 2^3 leaves: 4096 level-0 cells of 1 to 8 interior points, so
    the fused per-front sweeps run on the smallest fronts there are; at eps = 0
    the apply is a direct solve (1e-11 against a sparse solve)."""
    n, leaf = 32, 2
    a = log_uniform_field(n, -2, 2, 221)
    b = const_field(n, 0.0)
    f = normal_rhs(n, 222)
    ref = spla.spsolve(O.assemble(n, a, b).tocsc(), f)
    g = GpuHif(gpu_lib, n, leaf, 0.0, a, b)
    u = g.apply(f)
    assert np.linalg.norm(u - ref) <= 1e-11 * np.linalg.norm(ref)
    g.close()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n,leaf", [(64, 4), (128, 8)])
def test_fused_sweeps_match_general_path(gpu_lib, prec, n, leaf):
    """The fused per-front and per-face sweeps equal the gather / matrix-vector
    / scatter path up to the order of the FP64 sums (1e-12 relative).  64^3
    with 4^3 leaves: 4096 level-0 fronts of 27-64 interior points and faces
    of at most 49 points (one wave per face).  128^3 with 8^3 leaves: the
    1344 level-1 faces hold up to a few hundred points (one workgroup per
    face)."""
    a = log_uniform_field(n, -2, 2, 231)
    f = normal_rhs(n, 232)
    g = GpuHif(gpu_lib, n, leaf, 1e-4, a, const_field(n, 0.0), precision=prec)
    u0, u1 = _general_and_fused(g, f)
    assert np.linalg.norm(u1 - u0) <= 1e-12 * np.linalg.norm(u0)
    g.close()


def _general_and_fused(g, f):
    """F^{-1} f by the gather / matrix-vector / scatter sweeps, then by the
    fused ones (the library reads HIF_APPLY_FUSED at every application)."""
    import os
    old = os.environ.get("HIF_APPLY_FUSED")
    try:
        os.environ["HIF_APPLY_FUSED"] = "0"
        u0 = g.apply(f)
        os.environ["HIF_APPLY_FUSED"] = "1"
        u1 = g.apply(f)
    finally:
        if old is None:
            os.environ.pop("HIF_APPLY_FUSED", None)
        else:
            os.environ["HIF_APPLY_FUSED"] = old
    return u0, u1


@pytest.mark.parametrize("eps", [1e-2, 1e-6])
def test_fused_face_sweeps_at_other_skeleton_widths(gpu_lib, eps):
    """128^3 with 8^3 leaves, FP32 factor: at eps = 1e-2 the level-1 faces
    keep few skeleton points (narrow T and Y, a wide L_F̌^{-1}), at 1e-6 many
    (the reverse).  The level still has at least 1024 faces of more than 64
    points on average, so its skeleton step runs one workgroup per face, and
    the fused sweeps equal the general path to 1e-12."""
    n, leaf = 128, 8
    a = log_uniform_field(n, -2, 2, 241)
    g = GpuHif(gpu_lib, n, leaf, eps, a, const_field(n, 0.0), precision=1)
    st = gpu_lib.hif_factor_stats(g.F).as_dict()
    assert st["faces"][1] >= 1024 and st["face_dofs"][1] > 64 * st["faces"][1]
    ranks, sizes = gpu_lib.hif_factor_ranks(g.F, 1)
    k_med = float(np.median(np.array(ranks) / np.array(sizes)))
    assert (k_med < 0.5) if eps == 1e-2 else (k_med > 0.5), k_med
    f = normal_rhs(n, 242)
    u0, u1 = _general_and_fused(g, f)
    assert np.linalg.norm(u1 - u0) <= 1e-12 * np.linalg.norm(u0)
    g.close()
