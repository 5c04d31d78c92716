"""Batched multi-problem build (hif_build_batched) through the C ABI.

  * A batch of equally sized problems runs the same kernels with the same
    per-front arithmetic as single builds, so its factors must reproduce the
    single builds bit for bit.
  * A batch of mixed sizes and leaf widths at eps = 0 is exact nested
    dissection for every problem: F^{-1} f = A^{-1} f (sparse direct solve)
    to 1e-11 relative (FP64), and the eliminated counts per level are the
    oracle planner's.
  * At eps > 0 the ranks of a mixed batch are compared with the oracle face
    by face (every differing face counted; at least 98% must match), and PCG reaches a
    true residual of 1e-10 measured with the oracle's operator.
  * The full batched workload (48 problems of 32^3..96^3, FP32 factor at
    eps = 1e-4) is checked by properties that hold at any size: every PCG
    solve reaches a true relative residual of 1e-10.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from workloads import batched_workloads, const_field, log_uniform_field, normal_rhs

pytestmark = pytest.mark.gpu


def _t(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


class Batch:
    """Problems created one by one, factored together."""

    def __init__(self, H, specs, eps, precision):
        import torch
        self.H = H
        self.specs = specs  # (n, leaf, a, b)
        self.opts = [H.make_options(n, leaf, eps, precision) for n, leaf, _, _ in specs]
        self.keep = [(_t(a), _t(b)) for _, _, a, b in specs]
        self.A = [H.hif_problem_create(o, ta, tb) for o, (ta, tb) in zip(self.opts, self.keep)]
        self.F = H.hif_build_batched(self.A, self.opts)
        torch.cuda.synchronize()

    def apply(self, i, f):
        import torch
        tf = _t(f)
        tu = torch.empty_like(tf)
        self.H.hif_apply(self.F[i], tf, tu)
        torch.cuda.synchronize()
        return tu.cpu().numpy()

    def pcg(self, i, f, tol):
        import torch
        tf = _t(f)
        tu = torch.empty_like(tf)
        st, info = self.H.hif_pcg(self.A[i], self.F[i], tf, tu, tol=tol, maxit=300)
        torch.cuda.synchronize()
        return st, info[0], tu.cpu().numpy()

    def close(self):
        for F in self.F:
            self.H.hif_factor_destroy(F)
        for A in self.A:
            self.H.hif_problem_destroy(A)


def _single_apply(H, n, leaf, eps, prec, a, b, f):
    import torch
    opts = H.make_options(n, leaf, eps, prec)
    ta, tb = _t(a), _t(b)
    A = H.hif_problem_create(opts, ta, tb)
    F = H.hif_build(A, opts)
    tf = _t(f)
    tu = torch.empty_like(tf)
    H.hif_apply(F, tf, tu)
    torch.cuda.synchronize()
    ranks = [list(H.hif_factor_ranks(F, l)[0]) for l in range(H.hif_factor_stats(F).levels)]
    H.hif_factor_destroy(F)
    H.hif_problem_destroy(A)
    return tu.cpu().numpy(), ranks


@pytest.mark.parametrize("prec", [0, 1])
def test_equal_sizes_reproduce_single_builds(gpu_lib, prec):
    H = gpu_lib
    n, leaf, eps = 16, 4, 1e-5
    specs = [(n, leaf, log_uniform_field(n, -2, 2, 500 + i), const_field(n, 0.0))
             for i in range(3)]
    bt = Batch(H, specs, eps, prec)
    for i, (_, _, a, b) in enumerate(specs):
        f = normal_rhs(n, 510 + i)
        u_single, r_single = _single_apply(H, n, leaf, eps, prec, a, b, f)
        r_batch = [list(H.hif_factor_ranks(bt.F[i], l)[0]) for l in range(len(r_single))]
        assert r_batch == r_single
        assert np.array_equal(bt.apply(i, f), u_single)
    bt.close()


def test_mixed_sizes_eps0_exact(gpu_lib):
    H = gpu_lib
    grid = [(8, 2), (12, 3), (16, 4), (24, 6), (32, 8), (16, 8), (8, 4)]
    specs = [(n, leaf, log_uniform_field(n, -2, 2, 520 + k), const_field(n, 0.0))
             for k, (n, leaf) in enumerate(grid)]
    bt = Batch(H, specs, 0.0, 0)
    for i, (n, leaf, a, b) in enumerate(specs):
        f = normal_rhs(n, 540 + i)
        ref = spla.spsolve(O.assemble(n, a, b).tocsc(), f)
        u = bt.apply(i, f)
        assert np.linalg.norm(u - ref) / np.linalg.norm(ref) <= 1e-11
        st = H.hif_factor_stats(bt.F[i]).as_dict()
        counts, root = O.count_levels(n, leaf)
        assert st["eliminated"][:len(counts)] == counts
        assert st["root_size"] == root
    bt.close()


def test_same_problem_twice(gpu_lib):
    """One handle listed twice shares its cached level-0 plan; both factors are whole."""
    import torch
    H = gpu_lib
    n, leaf = 16, 4
    a = log_uniform_field(n, -1, 1, 560)
    b = const_field(n, 0.0)
    opts = H.make_options(n, leaf, 0.0)
    ta, tb = _t(a), _t(b)
    A = H.hif_problem_create(opts, ta, tb)
    F = H.hif_build_batched([A, A], [opts, opts])
    f = normal_rhs(n, 561)
    ref = spla.spsolve(O.assemble(n, a, b).tocsc(), f)
    for Fi in F:
        tf = _t(f)
        tu = torch.empty_like(tf)
        H.hif_apply(Fi, tf, tu)
        torch.cuda.synchronize()
        u = tu.cpu().numpy()
        assert np.linalg.norm(u - ref) / np.linalg.norm(ref) <= 1e-11
        H.hif_factor_destroy(Fi)
    H.hif_problem_destroy(A)


@pytest.mark.parametrize("prec", [0, 1])
def test_mixed_sizes_eps_ranks_and_pcg(gpu_lib, prec):
    H = gpu_lib
    eps = 1e-4
    grid = [(16, 4), (24, 6), (32, 8), (12, 3)]
    specs = [(n, leaf, log_uniform_field(n, -1, 1, 580 + k), const_field(n, 0.0))
             for k, (n, leaf) in enumerate(grid)]
    bt = Batch(H, specs, eps, prec)
    total, bad = 0, 0
    for i, (n, leaf, a, b) in enumerate(specs):
        fac = O.build(n, leaf, a, b, eps)
        for level, lev in enumerate(fac.levels):
            ranks, sizes = H.hif_factor_ranks(bt.F[i], level)
            assert list(sizes) == lev.face_sizes
            total += len(ranks)
            bad += int(np.sum(np.array(ranks) != np.array(lev.face_ranks)))
        A = O.assemble(n, a, b)
        f = normal_rhs(n, 600 + i)
        st, info, u = bt.pcg(i, f, 1e-10)
        assert st == 0 and info.converged
        assert np.linalg.norm(f - A @ u) / np.linalg.norm(f) <= 1e-10
    assert bad <= total // 50, (bad, total)
    bt.close()


def test_batch_reports_failing_problem(gpu_lib):
    """A non-SPD member fails the whole batch with ENOTSPD naming it; no handle escapes."""
    H = gpu_lib
    n, leaf = 8, 2
    good = (n, leaf, const_field(n, 1.0), const_field(n, 0.0))
    bad = (n, leaf, const_field(n, 1.0), const_field(n, -1e6))
    opts = [H.make_options(n, leaf, 0.0) for _ in range(3)]
    keep = [(_t(a), _t(b)) for _, _, a, b in (good, bad, good)]
    A = [H.hif_problem_create(o, ta, tb) for o, (ta, tb) in zip(opts, keep)]
    with pytest.raises(H.HifError) as ei:
        H.hif_build_batched(A, opts)
    assert ei.value.status == H.HIF_ENOTSPD
    assert "problem 1" in str(ei.value)
    mixed = [H.make_options(n, leaf, 0.0), H.make_options(n, leaf, 1e-3),
             H.make_options(n, leaf, 0.0)]
    with pytest.raises(H.HifError) as ei:
        H.hif_build_batched(A, mixed)
    assert ei.value.status == H.HIF_EINVAL
    for a in A:
        H.hif_problem_destroy(a)


def test_full_batched_workload(gpu_lib):
    """48 problems (32^3..96^3, 12.1M DOFs), FP32 factor at eps 1e-4: every PCG
    solve reaches a true relative residual of 1e-10; the residual is recomputed
    with the oracle's operator for the first problem of each size."""
    import torch
    H = gpu_lib
    wl = batched_workloads()
    opts = [H.make_options(w.n, w.leaf, w.eps, H.HIF_MIXED) for w in wl]
    keep = [(_t(w.a()), _t(w.b())) for w in wl]
    A = [H.hif_problem_create(o, ta, tb) for o, (ta, tb) in zip(opts, keep)]
    F = H.hif_build_batched(A, opts)
    checked = set()
    for i, w in enumerate(wl):
        f = w.f()
        tf = _t(f)
        tu = torch.empty_like(tf)
        st, info = H.hif_pcg(A[i], F[i], tf, tu, tol=1e-10, maxit=100)
        torch.cuda.synchronize()
        assert st == 0 and info[0].converged and info[0].relres <= 1e-10, (i, w.n)
        if w.n not in checked:
            checked.add(w.n)
            u = tu.cpu().numpy()
            Ao = O.assemble(w.n, w.a(), w.b())
            assert np.linalg.norm(f - Ao @ u) / np.linalg.norm(f) <= 1e-10, (i, w.n)
    for Fi in F:
        H.hif_factor_destroy(Fi)
    for a in A:
        H.hif_problem_destroy(a)


def test_batched_pcg_equals_single_solves(gpu_lib):
    """hif_pcg_batched runs one PCG per problem on concurrent streams: every
    solve does the same kernels in the same order as hif_pcg, so the solutions,
    iteration counts and residuals are identical bit for bit."""
    import torch
    H = gpu_lib
    grid = [(16, 4), (24, 6), (32, 8), (12, 3), (16, 8), (24, 3), (8, 2)]
    specs = [(n, leaf, log_uniform_field(n, -1, 1, 620 + k), const_field(n, 0.0))
             for k, (n, leaf) in enumerate(grid)]
    bt = Batch(H, specs, 1e-4, 1)
    fs = [_t(normal_rhs(n, 640 + i)) for i, (n, _, _, _) in enumerate(specs)]
    us = [torch.empty_like(f) for f in fs]
    st, info = H.hif_pcg_batched(bt.A, bt.F, fs, us, tol=1e-10, maxit=100)
    torch.cuda.synchronize()
    assert st == 0
    for i in range(len(specs)):
        u1 = torch.empty_like(fs[i])
        st1, info1 = H.hif_pcg(bt.A[i], bt.F[i], fs[i], u1, tol=1e-10, maxit=100)
        torch.cuda.synchronize()
        assert st1 == 0 and info1[0].iters == info[i].iters and info1[0].relres == info[i].relres
        assert torch.equal(u1, us[i])
    # a factor listed twice would share its scratch between two solves in flight
    with pytest.raises(H.HifError) as ei:
        H.hif_pcg_batched([bt.A[0], bt.A[0]], [bt.F[0], bt.F[0]], [fs[0], fs[0]],
                          [us[0], torch.empty_like(us[0])])
    assert ei.value.status == H.HIF_EINVAL
    # maxit = 1: every solve stops early and the call reports it
    st, info = H.hif_pcg_batched(bt.A, bt.F, fs, us, tol=1e-14, maxit=1)
    assert st == H.HIF_ENOCONV and all(x.iters == 1 and not x.converged for x in info)
    bt.close()
