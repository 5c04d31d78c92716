"""The forward operator F x (hif_apply_forward) and factor files
(hif_factor_save / hif_factor_load), through the C ABI.

  * F x against the oracle's apply_forward (the paper's product form of F,
    Section 2.4) element by element where the skeletons coincide (FP64:
    1e-11 relative to max |F x|); F (F^{-1} x) = x; at eps = 0, F x = A x;
    ||(A - F) x|| / ||A x|| shrinks with eps.
  * A factor written to a file and read back applies bit for bit like the
    original (F^{-1}, F and the PCG solve), in both precisions and both
    boundary conditions, with the same statistics, ranks and active sets;
    a missing or foreign file gives HIF_EINVAL and no handle.
"""
import os

import numpy as np
import pytest

import oracle as O
from workloads import const_field, log_uniform_field, normal_rhs

pytestmark = pytest.mark.gpu


def _t(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def _setup(H, n, leaf, eps, prec, bc, seed):
    import torch
    a = log_uniform_field(n, -2, 2, seed)
    b = const_field(n, 0.1 * n * n if bc == "periodic" else 0.0)
    o = H.make_options(n, leaf, eps, prec,
                       bc=H.HIF_PERIODIC if bc == "periodic" else H.HIF_DIRICHLET)
    keep = (_t(a), _t(b))
    A = H.hif_problem_create(o, *keep)
    F = H.hif_build(A, o)
    torch.cuda.synchronize()
    return a, b, A, F, keep


def _fwd(H, F, x):
    import torch
    tx = _t(x)
    ty = torch.empty_like(tx)
    H.hif_apply_forward(F, tx, ty)
    torch.cuda.synchronize()
    return ty.cpu().numpy()


def _inv(H, F, x):
    import torch
    tx = _t(x)
    ty = torch.empty_like(tx)
    H.hif_apply(F, tx, ty)
    torch.cuda.synchronize()
    return ty.cpu().numpy()


@pytest.mark.parametrize("n,leaf,eps,bc", [(16, 4, 1e-6, "dirichlet"), (32, 8, 1e-4, "dirichlet"),
                                           (16, 4, 1e-3, "periodic"), (16, 4, 0.0, "dirichlet")])
def test_forward_matches_oracle(gpu_lib, n, leaf, eps, bc):
    H = gpu_lib
    a, b, A, F, keep = _setup(H, n, leaf, eps, 0, bc, 51)
    fac = O.build(n, leaf, a, b, eps, bc)
    Ao = O.assemble(n, a, b, bc)
    x = normal_rhs(n, 52)
    y, yo = _fwd(H, F, x), O.apply_forward(fac, x)
    assert np.abs(y - yo).max() <= 1e-11 * np.abs(yo).max()
    back = _inv(H, F, y)
    assert np.linalg.norm(back - x) <= 1e-10 * np.linalg.norm(x)
    rel = np.linalg.norm(y - Ao @ x) / np.linalg.norm(Ao @ x)
    assert rel <= (1e-13 if eps == 0.0 else 10 * eps), rel
    H.hif_factor_destroy(F)
    H.hif_problem_destroy(A)


def test_forward_mixed_and_in_place(gpu_lib):
    """FP32 blocks: F (F^{-1} x) = x to FP32 rounding of the factor, and the
    in-place call gives the same vector."""
    import torch
    H = gpu_lib
    n, leaf = 32, 8
    a, b, A, F, keep = _setup(H, n, leaf, 1e-4, 1, "dirichlet", 53)
    x = normal_rhs(n, 54)
    y = _fwd(H, F, x)
    assert np.linalg.norm(_inv(H, F, y) - x) <= 1e-4 * np.linalg.norm(x)
    tx = _t(x)
    H.hif_apply_forward(F, tx, tx)
    torch.cuda.synchronize()
    assert np.array_equal(tx.cpu().numpy(), y)
    H.hif_factor_destroy(F)
    H.hif_problem_destroy(A)


@pytest.mark.parametrize("prec,bc,eps", [(0, "dirichlet", 1e-5), (1, "dirichlet", 1e-4),
                                         (0, "periodic", 1e-4), (0, "dirichlet", 0.0)])
def test_save_load_round_trip(gpu_lib, tmp_path, prec, bc, eps):
    import torch
    H = gpu_lib
    n, leaf = 24, 6
    a, b, A, F, keep = _setup(H, n, leaf, eps, prec, bc, 55)
    path = str(tmp_path / "factor.hif")
    H.hif_factor_save(F, path)
    G = H.hif_factor_load(path)
    s1, s2 = H.hif_factor_stats(F).as_dict(), H.hif_factor_stats(G).as_dict()
    assert {k: v for k, v in s1.items() if k not in ("e_s", "err_norm")} == \
        {k: v for k, v in s2.items() if k not in ("e_s", "err_norm")}
    for level in range(s1["levels"]):
        r1, z1 = H.hif_factor_ranks(F, level)
        r2, z2 = H.hif_factor_ranks(G, level)
        assert np.array_equal(r1, r2) and np.array_equal(z1, z2)
        assert np.array_equal(H.hif_factor_active(F, level, n ** 3),
                              H.hif_factor_active(G, level, n ** 3))
    x = normal_rhs(n, 56)
    assert np.array_equal(_inv(H, F, x), _inv(H, G, x))
    assert np.array_equal(_fwd(H, F, x), _fwd(H, G, x))
    tf = _t(x)
    u1, u2 = torch.empty_like(tf), torch.empty_like(tf)
    st1, i1 = H.hif_pcg(A, F, tf, u1, tol=1e-10)
    st2, i2 = H.hif_pcg(A, G, tf, u2, tol=1e-10)
    torch.cuda.synchronize()
    assert st1 == st2 == 0 and i1[0].iters == i2[0].iters and torch.equal(u1, u2)
    H.hif_factor_destroy(G)
    H.hif_factor_destroy(F)
    H.hif_problem_destroy(A)


def test_load_rejects_bad_files(gpu_lib, tmp_path):
    H = gpu_lib
    for content in (None, b"", b"not a factor file at all", b"HIFFACT1\x07\x00\x00\x00"):
        path = str(tmp_path / "bad.hif")
        if os.path.exists(path):
            os.remove(path)
        if content is not None:
            with open(path, "wb") as fh:
                fh.write(content)
        with pytest.raises(H.HifError) as ei:
            H.hif_factor_load(path)
        assert ei.value.status == H.HIF_EINVAL


def test_load_rejects_truncated_file(gpu_lib, tmp_path):
    """A factor file cut short fails with HIF_EINVAL (no handle, nothing
    leaks); the intact file still loads."""
    H = gpu_lib
    n, leaf = 16, 4
    a, b, A, F, keep = _setup(H, n, leaf, 1e-4, 0, "dirichlet", 57)
    path = str(tmp_path / "f.hif")
    H.hif_factor_save(F, path)
    data = open(path, "rb").read()
    cut = str(tmp_path / "cut.hif")
    for frac in (0.1, 0.5, 0.99):
        with open(cut, "wb") as fh:
            fh.write(data[:int(len(data) * frac)])
        with pytest.raises(H.HifError) as ei:
            H.hif_factor_load(cut)
        assert ei.value.status == H.HIF_EINVAL
    G = H.hif_factor_load(path)
    H.hif_factor_destroy(G)
    H.hif_factor_destroy(F)
    H.hif_problem_destroy(A)
