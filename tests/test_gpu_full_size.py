"""Full-size runs, checked by properties that hold at any size.

  * 128^3 high-contrast problem (the headline case), mixed eps = 1e-4 and
    FP64 eps = 1e-6: both PCG solves reach a true relative residual of 1e-10
    (the timed tolerance), recomputed with the oracle's CPU operator; driven
    on to 1e-13, the two solutions agree to 1e-10 relative.
  * 256^3 with 32 right-hand sides (block PCG sharing each block apply): every
    column reaches 1e-10; four sampled columns are rechecked with the oracle's
    operator; the stored factor fits the 288 GB of one GPU.
"""
import numpy as np
import pytest

import oracle as O
from workloads import WORKLOADS

pytestmark = pytest.mark.gpu


def _t(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def test_headline_128_mixed_and_fp64(gpu_lib):
    import torch
    H = gpu_lib
    wm, wd = WORKLOADS["c128_mixed"], WORKLOADS["c128_fp64"]
    a, b, f = wm.a(), wm.b(), wm.f()
    ta, tb, tf = _t(a), _t(b), _t(f)
    om = H.make_options(wm.n, wm.leaf, wm.eps, H.HIF_MIXED)
    od = H.make_options(wd.n, wd.leaf, wd.eps, H.HIF_FP64)
    A = H.hif_problem_create(om, ta, tb)
    sols, tight = [], []
    for o in (om, od):
        F = H.hif_build(A, o)
        tu = torch.empty_like(tf)
        st, info = H.hif_pcg(A, F, tf, tu, tol=1e-10, maxit=100)
        torch.cuda.synchronize()
        assert st == 0 and info[0].converged and info[0].iters <= 20
        sols.append(tu.cpu().numpy())
        st, info = H.hif_pcg(A, F, tf, tu, tol=1e-13, maxit=200)
        torch.cuda.synchronize()
        assert st == 0 and info[0].converged, info[0].relres
        tight.append(tu.cpu().numpy())
        H.hif_factor_destroy(F)
    H.hif_problem_destroy(A)
    Ao = O.assemble(wm.n, a, b)
    fn = np.linalg.norm(f)
    for u in sols:
        assert np.linalg.norm(f - Ao @ u) <= 1e-10 * fn
    for u in tight:
        assert np.linalg.norm(f - Ao @ u) <= 1e-13 * fn
    assert np.linalg.norm(tight[0] - tight[1]) <= 1e-10 * np.linalg.norm(tight[1])


def test_large_256_block_pcg(gpu_lib):
    import torch
    H = gpu_lib
    H.hif_release_cached_memory()  # blocks cached for the 128^3 sizes would not fit
    wl = WORKLOADS["c256_mixed"]
    nr = wl.extra["nrhs"]
    a, b = wl.a(), wl.b()
    F0 = wl.f(nrhs=nr)
    ta, tb, tf = _t(a), _t(b), _t(F0)
    o = H.make_options(wl.n, wl.leaf, wl.eps, H.HIF_MIXED)
    A = H.hif_problem_create(o, ta, tb)
    F = H.hif_build(A, o)
    stats = H.hif_factor_stats(F).as_dict()
    assert stats["levels"] == 5 and stats["factor_bytes"] < 288e9
    tu = torch.empty_like(tf)
    st, info = H.hif_pcg(A, F, tf, tu, nrhs=nr, tol=1e-10, maxit=100)
    torch.cuda.synchronize()
    assert st == 0 and all(x.converged and x.relres <= 1e-10 for x in info)
    H.hif_factor_destroy(F)
    H.hif_problem_destroy(A)
    Ao = O.assemble(wl.n, a, b)
    for j in (0, 7, 19, 31):
        u = tu[j].cpu().numpy()
        assert np.linalg.norm(F0[j] - Ao @ u) <= 1e-10 * np.linalg.norm(F0[j]), j
