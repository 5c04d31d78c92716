"""From the second single-vector PCG solve with a factor on, the
preconditioner application is replayed from a HIP graph (captured once per
factor, replayed every iteration with the solver's own kernels and host
synchronizations in between, and again by later solves).  The replays run the
same kernels in the same order as direct launches, so the iterates must be
identical bit for bit to the first solve (direct launches) and to one with
graphs switched off (HIF_APPLY_GRAPH=0)."""
import os

import numpy as np
import pytest

from workloads import const_field, log_uniform_field, normal_rhs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,nrhs", [(0, 1), (1, 1)])
def test_graph_replay_equals_direct(gpu_lib, prec, nrhs):
    import torch
    H = gpu_lib
    n, leaf = 24, 6
    a = log_uniform_field(n, -2, 2, 201)
    o = H.make_options(n, leaf, 1e-4, prec)
    ta = torch.tensor(a, dtype=torch.float64, device="cuda:0")
    tb = torch.tensor(const_field(n, 0.0), dtype=torch.float64, device="cuda:0")
    A = H.hif_problem_create(o, ta, tb)
    F = H.hif_build(A, o)
    tf = torch.tensor(normal_rhs(n, 202, nrhs=nrhs), dtype=torch.float64, device="cuda:0")
    res = []
    old = os.environ.get("HIF_APPLY_GRAPH")
    try:
        for flag in ("1", "0", "1", "1"):
            os.environ["HIF_APPLY_GRAPH"] = flag
            tu = torch.empty_like(tf)
            st, info = H.hif_pcg(A, F, tf, tu, nrhs=nrhs, tol=1e-12, maxit=100)
            torch.cuda.synchronize()
            assert st == 0
            res.append((tu.cpu().numpy(), [i.iters for i in info], [i.relres for i in info]))
    finally:
        if old is None:
            os.environ.pop("HIF_APPLY_GRAPH", None)
        else:
            os.environ["HIF_APPLY_GRAPH"] = old
    for u, its, rel in res[1:]:
        assert np.array_equal(u, res[0][0]) and its == res[0][1] and rel == res[0][2]
    assert max(res[0][1]) >= 3  # several replays per solve
    H.hif_factor_destroy(F)
    H.hif_problem_destroy(A)
