"""hif_apply_noalloc: the single-vector apply with every scratch vector in the
library's static device array.  It runs the same kernels in the same order
as hif_apply, so its result must equal hif_apply's bit for bit: on two calls
in a row (the second with a smaller problem, so the array holds the larger
call's leftovers), in place, and in both precisions.  A factor whose apply
needs more scratch than the array holds is refused before any launch."""
import numpy as np
import pytest

from workloads import const_field, log_uniform_field, normal_rhs

pytestmark = pytest.mark.gpu


def _t(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def _factor(H, n, leaf, eps, prec, seed):
    import torch
    a = log_uniform_field(n, -2, 2, seed)
    keep = (_t(a), _t(const_field(n, 0.0)))
    o = H.make_options(n, leaf, eps, prec)
    A = H.hif_problem_create(o, *keep)
    F = H.hif_build(A, o)
    torch.cuda.synchronize()
    return A, F, keep


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_apply_equals_apply(gpu_lib, prec):
    import torch
    H = gpu_lib
    for n, leaf, seed in ((64, 8, 301), (24, 6, 302)):  # second call: a smaller input
        A, F, keep = _factor(H, n, leaf, 1e-4, prec, seed)
        f = _t(normal_rhs(n, seed + 10))
        u_ref = torch.empty_like(f)
        u = torch.full_like(f, float("nan"))
        H.hif_apply(F, f, u_ref)
        H.hif_apply_noalloc(F, f, u)
        torch.cuda.synchronize()
        assert torch.equal(u, u_ref), (n, prec)
        g = f.clone()
        H.hif_apply_noalloc(F, g, g)  # in place
        torch.cuda.synchronize()
        assert torch.equal(g, u_ref), (n, prec)
        H.hif_factor_destroy(F)
        H.hif_problem_destroy(A)


def test_noalloc_rejects_too_large(gpu_lib):
    """160^3 with 5^3 leaves: the level-0 sweeps alone need about 84 MiB of
    scratch, more than the 64 MiB array; the call fails with HIF_EINVAL and
    leaves u untouched."""
    import torch
    H = gpu_lib
    n, leaf = 160, 5
    A, F, keep = _factor(H, n, leaf, 1e-2, 1, 303)
    f = _t(normal_rhs(n, 304))
    u = torch.zeros_like(f)
    with pytest.raises(H.HifError) as ei:
        H.hif_apply_noalloc(F, f, u)
    assert ei.value.status == H.HIF_EINVAL and "MiB" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((u == 0).all())
    H.hif_factor_destroy(F)
    H.hif_problem_destroy(A)
