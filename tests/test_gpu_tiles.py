"""Tile tuning mode: every output-overwriting GEMM runs with each candidate
tile.  All tile sizes take K in the same chunk order (chunks start at
multiples of 16, masked entries are exact zeros; the Gram's own tile runs
at every candidate size), so a factor built while tuning must equal one
built normally bit for bit, and the tuner must produce a table."""
import numpy as np
import pytest

from workloads import const_field, log_uniform_field, normal_rhs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [0, 1])
def test_tuning_mode_keeps_results(gpu_lib, prec, tmp_path):
    import torch
    H = gpu_lib
    n, leaf, eps = 32, 8, 1e-4
    a = log_uniform_field(n, -2, 2, 181)
    ta = torch.tensor(a, dtype=torch.float64, device="cuda:0")
    tb = torch.tensor(const_field(n, 0.0), dtype=torch.float64, device="cuda:0")
    tf = torch.tensor(normal_rhs(n, 182), dtype=torch.float64, device="cuda:0")
    o = H.make_options(n, leaf, eps, prec)
    A = H.hif_problem_create(o, ta, tb)
    out = []
    for tuning in (False, True):
        if tuning:
            H.hif_tune_begin()
        F = H.hif_build(A, o)
        if tuning:
            path = str(tmp_path / "tiles.tsv")
            keys = H.hif_tune_end(path)
            assert keys > 0
            rows = [l.split() for l in open(path) if not l.startswith("#")]
            assert len(rows) == keys and all(r[6] in ("32", "64", "128") for r in rows)
        tu = torch.empty_like(tf)
        H.hif_apply(F, tf, tu)
        torch.cuda.synchronize()
        out.append(tu.cpu().numpy())
        H.hif_factor_destroy(F)
    H.hif_problem_destroy(A)
    assert np.array_equal(out[0], out[1])
