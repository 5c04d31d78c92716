"""Autotuner of the batched-GEMM tile shapes, on the real workloads (GPU).

Every batched GEMM of the library runs square tiles of 32, 64 or (FP32
accumulation only) 128, picked per key: operand / accumulator types,
transposes, triangular flags and size bucket (the smallest power of two >= the
largest m or n of the batch, so fronts, faces and skeletons of similar size
share a bucket).  In tuning mode the library runs every GEMM that overwrites
its output with each candidate tile and times each run; this script drives
the factorizations and block solves the tiles are tuned for, then the library
writes the fastest tile per key (device time summed over the run) to
tiles.tsv beside itself, which every later process reads at its first GEMM.

Workloads: the 128^3 high-contrast problem (mixed eps 1e-4 and FP64 eps 1e-6,
each with a 32-vector block apply), the 48-problem batched build and the 256^3
problem (mixed eps 1e-4).

    python -m paper_1607_00346_amd.tune_tiles [--out PATH] [--skip-large]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1607_00346_amd import hif as H  # noqa: E402
from workloads import WORKLOADS, batched_workloads  # noqa: E402


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--out", default=os.path.join(HERE, "tiles.tsv"))
    p.add_argument("--skip-large", action="store_true", help="leave out the 256^3 problem")
    args = p.parse_args()
    import torch
    assert torch.cuda.is_available(), "the tuner runs on the GPU"
    dev = torch.device("cuda:0")

    def t(x):
        return torch.tensor(x, dtype=torch.float64, device=dev)

    H.hif_tune_begin()
    t0 = time.perf_counter()
    # the 128^3 problem, both precisions, with a block apply of 32 vectors
    w = WORKLOADS["c128_mixed"]
    ta, tb = t(w.a()), t(w.b())
    tf = torch.randn(32, w.n ** 3, dtype=torch.float64, device=dev)
    tu = torch.empty_like(tf)
    for prec, eps in ((H.HIF_MIXED, 1e-4), (H.HIF_FP64, 1e-6)):
        o = H.make_options(w.n, w.leaf, eps, prec)
        A = H.hif_problem_create(o, ta, tb)
        F = H.hif_build(A, o)
        H.hif_apply(F, tf, tu, nrhs=32)
        torch.cuda.synchronize()
        H.hif_factor_destroy(F)
        H.hif_problem_destroy(A)
        print(f"c128 precision {prec}: done ({time.perf_counter() - t0:.1f} s)", flush=True)
    del tf, tu, ta, tb
    # the batched workload
    wl = batched_workloads()
    opts = [H.make_options(x.n, x.leaf, x.eps, H.HIF_MIXED) for x in wl]
    keep = [(t(x.a()), t(x.b())) for x in wl]
    As = [H.hif_problem_create(o, a, b) for o, (a, b) in zip(opts, keep)]
    Fs = H.hif_build_batched(As, opts)
    torch.cuda.synchronize()
    for F in Fs:
        H.hif_factor_destroy(F)
    for A in As:
        H.hif_problem_destroy(A)
    del keep
    print(f"batched: done ({time.perf_counter() - t0:.1f} s)", flush=True)
    if not args.skip_large:
        w = WORKLOADS["c256_mixed"]
        ta, tb = t(w.a()), t(w.b())
        o = H.make_options(w.n, w.leaf, w.eps, H.HIF_MIXED)
        A = H.hif_problem_create(o, ta, tb)
        F = H.hif_build(A, o)
        torch.cuda.synchronize()
        H.hif_factor_destroy(F)
        H.hif_problem_destroy(A)
        print(f"c256: done ({time.perf_counter() - t0:.1f} s)", flush=True)
    keys = H.hif_tune_end(args.out)
    print(f"wrote {args.out} ({keys} keys)")


if __name__ == "__main__":
    main()
