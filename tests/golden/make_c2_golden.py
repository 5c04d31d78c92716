"""Write the stored oracle results for the 64^3 FP64 workload.

Calls only the CPU oracle (and the seeded input generators): the 64^3
high-contrast problem (log10 a ~ U(-2,2) per node, seed 201; b = 0; leaf 8^3;
eps = 1e-6; f ~ N(0,1), seed 202) is factored, and the following are written
to c2_64_fp64_eps1e-6.json beside this script:

  * per level, the rank and size of every face (face order of hif.h) and the
    number of points still active after the level, with a SHA-256 of the
    active mask (one byte per grid point, natural order);
  * |Sigma_L|;
  * e_s = ||x - F^{-1} A x|| / ||x|| for x ~ N(0,1), seed 203;
  * the oracle's PCG solve of A u = f to a true relative residual of 1e-13:
    iterations, residual, ||u||_2, max |u| and u at 2048 indices drawn
    with seed 204.

Run from the repository root: python tests/golden/make_c2_golden.py
(about four minutes on one core).
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from workloads import WORKLOADS, normal_rhs  # noqa: E402

OUT = os.path.join(HERE, "c2_64_fp64_eps1e-6.json")


def main():
    wl = WORKLOADS["c64_contrast"]
    n, leaf, eps = wl.n, wl.leaf, wl.eps
    a, b, f = wl.a(), wl.b(), wl.f()
    t0 = time.time()
    fac = O.build(n, leaf, a, b, eps)
    A = O.assemble(n, a, b)
    levels = []
    for l, lev in enumerate(fac.levels):
        act = O.active_after(fac, l).astype(np.uint8)
        levels.append({"face_ranks": [int(k) for k in lev.face_ranks],
                       "face_sizes": [int(s) for s in lev.face_sizes],
                       "active_after": int(act.sum()),
                       "active_sha256": hashlib.sha256(act.tobytes()).hexdigest()})
    x = normal_rhs(n, 203)
    es = O.relative_solve_error(fac, A, x)
    u, it, rel, ok = O.pcg(A, lambda r: O.apply_inverse(fac, r), f, 1e-13, 300)
    assert ok, "oracle PCG did not reach 1e-13"
    idx = np.sort(np.random.Generator(np.random.PCG64(204)).choice(n ** 3, 2048, replace=False))
    data = {
        "workload": "c64_contrast: 64^3, log10 a ~ U(-2,2) (seed 201), b = 0, leaf 8, "
                    "eps 1e-6, f ~ N(0,1) (seed 202)",
        "n": n, "leaf": leaf, "eps": eps,
        "levels": levels, "root_size": int(fac.root_size),
        "e_s": {"x_seed": 203, "value": es},
        "pcg": {"tol": 1e-13, "iters": int(it), "relres": rel,
                "u_norm2": float(np.linalg.norm(u)), "u_maxabs": float(np.abs(u).max()),
                "sample_seed": 204, "sample_idx": [int(i) for i in idx],
                "sample_u": [float(u[i]) for i in idx]},
        "oracle_seconds": time.time() - t0,
    }
    with open(OUT, "w") as fh:
        json.dump(data, fh, indent=0)
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
