"""CPU oracle for the hierarchical interpolative factorization.

TEST INFRASTRUCTURE ONLY.  A plain, slow FP64 implementation written from the
paper, sharing no code with the HIP path.  Only tests, the smoke check and
the benchmark's CPU-baseline leg may import anything from here.
"""
from .dense import (NotSPD, cholesky, cpqr, interp_decomp, ldl_signed, solve_lower, solve_lower_t,
                    solve_upper)
from .hif import (Factor, Geometry, active_after, apply_forward, apply_inverse, assemble, build, count_levels,
                  energy, gmres, pcg, relative_solve_error, power_norm_error)

__all__ = [
    "NotSPD", "cholesky", "cpqr", "interp_decomp", "ldl_signed", "solve_lower", "solve_lower_t", "solve_upper",
    "Factor", "Geometry", "active_after", "apply_forward", "apply_inverse", "assemble", "build", "count_levels",
    "energy", "gmres", "pcg",
    "relative_solve_error", "power_norm_error",
]
