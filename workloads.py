"""Seeded synthetic inputs for the variable-coefficient 7-point problem.

This module only draws random numbers: coefficient fields a(x), b(x) and
right-hand sides f, each in natural grid order (flat index x1 + n*x2 + n^2*x3,
x1 fastest).  It holds none of the factorization's arithmetic, so both the
CPU oracle and the GPU path can consume the same arrays.

The paper's experiments use formula-defined coefficient fields, not a dataset
(Section 4, Examples 1-3); the workloads below are the synthetic stand-ins
the measurements are quoted on.  Every draw uses numpy's PCG64 generator with
an explicit seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def _gen(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def log_uniform_field(n: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """a_j = 10**U(lo, hi), one independent draw per grid node (x1 fastest)."""
    return 10.0 ** _gen(seed).uniform(lo, hi, n ** 3)


def uniform_field(n: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """b_j = U(lo, hi) per grid node."""
    return _gen(seed).uniform(lo, hi, n ** 3)


def const_field(n: int, value: float) -> np.ndarray:
    return np.full(n ** 3, float(value))


def normal_rhs(n: int, seed: int, nrhs: int = 1) -> np.ndarray:
    """f ~ i.i.d. N(0,1); shape (N,) for one RHS, else (nrhs, N) row per RHS
    (each row is one column of the column-major N x nrhs block)."""
    g = _gen(seed)
    if nrhs == 1:
        return g.standard_normal(n ** 3)
    return g.standard_normal((nrhs, n ** 3))


def smoothed_binary_field(n: int, seed: int, lo: float = 0.1, hi: float = 1000.0,
                          sigma: float = 1.0) -> np.ndarray:
    """The high-contrast random field of the paper's Example 2 (Section 4): a
    uniform value in [0, 1) per grid point (x1 fastest), convolved
    periodically with an isotropic Gaussian of standard deviation `sigma` grid
    spacings (kernel normalised to sum 1, applied by FFT), then `lo` where
    the result is <= 0.5 and `hi` where it is above."""
    u = _gen(seed).uniform(0.0, 1.0, n ** 3).reshape(n, n, n)
    d = np.minimum(np.arange(n), n - np.arange(n)).astype(np.float64)  # periodic distance
    g1 = np.exp(-0.5 * (d / sigma) ** 2)
    ker = g1[:, None, None] * g1[None, :, None] * g1[None, None, :]
    ker /= ker.sum()
    sm = np.real(np.fft.ifftn(np.fft.fftn(u) * np.fft.fftn(ker)))
    return np.where(sm <= 0.5, lo, hi).ravel()


def checkerboard_field(n: int, block: int = 7, even: float = 1000.0,
                       odd: float = 0.1) -> np.ndarray:
    """The field of the paper's Example 3 (Section 4): `even` where
    floor(j1/block) + floor(j2/block) + floor(j3/block) is even (grid point
    j = (j1, j2, j3), x_i = j_i / n), `odd` elsewhere; x1 fastest."""
    j = np.arange(n) // block
    par = (j[:, None, None] + j[None, :, None] + j[None, None, :]) % 2
    return np.where(par == 0, even, odd).ravel()


@dataclass
class Workload:
    """One synthetic problem: grid n^3, leaf width m, coefficient recipe, ID tolerance."""
    name: str
    n: int
    leaf: int
    eps: float
    a_kind: str            # "const" | "logu" | "smooth01" | "checker"
    a_args: tuple
    b_kind: str            # "const" | "unif"
    b_args: tuple
    f_seed: int
    precision: str = "fp64"  # "fp64" | "mixed"
    extra: dict = field(default_factory=dict)
    bc: str = "dirichlet"    # "dirichlet" | "periodic"

    def a(self) -> np.ndarray:
        if self.a_kind == "const":
            return const_field(self.n, *self.a_args)
        if self.a_kind == "smooth01":
            return smoothed_binary_field(self.n, *self.a_args)
        if self.a_kind == "checker":
            return checkerboard_field(self.n, *self.a_args)
        return log_uniform_field(self.n, *self.a_args)

    def b(self) -> np.ndarray:
        if self.b_kind == "const":
            return const_field(self.n, *self.b_args)
        return uniform_field(self.n, *self.b_args)

    def f(self, nrhs: int = 1) -> np.ndarray:
        return normal_rhs(self.n, self.f_seed, nrhs)


# Named workloads.  "logu" args are (lo, hi, seed) of log10 a ~ U(lo, hi).
WORKLOADS = {
    # 16^3, a = 1, b = 0, leaf 4^3, eps 1e-6: the small case the oracle runs in seconds.
    "c16_const": Workload("c16_const", 16, 4, 1e-6, "const", (1.0,), "const", (0.0,), 101),
    # 64^3 high-contrast field, FP64, leaf 8^3, eps 1e-6.
    "c64_contrast": Workload("c64_contrast", 64, 8, 1e-6, "logu", (-2.0, 2.0, 201),
                             "const", (0.0,), 202),
    # 128^3 high-contrast field: the headline problem, mixed eps 1e-4 and FP64 eps 1e-6.
    "c128_mixed": Workload("c128_mixed", 128, 8, 1e-4, "logu", (-2.0, 2.0, 301),
                           "const", (0.0,), 302, precision="mixed"),
    "c128_fp64": Workload("c128_fp64", 128, 8, 1e-6, "logu", (-2.0, 2.0, 301),
                          "const", (0.0,), 302, precision="fp64"),
    # 256^3 high-contrast field, FP32 factor at eps 1e-4, 32 right-hand sides.
    "c256_mixed": Workload("c256_mixed", 256, 8, 1e-4, "logu", (-2.0, 2.0, 701),
                           "const", (0.0,), 702, precision="mixed", extra={"nrhs": 32}),
    # 32^3 high-contrast field used for mid-size parity and the CPU baseline sample.
    "c32_contrast": Workload("c32_contrast", 32, 8, 1e-6, "logu", (-2.0, 2.0, 211),
                             "const", (0.0,), 212),
    # The paper's three examples (Section 4): periodic on [0,1)^3, leaf 4^3 (blocks of
    # at most 64 points), b = 0.1 relative to the stencil taken without its 1/h^2
    # factor, i.e. b = 0.1 n^2 beside the 1/h^2 = n^2 stencil assembled here (the
    # reading under which the paper's 32^3 Example 1 figures are reproduced:
    # |Sigma_L| = 3440 and 6 GMRES steps).  Example 1: a = 1, eps 1e-3.
    "ex1_32": Workload("ex1_32", 32, 4, 1e-3, "const", (1.0,), "const", (0.1 * 32 ** 2,), 801,
                       bc="periodic"),
    # Example 2: smoothed, quantized random field a in {0.1, 1000}, eps 1e-5.
    "ex2_32": Workload("ex2_32", 32, 4, 1e-5, "smooth01", (802,), "const", (0.1 * 32 ** 2,),
                       803, bc="periodic"),
    # Example 3: checkerboard of 7-point blocks, a in {1000, 0.1}, eps 1e-4.
    "ex3_64": Workload("ex3_64", 64, 4, 1e-4, "checker", (7,), "const", (0.1 * 64 ** 2,), 804,
                       bc="periodic"),
    "ex1_128": Workload("ex1_128", 128, 4, 1e-3, "const", (1.0,), "const", (0.1 * 128 ** 2,),
                        805, bc="periodic"),
    "ex2_128": Workload("ex2_128", 128, 4, 1e-5, "smooth01", (806,), "const",
                        (0.1 * 128 ** 2,), 807, bc="periodic"),
    "ex3_128": Workload("ex3_128", 128, 4, 1e-4, "checker", (7,), "const", (0.1 * 128 ** 2,),
                        808, bc="periodic"),
}


def batched_leaf(n: int) -> int:
    """Leaf width for a batched problem: the largest m <= 8 with n / m a power of two."""
    for m in range(8, 1, -1):
        q, r = divmod(n, m)
        if r == 0 and q >= 1 and (q & (q - 1)) == 0:
            return m
    raise ValueError(f"no leaf width <= 8 divides {n} into a power of two")


def batched_workloads(count: int = 48, seed: int = 400,
                      sizes: tuple = (32, 48, 64, 96), eps: float = 1e-4) -> list:
    """Independent problems of a batched build: grid n drawn uniformly from `sizes`
    (seed `seed`), problem i with log10 a ~ U(-1, 1) (seed 1000 + i), b ~ U(0, 1)
    (seed 2000 + i) and f ~ N(0, 1) (seed 3000 + i); FP32 factor at `eps`."""
    ns = _gen(seed).choice(np.asarray(sizes), size=count)
    return [Workload(f"batch{i}_n{int(n)}", int(n), batched_leaf(int(n)), eps, "logu",
                     (-1.0, 1.0, 1000 + i), "unif", (0.0, 1.0, 2000 + i), 3000 + i,
                     precision="mixed")
            for i, n in enumerate(ns)]
