"""Thin ctypes binding of the HIF C ABI (include/hif.h).

Argument marshalling only: every step of the factorization, apply and solve
runs in the HIP kernels of libhif.so.  Device arrays are torch CUDA tensors
(float64, contiguous); streams are torch streams.  Loading fails loudly if
the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhif.so")

HIF_OK, HIF_EINVAL, HIF_ENOMEM, HIF_ENOTSPD, HIF_ENOCONV, HIF_EDEVICE = 0, -1, -2, -3, -4, -5
HIF_FP64, HIF_MIXED = 0, 1
HIF_DIRICHLET, HIF_PERIODIC = 0, 1
HIF_MAX_LEVELS = 16

EXPORTED = [
    "hif_problem_create", "hif_build", "hif_build_batched", "hif_apply", "hif_apply_noalloc",
    "hif_apply_forward",
    "hif_matvec", "hif_pcg", "hif_gmres", "hif_pcg_batched",
    "hif_factor_stats", "hif_factor_ranks", "hif_factor_active", "hif_factor_error",
    "hif_factor_save", "hif_factor_load", "hif_factor_destroy",
    "hif_problem_destroy", "hif_status_string", "hif_last_error", "hif_profile_begin",
    "hif_profile_end", "hif_profile_select", "hif_tune_begin", "hif_tune_end", "hif_release_cached_memory",
]


class hif_options(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("leaf", ctypes.c_int32), ("eps", ctypes.c_double),
                ("precision", ctypes.c_int32), ("bc", ctypes.c_int32)]


class hif_pcg_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("relres", ctypes.c_double)]


_M = HIF_MAX_LEVELS


class hif_stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("n_dof", ctypes.c_int64), ("root_size", ctypes.c_int64),
                ("cells", ctypes.c_int64 * (_M + 1)), ("faces", ctypes.c_int64 * _M),
                ("eliminated", ctypes.c_int64 * (_M + 1)), ("face_dofs", ctypes.c_int64 * _M),
                ("redundant", ctypes.c_int64 * _M), ("max_front", ctypes.c_int64 * (_M + 1)),
                ("level_seconds", ctypes.c_double * (_M + 1)), ("factor_flops", ctypes.c_double),
                ("factor_bytes", ctypes.c_int64), ("peak_bytes", ctypes.c_int64),
                ("build_seconds", ctypes.c_double),
                ("level_flops", ctypes.c_double * (_M + 1)),
                ("level_bytes", ctypes.c_int64 * (_M + 1)),
                ("e_s", ctypes.c_double), ("err_norm", ctypes.c_double)]

    def as_dict(self) -> dict:
        L = self.levels
        return {
            "levels": L, "precision": self.precision, "n_dof": self.n_dof,
            "root_size": self.root_size,
            "cells": list(self.cells[:L + 1]), "faces": list(self.faces[:L]),
            "eliminated": list(self.eliminated[:L + 1]), "face_dofs": list(self.face_dofs[:L]),
            "redundant": list(self.redundant[:L]), "max_front": list(self.max_front[:L + 1]),
            "level_seconds": list(self.level_seconds[:L + 1]),
            "factor_flops": self.factor_flops, "factor_bytes": self.factor_bytes,
            "peak_bytes": self.peak_bytes, "build_seconds": self.build_seconds,
            "level_flops": list(self.level_flops[:L + 1]),
            "level_bytes": list(self.level_bytes[:L + 1]),
            "e_s": self.e_s, "err_norm": self.err_norm,
        }


class hif_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", ctypes.c_int64),
                ("seconds", ctypes.c_double), ("flops", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class HifError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


_lib = None


def lib():
    """The loaded libhif.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        L.hif_problem_create.argtypes = [ctypes.POINTER(hif_options), vp, vp, vp,
                                         ctypes.POINTER(vp)]
        L.hif_build.argtypes = [vp, ctypes.POINTER(hif_options), vp, ctypes.POINTER(vp)]
        L.hif_build_batched.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(hif_options), vp,
                                        ctypes.POINTER(vp)]
        L.hif_apply.argtypes = [vp, vp, vp, i32, vp]
        L.hif_apply_noalloc.argtypes = [vp, vp, vp, vp]
        L.hif_apply_forward.argtypes = [vp, vp, vp, vp]
        L.hif_matvec.argtypes = [vp, vp, vp, i32, vp]
        L.hif_pcg.argtypes = [vp, vp, vp, vp, i32, f64, i32, ctypes.POINTER(hif_pcg_info), vp]
        L.hif_gmres.argtypes = [vp, vp, vp, vp, f64, i32, i32, ctypes.POINTER(hif_pcg_info), vp]
        L.hif_pcg_batched.argtypes = [i32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      ctypes.POINTER(vp), ctypes.POINTER(vp), f64, i32,
                                      ctypes.POINTER(hif_pcg_info), vp]
        L.hif_factor_stats.argtypes = [vp, ctypes.POINTER(hif_stats)]
        L.hif_factor_ranks.argtypes = [vp, i32, vp, vp, i32, ctypes.POINTER(i32)]
        L.hif_factor_active.argtypes = [vp, i32, vp]
        L.hif_factor_save.argtypes = [vp, ctypes.c_char_p, vp]
        L.hif_factor_load.argtypes = [ctypes.c_char_p, vp, ctypes.POINTER(vp)]
        L.hif_factor_error.argtypes = [vp, vp, vp, i32, ctypes.POINTER(f64),
                                       ctypes.POINTER(f64), vp]
        L.hif_factor_destroy.argtypes = [vp]
        L.hif_problem_destroy.argtypes = [vp]
        L.hif_profile_begin.argtypes = []
        L.hif_profile_end.argtypes = [vp, i32, ctypes.POINTER(i32)]
        L.hif_profile_select.argtypes = [ctypes.c_char_p]
        L.hif_release_cached_memory.argtypes = []
        L.hif_release_cached_memory.restype = ctypes.c_int
        L.hif_tune_begin.argtypes = []
        L.hif_tune_end.argtypes = [ctypes.c_char_p, ctypes.POINTER(i32)]
        L.hif_status_string.argtypes = [i32]
        L.hif_status_string.restype = ctypes.c_char_p
        L.hif_last_error.restype = ctypes.c_char_p
        for name in ("hif_problem_create", "hif_build", "hif_build_batched", "hif_apply",
                     "hif_apply_noalloc", "hif_apply_forward", "hif_gmres",
                     "hif_matvec", "hif_pcg", "hif_pcg_batched", "hif_factor_stats",
                     "hif_factor_ranks", "hif_factor_active", "hif_factor_error",
                     "hif_factor_save", "hif_factor_load",
                     "hif_profile_begin", "hif_profile_end", "hif_profile_select",
                     "hif_tune_begin", "hif_tune_end"):
            getattr(L, name).restype = ctypes.c_int
        L.hif_factor_destroy.restype = None
        L.hif_problem_destroy.restype = None
        _lib = L
    return _lib


def _check(status: int, where: str, allow=()) -> int:
    if status != HIF_OK and status not in allow:
        raise HifError(status, where, lib().hif_last_error().decode())
    return status


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(getattr(stream, "cuda_stream", stream))


def _dptr(t):
    import torch
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous(), "need contiguous CUDA f64"
    return ctypes.c_void_p(t.data_ptr())


def make_options(n: int, leaf: int, eps: float, precision: int = HIF_FP64,
                 bc: int = HIF_DIRICHLET) -> hif_options:
    return hif_options(int(n), int(leaf), float(eps), int(precision), int(bc))


def hif_problem_create(opts: hif_options, a, b, stream=None):
    h = ctypes.c_void_p()
    _check(lib().hif_problem_create(ctypes.byref(opts), _dptr(a), _dptr(b), _stream(stream),
                                    ctypes.byref(h)), "hif_problem_create")
    return h


def hif_build(A, opts: hif_options, stream=None):
    h = ctypes.c_void_p()
    _check(lib().hif_build(A, ctypes.byref(opts), _stream(stream), ctypes.byref(h)), "hif_build")
    return h


def hif_build_batched(problems, opts, stream=None):
    """Factor several problems with joint launches per level; opts[i] describes problems[i]."""
    count = len(problems)
    assert len(opts) == count and count >= 1
    A = (ctypes.c_void_p * count)(*[p.value if isinstance(p, ctypes.c_void_p) else p
                                    for p in problems])
    O = (hif_options * count)(*opts)
    out = (ctypes.c_void_p * count)()
    _check(lib().hif_build_batched(count, A, O, _stream(stream), out), "hif_build_batched")
    return [ctypes.c_void_p(out[i]) for i in range(count)]


def hif_apply(F, f, u, nrhs: int = 1, stream=None):
    _check(lib().hif_apply(F, _dptr(f), _dptr(u), int(nrhs), _stream(stream)), "hif_apply")


def hif_apply_noalloc(F, f, u, stream=None):
    """u = F^{-1} f (one vector) with the library's static scratch: no allocation."""
    _check(lib().hif_apply_noalloc(F, _dptr(f), _dptr(u), _stream(stream)), "hif_apply_noalloc")


def hif_apply_forward(F, x, y, stream=None):
    """y = F x (one vector): the factorization itself, the product form of F."""
    _check(lib().hif_apply_forward(F, _dptr(x), _dptr(y), _stream(stream)), "hif_apply_forward")


def hif_matvec(A, x, y, nrhs: int = 1, stream=None):
    _check(lib().hif_matvec(A, _dptr(x), _dptr(y), int(nrhs), _stream(stream)), "hif_matvec")


def hif_pcg(A, F, f, u, nrhs: int = 1, tol: float = 1e-10, maxit: int = 500, stream=None):
    """Returns (status, [hif_pcg_info]); HIF_ENOCONV is reported, not raised."""
    info = (hif_pcg_info * max(nrhs, 1))()
    st = _check(lib().hif_pcg(A, F, _dptr(f), _dptr(u), int(nrhs), float(tol), int(maxit),
                              info, _stream(stream)), "hif_pcg", allow=(HIF_ENOCONV,))
    return st, [info[i] for i in range(nrhs)]


def hif_gmres(A, F, f, u, tol: float = 1e-12, restart: int = 50, maxit: int = 500, stream=None):
    """GMRES(restart) with F^{-1} as a right preconditioner; returns (status, hif_pcg_info);
    HIF_ENOCONV is reported, not raised."""
    info = hif_pcg_info()
    st = _check(lib().hif_gmres(A, F, _dptr(f), _dptr(u), float(tol), int(restart), int(maxit),
                                ctypes.byref(info), _stream(stream)), "hif_gmres",
                allow=(HIF_ENOCONV,))
    return st, info


def hif_pcg_batched(problems, factors, fs, us, tol: float = 1e-10, maxit: int = 500, stream=None):
    """One single-vector PCG per problem, run concurrently; returns (status, [hif_pcg_info])."""
    count = len(problems)
    assert len(factors) == count and len(fs) == count and len(us) == count and count >= 1
    def arr(hs):
        return (ctypes.c_void_p * count)(*[h.value if isinstance(h, ctypes.c_void_p) else h
                                           for h in hs])
    F = (ctypes.c_void_p * count)(*[_dptr(t).value for t in fs])
    U = (ctypes.c_void_p * count)(*[_dptr(t).value for t in us])
    info = (hif_pcg_info * count)()
    st = _check(lib().hif_pcg_batched(count, arr(problems), arr(factors), F, U, float(tol),
                                      int(maxit), info, _stream(stream)),
                "hif_pcg_batched", allow=(HIF_ENOCONV,))
    return st, [info[i] for i in range(count)]


def hif_factor_stats(F) -> hif_stats:
    s = hif_stats()
    _check(lib().hif_factor_stats(F, ctypes.byref(s)), "hif_factor_stats")
    return s


def hif_factor_ranks(F, level: int):
    import numpy as np
    cnt = ctypes.c_int32()
    _check(lib().hif_factor_ranks(F, int(level), None, None, 0, ctypes.byref(cnt)),
           "hif_factor_ranks")
    ranks = np.zeros(cnt.value, dtype=np.int32)
    sizes = np.zeros(cnt.value, dtype=np.int32)
    _check(lib().hif_factor_ranks(F, int(level), ranks.ctypes.data_as(ctypes.c_void_p),
                                  sizes.ctypes.data_as(ctypes.c_void_p), cnt.value,
                                  ctypes.byref(cnt)), "hif_factor_ranks")
    return ranks, sizes


def hif_factor_save(F, path: str, stream=None):
    """Write the factorization to a file."""
    _check(lib().hif_factor_save(F, os.fsencode(path), _stream(stream)), "hif_factor_save")


def hif_factor_load(path: str, stream=None):
    """A new factor read from a file written by hif_factor_save."""
    h = ctypes.c_void_p()
    _check(lib().hif_factor_load(os.fsencode(path), _stream(stream), ctypes.byref(h)),
           "hif_factor_load")
    return h


def hif_factor_active(F, level: int, n_dof: int):
    import numpy as np
    m = np.zeros(n_dof, dtype=np.uint8)
    _check(lib().hif_factor_active(F, int(level), m.ctypes.data_as(ctypes.c_void_p)),
           "hif_factor_active")
    return m


def hif_factor_error(A, F, x, power_iters: int = 0, stream=None):
    """(e_s, ||I - F^{-1}A|| estimate or nan) for the device vector x."""
    es, nrm = ctypes.c_double(), ctypes.c_double()
    _check(lib().hif_factor_error(A, F, _dptr(x), int(power_iters), ctypes.byref(es),
                                  ctypes.byref(nrm), _stream(stream)), "hif_factor_error")
    return es.value, nrm.value


def hif_profile_begin():
    _check(lib().hif_profile_begin(), "hif_profile_begin")


def hif_profile_select(classes=None):
    """Record only these kernel classes (list or comma-separated string); None: all."""
    if classes is not None and not isinstance(classes, str):
        classes = ",".join(classes)
    _check(lib().hif_profile_select(classes.encode() if classes else None), "hif_profile_select")


def hif_profile_end():
    """Stop recording; returns {kernel class: {launches, seconds, flops, bytes}}."""
    cap = 256
    buf = (hif_kernel_stat * cap)()
    cnt = ctypes.c_int32()
    _check(lib().hif_profile_end(ctypes.cast(buf, ctypes.c_void_p), cap, ctypes.byref(cnt)),
           "hif_profile_end")
    out = {}
    for i in range(min(cnt.value, cap)):
        k = buf[i]
        out[k.name.decode()] = {"launches": k.launches, "seconds": k.seconds, "flops": k.flops,
                                "bytes": k.bytes}
    return out


def hif_release_cached_memory():
    """Return the library's cached device memory to the device."""
    _check(lib().hif_release_cached_memory(), "hif_release_cached_memory")


def hif_tune_begin():
    """Tile tuning mode: every output-overwriting batched GEMM is timed with each tile."""
    _check(lib().hif_tune_begin(), "hif_tune_begin")


def hif_tune_end(path: str | None = None) -> int:
    """Pick the fastest tile per key, write the table to path (if given), use it; returns keys."""
    keys = ctypes.c_int32()
    _check(lib().hif_tune_end(path.encode() if path else None, ctypes.byref(keys)),
           "hif_tune_end")
    return keys.value


def hif_factor_destroy(F):
    lib().hif_factor_destroy(F)


def hif_problem_destroy(A):
    lib().hif_problem_destroy(A)


def hif_status_string(s: int) -> str:
    return lib().hif_status_string(int(s)).decode()


def hif_last_error() -> str:
    return lib().hif_last_error().decode()
