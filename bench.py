"""Benchmark: HIF factor + PCG solve throughput (DOF/s) on one MI355X.

One step = hif_build of the 128^3 high-contrast problem (log10 a ~ U(-2,2)
per node, b = 0, leaf 8^3) followed by hif_pcg to a true relative residual of
1e-10.  `value` is the mixed-precision run (FP32 fronts, eps = 1e-4, FP64
PCG); the plain FP64 GPU HIF (eps = 1e-6) is timed beside it.  Inputs are
synthetic and already resident in HBM when timing starts.

Prints ONE JSON line (rank 0).  Only one GPU is supported: --gpus > 1 exits.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from workloads import WORKLOADS  # noqa: E402

PEAK = {"fp64_tflops": 78.6, "fp32_tflops": 157.3, "hbm_gbs": 8000.0}


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def run_gpu(args):
    import torch
    from paper_1607_00346_amd import hif as H

    wl_m = WORKLOADS[args.workload + "_mixed"]
    wl_d = WORKLOADS[args.workload + "_fp64"]
    n, leaf = wl_m.n, wl_m.leaf
    N = n ** 3
    dev = torch.device("cuda:0")
    a, b, f = wl_m.a(), wl_m.b(), wl_m.f()
    ta = torch.tensor(a, dtype=torch.float64, device=dev)
    tb = torch.tensor(b, dtype=torch.float64, device=dev)
    tf = torch.tensor(f, dtype=torch.float64, device=dev)
    tu = torch.zeros_like(tf)
    opt_m = H.make_options(n, leaf, wl_m.eps, H.HIF_MIXED)
    opt_d = H.make_options(n, leaf, wl_d.eps, H.HIF_FP64)
    A = H.hif_problem_create(opt_m, ta, tb)
    torch.cuda.synchronize()

    def step(opts, keep=False):
        t0 = time.perf_counter()
        F = H.hif_build(A, opts)
        t1 = time.perf_counter()
        st, info = H.hif_pcg(A, F, tf, tu, tol=args.tol, maxit=args.maxit)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        stats = H.hif_factor_stats(F).as_dict()
        if keep:
            return F, st, info[0], stats, t1 - t0, t2 - t1
        H.hif_factor_destroy(F)
        return None, st, info[0], stats, t1 - t0, t2 - t1

    def timed(opts, label):
        for i in range(args.warmup):
            _, st, info, _, tf_, ts_ = step(opts)
            log(f"[{label}] warmup {i}: factor {tf_:.3f}s pcg {ts_:.3f}s it={info.iters}")
        torch.cuda.synchronize()
        H.hif_profile_begin()
        t0 = time.perf_counter()
        rec = []
        for i in range(args.steps):
            _, st, info, stats, tf_, ts_ = step(opts)
            rec.append((st, info.iters, info.relres, info.converged, tf_, ts_))
            log(f"[{label}] step {i}: factor {tf_:.3f}s pcg {ts_:.3f}s it={info.iters} "
                f"relres={info.relres:.2e}")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = H.hif_profile_end()
        return (t1 - t0) / args.steps, rec, stats, prof

    def solve_error(opts):
        """e_s = |x - F^{-1} A x| / |x| for one seeded Gaussian x (the paper's
        relative solve error), on a factor built outside the timed region."""
        g = torch.Generator(device="cpu").manual_seed(7)
        x = torch.randn(N, generator=g, dtype=torch.float64).to(dev)
        y, z = torch.empty_like(x), torch.empty_like(x)
        F = H.hif_build(A, opts)
        H.hif_matvec(A, x, y)
        H.hif_apply(F, y, z)
        torch.cuda.synchronize()
        H.hif_factor_destroy(F)
        return float(torch.linalg.norm(x - z) / torch.linalg.norm(x))

    ms_m, rec_m, stats_m, prof_m = timed(opt_m, "mixed")
    u_m = tu.cpu().numpy().copy()
    out = {"mixed": {"s_per_step": ms_m, "rec": rec_m, "stats": stats_m, "u": u_m,
                     "prof": prof_m, "e_s": solve_error(opt_m)}}
    if not args.skip_fp64:
        ms_d, rec_d, stats_d, prof_d = timed(opt_d, "fp64")
        out["fp64"] = {"s_per_step": ms_d, "rec": rec_d, "stats": stats_d,
                       "u": tu.cpu().numpy().copy(), "prof": prof_d, "e_s": solve_error(opt_d)}
    H.hif_problem_destroy(A)
    out["N"] = N
    out["a"], out["b"], out["f"] = a, b, f
    return out


def run_batched(args):
    """48 independent problems (n drawn from 32^3..96^3, leaf per size, log10 a ~
    U(-1,1), b ~ U(0,1)), FP32 factor at eps 1e-4 + FP64 PCG to 1e-10 each:
    one joint build (hif_build_batched) and one joint solve (hif_pcg_batched)
    against one hif_build and one hif_pcg per problem."""
    import torch
    from paper_1607_00346_amd import hif as H
    from workloads import batched_workloads

    wl = batched_workloads()
    dev = torch.device("cuda:0")
    opts = [H.make_options(w.n, w.leaf, w.eps, H.HIF_MIXED) for w in wl]
    ins = [(torch.tensor(w.a(), dtype=torch.float64, device=dev),
            torch.tensor(w.b(), dtype=torch.float64, device=dev),
            torch.tensor(w.f(), dtype=torch.float64, device=dev)) for w in wl]
    A = [H.hif_problem_create(o, ta, tb) for o, (ta, tb, _) in zip(opts, ins)]
    outs = [torch.zeros_like(t[2]) for t in ins]
    torch.cuda.synchronize()
    total = sum(w.n ** 3 for w in wl)

    def solve_all(F, together):
        its, worst = [], 0.0
        if together:  # one call: the solves overlap on the library's streams
            st, infos = H.hif_pcg_batched(A, F, [x[2] for x in ins], outs, tol=args.tol,
                                          maxit=args.maxit)
        else:
            infos = []
            for i in range(len(wl)):
                st, info = H.hif_pcg(A[i], F[i], ins[i][2], outs[i], tol=args.tol,
                                     maxit=args.maxit)
                infos.append(info[0])
        for i, info in enumerate(infos):
            if not info.converged:
                raise RuntimeError(f"problem {i} did not converge")
            its.append(info.iters)
            worst = max(worst, info.relres)
        torch.cuda.synchronize()
        return its, worst

    peak = {}

    def joint():
        t0 = time.perf_counter()
        F = H.hif_build_batched(A, opts)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        its, worst = solve_all(F, True)
        t2 = time.perf_counter()
        peak["joint_gb"] = H.hif_factor_stats(F[0]).peak_bytes / 1e9
        peak["factor_gb"] = sum(H.hif_factor_stats(x).factor_bytes for x in F) / 1e9
        peak["level_s"] = H.hif_factor_stats(F[0]).as_dict()["level_seconds"]
        for x in F:
            H.hif_factor_destroy(x)
        return t1 - t0, t2 - t1, its, worst

    def separate():
        t0 = time.perf_counter()
        F = [H.hif_build(A[i], opts[i]) for i in range(len(wl))]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        its, worst = solve_all(F, False)
        t2 = time.perf_counter()
        for x in F:
            H.hif_factor_destroy(x)
        return t1 - t0, t2 - t1, its, worst

    for i in range(args.warmup):
        r = joint()
        log(f"[batched] warmup {i}: joint factor {r[0]:.3f}s pcg {r[1]:.3f}s")
        r = separate()
        log(f"[batched] warmup {i}: separate factor {r[0]:.3f}s pcg {r[1]:.3f}s")
    rj, rs = [], []
    for i in range(args.steps):
        rj.append(joint())
        rs.append(separate())
        log(f"[batched] step {i}: joint factor {rj[-1][0]:.3f}s pcg {rj[-1][1]:.3f}s | "
            f"separate factor {rs[-1][0]:.3f}s pcg {rs[-1][1]:.3f}s")
    for a in A:
        H.hif_problem_destroy(a)
    tj = float(np.mean([x[0] + x[1] for x in rj]))
    ts = float(np.mean([x[0] + x[1] for x in rs]))
    sizes = {}
    for w in wl:
        sizes[w.n] = sizes.get(w.n, 0) + 1
    return {
        "metric": "batched HIF factor+solve DOF/s, 48 problems 32^3..96^3 to PCG rel. "
                  "residual 1e-10",
        "value": total / tj, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": tj * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched: 48 problems, n ~ U{32,48,64,96} (seed 400), leaf "
                               "8 or 6, log10 a~U(-1,1), b~U(0,1), FP32 factor eps 1e-4, "
                               "FP64 PCG 1e-10",
                   "problems": len(wl), "dofs": total,
                   "sizes": {str(k): v for k, v in sorted(sizes.items())}},
        "extra": {"joint_t_factor_s": float(np.mean([x[0] for x in rj])),
                  "joint_t_pcg_s": float(np.mean([x[1] for x in rj])),
                  "separate_value": total / ts,
                  "separate_t_factor_s": float(np.mean([x[0] for x in rs])),
                  "separate_t_pcg_s": float(np.mean([x[1] for x in rs])),
                  "joint_over_separate": ts / tj,
                  "pcg_iters_max": int(max(max(x[2]) for x in rj)),
                  "joint_peak_gb": peak.get("joint_gb"), "factor_gb": peak.get("factor_gb"),
                  "joint_level_seconds_device": peak.get("level_s"),
                  "relres_max": float(max(x[3] for x in rj))},
    }


def run_large(args):
    """256^3 (16.8M DOFs), log10 a ~ U(-2,2), b = 0, leaf 8, FP32 factor at eps
    1e-4; 32 right-hand sides solved together by block PCG to 1e-10."""
    import torch
    from paper_1607_00346_amd import hif as H

    wl = WORKLOADS["c256_mixed"]
    n, nr = wl.n, wl.extra["nrhs"]
    N = n ** 3
    dev = torch.device("cuda:0")
    ta = torch.tensor(wl.a(), dtype=torch.float64, device=dev)
    tb = torch.tensor(wl.b(), dtype=torch.float64, device=dev)
    tf = torch.tensor(wl.f(nrhs=nr), dtype=torch.float64, device=dev)
    tu = torch.empty_like(tf)
    opts = H.make_options(n, wl.leaf, wl.eps, H.HIF_MIXED)
    A = H.hif_problem_create(opts, ta, tb)
    torch.cuda.synchronize()
    rec = []
    for i in range(args.warmup + args.steps):
        t0 = time.perf_counter()
        F = H.hif_build(A, opts)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, info = H.hif_pcg(A, F, tf, tu, nrhs=nr, tol=args.tol, maxit=args.maxit)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if st != 0 or not all(x.converged for x in info):
            raise RuntimeError("a right-hand side did not converge")
        stats = H.hif_factor_stats(F).as_dict()
        H.hif_factor_destroy(F)
        log(f"[large] {'warmup' if i < args.warmup else 'step'} {i}: factor {t1 - t0:.3f}s "
            f"pcg({nr} rhs) {t2 - t1:.3f}s it={max(x.iters for x in info)}")
        if i >= args.warmup:
            rec.append((t1 - t0, t2 - t1, max(x.iters for x in info),
                        max(x.relres for x in info), stats))
    H.hif_problem_destroy(A)
    tfac = float(np.mean([x[0] for x in rec]))
    tsol = float(np.mean([x[1] for x in rec]))
    stats = rec[-1][4]
    return {
        "metric": "HIF factor+solve DOF/s at 256^3, 32 RHS, to PCG rel. residual 1e-10",
        "value": N * nr / (tfac + tsol), "unit": "DOF/s (RHS-DOFs solved per second, factor "
                                                 "included)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": (tfac + tsol) * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c256_mixed: 256^3 7-point, log10 a~U(-2,2), b=0, leaf 8, FP32 "
                               "factor eps 1e-4, 32 RHS, block PCG 1e-10",
                   "n": n, "leaf": wl.leaf, "eps": wl.eps, "nrhs": nr},
        "extra": {"t_factor_s": tfac, "t_solve_all_rhs_s": tsol, "t_solve_per_rhs_s": tsol / nr,
                  "pcg_iters_max": rec[-1][2], "relres_max": rec[-1][3],
                  "factor_gb": stats["factor_bytes"] / 1e9, "peak_gb": stats["peak_bytes"] / 1e9,
                  "root_size": stats["root_size"], "levels": stats["levels"],
                  "level_seconds": stats["level_seconds"]},
    }


TRAFFIC_FILES = {"gemm_syrk": "profiles/gemm_syrk_c128_mixed_traffic.txt"}
KERNEL_SOURCE = "paper_1607_00346_amd/csrc/dense.hip"


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed counter summary of this kernel,
    or None when there is none or the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, TRAFFIC_FILES.get(kernel, ""))
    if kernel not in TRAFFIC_FILES or not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    sha = hashlib.sha256(open(os.path.join(ROOT, KERNEL_SOURCE), "rb").read()).hexdigest()
    if fields.get("source_sha256") != sha:
        return None
    return float(fields["traffic_bytes_per_launch"])


def by_class(prof):
    """Sum the per-level entries ("name@level") of each kernel class."""
    out = {}
    for key, v in prof.items():
        base = key.split("@")[0]
        o = out.setdefault(base, {"launches": 0, "seconds": 0.0, "flops": 0.0, "bytes": 0.0})
        for f in o:
            o[f] += v[f]
    return out


def roofline(prof, fp64: bool, counters: bool = True):
    """Dominant kernel class of the timed region against its roofline: flops
    for the matrix-core kernels, bytes for the sweeps."""
    name, k = max(prof.items(), key=lambda kv: kv[1]["seconds"])
    avg = k["seconds"] / max(k["launches"], 1)
    if k["flops"] > 0 and not name.startswith("apply") and name not in ("matvec", "pcg_dot"):
        peak = PEAK["fp64_tflops"] if (fp64 or name in ("gemm_gram", "gemm_interp")) \
            else PEAK["fp32_tflops"]
        ach = k["flops"] / k["seconds"] / 1e12
        return {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                "frac": ach / peak, "traffic": measured_traffic(name) if counters else None,
                "kernel": name,
                "launches": k["launches"], "avg_launch_us": avg * 1e6,
                "flops_per_launch": k["flops"] / max(k["launches"], 1)}
    ach = k["bytes"] / k["seconds"] / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": PEAK["hbm_gbs"], "unit": "GB/s",
            "frac": ach / PEAK["hbm_gbs"], "traffic": None, "kernel": name,
            "launches": k["launches"], "avg_launch_us": avg * 1e6,
            "bytes_per_launch": k["bytes"] / max(k["launches"], 1)}


def kernel_table(prof, steps):
    tot = sum(v["seconds"] for v in prof.values())
    rows = []
    for name, v in sorted(prof.items(), key=lambda kv: -kv[1]["seconds"]):
        r = {"kernel": name, "ms_per_step": 1e3 * v["seconds"] / steps,
             "share": v["seconds"] / tot if tot else 0.0, "launches": v["launches"] // steps}
        if v["flops"] > 0:
            r["tflops"] = v["flops"] / v["seconds"] / 1e12
        if v["bytes"] > 0:
            r["gbs"] = v["bytes"] / v["seconds"] / 1e9
        rows.append(r)
    return rows


def cpu_baseline(args):
    """The oracle (plain FP64 CPU HIF) on a bounded sample of the same law."""
    import oracle as O
    wl = WORKLOADS["c32_contrast"]
    n, leaf = wl.n, wl.leaf
    a, b, f = wl.a(), wl.b(), wl.f()
    reps = 2
    t0 = time.perf_counter()
    for _ in range(reps):
        fac = O.build(n, leaf, a, b, 1e-4)
        A = O.assemble(n, a, b)
        _, it, rel, ok = O.pcg(A, lambda r: O.apply_inverse(fac, r), f, args.tol, args.maxit)
    dt = (time.perf_counter() - t0) / reps
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    return {"value": n ** 3 / dt, "unit": "DOF/s", "cores": threads, "kind": "oracle",
            "sample": f"{n}^3 log10 a~U(-2,2), leaf {leaf}, eps 1e-4, oracle build + PCG to "
                      f"{args.tol:g} ({it} it, {dt:.1f} s per solve, {reps} solves)"}


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=2)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="c128",
                   help="c128 (the headline problem), batched (48 problems of 32^3..96^3) "
                        "or c256 (256^3 with 32 right-hand sides)")
    p.add_argument("--tol", type=float, default=1e-10)
    p.add_argument("--maxit", type=int, default=500)
    p.add_argument("--skip-fp64", action="store_true")
    p.add_argument("--skip-cpu", action="store_true")
    p.add_argument("--skip-extra", action="store_true",
                   help="leave out the batched and 256^3 workloads reported beside the headline "
                        "(also left out by --skip-cpu or --skip-fp64)")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 256 MiB device copy three times (scales the HBM "
                        "byte counters of a profiler run)")
    args = p.parse_args()
    if args.copy_calibration:
        import torch
        n = 256 * 1024 * 1024 // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "copies": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1"}))
        sys.exit(2)

    if args.workload == "batched":
        print(json.dumps(run_batched(args)))
        return
    if args.workload == "c256":
        print(json.dumps(run_large(args)))
        return
    r = run_gpu(args)
    N = r["N"]
    mixed = r["mixed"]
    value = N / mixed["s_per_step"]
    import scipy.sparse  # noqa: F401
    import oracle as O
    A = O.assemble(int(round(N ** (1 / 3))), r["a"], r["b"])
    fn = np.linalg.norm(r["f"])
    res_m = float(np.linalg.norm(r["f"] - A @ mixed["u"]) / fn)
    extra = {"mixed_relres_oracle_matvec": res_m,
             "mixed_pcg_iters": mixed["rec"][-1][1],
             "mixed_solve_error_e_s": mixed["e_s"],
             "mixed_t_factor_s": float(np.mean([x[4] for x in mixed["rec"]])),
             "mixed_t_pcg_s": float(np.mean([x[5] for x in mixed["rec"]])),
             "mixed_root_size": mixed["stats"]["root_size"],
             "mixed_factor_gb": mixed["stats"]["factor_bytes"] / 1e9,
             "mixed_peak_gb": mixed["stats"]["peak_bytes"] / 1e9}
    if "fp64" in r:
        d = r["fp64"]
        extra.update({
            "fp64_value": N / d["s_per_step"],
            "fp64_pcg_iters": d["rec"][-1][1],
            "fp64_solve_error_e_s": d["e_s"],
            "fp64_t_factor_s": float(np.mean([x[4] for x in d["rec"]])),
            "fp64_t_pcg_s": float(np.mean([x[5] for x in d["rec"]])),
            "fp64_relres_oracle_matvec": float(np.linalg.norm(r["f"] - A @ d["u"]) / fn),
            "mixed_vs_fp64_solution_diff": float(np.linalg.norm(mixed["u"] - d["u"])
                                                 / np.linalg.norm(d["u"])),
            "mixed_over_fp64": d["s_per_step"] / mixed["s_per_step"],
            "fp64_root_size": d["stats"]["root_size"],
        })
    line = {
        "metric": "HIF factor+solve DOF/s at 128^3 to PCG rel. residual 1e-10, mixed vs FP64",
        "value": value, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": mixed["s_per_step"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: 128^3 7-point, log10 a~U(-2,2), b=0, leaf 8, "
                               "mixed eps 1e-4 (FP32 fronts) vs FP64 eps 1e-6, PCG 1e-10",
                   "n": 128, "leaf": 8, "eps_mixed": 1e-4, "eps_fp64": 1e-6},
        "extra": extra,
    }
    pm = by_class(mixed["prof"])
    line["roofline"] = roofline(pm, fp64=False)
    apply_classes = {k: v for k, v in pm.items() if k.startswith("apply_")}
    if apply_classes:
        line["extra"]["roofline_apply"] = roofline(apply_classes, fp64=False)
    line["extra"]["kernels_mixed"] = kernel_table(pm, args.steps)
    line["extra"]["kernels_mixed_by_level"] = kernel_table(mixed["prof"], args.steps)[:40]
    if "fp64" in r:
        pd = by_class(r["fp64"]["prof"])
        # the committed counter runs cover the mixed factorization only
        line["extra"]["roofline_fp64"] = roofline(pd, fp64=True, counters=False)
        line["extra"]["kernels_fp64"] = kernel_table(pd, args.steps)
        line["extra"]["kernels_fp64_by_level"] = kernel_table(r["fp64"]["prof"], args.steps)[:40]
    line["extra"]["stats_mixed"] = {k: mixed["stats"][k] for k in (
        "cells", "faces", "eliminated", "face_dofs", "redundant", "max_front", "level_seconds",
        "factor_flops")}
    if not (args.skip_extra or args.skip_cpu or args.skip_fp64):
        # full runs only: the batched and large workloads, one warm-up and one
        # timed step each, reported beside the headline (a failure there does
        # not void it)
        sub = argparse.Namespace(**vars(args))
        sub.steps, sub.warmup = 1, 1
        from paper_1607_00346_amd import hif as H
        for key, fn in (("batched", run_batched), ("c256", run_large)):
            try:
                # blocks cached for the previous workload's sizes would not fit this one
                H.hif_release_cached_memory()
                r = fn(sub)
                line["extra"]["workload_" + key] = {
                    "metric": r["metric"], "value": r["value"], "unit": r["unit"],
                    "ms_per_step": r["ms_per_step"], "config": r["config"], "extra": r["extra"]}
            except Exception as e:  # noqa: BLE001
                line["extra"]["workload_" + key] = {"error": repr(e)}
    if not args.skip_cpu:
        line["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
