"""Benchmark: HIF factor + PCG solve throughput (DOF/s) on one MI355X.

One step = hif_build of the 128^3 high-contrast problem (log10 a ~ U(-2,2)
per node, b = 0, leaf 8^3) followed by hif_pcg to a true relative residual of
1e-10.  `value` is the mixed-precision run (FP32 fronts, eps = 1e-4, FP64
PCG); the plain FP64 GPU HIF (eps = 1e-6) is timed the same way beside it
(`fp64_value`).  Inputs are synthetic and already resident in HBM when timing
starts.  Each step is timed on its own (host clock, device synchronized at
both ends); `ms_per_step` is the median, with min, max and mean beside it.

Inside the timed region the library records HIP event pairs only around the
launches of the dominant kernel class (found in one profiled step before the
timed region), which gives that class's average launch duration for the
roofline.  Kernel tables of the profiled step go to --detail (a JSON file),
never to stdout.

Prints ONE short JSON line, the last line on stdout.  Only one GPU is
supported: --gpus > 1 exits with a message.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from workloads import WORKLOADS  # noqa: E402

PEAK = {"fp64_tflops": 78.6, "fp32_tflops": 157.3, "hbm_gbs": 8000.0}
METRIC = "HIF factor+solve DOF/s at 128^3 to PCG rel. residual 1e-10, mixed vs FP64"


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def by_class(prof):
    """Sum the per-level entries ("name@level") of each kernel class."""
    out = {}
    for key, v in prof.items():
        base = key.split("@")[0]
        o = out.setdefault(base, {"launches": 0, "seconds": 0.0, "flops": 0.0, "bytes": 0.0})
        for f in o:
            o[f] += v[f]
    return out


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


def is_sweep(name: str) -> bool:
    return name.startswith("apply") or name in ("matvec", "pcg_dot")


def dominant(prof_cls):
    return max(prof_cls.items(), key=lambda kv: kv[1]["seconds"])[0]


def roofline(name, k, fp64: bool, counters: bool = True):
    """One kernel class against its roofline: algorithmic flops per launch for
    the matrix-core kernels, algorithmic bytes for the sweeps, divided by the
    class's average event-timed launch duration."""
    launches = max(k["launches"], 1)
    avg = k["seconds"] / launches
    if k["flops"] > 0 and not is_sweep(name):
        peak = PEAK["fp64_tflops"] if (fp64 or name in ("gemm_gram", "gemm_interp")) \
            else PEAK["fp32_tflops"]
        ach = k["flops"] / launches / avg / 1e12
        return {"bound": "mfma", "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(ach / peak, 4),
                "traffic": measured_traffic(name) if counters else None,
                "kernel": name, "launches": k["launches"], "avg_launch_us": round(avg * 1e6, 1),
                "flops_per_launch": k["flops"] / launches}
    ach = k["bytes"] / launches / avg / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK["hbm_gbs"], "unit": "GB/s",
            "frac": round(ach / PEAK["hbm_gbs"], 4), "traffic": None, "kernel": name,
            "launches": k["launches"], "avg_launch_us": round(avg * 1e6, 1),
            "bytes_per_launch": k["bytes"] / launches}


def stats_of(times):
    return {"median": statistics.median(times), "min": min(times), "max": max(times),
            "mean": sum(times) / len(times)}


def run_c128(args, detail):
    import torch
    from paper_1607_00346_amd import hif as H

    wl_m = WORKLOADS["c128_mixed"]
    wl_d = WORKLOADS["c128_fp64"]
    n, leaf = wl_m.n, wl_m.leaf
    N = n ** 3
    dev = torch.device("cuda:0")
    a, b, f = wl_m.a(), wl_m.b(), wl_m.f()
    ta = torch.tensor(a, dtype=torch.float64, device=dev)
    tb = torch.tensor(b, dtype=torch.float64, device=dev)
    tf = torch.tensor(f, dtype=torch.float64, device=dev)
    opts = {"mixed": H.make_options(n, leaf, wl_m.eps, H.HIF_MIXED),
            "fp64": H.make_options(n, leaf, wl_d.eps, H.HIF_FP64)}
    A = H.hif_problem_create(opts["mixed"], ta, tb)
    torch.cuda.synchronize()

    def step(o, tu):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = H.hif_build(A, o)
        t1 = time.perf_counter()
        st, info = H.hif_pcg(A, F, tf, tu, tol=args.tol, maxit=args.maxit)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if st != 0 or not info[0].converged:
            raise RuntimeError(f"PCG did not converge (status {st})")
        stats = H.hif_factor_stats(F).as_dict()
        H.hif_factor_destroy(F)
        return t1 - t0, t2 - t1, info[0], stats

    out = {}
    labels = ["mixed"] if args.skip_fp64 else ["mixed", "fp64"]
    for label in labels:
        o = opts[label]
        tu = torch.zeros_like(tf)
        for i in range(args.warmup):
            tfac, tpcg, info, _ = step(o, tu)
        if args.warmup:
            log(f"[{label}] warm-up done: last factor {tfac:.3f}s pcg {tpcg:.3f}s it={info.iters}")
        # one profiled step outside the timed region: every kernel class
        H.hif_profile_select(None)
        H.hif_profile_begin()
        step(o, tu)
        prof_all = H.hif_profile_end()
        cls_all = by_class(prof_all)
        dom = dominant(cls_all)
        # the timed region: events around the dominant class's launches only
        H.hif_profile_select(dom)
        H.hif_profile_begin()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec = []
        for i in range(args.steps):
            rec.append(step(o, tu))
        torch.cuda.synchronize()
        t_region = time.perf_counter() - t0
        prof_dom = by_class(H.hif_profile_end())
        H.hif_profile_select(None)
        times = [r[0] + r[1] for r in rec]
        st = stats_of(times)
        its = [r[2].iters for r in rec]
        log(f"[{label}] {args.steps} steps: median {st['median'] * 1e3:.1f} ms "
            f"(min {st['min'] * 1e3:.1f}, max {st['max'] * 1e3:.1f}); factor median "
            f"{statistics.median(r[0] for r in rec) * 1e3:.1f} ms, PCG median "
            f"{statistics.median(r[1] for r in rec) * 1e3:.1f} ms, {its[-1]} iterations")
        out[label] = {
            "times": st, "t_region": t_region,
            "t_factor": statistics.median(r[0] for r in rec),
            "t_pcg": statistics.median(r[1] for r in rec),
            "iters": its[-1], "relres": rec[-1][2].relres, "stats": rec[-1][3],
            "u": tu.cpu().numpy().copy(),
            "dominant": dom, "prof_dom": prof_dom.get(dom),
        }
        detail[label] = {"kernels": kernel_table(cls_all, 1),
                         "kernels_by_level": kernel_table(prof_all, 1)[:60],
                         "stats": rec[-1][3],
                         "step_seconds": times}
        apply_cls = {k: v for k, v in cls_all.items() if k.startswith("apply_")}
        if apply_cls:
            an = dominant(apply_cls)
            detail[label]["roofline_apply"] = roofline(an, apply_cls[an], label == "fp64", False)
    # accuracy diagnostics outside the timed region
    g = torch.Generator(device="cpu").manual_seed(7)
    x = torch.randn(N, generator=g, dtype=torch.float64).to(dev)
    for label in labels:
        F = H.hif_build(A, opts[label])
        e_s, _ = H.hif_factor_error(A, F, x, power_iters=0)
        out[label]["e_s"] = e_s
        H.hif_factor_destroy(F)
    H.hif_problem_destroy(A)
    import oracle as O
    Ao = O.assemble(n, a, b)
    fn = np.linalg.norm(f)
    for label in labels:
        out[label]["relres_oracle"] = float(np.linalg.norm(f - Ao @ out[label]["u"]) / fn)
    if "fp64" in out:
        out["diff"] = float(np.linalg.norm(out["mixed"]["u"] - out["fp64"]["u"])
                            / np.linalg.norm(out["fp64"]["u"]))
    out["N"] = N
    return out


def run_batched(args, detail):
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
        if together:
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

    extra = {}

    def joint():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = H.hif_build_batched(A, opts)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        its, worst = solve_all(F, True)
        t2 = time.perf_counter()
        s0 = H.hif_factor_stats(F[0]).as_dict()
        extra["joint_peak_gb"] = s0["peak_bytes"] / 1e9
        extra["factor_gb"] = sum(H.hif_factor_stats(x).factor_bytes for x in F) / 1e9
        extra["level_seconds_device"] = s0["level_seconds"]
        for x in F:
            H.hif_factor_destroy(x)
        return t1 - t0, t2 - t1, its, worst

    def separate():
        torch.cuda.synchronize()
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
        joint()
        separate()
    rj, rs = [], []
    for i in range(args.steps):
        rj.append(joint())
        rs.append(separate())
        log(f"[batched] step {i}: joint factor {rj[-1][0]:.3f}s pcg {rj[-1][1]:.3f}s | "
            f"separate factor {rs[-1][0]:.3f}s pcg {rs[-1][1]:.3f}s")
    for a in A:
        H.hif_problem_destroy(a)
    sj = stats_of([x[0] + x[1] for x in rj])
    ss = stats_of([x[0] + x[1] for x in rs])
    sizes = {}
    for w in wl:
        sizes[w.n] = sizes.get(w.n, 0) + 1
    detail["batched"] = {"joint": [x[:2] for x in rj], "separate": [x[:2] for x in rs], **extra}
    return {
        "metric": "batched HIF factor+solve DOF/s, 48 problems 32^3..96^3 to PCG rel. "
                  "residual 1e-10",
        "value": total / sj["median"], "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sj["median"] * 1e3,
        "ms_per_step_min": sj["min"] * 1e3, "ms_per_step_max": sj["max"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "batched: 48 problems, n ~ U{32,48,64,96} (seed 400), leaf "
                               "8 or 6, log10 a~U(-1,1), b~U(0,1), FP32 factor eps 1e-4, "
                               "FP64 PCG 1e-10",
                   "problems": len(wl), "dofs": total,
                   "sizes": {str(k): v for k, v in sorted(sizes.items())}},
        "separate_value": total / ss["median"],
        "joint_over_separate": ss["median"] / sj["median"],
        "joint_t_factor_s": statistics.median(x[0] for x in rj),
        "joint_t_pcg_s": statistics.median(x[1] for x in rj),
        "pcg_iters_max": int(max(max(x[2]) for x in rj)),
        "relres_max": float(max(x[3] for x in rj)),
        "joint_peak_gb": extra.get("joint_peak_gb"), "factor_gb": extra.get("factor_gb"),
    }


def run_large(args, detail):
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
    s = stats_of([x[0] + x[1] for x in rec])
    tfac = statistics.median(x[0] for x in rec)
    tsol = statistics.median(x[1] for x in rec)
    stats = rec[-1][4]
    detail["c256"] = {"steps": [x[:4] for x in rec], "stats": stats}
    return {
        "metric": "HIF factor+solve DOF/s at 256^3, 32 RHS, to PCG rel. residual 1e-10",
        "value": N * nr / s["median"],
        "unit": "DOF/s (RHS-DOFs solved per second, factor included)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": s["median"] * 1e3, "ms_per_step_min": s["min"] * 1e3,
        "ms_per_step_max": s["max"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "c256_mixed: 256^3 7-point, log10 a~U(-2,2), b=0, leaf 8, FP32 "
                               "factor eps 1e-4, 32 RHS, block PCG 1e-10",
                   "n": n, "leaf": wl.leaf, "eps": wl.eps, "nrhs": nr},
        "t_factor_s": tfac, "t_solve_per_rhs_s": tsol / nr,
        "pcg_iters_max": rec[-1][2], "relres_max": rec[-1][3],
        "factor_gb": stats["factor_bytes"] / 1e9, "peak_gb": stats["peak_bytes"] / 1e9,
    }


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(args):
    """The oracle (plain FP64 CPU HIF, one Python process with BLAS pinned to
    one thread) on bounded samples: the 16^3 constant-coefficient problem and
    a 32^3 sample of the headline law (log10 a ~ U(-2,2), leaf 8^3), each a
    full build + PCG to the same tolerance.  `value` is the 32^3 rate."""
    from threadpoolctl import threadpool_limits
    import oracle as O

    def one(name, eps):
        wl = WORKLOADS[name]
        a, b, f = wl.a(), wl.b(), wl.f()
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            fac = O.build(wl.n, wl.leaf, a, b, eps)
            A = O.assemble(wl.n, a, b)
            _, it, rel, ok = O.pcg(A, lambda r: O.apply_inverse(fac, r), f, args.tol,
                                   args.maxit)
            dt = time.perf_counter() - t0
        return wl.n ** 3 / dt, dt, it
    v16, t16, i16 = one("c16_const", 1e-6)
    v32, t32, i32 = one("c32_contrast", 1e-4)
    return {"value": v32, "unit": "DOF/s", "cores": 1, "kind": "oracle",
            "sample": f"32^3 log10 a~U(-2,2) leaf 8 eps 1e-4: oracle build + PCG to {args.tol:g} "
                      f"({i32} it) in {t32:.1f} s; 16^3 a=1 leaf 4 eps 1e-6: {v16:.0f} DOF/s "
                      f"({t16:.2f} s, {i16} it); single process, BLAS 1 thread",
            "host": {"nproc": os.cpu_count(), "cpu": cpu_model()}}


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="c128",
                   help="c128 (the headline problem), batched (48 problems of 32^3..96^3) "
                        "or c256 (256^3 with 32 right-hand sides)")
    p.add_argument("--tol", type=float, default=1e-10)
    p.add_argument("--maxit", type=int, default=500)
    p.add_argument("--skip-fp64", action="store_true")
    p.add_argument("--skip-cpu", action="store_true")
    p.add_argument("--detail", default=None,
                   help="write kernel tables and per-step times to this JSON file")
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
        print(json.dumps({"error": "this build runs on exactly one GPU: the HIF here factors "
                                   "the whole problem on one device; --gpus must be 1"}))
        sys.exit(2)
    if args.steps < 1:
        raise SystemExit("--steps must be >= 1")
    detail = {}
    if args.workload == "batched":
        line = run_batched(args, detail)
    elif args.workload == "c256":
        line = run_large(args, detail)
    else:
        r = run_c128(args, detail)
        N = r["N"]
        m = r["mixed"]
        line = {
            "metric": METRIC, "value": N / m["times"]["median"], "unit": "DOF/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": m["times"]["median"] * 1e3,
            "ms_per_step_min": m["times"]["min"] * 1e3,
            "ms_per_step_max": m["times"]["max"] * 1e3,
            "ms_per_step_mean": m["times"]["mean"] * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": "c128: 128^3 7-point -div(a grad u), log10 a~U(-2,2) per node, "
                                   "b=0, Dirichlet, leaf 8^3; mixed = FP32 factor eps 1e-4 + FP64 "
                                   "PCG; fp64 = FP64 factor eps 1e-6 + FP64 PCG; PCG to 1e-10",
                       "n": 128, "leaf": 8, "eps_mixed": 1e-4, "eps_fp64": 1e-6},
            "t_factor_s": round(m["t_factor"], 5), "t_pcg_s": round(m["t_pcg"], 5),
            "pcg_iters": m["iters"], "relres_oracle_matvec": m["relres_oracle"],
            "e_s": m["e_s"], "root_size": m["stats"]["root_size"],
            "factor_gb": round(m["stats"]["factor_bytes"] / 1e9, 3),
            "peak_gb": round(m["stats"]["peak_bytes"] / 1e9, 3),
        }
        if "fp64" in r:
            d = r["fp64"]
            line.update({
                "fp64_value": N / d["times"]["median"],
                "fp64_ms_per_step": d["times"]["median"] * 1e3,
                "fp64_ms_per_step_min": d["times"]["min"] * 1e3,
                "fp64_ms_per_step_max": d["times"]["max"] * 1e3,
                "fp64_t_factor_s": round(d["t_factor"], 5), "fp64_t_pcg_s": round(d["t_pcg"], 5),
                "fp64_pcg_iters": d["iters"], "fp64_relres_oracle_matvec": d["relres_oracle"],
                "fp64_e_s": d["e_s"],
                "mixed_over_fp64": d["times"]["median"] / m["times"]["median"],
                "mixed_vs_fp64_solution_diff": r["diff"],
            })
        k = m["prof_dom"]
        if k:
            line["roofline"] = roofline(m["dominant"], k, fp64=False)
        if "fp64" in r and r["fp64"]["prof_dom"]:
            rf = roofline(r["fp64"]["dominant"], r["fp64"]["prof_dom"], fp64=True, counters=False)
            line["fp64_roofline"] = {x: rf[x] for x in ("kernel", "achieved", "peak", "unit",
                                                         "frac")}
    if not args.skip_cpu and args.workload == "c128":
        line["cpu_baseline"] = cpu_baseline(args)
    if args.detail:
        os.makedirs(os.path.dirname(os.path.abspath(args.detail)), exist_ok=True)
        with open(args.detail, "w") as fh:
            json.dump(detail, fh, indent=1, default=float)
    sys.stderr.flush()
    print(json.dumps(line, default=float), flush=True)


if __name__ == "__main__":
    main()
