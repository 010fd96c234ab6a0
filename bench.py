"""Benchmark of the MI355X FEAST hot path (one GPU).

One step = one complete FEAST solve (factorizations of the n_c shifted matrices, the filter
application Q = rho(A) X with its triangular solves and accumulation, Rayleigh-Ritz and the
residual test, iterated to convergence) on one synthetic problem resident in HBM.  The factor
cache is dropped before every step, so each step refactors.

Default workload (the configuration the headline metric is quoted on): complex Hermitian
A = U diag(lam) U^H with n = 8192, 200 eigenvalues in I = (-0.05, 0.05) of which 40 lie within
1e-3 inside each endpoint, 100 within 1e-3 outside each endpoint, the rest uniform on [-1, 1];
m0 = 300, n_c = 8, FP64.  Timed steps stop at max residual <= 1e-10 ||A|| (the metric's
threshold); the warm-up step runs the configuration's own tolerance 1e-12 and is checked
against the exact eigenvalues of the construction.

Prints one JSON line (see --help for options).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FEAST time-to-solution (res≤1e-10‖A‖) + filter-apply TFLOP/s, mixed vs FP64"
PEAK_FP64_MFMA = 78.6  # TFLOP/s, MI355X dense FP64 matrix
PEAK_FP32_MFMA = 157.3
# bf16x3 products: three bf16 matrix-core products per FP32 one (dense bf16 peak 2.5 PFLOP/s)
PEAK_BF16X3_MFMA = 2500.0 / 3
PEAKS = {0: PEAK_FP64_MFMA, 1: PEAK_FP32_MFMA, 2: PEAK_BF16X3_MFMA}
SWEEP_KERNEL = {0: "gemm_kernel<double>", 1: "gemm_kernel<float>", 2: "gemmx_kernel (bf16x3)"}
PEAK_HBM = 8000.0      # GB/s
PRECS = {"fp64": 0, "fp32ir": 1, "bf16x3ir": 2}


# HBM bytes per launch of the paired sweep GEMM on the default workload (FP64, n=8192), from
# rocprofv3 FETCH_SIZE and WRITE_SIZE runs scaled by a plain copy of known size; valid only
# while the sources of that kernel (gemm.hip), of its launches and block height (solve.hip)
# and their common header are the ones the counters were taken on.
SWEEP_TRAFFIC = {"sources": "c50978dcbb339c8e", "bytes_per_launch": 9.554e8}


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("gemm.hip", "solve.hip", "common.h"):
        with open(os.path.join(ROOT, "paper_1605_08771_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_problem(args, dev):
    from paper_1605_08771_amd import gen
    t0 = time.time()
    if args.workload == "c2":
        p = gen.config2(n=args.n or 8192, device=dev, basis=args.basis)
    elif args.workload == "c3":
        p = gen.config3(n=args.n or 16384, device=dev)
    elif args.workload == "c5":
        p = gen.config5(n=args.n or 32768, device=dev)
    else:
        raise SystemExit(f"unknown workload {args.workload}")
    log(f"[bench] generated {p.name} n={p.n} m0={p.m0} n_c={p.n_c} m_true={p.m_true} "
        f"in {time.time() - t0:.1f}s")
    return p


def cpu_baseline(p, iters, nodes_z):
    """The oracle timed on a bounded sample of the same workload, extrapolated by flop counts.

    Sample: the leading ns x ns principal block of A (ns = 1024) with the same m0: one
    partial-pivot LU of z_1 I - A_s, one pair of m0-column solves (Y and the adjoint Y'), and
    one Rayleigh-Ritz on an ns x m0 block.  Extrapolation: LU ~ n^3, solves and Rayleigh-Ritz
    ~ n^2 m0; n_c nodes run on min(n_c, threads) oracle threads (the oracle parallelises over
    nodes only); the GPU run's iteration count."""
    import oracle
    A = p.A.cpu().numpy() if hasattr(p.A, "cpu") else p.A
    X0 = p.X0.cpu().numpy() if hasattr(p.X0, "cpu") else p.X0
    ns = min(1024, p.n)
    As = np.asfortranarray(A[:ns, :ns])
    M = nodes_z[0] * np.eye(ns) - As
    t0 = time.perf_counter()
    LU, piv, _ = oracle.zlu(M)
    t_lu = time.perf_counter() - t0
    B = np.asfortranarray(X0[:ns, :p.m0])
    t0 = time.perf_counter()
    oracle.zlu_solve(LU, piv, B)
    oracle.zlu_solve(LU, piv, B, adjoint=True)
    t_solve = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.rayleigh_ritz("c128", As, B, p.emin, p.emax, p.anorm)
    t_rr = time.perf_counter() - t0
    s3 = (p.n / ns) ** 3
    s2 = (p.n / ns) ** 2
    threads = max(1, min(p.n_c, oracle.num_threads()))
    par = p.n_c / threads
    total = par * t_lu * s3 + iters * (par * t_solve * s2 + t_rr * s2)
    sample = (f"oracle on the leading {ns}x{ns} block: LU {t_lu:.2f}s, {p.m0}-column solve "
              f"pair {t_solve:.2f}s, Rayleigh-Ritz {t_rr:.2f}s; extrapolated by n^3 (LU) and "
              f"n^2 m0 (solves, RR) to n={p.n}, n_c={p.n_c} over {threads} threads, {iters} "
              f"iterations")
    return dict(value=round(total, 1), unit="s", cores=threads, kind="oracle", sample=sample,
                measured_s=round(t_lu + t_solve + t_rr, 2))


def bench_batched(args, dev):
    """Config 4: 64 independent complex Hermitian problems, n ~ U{256..4096}, each with its own
    interval holding ~8% of its spectrum and edge clusters; one step = solving all of them."""
    import torch
    import paper_1605_08771_amd as fm
    from paper_1605_08771_amd import gen
    t0 = time.time()
    specs = gen.config4_specs()
    probs = [gen.config4_problem(sp, device=dev) for sp in specs]
    log(f"[bench] generated {len(probs)} problems in {time.time() - t0:.1f}s")
    prec_name = args.prec or "fp32ir"
    prec = PRECS[prec_name]
    d = [dict(A=p.A, X0=p.X0, emin=p.emin, emax=p.emax, m0=p.m0, anorm=p.anorm) for p in probs]
    f = fm.Feast()

    def one(nstreams, pr=prec):
        f.invalidate()
        return f.solve_batched(d, n_c=8, tol=1e-10, max_iter=400, prec=pr, spurious=True,
                               nstreams=nstreams)

    def check(outs):
        errs, ok = [], True
        for p, o in zip(probs, outs):
            sel = (o["lam"] > p.emin) & (o["lam"] < p.emax)
            good = o["status"] == 0 and o["m"] == p.m_true
            ok &= good
            if good:
                ex = np.sort(p.lam[(p.lam > p.emin) & (p.lam < p.emax)])
                lam_in = np.sort(o["lam"][sel])
                # Ritz values that fail the filter test may sit in I; match the nearest ones
                errs.append(float(np.max(np.min(np.abs(lam_in[:, None] - ex[None, :]), axis=0))))
        return ok, (max(errs) if errs else float("nan"))

    for w in range(args.warmup):
        torch.cuda.synchronize()
        one(args.nstreams)
        torch.cuda.synchronize()
    f.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for k in range(args.steps):
        results.append(one(args.nstreams))
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    solve = f.kernel_stats("solve")
    f.set_profiling(False)
    bad, outs = results[-1]
    ok, err = check(outs)
    iters = [o["iters"] for o in outs]
    log(f"[bench] c4: bad={bad} ok={ok} max|dlam|={err:.2e} iters min/med/max "
        f"{min(iters)}/{int(np.median(iters))}/{max(iters)} time/step {total / args.steps:.3f}s")
    alg = sum(o["iters"] * 8 * 2 * 8.0 * p.n * p.n * p.m0 for p, o in zip(probs, outs)) * args.steps
    peak = PEAKS[prec]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    seq = one(1)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t1
    f.close()
    line = {
        "metric": METRIC, "value": round(total / args.steps, 4), "unit": "s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1000 * total / args.steps, 2), "higher_is_better": False,
        "scaling": "strong", "vs_baseline": None,
        "dtype": "f64" if prec == fm.FEAST_FP64 else "f32+f64", "data": "synthetic",
        "config": {"workload": f"C4: 64 complex Hermitian problems, n~U{{256..4096}} "
                               f"(sum n^2={sum(p.n * p.n for p in probs)}), own intervals with "
                               f"~8% of the spectrum and edge clusters, m0=ceil(1.5m), n_c=8, "
                               f"{prec_name}, {args.nstreams} streams, stop at res<=1e-10*||A||",
                   "problems": len(probs), "precision": prec_name, "nstreams": args.nstreams},
        "roofline": {"kernel": "gemm_kernel triangular sweeps (all workers; overlapping streams)",
                     "bound": "mfma",
                     "achieved": round(alg / (solve["ms"] * 1e-3) / 1e12, 2) if solve["ms"] else None,
                     "peak": peak, "unit": "TFLOP/s",
                     "frac": round(alg / (solve["ms"] * 1e-3) / 1e12 / peak, 4) if solve["ms"] else None,
                     "traffic": None, "launches": solve["launches"],
                     "note": "kernel time summed over concurrent streams"},
        "correct": ok and bad == 0, "max_eig_err": err,
        "iterations_min_median_max": [min(iters), int(np.median(iters)), max(iters)],
        "sequential_one_stream_s": round(t_seq, 4),
        "cpu_baseline": None,
    }
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5"])
    ap.add_argument("--nstreams", type=int, default=8, help="c4: concurrent worker streams")
    ap.add_argument("--n", type=int, default=0, help="override n (tests only)")
    ap.add_argument("--prec", default="", choices=["", *PRECS])
    ap.add_argument("--compare", default=None,
                    help="comma-separated precisions run after the timed steps on the same "
                         "input and threshold (default: the other of fp64/fp32ir; c3 adds "
                         "bf16x3ir, the split-precision factorization)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the run in the other precision")
    ap.add_argument("--basis", default="haar", choices=["haar", "householder"],
                    help="c2 eigenvectors: QR of a Gaussian matrix (default) or 8 dense "
                         "reflectors built without library factorizations (for counter runs)")
    ap.add_argument("--variants", default=None,
                    help="comma list of method:s[:precision] runs of the Sec. 2 variants "
                         "reported beside FEAST (default for c2: rfeast:2,rfeast:3,xfeast:2,"
                         "xfeast:3,xfeast:2:fp32ir; '' = none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        raise SystemExit(2)

    import torch
    import paper_1605_08771_amd as fm

    assert torch.cuda.is_available(), "bench.py needs the HIP device"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "c4":
        return bench_batched(args, dev)
    p = make_problem(args, dev)
    prec_name = args.prec or ("fp32ir" if args.workload in ("c3", "c5") else "fp64")
    prec = PRECS[prec_name]
    A = p.A
    X0 = p.X0
    f = fm.Feast()
    exact_in = np.sort(p.lam[(p.lam > p.emin) & (p.lam < p.emax)])

    def one(tol, max_iter=p.max_iter, pr=None, method="feast", expand=1):
        f.invalidate()
        out = f.solve(A, p.emin, p.emax, p.m0, n_c=p.n_c, tol=tol, max_iter=max_iter,
                      anorm=p.anorm, X0=X0, prec=prec if pr is None else pr, spurious=True,
                      refine_max=0, method=method, expand=expand)
        return out

    def check(out, tol):
        sel = (out["lam"] > p.emin) & (out["lam"] < p.emax) & (out["mu"] > 0.5)
        ok = out["status"] == 0 and out["m"] == p.m_true
        err = float(np.max(np.abs(out["lam"][sel] - exact_in))) if ok else float("nan")
        res = float(np.max(out["res"][sel])) if sel.any() else float("nan")
        return ok, err, res

    # warm-up at the configuration's own tolerance
    warm = {}
    for w in range(args.warmup):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = one(p.tol)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ok, err, res = check(out, p.tol)
        warm = dict(time_s=dt, iters=out["iters"], ok=ok, eig_err=err, res=res,
                    status=out["status"])
        log(f"[bench] warmup {w}: status={out['status']} iters={out['iters']} m={out['m']} "
            f"time={dt:.3f}s max|dlam|={err:.2e} max res={res:.2e}")

    # timed steps at the metric's threshold, kernel profiling on the library stream
    f.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs, phases, step_s = [], [], []
    for k in range(args.steps):
        ts = time.perf_counter()
        out = one(1e-10)  # returns after the solve's final stream sync (host outputs)
        step_s.append(time.perf_counter() - ts)
        outs.append(out)
        phases.append(f.timings())
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ms_per_step = 1000.0 * total / args.steps
    iters = [o["iters"] for o in outs]
    checks = [check(o, 1e-10) for o in outs]
    for k, (o, c) in enumerate(zip(outs, checks)):
        log(f"[bench] step {k}: status={o['status']} iters={o['iters']} m={o['m']} "
            f"max|dlam|={c[1]:.2e} max res={c[2]:.2e} phases={phases[k]}")
    solve = f.kernel_stats("solve")
    lu = f.kernel_stats("lu")
    rr = f.kernel_stats("rr")
    eig_main = f.kernel_stats("eig")
    sides = 2
    # filter applications: one per iteration plus the one that gives the last iterate's
    # filter values mu_k (the spurious-pair test is on)
    n_filters = sum(iters) + args.steps
    alg_solve = n_filters * p.n_c * sides * 8.0 * p.n * p.n * p.m0
    # algorithmic HBM bytes of the sweeps: each factor read once per sweep (forward and
    # backward; the two sides read complementary triangles) and each right-hand-side block
    # read and written once per sweep
    alg_solve_bytes = n_filters * p.n_c * 2 * (16.0 * p.n * p.n + sides * 2 * 16.0 * p.n * p.m0)
    achieved = alg_solve / (solve["ms"] * 1e-3) / 1e12 if solve["ms"] > 0 else 0.0
    peak = PEAKS[prec]
    filt_ms = sum(ph["solve_ms"] + ph["accumulate_ms"] for ph in phases)
    alg_filter = alg_solve + n_filters * p.n_c * sides * 8.0 * p.n * p.m0
    filter_tflops = alg_filter / (filt_ms * 1e-3) / 1e12 if filt_ms > 0 else 0.0
    f.set_profiling(False)

    # other precisions on the same input, to the same threshold (mixed vs FP64)
    cspec = args.compare
    if cspec is None:
        cspec = "fp32ir" if prec_name == "fp64" else "fp64"
        if args.workload == "c3":
            cspec += ",bf16x3ir"
    compares = []
    for other_name in [c for c in cspec.split(",") if c and c != prec_name]:
        if args.no_compare:
            break
        other = PRECS[other_name]
        one(1e-10, pr=other)  # warm-up of the other path's buffers
        f.set_profiling(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o2 = one(1e-10, pr=other)
        torch.cuda.synchronize()
        t_other = time.perf_counter() - t0
        lu2, solve2 = f.kernel_stats("lu"), f.kernel_stats("solve")
        f.set_profiling(False)
        ok2, err2, res2 = check(o2, 1e-10)
        rec = {"precision": other_name, "time_s": round(t_other, 4), "iterations": o2["iters"],
               "correct": ok2, "max_eig_err": err2, "max_residual": res2,
               "phase_ms": {k: round(v, 2) for k, v in f.timings().items()},
               "lu_gemm_ms": round(lu2["ms"], 2), "solve_gemm_ms": round(solve2["ms"], 2),
               "speedup_of_value_path": round(t_other / (total / args.steps), 3)}
        compares.append(rec)
        log(f"[bench] {other_name}: {rec}")
    compare = compares[0] if compares else None
    # the expanded-subspace variants of Sec. 2 on the same input and threshold
    variants = []
    vspec = args.variants
    if vspec is None:
        vspec = ("rfeast:2,rfeast:3,xfeast:2,xfeast:3,xfeast:2:fp32ir" if args.workload == "c2"
                 else "")
    for item in [v for v in vspec.split(",") if v]:
        parts = item.split(":")  # method:expand[:precision]
        meth, sx = parts[0], int(parts[1])
        vprec_name = parts[2] if len(parts) > 2 else prec_name
        vprec = PRECS[vprec_name]
        one(1e-10, max_iter=2, pr=vprec, method=meth, expand=sx)  # buffers, recorded sweeps
        f.set_profiling(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ov = one(1e-10, pr=vprec, method=meth, expand=sx)
        torch.cuda.synchronize()
        tv = time.perf_counter() - t0
        eig = f.kernel_stats("eig")
        f.set_profiling(False)
        okv, errv, resv = check(ov, 1e-10)
        rec = {"method": meth, "expand": sx, "precision": vprec_name, "time_s": round(tv, 4),
               "iterations": ov["iters"], "correct": okv, "max_eig_err": errv,
               "max_residual": resv,
               "phase_ms": {k: round(v, 2) for k, v in f.timings().items()},
               "eigensolves": {"ms": round(eig["ms"], 2), "sweeps": eig["launches"],
                               "calls": int(eig["dense_flops"])},
               "speedup_vs_feast": round((total / args.steps) / tv, 3)}
        variants.append(rec)
        log(f"[bench] variant {rec}")
    f.close()

    cpu = None
    if not args.no_cpu_baseline:
        from paper_1605_08771_amd import gen  # noqa: F401
        import oracle
        z, _ = oracle.contour(p.emin, p.emax, p.n_c)
        cpu = cpu_baseline(p, int(np.median(iters)), z)
        log(f"[bench] cpu baseline: {cpu}")

    traffic = None
    if (args.workload == "c2" and p.n == 8192 and prec == fm.FEAST_FP64
            and kernel_sources_hash() == SWEEP_TRAFFIC["sources"]):
        traffic = SWEEP_TRAFFIC["bytes_per_launch"]

    line = {
        "metric": METRIC,
        "value": round(total / args.steps, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64" if prec == fm.FEAST_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"{p.name}: complex Hermitian n={p.n}, {p.m_true} eigenvalues in "
                        f"I=({p.emin},{p.emax}) with edge clusters within 1e-3, m0={p.m0}, "
                        f"n_c={p.n_c}, {prec_name}, stop at res<=1e-10*||A||",
            "n": p.n, "m0": p.m0, "n_c": p.n_c, "precision": prec_name, "tol": 1e-10,
        },
        "roofline": {
            "kernel": f"{SWEEP_KERNEL[prec]} in the block triangular sweeps (Y and adjoint Y')",
            "bound": "mfma",
            "achieved": round(achieved, 2),
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": traffic,
            "traffic_unit": "bytes/launch",
            "launches": solve["launches"],
            "avg_launch_ms": round(solve["ms"] / max(1, solve["launches"]), 5),
            "algorithmic_flops_per_launch": alg_solve / max(1, solve["launches"]),
            "algorithmic_bytes_per_launch": alg_solve_bytes / max(1, solve["launches"]),
            "filter_applications": n_filters,
        },
        "filter_apply_tflops": round(filter_tflops, 2),
        "iterations": iters,
        "step_times_s": [round(x, 4) for x in step_s],
        "step_time_median_s": round(float(np.median(step_s)), 4),
        "step_time_min_s": round(float(np.min(step_s)), 4),
        "correct": all(c[0] for c in checks),
        "max_eig_err": max(c[1] for c in checks),
        "max_residual": max(c[2] for c in checks),
        "time_to_tol_1e-12_s": round(warm.get("time_s", float("nan")), 4),
        "iters_to_tol_1e-12": warm.get("iters"),
        "phase_ms_last_step": {k: round(v, 2) for k, v in phases[-1].items()},
        "lu_gemm_tflops": round(lu["dense_flops"] / (lu["ms"] * 1e-3) / 1e12, 2) if lu["ms"] else None,
        "rr_gemm_ms": round(rr["ms"], 2),
        "eigensolves": {"ms": round(eig_main["ms"], 2), "sweeps": eig_main["launches"],
                        "calls": int(eig_main["dense_flops"])},
        "other_precision": compare,
        "more_precisions": compares[1:],
        "variants": variants,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
