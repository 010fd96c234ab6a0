"""Benchmark of the MI355X FEAST hot path (one GPU).

One step = one complete FEAST solve (factorizations of the n_c shifted matrices, the filter
application Q = rho(A) X with its triangular solves and accumulation, Rayleigh-Ritz and the
residual test, iterated to convergence) on one synthetic problem resident in HBM.  The factor
cache is dropped before every step, so each step refactors.

Default workload: the largest single-GPU configuration, complex Hermitian A = U diag(lam) U^H
with n = 32768, 512 eigenvalues in I = (-0.05, 0.05) of which 64 lie within 1e-3 inside each
endpoint, the rest uniform on [-1, 1]; m0 = 768, n_c = 8; FP32 factors and solves with FP64
refinement (the timed value), and the plain FP64 path once on the same input and threshold
for comparison.  Timed steps stop at max residual <= 1e-10 ||A|| (the metric's threshold); the
first warm-up step runs to 1e-12 and reports its time.  Every solve is checked against the
exact eigenvalues of the construction.

Other workloads (--workload): c1 (real symmetric n = 500, plain FEAST), c2 (the n = 8192 hard
case in FP64, with the Sec. 2 variants beside it), c3 (n = 16384 mixed, with the bf16x3
variant), c4 (64 independent problems of uneven size).

Prints one JSON line (see --help for options).
"""
from __future__ import annotations

import argparse
import json
import math
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
PRECS = {"fp64": 0, "fp32ir": 1, "bf16x3ir": 2}
DEFAULT_PREC = {"c1": "fp64", "c2": "fp64", "c3": "fp32ir", "c4": "fp32ir", "c5": "fp32ir"}

# HBM bytes per launch of the paired sweep GEMM, from rocprofv3 FETCH_SIZE and WRITE_SIZE runs
# over the solver's sweep launches at the workload's order, block and node count (the sweeps
# microbenchmark) scaled by a plain copy of known size, keyed by (workload, precision); valid
# only while the sources of that kernel (gemm.hip), of its launches (solve.hip), of the block
# height table (sweep_tune.h) and their common header hash to the version the counters were
# taken on.
SWEEP_TRAFFIC = {
    ("c2", "fp64"): {"sources": "f3d143e28158b223", "bytes_per_launch": 1.286e9},
    ("c5", "fp32ir"): {"sources": "f3d143e28158b223", "bytes_per_launch": 3.677e9},
}


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("gemm.hip", "solve.hip", "sweep_tune.h", "common.h"):
        with open(os.path.join(ROOT, "paper_1605_08771_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"model": model, "nproc": os.cpu_count(), "usable": usable}


def make_problem(args, dev):
    from paper_1605_08771_amd import gen
    t0 = time.time()
    if args.workload == "c1":
        p = gen.config1(n=args.n or 500, device=dev)
    elif args.workload == "c2":
        p = gen.config2(n=args.n or 8192, device=dev, basis=args.basis)
    elif args.workload == "c3":
        p = gen.config3(n=args.n or 16384, device=dev)
    elif args.workload == "c5":
        p = gen.config5(n=args.n or 32768, device=dev, basis=args.basis)
    else:
        raise SystemExit(f"unknown workload {args.workload}")
    log(f"[bench] generated {p.name} n={p.n} m0={p.m0} n_c={p.n_c} m_true={p.m_true} "
        f"in {time.time() - t0:.1f}s")
    return p


# ---------------------------------------------------------------------------------------------
# CPU baseline: the oracle's cost per term, measured on small samples and extrapolated.
# ---------------------------------------------------------------------------------------------
def oracle_cost_model(A_block, X_block, z0, m0):
    """Time the oracle (single-threaded) on samples cut from the workload's own A and X0 and
    fit each term by its own exponent:
      LU of one shifted matrix          t_lu(ns) * (n / ns)^3
      solve pair (Y and adjoint Y')     t_solve(ns, ms) * (n / ns)^2 * (m0 / ms)
      Rayleigh-Ritz                     a n^2 m0 + b n m0^2 + c m0^3 (the n^2 m0 products A X,
                                        the n m0^2 Gram and basis products, the m0^3 reduced
                                        products and the two Jacobi eigensolves), a, b, c >= 0
                                        from a least-squares fit to four (ns, ms) samples.
    A_block: the leading square block of A (numpy, complex or real); X_block its rows of X0."""
    import oracle
    from scipy.optimize import nnls
    threads_before = oracle.num_threads()
    oracle.set_num_threads(1)
    is_c = np.iscomplexobj(A_block)
    dt = "c128" if is_c else "r64"
    Ac = A_block.astype(np.complex128)
    ns = min(1024, A_block.shape[0])
    M = z0 * np.eye(ns) - Ac[:ns, :ns]
    t0 = time.perf_counter()
    LU, piv, _ = oracle.zlu(M)
    t_lu = time.perf_counter() - t0
    ms = max(1, min(m0, X_block.shape[1], 256))
    B = np.asfortranarray(X_block[:ns, :ms].astype(np.complex128))
    t0 = time.perf_counter()
    oracle.zlu_solve(LU, piv, B)
    if is_c:
        oracle.zlu_solve(LU, piv, B, adjoint=True)
    t_solve = time.perf_counter() - t0
    pts, rows, ts = [], [], []
    nmax = A_block.shape[0]
    for (nr, mr) in ((nmax // 2, 48), (nmax, 48), (nmax // 2, 128), (3 * nmax // 4, 96)):
        mr = max(1, min(mr, nr, X_block.shape[1]))
        As = np.asfortranarray(A_block[:nr, :nr])
        Q = np.asfortranarray(X_block[:nr, :mr])
        t0 = time.perf_counter()
        oracle.rayleigh_ritz(dt, As, Q, -0.05, 0.05, 1.0)
        ts.append(time.perf_counter() - t0)
        rows.append([nr * nr * mr, nr * mr * mr, mr ** 3])
        pts.append((nr, mr))
    R = np.array(rows, dtype=float)
    scale = R.max(axis=0)
    coef, _ = nnls(R / scale, np.array(ts))
    coef = coef / scale
    oracle.set_num_threads(threads_before)
    return dict(ns=ns, t_lu=t_lu, ms=ms, t_solve=t_solve, rr_coef=[float(c) for c in coef],
                rr_samples=[(int(a), int(b), round(t, 3)) for (a, b), t in zip(pts, ts)],
                sample_s=t_lu + t_solve + sum(ts))


def oracle_estimate(cm, n, m0, n_c, iters, n_filters, threads):
    """Single-thread and node-parallel oracle time of one solve from the cost model."""
    lu = cm["t_lu"] * (n / cm["ns"]) ** 3
    solve = cm["t_solve"] * (n / cm["ns"]) ** 2 * (m0 / cm["ms"])
    a, b, c = cm["rr_coef"]
    rr = a * n * n * m0 + b * n * m0 * m0 + c * m0 ** 3
    per_node = lu + n_filters * solve
    single = n_c * per_node + iters * rr
    par = math.ceil(n_c / max(1, threads)) * per_node + iters * rr
    return dict(single_thread_s=single, node_parallel_s=par,
                terms_s={"lu_per_node": lu, "solve_pair_per_node_per_filter": solve,
                         "rayleigh_ritz_per_iteration": rr,
                         "rr_n2m0": a * n * n * m0, "rr_nm0^2": b * n * m0 * m0,
                         "rr_m0^3": c * m0 ** 3})


def cpu_baseline_single(p, iters, n_filters):
    import oracle
    z, _ = oracle.contour(p.emin, p.emax, p.n_c)
    nb = min(1024, p.n)
    Ab = p.A[:nb, :nb]
    Ab = Ab.cpu().numpy() if hasattr(Ab, "cpu") else np.asarray(Ab)
    Xb = p.X0[:nb, :]
    Xb = Xb.cpu().numpy() if hasattr(Xb, "cpu") else np.asarray(Xb)
    cm = oracle_cost_model(Ab, Xb, z[0], p.m0)
    threads = max(1, min(p.n_c, oracle.num_threads()))
    est = oracle_estimate(cm, p.n, p.m0, p.n_c, iters, n_filters, threads)
    info = cpu_info()
    sample = (f"oracle, single-threaded, on samples of this workload's A and X0: LU of one "
              f"{cm['ns']}x{cm['ns']} shifted block {cm['t_lu']:.2f}s, a {cm['ms']}-column "
              f"solve pair {cm['t_solve']:.2f}s, Rayleigh-Ritz at (n, m) = "
              f"{[s[:2] for s in cm['rr_samples']]} in {[s[2] for s in cm['rr_samples']]}s; "
              f"each term extrapolated by its own exponent (LU n^3; solves n^2 m0; "
              f"Rayleigh-Ritz a n^2 m0 + b n m0^2 + c m0^3 fitted) to n={p.n}, m0={p.m0}, "
              f"n_c={p.n_c}, {iters} iterations and {n_filters} filter applications; nodes run "
              f"in parallel on {threads} threads (the oracle parallelises over nodes only)")
    return dict(value=round(est["node_parallel_s"], 1), unit="s", cores=threads,
                kind="oracle", sample=sample, extrapolated=True,
                single_thread_s=round(est["single_thread_s"], 1),
                terms_s={k: round(v, 3) for k, v in est["terms_s"].items()},
                sample_s=round(cm["sample_s"], 2), cpu=info)


def cpu_baseline_c1(p):
    """Config 1 is small enough for the whole oracle solve (no extrapolation)."""
    import oracle
    threads = max(1, min(p.n_c, oracle.num_threads()))
    t0 = time.perf_counter()
    ref = oracle.feast_solve("r64", p.A, p.emin, p.emax, p.n_c, p.m0, 1e-10, p.max_iter,
                             p.anorm, p.X0)
    dt = time.perf_counter() - t0
    return dict(value=round(dt, 3), unit="s", cores=threads, kind="oracle",
                sample=f"the whole oracle solve of this workload to 1e-10 ({ref['iters']} "
                       f"iterations, status {ref['status']}), nodes on {threads} threads",
                extrapolated=False, cpu=cpu_info())


# ---------------------------------------------------------------------------------------------
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
    prec_name = args.prec or DEFAULT_PREC["c4"]
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
            good = o["status"] == 0 and o["m"] == p.m_true
            ok &= good
            if good:
                ex = np.sort(p.lam[(p.lam > p.emin) & (p.lam < p.emax)])
                lam_in = np.sort(o["lam"][o["counted"]])
                errs.append(float(np.max(np.abs(lam_in - ex))))
        return ok, (max(errs) if errs else float("nan"))

    for w in range(args.warmup):
        torch.cuda.synchronize()
        one(args.nstreams)
        torch.cuda.synchronize()
        log(f"[bench] warmup {w} done")
    f.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results, step_s = [], []
    for k in range(args.steps):
        ts = time.perf_counter()
        results.append(one(args.nstreams))
        step_s.append(time.perf_counter() - ts)
        log(f"[bench] step {k}: {step_s[-1]:.3f}s")
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    lu_st, solve_st = f.kernel_stats("lu"), f.kernel_stats("solve")
    f.set_profiling(False)
    bad, outs = results[-1]
    ok, err = check(outs)
    iters = [o["iters"] for o in outs]
    log(f"[bench] c4: bad={bad} ok={ok} max|dlam|={err:.2e} iters min/med/max "
        f"{min(iters)}/{int(np.median(iters))}/{max(iters)} time/step {total / args.steps:.3f}s")
    # whole-step rate: algorithmic LU and sweep flops of all problems per step over the step's
    # wall-clock time (the problems overlap on 8 streams, so per-launch durations would count
    # the same time several times)
    alg = sum(8 * (8.0 / 3.0) * p.n ** 3 + o["filter_columns"] * 8 * 2 * 8.0 * p.n * p.n
              for p, o in zip(probs, outs))
    peak = PEAKS[prec]
    step_mean = total / args.steps
    per_problem = sorted(
        ({"n": p.n, "m0": p.m0, "m": o["m"], "iters": o["iters"], "status": o["status"],
          "ms": round(o["time_ms"], 2)} for p, o in zip(probs, outs)),
        key=lambda r: -r["ms"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    one(1)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t1
    f.close()
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        # the cost model on the largest problem's own matrix, summed over all 64 problems
        big = max(probs, key=lambda q: q.n)
        z, _ = oracle.contour(big.emin, big.emax, 8)
        nb = min(1024, big.n)
        cm = oracle_cost_model(big.A[:nb, :nb].cpu().numpy(), big.X0[:nb, :].cpu().numpy(), z[0],
                               big.m0)
        threads = max(1, min(8, oracle.num_threads()))
        ests = [oracle_estimate(cm, p.n, p.m0, 8, o["iters"], o["iters"] + 1, threads)
                for p, o in zip(probs, outs)]
        cpu = dict(value=round(sum(e["node_parallel_s"] for e in ests), 1), unit="s",
                   cores=threads, kind="oracle", extrapolated=True,
                   single_thread_s=round(sum(e["single_thread_s"] for e in ests), 1),
                   sample=f"oracle cost model (single-threaded samples of the largest problem, "
                          f"n={big.n}: LU {cm['t_lu']:.2f}s at {cm['ns']}, solve pair "
                          f"{cm['t_solve']:.2f}s with {cm['ms']} columns, Rayleigh-Ritz fitted "
                          f"to {cm['rr_samples']}) summed over the 64 problems with their GPU "
                          f"iteration counts; problems one after another, nodes in parallel "
                          f"on {threads} threads", cpu=cpu_info())
        log(f"[bench] cpu baseline: {cpu}")
    line = {
        "metric": METRIC, "value": round(step_mean, 4), "unit": "s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1000 * step_mean, 2), "higher_is_better": False,
        "scaling": "strong", "vs_baseline": None,
        "dtype": "f64" if prec == fm.FEAST_FP64 else "f32+f64", "data": "synthetic",
        "config": {"workload": f"C4: 64 complex Hermitian problems, n~U{{256..4096}} "
                               f"(sum n^2={sum(p.n * p.n for p in probs)}), own intervals with "
                               f"~8% of the spectrum and edge clusters, m0=ceil(1.5m), n_c=8, "
                               f"{prec_name}, {args.nstreams} streams, stop at res<=1e-10*||A||",
                   "problems": len(probs), "precision": prec_name, "nstreams": args.nstreams},
        "roofline": {"kernel": "all LU trailing updates and triangular sweeps of the step "
                               "(whole-step rate; problems overlap on concurrent streams)",
                     "bound": "mfma",
                     "achieved": round(alg / step_mean / 1e12, 2),
                     "peak": peak, "unit": "TFLOP/s",
                     "frac": round(alg / step_mean / 1e12 / peak, 4),
                     "traffic": None,
                     "lu_kernel_ms": round(lu_st["ms"] / args.steps, 1),
                     "sweep_kernel_ms": round(solve_st["ms"] / args.steps, 1)},
        "correct": ok and bad == 0, "max_eig_err": err,
        "iterations_min_median_max": [min(iters), int(np.median(iters)), max(iters)],
        "step_times_s": [round(x, 4) for x in step_s],
        "sequential_one_stream_s": round(t_seq, 4),
        "slowest_problems": per_problem[:8],
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--nstreams", type=int, default=8, help="c4: concurrent worker streams")
    ap.add_argument("--n", type=int, default=0, help="override n (tests only)")
    ap.add_argument("--prec", default="", choices=["", *PRECS])
    ap.add_argument("--compare", default=None,
                    help="comma-separated precisions run once after the timed steps on the same "
                         "input and threshold (default: the other of fp64/fp32ir; c3 adds "
                         "bf16x3ir, the split-precision factorization)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the runs in the other precisions")
    ap.add_argument("--basis", default="haar", choices=["haar", "householder"],
                    help="c2/c5 eigenvectors: QR of a Gaussian matrix (default) or 8 dense "
                         "reflectors built without library factorizations (for counter runs)")
    ap.add_argument("--variants", default=None,
                    help="comma list of method:s[:precision] runs of the Sec. 2 variants "
                         "reported beside FEAST (default for c2: rfeast:3,xfeast:2,xfeast:3,"
                         "xfeast:2:fp32ir; '' = none)")
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
    prec_name = args.prec or DEFAULT_PREC[args.workload]
    prec = PRECS[prec_name]
    real = args.workload == "c1"
    # config 1 is plain FEAST (the paper's step 3); the others apply the filter-value test
    spurious = not real
    A = p.A
    X0 = p.X0
    f = fm.Feast()
    exact_in = np.sort(p.lam[(p.lam > p.emin) & (p.lam < p.emax)])

    def one(tol, max_iter=p.max_iter, pr=None, method="feast", expand=1):
        f.invalidate()
        out = f.solve(A, p.emin, p.emax, p.m0, n_c=p.n_c, tol=tol, max_iter=max_iter,
                      anorm=p.anorm, X0=X0, prec=prec if pr is None else pr,
                      spurious=spurious, refine_max=0, method=method, expand=expand)
        return out

    def check(out):
        sel = out["counted"]
        ok = out["status"] == 0 and out["m"] == p.m_true and len(sel) == p.m_true
        err = float(np.max(np.abs(np.sort(out["lam"][sel]) - exact_in))) if ok else float("nan")
        res = float(np.max(out["res"][sel])) if len(sel) else float("nan")
        return ok, err, res

    warm = {}
    for w in range(args.warmup):
        # the first warm-up step runs to the configuration's own tolerance
        tol_w = p.tol if w == 0 else 1e-10
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = one(tol_w)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ok, err, res = check(out)
        if w == 0:
            warm = dict(time_s=dt, iters=out["iters"], ok=ok, eig_err=err, res=res,
                        status=out["status"], tol=tol_w)
        log(f"[bench] warmup {w} (tol {tol_w:g}): status={out['status']} iters={out['iters']} "
            f"m={out['m']} time={dt:.3f}s max|dlam|={err:.2e} max res={res:.2e}")

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
        log(f"[bench] step {k}: {step_s[-1]:.3f}s iters={out['iters']} status={out['status']}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ms_per_step = 1000.0 * total / args.steps
    iters = [o["iters"] for o in outs]
    nfilt = [o["filter_applications"] for o in outs]
    ncols = [o["filter_columns"] for o in outs]
    checks = [check(o) for o in outs]
    for k, (o, c) in enumerate(zip(outs, checks)):
        log(f"[bench] step {k}: m={o['m']} max|dlam|={c[1]:.2e} max res={c[2]:.2e} "
            f"phases={phases[k]}")
    solve = f.kernel_stats("solve")
    lu = f.kernel_stats("lu")
    rr = f.kernel_stats("rr")
    eig_main = f.kernel_stats("eig")
    sides = 1 if real else 2
    n_filters = sum(nfilt)
    # right-hand-side columns filtered: m0 per application, fewer when the last application
    # only served the filter-value test of the Ritz pairs inside I
    n_cols = sum(ncols)
    alg_solve = n_cols * p.n_c * sides * 8.0 * p.n * p.n
    # algorithmic HBM bytes of the sweeps: each factor read once per sweep (forward and
    # backward; the two sides read complementary triangles) and each right-hand-side block
    # read and written once per sweep
    eb = 16.0 if prec == fm.FEAST_FP64 else 8.0
    alg_solve_bytes = (n_filters * p.n_c * 2 * eb * p.n * p.n
                       + n_cols * p.n_c * 2 * sides * 2 * eb * p.n)
    achieved = alg_solve / (solve["ms"] * 1e-3) / 1e12 if solve["ms"] > 0 else 0.0
    peak = PEAKS[prec]
    filt_ms = sum(ph["solve_ms"] + ph["accumulate_ms"] for ph in phases)
    alg_filter = alg_solve + n_cols * p.n_c * sides * 8.0 * p.n
    filter_tflops = alg_filter / (filt_ms * 1e-3) / 1e12 if filt_ms > 0 else 0.0
    f.set_profiling(False)

    # other precisions on the same input, to the same threshold (mixed vs FP64), run once
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
        f.set_profiling(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o2 = one(1e-10, pr=other)
        torch.cuda.synchronize()
        t_other = time.perf_counter() - t0
        lu2, solve2 = f.kernel_stats("lu"), f.kernel_stats("solve")
        f.set_profiling(False)
        ok2, err2, res2 = check(o2)
        rec = {"precision": other_name, "time_s": round(t_other, 4), "iterations": o2["iters"],
               "correct": ok2, "max_eig_err": err2, "max_residual": res2,
               "phase_ms": {k: round(v, 2) for k, v in f.timings().items()},
               "lu_gemm_ms": round(lu2["ms"], 2), "solve_gemm_ms": round(solve2["ms"], 2),
               "sweep_tflops": round(o2["filter_columns"] * p.n_c * sides * 8.0 * p.n *
                                     p.n / (solve2["ms"] * 1e-3) / 1e12, 2)
               if solve2["ms"] else None,
               "time_over_value": round(t_other / (total / args.steps), 3),
               "note": "one run, no separate warm-up (includes the first use of its buffers)"}
        compares.append(rec)
        log(f"[bench] {other_name}: {rec}")
    compare = compares[0] if compares else None
    # the expanded-subspace variants of Sec. 2 on the same input and threshold
    variants = []
    vspec = args.variants
    if vspec is None:
        vspec = "rfeast:3,xfeast:2,xfeast:3,xfeast:2:fp32ir" if args.workload == "c2" else ""
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
        okv, errv, resv = check(ov)
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
        if real:
            A_h = p.A.cpu().numpy() if hasattr(p.A, "cpu") else p.A
            X_h = p.X0.cpu().numpy() if hasattr(p.X0, "cpu") else p.X0
            q = type(p)(**{**p.__dict__, "A": np.asfortranarray(A_h),
                           "X0": np.asfortranarray(X_h)})
            cpu = cpu_baseline_c1(q)
        else:
            cpu = cpu_baseline_single(p, int(np.median(iters)), int(np.median(nfilt)))
        log(f"[bench] cpu baseline: {cpu}")

    traffic = None
    tr = SWEEP_TRAFFIC.get((args.workload, prec_name))
    if tr and p.n == {"c2": 8192, "c5": 32768}.get(args.workload) \
            and kernel_sources_hash() == tr["sources"]:
        traffic = tr["bytes_per_launch"]

    kind = "real symmetric" if real else "complex Hermitian"
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
        "dtype": "f64" if prec == fm.FEAST_FP64 else ("f32+f64" if prec == 1 else "bf16x3+f64"),
        "data": "synthetic",
        "config": {
            "workload": f"{p.name}: {kind} n={p.n}, {p.m_true} eigenvalues in "
                        f"I=({p.emin},{p.emax})"
                        + ("" if real else " with edge clusters within 1e-3")
                        + f", m0={p.m0}, n_c={p.n_c}, {prec_name}, stop at res<=1e-10*||A||",
            "n": p.n, "m0": p.m0, "n_c": p.n_c, "precision": prec_name, "tol": 1e-10,
        },
        "roofline": {
            "kernel": f"{SWEEP_KERNEL[prec]} in the block triangular sweeps"
                      + ("" if real else " (Y and adjoint Y')"),
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
            "filter_columns": n_cols,
        },
        "filter_apply_tflops": round(filter_tflops, 2),
        "iterations": iters,
        "step_times_s": [round(x, 4) for x in step_s],
        "step_time_median_s": round(float(np.median(step_s)), 4),
        "step_time_min_s": round(float(np.min(step_s)), 4),
        "correct": all(c[0] for c in checks),
        "max_eig_err": max(c[1] for c in checks),
        "max_residual": max(c[2] for c in checks),
        "time_to_own_tol_s": round(warm.get("time_s", float("nan")), 4),
        "own_tol": p.tol,
        "iters_to_own_tol": warm.get("iters"),
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
