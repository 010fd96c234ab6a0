"""Measure the sweep block height per precision class and order on this device, and write the
table the library builds in (csrc/sweep_tune.h; rebuild afterwards).

    python -m paper_1605_08771_amd.autotune [--reps 3] [--out PATH] [--report PATH]

The sweep block height nbt sets the rows of each block step of the triangular sweeps and of
the diagonal blocks inverted once per factorization; the factors are padded to a multiple of
it.  Taller blocks mean fewer, larger launches but more padding and more work in the
triangular products.  For each precision class (FP64 factors; FP32 factors with FP64
refinement) and each order n in SIZES, PROBLEMS synthetic problems of the batched workload's
kind (complex Hermitian, an interval holding 8 % of the spectrum with clusters at both ends,
centre and width drawn as in that workload, m0 = 1.5 m, 8 nodes) are solved to 1e-10 ||A||
with every candidate height (64, 128, 256, 512: the FP64 residual floor rules out taller
blocks) whose padding adds at most n / 8 rows (the library demotes taller ones); the height
with the smallest sum over the problems of the median time of `reps` timed solves (after one
untimed solve) among those that converge on every problem is kept.  Several problems per
order keep a problem whose residual sits near the threshold (one iteration more or less)
from deciding alone.  Each order's choice holds from the midpoint below it to the midpoint
above it; orders past the last size take 512, the height the n >= 8192 configurations were
validated with (their FP64 residual floor allows no taller block).
"""
from __future__ import annotations

import argparse
import math
import os
import statistics
import sys
import time

SIZES = (256, 384, 512, 768, 1024, 1536, 2048, 3072, 4096, 6144)
PROBLEMS = 3
CANDIDATES = (64, 128, 256, 512)
CLASSES = ((0, "FP64", 0), (1, "FP32+IR", 1))  # (class, name, solver precision code)

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "csrc", "sweep_tune.h")


def problems(n, count, device):
    from paper_1605_08771_amd import gen
    rng = gen.rng_for([7, n])
    m = int(round(0.08 * n))
    out = []
    for q in range(count):
        c, h = rng.uniform(-0.5, 0.5), rng.uniform(0.02, 0.1)
        spec = dict(n=n, emin=float(c - h), emax=float(c + h), m=m, m0=int(math.ceil(1.5 * m)),
                    tag=[7, n, q + 1])
        out.append(gen.config4_problem(spec, device=device))
    return out


def padding_ok(n, nbt):
    """The library demotes a height whose padding would add more than n / 8 rows."""
    return nbt == 64 or 8 * (-(-n // nbt) * nbt - n) <= n


def measure(f, p, prec, nbt, reps):
    import torch
    import paper_1605_08771_amd as fm
    fm.tune_sweep_block(nbt)
    times, out = [], None
    try:
        for r in range(reps + 1):
            f.invalidate()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = f.solve(p.A, p.emin, p.emax, p.m0, n_c=8, tol=1e-10, max_iter=200, prec=prec,
                          X0=p.X0, spurious=True, anorm=p.anorm, refine_max=0)
            torch.cuda.synchronize()
            if r > 0:
                times.append(time.perf_counter() - t0)
    finally:
        fm.tune_sweep_block(0)
    ok = out["status"] == 0 and out["m"] == p.m_true
    return statistics.median(times), out["iters"], ok


def rows_from(choice):
    """[(n, nbt)] ascending -> [(n_max, nbt)] with each order's choice up to the midpoint to
    the next order, equal neighbours merged."""
    rows = []
    for i, (n, nbt) in enumerate(choice):
        n_max = (n + choice[i + 1][0]) // 2 - 1 if i + 1 < len(choice) else n
        if rows and rows[-1][1] == nbt:
            rows[-1] = (n_max, nbt)
        else:
            rows.append((n_max, nbt))
    return rows


def header(table, device_name, reps):
    lines = [
        "// Sweep block heights (rows of the block triangular sweeps and of the inverted diagonal",
        "// blocks) per precision class of the factors (0: FP64, 1: FP32) and order n, measured on",
        f"// {device_name} by `python -m paper_1605_08771_amd.autotune --reps {reps}`: for each",
        "// order, the fastest converging height of 64, 128, 256 and 512 over whole solves of",
        f"// {PROBLEMS} synthetic problems of the batched workload's kind.  Orders past the last row",
        "// use 512.",
        "#pragma once",
        "",
        "namespace feast {",
        "",
        "struct SweepTuneRow {",
        "  int prec_class;",
        "  int n_max;",
        "  int nbt;",
        "};",
        "",
        "static const SweepTuneRow kSweepTune[] = {",
    ]
    for cls, rows in table:
        lines.append("    " + " ".join(f"{{{cls}, {n_max}, {nbt}}}," for n_max, nbt in rows))
    lines += ["};", "", "}  // namespace feast", ""]
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--report", default=None, help="also write the measurements (markdown)")
    ap.add_argument("--sizes", type=int, nargs="*", default=list(SIZES))
    a = ap.parse_args(argv)
    import torch
    import paper_1605_08771_amd as fm
    dev = "cuda:0"
    f = fm.Feast()
    # cells: summed median times over the problems, summed iteration counts
    report = ["| precision | n | m0 | " + " | ".join(f"nbt {c} (s, it.)" for c in CANDIDATES)
              + " | chosen |", "|---|---:|---:|" + "---:|" * len(CANDIDATES) + "---:|"]
    table = []
    probs = {}
    for cls, name, prec in CLASSES:
        choice = []
        for n in sorted(a.sizes):
            if n not in probs:
                probs[n] = problems(n, PROBLEMS, dev)
            res = {}
            for c in (c for c in CANDIDATES if padding_ok(n, c)):
                runs = [measure(f, p, prec, c, a.reps) for p in probs[n]]
                res[c] = (sum(r[0] for r in runs), sum(r[1] for r in runs), all(r[2] for r in runs))
            good = [c for c in res if res[c][2]]
            best = min(good, key=lambda c: res[c][0]) if good else 64
            choice.append((n, best))
            cells = " | ".join(("padding" if c not in res else
                                f"{res[c][0]:.4f}, {res[c][1]}" + ("" if res[c][2] else " (no)"))
                               for c in CANDIDATES)
            report.append(f"| {name} | {n} | {probs[n][0].m0} | {cells} | {best} |")
            print(report[-1], flush=True)
        table.append((cls, rows_from(choice)))
    f.close()
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", "").split(":")[0]
    text = header(table, f"{props.name} ({arch})" if arch else props.name, a.reps)
    with open(a.out, "w") as fh:
        fh.write(text)
    print(f"wrote {a.out}", flush=True)
    if a.report:
        with open(a.report, "w") as fh:
            fh.write("\n".join(report) + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
