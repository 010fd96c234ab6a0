"""Kernel-level microbenchmarks of the library's building blocks, for timing and counter runs.

    python -m paper_1605_08771_amd.microbench gemm --prec fp64 --shape 61440 300 512 --reps 4
    python -m paper_1605_08771_amd.microbench jacobi --m 300 --kind random --reps 3

`gemm` runs C = -op(A) op(B) + C through `feast_kern_gemm` (prec fp64, fp32 or bf16x3) on
seeded Gaussian operands (one untimed call first, then `reps` timed ones; a counter run sees
reps + 1 dispatches); `jacobi` runs `feast_kern_jacobi` on a seeded Hermitian matrix
(random, or a Gram matrix with eigenvalues from 1 to 1e-16).  Each prints one line with the
average time per call measured with HIP events on the library's stream.
"""
from __future__ import annotations

import argparse
import sys


def _gemm(a):
    import torch
    import paper_1605_08771_amd as fm
    dt = torch.complex128 if a.prec == "fp64" else torch.complex64
    M, N, K = a.shape
    g = torch.Generator(device="cuda").manual_seed(a.seed)

    def rnd(r, c):
        return fm.fortran(torch.randn(r, c, dtype=dt, device="cuda", generator=g))

    A = rnd(M, K) if a.opA == 0 else rnd(K, M)
    B = rnd(K, N) if a.opB == 0 else rnd(N, K)
    C = rnd(M, N)
    f = fm.Feast()
    s = f._stream
    split = a.prec == "bf16x3"
    if f.gemm(a.opA, a.opB, A, B, C, -1.0, 1.0, M=M, N=N, K=K, split_bf16=split) != 0:
        raise SystemExit("feast_kern_gemm failed")  # warm-up call (code load), not timed
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(s):
        e0.record()
        for _ in range(a.reps):
            st = f.gemm(a.opA, a.opB, A, B, C, -1.0, 1.0, M=M, N=N, K=K, split_bf16=split)
            if st != 0:
                raise SystemExit(f"feast_kern_gemm returned {st}")
        e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / a.reps
    print(f"gemm {a.prec} opA={a.opA} opB={a.opB} M={M} N={N} K={K}: {ms * 1e3:.1f} us/call, "
          f"{8.0 * M * N * K / (ms * 1e-3) / 1e12:.2f} TFLOP/s", flush=True)
    f.close()


def _jacobi(a):
    import numpy as np
    import torch
    import paper_1605_08771_amd as fm
    rng = np.random.default_rng(a.seed)
    m = a.m
    X = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    if a.kind == "random":
        H = X + X.conj().T
    else:
        Q, _ = np.linalg.qr(X)
        H = (Q * np.logspace(0, -16, m)) @ Q.conj().T
        H = 0.5 * (H + H.conj().T)
    Ht = torch.from_numpy(np.ascontiguousarray(H)).cuda()
    f = fm.Feast()
    times, sweeps = [], []
    for _ in range(a.reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sw, d, W = f.jacobi(Ht)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
        sweeps.append(sw)
    print(f"jacobi m={m} {a.kind}: {min(times):.2f} ms/call (min of {a.reps}), sweeps {sweeps[-1]}",
          flush=True)
    f.close()


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="what", required=True)
    g = sub.add_parser("gemm")
    g.add_argument("--prec", choices=["fp64", "fp32", "bf16x3"], default="fp64")
    g.add_argument("--shape", type=int, nargs=3, metavar=("M", "N", "K"), required=True)
    g.add_argument("--opA", type=int, default=0, choices=[0, 1, 2])
    g.add_argument("--opB", type=int, default=0, choices=[0, 1, 2])
    g.add_argument("--reps", type=int, default=4)
    g.add_argument("--seed", type=int, default=0)
    j = sub.add_parser("jacobi")
    j.add_argument("--m", type=int, required=True)
    j.add_argument("--kind", choices=["random", "gram"], default="random")
    j.add_argument("--reps", type=int, default=3)
    j.add_argument("--seed", type=int, default=0)
    a = ap.parse_args(argv)
    (_gemm if a.what == "gemm" else _jacobi)(a)


if __name__ == "__main__":
    sys.exit(main())
