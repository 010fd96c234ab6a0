"""Kernel-level microbenchmarks of the library's building blocks, for timing and counter runs.

    python -m paper_1605_08771_amd.microbench gemm --prec fp64 --shape 61440 300 512 --reps 4
    python -m paper_1605_08771_amd.microbench jacobi --m 300 --kind random --reps 3
    python -m paper_1605_08771_amd.microbench filter --n 32768 --m0 768 --prec fp32ir
    python -m paper_1605_08771_amd.microbench sweeps --n 32768 --m0 768 --prec fp32

`gemm` runs C = -op(A) op(B) + C through `feast_kern_gemm` (prec fp64, fp64x3 (three real
FP64 products per complex one), fp32 or bf16x3) on
seeded Gaussian operands (one untimed call first, then `rounds` rounds of `reps` timed ones,
the fastest round reported; a counter run with one round sees reps + 1 dispatches); with
`--vendor` it also times the same product through torch.addmm (the ROCm BLAS libraries, fp64
and fp32 only), alternating the two from round to round; `jacobi` runs `feast_kern_jacobi` on a seeded Hermitian matrix
(random, or a Gram matrix with eigenvalues from 1 to 1e-16).  Each prints one line with the
average time per call measured with HIP events on the library's stream.
"""
from __future__ import annotations

import argparse
import sys


def _gemm(a):
    import torch
    import paper_1605_08771_amd as fm
    dt = torch.complex128 if a.prec in ("fp64", "fp64x3") else torch.complex64
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

    def ours():
        st = f.gemm(a.opA, a.opB, A, B, C, -1.0, 1.0, M=M, N=N, K=K, split_bf16=split,
                    three_products=a.prec == "fp64x3")
        if st != 0:
            raise SystemExit(f"feast_kern_gemm returned {st}")

    def op(X, o):
        return X if o == 0 else (X.mT if o == 1 else X.mH)

    D = C.clone() if a.vendor and not split else None

    def vendor():
        torch.addmm(C, op(A, a.opA), op(B, a.opB), beta=1.0, alpha=-1.0, out=D)

    runs = [("gemm", ours)] + ([("vendor torch.addmm", vendor)] if D is not None else [])
    best = {}
    with torch.cuda.stream(s):
        for _, fn in runs:
            fn()  # warm-up call (code load), not timed
        for r in range(a.rounds):
            for name, fn in (runs if r % 2 == 0 else runs[::-1]):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(a.reps):
                    fn()
                e1.record()
                e1.synchronize()
                best[name] = min(best.get(name, 1e30), e0.elapsed_time(e1) / a.reps)
    torch.cuda.synchronize()
    for name, _ in runs:
        ms = best[name]
        print(f"{name} {a.prec} opA={a.opA} opB={a.opB} M={M} N={N} K={K}: {ms * 1e3:.1f} us/call, "
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


def _filter(a):
    """One filter application (feast_filter_apply) on a seeded random Hermitian matrix of
    order n with an m0-column block: the launch shapes of that workload's factorization and
    sweeps (the values do not change them).  Prints the phase times of the call."""
    import torch
    import paper_1605_08771_amd as fm
    g = torch.Generator(device="cuda").manual_seed(a.seed)
    n, m0 = a.n, a.m0
    A = torch.randn((n, n), dtype=torch.complex128, device="cuda", generator=g)
    A = (A + A.mH) * (0.5 / n ** 0.5)
    A = fm.fortran(A)
    X = fm.fortran(torch.randn((n, m0), dtype=torch.complex128, device="cuda", generator=g))
    f = fm.Feast()
    prec = {"fp64": 0, "fp32ir": 1, "bf16x3ir": 2}[a.prec]
    st, Q = f.filter_apply(A, X, -0.05, 0.05, a.nc, prec=prec)
    torch.cuda.synchronize()
    print(f"filter n={n} m0={m0} n_c={a.nc} {a.prec}: status {st}, phases {f.timings()}",
          flush=True)
    f.close()


def _sweeps(a):
    """The solver's block sweeps (both adjoint sides, all nodes) at order n with an m0-column
    block, on placeholder factors (identity diagonal, small off-diagonal entries): the launch
    shapes of one filter application's solves without the factorization before them."""
    import torch
    import paper_1605_08771_amd as fm
    prec = {"fp64": 0, "fp32": 1, "bf16x3": 2}[a.prec]
    dt = torch.complex128 if prec == 0 else torch.complex64
    f = fm.Feast()
    np_, nbt = f.sweep_shape(a.n, prec)
    base = torch.full((a.nc, np_, np_), 1e-4, dtype=dt, device="cuda")
    base.diagonal(dim1=1, dim2=2).fill_(1.0)
    LU = base.transpose(1, 2)
    invL = torch.empty((a.nc, nbt, np_), dtype=dt, device="cuda")
    invU = torch.empty_like(invL)
    B = torch.ones((a.nc, 2, a.m0, np_), dtype=dt, device="cuda")
    st = f.sweeps(LU, B, a.n, 2, prec=prec)  # computes the inverse blocks (untimed)
    if st != 0:
        raise SystemExit(f"feast_kern_sweeps returned {st}")
    lib = fm.lib()
    Z = torch.empty_like(B)
    times = []
    for _ in range(a.reps):
        B.fill_(1.0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(f._stream)
        st = lib.feast_kern_sweeps(prec, a.n, a.nc, a.m0, 2, fm._vp(base.data_ptr()),
                                   fm._vp(invL.data_ptr()), fm._vp(invU.data_ptr()), 0,
                                   fm._vp(B.data_ptr()), fm._vp(Z.data_ptr()), None, None,
                                   fm._vp(f._stream.cuda_stream))
        e1.record(f._stream)
        e1.synchronize()
        if st != 0:
            raise SystemExit(f"feast_kern_sweeps returned {st}")
        times.append(e0.elapsed_time(e1))
    print(f"sweeps n={a.n} np={np_} nbt={nbt} m0={a.m0} n_c={a.nc} {a.prec}: "
          f"{min(times):.3f} ms per filter application's sweeps (min of {a.reps})", flush=True)
    f.close()


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="what", required=True)
    g = sub.add_parser("gemm")
    g.add_argument("--prec", choices=["fp64", "fp64x3", "fp32", "bf16x3"], default="fp64")
    g.add_argument("--shape", type=int, nargs=3, metavar=("M", "N", "K"), required=True)
    g.add_argument("--opA", type=int, default=0, choices=[0, 1, 2])
    g.add_argument("--opB", type=int, default=0, choices=[0, 1, 2])
    g.add_argument("--reps", type=int, default=4)
    g.add_argument("--rounds", type=int, default=1,
                   help="timed rounds (alternating with --vendor); the fastest round is reported")
    g.add_argument("--seed", type=int, default=0)
    g.add_argument("--vendor", action="store_true", help="also time torch.addmm (ROCm BLAS)")
    j = sub.add_parser("jacobi")
    j.add_argument("--m", type=int, required=True)
    j.add_argument("--kind", choices=["random", "gram"], default="random")
    j.add_argument("--reps", type=int, default=3)
    j.add_argument("--seed", type=int, default=0)
    sw = sub.add_parser("sweeps")
    sw.add_argument("--n", type=int, required=True)
    sw.add_argument("--m0", type=int, required=True)
    sw.add_argument("--nc", type=int, default=8)
    sw.add_argument("--prec", choices=["fp64", "fp32", "bf16x3"], default="fp32")
    sw.add_argument("--reps", type=int, default=2)
    fl = sub.add_parser("filter")
    fl.add_argument("--n", type=int, required=True)
    fl.add_argument("--m0", type=int, required=True)
    fl.add_argument("--nc", type=int, default=8)
    fl.add_argument("--prec", choices=["fp64", "fp32ir", "bf16x3ir"], default="fp32ir")
    fl.add_argument("--seed", type=int, default=0)
    a = ap.parse_args(argv)
    {"gemm": _gemm, "jacobi": _jacobi, "filter": _filter, "sweeps": _sweeps}[a.what](a)


if __name__ == "__main__":
    sys.exit(main())
