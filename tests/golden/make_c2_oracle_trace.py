"""Writes c2_oracle_trace.txt: the FP64 CPU oracle's residual trace on config 2 at full size
(complex Hermitian n = 8192, 200 eigenvalues in I = (-0.05, 0.05) with edge clusters inside
and outside, m0 = 300, n_c = 8; the filter-value test on), for the first iterations of the
FEAST algorithm of the Appendix.  It calls only the oracle and the input generator; the GPU
path never contributes to the file.  Takes about three and a half hours on 8 cores.

    python tests/golden/make_c2_oracle_trace.py [iterations]
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1605_08771_amd import gen  # noqa: E402


def main():
    iters = int(sys.argv[1]) if len(sys.argv) > 1 else 12
    t0 = time.time()
    p = gen.config2()  # host arrays: the same draws as the device construction
    print(f"generated n={p.n} in {time.time() - t0:.0f}s", flush=True)
    t0 = time.time()
    out = oracle.feast_solve("c128", p.A, p.emin, p.emax, p.n_c, p.m0, 1e-30, iters, p.anorm,
                             p.X0, spurious=True)
    dt = time.time() - t0
    lines = [
        "# Appendix, FEAST algorithm, step 3: the largest residual ||A x_k - lambda_k x_k|| / ||A||",
        "# over the counted Ritz pairs (inside I, filter value mu_k > 1/2) after each iteration,",
        f"# of the FP64 CPU oracle on config 2 at full size (n = {p.n}, m0 = {p.m0}, n_c = {p.n_c},",
        "# I = (-0.05, 0.05), seeded input of the generator, start block X0), for the first",
        f"# {iters} iterations.  Written by make_c2_oracle_trace.py ({dt:.0f} s on "
        f"{oracle.num_threads()} threads).",
        f"iterations = {out['iters']}",
    ]
    lines += [f"trace_{i + 1} = {v:.17g}" for i, v in enumerate(out["trace"])]
    with open(os.path.join(HERE, "c2_oracle_trace.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
