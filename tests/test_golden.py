"""Values the paper prints, as cited fixtures under tests/golden/, checked against the oracle,
the closed-form filter and the input generator (CPU only)."""
import os

import numpy as np
import pytest

from paper_1605_08771_amd import gen
from tests.pins import rho_closed

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = (x.strip() for x in line.split("="))
                vals[k] = float(v)
    return vals


def test_sec1_rate_with_nc8_and_m0_1p5m(orc):
    """Sec. 1: n_c = 8 and m0 ~ 1.5 m give a per-iteration rate of about 1e4.  On a uniform
    spectrum the closed-form ratio rho(lambda_m) / rho(lambda_{m0+1}) is within a factor of
    ten of the printed value, and the oracle's FEAST residuals contract by at least 1e3 per
    iteration until they reach rounding level."""
    g = _read("sec1_convergence_rate.txt")
    nc = int(g["n_c"])
    rng = gen.rng_for([91, 1])
    n, emin, emax = 600, -0.1, 0.1
    lam = gen.uniform_spectrum(rng, n, emin, emax)
    m = int(np.sum((lam > emin) & (lam < emax)))
    m0 = int(round(g["m0_over_m"] * m))
    p = gen.make_problem(lam, emin, emax, m0, nc, 1e-13, 12, False, rng)
    rho = np.abs(rho_closed(p.lam, emin, emax, nc))
    inside = (p.lam > emin) & (p.lam < emax)
    predicted = np.min(rho[inside]) / np.sort(rho)[::-1][m0]
    assert g["rate"] / 10 <= predicted <= g["rate"] * 10, predicted
    out = orc.feast_solve("r64", p.A, emin, emax, nc, m0, 1e-13, 12, p.anorm, p.X0)
    assert out["status"] == 0
    tr = np.asarray(out["trace"])
    tr = tr[tr > 1e-12]
    assert len(tr) >= 3
    measured = np.exp(np.mean(np.log(tr[:-1] / tr[1:])))
    assert measured >= g["rate"] / 10, (measured, tr)


@pytest.mark.parametrize("kind", ["dense", "sparse"])
def test_sec3_test_matrices(kind):
    """Sec. 3: the generator's two n = 545 matrices have the printed dimension, count inside
    I = [-1, 1] and outer ranges; the XFEAST/RFEAST default m0 is the printed 51."""
    g = _read("sec3_test_matrices.txt")
    p = gen.fig2_problem(kind)
    hi = g["outer_hi_" + kind]
    assert p.n == int(g["n"]) and p.m0 == int(g["xr_m0"])
    assert (p.emin, p.emax) == (g["emin"], g["emax"])
    inside = (p.lam > p.emin) & (p.lam < p.emax)
    assert int(inside.sum()) == int(g["inside"]) == p.m_true
    outer = p.lam[~inside]
    assert len(outer) == int(g["n"]) - int(g["inside"])
    assert outer.min() >= g["outer_lo"] and outer.max() <= hi
    # the outer eigenvalues fill their range (not bunched at one end)
    assert outer.max() - outer.min() > 0.9 * (hi - g["outer_lo"])
