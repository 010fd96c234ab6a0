"""Pins of the oracle's generalized Hermitian-definite solver, A x = lambda B x with B positive
definite (the extension the paper states for its problem, Sec. 1 eq. 1), against facts that do
not come from the oracle:

* LAPACK's generalized Hermitian eigensolver (scipy.linalg.eigh(A, B)) and the construction
  (A = Z^{-H} diag(lam) Z^{-1}, B = Z^{-H} Z^{-1}, so the eigenvalues and B-orthonormal
  eigenvectors Z are known);
* the closed form of the filter on the pencil: rho(B^{-1} A) X = Z diag(rho(lam)) Z^{-1} X;
* B = I reduces to the standard solver;
* scaling both matrices leaves the pencil's eigenpairs unchanged;
* planted mistakes (the filter applied to X instead of B X, residuals without B, B' formed
  without B) each fail a pin.
"""
import numpy as np
import pytest
import scipy.linalg as sl

from paper_1605_08771_amd import gen
from tests.pins import orthonormal, rho_closed, sin_theta_max


def _pencil(dtype, n=160, tag=70, m0=36, half=0.2):
    rng = gen.rng_for([tag, n])
    lam = gen.uniform_spectrum(rng, n, -half, half)
    return gen.pencil_problem(lam, -half, half, m0, 8, 1e-12, 60, dtype == "c128", rng)


def _solve(orc, p, B="pencil", **kw):
    return orc.feast_solve_gen(p.dtype, p.A, p.B if B == "pencil" else B, p.emin, p.emax,
                               p.n_c, p.m0, p.tol, p.max_iter, p.anorm, p.X0, **kw)


def _gen_pins_pass(orc, dtype):
    p = _pencil(dtype)
    out = _solve(orc, p)
    if out["status"] != 0 or out["m"] != p.m_true:
        return False
    ins = (out["lam"] > p.emin) & (out["lam"] < p.emax)
    exact = np.sort(p.lam[(p.lam > p.emin) & (p.lam < p.emax)])
    if np.max(np.abs(out["lam"][ins] - exact)) > 1e-10 * p.anorm:
        return False
    Q = orc.filter_apply_gen(p.dtype, p.A, p.B, p.emin, p.emax, 8, p.X0)
    ref = p.Z @ (rho_closed(p.lam, p.emin, p.emax, 8)[:, None] * np.linalg.solve(p.Z, p.X0))
    return np.abs(Q - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("dtype", ["r64", "c128"])
def test_pencil_vs_lapack_and_construction(orc, dtype):
    p = _pencil(dtype)
    w = sl.eigh(p.A, p.B, eigvals_only=True)
    np.testing.assert_allclose(np.sort(w), np.sort(p.lam), rtol=0, atol=1e-13)  # the recipe
    out = _solve(orc, p)
    assert out["status"] == 0 and out["m"] == p.m_true
    ins = (out["lam"] > p.emin) & (out["lam"] < p.emax)
    exact = np.sort(p.lam[(p.lam > p.emin) & (p.lam < p.emax)])
    np.testing.assert_allclose(out["lam"][ins], exact, rtol=0, atol=1e-10 * p.anorm)
    wl = np.sort(w[(w > p.emin) & (w < p.emax)])
    np.testing.assert_allclose(out["lam"][ins], wl, rtol=0, atol=1e-10 * p.anorm)
    X = out["X"][:, ins]
    np.testing.assert_allclose(np.diag(X.conj().T @ p.B @ X).real, 1.0, rtol=0, atol=1e-12)
    assert np.max(out["res"][ins]) <= p.tol
    tin = (p.lam > p.emin) & (p.lam < p.emax)
    assert sin_theta_max(orthonormal(p.Z[:, tin]), orthonormal(X)) < 1e-8
    R = p.A @ X - (p.B @ X) * out["lam"][ins][None, :]
    np.testing.assert_allclose(np.linalg.norm(R, axis=0) / p.anorm, out["res"][ins], rtol=1e-3,
                               atol=1e-15)


@pytest.mark.parametrize("dtype,nc", [("r64", 4), ("c128", 8)])
def test_pencil_filter_closed_form(orc, dtype, nc):
    p = _pencil(dtype, n=90, tag=71, m0=5)
    Q = orc.filter_apply_gen(p.dtype, p.A, p.B, p.emin, p.emax, nc, p.X0)
    ref = p.Z @ (rho_closed(p.lam, p.emin, p.emax, nc)[:, None] * np.linalg.solve(p.Z, p.X0))
    assert np.abs(Q - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("dtype", ["r64", "c128"])
def test_identity_B_is_the_standard_problem(orc, dtype):
    p = gen.config1(n=200, seed_tag=72) if dtype == "r64" else None
    if p is None:
        rng = gen.rng_for(73)
        lam = gen.uniform_spectrum(rng, 200, -0.1, 0.1)
        p = gen.make_problem(lam, -0.1, 0.1, 30, 8, 1e-12, 40, True, rng)
    eye = np.eye(p.n)
    a = orc.feast_solve(p.dtype, p.A, p.emin, p.emax, p.n_c, p.m0, p.tol, 40, p.anorm, p.X0)
    b = orc.feast_solve_gen(p.dtype, p.A, eye, p.emin, p.emax, p.n_c, p.m0, p.tol, 40, p.anorm,
                            p.X0)
    assert a["status"] == b["status"] == 0 and a["iters"] == b["iters"]
    np.testing.assert_allclose(a["trace"], b["trace"], rtol=1e-6, atol=1e-15)
    np.testing.assert_allclose(a["lam"], b["lam"], rtol=0, atol=1e-13)


def test_pencil_scaling_invariance(orc):
    p = _pencil("c128", n=120, tag=74, m0=30)
    a = _solve(orc, p)
    b = orc.feast_solve_gen(p.dtype, 3.0 * p.A, 3.0 * p.B, p.emin, p.emax, 8, p.m0, p.tol,
                            p.max_iter, 3.0 * p.anorm, p.X0)
    assert a["status"] == b["status"] == 0
    ia = (a["lam"] > p.emin) & (a["lam"] < p.emax)
    ib = (b["lam"] > p.emin) & (b["lam"] < p.emax)
    np.testing.assert_allclose(a["lam"][ia], b["lam"][ib], rtol=0, atol=1e-12)


@pytest.mark.parametrize("fault", [9, 10, 11])
def test_pencil_pins_catch_planted_mistakes(orc, fault):
    assert _gen_pins_pass(orc, "c128")
    orc.set_fault(fault)
    try:
        assert not _gen_pins_pass(orc, "c128")
    finally:
        orc.set_fault(0)
