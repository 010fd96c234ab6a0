"""Pins of the oracle's expanded-subspace solvers (Sec. 2: XFEAST, Method 1, and RFEAST,
Method 2, as stated in the Appendix algorithms) against facts that do not come from the oracle:

* brute-force diagonalization of the test matrix (the converged pairs are the eigenpairs of A
  inside I);
* reductions that hold by construction: RFEAST with s = 1 is FEAST, and XFEAST with a window of
  one block is FEAST one iteration behind (its first Rayleigh-Ritz step sees X_0 itself);
* an invariant start (X_0 spanning eigenvectors exactly) converges at the first iteration,
  which needs the rank truncation of the Gram route when the window is exactly rank m0;
* the paper's Sec. 3 comparison on its n=545 test matrices: on the "dense" outer spectrum both
  variants with m0=51 beat FEAST with the same subspace size (m0=153) per iteration, and FEAST
  with m0=51 per linear-system right-hand side; on the "sparse" one FEAST with the larger
  subspace is ahead per iteration.
"""
import numpy as np
import pytest

from paper_1605_08771_amd import gen
from tests.pins import orthonormal, sin_theta_max


def _feast(orc, p, m0, iters, X0=None, tol=None):
    X0 = p.X0 if X0 is None else X0
    return orc.feast_solve(p.dtype, p.A, p.emin, p.emax, p.n_c, m0, tol or p.tol, iters, p.anorm,
                           X0)


def _xr(orc, v, p, s, iters, tol=None, spurious=False, X0=None, m0=None):
    return orc.xrfeast_solve(v, p.dtype, p.A, p.emin, p.emax, p.n_c, m0 or p.m0, s, tol or p.tol,
                             iters, p.anorm, p.X0 if X0 is None else X0, spurious=spurious)


def _check_converged(p, out, tol_lam=1e-10):
    """In-I pairs equal A's eigenpairs in I (ground truth from the construction)."""
    lam_true = np.sort(p.lam[(p.lam > p.emin) & (p.lam < p.emax)])
    inside = (out["lam"] > p.emin) & (out["lam"] < p.emax)
    assert out["m"] == len(lam_true)
    # the m lowest-residual inside pairs are the counted ones
    idx = np.flatnonzero(inside)
    idx = idx[np.argsort(out["res"][idx], kind="stable")][: len(lam_true)]
    idx = np.sort(idx)
    np.testing.assert_allclose(out["lam"][idx], lam_true, rtol=0, atol=tol_lam * p.anorm)
    U = np.asarray(p.U)
    order = np.argsort(p.lam)
    Ut = U[:, order[(np.sort(p.lam) > p.emin) & (np.sort(p.lam) < p.emax)]]
    assert sin_theta_max(orthonormal(Ut), orthonormal(out["X"][:, idx])) < 1e-7
    return idx


@pytest.fixture(scope="module")
def small(orc):
    """n=160 real symmetric with a sparse outer spectrum: 12 inside (-0.1, 0.1)."""
    rng = gen.rng_for(61)
    lam = np.concatenate([gen.uniform_spectrum(rng, 12, -0.1, 0.1, lo=-0.1, hi=0.1),
                          rng.uniform(0.12, 1.0, size=74), rng.uniform(-1.0, -0.12, size=74)])
    return gen.make_problem(lam, -0.1, 0.1, 18, 4, 1e-12, 30, False, rng, name="xr-small")


@pytest.mark.parametrize("variant,s", [("x", 2), ("x", 3), ("r", 2), ("r", 3)])
def test_xr_converges_to_eigenpairs(orc, small, variant, s):
    out = _xr(orc, variant, small, s, 30)
    assert out["status"] == 0, out["trace"]
    idx = _check_converged(small, out)
    assert np.all(out["res"][idx] <= 1e-12)


@pytest.mark.parametrize("variant", ["x", "r"])
def test_xr_complex_converges(orc, variant):
    """Complex Hermitian, with the filter-value test on: here the expanded bases produce
    inside pairs that A does not have (Sec. 2 warns of them for both methods) and, with
    m0 - m = 5 slots, they crowd out the outer pairs the selection would otherwise keep;
    mu_k = Re(x_k^H rho(A) x_k) > 1/2 excludes them from the count."""
    rng = gen.rng_for(62)
    lam = np.concatenate([gen.uniform_spectrum(rng, 10, -0.2, 0.2, lo=-0.2, hi=0.2),
                          rng.uniform(0.25, 1.0, size=60), rng.uniform(-1.0, -0.25, size=60)])
    p = gen.make_problem(lam, -0.2, 0.2, 15, 4, 1e-12, 30, True, rng, name="xr-complex")
    out = _xr(orc, variant, p, 2, 30, spurious=True)
    assert out["status"] == 0, out["trace"]
    _check_converged(p, out)


def test_rfeast_one_step_is_feast(orc, small):
    """RFEAST with s=1 runs one Rayleigh-Ritz step on rho(A) X_i and keeps all m0 pairs: the
    FEAST iteration (Appendix FEAST box)."""
    f = _feast(orc, small, small.m0, 6)
    r = _xr(orc, "r", small, 1, 6)
    k = min(len(f["trace"]), len(r["trace"]))
    assert k >= 4
    a, b = f["trace"][:k], r["trace"][:k]
    assert np.all(np.abs(a - b) <= 1e-6 * np.maximum(a, b) + 1e-14), (a, b)


def test_xfeast_one_block_is_feast_delayed(orc, small):
    """XFEAST with a window of one block: iteration 1 is Rayleigh-Ritz on X_0 itself, and
    iteration k+1 is FEAST's iteration k."""
    f = _feast(orc, small, small.m0, 5)
    x = _xr(orc, "x", small, 1, 6)
    k = min(len(f["trace"]), len(x["trace"]) - 1)
    assert k >= 4
    a, b = f["trace"][:k], x["trace"][1:k + 1]
    assert np.all(np.abs(a - b) <= 1e-6 * np.maximum(a, b) + 1e-14), (a, b)
    assert x["trace"][0] > 2 * f["trace"][0]  # unfiltered X_0 is farther from converged


@pytest.mark.parametrize("variant,s", [("x", 2), ("x", 3), ("r", 3)])
def test_invariant_start_converges_at_once(orc, variant, s):
    """X_0 = unit vectors of 6 eigenvectors inside I and 3 outside of a diagonal A: span X_0 is
    invariant, so the first Rayleigh-Ritz step is exact.  For XFEAST the window
    [X_0, rho X_0, rho^2 X_0] has rank m0 exactly; the Gram route must drop the null part."""
    lam = np.linspace(-1.0, 1.0, 41)[1:-1]
    lam = lam[np.abs(lam) > 1e-9]  # keep away from the open interval's centre
    n = len(lam)
    A = np.diag(lam)
    inside = np.flatnonzero(np.abs(lam) < 0.16)
    outside = np.flatnonzero((np.abs(lam) > 0.16) & (np.abs(lam) < 0.3))[:3]
    cols = np.concatenate([inside, outside])
    X0 = np.eye(n)[:, cols]
    out = orc.xrfeast_solve(variant, "r64", A, -0.16, 0.16, 4, len(cols), s, 1e-13, 3, 1.0, X0)
    assert out["status"] == 0 and out["iters"] == 1, out
    assert out["m"] == len(inside)
    np.testing.assert_allclose(np.sort(out["lam"][np.abs(out["lam"]) < 0.16]),
                               np.sort(lam[inside]), atol=1e-15)


# ------------------------------------------------------------- Sec. 3 comparison (n = 545)
@pytest.fixture(scope="module")
def dense_runs(orc):
    p = gen.fig2_problem("dense")
    X0_153 = gen.gaussian_block(gen.rng_for([6, 0, 153]), p.n, 153, False)
    return dict(
        p=p,
        f51=_feast(orc, p, 51, 9)["trace"],
        f153=_feast(orc, p, 153, 6, X0=X0_153)["trace"],
        x3=_xr(orc, "x", p, 3, 6)["trace"],
        r3=_xr(orc, "r", p, 3, 6)["trace"],
    )


def test_dense_outer_spectrum_per_iteration(dense_runs):
    """Sec. 3, dense outer spectrum: XFEAST and RFEAST (m0=51, s=3) beat FEAST with the same
    subspace size (m0=153) at every iteration (after the first for XFEAST, whose first
    Rayleigh-Ritz step includes the unfiltered X_0)."""
    f153, x3, r3 = dense_runs["f153"], dense_runs["x3"], dense_runs["r3"]
    assert len(f153) == len(x3) == len(r3) == 6
    assert np.all(r3 < 0.1 * f153), (r3, f153)
    assert np.all(x3[1:] < f153[1:]), (x3, f153)


def test_dense_outer_spectrum_per_rhs(dense_runs):
    """Sec. 3, residual against right-hand sides solved: at equal numbers of solves XFEAST
    (2 m0 extra for the initial window) and RFEAST are ahead of FEAST with m0=51."""
    f51, x3, r3 = dense_runs["f51"], dense_runs["x3"], dense_runs["r3"]
    for k in range(6):  # after iteration k+1 both variants have solved (k+1)(+2) blocks
        assert r3[k] < 0.01 * f51[k], (k, r3, f51)
        if k >= 1 and k + 2 < len(f51):
            assert x3[k] < f51[k + 2], (k, x3, f51)


def test_rfeast_dense_converges_to_true_count(orc):
    """RFEAST's count of expected pairs (pairs inside I at the first Rayleigh-Ritz step) keeps
    the spurious inside pairs of the expanded basis out of the test: it stops with the 50
    true eigenpairs."""
    p = gen.fig2_problem("dense")
    out = _xr(orc, "r", p, 3, 12, tol=1e-11)
    assert out["status"] == 0, out["trace"]
    _check_converged(p, out, tol_lam=1e-9)


def test_sparse_outer_spectrum_feast_ahead(orc):
    """Sec. 3, sparse outer spectrum: there the expansion does not pay per iteration; FEAST
    with m0=153 is ahead of both variants with m0=51 (n_c=3)."""
    p = gen.fig2_problem("sparse")
    X0_153 = gen.gaussian_block(gen.rng_for([6, 1, 153]), p.n, 153, False)
    f153 = _feast(orc, p, 153, 3, X0=X0_153)["trace"]
    x3 = _xr(orc, "x", p, 3, 3)["trace"]
    r3 = _xr(orc, "r", p, 3, 3)["trace"]
    assert np.all(f153[1:] < x3[1:]) and np.all(f153[1:] < r3[1:]), (f153, x3, r3)


def _xr_pins_pass(orc, small, dense_runs):
    for variant in ("x", "r"):
        out = _xr(orc, variant, small, 3, 30)
        if out["status"] != 0:
            return False
        try:
            _check_converged(small, out)
        except AssertionError:
            return False
    f = _feast(orc, small, small.m0, 5)["trace"]
    x = _xr(orc, "x", small, 1, 6)["trace"]
    if not np.all(np.abs(f[:4] - x[1:5]) <= 1e-6 * np.maximum(f[:4], x[1:5]) + 1e-14):
        return False
    p = dense_runs["p"]
    runs = dict(dense_runs, x3=_xr(orc, "x", p, 3, 6)["trace"], r3=_xr(orc, "r", p, 3, 6)["trace"])
    try:
        test_dense_outer_spectrum_per_iteration(runs)
        test_dense_outer_spectrum_per_rhs(runs)
    except AssertionError:
        return False
    return True


def _selection_ok(orc, trials=200):
    rng = np.random.default_rng(5)
    for _ in range(trials):
        r = int(rng.integers(1, 40))
        m0 = int(rng.integers(1, 30))
        lam = np.sort(rng.uniform(-2, 2, size=r))
        res = rng.uniform(0, 1, size=r)
        if not _selection_properties(orc, lam, res, -0.7, 0.9, m0):
            return False
    return True


def _selection_properties(orc, lam, res, emin, emax, m0):
    sel = orc.select_pairs(lam, res, emin, emax, m0)
    r = len(lam)
    if len(sel) != min(m0, r) or len(set(sel.tolist())) != len(sel):
        return False
    if np.any(np.diff(lam[sel]) < 0):
        return False
    inside = (lam > emin) & (lam < emax)
    chosen = np.zeros(r, bool)
    chosen[sel] = True
    if inside.sum() <= m0:  # every inside pair, then the best outside ones
        if not np.all(chosen[inside]):
            return False
        out_c, out_u = res[chosen & ~inside], res[~chosen & ~inside]
        return not (len(out_c) and len(out_u) and out_c.max() > out_u.min())
    # more inside pairs than m0: the m0 inside ones with the lowest residuals
    if np.any(chosen & ~inside):
        return False
    return res[chosen].max() <= res[inside & ~chosen].min()


def test_selection_rule_properties(orc):
    """Sec. 2 (Method 1) selection: all pairs inside I, then outside pairs by increasing
    residual, m0 in total, returned in ascending lambda; with more than m0 inside (a case the
    paper leaves open) the m0 inside pairs with the lowest residuals."""
    assert _selection_ok(orc)


@pytest.mark.parametrize("fault", [5, 6, 7, 8])
def test_xr_pins_catch_planted_mistakes(orc, small, dense_runs, fault):
    """Planted oracle mistakes in the expanded-subspace path (S^{-1} dropped in the B'
    reduction, outside pairs chosen by highest residual, the XFEAST window never slid, the
    RFEAST basis never grown by the residual block) each make a pin above fail.  (A wrong
    sign or a missing X Lambda term in R would not: the basis already holds X, so the span
    is unchanged.)"""
    orc.set_fault(fault)
    try:
        assert not (_selection_ok(orc) and _xr_pins_pass(orc, small, dense_runs))
    finally:
        orc.set_fault(0)
