"""The configurations and code paths the benchmark reaches that the other GPU tests do not:
config 5 at full size (n = 32768, m0 = 768, n_c = 8, FP32 factors with FP64 refinement, the
default benchmark step), all 64 problems of config 4 through the batched entry point, config
3 with the bf16x3 split-precision products, oracle parity where the sweeps use 256-row blocks
(2048 <= n < 8192), and the degenerate sizes (n below one 64-row tile, m0 = 1, m0 = n).

Full-size results are checked against the construction A = U diag(lam) U^H (the oracle, an
FP64 CPU FEAST, would take hours there): every eigenvalue inside I to 1e-10 ||A||, residuals
at most the tolerance, and the span of the counted Ritz vectors against U[:, inside] within
the Davis-Kahan bound (see test_gpu_fullsize.py).  Smaller cases are compared with the oracle
on the same seeded inputs: filtered blocks to 1e-11 relative, eigenvalues to 1e-10 ||A||,
subspaces to sin(theta_max) <= 1e-8, equal statuses and counts."""
import numpy as np
import pytest

from paper_1605_08771_amd import gen
from tests.pins import orthonormal, sin_theta_max
from tests.test_gpu_fullsize import _check_converged

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fe():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the HIP device"
    import paper_1605_08771_amd as fm
    f = fm.Feast()
    yield f
    f.close()
    torch.cuda.empty_cache()


def _dev(a):
    import torch
    import paper_1605_08771_amd as fm
    return fm.fortran(torch.from_numpy(np.asarray(a)).cuda())


def test_c5_mixed_solve_full_size(fe):
    """Config 5 as the benchmark times it: FP32+IR, filter-value test on, stop at 1e-10 ||A||."""
    import torch
    p = gen.config5(device=torch.device("cuda"))
    assert p.n == 32768 and p.m0 == 768 and p.n_c == 8 and p.m_true == 512
    fe.invalidate()
    out = fe.solve(p.A, p.emin, p.emax, p.m0, n_c=p.n_c, tol=1e-10, max_iter=p.max_iter,
                   anorm=p.anorm, X0=p.X0, prec=1, spurious=True, refine_max=0)
    torch.cuda.synchronize()
    fe.invalidate()
    try:
        _check_converged(p, out, 1e-10)
        assert len(out["trace"]) == out["iters"] and out["trace"][-1] <= 1e-10
        assert out["filter_applications"] in (out["iters"], out["iters"] + 1)
        fa, fc = out["filter_applications"], out["filter_columns"]
        n_in = int(np.sum((out["lam"] > p.emin) & (out["lam"] < p.emax)))
        assert fc in (fa * p.m0, (fa - 1) * p.m0 + n_in), (fa, fc, n_in)
    finally:
        del p, out
        torch.cuda.empty_cache()


def test_c4_all_problems_batched(fe):
    """All 64 problems of config 4 (n ~ U{256..4096}, own intervals, FP32+IR) on 8 worker
    streams, as the benchmark runs them; the per-problem report (iterations, trace, filter
    applications, time) comes back through the C-ABI."""
    import torch
    specs = gen.config4_specs()
    probs = [gen.config4_problem(sp, device=torch.device("cuda")) for sp in specs]
    assert len(probs) == 64
    d = [dict(A=p.A, X0=p.X0, emin=p.emin, emax=p.emax, m0=p.m0, anorm=p.anorm) for p in probs]
    fe.invalidate()
    bad, outs = fe.solve_batched(d, n_c=8, tol=1e-10, max_iter=400, prec=1, spurious=True,
                                 nstreams=8)
    torch.cuda.synchronize()
    fe.invalidate()
    assert bad == 0, [o["status"] for o in outs]
    for p, o in zip(probs, outs):
        _check_converged(p, o, 1e-10)
        assert len(o["trace"]) == o["iters"] and o["trace"][-1] <= 1e-10
        assert o["time_ms"] > 0 and o["filter_applications"] >= o["iters"]
    iters = sorted(o["iters"] for o in outs)
    assert iters[0] >= 1 and iters[-1] <= 400
    del probs, d, outs
    torch.cuda.empty_cache()


def test_c3_bf16x3_solve_full_size(fe):
    """Config 3 (n = 16384, m0 = 400, n_c = 16) with the bf16x3 split-precision products and
    FP64 refinement, to the benchmark's threshold."""
    import torch
    p = gen.config3(device=torch.device("cuda"))
    fe.invalidate()
    out = fe.solve(p.A, p.emin, p.emax, p.m0, n_c=p.n_c, tol=1e-10, max_iter=p.max_iter,
                   anorm=p.anorm, X0=p.X0, prec=2, spurious=True, refine_max=0)
    torch.cuda.synchronize()
    fe.invalidate()
    try:
        _check_converged(p, out, 1e-10)
    finally:
        del p, out
        torch.cuda.empty_cache()


# ---------------------------------------------------------------- 256-row sweep blocks
def _n2048_hard(m0=80):
    """Config-2 recipe (edge clusters inside and outside I) at n = 2048: sweep and inverse
    blocks of 256 rows."""
    return gen.config2(n=2048, seed_tag=2048, n_in=60, n_in_edge=12, n_out_edge=30, m0=m0,
                       n_c=8, max_iter=200)


@pytest.mark.parametrize("prec", [0, 1])
def test_sweep_block_256_filter_vs_oracle(fe, orc, prec):
    import torch
    p = _n2048_hard()
    ref = orc.filter_apply("c128", p.A, p.emin, p.emax, 8, p.X0)
    fe.invalidate()
    st, Q = fe.filter_apply(_dev(p.A), _dev(p.X0), p.emin, p.emax, 8, prec=prec)
    torch.cuda.synchronize()
    fe.invalidate()
    assert st == 0
    err = np.abs(Q.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < 1e-11, err


@pytest.mark.parametrize("prec", [0, 1])
def test_sweep_block_256_solve_vs_oracle(fe, orc, prec):
    """A full solve at n = 2048 (uniform spectrum, 40-odd eigenvalues in I, m0 = 64): same
    status, count, eigenvalues and subspace as the oracle, FP64 and FP32+IR."""
    import torch
    rng = gen.rng_for([2048, 1])
    emin, emax = -0.02, 0.02
    lam = gen.uniform_spectrum(rng, 2048, emin, emax)
    p = gen.make_problem(lam, emin, emax, 64, 8, 1e-12, 40, True, rng, name="n2048")
    assert p.m_true < 64
    ref = orc.feast_solve("c128", p.A, emin, emax, 8, p.m0, p.tol, p.max_iter, p.anorm, p.X0,
                          spurious=True)
    fe.invalidate()
    out = fe.solve(_dev(p.A), emin, emax, p.m0, n_c=8, tol=p.tol, max_iter=p.max_iter,
                   anorm=p.anorm, X0=_dev(p.X0), prec=prec, spurious=True, refine_max=0)
    torch.cuda.synchronize()
    fe.invalidate()
    assert out["status"] == 0 and ref["status"] == 0
    assert out["m"] == ref["m"] == p.m_true
    sg = out["counted"]
    so = (ref["lam"] > emin) & (ref["lam"] < emax) & (ref["mu"] > 0.5)
    np.testing.assert_allclose(out["lam"][sg], ref["lam"][so], rtol=0, atol=1e-10 * p.anorm)
    assert np.max(out["res"][sg]) <= p.tol
    assert sin_theta_max(ref["X"][:, so], out["X"].cpu().numpy()[:, sg]) < 1e-8
    assert abs(out["iters"] - ref["iters"]) <= 1


# ---------------------------------------------------------------- degenerate sizes
def _small(n=40, tag=4040):
    rng = gen.rng_for([tag, n])
    lam = np.sort(gen.uniform_spectrum(rng, n, -0.9, 0.9))
    return rng, lam


def _parity(fe, orc, p, spurious=False, prec=0):
    import torch
    ref = orc.feast_solve("c128", p.A, p.emin, p.emax, p.n_c, p.m0, p.tol, p.max_iter, p.anorm,
                          p.X0, spurious=spurious)
    fe.invalidate()
    out = fe.solve(_dev(p.A), p.emin, p.emax, p.m0, n_c=p.n_c, tol=p.tol, max_iter=p.max_iter,
                   anorm=p.anorm, X0=_dev(p.X0), prec=prec, spurious=spurious, refine_max=0)
    torch.cuda.synchronize()
    fe.invalidate()
    assert out["status"] == ref["status"]
    assert out["m"] == ref["m"]
    return out, ref


def test_m0_equal_n_below_one_tile(fe, orc):
    """n = 40 < 64 (one padded tile) and m0 = n: the basis is the whole space, so the first
    Rayleigh-Ritz step is exact; both sides converge at once to every eigenvalue in I."""
    rng, lam = _small()
    p = gen.make_problem(lam, -0.9, 0.9, 40, 8, 1e-12, 10, True, rng, name="m0=n")
    out, ref = _parity(fe, orc, p)
    assert out["status"] == 0 and out["m"] == p.m_true and out["iters"] <= 2
    sg = out["counted"]
    exact = np.sort(lam[(lam > -0.9) & (lam < 0.9)])
    np.testing.assert_allclose(out["lam"][sg], exact, rtol=0, atol=1e-10 * p.anorm)
    so = (ref["lam"] > -0.9) & (ref["lam"] < 0.9)
    assert sin_theta_max(ref["X"][:, so], out["X"].cpu().numpy()[:, sg]) < 1e-8


@pytest.mark.parametrize("m0", [1, 2])
def test_single_eigenvalue_interval(fe, orc, m0):
    """n = 40 with exactly one eigenvalue in I: m0 = 1 violates the precondition m < m0 (the
    run either converges at the first iteration or stops with M0_TOO_SMALL, the same on both
    sides); m0 = 2 converges to that eigenvalue."""
    rng, lam = _small(tag=4041)
    k = 20
    a, b = 0.5 * (lam[k - 1] + lam[k]), 0.5 * (lam[k] + lam[k + 1])
    p = gen.make_problem(lam, a, b, m0, 8, 1e-12, 20, True, rng, name="one")
    assert p.m_true == 1
    out, ref = _parity(fe, orc, p)
    if m0 == 2:
        assert out["status"] == 0
    assert out["status"] in (0, 2)
    if out["status"] == 0:
        np.testing.assert_allclose(out["lam"][out["counted"]], [lam[k]], rtol=0,
                                   atol=1e-10 * p.anorm)
        so = (ref["lam"] > a) & (ref["lam"] < b)
        np.testing.assert_allclose(ref["lam"][so], [lam[k]], rtol=0, atol=1e-10 * p.anorm)
