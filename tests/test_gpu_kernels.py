"""Kernel-level parity of the HIP building blocks against plain fp64 references on the host:
the matrix-core complex GEMM (all op combinations, ragged shapes; FP64, FP32 and bf16x3
products), the batched partial-pivot
LU of the shifted matrices, and the Jacobi reduced eigensolver."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fe():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the HIP device"
    import paper_1605_08771_amd as fm
    f = fm.Feast()
    yield f
    f.close()


def _dev(a, dtype=None):
    import torch
    import paper_1605_08771_amd as fm
    t = torch.from_numpy(np.asarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return fm.fortran(t.cuda())


def _crand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


OPS = {0: lambda a: a, 1: lambda a: a.T, 2: lambda a: a.conj().T}


@pytest.mark.parametrize("three", [False, True])
@pytest.mark.parametrize("opA", [0, 1, 2])
@pytest.mark.parametrize("opB", [0, 1, 2])
@pytest.mark.parametrize("shape", [(1, 1, 1), (17, 5, 33), (64, 64, 16), (130, 77, 70),
                                   (65, 129, 0), (200, 31, 257)])
def test_zgemm_fp64(fe, opA, opB, shape, three):
    """Four-product and three-product (factorization, Rayleigh-Ritz) FP64 forms."""
    import torch
    M, N, K = shape
    rng = np.random.default_rng(M * 1000 + N * 10 + K + 7 * opA + opB)
    A = _crand(rng, M, K) if opA == 0 else _crand(rng, K, M)
    B = _crand(rng, K, N) if opB == 0 else _crand(rng, N, K)
    C = _crand(rng, M, N)
    alpha, beta = 0.7 - 0.3j, -1.1 + 0.4j
    ref = alpha * OPS[opA](A) @ OPS[opB](B) + beta * C
    dA, dB, dC = _dev(A), _dev(B), _dev(C)
    st = fe.gemm(opA, opB, dA, dB, dC, alpha, beta, M=M, N=N, K=K, three_products=three)
    torch.cuda.synchronize()
    assert st == 0
    got = dC.cpu().numpy()
    scale = (np.abs(A).max() if A.size else 1) * (np.abs(B).max() if B.size else 1) * max(K, 1)
    assert np.abs(got - ref).max() <= 1e-14 * scale + 1e-14


@pytest.mark.parametrize("opA,opB", [(0, 0), (2, 0), (0, 2)])
def test_cgemm_fp32(fe, opA, opB):
    import torch
    M, N, K = 150, 70, 99
    rng = np.random.default_rng(11)
    A = _crand(rng, M, K) if opA == 0 else _crand(rng, K, M)
    B = _crand(rng, K, N) if opB == 0 else _crand(rng, N, K)
    C = np.zeros((M, N), dtype=np.complex128)
    ref = OPS[opA](A) @ OPS[opB](B)
    dA, dB = _dev(A, torch.complex64), _dev(B, torch.complex64)
    dC = _dev(C, torch.complex64)
    assert fe.gemm(opA, opB, dA, dB, dC, 1.0, 0.0, M=M, N=N, K=K) == 0
    torch.cuda.synchronize()
    got = dC.cpu().numpy().astype(np.complex128)
    assert np.abs(got - ref).max() <= 2e-5 * np.abs(ref).max()


@pytest.mark.parametrize("opA,opB", [(0, 0), (1, 0), (2, 0), (0, 2), (0, 1)])
def test_cgemm_fp32_large_ragged(fe, opA, opB):
    """FP32 products over about 2000 output tiles (more than the chip holds at once, so the
    XCD-aware tile order wraps): ragged M, N and K, op(A) and op(B) variants, alpha and beta,
    against the FP32 error bound 4 K 2^-24 sum |a||b| + |beta c| terms."""
    import torch
    M, N, K = 8201, 1003, 45
    rng = np.random.default_rng(17 + 3 * opA + opB)
    A = _crand(rng, M, K) if opA == 0 else _crand(rng, K, M)
    B = _crand(rng, K, N) if opB == 0 else _crand(rng, N, K)
    C = _crand(rng, M, N)
    A, B, C = (x.astype(np.complex64).astype(np.complex128) for x in (A, B, C))
    alpha, beta = 0.5 + 0.25j, -0.75 + 0.5j
    ref = alpha * OPS[opA](A) @ OPS[opB](B) + beta * C
    dA, dB, dC = (_dev(x, torch.complex64) for x in (A, B, C))
    assert fe.gemm(opA, opB, dA, dB, dC, alpha, beta, M=M, N=N, K=K) == 0
    torch.cuda.synchronize()
    got = dC.cpu().numpy().astype(np.complex128)
    bound = 4 * K * 2.0**-24 * (np.abs(alpha) * (np.abs(OPS[opA](A)) @ np.abs(OPS[opB](B)))
                                + np.abs(beta * C))
    assert np.all(np.abs(got - ref) <= bound + 1e-30), np.max(np.abs(got - ref) / bound)


@pytest.mark.parametrize("opA", [0, 1, 2])
@pytest.mark.parametrize("opB", [0, 1, 2])
@pytest.mark.parametrize("shape", [(1, 1, 1), (130, 77, 70), (65, 129, 0), (200, 31, 257)])
def test_cgemm_bf16x3(fe, opA, opB, shape):
    """bf16x3 products of complex64 operands against the exact product of the same operands.
    With bf16 (8 significant bits, unit roundoff 2^-8) hi = RN(x), lo = RN(x - hi):
    |x - hi - lo| <= 2^-16 |x|, and dropping lo_a lo_b adds at most 2^-16 |a||b|, so a real
    product errs by at most ~3 2^-16 |a||b|; FP32 accumulation adds K 2^-24 sum |a||b|.  A
    complex entry therefore errs by at most (3 2^-16 + K 2^-23) sum_k 2 |a_ik| |b_kj|.  A
    dropped cross term (error ~2^-9 per product) exceeds this bound for these K."""
    import torch
    M, N, K = shape
    rng = np.random.default_rng(M * 1000 + N * 10 + K + 7 * opA + opB + 5)
    A = _crand(rng, M, K) if opA == 0 else _crand(rng, K, M)
    B = _crand(rng, K, N) if opB == 0 else _crand(rng, N, K)
    C = _crand(rng, M, N)
    A = A.astype(np.complex64).astype(np.complex128)
    B = B.astype(np.complex64).astype(np.complex128)
    C = C.astype(np.complex64).astype(np.complex128)
    alpha, beta = 0.75 - 0.25j, -1.0 + 0.5j
    oA, oB = OPS[opA](A), OPS[opB](B)
    ref = alpha * oA @ oB + beta * C
    dA, dB, dC = (_dev(x, torch.complex64) for x in (A, B, C))
    st = fe.gemm(opA, opB, dA, dB, dC, alpha, beta, M=M, N=N, K=K, split_bf16=True)
    torch.cuda.synchronize()
    assert st == 0
    got = dC.cpu().numpy().astype(np.complex128)
    bound = (3 * 2.0**-16 + K * 2.0**-23) * 2 * np.abs(alpha) * (np.abs(oA) @ np.abs(oB))
    bound += 4 * 2.0**-24 * (np.abs(ref) + np.abs(beta * C)) + 1e-30
    assert np.all(np.abs(got - ref) <= bound), np.max(np.abs(got - ref) / bound)


def test_cgemm_bf16x3_beats_bf16(fe):
    """The lo parts matter: the bf16x3 error is far below a product of bf16-rounded operands."""
    import torch
    rng = np.random.default_rng(21)
    M, N, K = 256, 128, 512
    A = _crand(rng, M, K).astype(np.complex64).astype(np.complex128)
    B = _crand(rng, K, N).astype(np.complex64).astype(np.complex128)
    ref = A @ B
    dA, dB = _dev(A, torch.complex64), _dev(B, torch.complex64)
    dC = _dev(np.zeros((M, N)), torch.complex64)
    assert fe.gemm(0, 0, dA, dB, dC, 1.0, 0.0, split_bf16=True) == 0
    torch.cuda.synchronize()
    err = np.abs(dC.cpu().numpy().astype(np.complex128) - ref).max()

    def bf16(x):  # round to nearest even at 8 significant bits
        return torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()

    err_bf16 = np.abs((bf16(A.real) + 1j * bf16(A.imag)) @ (bf16(B.real) + 1j * bf16(B.imag))
                      - ref).max()
    assert err < err_bf16 / 64, (err, err_bf16)


def test_zgemm_beta_zero_ignores_nan(fe):
    import torch
    rng = np.random.default_rng(3)
    A, B = _crand(rng, 40, 20), _crand(rng, 20, 30)
    C = np.full((40, 30), np.nan + 1j * np.nan)
    dA, dB, dC = _dev(A), _dev(B), _dev(C)
    assert fe.gemm(0, 0, dA, dB, dC, 1.0, 0.0) == 0
    torch.cuda.synchronize()
    np.testing.assert_allclose(dC.cpu().numpy(), A @ B, rtol=0, atol=1e-12)


@pytest.mark.parametrize("n,prec", [(60, 0), (200, 0), (500, 0), (1030, 0), (300, 1), (300, 2),
                                    (1030, 2)])
def test_batched_lu(fe, n, prec):
    """P_j (z_j I - A) = L_j U_j for every node, with |L| <= 1 (partial pivoting)."""
    import torch
    rng = np.random.default_rng(n)
    G = _crand(rng, n, n)
    A = 0.5 * (G + G.conj().T) / np.sqrt(n)
    z = np.array([0.1 + 0.05j, -0.3 + 0.001j, 0.7 + 0.4j])
    st, LU, perm = fe.lu(_dev(A), z, prec=prec)
    torch.cuda.synchronize()
    assert st == 0
    LU = LU.cpu().numpy().astype(np.complex128)
    perm = perm.cpu().numpy()
    np_ = LU.shape[1]
    # prec 2: trailing updates as bf16x3 products, ~3 2^-16 relative per product term
    eps = {0: np.finfo(np.float64).eps, 1: np.finfo(np.float32).eps, 2: 2.0**-16}[prec]
    for j, zj in enumerate(z):
        M = np.eye(np_, dtype=np.complex128)
        M[:n, :n] = zj * np.eye(n) - A
        L = np.tril(LU[j], -1) + np.eye(np_)
        U = np.triu(LU[j])
        assert sorted(perm[j]) == list(range(np_))
        assert np.all(np.abs(L) <= 1 + 1e-6)
        be = np.linalg.norm(M[perm[j]] - L @ U) / (np.linalg.norm(M) * np_ * eps)
        assert be < 5.0, (j, be)


@pytest.mark.parametrize("n,prec", [(60, 0), (300, 0), (1100, 0), (1500, 1), (2100, 1),
                                    (700, 2), (2100, 2)])
def test_short_panel_groups_match_column_steps(fe, n, prec):
    """The short-panel path (a group of column steps per launch once at most 1024 (FP64) or
    2048 (FP32) rows remain) gives bit-identical factors and permutations to one launch per
    column; n = 1100 (FP64) and 2100 (FP32) start with long panels and end with short ones."""
    import torch
    rng = np.random.default_rng(n + 7 * prec)
    G = _crand(rng, n, n)
    A = 0.5 * (G + G.conj().T) / np.sqrt(n)
    z = np.array([0.1 + 0.05j, -0.3 + 0.001j, 0.7 + 0.4j])
    st1, LU1, p1 = fe.lu(_dev(A), z, prec=prec)
    st2, LU2, p2 = fe.lu(_dev(A), z, prec=prec, column_steps=True)
    torch.cuda.synchronize()
    assert st1 == 0 and st2 == 0
    assert torch.equal(p1, p2)
    assert torch.equal(torch.view_as_real(LU1.contiguous()), torch.view_as_real(LU2.contiguous()))


@pytest.mark.parametrize("n,prec,sides", [(300, 0, 2), (700, 1, 2), (1100, 0, 1), (1500, 1, 2),
                                          (2100, 0, 2)])
def test_kern_sweeps_solve_both_adjoint_systems(fe, n, prec, sides):
    """The solver's block sweeps on feast_kern_lu's factors: side 0 solves (L U) y = b and side
    1 solves (L U)^H y = b, each to a backward error of a few units of the factors' precision."""
    import torch
    rng = np.random.default_rng(n + 11 * prec)
    G = _crand(rng, n, n)
    A = 0.5 * (G + G.conj().T) / np.sqrt(n)
    z = np.array([0.1 + 0.05j, -0.3 + 0.02j])
    st, LU, perm = fe.lu(_dev(A), z, prec=prec)
    assert st == 0
    np_, nbt = fe.sweep_shape(n, prec)
    assert LU.shape[1] == np_
    m0 = 23
    dt = torch.complex128 if prec == 0 else torch.complex64
    B0 = rng.standard_normal((2, sides, m0, np_)) + 1j * rng.standard_normal((2, sides, m0, np_))
    B = torch.from_numpy(B0).to(dt).cuda().contiguous()
    assert fe.sweeps(LU, B, n, sides, prec=prec) == 0
    torch.cuda.synchronize()
    Y = B.cpu().numpy().astype(np.complex128)
    LUh = LU.cpu().numpy().astype(np.complex128)
    eps = np.finfo(np.float64 if prec == 0 else np.float32).eps
    for j in range(2):
        L = np.tril(LUh[j], -1) + np.eye(np_)
        U = np.triu(LUh[j])
        for sd in range(sides):
            Mj = L @ U if sd == 0 else (L @ U).conj().T
            rhs = B0[j, sd].T.astype(np.complex128 if prec == 0 else np.complex64)
            rhs = rhs.astype(np.complex128)
            y = Y[j, sd].T
            be = np.linalg.norm(Mj @ y - rhs) / (np.linalg.norm(Mj) * np.linalg.norm(y) * np_ * eps)
            assert be < 5.0, (j, sd, be)


@pytest.mark.parametrize("m,k", [(300, 40), (700, 150), (96, 20), (513, 9)])
def test_jacobi_structured(fe, m, k):
    """A reduced matrix of the kind FEAST produces once most Ritz pairs have converged: a
    diagonal part with couplings below the convergence floor and a dense coupled block on k
    scattered indices; eigenvalues and eigenvectors against LAPACK."""
    import torch
    rng = np.random.default_rng(1000 + m + k)
    H = np.diag(rng.uniform(-1.0, 1.0, m)).astype(complex)
    E = 1e-18 * (rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    H += 0.5 * (E + E.conj().T)
    S = np.sort(rng.choice(m, size=k, replace=False))
    G = _crand(rng, k, k)
    H[np.ix_(S, S)] += 0.25 * (G + G.conj().T)
    sweeps, d, W = fe.jacobi(torch.from_numpy(H).cuda())
    torch.cuda.synchronize()
    assert sweeps >= 0
    d = d.cpu().numpy()
    W = W.cpu().numpy()
    tol = max(1e-13, 4 * m * np.finfo(float).eps) * np.linalg.norm(H, 2)
    np.testing.assert_allclose(d, np.linalg.eigvalsh(H), rtol=0, atol=tol)
    np.testing.assert_allclose(W.conj().T @ W, np.eye(m), rtol=0, atol=1e-12)
    np.testing.assert_allclose(H @ W, W * d, rtol=0, atol=1e-12 * np.linalg.norm(H, 2))


@pytest.mark.parametrize("m", [1, 2, 7, 31, 33, 64, 75, 301, 512, 513, 900])
def test_jacobi_vs_lapack(fe, m):
    import torch
    rng = np.random.default_rng(m)
    G = _crand(rng, m, m)
    H = 0.5 * (G + G.conj().T)
    sweeps, d, W = fe.jacobi(torch.from_numpy(H).cuda())
    torch.cuda.synchronize()
    assert sweeps >= 0
    d = d.cpu().numpy()
    W = W.cpu().numpy()
    scale = np.linalg.norm(H, 2)
    tol = max(1e-13, 4 * m * np.finfo(float).eps)  # a small multiple of m eps ||H||_2
    np.testing.assert_allclose(d, np.linalg.eigvalsh(H), rtol=0, atol=tol * scale)
    np.testing.assert_allclose(W.conj().T @ W, np.eye(m), rtol=0, atol=tol)
    np.testing.assert_allclose(H @ W, W * d, rtol=0, atol=tol * scale)


@pytest.mark.parametrize("m", [96, 600])
def test_jacobi_gram_spectrum(fe, m):
    """A Gram matrix B^H B whose eigenvalues fall from 1 to 1e-16 (the orthogonalization of
    the expanded subspaces): eigenvalues to 1e-13 ||G|| absolutely, and the eigenvectors of the
    eigenvalues above 1e-8 span LAPACK's invariant subspace to the Davis-Kahan bound: the
    sweeps stop once every off-diagonal entry is below 4 eps ||G||_F, so the angle between the
    computed and the exact invariant subspace is at most about that residual over the
    eigenvalue gap at the cut (a factor 8 allows for the norm of the residual block)."""
    import torch
    from tests.pins import sin_theta_max
    rng = np.random.default_rng(m + 7)
    Q, _ = np.linalg.qr(_crand(rng, m, m))
    ev = np.logspace(0, -16, m)
    G = (Q * ev) @ Q.conj().T
    G = 0.5 * (G + G.conj().T)
    sweeps, d, W = fe.jacobi(torch.from_numpy(G).cuda())
    torch.cuda.synchronize()
    assert sweeps >= 0
    d = d.cpu().numpy()
    W = W.cpu().numpy()
    dr, Wr = np.linalg.eigh(G)
    np.testing.assert_allclose(d, dr, rtol=0, atol=1e-13)
    big = dr > 1e-8
    k = int(np.argmax(big))  # first eigenvalue above the cut (ascending order)
    gap = dr[k] - dr[k - 1]
    bound = 8 * 4 * 2.2e-16 * np.linalg.norm(G) / gap
    assert sin_theta_max(Wr[:, big], W[:, d > 1e-8]) < bound
    # a graded spectrum takes ~3x the sweeps of a random one; each plane rotation is unitary to
    # one rounding error, and a sweep composes them into m / 16 - 1 block transforms of V, each
    # a product of 31 rotations applied as 32-term sums, so orthonormality is held to a
    # multiple of m eps
    np.testing.assert_allclose(W.conj().T @ W, np.eye(m), rtol=0, atol=max(1e-13, 16 * m * 2.2e-16))


def test_binding_refuses_real_input_to_complex_calls(fe):
    """A real tensor handed to a complex-only building block is refused before any launch."""
    import torch
    H = torch.eye(8, dtype=torch.float64, device="cuda")
    with pytest.raises(TypeError):
        fe.jacobi(H)
    with pytest.raises(TypeError):
        fe.lu(H, np.array([1j]))
    A = fm_fortran(torch.eye(8, dtype=torch.complex128, device="cuda"))
    Xr = fm_fortran(torch.zeros(8, 2, dtype=torch.float64, device="cuda"))
    with pytest.raises(TypeError):
        fe.filter_apply(A, Xr, -1.0, 1.0, 4)
    with pytest.raises(TypeError):
        fe.solve(A, -1.0, 1.0, 2, X0=Xr)


def fm_fortran(t):
    import paper_1605_08771_amd as fm
    return fm.fortran(t)
