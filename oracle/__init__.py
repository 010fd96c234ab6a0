"""TEST INFRASTRUCTURE ONLY: ctypes wrapper of the plain FP64 CPU FEAST oracle
(feast_oracle.c).  Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package; the GPU product never does.

Arrays are numpy, column-major (Fortran order).  dtype "r64" = real symmetric A / real X,
"c128" = complex Hermitian A / complex X.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libfeast_oracle.so")
_SO_FAULTS = os.path.join(_HERE, "libfeast_oracle_faults.so")
_lib = None
_ref = None      # the reference library
_faults = None   # the test build with planted mistakes (mutation tests only)

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force=False):
    """Compile the oracle with the host C compiler (no GPU code involved): the reference
    library, and a separate test build with the planted mistakes of the mutation tests
    (-DORACLE_FAULTS); the reference library holds no fault branches."""
    src = os.path.join(_HERE, "feast_oracle.c")
    hdr = os.path.join(_HERE, "feast_oracle.h")
    newest = max(os.path.getmtime(src), os.path.getmtime(hdr))
    for so, extra in ((_SO, []), (_SO_FAULTS, ["-DORACLE_FAULTS"])):
        if force or not os.path.exists(so) or os.path.getmtime(so) < newest:
            cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-fcx-fortran-rules",
                   "-std=c11", "-D_DEFAULT_SOURCE", "-Wall", *extra, src, "-o", so + ".tmp",
                   "-lm"]
            subprocess.check_call(cmd)
            os.replace(so + ".tmp", so)
    return _SO


def lib():
    """The library the oracle functions call: the reference build, or the fault build while
    set_fault(code != 0) is in effect."""
    global _lib, _ref
    if _lib is None:
        if _ref is None:
            _ref = _load(_SO)
        _lib = _ref
    return _lib


def _load(path):
    if not os.path.exists(path):
        build()
    L = ctypes.CDLL(path)
    L.or_gauss_legendre.argtypes = [ctypes.c_int, _dp, _dp]
    L.or_contour.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp, _dp]
    L.or_zlu.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _ip]
    L.or_zlu_solve.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _ip, ctypes.c_int, _dp,
                               ctypes.c_int, ctypes.c_int]
    L.or_jacobi_eigh.argtypes = [ctypes.c_int, _dp, ctypes.c_int, _dp, _dp, ctypes.c_int]
    L.or_filter_apply.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp,
                                  ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int]
    L.or_rayleigh_ritz.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, _dp, _dp, _ip]
    L.or_feast_solve.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_double, _dp, ctypes.c_int, _dp, ctypes.c_int,
                                 _dp, _dp, _ip, _ip, _dp]
    L.or_feast_solve_ex.argtypes = L.or_feast_solve.argtypes + [ctypes.c_int, _dp]
    L.or_xrfeast_solve.argtypes = [ctypes.c_int] + L.or_feast_solve.argtypes[:7] + [
        ctypes.c_int, ctypes.c_int] + L.or_feast_solve.argtypes[8:] + [ctypes.c_int, _dp]
    L.or_feast_solve_gen.argtypes = L.or_feast_solve.argtypes[:4] + [_dp, ctypes.c_int] + \
        L.or_feast_solve.argtypes[4:] + [ctypes.c_int, _dp]
    L.or_filter_apply_gen.argtypes = L.or_filter_apply.argtypes[:4] + [_dp, ctypes.c_int] + \
        L.or_filter_apply.argtypes[4:]
    L.or_select_pairs.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_int, _ip]
    L.or_num_threads.restype = ctypes.c_int
    L.or_set_num_threads.argtypes = [ctypes.c_int]
    if hasattr(L, "or_set_fault"):
        L.or_set_fault.argtypes = [ctypes.c_int]
    return L


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _dt(dtype):
    return {"r64": 0, "c128": 1}[dtype]


def _fort(a, dtype):
    want = np.complex128 if dtype == "c128" else np.float64
    return np.asfortranarray(np.asarray(a, dtype=want))


def set_fault(code: int):
    """Plant a known mistake in the oracle (0 = none); for the mutation tests of the pins.
    A nonzero code routes every oracle call to the separate fault build until set_fault(0)
    returns them to the reference library."""
    global _lib, _faults
    if code:
        if _faults is None:
            _faults = _load(_SO_FAULTS)
        _faults.or_set_fault(int(code))
        _lib = _faults
    else:
        if _faults is not None:
            _faults.or_set_fault(0)
        _lib = None


def num_threads() -> int:
    return lib().or_num_threads()


def set_num_threads(n: int):
    lib().or_set_num_threads(int(n))


def gauss_legendre(n):
    x = np.zeros(n)
    w = np.zeros(n)
    st = lib().or_gauss_legendre(n, _ptr(x), _ptr(w))
    if st:
        raise ValueError(st)
    return x, w


def contour(emin, emax, nc):
    z = np.zeros(2 * nc)
    om = np.zeros(2 * nc)
    st = lib().or_contour(emin, emax, nc, _ptr(z), _ptr(om))
    if st:
        raise ValueError(st)
    return z.view(np.complex128), om.view(np.complex128)


def zlu(M):
    M = _fort(M, "c128").copy(order="F")
    n = M.shape[0]
    piv = np.zeros(n, dtype=np.int32)
    st = lib().or_zlu(n, _ptr(M), n, piv.ctypes.data_as(_ip))
    return M, piv, st


def zlu_solve(LU, piv, B, adjoint=False):
    B = _fort(B, "c128").copy(order="F")
    n = LU.shape[0]
    nrhs = B.shape[1]
    LU = _fort(LU, "c128")
    piv = np.ascontiguousarray(piv, dtype=np.int32)
    lib().or_zlu_solve(n, _ptr(LU), n, piv.ctypes.data_as(_ip), nrhs, _ptr(B), n, int(adjoint))
    return B


def jacobi_eigh(H):
    H = _fort(H, "c128").copy(order="F")
    n = H.shape[0]
    d = np.zeros(n)
    V = np.zeros((n, n), dtype=np.complex128, order="F")
    sweeps = lib().or_jacobi_eigh(n, _ptr(H), n, _ptr(d), _ptr(V), n)
    return d, V, sweeps


def filter_apply(dtype, A, emin, emax, nc, X):
    A = _fort(A, dtype)
    X = _fort(X, dtype)
    n, m0 = X.shape
    Q = np.zeros((n, m0), dtype=A.dtype, order="F")
    st = lib().or_filter_apply(_dt(dtype), n, _ptr(A), n, emin, emax, nc, _ptr(X), n, m0,
                               _ptr(Q), n)
    if st:
        raise RuntimeError(f"oracle filter_apply status {st}")
    return Q


def rayleigh_ritz(dtype, A, Q, emin, emax, anorm):
    A = _fort(A, dtype)
    Q = _fort(Q, dtype).copy(order="F")
    n, m0 = Q.shape
    lam = np.zeros(m0)
    res = np.zeros(m0)
    m = ctypes.c_int(0)
    st = lib().or_rayleigh_ritz(_dt(dtype), n, _ptr(A), n, _ptr(Q), n, m0, emin, emax, anorm,
                                _ptr(lam), _ptr(res), ctypes.byref(m))
    return dict(status=st, X=Q, lam=lam, res=res, m=m.value)


def feast_solve(dtype, A, emin, emax, nc, m0, tol, max_iter, anorm, X0, spurious=False):
    """spurious=True: only Ritz pairs inside I whose filter Rayleigh quotient exceeds 1/2
    count (see or_feast_solve_ex); the result then also carries 'mu'."""
    A = _fort(A, dtype)
    X0 = _fort(X0, dtype)
    n = A.shape[0]
    X = np.zeros((n, m0), dtype=A.dtype, order="F")
    lam = np.zeros(m0)
    res = np.zeros(m0)
    m = ctypes.c_int(0)
    iters = ctypes.c_int(0)
    trace = np.zeros(max_iter)
    mu = np.zeros(m0)
    st = lib().or_feast_solve_ex(_dt(dtype), n, _ptr(A), n, emin, emax, nc, m0, tol, max_iter,
                                 anorm, _ptr(X0), n, _ptr(X), n, _ptr(lam), _ptr(res),
                                 ctypes.byref(m), ctypes.byref(iters), _ptr(trace),
                                 int(spurious), _ptr(mu))
    out = dict(status=st, X=X, lam=lam, res=res, m=m.value, iters=iters.value,
               trace=trace[: iters.value])
    if spurious:
        out["mu"] = mu
    return out


def filter_apply_gen(dtype, A, B, emin, emax, nc, X):
    """Q = rho(B^{-1} A) X for the Hermitian-definite pencil (A, B)."""
    A = _fort(A, dtype)
    B = _fort(B, dtype)
    X = _fort(X, dtype)
    n, m0 = X.shape
    Q = np.zeros((n, m0), dtype=A.dtype, order="F")
    st = lib().or_filter_apply_gen(_dt(dtype), n, _ptr(A), n, _ptr(B), n, emin, emax, nc,
                                   _ptr(X), n, m0, _ptr(Q), n)
    if st:
        raise RuntimeError(f"oracle filter_apply_gen status {st}")
    return Q


def feast_solve_gen(dtype, A, B, emin, emax, nc, m0, tol, max_iter, anorm, X0, spurious=False):
    """FEAST on A x = lambda B x (B Hermitian positive definite); B=None is B = I.  Ritz
    vectors are B-normalized and res_k = ||A x_k - lambda_k B x_k|| / anorm."""
    A = _fort(A, dtype)
    X0 = _fort(X0, dtype)
    Bf = _fort(B, dtype) if B is not None else None
    n = A.shape[0]
    X = np.zeros((n, m0), dtype=A.dtype, order="F")
    lam = np.zeros(m0)
    res = np.zeros(m0)
    m = ctypes.c_int(0)
    iters = ctypes.c_int(0)
    trace = np.zeros(max_iter)
    mu = np.zeros(m0)
    st = lib().or_feast_solve_gen(_dt(dtype), n, _ptr(A), n,
                                  _ptr(Bf) if Bf is not None else None, n, emin, emax, nc, m0,
                                  tol, max_iter, anorm, _ptr(X0), n, _ptr(X), n, _ptr(lam),
                                  _ptr(res), ctypes.byref(m), ctypes.byref(iters), _ptr(trace),
                                  int(spurious), _ptr(mu))
    out = dict(status=st, X=X, lam=lam, res=res, m=m.value, iters=iters.value,
               trace=trace[: iters.value])
    if spurious:
        out["mu"] = mu
    return out


def select_pairs(lam, res, emin, emax, m0):
    """Indices of the m0 pairs the expanded-subspace methods keep (Sec. 2, Method 1)."""
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    res = np.ascontiguousarray(res, dtype=np.float64)
    sel = np.zeros(max(m0, 1), dtype=np.int32)
    k = lib().or_select_pairs(len(lam), _ptr(lam), _ptr(res), emin, emax, m0,
                              sel.ctypes.data_as(_ip))
    return sel[:k]


def xrfeast_solve(variant, dtype, A, emin, emax, nc, m0, s, tol, max_iter, anorm, X0,
                  spurious=False):
    """variant "x" = XFEAST, "r" = RFEAST (Sec. 2, Appendix boxes); s = blocks in the window
    (XFEAST) or Rayleigh-Ritz steps per filter application (RFEAST)."""
    A = _fort(A, dtype)
    X0 = _fort(X0, dtype)
    n = A.shape[0]
    X = np.zeros((n, m0), dtype=A.dtype, order="F")
    lam = np.zeros(m0)
    res = np.zeros(m0)
    m = ctypes.c_int(0)
    iters = ctypes.c_int(0)
    trace = np.zeros(max_iter)
    mu = np.zeros(m0)
    st = lib().or_xrfeast_solve({"x": 1, "r": 2}[variant], _dt(dtype), n, _ptr(A), n, emin,
                                emax, nc, m0, s, tol, max_iter, anorm, _ptr(X0), n, _ptr(X), n,
                                _ptr(lam), _ptr(res), ctypes.byref(m), ctypes.byref(iters),
                                _ptr(trace), int(spurious), _ptr(mu))
    return dict(status=st, X=X, lam=lam, res=res, m=m.value, iters=iters.value,
                trace=trace[: iters.value], mu=mu)
