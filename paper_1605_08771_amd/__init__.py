"""Python binding of libfeast_mi355x.so (the MI355X FEAST hot path, include/feast.h).

Argument marshalling only: device arrays are torch tensors on a HIP device, passed to the
C-ABI by pointer; every step of the computation runs in the library's kernels.  Matrices
must be column-major (torch stride (1, ld)); `fortran(t)` makes such a copy.  dtype is
chosen from the tensor: float64 -> FEAST_R64 (real symmetric), complex128 -> FEAST_C128
(complex Hermitian).

There is no CPU fallback: if the shared library is missing, `lib()` raises.
"""
from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfeast_mi355x.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "feast.h")

FEAST_R64, FEAST_C128 = 0, 1
FEAST_FP64, FEAST_FP32_IR, FEAST_BF16X3_IR = 0, 1, 2
STATUS = {0: "OK", 1: "NOT_CONVERGED", 2: "M0_TOO_SMALL", 3: "NO_EIGENVALUES",
          4: "B_NOT_SPD", 5: "NONFINITE", 6: "ZERO_PIVOT", 7: "EIG_FAILED", -100: "ERR_ALLOC",
          -101: "ERR_HIP", -102: "ERR_UNSUPPORTED"}
KCLASS = {"lu": 0, "solve": 1, "rr": 2, "refine": 3, "other": 4, "eig": 5}


METHODS = {"feast": 0, "xfeast": 1, "rfeast": 2}


class FeastOpts(ctypes.Structure):
    _fields_ = [("n_c", ctypes.c_int), ("m0", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("refine_max", ctypes.c_int), ("tol", ctypes.c_double),
                ("anorm", ctypes.c_double), ("prec", ctypes.c_int),
                ("seed", ctypes.c_ulonglong), ("spurious", ctypes.c_int),
                ("method", ctypes.c_int), ("expand", ctypes.c_int)]


class FeastSolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("filter_applications", ctypes.c_int),
                ("counted", ctypes.c_int), ("max_res", ctypes.c_double),
                ("time_ms", ctypes.c_double), ("filter_columns", ctypes.c_longlong)]


class FeastProblem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("lda", ctypes.c_int), ("ldx", ctypes.c_int),
                ("m0", ctypes.c_int), ("A", ctypes.c_void_p), ("emin", ctypes.c_double),
                ("emax", ctypes.c_double), ("anorm", ctypes.c_double), ("X0", ctypes.c_void_p),
                ("X", ctypes.c_void_p), ("lambda_", ctypes.POINTER(ctypes.c_double)),
                ("res", ctypes.POINTER(ctypes.c_double)), ("m", ctypes.POINTER(ctypes.c_int)),
                ("iters", ctypes.POINTER(ctypes.c_int)), ("status", ctypes.POINTER(ctypes.c_int)),
                ("mu", ctypes.POINTER(ctypes.c_double)),
                ("counted", ctypes.POINTER(ctypes.c_int)),
                ("trace", ctypes.POINTER(ctypes.c_double)),
                ("info", ctypes.POINTER(FeastSolveInfo))]


_lib = None
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def header_functions():
    """Names of the functions declared in include/feast.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(feast_[a-z_0-9]+)\s*\(", txt)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        L.feast_create.argtypes = [ctypes.POINTER(_vp), _vp]
        L.feast_destroy.argtypes = [_vp]
        L.feast_status_string.argtypes = [ctypes.c_int]
        L.feast_status_string.restype = ctypes.c_char_p
        L.feast_last_error.argtypes = [_vp]
        L.feast_last_error.restype = ctypes.c_char_p
        L.feast_invalidate.argtypes = [_vp]
        L.feast_invalidate.restype = None
        L.feast_filter_apply.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                         ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, _vp,
                                         ctypes.c_int]
        L.feast_rayleigh_ritz.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int,
                                          _vp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, _dp, _dp, _ip]
        L.feast_solve.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int,
                                  ctypes.c_double, ctypes.c_double, ctypes.POINTER(FeastOpts),
                                  _vp, _vp, ctypes.c_int, _dp, _dp, _ip, _ip, _dp]
        L.feast_solve_gen.argtypes = L.feast_solve.argtypes[:5] + [_vp, ctypes.c_int] + \
            L.feast_solve.argtypes[5:]
        L.feast_filter_apply_gen.argtypes = L.feast_filter_apply.argtypes[:5] + \
            [_vp, ctypes.c_int] + L.feast_filter_apply.argtypes[5:]
        L.feast_get_timings.argtypes = [_vp, _dp, ctypes.c_int]
        L.feast_get_filter_values.argtypes = [_vp, _dp, ctypes.c_int]
        L.feast_get_solve_info.argtypes = [_vp, ctypes.POINTER(FeastSolveInfo), _ip,
                                           ctypes.c_int]
        L.feast_solve_batched.argtypes = [_vp, ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(FeastProblem), ctypes.POINTER(FeastOpts),
                                          ctypes.c_int]
        L.feast_set_profiling.argtypes = [_vp, ctypes.c_int]
        L.feast_get_kernel_stats.argtypes = [_vp, ctypes.c_int, _dp,
                                             ctypes.POINTER(ctypes.c_longlong), _dp]
        ci, cl = ctypes.c_int, ctypes.c_long
        L.feast_kern_gemm.argtypes = [ci, ci, ci, ci, ci, ci, _dp, _vp, cl, _vp, cl, _dp, _vp,
                                      cl, _vp]
        L.feast_kern_lu.argtypes = [ci, _vp, ci, ci, ci, _dp, _vp, _ip, _ip, _vp]
        L.feast_kern_jacobi.argtypes = [_vp, ci, _vp, _vp, _vp]
        L.feast_tune_sweep_block.argtypes = [ci]
        L.feast_tune_split_filter.argtypes = [ci]
        L.feast_kern_sweeps.argtypes = [ci, ci, ci, ci, ci, _vp, _vp, _vp, ci, _vp, _vp, _ip,
                                        _ip, _vp]
        _lib = L
    return _lib


def tune_sweep_block(nbt):
    """Process-wide sweep block height for later factorizations (64, 128, 256 or 512; 0: the
    built-in tuned table).  Set it only while no solve is running."""
    st = lib().feast_tune_sweep_block(int(nbt))
    if st != 0:
        raise ValueError(f"sweep block height must be 0, 64, 128, 256 or 512, not {nbt}")


def tune_split_filter(mode):
    """Process-wide test hook: 1 splits every filter application made for the filter-value
    test into the Ritz vectors inside I and the rest (0, the default: only at a likely last
    iteration).  Both give the same iterates.  Set it only while no solve is running."""
    st = lib().feast_tune_split_filter(int(mode))
    if st != 0:
        raise ValueError(f"split-filter mode must be 0 or 1, not {mode}")


def fortran(t):
    """Column-major copy of a 2-D torch tensor (stride (1, rows))."""
    return t.mT.contiguous().mT


def _ld(t, name):
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    if t.numel() == 0:
        return max(1, t.shape[0])
    if t.shape[1] == 1:  # a one-column tensor's column stride carries no layout (torch sets 1)
        if t.stride(0) != 1 and t.shape[0] > 1:
            raise ValueError(f"{name} must be column-major (use fortran(t))")
        if t.device.type != "cuda":
            raise ValueError(f"{name} must live on the HIP device")
        return max(1, t.shape[0])
    if t.stride(0) != 1 or t.stride(1) < max(1, t.shape[0]):
        raise ValueError(f"{name} must be column-major (use fortran(t))")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the HIP device")
    return t.stride(1)


def _need(t, name, dtype, rows=None, cols=None):
    """Refuse a tensor whose dtype, rank or shape does not match what the C-ABI will read or
    write (the library trusts its pointers and sizes)."""
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    if rows is not None and t.shape[0] < rows:
        raise ValueError(f"{name} has {t.shape[0]} rows, needs {rows}")
    if cols is not None and t.shape[1] < cols:
        raise ValueError(f"{name} has {t.shape[1]} columns, needs {cols}")


def _square(A, name="A"):
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError(f"{name} must be square")
    return A.shape[0]


def _dtype_code(t):
    import torch
    if t.dtype == torch.complex128:
        return FEAST_C128
    if t.dtype == torch.float64:
        return FEAST_R64
    raise TypeError("A must be float64 (real symmetric) or complex128 (Hermitian)")


class FeastError(RuntimeError):
    def __init__(self, code, where, msg=""):
        super().__init__(f"{where}: status {code} ({STATUS.get(code, 'invalid argument')}) {msg}")
        self.code = code


class Feast:
    """One library handle bound to the current torch stream of the current device."""

    def __init__(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        h = _vp()
        st = lib().feast_create(ctypes.byref(h), _vp(stream.cuda_stream))
        if st != 0:
            raise FeastError(st, "feast_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().feast_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self):
        return lib().feast_last_error(self.h).decode()

    def invalidate(self):
        lib().feast_invalidate(self.h)

    # ---------------------------------------------------------------- entry points
    def filter_apply(self, A, X, emin, emax, n_c, prec=FEAST_FP64, Q=None):
        import torch
        dt = _dtype_code(A)
        n = _square(A)
        _need(X, "X", A.dtype, rows=n)
        lda, ldx = _ld(A, "A"), _ld(X, "X")
        m0 = X.shape[1]
        if Q is None:
            Q = fortran(torch.empty((n, m0), dtype=X.dtype, device=X.device))
        _need(Q, "Q", A.dtype, rows=n, cols=m0)
        ldq = _ld(Q, "Q")
        st = lib().feast_filter_apply(self.h, dt, n, _vp(A.data_ptr()), lda, emin, emax, n_c,
                                      prec, _vp(X.data_ptr()), ldx, m0, _vp(Q.data_ptr()), ldq)
        return st, Q

    def rayleigh_ritz(self, A, Q, emin, emax, anorm):
        """Q is overwritten by the Ritz vectors. Returns (status, lam, res, m)."""
        import numpy as np
        dt = _dtype_code(A)
        n = _square(A)
        _need(Q, "Q", A.dtype, rows=n)
        lda, ldq = _ld(A, "A"), _ld(Q, "Q")
        m0 = Q.shape[1]
        lam = np.zeros(m0)
        res = np.zeros(m0)
        m = ctypes.c_int(0)
        st = lib().feast_rayleigh_ritz(self.h, dt, n, _vp(A.data_ptr()), lda,
                                       _vp(Q.data_ptr()), ldq, m0, emin, emax, anorm,
                                       lam.ctypes.data_as(_dp), res.ctypes.data_as(_dp),
                                       ctypes.byref(m))
        return st, lam, res, m.value

    def solve(self, A, emin, emax, m0, n_c=8, tol=1e-12, max_iter=50, anorm=0.0,
              prec=FEAST_FP64, refine_max=4, X0=None, seed=0, X=None, spurious=False,
              method="feast", expand=1):
        """method: "feast", "xfeast" or "rfeast" (expand = blocks kept / Rayleigh-Ritz steps
        per filter application)."""
        import numpy as np
        import torch
        dt = _dtype_code(A)
        lda = _ld(A, "A")
        n = _square(A)
        if X is None:
            X = fortran(torch.empty((n, m0), dtype=A.dtype, device=A.device))
        _need(X, "X", A.dtype, rows=n, cols=m0)
        ldx = _ld(X, "X")
        if X0 is not None:
            _need(X0, "X0", A.dtype, rows=n, cols=m0)
            if _ld(X0, "X0") != ldx:
                raise ValueError("X0 and X must share the leading dimension")
        opts = FeastOpts(n_c=n_c, m0=m0, max_iter=max_iter, refine_max=refine_max, tol=tol,
                         anorm=anorm, prec=prec, seed=seed, spurious=int(spurious),
                         method=METHODS[method], expand=expand)
        lam = np.zeros(m0)
        res = np.zeros(m0)
        trace = np.zeros(max_iter)
        m = ctypes.c_int(0)
        iters = ctypes.c_int(0)
        st = lib().feast_solve(self.h, dt, n, _vp(A.data_ptr()), lda, emin, emax,
                               ctypes.byref(opts), _vp(X0.data_ptr()) if X0 is not None else None,
                               _vp(X.data_ptr()), ldx, lam.ctypes.data_as(_dp),
                               res.ctypes.data_as(_dp), ctypes.byref(m), ctypes.byref(iters),
                               trace.ctypes.data_as(_dp))
        out = dict(status=st, X=X, lam=lam, res=res, m=m.value, iters=iters.value,
                   trace=trace[: iters.value])
        self._outcome(out, m0)
        if spurious or prec != FEAST_FP64:
            mu = np.zeros(m0)
            lib().feast_get_filter_values(self.h, mu.ctypes.data_as(_dp), m0)
            out["mu"] = mu
        return out

    def _outcome(self, out, m0):
        """The library's step-3 decision and counts for the last solve on this handle."""
        import numpy as np
        info = FeastSolveInfo()
        counted = np.zeros(m0, dtype=np.int32)
        lib().feast_get_solve_info(self.h, ctypes.byref(info), counted.ctypes.data_as(_ip), m0)
        out["counted"] = np.flatnonzero(counted)
        out["filter_applications"] = info.filter_applications
        out["filter_columns"] = info.filter_columns
        out["time_ms"] = info.time_ms

    def filter_apply_gen(self, A, B, X, emin, emax, n_c, Q=None):
        """Q = rho(B^{-1} A) X for the Hermitian-definite pencil (A, B) (FP64)."""
        import torch
        dt = _dtype_code(A)
        n = _square(A)
        _need(B, "B", A.dtype, rows=n, cols=n)
        _need(X, "X", A.dtype, rows=n)
        lda, ldb, ldx = _ld(A, "A"), _ld(B, "B"), _ld(X, "X")
        m0 = X.shape[1]
        if Q is None:
            Q = fortran(torch.empty((n, m0), dtype=X.dtype, device=X.device))
        _need(Q, "Q", A.dtype, rows=n, cols=m0)
        ldq = _ld(Q, "Q")
        st = lib().feast_filter_apply_gen(self.h, dt, n, _vp(A.data_ptr()), lda,
                                          _vp(B.data_ptr()), ldb, emin, emax, n_c, FEAST_FP64,
                                          _vp(X.data_ptr()), ldx, m0, _vp(Q.data_ptr()), ldq)
        return st, Q

    def solve_gen(self, A, B, emin, emax, m0, n_c=8, tol=1e-12, max_iter=50, anorm=0.0,
                  X0=None, seed=0, X=None, spurious=False):
        """FEAST on A x = lambda B x (B Hermitian positive definite), FP64.  Ritz vectors are
        B-normalized; res_k = ||A x_k - lambda_k B x_k|| / anorm."""
        import numpy as np
        import torch
        dt = _dtype_code(A)
        n = _square(A)
        _need(B, "B", A.dtype, rows=n, cols=n)
        lda, ldb = _ld(A, "A"), _ld(B, "B")
        if X is None:
            X = fortran(torch.empty((n, m0), dtype=A.dtype, device=A.device))
        _need(X, "X", A.dtype, rows=n, cols=m0)
        ldx = _ld(X, "X")
        if X0 is not None:
            _need(X0, "X0", A.dtype, rows=n, cols=m0)
            if _ld(X0, "X0") != ldx:
                raise ValueError("X0 and X must share the leading dimension")
        opts = FeastOpts(n_c=n_c, m0=m0, max_iter=max_iter, refine_max=0, tol=tol, anorm=anorm,
                         prec=FEAST_FP64, seed=seed, spurious=int(spurious))
        lam, res, trace = np.zeros(m0), np.zeros(m0), np.zeros(max_iter)
        m, iters = ctypes.c_int(0), ctypes.c_int(0)
        st = lib().feast_solve_gen(self.h, dt, n, _vp(A.data_ptr()), lda, _vp(B.data_ptr()), ldb,
                                   emin, emax, ctypes.byref(opts),
                                   _vp(X0.data_ptr()) if X0 is not None else None,
                                   _vp(X.data_ptr()), ldx, lam.ctypes.data_as(_dp),
                                   res.ctypes.data_as(_dp), ctypes.byref(m), ctypes.byref(iters),
                                   trace.ctypes.data_as(_dp))
        out = dict(status=st, X=X, lam=lam, res=res, m=m.value, iters=iters.value,
                   trace=trace[: iters.value])
        self._outcome(out, m0)
        if spurious:
            mu = np.zeros(m0)
            lib().feast_get_filter_values(self.h, mu.ctypes.data_as(_dp), m0)
            out["mu"] = mu
        return out

    def solve_batched(self, problems, n_c=8, tol=1e-12, max_iter=200, prec=FEAST_FP64,
                      refine_max=0, spurious=False, nstreams=8):
        """problems: list of dicts with A, emin, emax, m0 and optional anorm, X0 (device,
        column-major, one dtype for all).  Returns (count_not_ok, list of result dicts)."""
        import numpy as np
        import torch
        if not problems:
            return 0, []
        dt = _dtype_code(problems[0]["A"])
        arr = (FeastProblem * len(problems))()
        keep = []
        outs = []
        for i, pr in enumerate(problems):
            A = pr["A"]
            if _dtype_code(A) != dt:
                raise TypeError("all problems of a batch must share one dtype")
            n = _square(A)
            m0 = pr["m0"]
            X = fortran(torch.empty((n, m0), dtype=A.dtype, device=A.device))
            lam, res, mu = np.zeros(m0), np.zeros(m0), np.zeros(m0)
            counted, trace = np.zeros(m0, dtype=np.int32), np.zeros(max_iter)
            info = FeastSolveInfo()
            m, it, st = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(-999)
            X0 = pr.get("X0")
            if X0 is not None:
                _need(X0, "X0", A.dtype, rows=n, cols=m0)
                if _ld(X0, "X0") != _ld(X, "X"):
                    raise ValueError("X0 must be column-major with leading dimension n")
            arr[i] = FeastProblem(n=n, lda=_ld(A, "A"), ldx=_ld(X, "X"), m0=m0,
                                  A=A.data_ptr(), emin=pr["emin"], emax=pr["emax"],
                                  anorm=pr.get("anorm", 0.0),
                                  X0=X0.data_ptr() if X0 is not None else None,
                                  X=X.data_ptr(), lambda_=lam.ctypes.data_as(_dp),
                                  res=res.ctypes.data_as(_dp), m=ctypes.pointer(m),
                                  iters=ctypes.pointer(it), status=ctypes.pointer(st),
                                  mu=mu.ctypes.data_as(_dp),
                                  counted=counted.ctypes.data_as(_ip),
                                  trace=trace.ctypes.data_as(_dp), info=ctypes.pointer(info))
            keep += [X, lam, res, m, it, st, mu, counted, trace, info]
            outs.append((X, lam, res, m, it, st, mu, counted, trace, info))
        opts = FeastOpts(n_c=n_c, m0=1, max_iter=max_iter, refine_max=refine_max, tol=tol,
                         anorm=0.0, prec=prec, seed=0, spurious=int(spurious))
        torch.cuda.synchronize()
        bad = lib().feast_solve_batched(self.h, dt, len(problems), arr, ctypes.byref(opts),
                                        nstreams)
        results = [dict(status=st.value, X=X, lam=lam, res=res, m=m.value, iters=it.value,
                        mu=mu, counted=np.flatnonzero(counted), trace=trace[: it.value],
                        filter_applications=info.filter_applications,
                        filter_columns=info.filter_columns, time_ms=info.time_ms)
                   for (X, lam, res, m, it, st, mu, counted, trace, info) in outs]
        return bad, results

    def solve_slices(self, A, edges, m0, anorm=0.0, X0=None, n_c=8, tol=1e-12, max_iter=200,
                     prec=FEAST_FP64, refine_max=0, spurious=True, nstreams=8):
        """Eigenpairs of one matrix A in the open slices (edges[k], edges[k+1]), solved as
        independent intervals (Sec. 1) on concurrent streams.  m0: one size for all slices or
        one per slice; X0: None (seeded starts) or one start block per slice.  Returns
        (count_not_ok, per-slice results, eigenvalues of all slices in ascending order).  The
        pairs of a slice are those the library's step 3 counted for it ("counted"); each
        slice's result also carries its residual trace, iteration count, filter applications
        and solve time, so the imbalance between slices of uneven spectral density shows."""
        import numpy as np
        edges = [float(e) for e in edges]
        if len(edges) < 2 or any(b <= a for a, b in zip(edges, edges[1:])):
            raise ValueError("edges must increase")
        k = len(edges) - 1
        m0s = list(m0) if hasattr(m0, "__len__") else [int(m0)] * k
        if len(m0s) != k:
            raise ValueError("one m0 per slice")
        probs = []
        for i in range(k):
            pr = dict(A=A, emin=edges[i], emax=edges[i + 1], m0=m0s[i], anorm=anorm)
            if X0 is not None:
                pr["X0"] = X0[i]
            probs.append(pr)
        bad, outs = self.solve_batched(probs, n_c=n_c, tol=tol, max_iter=max_iter, prec=prec,
                                       refine_max=refine_max, spurious=spurious,
                                       nstreams=nstreams)
        found = [o["lam"][o["counted"]] for o in outs]
        return bad, outs, np.sort(np.concatenate(found)) if found else np.zeros(0)

    # ---------------------------------------------------------------- building blocks
    def gemm(self, opA, opB, A, B, C, alpha=1.0, beta=0.0, M=None, N=None, K=None,
             split_bf16=False, three_products=False):
        """C = alpha op(A) op(B) + beta C on the matrix cores (complex128 or complex64;
        split_bf16 with complex64: bf16x3 products with FP32 accumulation; three_products with
        complex128: each complex product from three real FP64 products)."""
        import torch
        if A.dtype not in (torch.complex128, torch.complex64):
            raise TypeError("gemm takes complex128 or complex64 operands")
        if split_bf16 and A.dtype != torch.complex64:
            raise TypeError("split_bf16 takes complex64 operands")
        if three_products and A.dtype != torch.complex128:
            raise TypeError("three_products selects the FP64 form (complex128 operands)")
        prec = (3 if three_products else 0) if A.dtype == torch.complex128 else \
            (2 if split_bf16 else 1)
        M = C.shape[0] if M is None else M
        N = C.shape[1] if N is None else N
        if K is None:
            K = A.shape[1] if opA == 0 else A.shape[0]
        if K > 0:
            _need(A, "A", A.dtype, *((M, K) if opA == 0 else (K, M)))
            _need(B, "B", A.dtype, *((K, N) if opB == 0 else (N, K)))
        _need(C, "C", A.dtype, M, N)
        lda, ldb, ldc = _ld(A, "A"), _ld(B, "B"), _ld(C, "C")
        al = (ctypes.c_double * 2)(complex(alpha).real, complex(alpha).imag)
        be = (ctypes.c_double * 2)(complex(beta).real, complex(beta).imag)
        st = lib().feast_kern_gemm(prec, opA, opB, M, N, K, al, _vp(A.data_ptr()), lda,
                                   _vp(B.data_ptr()), ldb, be, _vp(C.data_ptr()), ldc,
                                   _vp(self._stream.cuda_stream))
        return st

    def lu(self, A, z, prec=0, column_steps=False):
        """Factors of z_j I - A for the nodes z (numpy complex array); prec 0 FP64, 1 FP32,
        2 FP32 with bf16x3 trailing updates; column_steps: one launch per panel column
        throughout (the reference schedule of the short-panel groups).  Returns (status,
        LU [nc, np, np] tensor in column-major blocks, perm [nc, np])."""
        import numpy as np
        import torch
        _need(A, "A", torch.complex128)
        n = _square(A)
        lda = _ld(A, "A")
        zz = np.ascontiguousarray(np.asarray(z, dtype=np.complex128)).view(np.float64)
        nc = len(zz) // 2
        npo = ctypes.c_int()
        lib().feast_kern_lu(prec, _vp(A.data_ptr()), lda, n, nc, zz.ctypes.data_as(_dp), None,
                            None, ctypes.byref(npo), None)
        np_ = npo.value
        dt = torch.complex128 if prec == 0 else torch.complex64
        LU = torch.empty((nc, np_, np_), dtype=dt, device=A.device)
        perm = torch.empty((nc, np_), dtype=torch.int32, device=A.device)
        st = lib().feast_kern_lu(prec | (8 if column_steps else 0), _vp(A.data_ptr()), lda, n,
                                 nc, zz.ctypes.data_as(_dp),
                                 _vp(LU.data_ptr()), ctypes.cast(ctypes.c_void_p(perm.data_ptr()), _ip),
                                 None, _vp(self._stream.cuda_stream))
        # blocks are column-major: element (r, c) of node j at LU[j].flatten()[r + c*np]
        return st, LU.transpose(1, 2), perm

    def sweep_shape(self, n, prec=0):
        """(np, nbt): the padded order and sweep block height the solver uses for order n."""
        npo, nbo = ctypes.c_int(), ctypes.c_int()
        st = lib().feast_kern_sweeps(prec, n, 1, 1, 1, None, None, None, 0, None, None,
                                     ctypes.byref(npo), ctypes.byref(nbo), None)
        if st != 0:
            raise ValueError(f"feast_kern_sweeps returned {st}")
        return npo.value, nbo.value

    def sweeps(self, LU, B, n, sides, invL=None, invU=None, prec=0):
        """The solver's block sweeps on factors LU [nc, np, np] (as lu() returns them) for
        right-hand sides B [nc, sides, m0, np] (each block column-major, modified in place:
        side 0 -> (L U)^{-1} B_0, side 1 -> (L U)^{-H} B_1).  The diagonal-block inverses are
        computed here unless invL and invU [nc, nbt, np] are given.  Returns the status."""
        import torch
        nc = LU.shape[0]
        np_, nbt = self.sweep_shape(n, prec)
        m0 = B.shape[2]
        dt = torch.complex128 if prec == 0 else torch.complex64
        if tuple(LU.shape) != (nc, np_, np_) or LU.dtype != dt:
            raise ValueError("LU must be [nc, np, np] of the precision's dtype")
        if tuple(B.shape) != (nc, sides, m0, np_) or B.dtype != dt or not B.is_contiguous():
            raise ValueError("B must be a contiguous [nc, sides, m0, np] tensor")
        comp = invL is None
        if comp:
            invL = torch.empty((nc, nbt, np_), dtype=dt, device=LU.device)
            invU = torch.empty_like(invL)
        Z = torch.empty_like(B)
        # lu() hands back column-major blocks as transposed views of contiguous storage
        base = LU.transpose(1, 2)
        if not base.is_contiguous():
            raise ValueError("LU must be the column-major blocks lu() returns")
        return lib().feast_kern_sweeps(prec, n, nc, m0, sides, _vp(base.data_ptr()),
                                       _vp(invL.data_ptr()), _vp(invU.data_ptr()), int(comp),
                                       _vp(B.data_ptr()), _vp(Z.data_ptr()), None, None,
                                       _vp(self._stream.cuda_stream))

    def jacobi(self, H):
        import torch
        _need(H, "H", torch.complex128)
        m = _square(H, "H")
        if H.device.type != "cuda":
            raise ValueError("H must live on the HIP device")
        Hf = fortran(H)
        d = torch.empty(m, dtype=torch.float64, device=H.device)
        W = fortran(torch.empty((m, m), dtype=H.dtype, device=H.device))
        sweeps = lib().feast_kern_jacobi(_vp(Hf.data_ptr()), m, _vp(d.data_ptr()),
                                         _vp(W.data_ptr()), _vp(self._stream.cuda_stream))
        return sweeps, d, W

    # ---------------------------------------------------------------- measurement
    def timings(self):
        out = (ctypes.c_double * 6)()
        lib().feast_get_timings(self.h, out, 6)
        keys = ["factor_ms", "solve_ms", "accumulate_ms", "rr_ms", "refine_ms", "total_ms"]
        return dict(zip(keys, list(out)))

    def set_profiling(self, on=True):
        lib().feast_set_profiling(self.h, int(on))

    def kernel_stats(self, kclass):
        ms = ctypes.c_double(0)
        n = ctypes.c_longlong(0)
        fl = ctypes.c_double(0)
        lib().feast_get_kernel_stats(self.h, KCLASS[kclass], ctypes.byref(ms), ctypes.byref(n),
                                     ctypes.byref(fl))
        return dict(ms=ms.value, launches=n.value, dense_flops=fl.value)
