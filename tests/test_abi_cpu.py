"""Host-side checks of the C-ABI library that need no GPU: it loads, exports every function
declared in include/*.h, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import pytest

import paper_1605_08771_amd as fm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(feast_[a-z_0-9]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = fm.lib()
    names = _declared()
    assert "feast_solve" in names and "feast_filter_apply" in names
    assert "feast_rayleigh_ritz" in names
    for name in names:
        assert hasattr(L, name), name


def test_status_strings():
    L = fm.lib()
    for code in (0, 1, 2, 3, 4, 5, 6, 7, -100, -101, -102, -103, -3):
        assert len(L.feast_status_string(code)) > 0


BAD = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first
DEV = ctypes.c_void_p(0x2000)


def test_filter_apply_argument_checks():
    L = fm.lib()
    f = L.feast_filter_apply
    ok = dict(h=BAD, dt=1, n=10, A=DEV, lda=10, emin=-1.0, emax=1.0, nc=8, prec=0, X=DEV,
              ldx=10, m0=4, Q=ctypes.c_void_p(0x3000), ldq=10)

    def call(**kw):
        a = dict(ok)
        a.update(kw)
        return f(a["h"], a["dt"], a["n"], a["A"], a["lda"], a["emin"], a["emax"], a["nc"],
                 a["prec"], a["X"], a["ldx"], a["m0"], a["Q"], a["ldq"])

    assert call(h=None) == -1
    assert call(dt=7) == -2
    assert call(n=0) == -3
    assert call(A=None) == -4
    assert call(lda=9) == -5
    assert call(emin=float("nan")) == -6
    assert call(emin=1.0, emax=1.0) == -7
    assert call(emin=2.0, emax=1.0) == -7
    assert call(nc=0) == -8
    assert call(prec=5) == -9
    assert call(X=None) == -10
    assert call(ldx=3) == -11
    assert call(m0=0) == -12
    assert call(m0=11) == -12
    assert call(Q=None) == -13
    assert call(Q=DEV) == -13  # aliasing X
    assert call(ldq=1) == -14


def test_rayleigh_ritz_argument_checks():
    L = fm.lib()
    f = L.feast_rayleigh_ritz
    lam = (ctypes.c_double * 4)()
    res = (ctypes.c_double * 4)()
    m = ctypes.c_int()
    dp = ctypes.POINTER(ctypes.c_double)
    args = [BAD, 1, 10, DEV, 10, DEV, 10, 4, -1.0, 1.0, 1.0, ctypes.cast(lam, dp),
            ctypes.cast(res, dp), ctypes.byref(m)]

    def call(i, v):
        a = list(args)
        a[i] = v
        return f(*a)

    assert call(0, None) == -1
    assert call(1, 3) == -2
    assert call(2, -1) == -3
    assert call(3, None) == -4
    assert call(4, 2) == -5
    assert call(5, None) == -6
    assert call(6, 5) == -7
    assert call(7, 0) == -8
    assert call(9, -1.0) == -10
    assert call(10, 0.0) == -11
    assert call(11, None) == -12
    assert call(12, None) == -13
    assert call(13, None) == -14


def test_solve_argument_checks():
    L = fm.lib()
    f = L.feast_solve
    lam = (ctypes.c_double * 8)()
    res = (ctypes.c_double * 8)()
    m = ctypes.c_int()
    it = ctypes.c_int()
    dp = ctypes.POINTER(ctypes.c_double)
    good = fm.FeastOpts(n_c=8, m0=4, max_iter=10, refine_max=2, tol=1e-12, anorm=1.0, prec=0,
                        seed=1)

    def call(opts=good, **kw):
        a = dict(h=BAD, dt=1, n=10, A=DEV, lda=10, emin=-1.0, emax=1.0, X0=None,
                 X=ctypes.c_void_p(0x3000), ldx=10)
        a.update(kw)
        return f(a["h"], a["dt"], a["n"], a["A"], a["lda"], a["emin"], a["emax"],
                 ctypes.byref(opts) if opts is not None else None, a["X0"], a["X"], a["ldx"],
                 ctypes.cast(lam, dp), ctypes.cast(res, dp), ctypes.byref(m), ctypes.byref(it),
                 None)

    assert call(h=None) == -1
    assert call(dt=2) == -2
    assert call(n=0) == -3
    assert call(A=None) == -4
    assert call(lda=4) == -5
    assert call(emax=-2.0) == -7
    assert call(opts=None) == -8
    for bad in (dict(n_c=0), dict(m0=0), dict(m0=11), dict(max_iter=0), dict(tol=0.0),
                dict(prec=9), dict(prec=3), dict(prec=1, refine_max=-1), dict(prec=2, refine_max=-1),
                dict(method=3), dict(method=-1),
                dict(method=1, expand=0), dict(method=2, expand=0), dict(method=1, expand=3),
                dict(method=2, expand=3)):
        o = fm.FeastOpts(n_c=8, m0=4, max_iter=10, refine_max=2, tol=1e-12, anorm=1.0, prec=0,
                         seed=1)
        for k, v in bad.items():
            setattr(o, k, v)
        assert call(opts=o) == -8, bad
    assert call(X=None) == -10
    assert call(ldx=2) == -11


def test_kernel_api_argument_checks():
    L = fm.lib()
    al = ctypes.cast((ctypes.c_double * 2)(1.0, 0.0), ctypes.POINTER(ctypes.c_double))
    assert L.feast_kern_gemm(4, 0, 0, 4, 4, 4, al, DEV, 4, DEV, 4, al, DEV, 4, None) == -1
    assert L.feast_kern_gemm(0, 5, 0, 4, 4, 4, al, DEV, 4, DEV, 4, al, DEV, 4, None) == -2
    assert L.feast_kern_gemm(0, 0, 0, 4, 4, 4, al, DEV, 3, DEV, 4, al, DEV, 4, None) == -9
    npo = ctypes.c_int()
    z = (ctypes.c_double * 2)(0.0, 1.0)
    assert L.feast_kern_lu(0, DEV, 500, 500, 1, ctypes.cast(z, ctypes.POINTER(ctypes.c_double)),
                           None, None, ctypes.byref(npo), None) == 0
    assert npo.value == 512
    zp = ctypes.cast(z, ctypes.POINTER(ctypes.c_double))
    for prec in (8, 9, 10):  # + 8: one launch per panel column (same factors)
        assert L.feast_kern_lu(prec, DEV, 500, 500, 1, zp, None, None, ctypes.byref(npo), None) == 0
    for prec in (3, 11, 16, -1):
        assert L.feast_kern_lu(prec, DEV, 500, 500, 1, zp, None, None, ctypes.byref(npo),
                               None) == -1
    assert L.feast_kern_jacobi(None, 4, None, None, None) == -1


def test_kern_sweeps_argument_checks_and_shape_query():
    L = fm.lib()
    npo, nbo = ctypes.c_int(), ctypes.c_int()

    def q(prec=0, n=300, nc=1, m0=4, sides=2):
        return L.feast_kern_sweeps(prec, n, nc, m0, sides, None, None, None, 0, None, None,
                                   ctypes.byref(npo), ctypes.byref(nbo), None)
    assert q(prec=3) == -1 and q(n=0) == -2 and q(nc=0) == -3 and q(m0=0) == -4
    assert q(sides=3) == -5
    for n in (1, 63, 300, 1000, 2100, 5000, 8192, 20000):
        for prec in (0, 1):
            assert q(prec=prec, n=n) == 0
            assert npo.value % nbo.value == 0 and npo.value >= n
            assert nbo.value == 64 or 8 * (npo.value - n) <= n
    assert L.feast_kern_sweeps(0, 300, 1, 4, 2, DEV, None, DEV, 0, DEV, DEV, None, None,
                               None) == -6
    assert L.feast_kern_sweeps(0, 300, 1, 4, 2, DEV, DEV, DEV, 0, DEV, DEV, None, None,
                               None) == -7


def test_split_filter_hook_argument_checks():
    """The split-filter test hook takes 0 or 1 and rejects anything else unchanged."""
    L = fm.lib()
    try:
        assert L.feast_tune_split_filter(2) == -1 and L.feast_tune_split_filter(-1) == -1
        assert L.feast_tune_split_filter(1) == 0
        with pytest.raises(ValueError):
            fm.tune_split_filter(3)
    finally:
        assert L.feast_tune_split_filter(0) == 0


def test_sweep_block_override():
    """The tuning hook: heights 64..512 change the padding the factorizations use; 0 restores
    the table; anything else is rejected and leaves the setting alone."""
    L = fm.lib()
    npo = ctypes.c_int()
    zp = ctypes.cast((ctypes.c_double * 2)(0.0, 1.0), ctypes.POINTER(ctypes.c_double))

    def np_for(n, prec=0):
        assert L.feast_kern_lu(prec, DEV, n, n, 1, zp, None, None, ctypes.byref(npo), None) == 0
        return npo.value
    try:
        base = np_for(300)
        assert base % 64 == 0 and 300 <= base <= 300 + 300 // 8  # padding rule of the table
        fm.tune_sweep_block(512)
        assert np_for(300) == 512 and np_for(300, 1) == 512
        assert L.feast_tune_sweep_block(100) == -1
        assert np_for(300) == 512
        fm.tune_sweep_block(64)
        assert np_for(300) == 320 and np_for(1000, 1) == 1024
        with pytest.raises(ValueError):
            fm.tune_sweep_block(1024)
    finally:
        fm.tune_sweep_block(0)
    assert np_for(300) == base


def test_binding_rejects_missing_library(monkeypatch, tmp_path):
    monkeypatch.setattr(fm, "_lib", None)
    monkeypatch.setattr(fm, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        fm.lib()


def test_batched_argument_checks():
    L = fm.lib()
    o = fm.FeastOpts(n_c=8, m0=4, max_iter=10, refine_max=0, tol=1e-12, anorm=1.0, prec=0, seed=1)
    arr = (fm.FeastProblem * 1)()
    f = L.feast_solve_batched
    assert f(None, 1, 1, arr, ctypes.byref(o), 4) == -1
    assert f(BAD, 5, 1, arr, ctypes.byref(o), 4) == -2
    assert f(BAD, 1, -1, arr, ctypes.byref(o), 4) == -3
    assert f(BAD, 1, 1, None, ctypes.byref(o), 4) == -4
    assert f(BAD, 1, 1, arr, None, 4) == -5
    assert f(BAD, 1, 1, arr, ctypes.byref(o), 0) == -6
    assert f(BAD, 1, 1, arr, ctypes.byref(o), 33) == -6
    assert f(BAD, 1, 0, arr, ctypes.byref(o), 4) == 0


def test_noalloc_argument_checks():
    """The allocation-free filter entry point validates its arguments and its scratch limit on
    the host, before any device work."""
    L = fm.lib()
    f = L.feast_filter_apply_noalloc
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                  ctypes.c_double, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                  ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    ok = dict(dt=1, n=100, A=DEV, lda=100, emin=-0.1, emax=0.1, n_c=8, X=DEV, ldx=100, m0=10,
              Q=BAD, ldq=100)

    def call(**kw):
        a = {**ok, **kw}
        return f(a["dt"], a["n"], a["A"], a["lda"], a["emin"], a["emax"], a["n_c"], a["X"],
                 a["ldx"], a["m0"], a["Q"], a["ldq"], None)
    assert call(dt=3) == -1
    assert call(n=0) == -2
    assert call(A=None) == -3
    assert call(lda=99) == -4
    assert call(emin=float("nan")) == -5
    assert call(emax=-0.2) == -6
    assert call(n_c=0) == -7
    assert call(X=None) == -8
    assert call(ldx=50) == -9
    assert call(m0=101) == -10
    assert call(Q=DEV) == -11
    assert call(ldq=1) == -12
    # 8 complex factors of order 4096 alone exceed the 256 MiB array
    assert call(n=4096, lda=4096, ldx=4096, ldq=4096) == -103
    assert b"scratch" in L.feast_status_string(-103)


def test_solve_info_argument_checks():
    L = fm.lib()
    info = fm.FeastSolveInfo()
    assert L.feast_get_solve_info(None, ctypes.byref(info), None, 0) == -1
    # the binding's structures have the C layout of include/feast.h (LP64: 136 and 40 bytes)
    assert ctypes.sizeof(fm.FeastProblem) == 136
    assert ctypes.sizeof(fm.FeastSolveInfo) == 40
    _check_layout_against_header(fm.FeastSolveInfo, "feast_solve_info")
    _check_layout_against_header(fm.FeastProblem, "feast_problem")


def _check_layout_against_header(cls, cname):
    """Sizes and field offsets of a binding structure equal those a C compiler gives the
    declaration in include/feast.h."""
    import os
    import shutil
    import subprocess
    import tempfile
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    names = [f[0] for f in cls._fields_]
    # a trailing underscore marks a C member named like a Python keyword (lambda)
    body = "".join(f'  printf("%zu\\n", offsetof({cname}, {n.rstrip("_")}));\n' for n in names)
    src = ("#include <stddef.h>\n#include <stdio.h>\n#include \"feast.h\"\nint main(void) {\n"
           f'  printf("%zu\\n", sizeof({cname}));\n' + body + "  return 0;\n}\n")
    with tempfile.TemporaryDirectory() as d:
        c, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        open(c, "w").write(src)
        subprocess.run([cc, "-I", inc, c, "-o", exe], check=True, capture_output=True)
        got = [int(v) for v in subprocess.run([exe], check=True, capture_output=True,
                                               text=True).stdout.split()]
    assert got[0] == ctypes.sizeof(cls)
    assert got[1:] == [getattr(cls, n).offset for n in names]


def test_binding_refuses_mismatched_tensors():
    """The C-ABI trusts pointers and sizes, so the binding refuses tensors whose dtype or shape
    differs from what the call will read or write (checked before any library call)."""
    import torch
    with pytest.raises(TypeError):
        fm._need(torch.zeros(4, 4, dtype=torch.float64), "H", torch.complex128)
    with pytest.raises(ValueError):
        fm._need(torch.zeros(3, 2, dtype=torch.complex128), "X", torch.complex128, rows=4)
    with pytest.raises(ValueError):
        fm._need(torch.zeros(4, 2, dtype=torch.complex128), "X", torch.complex128, cols=3)
    with pytest.raises(ValueError):
        fm._square(torch.zeros(4, 3, dtype=torch.complex128))
    fm._need(torch.zeros(4, 3, dtype=torch.complex128), "X", torch.complex128, rows=4, cols=3)
    with pytest.raises(TypeError):
        fm._dtype_code(torch.zeros(2, 2, dtype=torch.float32))


def test_pencil_entry_points_argument_checks():
    """feast_solve_gen / feast_filter_apply_gen reject bad arguments before any launch."""
    L = fm.lib()
    lam = (ctypes.c_double * 8)()
    res = (ctypes.c_double * 8)()
    m = ctypes.c_int()
    it = ctypes.c_int()
    dp = ctypes.POINTER(ctypes.c_double)
    good = fm.FeastOpts(n_c=8, m0=4, max_iter=10, refine_max=0, tol=1e-12, anorm=1.0, prec=0,
                        seed=1)

    def solve(opts=good, **kw):
        a = dict(h=BAD, dt=1, n=10, A=DEV, lda=10, B=DEV, ldb=10, emin=-1.0, emax=1.0, X0=None,
                 X=ctypes.c_void_p(0x3000), ldx=10)
        a.update(kw)
        return L.feast_solve_gen(a["h"], a["dt"], a["n"], a["A"], a["lda"], a["B"], a["ldb"],
                                 a["emin"], a["emax"],
                                 ctypes.byref(opts) if opts is not None else None, a["X0"],
                                 a["X"], a["ldx"], ctypes.cast(lam, dp), ctypes.cast(res, dp),
                                 ctypes.byref(m), ctypes.byref(it), None)

    assert solve(h=None) == -1
    assert solve(dt=3) == -2
    assert solve(B=None) == -6
    assert solve(ldb=9) == -7
    assert solve(emax=-3.0) == -9
    assert solve(opts=None) == -10
    for bad in (dict(prec=1), dict(method=1, expand=1), dict(m0=11)):
        o = fm.FeastOpts(n_c=8, m0=4, max_iter=10, refine_max=0, tol=1e-12, anorm=1.0, prec=0,
                         seed=1)
        for k, v in bad.items():
            setattr(o, k, v)
        assert solve(opts=o) == -10, bad
    assert solve(X=None) == -12

    def filt(**kw):
        a = dict(h=BAD, dt=1, n=10, A=DEV, lda=10, B=DEV, ldb=10, emin=-1.0, emax=1.0, nc=8,
                 prec=0, X=DEV, ldx=10, m0=4, Q=ctypes.c_void_p(0x3000), ldq=10)
        a.update(kw)
        return L.feast_filter_apply_gen(a["h"], a["dt"], a["n"], a["A"], a["lda"], a["B"],
                                        a["ldb"], a["emin"], a["emax"], a["nc"], a["prec"],
                                        a["X"], a["ldx"], a["m0"], a["Q"], a["ldq"])

    assert filt(B=None) == -6
    assert filt(prec=1) == -11
    assert filt(Q=DEV) == -15
    assert filt(ldq=3) == -16
