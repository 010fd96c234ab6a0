"""The allocation-free filter entry point (include/feast_noalloc.h) against feast_filter_apply
(FP64) on the same inputs, through the C-ABI: two calls in a row, the second with a smaller
problem (the static scratch array keeps the first call's contents), for complex Hermitian and
real symmetric A; and the size limit is reported before any device work."""
import ctypes

import numpy as np
import pytest

from paper_1605_08771_amd import gen

pytestmark = pytest.mark.gpu

_vp = ctypes.c_void_p


def _lib():
    import paper_1605_08771_amd as fm
    L = fm.lib()
    L.feast_filter_apply_noalloc.argtypes = [ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int,
                                             ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                             _vp, ctypes.c_int, ctypes.c_int, _vp,
                                             ctypes.c_int, _vp]
    return L


def _noalloc(A, X, emin, emax, n_c, stream):
    import torch
    import paper_1605_08771_amd as fm
    n, m0 = X.shape
    Q = fm.fortran(torch.full((n, m0), float("nan"), dtype=X.dtype, device=X.device))
    dt = 1 if A.dtype == torch.complex128 else 0
    st = _lib().feast_filter_apply_noalloc(dt, n, _vp(A.data_ptr()), A.stride(1), emin, emax,
                                           n_c, _vp(X.data_ptr()), X.stride(1), m0,
                                           _vp(Q.data_ptr()), Q.stride(1),
                                           _vp(stream.cuda_stream))
    return st, Q


@pytest.mark.parametrize("complex_", [True, False])
def test_noalloc_filter_matches_filter_apply(complex_):
    import torch
    import paper_1605_08771_amd as fm
    assert torch.cuda.is_available(), "GPU tests need the HIP device"
    f = fm.Feast()
    stream = torch.cuda.current_stream()
    try:
        # first a larger problem (several 128-row sweep blocks and a ragged tail), then a
        # smaller one (64-row blocks) that reuses the same scratch array
        for n, m0, n_c, tag in ((900, 96, 8, 1), (300, 40, 6, 2)):
            rng = gen.rng_for([7007, n, int(complex_)])
            lam = gen.uniform_spectrum(rng, n, -0.1, 0.1)
            p = gen.make_problem(lam, -0.1, 0.1, m0, n_c, 1e-12, 10, complex_, rng)
            A = fm.fortran(torch.from_numpy(p.A).cuda())
            X = fm.fortran(torch.from_numpy(p.X0).cuda())
            f.invalidate()
            st_ref, Qref = f.filter_apply(A, X, p.emin, p.emax, n_c)
            st, Q = _noalloc(A, X, p.emin, p.emax, n_c, stream)
            torch.cuda.synchronize()
            assert st_ref == 0 and st == 0, (st_ref, st)
            ref = Qref.cpu().numpy()
            got = Q.cpu().numpy()
            err = np.abs(got - ref).max() / np.abs(ref).max()
            assert err < 1e-11, (n, err)
    finally:
        f.close()


def test_noalloc_rejects_sizes_beyond_the_scratch():
    import torch
    import paper_1605_08771_amd as fm
    n = 4096  # factors alone: 8 * 4096^2 * 16 B = 2 GiB > 256 MiB
    A = fm.fortran(torch.zeros((n, n), dtype=torch.complex128, device="cuda"))
    X = fm.fortran(torch.zeros((n, 8), dtype=torch.complex128, device="cuda"))
    st, _ = _noalloc(A, X, -0.1, 0.1, 8, torch.cuda.current_stream())
    assert st == -103
