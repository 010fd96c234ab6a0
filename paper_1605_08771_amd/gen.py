"""Seeded synthetic inputs for the FEAST hot path (shared by the tests, the benchmark and the
smoke check).  This module holds no arithmetic of the eigensolver itself: it only draws
spectra, Haar-like unitary bases and Gaussian start blocks.

The matrices are A = U diag(lam) U^H (U from the QR factorization of a seeded Gaussian matrix,
complex for Hermitian problems, real for symmetric ones), so the exact eigenvalues are known.
Spectra follow the paper's hard case (Sec. 1 and Sec. 3 test matrices): eigenvalues packed
densely just outside the search interval, here within 1e-3 of each endpoint.

Random numbers come from numpy's PCG64 seeded with SeedSequence([1605, 8771, tag]); the draw
order is spectrum, then the Gaussian for U, then X0.  For the largest matrices built on the
device (n >= DEVICE_GAUSSIAN_N) the Gaussian for U is drawn by torch's device generator
(Philox), seeded by one 63-bit integer drawn from the same PCG64 stream at that point of the
order: drawing 2 n^2 normals on the host would dominate the set-up time.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

DELTA = 5e-5          # eigenvalues are kept at least this far from either endpoint
DEVICE_GAUSSIAN_N = 32768  # from this order on, the Gaussian for U is drawn on the device
EDGE_WIDTH = 1e-3     # width of the edge clusters just inside / just outside the interval


def rng_for(tag) -> np.random.Generator:
    tag = list(tag) if isinstance(tag, (list, tuple)) else [int(tag)]
    return np.random.default_rng(np.random.SeedSequence([1605, 8771] + [int(t) for t in tag]))


@dataclasses.dataclass
class Problem:
    n: int
    dtype: str            # "r64" (real symmetric) or "c128" (complex Hermitian)
    emin: float
    emax: float
    m0: int
    n_c: int
    tol: float
    max_iter: int
    lam: np.ndarray        # exact eigenvalues, ascending order not implied
    m_true: int            # eigenvalues strictly inside (emin, emax)
    anorm: float           # ||A||_2 = max |lam|
    A: object = None       # numpy (CPU) or torch tensor (device), column-major values
    U: object = None
    X0: object = None
    name: str = ""


def _uniform_avoiding(rng, count, lo, hi, holes):
    """count values uniform on [lo, hi] minus the union of the open intervals in holes."""
    segs = [(lo, hi)]
    for a, b in holes:
        nxt = []
        for s0, s1 in segs:
            if b <= s0 or a >= s1:
                nxt.append((s0, s1))
                continue
            if a > s0:
                nxt.append((s0, a))
            if b < s1:
                nxt.append((b, s1))
        segs = nxt
    lens = np.array([s1 - s0 for s0, s1 in segs])
    u = rng.uniform(0.0, lens.sum(), size=count)
    cum = np.concatenate([[0.0], np.cumsum(lens)])
    idx = np.clip(np.searchsorted(cum, u, side="right") - 1, 0, len(segs) - 1)
    return np.array([segs[i][0] for i in idx]) + (u - cum[idx])


def edge_cluster_spectrum(rng, n, emin, emax, n_in_edge, n_out_edge, n_in_total,
                          width=EDGE_WIDTH, delta=DELTA, bulk=(-1.0, 1.0)):
    """n eigenvalues: n_in_total strictly inside (emin, emax), of which n_in_edge lie within
    `width` inside each endpoint; n_out_edge lie within `width` outside each endpoint; the
    rest are uniform on `bulk` outside [emin - width, emax + width].  Nothing is closer than
    `delta` to an endpoint."""
    interior = n_in_total - 2 * n_in_edge
    assert interior >= 0
    lam = [
        rng.uniform(emin + width, emax - width, size=interior),
        rng.uniform(emin + delta, emin + width, size=n_in_edge),
        rng.uniform(emax - width, emax - delta, size=n_in_edge),
        rng.uniform(emin - width, emin - delta, size=n_out_edge),
        rng.uniform(emax + delta, emax + width, size=n_out_edge),
    ]
    n_bulk = n - n_in_total - 2 * n_out_edge
    assert n_bulk >= 0
    lam.append(_uniform_avoiding(rng, n_bulk, bulk[0], bulk[1], [(emin - width, emax + width)]))
    return np.concatenate(lam)


def uniform_spectrum(rng, n, emin, emax, delta=DELTA, lo=-1.0, hi=1.0):
    """n eigenvalues uniform on [lo, hi], redrawn when closer than delta to an endpoint."""
    lam = rng.uniform(lo, hi, size=n)
    for _ in range(100):
        bad = (np.abs(lam - emin) < delta) | (np.abs(lam - emax) < delta)
        if not bad.any():
            break
        lam[bad] = rng.uniform(lo, hi, size=int(bad.sum()))
    return lam


def haar_basis(rng, n, complex_, device=None):
    """Q factor of the QR factorization of a seeded i.i.d. Gaussian n x n matrix."""
    if device is not None and n >= DEVICE_GAUSSIAN_N:
        import torch
        gen = torch.Generator(device=device)
        gen.manual_seed(int(rng.integers(0, 2 ** 63 - 1)))
        dt = torch.complex128 if complex_ else torch.float64
        gt = torch.randn((n, n), dtype=dt, device=device, generator=gen)
        if complex_:
            gt *= 2 ** 0.5  # torch's complex normal has unit variance: re, im each N(0, 1/2)
        q, _ = torch.linalg.qr(gt)
        del gt
        return q
    g = rng.standard_normal((n, n))
    if complex_:
        g = g + 1j * rng.standard_normal((n, n))
    if device is None:
        q, _ = np.linalg.qr(g)
        return np.asfortranarray(q)
    import torch
    gt = torch.from_numpy(g).to(device)
    del g
    q, _ = torch.linalg.qr(gt)
    del gt
    return q


def assemble(lam, U, device=None):
    """A = U diag(lam) U^H, made exactly Hermitian; returned column-major."""
    if device is None:
        A = (U * lam[None, :]) @ U.conj().T
        A = 0.5 * (A + A.conj().T)
        return np.asfortranarray(A)
    import torch
    lt = torch.from_numpy(np.asarray(lam)).to(device=device, dtype=U.real.dtype if U.is_complex() else U.dtype)
    A = (U * lt[None, :]) @ U.conj().T
    A = 0.5 * (A + A.conj().T)
    return A.mT.contiguous().mT   # column-major storage


def gaussian_block(rng, n, m0, complex_, device=None):
    x = rng.standard_normal((n, m0))
    if complex_:
        x = x + 1j * rng.standard_normal((n, m0))
    x = np.asfortranarray(x)
    if device is None:
        return x
    import torch
    return torch.from_numpy(x).to(device).mT.contiguous().mT


def householder_assemble(rng, lam, complex_, device, k=8):
    """A = H_k ... H_1 diag(lam) H_1 ... H_k with k seeded dense reflectors H = I - 2 v v^H
    (|v| = 1), built with elementwise products and row sums only (no library factorization or
    matrix product).  The same eigenvalues and dense storage as the Haar construction, with
    eigenvectors U = H_k ... H_1 (not formed).  Device tensors only."""
    import torch
    n = len(lam)
    dt = torch.complex128 if complex_ else torch.float64
    A = torch.diag(torch.from_numpy(np.asarray(lam, dtype=np.float64)).to(device)).to(dt)
    for _ in range(k):
        v = rng.standard_normal(n)
        if complex_:
            v = v + 1j * rng.standard_normal(n)
        v = torch.from_numpy(v / np.linalg.norm(v)).to(device=device, dtype=dt)
        w = (A * v[None, :]).sum(dim=1)                       # A v
        c = (v.conj() * w).sum()                              # v^H A v
        A = A - 2 * (v[:, None] * w.conj()[None, :]) - 2 * (w[:, None] * v.conj()[None, :]) \
            + 4 * c * (v[:, None] * v.conj()[None, :])
    A = 0.5 * (A + A.conj().T)
    return A.mT.contiguous().mT


def make_problem(lam, emin, emax, m0, n_c, tol, max_iter, complex_, rng, device=None, name="",
                 basis="haar"):
    """basis "haar" (default): U from the QR of a Gaussian matrix, kept in the result;
    "householder" (device only): the reflector construction, U not formed (None)."""
    n = len(lam)
    if basis == "householder":
        A = householder_assemble(rng, lam, complex_, device)
        X0 = gaussian_block(rng, n, m0, complex_, device)
        m_true = int(np.sum((lam > emin) & (lam < emax)))
        return Problem(n=n, dtype="c128" if complex_ else "r64", emin=emin, emax=emax, m0=m0,
                       n_c=n_c, tol=tol, max_iter=max_iter, lam=np.asarray(lam), m_true=m_true,
                       anorm=float(np.max(np.abs(lam))), A=A, U=None, X0=X0, name=name)
    U = haar_basis(rng, n, complex_, device)
    A = assemble(lam, U, device)
    X0 = gaussian_block(rng, n, m0, complex_, device)
    m_true = int(np.sum((lam > emin) & (lam < emax)))
    return Problem(n=n, dtype="c128" if complex_ else "r64", emin=emin, emax=emax, m0=m0,
                   n_c=n_c, tol=tol, max_iter=max_iter, lam=np.asarray(lam), m_true=m_true,
                   anorm=float(np.max(np.abs(lam))), A=A, U=U, X0=X0, name=name)


# --------------------------------------------------------------------------------------
# The five workloads.  Sizes can be scaled down (n=...) for tests; the recipe is unchanged.
# --------------------------------------------------------------------------------------

def fig2_problem(kind="dense", m0=51, n_c=None, complex_=False, tol=1e-12, max_iter=40,
                 device=None, seed_tag=6, n=545, n_in=50):
    """The two n=545 test matrices of Sec. 3 (the comparison of FEAST, XFEAST and RFEAST):
    the same eigenvectors, n_in eigenvalues inside I=(-1, 1) and the other n - n_in uniform on
    [1.01, 1.1] ("dense" outer spectrum) or [1.01, 20.81] ("sparse").  The paper does not say
    how the inside eigenvalues are placed: here uniform on (-1, 1), at least DELTA from the
    endpoints.  n_c defaults to the paper's choice for each matrix (8 dense, 3 sparse)."""
    rng = rng_for([seed_tag, 0 if kind == "dense" else 1])
    hi = {"dense": 1.1, "sparse": 20.81}[kind]
    lam = np.concatenate([uniform_spectrum(rng, n_in, -1.0, 1.0, lo=-1.0, hi=1.0),
                          rng.uniform(1.01, hi, size=n - n_in)])
    if n_c is None:
        n_c = 8 if kind == "dense" else 3
    return make_problem(lam, -1.0, 1.0, m0, n_c, tol, max_iter, complex_, rng, device,
                        name=f"fig2-{kind}")


@dataclasses.dataclass
class PencilProblem(Problem):
    B: object = None       # Hermitian positive definite, column-major
    Z: object = None       # B-orthonormal eigenvectors (A Z = B Z diag(lam)), numpy only


def pencil_problem(lam, emin, emax, m0, n_c, tol, max_iter, complex_, rng, s_range=(0.6, 1.5),
                   name=""):
    """A Hermitian-definite pencil with known eigenpairs: Z = U diag(s) W (U, W Haar-like
    unitary, s uniform on s_range), B = Z^{-H} Z^{-1} = U diag(1/s^2) U^H and
    A = Z^{-H} diag(lam) Z^{-1}, so A z_i = lam_i B z_i with z_i^H B z_j = delta_ij and A, B do
    not commute.  Draw order: lam (given), U, s, W, X0.  Host (numpy) arrays."""
    n = len(lam)
    U = haar_basis(rng, n, complex_)
    s = rng.uniform(s_range[0], s_range[1], size=n)
    W = haar_basis(rng, n, complex_)
    # Z^{-1} = W^H diag(1/s) U^H;  M = Z^{-H} = U diag(1/s) W
    M = (U / s[None, :]) @ W
    A = (M * np.asarray(lam)[None, :]) @ M.conj().T
    A = np.asfortranarray(0.5 * (A + A.conj().T))
    B = (U / (s * s)[None, :]) @ U.conj().T
    B = np.asfortranarray(0.5 * (B + B.conj().T))
    Z = np.asfortranarray((U * s[None, :]) @ W)
    X0 = gaussian_block(rng, n, m0, complex_)
    m_true = int(np.sum((np.asarray(lam) > emin) & (np.asarray(lam) < emax)))
    anorm = float(np.linalg.norm(A, 2))
    return PencilProblem(n=n, dtype="c128" if complex_ else "r64", emin=emin, emax=emax, m0=m0,
                         n_c=n_c, tol=tol, max_iter=max_iter, lam=np.asarray(lam),
                         m_true=m_true, anorm=anorm, A=A, U=None, X0=X0, name=name, B=B, Z=Z)


def config1(n=500, device=None, seed_tag=1):
    """Real symmetric, lam ~ U[-1,1], I = (-0.1, 0.1), m0 = 75, n_c = 8, tol 1e-12, 20 its."""
    rng = rng_for(seed_tag)
    emin, emax = -0.1, 0.1
    lam = uniform_spectrum(rng, n, emin, emax)
    m0 = 75 if n == 500 else max(4, int(math.ceil(1.5 * 0.1 * n)))
    return make_problem(lam, emin, emax, m0, 8, 1e-12, 20, False, rng, device, "C1")


def config2(n=8192, device=None, seed_tag=2, n_in=200, n_in_edge=40, n_out_edge=100, m0=300,
            n_c=8, half_width=0.05, max_iter=200, basis="haar"):
    """Complex Hermitian hard case: n_in eigenvalues in I = (-0.05, 0.05) with n_in_edge
    within 1e-3 inside each endpoint, n_out_edge within 1e-3 outside each endpoint, the rest
    uniform on [-1, 1] outside the clusters; m0 = 300, n_c = 8, tol 1e-12."""
    rng = rng_for(seed_tag)
    emin, emax = -half_width, half_width
    lam = edge_cluster_spectrum(rng, n, emin, emax, n_in_edge, n_out_edge, n_in)
    return make_problem(lam, emin, emax, m0, n_c, 1e-12, max_iter, True, rng, device, "C2",
                        basis=basis)


def config3(n=16384, device=None, seed_tag=3):
    """Same recipe as config2 at n = 16384, m0 = 400, n_c = 16."""
    p = config2(n=n, device=device, seed_tag=seed_tag, m0=400, n_c=16)
    p.name = "C3"
    return p


def config5(n=32768, device=None, seed_tag=5, basis="haar"):
    """n = 32768, 512 eigenvalues in I = (-0.05, 0.05) with 64 within 1e-3 inside each edge,
    no outer cluster, bulk uniform outside; m0 = 768, n_c = 8."""
    p = config2(n=n, device=device, seed_tag=seed_tag, n_in=512, n_in_edge=64, n_out_edge=0,
                m0=768, n_c=8, basis=basis)
    p.name = "C5"
    return p


def config4_specs(count=64, seed_tag=4, n_lo=256, n_hi=4096):
    """Sizes and intervals of the batched workload: n_p ~ U{n_lo..n_hi}; interval centre
    c_p ~ U[-0.5, 0.5], half-width h_p ~ U[0.02, 0.1]; m_p = round(0.08 n_p) inside with 10
    within 1e-3 inside each endpoint, 10 within 1e-3 outside each endpoint; m0_p = ceil(1.5 m_p)."""
    rng = rng_for([seed_tag, 0])
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    cs = rng.uniform(-0.5, 0.5, size=count)
    hs = rng.uniform(0.02, 0.1, size=count)
    specs = []
    for p in range(count):
        m_p = int(round(0.08 * ns[p]))
        specs.append(dict(n=int(ns[p]), emin=float(cs[p] - hs[p]), emax=float(cs[p] + hs[p]),
                          m=m_p, m0=int(math.ceil(1.5 * m_p)), tag=[seed_tag, p + 1]))
    return specs


def config4_problem(spec, device=None):
    rng = rng_for(spec["tag"])
    lam = edge_cluster_spectrum(rng, spec["n"], spec["emin"], spec["emax"], 10, 10, spec["m"])
    return make_problem(lam, spec["emin"], spec["emax"], spec["m0"], 8, 1e-12, 200, True, rng,
                        device, "C4")
