"""Independent reference values used to pin the oracle (no oracle code here): closed forms of
the quadrature filter, brute-force eigendecompositions via numpy/LAPACK, and subspace angles."""
import numpy as np


def rho_closed(lam, emin, emax, nc):
    """Real closed form of the n_c-point Gauss-Legendre filter on the circle around I:
    with t = (lam - c)/r and s_j = sin(pi x_j / 2),
        rho(t) = sum_j (w_j / 2) (1 - t s_j) / (1 - 2 t s_j + t^2).
    Derived from Re[e^{i th}/(e^{i th} - t)] = (1 - t cos th)/(1 - 2 t cos th + t^2) with
    th_j = (pi/2)(1 - x_j), cos th_j = sin(pi x_j / 2).  Nodes/weights from numpy's leggauss."""
    x, w = np.polynomial.legendre.leggauss(nc)
    c, r = 0.5 * (emin + emax), 0.5 * (emax - emin)
    t = (np.asarray(lam, dtype=float) - c) / r
    s = np.sin(0.5 * np.pi * x)
    t = t[..., None]
    return np.sum(0.5 * w * (1.0 - t * s) / (1.0 - 2.0 * t * s + t * t), axis=-1)


def sin_theta_max(Xa, Xb):
    """Largest principal angle (as its sine) between span(Xa) and span(Xb), both with
    orthonormal columns: || Xb - Xa (Xa^H Xb) ||_2 (no arccos of the smallest cosine)."""
    Xa = np.asarray(Xa)
    Xb = np.asarray(Xb)
    return np.linalg.norm(Xb - Xa @ (Xa.conj().T @ Xb), 2)


def orthonormal(X):
    q, _ = np.linalg.qr(X)
    return q
