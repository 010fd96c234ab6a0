/* feast_oracle.c -- TEST INFRASTRUCTURE ONLY (see feast_oracle.h).
 *
 * Plain FP64 CPU FEAST, written from Gavin & Polizzi, arXiv 1605.08771:
 *   - spectral projector rho(A) as a contour integral, Sec. 1 eq. (contour_int);
 *   - its n_c-point Gauss quadrature, Sec. 1 eq. (contour_int_quad);
 *   - each term (z_i I - A)^{-1} X by a linear solve with the columns of X as right-hand
 *     sides, Sec. 1 (text after eq. contour_int_quad);
 *   - the FEAST algorithm of the Appendix: step 1 filter, step 2 Rayleigh-Ritz with
 *     A' = X'^H A X', B' = X'^H X', step 3 residual test over the Ritz pairs inside I.
 *   - B' is reduced the way Sec. 2 (Method 1) orthogonalizes a subspace: diagonalize
 *     B' = V S^2 V^H and use V S^{-1}.
 *
 * Where the paper is silent the readings are (also listed in the design notes):
 *   - contour: circle with centre c = (emin+emax)/2, radius r = (emax-emin)/2; Gauss-Legendre
 *     nodes on the upper half circle, theta_j = (pi/2)(1 - x_j); the lower half is folded in
 *     by conjugate symmetry (adjoint solves for complex A, a real part for real A);
 *   - n_c = number of upper-half nodes = number of factorizations;
 *   - solver: LU with partial pivoting (largest modulus, ties to the lowest row);
 *   - reduced eigenproblems: cyclic-by-rows complex Jacobi (Golub & Van Loan, sym.schur2
 *     after removing the phase of the off-diagonal entry);
 *   - residual r_k = ||A x_k - lambda_k x_k||_2 / anorm with ||x_k||_2 = 1.
 *
 * Everything is unblocked textbook code; no blocking, fusion or reordering beyond the
 * definitions.  OpenMP is used only across the independent quadrature nodes; the
 * accumulation over nodes runs afterwards in node order, so results do not depend on the
 * thread count.
 */
#include "feast_oracle.h"

#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex zc;

/* Planted-mistake switch for the mutation tests of the pins.  Only the separate test build
 * compiled with -DORACLE_FAULTS has it; in the reference build g_fault is the constant 0, so
 * every planted branch below folds away at compile time and the library holds none of them. */
#ifdef ORACLE_FAULTS
static int g_fault = 0;
void or_set_fault(int code) { g_fault = code; }
#else
#define g_fault 0
#endif

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
void or_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ---------------------------------------------------------------------------------------
 * Gauss-Legendre rule on [-1, 1] (the "Gauss quadrature" of Sec. 1).  Roots of P_n by Newton
 * iteration with the three-term recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1};
 * weights w = 2 / ((1 - x^2) P_n'(x)^2).  Output ascending in x.
 * ------------------------------------------------------------------------------------- */
static void legendre_eval(int n, double t, double* pn, double* dpn) {
  double pkm1 = 1.0, pk = t;
  if (n == 0) { *pn = 1.0; *dpn = 0.0; return; }
  for (int k = 1; k < n; k++) {
    double pk1 = ((2.0 * k + 1.0) * t * pk - k * pkm1) / (k + 1.0);
    pkm1 = pk;
    pk = pk1;
  }
  *pn = pk;
  *dpn = n * (t * pk - pkm1) / (t * t - 1.0);
}

int or_gauss_legendre(int n, double* x, double* w) {
  if (n < 1 || !x || !w) return -1;
  for (int i = 0; i < n; i++) {
    double t = cos(M_PI * (i + 0.75) / (n + 0.5)); /* i-th root from the top */
    double p, dp;
    for (int it = 0; it < 100; it++) {
      legendre_eval(n, t, &p, &dp);
      double dt = p / dp;
      t -= dt;
      if (fabs(dt) <= 1e-16) break;
    }
    legendre_eval(n, t, &p, &dp);
    x[n - 1 - i] = t;
    w[n - 1 - i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
  return 0;
}

/* ---------------------------------------------------------------------------------------
 * Nodes z_j and weights omega_j of eq. (contour_int_quad) on the circle around I.
 *   rho(A) = 1/(2 pi i) \oint (zI-A)^{-1} dz, z = c + r e^{i theta}, dz = i r e^{i theta} dtheta
 *          = 1/(2 pi) \int_0^{2pi} r e^{i theta} (zI - A)^{-1} dtheta.
 * The lower half (theta -> 2pi - theta) is the conjugate node with the conjugate factor, so
 *   rho(A) X = 1/(2 pi) \int_0^pi [ r e^{i theta} (zI-A)^{-1} + r e^{-i theta} (zbar I-A)^{-1} ] X
 * and Gauss-Legendre on theta = (pi/2)(1 - x) in [0, pi] (dtheta = (pi/2) dx) gives
 *   rho(A) X ~= sum_j [ omega_j (z_j I - A)^{-1} + conj(omega_j) (conj(z_j) I - A)^{-1} ] X,
 *   omega_j = (w_j / 4) r e^{i theta_j}.
 * z and omega are interleaved complex arrays of length nc.
 * ------------------------------------------------------------------------------------- */
int or_contour(double emin, double emax, int nc, double* z, double* omega) {
  if (!(emin < emax) || nc < 1) return -1;
  double* x = malloc(sizeof(double) * nc);
  double* w = malloc(sizeof(double) * nc);
  or_gauss_legendre(nc, x, w);
  double c = 0.5 * (emin + emax), r = 0.5 * (emax - emin);
  for (int j = 0; j < nc; j++) {
    double th = 0.5 * M_PI * (1.0 - x[j]);
    zc e = cexp(I * th);
    zc zj = c + r * e;
    zc oj = 0.25 * w[j] * r * (g_fault == 2 ? conj(e) : e); /* planted: weight phase sign */
    z[2 * j] = creal(zj);
    z[2 * j + 1] = cimag(zj);
    omega[2 * j] = creal(oj);
    omega[2 * j + 1] = cimag(oj);
  }
  free(x);
  free(w);
  return 0;
}

/* ---------------------------------------------------------------------------------------
 * Complex LU with partial pivoting, unblocked (textbook Doolittle, right-looking).
 * M (n x n, column-major, ld) is overwritten by L (unit, strictly lower) and U (upper);
 * piv[k] = row exchanged with row k at step k (0-based), applied to whole rows, so that
 * P M = L U with P = S_{n-1} ... S_0.  Returns 0, or k+1 if column k has only zeros.
 * ------------------------------------------------------------------------------------- */
static int zlu(int n, zc* M, int ld, int* piv) {
  for (int k = 0; k < n; k++) {
    int p = k;
    double best = cabs(M[k + (size_t)k * ld]);
    for (int i = k + 1; i < n; i++) {
      double a = cabs(M[i + (size_t)k * ld]);
      if (a > best) { best = a; p = i; }
    }
    piv[k] = p;
    if (best == 0.0) return k + 1;
    if (p != k && g_fault != 4) {
      for (int j = 0; j < n; j++) {
        zc t = M[k + (size_t)j * ld];
        M[k + (size_t)j * ld] = M[p + (size_t)j * ld];
        M[p + (size_t)j * ld] = t;
      }
    }
    zc piv_val = M[k + (size_t)k * ld];
    for (int i = k + 1; i < n; i++) M[i + (size_t)k * ld] /= piv_val;
    for (int j = k + 1; j < n; j++) {
      zc ukj = M[k + (size_t)j * ld];
      if (ukj == 0.0) continue;
      zc* colj = M + (size_t)j * ld;
      const zc* colk = M + (size_t)k * ld;
      for (int i = k + 1; i < n; i++) colj[i] -= colk[i] * ukj;
    }
  }
  return 0;
}

/* Solve M Y = B (adjoint = 0) or M^H Y = B (adjoint = 1) with the factors of zlu, in place.
 *   M   = P^T L U      ->  Y = U^{-1} L^{-1} (P B)
 *   M^H = U^H L^H P    ->  Y = P^T L^{-H} U^{-H} B                                        */
static void zlu_solve(int n, const zc* LU, int ld, const int* piv, int nrhs, zc* B, int ldb,
                      int adjoint) {
  for (int c = 0; c < nrhs; c++) {
    zc* b = B + (size_t)c * ldb;
    if (!adjoint) {
      for (int k = 0; k < n; k++) {
        int p = piv[k];
        if (p != k) { zc t = b[k]; b[k] = b[p]; b[p] = t; }
      }
      for (int j = 0; j < n; j++) { /* L unit lower, forward */
        zc bj = b[j];
        if (bj == 0.0) continue;
        const zc* col = LU + (size_t)j * ld;
        for (int i = j + 1; i < n; i++) b[i] -= col[i] * bj;
      }
      for (int j = n - 1; j >= 0; j--) { /* U upper, backward */
        const zc* col = LU + (size_t)j * ld;
        b[j] /= col[j];
        zc bj = b[j];
        if (bj == 0.0) continue;
        for (int i = 0; i < j; i++) b[i] -= col[i] * bj;
      }
    } else {
      for (int i = 0; i < n; i++) { /* U^H lower, forward: row i of U^H = conj(column i of U) */
        const zc* col = LU + (size_t)i * ld;
        zc s = b[i];
        for (int k = 0; k < i; k++) s -= conj(col[k]) * b[k];
        b[i] = s / conj(col[i]);
      }
      for (int i = n - 1; i >= 0; i--) { /* L^H unit upper, backward */
        const zc* col = LU + (size_t)i * ld;
        zc s = b[i];
        for (int k = i + 1; k < n; k++) s -= conj(col[k]) * b[k];
        b[i] = s;
      }
      for (int k = n - 1; k >= 0; k--) {
        int p = piv[k];
        if (p != k) { zc t = b[k]; b[k] = b[p]; b[p] = t; }
      }
    }
  }
}

int or_zlu(int n, double* M, int ld, int* piv) {
  if (n < 1 || ld < n || !M || !piv) return -1;
  return zlu(n, (zc*)M, ld, piv);
}

int or_zlu_solve(int n, const double* LU, int ld, const int* piv, int nrhs, double* B, int ldb,
                 int adjoint) {
  if (n < 1 || ld < n || ldb < n || nrhs < 0) return -1;
  zlu_solve(n, (const zc*)LU, ld, piv, nrhs, (zc*)B, ldb, adjoint);
  return 0;
}

/* ---------------------------------------------------------------------------------------
 * Cyclic-by-rows Jacobi for a complex Hermitian H (n x n, column-major, overwritten).
 * For each pair (p, q): write h_pq = |h_pq| e^{i phi}; D = diag(1, e^{-i phi}) makes the 2x2
 * block real symmetric, then the Golub & Van Loan sym.schur2 rotation J = [c s; -s c] with
 *   tau = (h_qq - h_pp) / (2 |h_pq|),  t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
 *   c = 1/sqrt(1 + t^2), s = t c
 * zeroes it.  G = D J; H <- G^H H G; V <- V G.  A rotation is skipped when
 * |h_pq| <= 1e-17 sqrt(|h_pp h_qq|) (relative threshold); sweeps stop when a whole sweep
 * skips every pair.  Outputs d[k] = H_kk (unsorted) and V with H_in V = V diag(d).
 * Returns the number of sweeps, or -1 if 100 sweeps did not converge.
 * ------------------------------------------------------------------------------------- */
static int jacobi(int n, zc* H, int ld, double* d, zc* V, int ldv) {
  for (int j = 0; j < n; j++)
    for (int i = 0; i < n; i++) V[i + (size_t)j * ldv] = (i == j) ? 1.0 : 0.0;
  int sweeps = 0, converged = 0;
  for (; sweeps < 100 && !converged; sweeps++) {
    int rotated = 0;
    for (int p = 0; p < n - 1; p++) {
      for (int q = p + 1; q < n; q++) {
        zc hpq = H[p + (size_t)q * ld];
        double a = cabs(hpq);
        double hpp = creal(H[p + (size_t)p * ld]), hqq = creal(H[q + (size_t)q * ld]);
        if (a == 0.0 || a <= 1e-17 * sqrt(fabs(hpp * hqq))) continue;
        rotated = 1;
        zc e = conj(hpq) / a; /* e^{-i phi} */
        double tau = (hqq - hpp) / (2.0 * a);
        double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        zc gpp = c, gpq = s, gqp = -s * e, gqq = c * e;
        for (int k = 0; k < n; k++) { /* columns: H <- H G */
          zc hkp = H[k + (size_t)p * ld], hkq = H[k + (size_t)q * ld];
          H[k + (size_t)p * ld] = hkp * gpp + hkq * gqp;
          H[k + (size_t)q * ld] = hkp * gpq + hkq * gqq;
        }
        for (int k = 0; k < n; k++) { /* rows: H <- G^H H */
          zc hpk = H[p + (size_t)k * ld], hqk = H[q + (size_t)k * ld];
          H[p + (size_t)k * ld] = conj(gpp) * hpk + conj(gqp) * hqk;
          H[q + (size_t)k * ld] = conj(gpq) * hpk + conj(gqq) * hqk;
        }
        H[p + (size_t)p * ld] = hpp - t * a;
        H[q + (size_t)q * ld] = hqq + t * a;
        H[p + (size_t)q * ld] = 0.0;
        H[q + (size_t)p * ld] = 0.0;
        for (int k = 0; k < n; k++) { /* V <- V G */
          zc vkp = V[k + (size_t)p * ldv], vkq = V[k + (size_t)q * ldv];
          V[k + (size_t)p * ldv] = vkp * gpp + vkq * gqp;
          V[k + (size_t)q * ldv] = vkp * gpq + vkq * gqq;
        }
      }
    }
    if (!rotated) converged = 1;
  }
  for (int k = 0; k < n; k++) d[k] = creal(H[k + (size_t)k * ld]);
  return converged ? sweeps : -1;
}

int or_jacobi_eigh(int n, double* H, int ld, double* d, double* V, int ldv) {
  if (n < 1 || ld < n || ldv < n) return -1;
  return jacobi(n, (zc*)H, ld, d, (zc*)V, ldv);
}

/* ---------------------------------------------------------------------------------------
 * Helpers: load a real or complex column-major array into a dense complex copy.
 * ------------------------------------------------------------------------------------- */
static zc* load_matrix(int dtype, int rows, int cols, const double* src, int ld) {
  zc* out = malloc(sizeof(zc) * (size_t)rows * cols);
  for (int j = 0; j < cols; j++)
    for (int i = 0; i < rows; i++) {
      size_t s = i + (size_t)j * ld;
      out[i + (size_t)j * rows] = dtype ? (src[2 * s] + I * src[2 * s + 1]) : src[s];
    }
  return out;
}

static void store_matrix(int dtype, int rows, int cols, const zc* src, double* dst, int ld) {
  for (int j = 0; j < cols; j++)
    for (int i = 0; i < rows; i++) {
      size_t s = i + (size_t)j * ld;
      zc v = src[i + (size_t)j * rows];
      if (dtype) { dst[2 * s] = creal(v); dst[2 * s + 1] = cimag(v); }
      else dst[s] = creal(v);
    }
}

static int all_finite(const zc* a, size_t count) {
  for (size_t i = 0; i < count; i++)
    if (!isfinite(creal(a[i])) || !isfinite(cimag(a[i]))) return 0;
  return 1;
}

/* Factorizations of z_j I - A at all nodes, kept for the whole FEAST run (z_j, A fixed). */
typedef struct {
  int n, nc;
  zc* z;
  zc* omega;
  zc* lu;   /* nc blocks of n x n */
  int* piv; /* nc blocks of n */
} factors_t;

static void factors_free(factors_t* f) {
  free(f->z); free(f->omega); free(f->lu); free(f->piv);
  memset(f, 0, sizeof(*f));
}

/* Bm == NULL: the standard problem (B = I). */
static int factors_build(factors_t* f, const zc* A, const zc* Bm, int n, double emin,
                         double emax, int nc) {
  f->n = n; f->nc = nc;
  f->z = malloc(sizeof(zc) * nc);
  f->omega = malloc(sizeof(zc) * nc);
  f->lu = malloc(sizeof(zc) * (size_t)nc * n * n);
  f->piv = malloc(sizeof(int) * (size_t)nc * n);
  if (!f->z || !f->omega || !f->lu || !f->piv) return -100;
  or_contour(emin, emax, nc, (double*)f->z, (double*)f->omega);
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
  for (int j = 0; j < nc; j++) {
    zc* M = f->lu + (size_t)j * n * n;
    if (Bm) {
      for (size_t k = 0; k < (size_t)n * n; k++) M[k] = f->z[j] * Bm[k] - A[k]; /* z_j B - A */
    } else {
      for (size_t k = 0; k < (size_t)n * n; k++) M[k] = -A[k]; /* M = z_j I - A */
      for (int i = 0; i < n; i++) M[i + (size_t)i * n] += f->z[j];
    }
    if (zlu(n, M, n, f->piv + (size_t)j * n) != 0) bad = 1;
  }
  return bad ? 6 : 0;
}

/* Eq. (contour_int_quad): Q = sum_j [omega_j Y_j + conj(omega_j) Y'_j] with
 * Y_j = (z_j I - A)^{-1} X and Y'_j = (conj z_j I - A)^{-1} X = (z_j I - A)^{-H} X (A Hermitian).
 * For real symmetric A and real X, Y'_j = conj(Y_j), so Q = sum_j 2 Re(omega_j Y_j).          */
static void filter_with_factors(const factors_t* f, int dtype, const zc* X, int m0, zc* Q) {
  int n = f->n, nc = f->nc;
  size_t blk = (size_t)n * m0;
  int sides = dtype ? 2 : 1;
  zc* Y = malloc(sizeof(zc) * blk * nc * sides);
#pragma omp parallel for schedule(dynamic, 1)
  for (int js = 0; js < nc * sides; js++) {
    int j = js / sides, adj = js % sides;
    zc* y = Y + blk * js;
    memcpy(y, X, sizeof(zc) * blk);
    zlu_solve(n, f->lu + (size_t)j * n * n, n, f->piv + (size_t)j * n, m0, y, n, adj);
  }
  for (size_t k = 0; k < blk; k++) Q[k] = 0.0;
  for (int j = 0; j < nc; j++) {
    zc om = f->omega[j];
    if (dtype) {
      const zc* y = Y + blk * (2 * j);
      const zc* yh = Y + blk * (2 * j + 1);
      zc omb = (g_fault == 1) ? om : conj(om); /* planted: adjoint weight not conjugated */
      for (size_t k = 0; k < blk; k++) Q[k] += om * y[k] + omb * yh[k];
    } else {
      const zc* y = Y + blk * j;
      for (size_t k = 0; k < blk; k++) Q[k] += 2.0 * creal(om * y[k]);
    }
  }
  free(Y);
}

int or_filter_apply(int dtype, int n, const double* A, int lda, double emin, double emax, int nc,
                    const double* X, int ldx, int m0, double* Q, int ldq) {
  if (dtype != 0 && dtype != 1) return -1;
  if (n < 1) return -2;
  if (!A) return -3;
  if (lda < n) return -4;
  if (!(emin < emax)) return -5;
  if (nc < 1) return -7;
  if (!X) return -8;
  if (ldx < n) return -9;
  if (m0 < 1 || m0 > n) return -10;
  if (!Q) return -11;
  if (ldq < n) return -12;
  zc* Az = load_matrix(dtype, n, n, A, lda);
  zc* Xz = load_matrix(dtype, n, m0, X, ldx);
  factors_t f;
  memset(&f, 0, sizeof(f));
  int st = factors_build(&f, Az, NULL, n, emin, emax, nc);
  if (st == 0) {
    zc* Qz = malloc(sizeof(zc) * (size_t)n * m0);
    filter_with_factors(&f, dtype, Xz, m0, Qz);
    store_matrix(dtype, n, m0, Qz, Q, ldq);
    free(Qz);
  }
  factors_free(&f);
  free(Az);
  free(Xz);
  return st;
}

/* Plain products used by Rayleigh-Ritz. C (r x c) = op(A) B with op = H when ah. */
static void matmul(int ah, int r, int c, int kdim, const zc* A, int lda, const zc* B, int ldb,
                   zc* C) {
  for (int j = 0; j < c; j++)
    for (int i = 0; i < r; i++) {
      zc s = 0.0;
      for (int k = 0; k < kdim; k++) {
        zc a = ah ? conj(A[k + (size_t)i * lda]) : A[i + (size_t)k * lda];
        if (ah && g_fault == 3) a = A[k + (size_t)i * lda]; /* planted: transpose, no conj */
        s += a * B[k + (size_t)j * ldb];
      }
      C[i + (size_t)j * r] = s;
    }
}

static void hermitize(int m, zc* H) {
  for (int j = 0; j < m; j++)
    for (int i = 0; i <= j; i++) {
      zc a = 0.5 * (H[i + (size_t)j * m] + conj(H[j + (size_t)i * m]));
      H[i + (size_t)j * m] = a;
      H[j + (size_t)i * m] = conj(a);
    }
  for (int i = 0; i < m; i++) H[i + (size_t)i * m] = creal(H[i + (size_t)i * m]);
}

/* Appendix, FEAST step 2 (and step 3's residuals).  In: Q = X' (n x m0 basis).
 * Out: Q = Ritz vectors x_k (unit B-norm, ascending lambda), lambda, res_k =
 * ||A x_k - lambda_k B x_k|| / anorm, m = #{lambda_k in (emin, emax)}.  Bm == NULL: B = I.
 *   A' = X'^H A X',  B' = X'^H B X'  (both made exactly Hermitian)
 *   B' = V S^2 V^H (Jacobi), T = V S^{-1}   [Sec. 2, Method 1: U = X' V S^{-1}]
 *   C = T^H A' T = Z Lambda Z^H (Jacobi), W = T Z  solves A' W = B' W Lambda
 *   X = X' W.                                                                            */
static int rr_core(int n, const zc* A, const zc* Bm, zc* Qb, int m0, double emin, double emax,
                   double anorm, double* lambda, double* res, int* m) {
  int st = 0;
  zc* AQ = malloc(sizeof(zc) * (size_t)n * m0);
  zc* BQ = malloc(sizeof(zc) * (size_t)n * m0);
  zc* Ap = malloc(sizeof(zc) * (size_t)m0 * m0);
  zc* Bp = malloc(sizeof(zc) * (size_t)m0 * m0);
  zc* V = malloc(sizeof(zc) * (size_t)m0 * m0);
  zc* T = malloc(sizeof(zc) * (size_t)m0 * m0);
  zc* TA = malloc(sizeof(zc) * (size_t)m0 * m0);
  zc* C = malloc(sizeof(zc) * (size_t)m0 * m0);
  zc* Z = malloc(sizeof(zc) * (size_t)m0 * m0);
  zc* W = malloc(sizeof(zc) * (size_t)m0 * m0);
  zc* Xn = malloc(sizeof(zc) * (size_t)n * m0);
  double* s2 = malloc(sizeof(double) * m0);
  double* lam = malloc(sizeof(double) * m0);
  int* order = malloc(sizeof(int) * m0);

  matmul(0, n, m0, n, A, n, Qb, n, AQ);   /* A X'        */
  matmul(1, m0, m0, n, Qb, n, AQ, n, Ap); /* X'^H A X'   */
  if (Bm && g_fault != 11) { /* planted (11): B' = X'^H X' whatever B */
    matmul(0, n, m0, n, Bm, n, Qb, n, BQ);
    matmul(1, m0, m0, n, Qb, n, BQ, n, Bp); /* X'^H B X' */
  } else {
    matmul(1, m0, m0, n, Qb, n, Qb, n, Bp); /* X'^H X'     */
  }
  hermitize(m0, Ap);
  hermitize(m0, Bp);
  if (!all_finite(Ap, (size_t)m0 * m0) || !all_finite(Bp, (size_t)m0 * m0)) { st = 5; goto done; }

  jacobi(m0, Bp, m0, s2, V, m0);
  double smax = 0.0, smin = INFINITY;
  for (int k = 0; k < m0; k++) { if (s2[k] > smax) smax = s2[k]; if (s2[k] < smin) smin = s2[k]; }
  if (!(smin > 1e-26 * smax) || !(smax > 0.0)) { st = 4; goto done; }
  for (int j = 0; j < m0; j++) {
    double sinv = (g_fault == 5) ? 1.0 : 1.0 / sqrt(s2[j]); /* planted: S^{-1} dropped */
    for (int i = 0; i < m0; i++) T[i + (size_t)j * m0] = V[i + (size_t)j * m0] * sinv;
  }
  matmul(1, m0, m0, m0, T, m0, Ap, m0, TA); /* T^H A'    */
  matmul(0, m0, m0, m0, TA, m0, T, m0, C);  /* T^H A' T  */
  hermitize(m0, C);
  jacobi(m0, C, m0, lam, Z, m0);
  matmul(0, m0, m0, m0, T, m0, Z, m0, W);   /* W = T Z   */
  matmul(0, n, m0, m0, Qb, n, W, m0, Xn);   /* X = X' W  */

  /* ascending eigenvalues, ties by index (stable insertion sort) */
  for (int k = 0; k < m0; k++) order[k] = k;
  for (int k = 1; k < m0; k++) {
    int v = order[k], i = k - 1;
    while (i >= 0 && lam[order[i]] > lam[v]) { order[i + 1] = order[i]; i--; }
    order[i + 1] = v;
  }
  /* B x for the normalization x^H B x = 1 (2-norm when B = I) */
  if (Bm) matmul(0, n, m0, n, Bm, n, Xn, n, BQ);
  int cnt = 0;
  for (int k = 0; k < m0; k++) {
    int src = order[k];
    double nrm = 0.0;
    for (int i = 0; i < n; i++) {
      zc v = Xn[i + (size_t)src * n];
      if (Bm) nrm += creal(conj(v) * BQ[i + (size_t)src * n]);
      else nrm += creal(v) * creal(v) + cimag(v) * cimag(v);
    }
    nrm = sqrt(nrm);
    for (int i = 0; i < n; i++) Qb[i + (size_t)k * n] = Xn[i + (size_t)src * n] / nrm;
    lambda[k] = lam[src];
    if (lambda[k] > emin && lambda[k] < emax) cnt++;
  }
  *m = cnt;
  /* residuals r_k = || A x_k - lambda_k B x_k ||_2 / anorm (Appendix, FEAST step 3) */
  matmul(0, n, m0, n, A, n, Qb, n, AQ);
  if (Bm) matmul(0, n, m0, n, Bm, n, Qb, n, BQ);
  for (int k = 0; k < m0; k++) {
    double s = 0.0;
    for (int i = 0; i < n; i++) {
      zc bx = (Bm && g_fault != 10) ? BQ[i + (size_t)k * n] /* planted (10): B dropped */
                                    : Qb[i + (size_t)k * n];
      zc r = AQ[i + (size_t)k * n] - lambda[k] * bx;
      s += creal(r) * creal(r) + cimag(r) * cimag(r);
    }
    res[k] = sqrt(s) / anorm;
  }
  for (int k = 0; k < m0; k++)
    if (!isfinite(lambda[k]) || !isfinite(res[k])) st = 5;
done:
  free(AQ); free(BQ); free(Ap); free(Bp); free(V); free(T); free(TA); free(C); free(Z); free(W);
  free(Xn); free(s2); free(lam); free(order);
  return st;
}

int or_rayleigh_ritz(int dtype, int n, const double* A, int lda, double* Q, int ldq, int m0,
                     double emin, double emax, double anorm, double* lambda, double* res, int* m) {
  if (dtype != 0 && dtype != 1) return -1;
  if (n < 1) return -2;
  if (!A) return -3;
  if (lda < n) return -4;
  if (!Q) return -5;
  if (ldq < n) return -6;
  if (m0 < 1 || m0 > n) return -7;
  if (!(emin < emax)) return -8;
  if (!(anorm > 0.0)) return -10;
  if (!lambda || !res || !m) return -11;
  zc* Az = load_matrix(dtype, n, n, A, lda);
  zc* Qz = load_matrix(dtype, n, m0, Q, ldq);
  int st = rr_core(n, Az, NULL, Qz, m0, emin, emax, anorm, lambda, res, m);
  if (st == 0) store_matrix(dtype, n, m0, Qz, Q, ldq);
  free(Az);
  free(Qz);
  return st;
}

/* Appendix, FEAST algorithm: X' = rho(A) X_i; Rayleigh-Ritz; X_{i+1} = X' W (all m0 Ritz
 * vectors); stop when r = max_{lambda_k in I} res_k <= tol.  Status rules (the paper only
 * states the precondition "fewer than m0 eigenvalues in I"): m >= m0 at iteration >= 2 ->
 * 2; m = 0 at two consecutive iterations -> 3; max_iter reached -> 1.  trace[it-1] = r.
 *
 * spurious = 1 (an option beyond the paper's step 3): a Ritz pair inside I counts only if
 * its filter Rayleigh quotient mu_k = Re(x_k^H rho(A) x_k) exceeds 1/2.  For the n_c-point
 * rule on the circle, rho(t) - 1/2 = ((1 - t^2)/4) sum_j w_j / |e^{i theta_j} - t|^2, so
 * rho > 1/2 exactly on I; a Ritz vector made of eigenvectors outside I has mu < 1/2.  mu_k is
 * computed by applying the filter to the Ritz vectors, which is also the next iteration's
 * step 1.  mu_out (nullable) receives mu of the returned Ritz vectors (spurious = 1).      */
/* The FEAST loop of the Appendix on the pencil (A, B) (Bz == NULL: B = I): Xz (n x m0) holds
 * X_0 on entry and the last Ritz vectors on exit.  With B, the filter of Sec. 1 is applied to
 * B X (rho(B^{-1}A) X = sum_j omega_j (z_j B - A)^{-1} B X + adjoint terms), Rayleigh-Ritz
 * uses B' = Q^H B Q, and mu_k = Re(x_k^H B rho x_k). */
static int feast_loop(int dtype, int n, const zc* Az, const zc* Bz, double emin, double emax,
                      int nc, int m0, double tol, int max_iter, double anorm, zc* Xz,
                      double* lambda, double* res, int* m, int* iters, double* trace,
                      int spurious, double* mu_out) {
  zc* Qz = malloc(sizeof(zc) * (size_t)n * m0);
  zc* BX = Bz ? malloc(sizeof(zc) * (size_t)n * m0) : NULL;
  double* mu = malloc(sizeof(double) * m0);
  factors_t f;
  memset(&f, 0, sizeof(f));
  int st = factors_build(&f, Az, Bz, n, emin, emax, nc);
  int it = 0, prev_m = -1;
  *m = 0;
  if (st == 0) {
    st = 1;
    if (Bz) matmul(0, n, m0, n, Bz, n, Xz, n, BX);
    /* planted (9): the filter applied to X instead of B X */
    filter_with_factors(&f, dtype, (Bz && g_fault != 9) ? BX : Xz, m0, Qz); /* step 1 */
    for (it = 1; it <= max_iter; it++) {
      int mm = 0;
      int rst = rr_core(n, Az, Bz, Qz, m0, emin, emax, anorm, lambda, res, &mm); /* step 2 */
      memcpy(Xz, Qz, sizeof(zc) * (size_t)n * m0);
      if (rst != 0) { *m = mm; st = rst; break; }
      if (Bz) matmul(0, n, m0, n, Bz, n, Xz, n, BX);
      filter_with_factors(&f, dtype, (Bz && g_fault != 9) ? BX : Xz, m0, Qz); /* next step 1 */
      double r = 0.0; /* step 3 */
      int cnt = 0;
      for (int k = 0; k < m0; k++) {
        if (!(lambda[k] > emin && lambda[k] < emax)) continue;
        if (spurious) {
          const zc* bx = Bz ? BX : Xz;
          double d = 0.0;
          for (int i = 0; i < n; i++)
            d += creal(conj(bx[i + (size_t)k * n]) * Qz[i + (size_t)k * n]);
          mu[k] = d;
          if (!(d > 0.5)) continue;
        }
        cnt++;
        if (res[k] > r) r = res[k];
      }
      if (!spurious) cnt = mm;
      mm = cnt;
      *m = mm;
      if (trace) trace[it - 1] = r;
      if (mm == 0) {
        if (prev_m == 0) { st = 3; break; }
      } else if (mm >= m0 && it >= 2) {
        st = 2; break;
      } else if (r <= tol) {
        st = 0; break;
      }
      prev_m = mm;
    }
    if (it > max_iter) it = max_iter;
  }
  if (mu_out && spurious) {
    const zc* bx = Bz ? BX : Xz;
    if (Bz) matmul(0, n, m0, n, Bz, n, Xz, n, BX);
    for (int k = 0; k < m0; k++) {
      double d = 0.0;
      for (int i = 0; i < n; i++) d += creal(conj(bx[i + (size_t)k * n]) * Qz[i + (size_t)k * n]);
      mu_out[k] = d;
    }
  }
  *iters = it;
  factors_free(&f);
  free(Qz);
  free(BX);
  free(mu);
  return st;
}

int or_feast_solve_ex(int dtype, int n, const double* A, int lda, double emin, double emax,
                      int nc, int m0, double tol, int max_iter, double anorm, const double* X0,
                      int ldx0, double* X, int ldx, double* lambda, double* res, int* m,
                      int* iters, double* trace, int spurious, double* mu_out) {
  return or_feast_solve_gen(dtype, n, A, lda, NULL, 0, emin, emax, nc, m0, tol, max_iter, anorm,
                            X0, ldx0, X, ldx, lambda, res, m, iters, trace, spurious, mu_out);
}

int or_feast_solve_gen(int dtype, int n, const double* A, int lda, const double* B, int ldb,
                       double emin, double emax, int nc, int m0, double tol, int max_iter,
                       double anorm, const double* X0, int ldx0, double* X, int ldx,
                       double* lambda, double* res, int* m, int* iters, double* trace,
                       int spurious, double* mu_out) {
  if (dtype != 0 && dtype != 1) return -1;
  if (n < 1) return -2;
  if (!A) return -3;
  if (lda < n) return -4;
  if (B && ldb < n) return -6;
  if (!(emin < emax)) return -7;
  if (nc < 1) return -9;
  if (m0 < 1 || m0 > n) return -10;
  if (!(tol > 0.0)) return -11;
  if (max_iter < 1) return -12;
  if (!(anorm > 0.0)) return -13;
  if (!X0) return -14;
  if (ldx0 < n) return -15;
  if (!X) return -16;
  if (ldx < n) return -17;
  if (!lambda || !res || !m || !iters) return -18;

  zc* Az = load_matrix(dtype, n, n, A, lda);
  zc* Bz = B ? load_matrix(dtype, n, n, B, ldb) : NULL;
  if (!all_finite(Az, (size_t)n * n) || (Bz && !all_finite(Bz, (size_t)n * n))) {
    free(Az); free(Bz);
    return 5;
  }
  zc* Xz = load_matrix(dtype, n, m0, X0, ldx0);
  int st = feast_loop(dtype, n, Az, Bz, emin, emax, nc, m0, tol, max_iter, anorm, Xz, lambda,
                      res, m, iters, trace, spurious, mu_out);
  store_matrix(dtype, n, m0, Xz, X, ldx);
  free(Az);
  free(Bz);
  free(Xz);
  return st;
}

/* Sec. 1 eq. (contour_int_quad) on the pencil: Q = rho(B^{-1} A) X. */
int or_filter_apply_gen(int dtype, int n, const double* A, int lda, const double* B, int ldb,
                        double emin, double emax, int nc, const double* X, int ldx, int m0,
                        double* Q, int ldq) {
  if (dtype != 0 && dtype != 1) return -1;
  if (n < 1) return -2;
  if (!A || lda < n) return -3;
  if (!B || ldb < n) return -5;
  if (!(emin < emax)) return -7;
  if (nc < 1) return -9;
  if (!X || ldx < n) return -10;
  if (m0 < 1 || m0 > n) return -12;
  if (!Q || ldq < n) return -13;
  zc* Az = load_matrix(dtype, n, n, A, lda);
  zc* Bz = load_matrix(dtype, n, n, B, ldb);
  zc* Xz = load_matrix(dtype, n, m0, X, ldx);
  zc* BX = malloc(sizeof(zc) * (size_t)n * m0);
  matmul(0, n, m0, n, Bz, n, Xz, n, BX);
  factors_t f;
  memset(&f, 0, sizeof(f));
  int st = factors_build(&f, Az, Bz, n, emin, emax, nc);
  if (st == 0) {
    zc* Qz = malloc(sizeof(zc) * (size_t)n * m0);
    filter_with_factors(&f, dtype, g_fault == 9 ? Xz : BX, m0, Qz);
    store_matrix(dtype, n, m0, Qz, Q, ldq);
    free(Qz);
  }
  factors_free(&f);
  free(Az); free(Bz); free(Xz); free(BX);
  return st;
}

int or_feast_solve(int dtype, int n, const double* A, int lda, double emin, double emax, int nc,
                   int m0, double tol, int max_iter, double anorm, const double* X0, int ldx0,
                   double* X, int ldx, double* lambda, double* res, int* m, int* iters,
                   double* trace) {
  return or_feast_solve_ex(dtype, n, A, lda, emin, emax, nc, m0, tol, max_iter, anorm, X0, ldx0,
                           X, ldx, lambda, res, m, iters, trace, 0, NULL);
}


/* =======================================================================================
 * Expanded-subspace variants of Sec. 2 (Appendix, XFEAST and RFEAST algorithms).
 * ===================================================================================== */

/* Orthonormal basis of span(B) (n x k) by the Gram route of Sec. 2 (Method 1), applied to B
 * with its columns first scaled to unit length (a diagonal scaling leaves the span, and so the
 * Rayleigh-Ritz pairs, unchanged; without it the residual columns of RFEAST, orders of
 * magnitude shorter than the filtered ones, would sit below any rank threshold):
 * B^H B = V S^2 V^H (Jacobi), U = B V S^{-1}, keeping the directions with
 * s^2 > 1e-14 s^2_max (the numerically independent part).  Returns the rank r; U is n x r. */
static int gram_orthonormal(int n, int k, const zc* B, zc* U) {
  zc* Bn = malloc(sizeof(zc) * (size_t)n * k);
  zc* G = malloc(sizeof(zc) * (size_t)k * k);
  zc* V = malloc(sizeof(zc) * (size_t)k * k);
  double* s2 = malloc(sizeof(double) * k);
  for (int j = 0; j < k; j++) {
    double nrm = 0.0;
    for (int i = 0; i < n; i++) {
      zc v = B[i + (size_t)j * n];
      nrm += creal(v) * creal(v) + cimag(v) * cimag(v);
    }
    nrm = sqrt(nrm);
    double sc = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int i = 0; i < n; i++) Bn[i + (size_t)j * n] = B[i + (size_t)j * n] * sc;
  }
  matmul(1, k, k, n, Bn, n, Bn, n, G);
  hermitize(k, G);
  jacobi(k, G, k, s2, V, k);
  double smax = 0.0;
  for (int j = 0; j < k; j++) if (s2[j] > smax) smax = s2[j];
  int r = 0;
  for (int j = 0; j < k; j++) {
    if (!(s2[j] > 1e-14 * smax)) continue;
    double sinv = 1.0 / sqrt(s2[j]);
    for (int i = 0; i < n; i++) {
      zc acc = 0.0;
      for (int l = 0; l < k; l++) acc += Bn[i + (size_t)l * n] * V[l + (size_t)j * k];
      U[i + (size_t)r * n] = acc * sinv;
    }
    r++;
  }
  free(Bn); free(G); free(V); free(s2);
  return r;
}

/* Rayleigh-Ritz on the orthogonalized basis U (n x r): step 2.i of the XFEAST and RFEAST
 * algorithms, A' q = lambda B' q with A' = U^H A U and B' = U^H U (rr_core: unit Ritz vectors
 * Y, ascending lambda, residuals ||A y - lambda y|| / anorm).  Returns rr_core's status. */
static int rr_all(int n, const zc* A, const zc* U, int r, double anorm, zc* Y, double* lam,
                  double* res) {
  int mdummy = 0;
  memcpy(Y, U, sizeof(zc) * (size_t)n * r);
  return rr_core(n, A, NULL, Y, r, 0.0, 0.0, anorm, lam, res, &mdummy);
}

/* Selection of Sec. 2 (Method 1, also used by Method 2): every pair inside I, and if fewer
 * than m0 are inside, the pairs outside with the lowest residuals.  Reading for the case the
 * paper leaves open: with more than m0 inside, the m0 inside pairs with the lowest residuals.
 * Writes sel[0..m0) (indices into the r pairs, ascending by lambda) and returns the count
 * selected (min(m0, r)). */
static int select_pairs(int r, const double* lam, const double* res, double emin, double emax,
                        int m0, int* sel) {
  int* idx = malloc(sizeof(int) * r);
  int cnt = 0;
  /* inside, by residual */
  for (int k = 0; k < r; k++) if (lam[k] > emin && lam[k] < emax) idx[cnt++] = k;
  int nin = cnt;
  for (int a = 1; a < nin; a++) {
    int v = idx[a], b = a - 1;
    while (b >= 0 && res[idx[b]] > res[v]) { idx[b + 1] = idx[b]; b--; }
    idx[b + 1] = v;
  }
  for (int k = 0; k < r; k++) if (!(lam[k] > emin && lam[k] < emax)) idx[cnt++] = k;
  for (int a = nin + 1; a < r; a++) {
    int v = idx[a], b = a - 1;
    /* planted (6): highest residual first */
    while (b >= nin && (g_fault == 6 ? res[idx[b]] < res[v] : res[idx[b]] > res[v])) {
      idx[b + 1] = idx[b];
      b--;
    }
    idx[b + 1] = v;
  }
  int take = r < m0 ? r : m0;
  for (int a = 0; a < take; a++) sel[a] = idx[a];
  /* ascending by lambda */
  for (int a = 1; a < take; a++) {
    int v = sel[a], b = a - 1;
    while (b >= 0 && lam[sel[b]] > lam[v]) { sel[b + 1] = sel[b]; b--; }
    sel[b + 1] = v;
  }
  free(idx);
  return take;
}

int or_select_pairs(int r, const double* lam, const double* res, double emin, double emax,
                    int m0, int* sel) {
  if (r < 0 || m0 < 1 || (r > 0 && (!lam || !res || !sel))) return -1;
  return select_pairs(r, lam, res, emin, emax, m0, sel);
}

/* XFEAST (Appendix): X' = [X_0, rho X_0, ..., rho^{s-1} X_0]; repeat: orthogonalize X'
 * (Gram route), Rayleigh-Ritz on span X', select m0 pairs, stop if their largest residual
 * inside I is <= tol, else filter the selected block and slide the window of s blocks.
 * variant = 1 (XFEAST) or 2 (RFEAST: X' = rho X_i, then s Rayleigh-Ritz steps each
 * expanding X' by the residual block R = A X - X Lambda of the selected pairs; the number of
 * pairs inside I at the first step, m_e, fixes how many inside pairs (lowest residuals)
 * count in step 3).  spurious = 1 additionally requires mu_k = Re(x^H rho(A) x) > 1/2 for a
 * counted pair (as in or_feast_solve_ex).  trace[it-1] = r of outer iteration it. */
int or_xrfeast_solve(int variant, int dtype, int n, const double* A, int lda, double emin,
                     double emax, int nc, int m0, int s, double tol, int max_iter, double anorm,
                     const double* X0, int ldx0, double* X, int ldx, double* lambda, double* res,
                     int* m, int* iters, double* trace, int spurious, double* mu_out) {
  if (variant != 1 && variant != 2) return -1;
  if (dtype != 0 && dtype != 1) return -2;
  if (n < 1) return -3;
  if (!A || lda < n) return -4;
  if (!(emin < emax)) return -6;
  if (nc < 1) return -8;
  if (m0 < 1 || m0 > n) return -9;
  if (s < 1 || s * m0 > n) return -10;
  if (!(tol > 0.0) || max_iter < 1 || !(anorm > 0.0)) return -11;
  if (!X0 || ldx0 < n || !X || ldx < n || !lambda || !res || !m || !iters) return -15;
  zc* Az = load_matrix(dtype, n, n, A, lda);
  if (!all_finite(Az, (size_t)n * n)) { free(Az); return 5; }
  const int K = s * m0 + m0; /* room for the RFEAST expansion */
  zc* Xs = load_matrix(dtype, n, m0, X0, ldx0);
  zc* Bw = malloc(sizeof(zc) * (size_t)n * K);  /* X' (window or expanded basis) */
  zc* U = malloc(sizeof(zc) * (size_t)n * K);
  zc* Y = malloc(sizeof(zc) * (size_t)n * K);
  zc* Fq = malloc(sizeof(zc) * (size_t)n * m0);
  double* lam = malloc(sizeof(double) * K);
  double* rs = malloc(sizeof(double) * K);
  int* sel = malloc(sizeof(int) * m0);
  double* mu = malloc(sizeof(double) * m0);
  factors_t f;
  memset(&f, 0, sizeof(f));
  int st = factors_build(&f, Az, NULL, n, emin, emax, nc);
  int it = 0, prev_m = -1, mm = 0, kcols = 0;
  if (st == 0 && variant == 1) { /* step 0: the Krylov-like window of filtered blocks */
    memcpy(Bw, Xs, sizeof(zc) * (size_t)n * m0);
    for (int b = 1; b < s; b++)
      filter_with_factors(&f, dtype, Bw + (size_t)(b - 1) * n * m0, m0, Bw + (size_t)b * n * m0);
    kcols = s * m0;
  }
  if (st == 0) {
    st = 1;
    for (it = 1; it <= max_iter; it++) {
      int take = 0, me = -1;
      if (variant == 1) {
        int r = gram_orthonormal(n, kcols, Bw, U);
        if (r < 1) { st = 4; break; }
        st = rr_all(n, Az, U, r, anorm, Y, lam, rs);
        if (st) break;
        st = 1;
        take = select_pairs(r, lam, rs, emin, emax, m0, sel);
      } else {
        /* step 1: rho(A) X_i, already formed at the end of the previous iteration */
        if (it == 1) filter_with_factors(&f, dtype, Xs, m0, Bw);
        else memcpy(Bw, Fq, sizeof(zc) * (size_t)n * m0);
        kcols = m0;
        for (int j = 1; j <= s; j++) { /* step 2 */
          int r = gram_orthonormal(n, kcols, Bw, U);
          if (r < 1) { st = 4; break; }
          st = rr_all(n, Az, U, r, anorm, Y, lam, rs);
          if (st) break;
          st = 1;
          take = select_pairs(r, lam, rs, emin, emax, m0, sel);
          if (j == 1) {
            me = 0;
            for (int a = 0; a < r; a++) if (lam[a] > emin && lam[a] < emax) me++;
          }
          if (j < s) { /* R = A X - X Lambda appended to X' */
            for (int a = 0; a < take; a++) {
              const zc* y = Y + (size_t)sel[a] * n;
              zc* rcol = Bw + (size_t)(kcols + a) * n;
              for (int i = 0; i < n; i++) {
                zc acc = 0.0;
                for (int l = 0; l < n; l++) acc += Az[i + (size_t)l * n] * y[l];
                rcol[i] = acc - lam[sel[a]] * y[i];
              }
            }
            if (g_fault != 8) kcols += take; /* planted (8): basis never grows */
          }
        }
        if (st != 1) break;
      }
      /* the m0 selected pairs become X_{i+1} */
      double lam_sel[m0 > 0 ? m0 : 1], res_sel[m0 > 0 ? m0 : 1];
      for (int a = 0; a < take; a++) {
        memcpy(Xs + (size_t)a * n, Y + (size_t)sel[a] * n, sizeof(zc) * n);
        lam_sel[a] = lam[sel[a]];
        res_sel[a] = rs[sel[a]];
      }
      for (int a = take; a < m0; a++) { lam_sel[a] = INFINITY; res_sel[a] = INFINITY; }
      for (int a = 0; a < m0; a++) { lambda[a] = lam_sel[a]; res[a] = res_sel[a]; }
      filter_with_factors(&f, dtype, Xs, m0, Fq); /* rho(A) X_{i+1}: next window block / mu */
      for (int a = 0; a < take; a++) {
        double d = 0.0;
        for (int i = 0; i < n; i++) d += creal(conj(Xs[i + (size_t)a * n]) * Fq[i + (size_t)a * n]);
        mu[a] = d;
      }
      /* step 3 */
      int cand[m0 > 0 ? m0 : 1], nc_in = 0;
      for (int a = 0; a < take; a++) {
        if (!(lambda[a] > emin && lambda[a] < emax)) continue;
        if (spurious && !(mu[a] > 0.5)) continue;
        cand[nc_in++] = a;
      }
      if (variant == 2 && !spurious && me >= 0 && nc_in > me) { /* keep the me lowest residuals */
        for (int a = 1; a < nc_in; a++) {
          int v = cand[a], b = a - 1;
          while (b >= 0 && res[cand[b]] > res[v]) { cand[b + 1] = cand[b]; b--; }
          cand[b + 1] = v;
        }
        nc_in = me;
      }
      double r = 0.0;
      for (int a = 0; a < nc_in; a++) if (res[cand[a]] > r) r = res[cand[a]];
      mm = nc_in;
      *m = mm;
      if (trace) trace[it - 1] = r;
      if (mm == 0) {
        if (prev_m == 0) { st = 3; break; }
      } else if (mm >= m0 && it >= 2) {
        st = 2; break;
      } else if (r <= tol) {
        st = 0; break;
      }
      prev_m = mm;
      if (variant == 1 && g_fault != 7) { /* step 4: slide the window (planted 7: not) */
        memmove(Bw, Bw + (size_t)n * m0, sizeof(zc) * (size_t)n * m0 * (s - 1));
        memcpy(Bw + (size_t)(s - 1) * n * m0, Fq, sizeof(zc) * (size_t)n * m0);
      }
    }
    if (it > max_iter) it = max_iter;
  }
  if (mu_out) for (int a = 0; a < m0; a++) mu_out[a] = mu[a];
  *iters = it;
  store_matrix(dtype, n, m0, Xs, X, ldx);
  factors_free(&f);
  free(Az); free(Xs); free(Bw); free(U); free(Y); free(Fq); free(lam); free(rs); free(sel);
  free(mu);
  return st;
}
