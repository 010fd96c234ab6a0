/* feast_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the FEAST eigensolver for the Hermitian
 * standard problem A x = lambda x on an open interval I = (emin, emax), written from
 * Gavin & Polizzi, "Enhancing the Performance and Robustness of the FEAST Eigensolver"
 * (arXiv 1605.08771): the quadrature filter of Sec. 1, eq. (contour_int_quad), and the
 * FEAST algorithm of the Appendix (filter, Rayleigh-Ritz, residual test), the expanded-subspace
 * variants of Sec. 2, and the generalized Hermitian-definite problem A x = lambda B x.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may load this
 * library.  The GPU product never links, loads or calls it, and it shares no code with the
 * GPU path.
 *
 * Conventions: column-major arrays with a leading dimension; complex numbers are interleaved
 * (re, im) double pairs.  dtype 0 = real symmetric A and real X (arrays of double),
 * dtype 1 = complex Hermitian A and complex X (arrays of 2*... doubles).
 *
 * Status codes (shared meaning with the product's header, no shared code):
 *   0 converged, 1 not converged, 2 m0 too small, 3 no eigenvalues, 4 B' not positive
 *   definite, 5 non-finite value, 6 exact zero pivot, negative = invalid argument.
 */
#ifndef FEAST_ORACLE_H
#define FEAST_ORACLE_H
#ifdef __cplusplus
extern "C" {
#endif

int or_gauss_legendre(int n, double* x, double* w);
int or_contour(double emin, double emax, int nc, double* z, double* omega);
int or_zlu(int n, double* M, int ld, int* piv);
int or_zlu_solve(int n, const double* LU, int ld, const int* piv, int nrhs, double* B, int ldb,
                 int adjoint);
int or_jacobi_eigh(int n, double* H, int ld, double* d, double* V, int ldv);
int or_filter_apply(int dtype, int n, const double* A, int lda, double emin, double emax, int nc,
                    const double* X, int ldx, int m0, double* Q, int ldq);
int or_rayleigh_ritz(int dtype, int n, const double* A, int lda, double* Q, int ldq, int m0,
                     double emin, double emax, double anorm, double* lambda, double* res, int* m);
int or_feast_solve(int dtype, int n, const double* A, int lda, double emin, double emax, int nc,
                   int m0, double tol, int max_iter, double anorm, const double* X0, int ldx0,
                   double* X, int ldx, double* lambda, double* res, int* m, int* iters,
                   double* trace);
int or_feast_solve_ex(int dtype, int n, const double* A, int lda, double emin, double emax,
                      int nc, int m0, double tol, int max_iter, double anorm, const double* X0,
                      int ldx0, double* X, int ldx, double* lambda, double* res, int* m,
                      int* iters, double* trace, int spurious, double* mu_out);
int or_feast_solve_gen(int dtype, int n, const double* A, int lda, const double* B, int ldb,
                       double emin, double emax, int nc, int m0, double tol, int max_iter,
                       double anorm, const double* X0, int ldx0, double* X, int ldx,
                       double* lambda, double* res, int* m, int* iters, double* trace,
                       int spurious, double* mu_out);
int or_filter_apply_gen(int dtype, int n, const double* A, int lda, const double* B, int ldb,
                        double emin, double emax, int nc, const double* X, int ldx, int m0,
                        double* Q, int ldq);
int or_xrfeast_solve(int variant, int dtype, int n, const double* A, int lda, double emin,
                     double emax, int nc, int m0, int s, double tol, int max_iter, double anorm,
                     const double* X0, int ldx0, double* X, int ldx, double* lambda, double* res,
                     int* m, int* iters, double* trace, int spurious, double* mu_out);
int or_select_pairs(int r, const double* lam, const double* res, double emin, double emax,
                    int m0, int* sel);
int or_num_threads(void);
void or_set_num_threads(int n);
/* Test build only (compiled with -DORACLE_FAULTS): plant mistake `code` (0 = none). */
#ifdef ORACLE_FAULTS
void or_set_fault(int code);
#endif

#ifdef __cplusplus
}
#endif
#endif
