/* feast.h -- C-ABI of the MI355X FEAST hot path (libfeast_mi355x.so, gfx950).
 *
 * FEAST (Gavin & Polizzi, "Enhancing the Performance and Robustness of the FEAST
 * Eigensolver", arXiv 1605.08771) finds the eigenpairs (lambda, x) of a Hermitian matrix,
 * A x = lambda x, with lambda in an open interval I = (emin, emax) (Sec. 1, eq. 1 with B = I).
 * The library exposes the two steps of the FEAST iteration (Appendix, FEAST algorithm) and
 * the whole iteration:
 *   feast_filter_apply   step 1, Q = rho(A) X by the quadrature of Sec. 1 eq.
 *                        (contour_int_quad);
 *   feast_rayleigh_ritz  step 2 (A' = Q^H A Q on an orthonormalised Q, reduced
 *                        eigenproblem, X = Q W) plus the residuals of step 3;
 *   feast_solve          the loop 1-2-3 until max_{lambda_k in I} res_k <= tol.
 *
 * Conventions for every entry point
 *   - Matrices are column-major with a leading dimension (LAPACK layout).  Complex data is
 *     interleaved (re, im) double pairs (std::complex<double>, numpy/torch complex128).
 *     A row-major Hermitian A read as column-major is conj(A): pass column-major storage.
 *   - A, X, X0 and Q are DEVICE pointers owned by the caller; the library never frees them.
 *     lambda, res, m, iters and trace are HOST pointers, written after the call has
 *     synchronised its stream.  The library allocates its own workspace on the handle's
 *     device (factor cache, right-hand-side blocks, reduced matrices) and frees it in
 *     feast_destroy.
 *   - dtype FEAST_R64: A real symmetric (double), X/Q real (double).  FEAST_C128: A complex
 *     Hermitian, X/Q complex.  Only the lower or upper triangle is not enough: the full A is
 *     read.
 *   - The quadrature (readings of Sec. 1, which only says "Gauss quadrature"): circle with
 *     centre c = (emin+emax)/2 and radius r = (emax-emin)/2, n_c Gauss-Legendre nodes on the
 *     upper half circle theta_j = (pi/2)(1 - x_j), z_j = c + r e^{i theta_j}, weights
 *     omega_j = (w_j/4) r e^{i theta_j}; the lower half enters through the adjoint solves
 *     (complex A) or a real part (real A).  n_c is the number of factorizations.
 *   - A handle is bound to the HIP device current at feast_create and to one stream; it is
 *     not thread-safe.
 *
 * Return codes: 0 success; -i argument i invalid (checked on the host before any device
 * work); FEAST_ERR_ALLOC (-100) device allocation failed; FEAST_ERR_HIP (-101) HIP runtime
 * error (message in feast_last_error); FEAST_ERR_UNSUPPORTED (-102) option not available;
 * positive codes are the FEAST outcomes listed below.
 */
#ifndef FEAST_MI355X_H
#define FEAST_MI355X_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct feast_ctx* feast_handle;

typedef enum { FEAST_R64 = 0, FEAST_C128 = 1 } feast_dtype;

/* Arithmetic of the shifted factorizations and solves.  FEAST_FP64: everything in FP64.
 * FEAST_FP32_IR: LU factors and correction solves in FP32 complex (FP32 matrix cores), with
 * iterative refinement whose residuals X - (z_j I - A) Y and updates are FP64, to the FP64
 * accuracy of the filtered block.  FEAST_BF16X3_IR: as FEAST_FP32_IR (FP32 factor storage,
 * same refinement), but the matrix-core products of the factorization and of the solves split
 * each FP32 operand into bf16 hi + lo parts and sum three bf16 products (hi hi, hi lo, lo hi)
 * in FP32, about 16 significant bits per product.  The Rayleigh-Ritz step is FP64 in every
 * mode. */
typedef enum { FEAST_FP64 = 0, FEAST_FP32_IR = 1, FEAST_BF16X3_IR = 2 } feast_precision;

/* The subspace iteration run by feast_solve.
 * FEAST_METHOD_FEAST: the FEAST algorithm (Appendix).
 * FEAST_METHOD_XFEAST: Sec. 2, Method 1 (Appendix, XFEAST algorithm): X' holds the last
 *   `expand` filtered blocks, [X_0, rho X_0, ..., rho^{s-1} X_0] at the start; each iteration
 *   orthogonalizes X', runs Rayleigh-Ritz on it, keeps m0 pairs (every pair inside I, then
 *   the lowest residuals outside), and puts the filtered kept block in place of the oldest.
 * FEAST_METHOD_RFEAST: Sec. 2, Method 2 (Appendix, RFEAST algorithm): X' = rho(A) X_i, then
 *   `expand` Rayleigh-Ritz steps, each after the first on X' grown by the residual block
 *   A X - X Lambda of the pairs kept by the previous step; unless opt->spurious is set, the
 *   number of pairs inside I at the first step bounds how many pairs inside I (lowest
 *   residuals) count in the convergence test.
 * Both variants orthogonalize X' by its Gram matrix (X'^H X' = V S^2 V^H, U = X' V S^{-1}),
 * with the columns of X' first scaled to unit length and directions with
 * s^2 <= 1e-14 s^2_max dropped, then run Rayleigh-Ritz on U.  Both solve n_c * m0
 * right-hand sides per iteration, like FEAST with the same m0. */
typedef enum {
  FEAST_METHOD_FEAST = 0,
  FEAST_METHOD_XFEAST = 1,
  FEAST_METHOD_RFEAST = 2
} feast_method;

typedef struct {
  int n_c;          /* quadrature nodes on the upper half circle (>= 1) */
  int m0;           /* subspace size, more than the number of eigenvalues in I */
  int max_iter;     /* FEAST iterations (>= 1) */
  int refine_max;   /* FP32_IR, BF16X3_IR: classic refinement steps (FP64 residual with A) when the
                       filter has no Ritz information, i.e. the first iteration (>= 0) */
  double tol;       /* stop when max residual over Ritz values in I <= tol (> 0) */
  double anorm;     /* ||A||_2 used to scale residuals; <= 0: estimated by power iteration */
  feast_precision prec;
  unsigned long long seed; /* seeds the Gaussian start block when X0 == NULL */
  int spurious;     /* 0: step 3 of the paper (every Ritz pair inside I counts);
                       1: a Ritz pair inside I counts only if its filter Rayleigh quotient
                       mu_k = Re(x_k^H rho(A) x_k) > 1/2.  For this quadrature
                       rho(t) - 1/2 = ((1 - t^2)/4) sum_j w_j / |e^{i theta_j} - t|^2 with
                       t = (lambda - c)/r, so rho > 1/2 exactly on I and a Ritz vector built
                       from eigenvectors outside I has mu < 1/2.  mu_k is read off the next
                       iteration's filtered block, so a converged run applies the filter once
                       more than it runs Rayleigh-Ritz.  The mixed modes always apply this
                       test: FP32 solves leave the strongly damped directions of the filtered
                       block at the FP32 noise floor, and Rayleigh-Ritz turns that noise into
                       Ritz pairs inside I with large residuals. */
  int method;       /* feast_method; 0 = FEAST */
  int expand;       /* XFEAST: blocks kept in X'; RFEAST: Rayleigh-Ritz steps per filter
                       application; >= 1 with expand * m0 <= n (ignored by FEAST) */
} feast_opts;

#define FEAST_OK 0
#define FEAST_NOT_CONVERGED 1 /* max_iter reached; outputs hold the last iterate */
#define FEAST_M0_TOO_SMALL 2  /* >= m0 Ritz values inside I at iteration >= 2 */
#define FEAST_NO_EIGENVALUES 3 /* no Ritz value inside I at two consecutive iterations */
#define FEAST_B_NOT_SPD 4      /* the filtered block is rank deficient (Q^H Q singular) */
#define FEAST_NONFINITE 5      /* NaN/Inf in A, X or an intermediate */
#define FEAST_ZERO_PIVOT 6     /* exact zero pivot in a shifted factorization */
#define FEAST_EIG_FAILED 7     /* the dense Hermitian eigensolve of a Rayleigh-Ritz step (or of
                                  the Gram matrix of XFEAST/RFEAST) did not converge */
#define FEAST_ERR_ALLOC (-100)
#define FEAST_ERR_HIP (-101)
#define FEAST_ERR_UNSUPPORTED (-102)

/* Create a handle on the current HIP device.  hip_stream: a hipStream_t to run on, or NULL:
 * the handle then creates its own blocking stream (ordered with the legacy null stream, so
 * work the caller queued there completes first).  Every entry point synchronises its stream
 * before returning.  Returns 0 or -1 (h NULL) / FEAST_ERR_HIP. */
int feast_create(feast_handle* h, void* hip_stream);
/* Release all workspace of h.  Safe on NULL. */
int feast_destroy(feast_handle h);
/* Static text for a return code. */
const char* feast_status_string(int status);
/* Text of the last HIP error seen by h (empty if none). */
const char* feast_last_error(feast_handle h);
/* Drop the cached factorizations (call after modifying A in place); also those of the batch
 * workers. */
void feast_invalidate(feast_handle h);

/* Step 1 of the FEAST algorithm (Appendix) with the quadrature of Sec. 1 eq.
 * (contour_int_quad):  Q = sum_j [omega_j (z_j I - A)^{-1} + conj(omega_j) (conj(z_j) I - A)^{-1}] X
 * (for FEAST_R64: Q = sum_j 2 Re(omega_j (z_j I - A)^{-1} X)).
 *   A: n x n (lda >= n); X: n x m0 (ldx >= n); Q: n x m0 output (ldq >= n), must not alias X.
 *   The n_c factorizations of z_j I - A are cached in h, keyed by (A pointer, n, lda, dtype,
 *   emin, emax, n_c, prec); call feast_invalidate after changing A in place.
 * Mixed modes refine each system's solution (FP64 residuals X - (z_j I - A) Y, corrections
 * through the low-precision factors) until the largest residual entry no longer drops below
 * 0.9 of the previous one, at most 10 steps (FEAST_FP32_IR) or 30 (FEAST_BF16X3_IR).
 * Argument positions for negative codes: h=1 dt=2 n=3 A=4 lda=5 emin=6 emax=7 (needs
 * emin < emax) n_c=8 prec=9 X=10 ldx=11 m0=12 (1 <= m0 <= n) Q=13 ldq=14.
 * Positive returns: FEAST_ZERO_PIVOT, FEAST_NONFINITE. */
int feast_filter_apply(feast_handle h, feast_dtype dt, int n, const void* A, int lda,
                       double emin, double emax, int n_c, feast_precision prec, const void* X,
                       int ldx, int m0, void* Q, int ldq);

/* Step 2 of the FEAST algorithm (Appendix) and the residuals of step 3.
 *   In: Q (n x m0, ldq), any basis of full rank.  Q is orthonormalised (Cholesky-QR, twice),
 *   A' = Q^H A Q is diagonalised (FP64 Jacobi), and Q is overwritten by the Ritz vectors
 *   X = Q W (unit 2-norm, ascending Ritz values).
 *   Out (host): lambda[m0] ascending, res[m0] = ||A x_k - lambda_k x_k||_2 / anorm,
 *   *m = number of lambda_k in the open interval (emin, emax).
 * Argument positions: h=1 dt=2 n=3 A=4 lda=5 Q=6 ldq=7 m0=8 emin=9 emax=10 anorm=11 (> 0)
 * lambda=12 res=13 m=14.  Positive returns: FEAST_B_NOT_SPD, FEAST_NONFINITE. */
int feast_rayleigh_ritz(feast_handle h, feast_dtype dt, int n, const void* A, int lda, void* Q,
                        int ldq, int m0, double emin, double emax, double anorm, double* lambda,
                        double* res, int* m);

/* The FEAST algorithm (Appendix), or the variant opt->method selects: X_0 = X0 (n x m0,
 * leading dimension ldx; or a seeded Gaussian block when X0 == NULL);
 * repeat  Q = rho(A) X_i;  Rayleigh-Ritz on Q;  X_{i+1} = all m0 Ritz vectors  until the
 * largest residual of the Ritz pairs inside I is <= opt->tol.  For XFEAST/RFEAST, lambda and
 * res hold the m0 kept pairs (ascending lambda; +inf past the basis rank).
 *   X: n x m0 output (ldx >= n), may equal X0 only if ldx matches.
 *   lambda[m0], res[m0], *m, *iters: host outputs of the last iterate (*m counts the pairs
 *   inside I that pass the opt->spurious test).
 *   trace: NULL or host array of opt->max_iter doubles; trace[i-1] = largest in-interval
 *   residual after iteration i.
 * Argument positions: h=1 dt=2 n=3 A=4 lda=5 emin=6 emax=7 opt=8 (n_c, m0, max_iter, tol,
 * prec, refine_max, method, expand checked) X0=9 X=10 ldx=11 lambda=12 res=13 m=14 iters=15.
 * Returns FEAST_OK, FEAST_NOT_CONVERGED, FEAST_M0_TOO_SMALL, FEAST_NO_EIGENVALUES,
 * FEAST_B_NOT_SPD, FEAST_NONFINITE, FEAST_ZERO_PIVOT or an error. */
int feast_solve(feast_handle h, feast_dtype dt, int n, const void* A, int lda, double emin,
                double emax, const feast_opts* opt, const void* X0, void* X, int ldx,
                double* lambda, double* res, int* m, int* iters, double* trace);

/* The generalized Hermitian-definite problem A x = lambda B x (Sec. 1, eq. 1), B Hermitian
 * positive definite (real symmetric for FEAST_R64), n x n, ldb >= n, same dtype as A.
 * The filter of eq. (contour_int_quad) becomes rho(B^{-1} A) X = sum_j omega_j (z_j B - A)^{-1}
 * B X + the adjoint terms (the factors of z_j B - A serve both sides); Rayleigh-Ritz uses
 * A' = Q^H A Q and B' = Q^H B Q (Cholesky-QR in the B inner product, twice).  Ritz vectors
 * are returned with x^H B x = 1, res_k = ||A x_k - lambda_k B x_k||_2 / anorm (anorm <= 0:
 * ||A||_2 estimated), and with opt->spurious = 1 the filter value is mu_k = Re(x_k^H B rho x_k).
 * FP64 and the FEAST method only (opt->prec = FEAST_FP64, opt->method = FEAST_METHOD_FEAST).
 * The factor cache is keyed by (A, B) pointers as well: call feast_invalidate if either
 * changes in place.
 * Argument positions: h=1 dt=2 n=3 A=4 lda=5 B=6 ldb=7 emin=8 emax=9 opt=10 X0=11 X=12
 * ldx=13 lambda=14 res=15 m=16 iters=17; returns as feast_solve. */
int feast_solve_gen(feast_handle h, feast_dtype dt, int n, const void* A, int lda, const void* B,
                    int ldb, double emin, double emax, const feast_opts* opt, const void* X0,
                    void* X, int ldx, double* lambda, double* res, int* m, int* iters,
                    double* trace);

/* Q = rho(B^{-1} A) X for the pencil (A, B) as above (prec must be FEAST_FP64).
 * Argument positions: h=1 dt=2 n=3 A=4 lda=5 B=6 ldb=7 emin=8 emax=9 n_c=10 prec=11 X=12
 * ldx=13 m0=14 Q=15 (!= X) ldq=16. */
int feast_filter_apply_gen(feast_handle h, feast_dtype dt, int n, const void* A, int lda,
                           const void* B, int ldb, double emin, double emax, int n_c,
                           feast_precision prec, const void* X, int ldx, int m0, void* Q,
                           int ldq);

/* Outcome of the last feast_solve / feast_solve_gen on a handle (host values). */
typedef struct {
  int iters;               /* iterations run */
  int filter_applications; /* applications of rho(A) (each solves the n_c shifted systems for
                              m0 right-hand sides, both adjoint sides for complex A) */
  int counted;             /* Ritz pairs that step 3 counted (the *m of the call) */
  double max_res;          /* largest residual over the counted pairs at the last iteration */
  double time_ms;          /* duration of the call on the handle's stream (HIP events) */
  long long filter_columns; /* right-hand-side columns filtered in all: m0 per application,
                               except that an application made for the filter-value test at
                               what step 3 then finds to be the last iteration filters only
                               the Ritz vectors inside I */
} feast_solve_info;

/* The step-3 decision of the last feast_solve / feast_solve_gen on h (Appendix, FEAST step 3;
 * RFEAST step 3 for the variant).  info: NULL or filled as above.  counted: NULL or host array
 * of m0 ints, counted[k] = 1 when Ritz pair k is one the convergence test counts: lambda_k
 * inside I and, with the filter-value test on, mu_k > 1/2 (or, for RFEAST without it, one of
 * the m_e lowest residuals inside I); 0 otherwise.  When the last iterate met step 3 as the
 * paper states it (every pair inside I at or below tol), the filter-value test is not needed
 * and mu_k (feast_get_filter_values) holds the scalar filter rho(lambda_k) instead of a
 * measured x_k^H rho(A) x_k.  Returns the number of counted pairs, or -1 (h NULL) / -4. */
int feast_get_solve_info(feast_handle h, feast_solve_info* info, int* counted, int m0);

/* One problem of a batch (device arrays owned by the caller, host outputs as in feast_solve).
 * X0 may be NULL (seeded Gaussian start); X0 and X share ldx. */
typedef struct {
  int n, lda, ldx, m0;
  const void* A;
  double emin, emax;
  double anorm;      /* <= 0: estimated */
  const void* X0;
  void* X;
  double* lambda;    /* host, m0 */
  double* res;       /* host, m0 */
  int* m;            /* host */
  int* iters;        /* host */
  int* status;       /* host: the feast_solve return code of this problem */
  double* mu;        /* host, m0, or NULL: filter values mu_k of the returned Ritz vectors
                        (written when opt->spurious = 1 or opt->prec is a mixed mode) */
  int* counted;      /* host, m0, or NULL: the step-3 mask of feast_get_solve_info */
  double* trace;     /* host, opt->max_iter, or NULL: the residual trace of feast_solve */
  feast_solve_info* info; /* host, or NULL: iterations, filter applications, time */
} feast_problem;

/* Independent FEAST problems (Sec. 1: disjoint intervals, or independent matrices, are solved
 * independently and in parallel).  Problems are ordered by decreasing n^3 (largest first)
 * and handed to nstreams workers, each with its own HIP stream (default priority) and its own
 * workspace, so small problems overlap on the device.  opt supplies n_c, max_iter, tol, prec,
 * refine_max, spurious and seed; m0 and anorm come from each problem.  Work already queued on
 * the handle's stream (for example the writes of A and X0) completes before any worker reads
 * the inputs: every worker stream waits for an event recorded on it at entry.  The call
 * returns after every worker has synchronised its stream.
 * Argument positions: h=1 dt=2 nprob=3 probs=4 opt=5 nstreams=6 (1..32).
 * Returns 0 when every problem returned FEAST_OK, else the number of problems that did not
 * (their own codes are in *status). */
int feast_solve_batched(feast_handle h, feast_dtype dt, int nprob, const feast_problem* probs,
                        const feast_opts* opt, int nstreams);

/* mu_k of the Ritz vectors returned by the last feast_solve with opt->spurious = 1 (host
 * array of m0 doubles).  When the last filter application covered only the Ritz vectors
 * inside I (see filter_columns above), mu_k of the pairs outside I is the scalar filter
 * rho(lambda_k).  Returns the number of values written. */
int feast_get_filter_values(feast_handle h, double* mu, int m0);

/* Phase timings of the last feast_solve / feast_filter_apply / feast_rayleigh_ritz call, in
 * milliseconds measured with HIP events on the handle's stream:
 * out[0] factorization (shift + LU + diagonal-block inverses), out[1] triangular solves,
 * out[2] accumulation, out[3] Rayleigh-Ritz, out[4] refinement (mixed modes), out[5] total.
 * Returns the number of values written (<= count). */
int feast_get_timings(feast_handle h, double* out, int count);

/* Kernel-level profiling: when enabled, every matrix-core GEMM launch is bracketed with HIP
 * events on the handle's stream and attributed to a class.  Classes: 0 LU trailing update,
 * 1 triangular-solve sweeps, 2 Rayleigh-Ritz, 3 refinement residual, 4 other.
 * feast_get_kernel_stats returns total kernel milliseconds, launch count and dense GEMM
 * flops (8 M N K per complex product) accumulated since profiling was enabled, summed over h
 * and its batch workers (whose kernels overlap in time).  Class 5 covers the dense Hermitian
 * eigensolves (Rayleigh-Ritz and the Gram matrices of XFEAST/RFEAST): milliseconds, Jacobi
 * sweeps in place of launches, and the number of eigensolves in place of flops. */
int feast_set_profiling(feast_handle h, int on);
int feast_get_kernel_stats(feast_handle h, int kclass, double* total_ms, long long* launches,
                           double* dense_flops);

#ifdef __cplusplus
}
#endif
#endif
