/* feast_kernels.h -- building blocks of the MI355X FEAST hot path, exported for kernel-level
 * parity tests and measurements.  Same conventions as feast.h: column-major, interleaved
 * complex, device pointers owned by the caller, hip_stream may be NULL.  Every call is
 * asynchronous on hip_stream except where it says it synchronises.  Returns 0, a negative
 * argument position, or FEAST_ERR_HIP (-101).
 */
#ifndef FEAST_MI355X_KERNELS_H
#define FEAST_MI355X_KERNELS_H
#ifdef __cplusplus
extern "C" {
#endif

/* C = alpha op(A) op(B) + beta C on the matrix cores; op: 0 = N, 1 = T, 2 = C (conjugate
 * transpose).  prec 0: complex128 data and FP64 MFMA; prec 1: complex64 data and FP32 MFMA;
 * prec 2: complex64 data, each operand split into bf16 hi + lo parts, three bf16 MFMA products
 * (hi hi + hi lo + lo hi) with FP32 accumulation (relative error ~2^-16 per product term);
 * prec 3: complex128 data, each complex product from three real FP64 MFMA products
 * (Re Re, Im Im, (Re + Im)(Re + Im)), the form the Rayleigh-Ritz products use.
 * Complex64 products (prec 1) always use the three-product form.
 * alpha, beta: host arrays {re, im}.  A and B may be NULL when K == 0 (C = beta C).  This is the dense contraction used by the LU trailing
 * updates, the block triangular sweeps and Q^H A Q (Sec. 1 linear solves; Appendix step 2).
 * Argument positions: prec=1 opA=2 opB=3 M=4 N=5 K=6 alpha=7 A=8 lda=9 B=10 ldb=11 beta=12
 * C=13 ldc=14. */
int feast_kern_gemm(int prec, int opA, int opB, int M, int N, int K, const double* alpha,
                    const void* A, long lda, const void* B, long ldb, const double* beta,
                    void* C, long ldc, void* hip_stream);

/* Batched LU with partial pivoting of M_j = z_j I - A (complex Hermitian A, n x n, lda), the
 * factorizations behind each quadrature term of Sec. 1 eq. (contour_int_quad).
 * z: host array of 2*nc doubles (interleaved nodes).  np = n rounded up as the library pads
 * (returned in *np_out when LU is NULL, without other work).  LU: nc blocks of np x np
 * (ld np, complex128 for prec 0, complex64 for prec 1 and 2; the trailing updates are
 * four-product FP64 (prec 0) or three-product FP32 (prec 1) products, or bf16x3 products
 * (prec 2), see feast_kern_gemm) receiving unit-lower L and U; perm:
 * nc blocks of np ints with (P M)[r] = M[perm[r]].  prec + 8: the same factorization with
 * one launch per panel column throughout (the solver runs a panel's column groups as single
 * launches once few rows remain; both schedules give bit-identical factors).  Synchronises
 * the stream; returns 6 on an exact zero pivot. */
int feast_kern_lu(int prec, const void* A, int lda, int n, int nc, const double* z, void* LU,
                  int* perm, int* np_out, void* hip_stream);

/* The block triangular sweeps of the Sec. 1 linear solves on given factors (the solver's own
 * launches, for tests and counter runs).  LU: nc blocks of np x np (ld np; complex128 for
 * prec 0, complex64 for prec 1 and 2, as feast_kern_lu writes them: unit-lower L and U of
 * P M_j).  invL, invU: nc blocks of np x nbt receiving (compute_inverses != 0) or holding the
 * inverses of the nbt x nbt diagonal blocks of L and U.  B: nc blocks of sides x np x m0
 * (ld np): on entry the right-hand sides, on exit side 0 holds (L U)^{-1} B_0 and side 1
 * (L U)^{-H} B_1 (both adjoint systems of the quadrature share the factors); Z: scratch of
 * B's size.  With LU NULL only np and nbt are returned (*np_out, *nbt_out).  Synchronises the
 * stream.  Returns 0, -1..-7 for an invalid argument (prec, n, nc, m0, sides, invL/invU,
 * B/Z), -101 on a HIP error. */
int feast_kern_sweeps(int prec, int n, int nc, int m0, int sides, const void* LU, void* invL,
                      void* invU, int compute_inverses, void* B, void* Z, int* np_out,
                      int* nbt_out, void* hip_stream);

/* Tuning hook for the block triangular sweeps of the Sec. 1 linear solves: every later
 * factorization (and its solves) uses sweep blocks of nbt rows (64, 128, 256 or 512) and pads
 * the factors to a multiple of nbt; nbt = 0 restores the built-in table (measured per
 * precision and order by the package's autotune module).  Process-wide: set it only while no
 * solve is running.  Returns 0, or -1 for any other nbt (the setting is then unchanged). */
int feast_tune_sweep_block(int nbt);

/* Test hook for the filter application that a FEAST iteration with the filter-value test on
 * makes after Rayleigh-Ritz (Appendix FEAST step 3 reads mu_k only inside I).  mode 0 (the
 * default): when every pair counted at the previous iteration now has a residual at most
 * tol, the Ritz vectors inside I are filtered first and the other columns only if step 3 does
 * not stop; mode 1: that split is made at every such application.  Each column is filtered
 * on its own, so both modes give the same iterates; mode 1 exists to exercise the second
 * half of the split.  Process-wide: set it only while no solve is running.  Returns 0, or -1
 * for any other mode (the setting is then unchanged). */
int feast_tune_split_filter(int mode);

/* Parallel-order two-sided Jacobi eigendecomposition of a Hermitian m x m matrix H
 * (ld m, complex128, not modified): the reduced eigenproblem of the Appendix, step 2.i.
 * d: device m doubles (eigenvalues ascending); W: device m x m eigenvectors (ld m).
 * Synchronises the stream; returns the sweep count (>= 0) or -1 if not converged. */
int feast_kern_jacobi(const void* H, int m, double* d, void* W, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
