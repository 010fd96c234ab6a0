/* feast_noalloc.h -- allocation-free variant of feast_filter_apply (libfeast_mi355x.so).
 *
 * For callers that cannot allocate device memory: code recorded under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same computation as
 * feast_filter_apply with prec = FEAST_FP64 (feast.h): Q = rho(A) X by the quadrature of
 * Sec. 1 eq. (contour_int_quad), refactoring z_j I - A on every call (no factor cache).
 *
 * Every intermediate (the n_c factorizations, the inverted diagonal blocks, the right-hand-side
 * blocks, the LU workspace and the quadrature nodes) lives in one static device array of
 * FEAST_NOALLOC_SCRATCH_MB MiB that each GPU running the library holds until the process
 * ends; the call makes no hipMalloc, hipFree or other allocating call.  With nbt the sweep
 * block height (64 for n < 384, 128 below 2048, 256 below 8192, else 512), np = n rounded up
 * to a multiple of nbt and sides = 2 (FEAST_C128) or 1 (FEAST_R64), the call needs about
 *   16 * n_c * (np^2 + 2 np nbt + 2 sides np m0) + 16 np nbt  (+ 32 n m0 for FEAST_R64)
 * bytes; a larger problem returns FEAST_ERR_SCRATCH before any device work (n = 1024,
 * n_c = 8, m0 = 128 complex fits).
 *
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU (from several
 * streams or threads) race and must be serialised by the caller.  The array keeps the last
 * call's contents; what must start at zero is cleared by each call.
 *
 * Arguments as feast_filter_apply without the handle and precision: A, X, Q are device
 * pointers owned by the caller (column-major, interleaved complex for FEAST_C128); hip_stream
 * may be NULL (the legacy default stream).  The call synchronises hip_stream before it
 * returns.  Argument positions for negative codes: dt=1 n=2 A=3 lda=4 emin=5 emax=6
 * (emin < emax) n_c=7 (1..128) X=8 ldx=9 m0=10 (1 <= m0 <= n) Q=11 (!= X) ldq=12.
 * Returns 0, a negative argument position, FEAST_ERR_SCRATCH, FEAST_NONFINITE,
 * FEAST_ZERO_PIVOT or FEAST_ERR_HIP.
 */
#ifndef FEAST_MI355X_NOALLOC_H
#define FEAST_MI355X_NOALLOC_H
#include "feast.h"

#ifdef __cplusplus
extern "C" {
#endif

#define FEAST_NOALLOC_SCRATCH_MB 256
#define FEAST_ERR_SCRATCH (-103) /* the problem needs more than the static scratch array */

int feast_filter_apply_noalloc(feast_dtype dt, int n, const void* A, int lda, double emin,
                               double emax, int n_c, const void* X, int ldx, int m0, void* Q,
                               int ldq, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
