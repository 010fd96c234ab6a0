// Internal launchers of the FEAST MI355X library.  All device pointers; every launch is
// asynchronous on the given stream.
#pragma once
#include "common.h"

namespace feast {

// Two nested strided batch dimensions (element strides), n1 x n2 problems.
// With splitk > 0 the first batch dimension instead cuts K into chunks of splitk (the
// n1 partial products go to C + b1 * sC1; sA1/sB1 are ignored).
// tri = 1 (2): op(A) is square lower (upper) triangular, M = K; each row tile multiplies only
// the K range of the nonzero part (the zero part of A is never read).
struct Batch {
  int n1 = 1, n2 = 1;
  long sA1 = 0, sA2 = 0, sB1 = 0, sB2 = 0, sC1 = 0, sC2 = 0;
  int splitk = 0;
  int tri = 0;
};

// Optional per-thread hook that brackets every GEMM launch (kernel-level profiling).
struct GemmProfiler {
  virtual void begin(hipStream_t s) = 0;
  virtual void end(hipStream_t s, double dense_flops) = 0;
  virtual ~GemmProfiler() {}
};
extern thread_local GemmProfiler* g_gemm_prof;

// When set (per thread), complex FP32 products (cgemm, cgemm_pair) run as bf16x3: each FP32
// operand split into bf16 hi + lo, three bf16 matrix-core products with FP32 accumulation.
extern thread_local bool g_split_bf16;
struct SplitBf16Scope {
  bool saved;
  explicit SplitBf16Scope(bool on) : saved(g_split_bf16) { g_split_bf16 = on; }
  ~SplitBf16Scope() { g_split_bf16 = saved; }
};

// When set (per thread), complex FP64 products (zgemm, zgemm_pair, zgemm_nn_split) run as
// three real MFMA products (Re Re, Im Im, (Re + Im)(Re + Im)) instead of four: a quarter less
// matrix-core work, with a normwise error bound a few times the four-product one.  The
// Rayleigh-Ritz step sets it; the factorization and the sweeps, whose errors set the FP64
// residual floor, do not.  FP32 products always use the three-product form.
extern thread_local bool g_z3m;
struct Z3mScope {
  bool saved;
  explicit Z3mScope(bool on) : saved(g_z3m) { g_z3m = on; }
  ~Z3mScope() { g_z3m = saved; }
};

// C = alpha op(A) op(B) + beta C (column-major, complex; FP64 or FP32 matrix cores).
void zgemm(hipStream_t s, int opA, int opB, int M, int N, int K, zd alpha, const zd* A, long lda,
           const zd* B, long ldb, zd beta, zd* C, long ldc, const Batch& bt = Batch());
void cgemm(hipStream_t s, int opA, int opB, int M, int N, int K, zf alpha, const zf* A, long lda,
           const zf* B, long ldb, zf beta, zf* C, long ldc, const Batch& bt = Batch());

// K-chunk count for C = A B (FP64, op N/N; K = the inner length) that spreads the output
// tiles of all chunks more evenly over the workgroups the device holds at once of the kernel
// the calling thread's product form selects (1 = no split; at most 8, chunks of at least 256).
int zgemm_kchunks(int M, int N, int K);
// C = A B (beta = 0).  nchunk > 1: partial products of K chunks into part
// (nchunk * M * N elements, ld M), then summed into C in chunk order.
void zgemm_nn_split(hipStream_t s, int M, int N, int K, const zd* A, long lda, const zd* B,
                    long ldb, zd* C, long ldc, int nchunk, zd* part);

// Two problems with equal M, N, K (own pointers, leading dimensions, op(A)) in one launch.
void zgemm_pair(hipStream_t s, int opA0, int opA1, int opB, int M, int N, int K, zd alpha,
                const zd* const A[2], const long lda[2], const zd* const B[2], const long ldb[2],
                zd beta, zd* const C[2], const long ldc[2], const Batch& bt = Batch());
void cgemm_pair(hipStream_t s, int opA0, int opA1, int opB, int M, int N, int K, zf alpha,
                const zf* const A[2], const long lda[2], const zf* const B[2], const long ldb[2],
                zf beta, zf* const C[2], const long ldc[2], const Batch& bt = Batch());

// Quadrature of the filter (feast_api.hip): z[j], omega[j] for j < nc on the host.
void quadrature_nodes(double emin, double emax, int nc, zd* z, zd* omega);

// ---- LU (lu.hip) ---------------------------------------------------------------------
// Shifted copies M_j = z_j B - A (j < nc; B = I when B == nullptr) of real (is_real) or
// complex n x n matrices into np x np factor storage (ld = np, batch stride np*np);
// rows/cols n..np-1 set to identity.  *flag (device int, cleared by the caller) becomes
// nonzero when a shifted entry is not finite in the storage precision.
void shift_matrices(hipStream_t s, const void* A, long lda, int is_real, int n, int np,
                    const zd* z_dev, int nc, zd* M, int* flag, const void* B = nullptr,
                    long ldb = 0);
void shift_matrices_f32(hipStream_t s, const void* A, long lda, int is_real, int n, int np,
                        const zd* z_dev, int nc, zf* M, int* flag, const void* B = nullptr,
                        long ldb = 0);

// Workspace for the batched LU with partial pivoting.
struct LuWork {
  int* retired = nullptr;   // nc * np, panel stamp of rows chosen as pivots
  double* pval = nullptr;   // 2 * nc * maxwg, pivot-search partials (value)
  int* prow = nullptr;      // 2 * nc * maxwg, pivot-search partials (row)
  int* pivrows = nullptr;   // nc * 64, pivot rows of the current panel
  int* moves = nullptr;     // nc * (4 * 64 + 1): per node a count, then up to 2 * 64
                            // (dst, src) row moves of the current panel
  int* perm = nullptr;      // nc * np, P as a row gather: (P X)[r] = X[perm[r]]
  int* pinv = nullptr;      // nc * np, inverse of perm
  int* flag = nullptr;      // 1 int: set to 1 + column of the first exact zero pivot
  void* linv = nullptr;     // 8 * nc * 64 * 64 complex: inverses of the L11 blocks of the
                            // current outer panel's sub-panels
  void* u12 = nullptr;      // nc * 64 * np complex: staging copy of the panel's rows of A12
  bool column_steps = false;  // one launch per panel column throughout (no short-panel
                              // groups); the same factors, a reference schedule for tests
};
size_t lu_work_bytes(int np, int nc);
void lu_work_carve(LuWork& w, void* base, int np, int nc);

// In-place batched LU with partial pivoting of nc matrices (np x np, ld = np).
void lu_factor_f64(hipStream_t s, zd* M, int np, int nc, LuWork& w);
void lu_factor_f32(hipStream_t s, zf* M, int np, int nc, LuWork& w);

// ---- triangular solves (solve.hip) -----------------------------------------------------
// Inverses of the nbt x nbt diagonal blocks of the unit-lower L and upper U factors
// (nb = np / nbt blocks per node, stored densely with ld = nbt, node stride np*nbt).
void tri_inverse_blocks_f64(hipStream_t s, const zd* LU, int np, int nc, int nbt, zd* invL,
                            zd* invU, zd* tmp);
void tri_inverse_blocks_f32(hipStream_t s, const zf* LU, int np, int nc, int nbt, zf* invL,
                            zf* invU, zf* tmp);

// Rows of X gathered by the node permutations: B0_j[r] = X[perm_j[r]] (side 0) and
// B1_j = X (side 1); X is n x m0 (ldx), B is np x m0 per (node, side), padded with zeros.
void gather_rhs(hipStream_t s, const zd* X, long ldx, int n, int np, int m0, int nc, int sides,
                const int* perm, zd* B);
void gather_rhs_f32(hipStream_t s, const zd* X, long ldx, int n, int np, int m0, int nc,
                    int sides, const int* perm, zf* B);

// Height of the sweep blocks (and of the inverted diagonal blocks) for order n and the
// factors' precision class (0: FP64, 1: FP32 factors): the factors are padded to a multiple
// of it.  set_sweep_block_override(nbt) makes every later call return nbt (64, 128, 256 or
// 512; 0 restores the table), for tuning runs; returns -1 on any other value.
int sweep_block(int n, int prec_class);
int set_sweep_block_override(int nbt);
// Forward then backward block sweeps for all (node, side) systems.  B (input RHS, destroyed)
// and Y (output) are [nc][sides] blocks of np x m0.
void solve_sweeps_f64(hipStream_t s, const zd* LU, const zd* invL, const zd* invU, int np,
                      int nc, int nbt, int sides, int m0, zd* B, zd* Y);
void solve_sweeps_f32(hipStream_t s, const zf* LU, const zf* invL, const zf* invU, int np,
                      int nc, int nbt, int sides, int m0, zf* B, zf* Y);

// Q = sum_j omega_j Y0_j + conj(omega_j) P_j^T Y1_j (sides == 2) or sum_j 2 Re(omega_j Y0_j)
// (sides == 1); Q is n x m0 (ldq).
void accumulate(hipStream_t s, const zd* Y, int n, int np, int m0, int nc, int sides,
                const zd* omega_dev, const int* pinv, zd* Q, long ldq);

// ---- mixed precision (mixed.hip) -------------------------------------------------------
void seeded_rhs(hipStream_t s, const zd* R, long ldr, const double* lam, const zd* z,
                const int* perm, int n, int np, int m0, int nc, int sides, zf* B);
void filter_values(hipStream_t s, const double* lam, const zd* z, const zd* omega, int nc, int m0,
                   double* rho);
void accumulate_mixed(hipStream_t s, const zd* X, long ldx, const double* rho, const zf* D, int n,
                      int np, int m0, int nc, int sides, const zd* omega, const int* pinv, zd* Q,
                      long ldq);
void unpermute_to64(hipStream_t s, const zf* D, const int* pinv, int n, int np, int m0, int nc,
                    int sides, int add, zd* Y);
// rmax (device, nullable): receives max |R| over all entries as the bits of a double.
void refine_rhs(hipStream_t s, const zd* X, long ldx, const zd* Y, const zd* AY, const zd* z,
                const int* perm, int n, int np, int m0, int nc, int sides, zf* B,
                unsigned long long* rmax = nullptr);
void accumulate_plain(hipStream_t s, const zd* Y, int n, int np, int m0, int nc, int sides,
                      const zd* omega, zd* Q, long ldq);

// ---- Rayleigh-Ritz helpers (rr.hip) -------------------------------------------------------
void reduce_partials_hermitian(hipStream_t s, const zd* part, int nparts, int m, zd* G, int ldg);
// Blocked Cholesky G = R^H R (upper R, in place, ld = ldg); *flag set on breakdown.
void cholesky_upper(hipStream_t s, zd* G, int m, int ldg, int* flag, zd* tmp);
// Rinv = R^{-1} for upper triangular R (m x m); Rinv must be zeroed by the call.
void upper_inverse(hipStream_t s, const zd* R, int m, int ldr, zd* Rinv, int ldi, zd* tmp);
// Cyclic two-sided Jacobi on the Hermitian m x m matrix H (ld = m, not modified) in a
// block-pair parallel ordering (blocks of 16 indices; per outer round each pair of blocks
// runs one inner sweep in LDS, then the round's block rotations are applied to the rest).
// A rotation is skipped when |h_pq| <= max(1e-17 sqrt(|h_pp h_qq|), eps ||H||_F); a sweep
// ends the iteration when no off-diagonal entry exceeds max(1e-17 sqrt(|h_pp h_qq|), 4 eps ||H||_F).
// Returns sweeps used (host sync per sweep) or -1.  d (device, mp) eigenvalues unsorted,
// V (device, mp x mp, ld mp) eigenvectors; work: jacobi_work(mp) complex.
// One sweep is recorded as a HIP graph (rounds, then a fill kernel and the check: no memset
// node) and replayed per sweep when cache is given; the graph is re-recorded when the sizes
// or buffers change.
struct JacobiGraph {
  void* graph = nullptr;
  void* exec = nullptr;
  int mp = 0;
  const void* A0 = nullptr;
  const void* V = nullptr;
  const void* flag = nullptr;
  JacobiGraph() = default;
  JacobiGraph(const JacobiGraph&) = delete;
  JacobiGraph& operator=(const JacobiGraph&) = delete;
  ~JacobiGraph();
};
// mp = padded order (a multiple of 32, >= m; rows/columns beyond m are decoupled and sort
// last).
int jacobi_eigh(hipStream_t s, zd* H, int m, double* d, zd* V, zd* work, int* dflag,
                int max_sweeps, JacobiGraph* cache, int mp);
inline int jacobi_order(int m) { return (m + 31) / 32 * 32; }
// Complex entries of jacobi_eigh's work array at padded order mp.
inline size_t jacobi_work(int mp) { return (size_t)mp * mp + 32 * (size_t)mp + 40; }
// Padded order used by callers that record sweeps for several nearby sizes.
inline int jacobi_order_quantized(int m) { return jacobi_order(m); }
// Stable ascending sort of d; Wout = V[:, order] (first m columns), lam = d[order].
void sort_eigen(hipStream_t s, const double* d, const zd* V, int m, int mp, double* lam, zd* W,
                int* rank);
// R = AX - X diag(lam) (n x m0, ld n).
void ritz_residual(hipStream_t s, const zd* AX, long ldax, const zd* X, long ldx,
                   const double* lam, int n, int m0, zd* R);
// res_k = || AX_k - lam_k X_k ||_2 / anorm.
void residual_norms(hipStream_t s, const zd* AX, long ldax, const zd* X, long ldx,
                    const double* lam, int n, int m0, double anorm, double* res);
// out[k] = Re(sum_i conj(X[i,k]) Y[i,k]), k < m0.
void coldot_re(hipStream_t s, const zd* X, long ldx, const zd* Y, long ldy, int n, int m0,
               double* out);
void copy_matrix(hipStream_t s, const zd* src, long lds, zd* dst, long ldd, int rows, int cols);
void real_to_complex(hipStream_t s, const double* src, long lds, zd* dst, long ldd, int rows,
                     int cols);
void complex_to_real(hipStream_t s, const zd* src, long lds, double* dst, long ldd, int rows,
                     int cols);
void fill_zero(hipStream_t s, void* p, size_t bytes);
// diag[k] = Re G[k, k] (k < m).
void diag_real(hipStream_t s, const zd* G, int m, int ldg, double* diag);
// G[k, k] += sigma (k < m).
void add_diag(hipStream_t s, zd* G, int m, int ldg, double sigma);
// Seeded Gaussian block (counter-based splitmix64 + Box-Muller): complex entries get
// independent N(0,1) real and imaginary parts, real entries (is_real) N(0,1).
void gaussian_fill(hipStream_t s, void* X, long ldx, int rows, int cols, int is_real,
                   unsigned long long seed);
// Power-iteration estimate of ||A||_2 (iters steps from a seeded start vector).
double norm2_estimate(hipStream_t s, const zd* A, long lda, int n, int iters, zd* work,
                      double* dnorm);
int nonfinite_check(hipStream_t s, const zd* a, long ld, int rows, int cols, int* dflag);

// ---- Expanded-subspace variants (xr.hip) ------------------------------------------------
// B[:, c] /= ||B[:, c]||_2 for c < k (zero columns stay zero).
void normalize_columns(hipStream_t s, zd* B, long ldb, int n, int k);
// T (k x r, ld k) = V[:, keep[j]] / sqrt(d[keep[j]]), j < r.
void gram_basis(hipStream_t s, const double* d, const zd* V, long ldv, const int* keep, int k,
                int r, zd* T);
// dst[:, a] = src[:, idx[a]] (n rows), a < cnt.
void gather_columns(hipStream_t s, const zd* src, long lds, const int* idx, int n, int cnt, zd* dst,
                    long ldd);
// dst[a] = src[idx[a]], a < cnt.
void gather_values(hipStream_t s, const double* src, const int* idx, int cnt, double* dst);

}  // namespace feast
