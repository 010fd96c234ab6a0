// C-ABI of the FEAST hot path: handle, factor cache, filter application, Rayleigh-Ritz and
// the FEAST loop (Appendix, FEAST algorithm).  Host code only orchestrates launches on the
// handle's stream; every arithmetic step of the path runs in this library's kernels.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/feast.h"
#include "../../include/feast_noalloc.h"
#include "common.h"
#include "kernels.h"

using namespace feast;

namespace {

void gauss_legendre_gw(int n, std::vector<double>& x, std::vector<double>& w);

}  // namespace

// Nodes and weights of the quadrature (readings of Sec. 1, eq. contour_int_quad): circle of
// centre c = (emin + emax)/2 and radius r = (emax - emin)/2, Gauss-Legendre abscissae x_j on
// the upper half circle theta_j = (pi/2)(1 - x_j), z_j = c + r e^{i theta_j},
// omega_j = (w_j / 4) r e^{i theta_j}.
void feast::quadrature_nodes(double emin, double emax, int nc, zd* z, zd* omega) {
  std::vector<double> x, w;
  gauss_legendre_gw(nc, x, w);
  const double c = 0.5 * (emin + emax), r = 0.5 * (emax - emin);
  for (int j = 0; j < nc; ++j) {
    double th = 0.5 * M_PI * (1.0 - x[j]);
    double ct = std::cos(th), st = std::sin(th);
    z[j] = zmake(c + r * ct, r * st);
    omega[j] = zmake(0.25 * w[j] * r * ct, 0.25 * w[j] * r * st);
  }
}

namespace {

// ---------------------------------------------------------------------------------------
// Gauss-Legendre nodes/weights (the "Gauss quadrature" of Sec. 1) by the Golub-Welsch
// characterisation: the nodes are the eigenvalues of the symmetric tridiagonal Jacobi matrix
// of the Legendre recurrence (zero diagonal, off-diagonal k / sqrt(4k^2 - 1)), found here by
// Sturm-sequence bisection; the weight of node x is 2 v_0^2 = 1 / sum_k p_k(x)^2 with p_k
// the Legendre polynomials normalised on [-1, 1] (Christoffel function).
// ---------------------------------------------------------------------------------------
int sturm_count(int n, double x) {  // number of eigenvalues < x
  int cnt = 0;
  double q = -x;
  if (q < 0) cnt++;
  for (int k = 1; k < n; ++k) {
    double b2 = (double)k * k / (4.0 * k * k - 1.0);
    if (q == 0.0) q = 1e-300;
    q = -x - b2 / q;
    if (q < 0) cnt++;
  }
  return cnt;
}

void gauss_legendre_gw(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {  // i-th smallest eigenvalue in (-1, 1)
    double lo = -1.0, hi = 1.0;
    for (int it = 0; it < 200 && hi - lo > 0; ++it) {
      double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (sturm_count(n, mid) > i) hi = mid;
      else lo = mid;
    }
    double xi = 0.5 * (lo + hi);
    // orthonormal Legendre values p_k(x) = sqrt((2k+1)/2) P_k(x)
    double pkm1 = 1.0, pk = xi, s = 0.5;  // p_0^2 = 1/2
    if (n > 1) s += 1.5 * xi * xi;
    for (int k = 1; k + 1 < n; ++k) {
      double pk1 = ((2.0 * k + 1.0) * xi * pk - k * pkm1) / (k + 1.0);
      pkm1 = pk;
      pk = pk1;
      s += (2.0 * (k + 1) + 1.0) / 2.0 * pk * pk;
    }
    x[i] = xi;
    w[i] = 1.0 / s;
  }
}

// ---------------------------------------------------------------------------------------
// Device buffer owned by a handle; grows on demand and is freed with the handle (every Buf
// member, including those feast_destroy does not list, through this destructor).
struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  Buf() = default;
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  ~Buf() { release(); }
  template <typename T>
  T* get(size_t count) {
    size_t need = count * sizeof(T);
    if (need == 0) need = 256;
    if (need > bytes) {
      if (p) FEAST_HIP(hipFree(p));
      p = nullptr;
      bytes = 0;
      hipError_t e = hipMalloc(&p, need);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        throw std::bad_alloc();
      }
      bytes = need;
    }
    return (T*)p;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

struct EventPool {
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  hipEvent_t take() {
    if (used == ev.size()) {
      hipEvent_t e;
      FEAST_HIP(hipEventCreate(&e));
      ev.push_back(e);
    }
    return ev[used++];
  }
  void reset() { used = 0; }
  ~EventPool() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

// Sweep cap of the dense Hermitian eigensolves: the block-pair Jacobi takes about 10 sweeps
// on random Hermitian matrices and 30-33 on the strongly graded Gram matrices of the
// expanded-subspace methods; a solve that needs more than this reports FEAST_EIG_FAILED.
constexpr int kJacobiMaxSweeps = 60;

// 1: every filter application made for the filter-value test filters the Ritz vectors inside
// I first and the other columns after step 3 (a test hook for that path); 0: only when the
// iteration is likely the last.
std::atomic<int> g_split_filter{0};

constexpr int NCLASS = 6;
enum { K_LU = 0, K_SOLVE = 1, K_RR = 2, K_REFINE = 3, K_OTHER = 4, K_EIG = 5 };

struct KernelProfiler : GemmProfiler {
  bool on = false;
  int cls = K_OTHER;
  EventPool pool;
  struct Rec {
    hipEvent_t a, b;
    int cls;
    double flops;
  };
  std::vector<Rec> pending;
  hipEvent_t cur_a = nullptr;
  double ms[NCLASS] = {0}, flops[NCLASS] = {0};
  long long launches[NCLASS] = {0};
  void begin(hipStream_t s) override {
    cur_a = pool.take();
    FEAST_HIP(hipEventRecord(cur_a, s));
  }
  void end(hipStream_t s, double f) override {
    hipEvent_t b = pool.take();
    FEAST_HIP(hipEventRecord(b, s));
    pending.push_back({cur_a, b, cls, f});
  }
  // An eigensolve: its time (events a..b), sweeps counted as launches, one per call as flops.
  std::vector<std::pair<long long, int>> eig_pending;
  void eig(hipStream_t s, hipEvent_t a, int sweeps) {
    hipEvent_t b = pool.take();
    FEAST_HIP(hipEventRecord(b, s));
    pending.push_back({a, b, K_EIG, 1.0});
    eig_pending.push_back({(long long)std::max(sweeps, 0), 1});
  }
  void flush() {  // stream must be synchronised; an eigensolve counts its sweeps (>= 0)
    for (auto& e : eig_pending) launches[K_EIG] += e.first - 1;  // the record below adds 1
    eig_pending.clear();
    for (auto& r : pending) {
      float t = 0;
      FEAST_HIP(hipEventElapsedTime(&t, r.a, r.b));
      ms[r.cls] += t;
      flops[r.cls] += r.flops;
      launches[r.cls] += 1;
    }
    pending.clear();
    pool.reset();
  }
};

enum { P_FACTOR = 0, P_SOLVE = 1, P_ACC = 2, P_RR = 3, P_REFINE = 4, P_TOTAL = 5 };

// Phase timer: pairs of events accumulated into phase totals at flush().  The whole call is
// bracketed by two events of its own (begin_total / end_total), which the pool's reuse after
// each flush never hands out again.
struct PhaseTimer {
  EventPool pool;
  struct Rec {
    hipEvent_t a, b;
    int phase;
  };
  std::vector<Rec> pending;
  double ms[6] = {0};
  hipEvent_t t_begin = nullptr, t_end = nullptr;
  bool total_open = false;
  hipEvent_t mark(hipStream_t s) {
    hipEvent_t e = pool.take();
    FEAST_HIP(hipEventRecord(e, s));
    return e;
  }
  void add(hipEvent_t a, hipEvent_t b, int phase) { pending.push_back({a, b, phase}); }
  void begin_total(hipStream_t s) {
    if (!t_begin) FEAST_HIP(hipEventCreate(&t_begin));
    if (!t_end) FEAST_HIP(hipEventCreate(&t_end));
    FEAST_HIP(hipEventRecord(t_begin, s));
    total_open = true;
  }
  // Records the end of the call; the caller synchronises the stream, then flushes.
  void end_total(hipStream_t s) {
    if (!total_open) return;
    FEAST_HIP(hipEventRecord(t_end, s));
    pending.push_back({t_begin, t_end, P_TOTAL});
    total_open = false;
  }
  void flush() {
    for (auto& r : pending) {
      float t = 0;
      FEAST_HIP(hipEventElapsedTime(&t, r.a, r.b));
      ms[r.phase] += t;
    }
    pending.clear();
    pool.reset();
  }
  void clear() {
    for (double& v : ms) v = 0;
    total_open = false;
  }
  ~PhaseTimer() {
    if (t_begin) (void)hipEventDestroy(t_begin);
    if (t_end) (void)hipEventDestroy(t_end);
  }
};

struct ScopedProf {
  KernelProfiler* kp;
  int saved;
  ScopedProf(KernelProfiler& p, int cls) : kp(&p), saved(p.cls) {
    p.cls = cls;
    g_gemm_prof = p.on ? &p : nullptr;
  }
  ~ScopedProf() {
    kp->cls = saved;
    g_gemm_prof = nullptr;
  }
};

}  // namespace

struct feast_ctx {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  std::string last_error;
  // factor cache
  bool f_valid = false;
  const void* f_A = nullptr;
  const void* f_B = nullptr;  // pencil (A, B); nullptr: B = I
  int f_n = 0, f_lda = 0, f_ldb = 0, f_dt = -1, f_nc = 0, f_prec = -1, f_np = 0, f_nbt = 0;
  double f_emin = 0, f_emax = 0;
  std::vector<zd> z, omega;
  Buf b_fac, b_invL, b_invU, b_tri_tmp, b_luw, b_z, b_omega;
  LuWork luw;
  // complex copies of a real A and B (Rayleigh-Ritz operands)
  const void* ac_A = nullptr;
  int ac_n = 0, ac_lda = 0;
  bool ac_valid = false;
  Buf b_Ac;
  const void* bc_B = nullptr;
  int bc_n = 0, bc_ldb = 0;
  bool bc_valid = false;
  Buf b_Bc, b_BQ, b_BX, b_BXf;
  // right-hand sides / solutions
  Buf b_B, b_Z, b_Xc, b_Qc, b_X0c;
  // Rayleigh-Ritz
  Buf b_Q1, b_Q2, b_AQ, b_AX, b_G, b_part, b_Rinv, b_rrtmp, b_H, b_jac, b_V, b_d, b_lam, b_res,
      b_rank, b_W, b_flag, b_diag, b_pow, b_mu, b_Reig, b_Y64, b_AY, b_rho, b_rmax, b_kpart;
  std::vector<double> mu;
  // outcome of the last solve: step 3's counted pairs, filter applications, iterations
  std::vector<int> counted;
  int last_filters = 0, last_iters = 0, last_count = 0;
  long long last_filter_cols = 0;  // right-hand-side columns filtered by the last solve
  double last_max_res = 0;
  PhaseTimer timer;
  KernelProfiler prof;
  std::map<int, JacobiGraph> jgraphs;  // recorded Jacobi sweeps, by padded order
  // expanded-subspace variants
  Buf b_win, b_U, b_Rsel, b_lsel, b_keep, b_sel, b_T;
  std::vector<int> keep_h, sel_h;
  // batched workers (each with its own stream and workspace)
  std::vector<feast_ctx*> workers;
  std::vector<hipStream_t> worker_streams;
};

namespace {

int fail_hip(feast_ctx* h, const HipError& e) {
  h->last_error = std::string(e.what) + ": " + hipGetErrorString(e.err);
  return FEAST_ERR_HIP;
}

// Factorizations of z_j I - A for all nodes (cached).
int ensure_factors(feast_ctx* h, int dt, int n, const void* A, int lda, double emin, double emax,
                   int nc, int prec, const void* B = nullptr, int ldb = 0) {
  if (h->f_valid && h->f_A == A && h->f_n == n && h->f_lda == lda && h->f_dt == dt &&
      h->f_nc == nc && h->f_prec == prec && h->f_emin == emin && h->f_emax == emax &&
      h->f_B == B && h->f_ldb == ldb)
    return 0;
  h->f_valid = false;
  hipStream_t s = h->stream;
  const int nbt = sweep_block(n, prec == FEAST_FP64 ? 0 : 1);
  const int np = (n + nbt - 1) / nbt * nbt;
  // nodes and weights
  h->z.resize(nc);
  h->omega.resize(nc);
  quadrature_nodes(emin, emax, nc, h->z.data(), h->omega.data());
  zd* zdev = h->b_z.get<zd>(nc);
  zd* odev = h->b_omega.get<zd>(nc);
  FEAST_HIP(hipMemcpyAsync(zdev, h->z.data(), sizeof(zd) * nc, hipMemcpyHostToDevice, s));
  FEAST_HIP(hipMemcpyAsync(odev, h->omega.data(), sizeof(zd) * nc, hipMemcpyHostToDevice, s));

  void* luw = h->b_luw.get<char>(lu_work_bytes(np, nc));
  lu_work_carve(h->luw, luw, np, nc);
  hipEvent_t e0 = h->timer.mark(s);
  int st = 0;
  // The shift flags non-finite shifted entries (NaN/Inf in A or B; for FP32 factors also
  // entries beyond the FP32 range) before any factorization work.
  auto shifted_finite = [&]() {
    int flag = 0;
    FEAST_HIP(hipMemcpyAsync(&flag, h->luw.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    FEAST_HIP(hipStreamSynchronize(s));
    return flag == 0;
  };
  fill_zero(s, h->luw.flag, sizeof(int));
  if (prec == FEAST_FP64) {
    zd* F = h->b_fac.get<zd>((size_t)nc * np * np);
    shift_matrices(s, A, lda, dt == FEAST_R64, n, np, zdev, nc, F, h->luw.flag, B, ldb);
    if (!shifted_finite()) return FEAST_NONFINITE;
    {
      ScopedProf sp(h->prof, K_LU);
      lu_factor_f64(s, F, np, nc, h->luw);
    }
    int flag = 0;
    FEAST_HIP(hipMemcpyAsync(&flag, h->luw.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    FEAST_HIP(hipStreamSynchronize(s));
    if (flag) st = FEAST_ZERO_PIVOT;
    zd* iL = h->b_invL.get<zd>((size_t)nc * np * nbt);
    zd* iU = h->b_invU.get<zd>((size_t)nc * np * nbt);
    zd* tmp = h->b_tri_tmp.get<zd>((size_t)np * nbt);
    {
      ScopedProf sp(h->prof, K_LU);
      tri_inverse_blocks_f64(s, F, np, nc, nbt, iL, iU, tmp);
    }
  } else {
    // FEAST_BF16X3_IR: the FP32 factorization's matrix-core products run as bf16x3.
    SplitBf16Scope split(prec == FEAST_BF16X3_IR);
    zf* F = h->b_fac.get<zf>((size_t)nc * np * np);
    shift_matrices_f32(s, A, lda, dt == FEAST_R64, n, np, zdev, nc, F, h->luw.flag, B, ldb);
    if (!shifted_finite()) return FEAST_NONFINITE;
    {
      ScopedProf sp(h->prof, K_LU);
      lu_factor_f32(s, F, np, nc, h->luw);
    }
    int flag = 0;
    FEAST_HIP(hipMemcpyAsync(&flag, h->luw.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    FEAST_HIP(hipStreamSynchronize(s));
    if (flag) st = FEAST_ZERO_PIVOT;
    zf* iL = h->b_invL.get<zf>((size_t)nc * np * nbt);
    zf* iU = h->b_invU.get<zf>((size_t)nc * np * nbt);
    zf* tmp = h->b_tri_tmp.get<zf>((size_t)np * nbt);
    {
      ScopedProf sp(h->prof, K_LU);
      tri_inverse_blocks_f32(s, F, np, nc, nbt, iL, iU, tmp);
    }
  }
  hipEvent_t e1 = h->timer.mark(s);
  h->timer.add(e0, e1, P_FACTOR);
  if (st) return st;
  h->f_valid = true;
  h->f_A = A;
  h->f_B = B;
  h->f_ldb = ldb;
  h->f_n = n;
  h->f_lda = lda;
  h->f_dt = dt;
  h->f_nc = nc;
  h->f_prec = prec;
  h->f_emin = emin;
  h->f_emax = emax;
  h->f_np = np;
  h->f_nbt = nbt;
  return 0;
}

// Complex n x n copy of a real A (FEAST_R64), or A itself.
const zd* complex_A(feast_ctx* h, int dt, int n, const void* A, int lda, long* ld_out) {
  if (dt == FEAST_C128) {
    *ld_out = lda;
    return (const zd*)A;
  }
  if (!(h->ac_valid && h->ac_A == A && h->ac_n == n && h->ac_lda == lda)) {
    zd* Ac = h->b_Ac.get<zd>((size_t)n * n);
    real_to_complex(h->stream, (const double*)A, lda, Ac, n, n, n);
    h->ac_valid = true;
    h->ac_A = A;
    h->ac_n = n;
    h->ac_lda = lda;
  }
  *ld_out = n;
  return (const zd*)h->b_Ac.p;
}

// Complex n x n copy of a real B (FEAST_R64), or B itself.
const zd* complex_B(feast_ctx* h, int dt, int n, const void* B, int ldb, long* ld_out) {
  if (dt == FEAST_C128) {
    *ld_out = ldb;
    return (const zd*)B;
  }
  if (!(h->bc_valid && h->bc_B == B && h->bc_n == n && h->bc_ldb == ldb)) {
    zd* Bc = h->b_Bc.get<zd>((size_t)n * n);
    real_to_complex(h->stream, (const double*)B, ldb, Bc, n, n, n);
    h->bc_valid = true;
    h->bc_B = B;
    h->bc_n = n;
    h->bc_ldb = ldb;
  }
  *ld_out = n;
  return (const zd*)h->b_Bc.p;
}

// The pencil's B for Rayleigh-Ritz and the filter's right-hand side (nullptr: B = I).
struct PencilB {
  const zd* B = nullptr;
  long ld = 0;
};

// Ritz information of the block handed to the filter (FEAST loop, iteration >= 2): X are Ritz
// vectors with values lam (device) and FP64 residual R = A X - X diag(lam) (n x m0, ld n).
struct RitzInfo {
  const zd* R;
  const double* lam;
};

// Q (n x m0 complex, ldq) = rho(A) X with X n x m0 complex (ldx).  Factors must be ready.
// Mixed modes: with ritz, the Ritz-seeded correction; without, low-precision solves plus
// `refine` classic refinement steps whose residuals X - (z I - A) Y are FP64 (A: complex
// n x n, lda).  adaptive: `refine` is a cap, and refinement stops once the largest residual
// entry no longer falls below 0.9 of the previous one (it has reached its FP64 floor).
int filter_core(feast_ctx* h, int dt, int n, int m0, const zd* X, long ldx, zd* Q, long ldq,
                const zd* A = nullptr, long lda = 0, const RitzInfo* ritz = nullptr,
                int refine = 0, bool adaptive = false, bool count = true) {
  hipStream_t s = h->stream;
  if (count) h->last_filters++;  // false: more columns of an application already counted
  h->last_filter_cols += m0;
  const int np = h->f_np, nc = h->f_nc, nbt = h->f_nbt;
  const int sides = (dt == FEAST_C128) ? 2 : 1;
  const size_t blk = (size_t)nc * sides * np * m0;
  const int* perm = h->luw.perm;
  const int* pinv = h->luw.pinv;
  const zd* zdev = (const zd*)h->b_z.p;
  const zd* odev = (const zd*)h->b_omega.p;
  if (h->f_prec == FEAST_FP64) {
    zd* B = h->b_B.get<zd>(blk);
    zd* Z = h->b_Z.get<zd>(blk);
    hipEvent_t e0 = h->timer.mark(s);
    gather_rhs(s, X, ldx, n, np, m0, nc, sides, perm, B);
    {
      ScopedProf sp(h->prof, K_SOLVE);
      solve_sweeps_f64(s, (const zd*)h->b_fac.p, (const zd*)h->b_invL.p, (const zd*)h->b_invU.p,
                       np, nc, nbt, sides, m0, B, Z);
    }
    hipEvent_t e1 = h->timer.mark(s);
    accumulate(s, B, n, np, m0, nc, sides, odev, pinv, Q, ldq);
    hipEvent_t e2 = h->timer.mark(s);
    h->timer.add(e0, e1, P_SOLVE);
    h->timer.add(e1, e2, P_ACC);
    return 0;
  }
  // FP32 factors (and, for FEAST_BF16X3_IR, bf16x3 products in the sweeps)
  SplitBf16Scope split(h->f_prec == FEAST_BF16X3_IR);
  zf* B32 = h->b_B.get<zf>(blk);
  zf* Z32 = h->b_Z.get<zf>(blk);
  const zf* F = (const zf*)h->b_fac.p;
  const zf* iL = (const zf*)h->b_invL.p;
  const zf* iU = (const zf*)h->b_invU.p;
  auto sweep32 = [&]() {
    hipEvent_t a = h->timer.mark(s);
    {
      ScopedProf sp(h->prof, K_SOLVE);
      solve_sweeps_f32(s, F, iL, iU, np, nc, nbt, sides, m0, B32, Z32);
    }
    hipEvent_t b = h->timer.mark(s);
    h->timer.add(a, b, P_SOLVE);
  };
  if (ritz) {
    hipEvent_t e0 = h->timer.mark(s);
    seeded_rhs(s, ritz->R, n, ritz->lam, zdev, perm, n, np, m0, nc, sides, B32);
    double* rho = h->b_rho.get<double>(m0);
    filter_values(s, ritz->lam, zdev, odev, nc, m0, rho);
    hipEvent_t e1 = h->timer.mark(s);
    h->timer.add(e0, e1, P_REFINE);
    sweep32();
    hipEvent_t e2 = h->timer.mark(s);
    accumulate_mixed(s, X, ldx, rho, B32, n, np, m0, nc, sides, odev, pinv, Q, ldq);
    hipEvent_t e3 = h->timer.mark(s);
    h->timer.add(e2, e3, P_ACC);
    return 0;
  }
  gather_rhs_f32(s, X, ldx, n, np, m0, nc, sides, perm, B32);
  sweep32();
  if (refine <= 0) {
    hipEvent_t e2 = h->timer.mark(s);
    accumulate_mixed(s, nullptr, 0, nullptr, B32, n, np, m0, nc, sides, odev, pinv, Q, ldq);
    hipEvent_t e3 = h->timer.mark(s);
    h->timer.add(e2, e3, P_ACC);
    return 0;
  }
  zd* Y = h->b_Y64.get<zd>(blk);
  zd* AY = h->b_AY.get<zd>(blk);
  unpermute_to64(s, B32, pinv, n, np, m0, nc, sides, 0, Y);
  unsigned long long* rmax = adaptive ? h->b_rmax.get<unsigned long long>(1) : nullptr;
  double prev = INFINITY;
  for (int it = 0; it < refine; ++it) {
    hipEvent_t e0 = h->timer.mark(s);
    {
      ScopedProf sp(h->prof, K_REFINE);
      zgemm(s, OP_N, OP_N, n, nc * sides * m0, n, zmake(1, 0), A, lda, Y, np, zmake(0, 0), AY, np);
    }
    refine_rhs(s, X, ldx, Y, AY, zdev, perm, n, np, m0, nc, sides, B32, rmax);
    hipEvent_t e1 = h->timer.mark(s);
    h->timer.add(e0, e1, P_REFINE);
    if (adaptive) {
      unsigned long long bits = 0;
      FEAST_HIP(hipMemcpyAsync(&bits, rmax, sizeof(bits), hipMemcpyDeviceToHost, s));
      FEAST_HIP(hipStreamSynchronize(s));
      double r;
      std::memcpy(&r, &bits, sizeof(r));
      if (!(r < 0.9 * prev)) break;  // stagnated at the FP64 floor (or not finite)
      prev = r;
    }
    sweep32();
    unpermute_to64(s, B32, pinv, n, np, m0, nc, sides, 1, Y);
  }
  hipEvent_t e2 = h->timer.mark(s);
  accumulate_plain(s, Y, n, np, m0, nc, sides, odev, Q, ldq);
  hipEvent_t e3 = h->timer.mark(s);
  h->timer.add(e2, e3, P_ACC);
  return 0;
}

// C = A B for a tall product (n x n times n x k, FP64 complex): K is cut into chunks whose
// partial products are summed when that spreads the output tiles more evenly over the device.
void tall_product(feast_ctx* h, int M, int N, int K, const zd* A, long lda, const zd* B,
                  long ldb, zd* C, long ldc) {
  const int nk = zgemm_kchunks(M, N, K);
  zd* part = nk > 1 ? h->b_kpart.get<zd>((size_t)nk * M * N) : nullptr;
  zgemm_nn_split(h->stream, M, N, K, A, lda, B, ldb, C, ldc, nk, part);
}

// Q <- Q R^{-1} with G = Q^H Q = R^H R; Q1 (nq x m0 zero-padded rows) -> Q2.
// Returns 0, 1 on Cholesky breakdown.
// G = Q1^H Q1, or Q1^H (B Q1) for a pencil (split-K products, Hermitian reduction).
void gram_matrix(feast_ctx* h, int n, int m0, const zd* Q1, const PencilB& pb, zd* G) {
  hipStream_t s = h->stream;
  const int nsplit = std::max(1, std::min(32, n / 256));
  const int kc = (n + nsplit - 1) / nsplit;
  zd* part = h->b_part.get<zd>((size_t)nsplit * m0 * m0);
  const zd* R = Q1;
  if (pb.B) {
    zd* BQ = h->b_BQ.get<zd>((size_t)n * m0);
    tall_product(h, n, m0, n, pb.B, pb.ld, Q1, n, BQ, n);
    R = BQ;
  }
  Batch b;
  b.n1 = nsplit;
  b.splitk = kc;
  b.sC1 = (long)m0 * m0;
  zgemm(s, OP_C, OP_N, m0, m0, n, zmake(1, 0), Q1, n, R, n, zmake(0, 0), part, m0, b);
  reduce_partials_hermitian(s, part, nsplit, m0, G, m0);
}

int cholqr_pass(feast_ctx* h, int n, int m0, const zd* Q1, zd* Q2, double shift_rel,
                const PencilB& pb) {
  hipStream_t s = h->stream;
  zd* G = h->b_G.get<zd>((size_t)m0 * m0);
  int* flag = h->b_flag.get<int>(64);
  gram_matrix(h, n, m0, Q1, pb, G);
  if (shift_rel > 0) {
    // sigma = shift_rel * trace(G) (trace bounds ||G||_2)
    double* dg = h->b_diag.get<double>(m0);
    diag_real(s, G, m0, m0, dg);
    std::vector<double> hd(m0);
    FEAST_HIP(hipMemcpyAsync(hd.data(), dg, sizeof(double) * m0, hipMemcpyDeviceToHost, s));
    FEAST_HIP(hipStreamSynchronize(s));
    double tr = 0;
    for (double v : hd) tr += v;
    add_diag(s, G, m0, m0, shift_rel * tr);
  }
  fill_zero(s, flag, sizeof(int));
  cholesky_upper(s, G, m0, m0, flag, nullptr);
  int hflag = 0;
  FEAST_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  FEAST_HIP(hipStreamSynchronize(s));
  if (hflag) return 1;
  zd* Rinv = h->b_Rinv.get<zd>((size_t)m0 * m0);
  zd* tmp = h->b_rrtmp.get<zd>((size_t)m0 * 64);
  fill_zero(s, Rinv, sizeof(zd) * (size_t)m0 * m0);
  upper_inverse(s, G, m0, m0, Rinv, m0, tmp);
  zgemm(s, OP_N, OP_N, n, m0, m0, zmake(1, 0), Q1, n, Rinv, m0, zmake(0, 0), Q2, n);
  return 0;
}

// Rayleigh-Ritz on Qin (n x m0 complex, ldq); Ritz vectors written back to Qin.
int rr_core(feast_ctx* h, const zd* A, long lda, int n, zd* Qin, long ldq, int m0, double emin,
            double emax, double anorm, double* lam_h, double* res_h, int* m_out,
            zd* Reig = nullptr, bool quant = false, const PencilB& pb = PencilB()) {
  hipStream_t s = h->stream;
  ScopedProf sp(h->prof, K_RR);
  // The Rayleigh-Ritz products take the three-product FP64 form: measured on config 2, the
  // residual floor stays at 5.5e-13 (the factorization and the sweeps, whose errors set that
  // floor, keep four products: with three there it rose to 3e-11).
  Z3mScope z3(true);
  hipEvent_t e0 = h->timer.mark(s);
  zd* Q1 = h->b_Q1.get<zd>((size_t)n * m0);
  zd* Q2 = h->b_Q2.get<zd>((size_t)n * m0);
  copy_matrix(s, Qin, ldq, Q1, n, n, m0);
  // zero columns -> rank deficient (B' singular)
  {
    const int nsplit = std::max(1, std::min(32, n / 256));
    (void)nsplit;
  }
  // Cholesky-QR twice; shifted Cholesky-QR3 when the first Cholesky breaks down.
  {
    // column norms from the first Gram matrix decide exact rank deficiency
    zd* G = h->b_G.get<zd>((size_t)m0 * m0);
    gram_matrix(h, n, m0, Q1, pb, G);
    double* dg = h->b_diag.get<double>(m0);
    diag_real(s, G, m0, m0, dg);
    std::vector<double> hd(m0);
    FEAST_HIP(hipMemcpyAsync(hd.data(), dg, sizeof(double) * m0, hipMemcpyDeviceToHost, s));
    FEAST_HIP(hipStreamSynchronize(s));
    double mx = 0, mn = INFINITY;
    for (double v : hd) {
      if (!std::isfinite(v)) return FEAST_NONFINITE;
      mx = std::max(mx, v);
      mn = std::min(mn, v);
    }
    if (!(mx > 0) || !(mn > 1e-26 * mx)) return FEAST_B_NOT_SPD;
  }
  if (cholqr_pass(h, n, m0, Q1, Q2, 0.0, pb) == 0) {
    if (cholqr_pass(h, n, m0, Q2, Q1, 0.0, pb) != 0) return FEAST_B_NOT_SPD;
  } else {
    const double u = 1.1102230246251565e-16;
    const double shift = 11.0 * ((double)m0 * n + (double)m0 * (m0 + 1)) * u;
    if (cholqr_pass(h, n, m0, Q1, Q2, shift, pb) != 0) return FEAST_B_NOT_SPD;
    if (cholqr_pass(h, n, m0, Q2, Q1, 0.0, pb) != 0) return FEAST_B_NOT_SPD;
    if (cholqr_pass(h, n, m0, Q1, Q2, 0.0, pb) != 0) return FEAST_B_NOT_SPD;
    std::swap(Q1, Q2);
  }
  // Q1 orthonormal (B-orthonormal for a pencil).  A' = Q^H (A Q).
  zd* AQ = h->b_AQ.get<zd>((size_t)n * m0);
  tall_product(h, n, m0, n, A, lda, Q1, n, AQ, n);
  const int nsplit = std::max(1, std::min(32, n / 256));
  const int kc = (n + nsplit - 1) / nsplit;
  zd* part = h->b_part.get<zd>((size_t)nsplit * m0 * m0);
  zd* H = h->b_H.get<zd>((size_t)m0 * m0);
  {
    Batch b;
    b.n1 = nsplit;
    b.splitk = kc;
    b.sC1 = (long)m0 * m0;
    zgemm(s, OP_C, OP_N, m0, m0, n, zmake(1, 0), Q1, n, AQ, n, zmake(0, 0), part, m0, b);
    reduce_partials_hermitian(s, part, nsplit, m0, H, m0);
  }
  const int mp = quant ? jacobi_order_quantized(m0) : jacobi_order(m0);
  double* d = h->b_d.get<double>(mp);
  zd* V = h->b_V.get<zd>((size_t)mp * mp);
  zd* jw = h->b_jac.get<zd>(jacobi_work(mp));
  int* dflag = h->b_flag.get<int>(64);
  hipEvent_t ej = h->prof.on ? h->prof.pool.take() : nullptr;
  if (ej) FEAST_HIP(hipEventRecord(ej, s));
  int sweeps = jacobi_eigh(s, H, m0, d, V, jw, dflag, kJacobiMaxSweeps, &h->jgraphs[mp], mp);
  if (ej) h->prof.eig(s, ej, sweeps);
  if (sweeps < 0) return FEAST_EIG_FAILED;
  double* lam = h->b_lam.get<double>(mp);
  zd* W = h->b_W.get<zd>((size_t)m0 * m0);
  int* rank = h->b_rank.get<int>(mp);
  sort_eigen(s, d, V, m0, mp, lam, W, rank);
  zd* AX = h->b_AX.get<zd>((size_t)n * m0);
  zgemm(s, OP_N, OP_N, n, m0, m0, zmake(1, 0), Q1, n, W, m0, zmake(0, 0), Q2, n);   // X
  zgemm(s, OP_N, OP_N, n, m0, m0, zmake(1, 0), AQ, n, W, m0, zmake(0, 0), AX, n);   // A X
  const zd* BX = Q2;  // B X (X itself when B = I)
  if (pb.B) {
    zd* bx = h->b_BX.get<zd>((size_t)n * m0);
    tall_product(h, n, m0, n, pb.B, pb.ld, Q2, n, bx, n);
    BX = bx;
  }
  double* res = h->b_res.get<double>(m0);
  residual_norms(s, AX, n, BX, n, lam, n, m0, anorm, res);
  if (Reig) ritz_residual(s, AX, n, BX, n, lam, n, m0, Reig);
  copy_matrix(s, Q2, n, Qin, ldq, n, m0);
  FEAST_HIP(hipMemcpyAsync(lam_h, lam, sizeof(double) * m0, hipMemcpyDeviceToHost, s));
  FEAST_HIP(hipMemcpyAsync(res_h, res, sizeof(double) * m0, hipMemcpyDeviceToHost, s));
  hipEvent_t e1 = h->timer.mark(s);
  h->timer.add(e0, e1, P_RR);
  FEAST_HIP(hipStreamSynchronize(s));
  int cnt = 0;
  for (int k = 0; k < m0; ++k) {
    if (!std::isfinite(lam_h[k]) || !std::isfinite(res_h[k])) return FEAST_NONFINITE;
    if (lam_h[k] > emin && lam_h[k] < emax) cnt++;
  }
  *m_out = cnt;
  return 0;
}

void finish_timing(feast_ctx* h) {
  h->timer.flush();
  h->prof.flush();
}


// Set-up shared by the FEAST loop and its expanded-subspace variants: the complex operand
// for Rayleigh-Ritz, ||A||_2 (given or estimated), the factors of the n_c shifted matrices
// and the start block Xw (n x m0, from X0 or seeded Gaussian).  Returns 0 or a status.
int solve_setup(feast_ctx* h, feast_dtype dt, int n, const void* A, int lda, double emin,
                double emax, const feast_opts* opt, const void* X0, int ldx, const zd** Ac_out,
                long* ldac, double* anorm_out, zd* Xw, const void* B = nullptr, int ldb = 0) {
  hipStream_t s = h->stream;
  const int m0 = opt->m0;
  const zd* Ac = complex_A(h, dt, n, A, lda, ldac);
  *Ac_out = Ac;
  double anorm = opt->anorm;
  if (!(anorm > 0)) {
    zd* pw = h->b_pow.get<zd>(2 * (size_t)n);
    double* dn = h->b_diag.get<double>(64);
    anorm = norm2_estimate(s, Ac, *ldac, n, 30, pw, dn);
    if (!(anorm > 0)) anorm = 1.0;
  }
  *anorm_out = anorm;
  int st = ensure_factors(h, dt, n, A, lda, emin, emax, opt->n_c, opt->prec, B, ldb);
  if (st) return st;
  if (X0) {
    if (dt == FEAST_R64) real_to_complex(s, (const double*)X0, ldx, Xw, n, n, m0);
    else copy_matrix(s, (const zd*)X0, ldx, Xw, n, n, m0);
  } else {
    if (dt == FEAST_R64) {
      double* tmp = (double*)h->b_Xc.get<zd>((size_t)n * m0);
      gaussian_fill(s, tmp, n, n, m0, 1, opt->seed);
      real_to_complex(s, tmp, n, Xw, n, n, m0);
    } else {
      gaussian_fill(s, Xw, n, n, m0, 0, opt->seed);
    }
  }
  if (nonfinite_check(s, Xw, n, n, m0, h->b_flag.get<int>(64))) return FEAST_NONFINITE;
  return 0;
}

// ---- Expanded-subspace variants (Sec. 2; Appendix, XFEAST and RFEAST algorithms) ---------

// Orthonormal basis U (n x r, ld n) of span(B) (n x k, ld n) by the Gram route of Sec. 2
// (Method 1), after scaling B's columns to unit length in place (a diagonal scaling keeps the
// span; it keeps RFEAST's short residual columns above the rank threshold):
// B^H B = V S^2 V^H (Jacobi), U = B V S^{-1} over the directions with s^2 > 1e-14 s^2_max.
// Returns r (0: no direction left), -1 if the Gram matrix is not finite or -2 if its
// eigensolve did not converge.
int gram_orthonormal(feast_ctx* h, int n, int k, zd* B, zd* U) {
  hipStream_t s = h->stream;
  // four-product Gram matrix: its eigenvalues decide the rank at 1e-14 of the largest
  Z3mScope z3(false);
  normalize_columns(s, B, n, n, k);
  const int nsplit = std::max(1, std::min(32, n / 256));
  const int kc = (n + nsplit - 1) / nsplit;
  zd* part = h->b_part.get<zd>((size_t)nsplit * k * k);
  zd* G = h->b_G.get<zd>((size_t)k * k);
  Batch b;
  b.n1 = nsplit;
  b.splitk = kc;
  b.sC1 = (long)k * k;
  zgemm(s, OP_C, OP_N, k, k, n, zmake(1, 0), B, n, B, n, zmake(0, 0), part, k, b);
  reduce_partials_hermitian(s, part, nsplit, k, G, k);
  const int mp = jacobi_order_quantized(k);
  double* d = h->b_d.get<double>(mp);
  zd* V = h->b_V.get<zd>((size_t)mp * mp);
  zd* jw = h->b_jac.get<zd>(jacobi_work(mp));
  int* dflag = h->b_flag.get<int>(64);
  hipEvent_t ej = h->prof.on ? h->prof.pool.take() : nullptr;
  if (ej) FEAST_HIP(hipEventRecord(ej, s));
  int sweeps = jacobi_eigh(s, G, k, d, V, jw, dflag, kJacobiMaxSweeps, &h->jgraphs[mp], mp);
  if (ej) h->prof.eig(s, ej, sweeps);
  if (sweeps < 0) return -2;
  std::vector<double> hd(k);
  FEAST_HIP(hipMemcpyAsync(hd.data(), d, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  FEAST_HIP(hipStreamSynchronize(s));
  double mx = 0;
  for (double v : hd) {
    if (!std::isfinite(v)) return -1;
    mx = std::max(mx, v);
  }
  h->keep_h.clear();
  for (int j = 0; j < k; ++j)
    if (hd[j] > 1e-14 * mx) h->keep_h.push_back(j);
  const int r = (int)h->keep_h.size();
  if (r == 0) return 0;
  int* dkeep = h->b_keep.get<int>(r);
  FEAST_HIP(hipMemcpyAsync(dkeep, h->keep_h.data(), sizeof(int) * r, hipMemcpyHostToDevice, s));
  zd* T = h->b_T.get<zd>((size_t)k * r);
  gram_basis(s, d, V, mp, dkeep, k, r, T);
  zgemm(s, OP_N, OP_N, n, r, k, zmake(1, 0), B, n, T, k, zmake(0, 0), U, n);
  FEAST_HIP(hipStreamSynchronize(s));  // keep_h is reused by the next call
  return r;
}

// mu_k (host, k < cnt) for Ritz pairs whose filter value was not measured because the last
// iterate met step 3 as the paper states it: the scalar filter rho(lambda_k) of the
// quadrature, which x_k^H rho(A) x_k equals up to the square of the (converged) residual.
void scalar_filter_mu(feast_ctx* h, const double* lam_dev, int cnt) {
  hipStream_t s = h->stream;
  double* rho = h->b_rho.get<double>(std::max(cnt, 1));
  filter_values(s, lam_dev, (const zd*)h->b_z.p, (const zd*)h->b_omega.p, h->f_nc, cnt, rho);
  h->mu.assign(cnt, 0.0);
  FEAST_HIP(hipMemcpyAsync(h->mu.data(), rho, sizeof(double) * cnt, hipMemcpyDeviceToHost, s));
  FEAST_HIP(hipStreamSynchronize(s));
}

// Step 3 as the paper states it: every Ritz pair inside I counts, and the iteration stops
// when their largest residual is at most tol (and fewer than m0 lie inside I after the first
// iteration).  Pairs inside I with a residual at most tol are eigenpairs inside I (their
// eigenvalue lies within res * anorm of lambda_k), so when this test passes the filter-value
// test cannot remove any of them and is not needed.
bool plain_step3_converged(const double* lam, const double* res, int cnt, double emin,
                           double emax, double tol, int m0, int it) {
  int in = 0;
  double r = 0;
  for (int k = 0; k < cnt; ++k)
    if (lam[k] > emin && lam[k] < emax) {
      in++;
      r = std::max(r, res[k]);
    }
  return in > 0 && r <= tol && !(in >= m0 && it >= 2);
}

// Status of a gram_orthonormal result r (0 when r is a usable basis width).
int gram_status(int r) {
  return r == -2 ? FEAST_EIG_FAILED : r < 0 ? FEAST_NONFINITE : r == 0 ? FEAST_B_NOT_SPD : 0;
}

// Selection of Sec. 2 (Method 1; Method 2 uses the same): every pair inside I, then the pairs
// outside by increasing residual, m0 in all; with more than m0 inside (left open by the
// paper), the m0 inside pairs with the lowest residuals.  Ties keep the lower index.
// sel = chosen indices in ascending lambda order; returns min(m0, r).
int select_pairs(int r, const double* lam, const double* res, double emin, double emax, int m0,
                 std::vector<int>& sel) {
  std::vector<int> in, out;
  for (int k = 0; k < r; ++k) (lam[k] > emin && lam[k] < emax ? in : out).push_back(k);
  auto by_res = [&](int a, int b) { return res[a] < res[b]; };
  std::stable_sort(in.begin(), in.end(), by_res);
  std::stable_sort(out.begin(), out.end(), by_res);
  sel.assign(in.begin(), in.end());
  sel.insert(sel.end(), out.begin(), out.end());
  const int take = std::min(m0, r);
  sel.resize(take);
  std::stable_sort(sel.begin(), sel.end(), [&](int a, int b) { return lam[a] < lam[b]; });
  return take;
}

// XFEAST (opt->method 1): X' = [X_0, rho X_0, ..., rho^{s-1} X_0]; each iteration
// orthogonalizes X', runs Rayleigh-Ritz on it, keeps m0 pairs, tests them, filters the kept
// block and puts it in place of the oldest block.  RFEAST (method 2): X' = rho(A) X_i, then s
// Rayleigh-Ritz steps, each after the first on X' grown by the residual block R = A X - X Lambda
// of the pairs kept by the previous one; m_e, the number of pairs inside I at the first step,
// caps the pairs that count in the test (the lowest residuals among those inside I).
// Xs holds X_0 on entry (n x m0, complex).  Outputs as feast_solve.
int xr_solve(feast_ctx* h, feast_dtype dt, int n, const zd* Ac, long ldac, double anorm,
             double emin, double emax, const feast_opts* opt, zd* Xs, void* X, int ldx,
             double* lambda, double* res, int* m, int* iters, double* trace) {
  hipStream_t s = h->stream;
  const int m0 = opt->m0, sx = opt->expand, variant = opt->method;
  const int K = sx * m0;
  const bool mixed = opt->prec != FEAST_FP64;
  const bool spur = opt->spurious != 0 || mixed;
  // Buffers sized once for the widest basis, so device pointers (and the recorded Jacobi
  // sweeps that capture them) stay fixed while the basis width changes.
  zd* W = h->b_win.get<zd>((size_t)n * K);
  zd* U = h->b_U.get<zd>((size_t)n * K);
  zd* Reig = h->b_Reig.get<zd>((size_t)n * K);
  {
    const int mq = jacobi_order_quantized(K);
    h->b_d.get<double>(mq);
    h->b_V.get<zd>((size_t)mq * mq);
    h->b_jac.get<zd>(jacobi_work(mq));
    h->b_flag.get<int>(64);
  }
  zd* Rsel = h->b_Rsel.get<zd>((size_t)n * m0);
  double* lsel = h->b_lsel.get<double>(m0);
  int* dsel = h->b_sel.get<int>(m0);
  double* dmu = h->b_mu.get<double>(m0);
  std::vector<double> lam_h(K), res_h(K);
  h->mu.assign(m0, 0.0);
  std::vector<int>& sel = h->sel_h;
  auto upload_sel = [&](int take) {
    FEAST_HIP(hipMemcpyAsync(dsel, sel.data(), sizeof(int) * take, hipMemcpyHostToDevice, s));
  };

  int fs = 0, kcols = 0, slot = 0;
  if (variant == FEAST_METHOD_XFEAST) {  // step 0
    copy_matrix(s, Xs, n, W, n, n, m0);
    for (int b = 1; b < sx && !fs; ++b)
      fs = filter_core(h, dt, n, m0, W + (size_t)(b - 1) * n * m0, n, W + (size_t)b * n * m0, n,
                       Ac, ldac, nullptr, opt->refine_max);
    kcols = K;
  } else {  // step 1 of the first iteration
    fs = filter_core(h, dt, n, m0, Xs, n, W, n, Ac, ldac, nullptr, opt->refine_max);
  }
  int st = fs ? fs : FEAST_NOT_CONVERGED;
  int it = 0, prev_m = -1, mm = 0;
  for (it = 1; fs == 0 && it <= opt->max_iter; ++it) {
    int take = 0, me = -1, rs = 0, mcount = 0;
    if (variant == FEAST_METHOD_XFEAST) {
      int r = gram_orthonormal(h, n, kcols, W, U);  // step 1
      rs = gram_status(r);
      if (!rs)
        rs = rr_core(h, Ac, ldac, n, U, n, r, emin, emax, anorm, lam_h.data(), res_h.data(),
                     &mcount, mixed ? Reig : nullptr, true);  // step 2.i
      if (!rs) take = select_pairs(r, lam_h.data(), res_h.data(), emin, emax, m0, sel);  // 2.ii
    } else {
      kcols = m0;
      for (int j = 1; j <= sx && !rs; ++j) {  // step 2
        int r = gram_orthonormal(h, n, kcols, W, U);
        rs = gram_status(r);
        if (!rs)
          rs = rr_core(h, Ac, ldac, n, U, n, r, emin, emax, anorm, lam_h.data(), res_h.data(),
                       &mcount, Reig, true);
        if (rs) break;
        take = select_pairs(r, lam_h.data(), res_h.data(), emin, emax, m0, sel);
        if (j == 1) me = mcount;
        if (j < sx) {  // step 2.iii: X' = [X' R]
          upload_sel(take);
          gather_columns(s, Reig, n, dsel, n, take, W + (size_t)kcols * n, n);
          kcols += take;
        }
      }
    }
    if (rs) {
      finish_timing(h);
      st = rs;
      break;
    }
    // X_{i+1}: the kept Ritz vectors (columns past `take` keep the previous block)
    upload_sel(take);
    gather_columns(s, U, n, dsel, n, take, Xs, n);
    for (int a = 0; a < m0; ++a) {
      lambda[a] = a < take ? lam_h[sel[a]] : INFINITY;
      res[a] = a < take ? res_h[sel[a]] : INFINITY;
    }
    const bool seeded = mixed && take == m0;
    const bool plain = spur && plain_step3_converged(lambda, res, take, emin, emax, opt->tol,
                                                     m0, it);
    if (seeded || plain) gather_values(s, (const double*)h->b_lam.p, dsel, take, lsel);
    if (seeded) gather_columns(s, Reig, n, dsel, n, take, Rsel, n);
    RitzInfo ri{Rsel, lsel};
    // rho(A) X_{i+1}: XFEAST's newest block (in place of the oldest), RFEAST's next X'
    zd* dst = variant == FEAST_METHOD_XFEAST ? W + (size_t)slot * n * m0 : W;
    auto filter_next = [&]() {
      return filter_core(h, dt, n, m0, Xs, n, dst, n, Ac, ldac, seeded ? &ri : nullptr,
                         opt->refine_max);
    };
    if (plain) {
      scalar_filter_mu(h, lsel, take);
      h->mu.resize(m0, 0.0);
    } else if (spur) {
      fs = filter_next();
      if (fs) {
        st = fs;
        break;
      }
      coldot_re(s, Xs, n, dst, n, n, take, dmu);
      FEAST_HIP(hipMemcpyAsync(h->mu.data(), dmu, sizeof(double) * take, hipMemcpyDeviceToHost,
                               s));
      FEAST_HIP(hipStreamSynchronize(s));
    }
    finish_timing(h);
    // step 3
    std::vector<int> cand;
    for (int a = 0; a < take; ++a) {
      if (!(lambda[a] > emin && lambda[a] < emax)) continue;
      if (spur && !plain && !(h->mu[a] > 0.5)) continue;
      cand.push_back(a);
    }
    if (variant == FEAST_METHOD_RFEAST && !spur && me >= 0 && (int)cand.size() > me) {
      std::stable_sort(cand.begin(), cand.end(), [&](int a, int b) { return res[a] < res[b]; });
      cand.resize(me);
    }
    double r = 0;
    for (int a : cand) r = std::max(r, res[a]);
    mm = (int)cand.size();
    h->counted.assign(m0, 0);
    for (int a : cand) h->counted[a] = 1;
    h->last_max_res = r;
    if (trace) trace[it - 1] = r;
    if (mm == 0) {
      if (prev_m == 0) {
        st = FEAST_NO_EIGENVALUES;
        break;
      }
    } else if (mm >= m0 && it >= 2) {
      st = FEAST_M0_TOO_SMALL;
      break;
    } else if (r <= opt->tol) {
      st = FEAST_OK;
      break;
    }
    prev_m = mm;
    if (!spur && it < opt->max_iter) {
      fs = filter_next();
      if (fs) {
        st = fs;
        break;
      }
    }
    if (variant == FEAST_METHOD_XFEAST) slot = (slot + 1) % sx;  // step 4.ii
  }
  if (it > opt->max_iter) it = opt->max_iter;
  *iters = it;
  *m = mm;
  h->last_iters = it;
  h->last_count = mm;
  if (dt == FEAST_R64) complex_to_real(s, Xs, n, (double*)X, ldx, n, m0);
  else copy_matrix(s, Xs, n, (zd*)X, ldx, n, m0);
  h->timer.end_total(s);
  FEAST_HIP(hipStreamSynchronize(s));
  finish_timing(h);
  return st;
}
}  // namespace

// =======================================================================================
extern "C" {

int feast_create(feast_handle* out, void* hip_stream) {
  if (!out) return -1;
  feast_ctx* h = new feast_ctx();
  h->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    *out = nullptr;
    return FEAST_ERR_HIP;
  }
  if (!h->stream) {  // own blocking stream: ordered with the legacy default stream
    if (hipStreamCreate(&h->stream) != hipSuccess) {
      delete h;
      *out = nullptr;
      return FEAST_ERR_HIP;
    }
    h->own_stream = true;
  }
  *out = h;
  return 0;
}

int feast_destroy(feast_handle h) {
  if (!h) return 0;
  (void)hipStreamSynchronize(h->stream);
  for (size_t w = 0; w < h->workers.size(); ++w) {
    feast_destroy(h->workers[w]);
    (void)hipStreamDestroy(h->worker_streams[w]);
  }
  h->workers.clear();
  Buf* bufs[] = {&h->b_fac, &h->b_invL, &h->b_invU, &h->b_tri_tmp, &h->b_luw, &h->b_z,
                 &h->b_omega, &h->b_Ac, &h->b_B, &h->b_Z, &h->b_Xc, &h->b_Qc, &h->b_X0c,
                 &h->b_Q1, &h->b_Q2, &h->b_AQ, &h->b_AX, &h->b_G, &h->b_part, &h->b_Rinv,
                 &h->b_rrtmp, &h->b_H, &h->b_jac, &h->b_V, &h->b_d, &h->b_lam, &h->b_res,
                 &h->b_rank, &h->b_W, &h->b_flag, &h->b_diag, &h->b_pow, &h->b_mu,
                 &h->b_Reig, &h->b_Y64, &h->b_AY, &h->b_rho, &h->b_rmax, &h->b_kpart};
  for (Buf* b : bufs) b->release();
  if (h->own_stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return 0;
}

const char* feast_status_string(int st) {
  switch (st) {
    case FEAST_OK: return "converged";
    case FEAST_NOT_CONVERGED: return "maximum number of iterations reached";
    case FEAST_M0_TOO_SMALL: return "m0 too small: at least m0 Ritz values inside the interval";
    case FEAST_NO_EIGENVALUES: return "no eigenvalue inside the interval";
    case FEAST_B_NOT_SPD: return "filtered block is rank deficient (B' not positive definite)";
    case FEAST_NONFINITE: return "non-finite value in the input or an intermediate";
    case FEAST_ZERO_PIVOT: return "exact zero pivot in a shifted factorization";
    case FEAST_EIG_FAILED: return "the dense reduced eigensolver did not converge";
    case FEAST_ERR_ALLOC: return "device allocation failed";
    case FEAST_ERR_HIP: return "HIP runtime error";
    case FEAST_ERR_UNSUPPORTED: return "unsupported option";
    case FEAST_ERR_SCRATCH:
      return "the problem needs more than the static scratch array of the allocation-free "
             "entry point";
    default: return st < 0 ? "invalid argument" : "unknown status";
  }
}

const char* feast_last_error(feast_handle h) { return h ? h->last_error.c_str() : ""; }

void feast_invalidate(feast_handle h) {
  if (!h) return;
  h->f_valid = false;
  h->ac_valid = false;
  for (feast_ctx* w : h->workers) feast_invalidate(w);
}

int feast_filter_apply(feast_handle h, feast_dtype dt, int n, const void* A, int lda,
                       double emin, double emax, int n_c, feast_precision prec, const void* X,
                       int ldx, int m0, void* Q, int ldq) {
  if (!h) return -1;
  if (dt != FEAST_R64 && dt != FEAST_C128) return -2;
  if (n < 1) return -3;
  if (!A) return -4;
  if (lda < n) return -5;
  if (!std::isfinite(emin)) return -6;
  if (!std::isfinite(emax) || !(emin < emax)) return -7;
  if (n_c < 1 || n_c > 128) return -8;
  if (prec != FEAST_FP64 && prec != FEAST_FP32_IR && prec != FEAST_BF16X3_IR) return -9;
  if (!X) return -10;
  if (ldx < n) return -11;
  if (m0 < 1 || m0 > n) return -12;
  if (!Q || Q == X) return -13;
  if (ldq < n) return -14;
  try {
    hipStream_t s = h->stream;
    h->timer.clear();
    h->timer.begin_total(s);
    int st = ensure_factors(h, dt, n, A, lda, emin, emax, n_c, prec);
    if (st) {
      finish_timing(h);
      return st;
    }
    const zd* Xc;
    long ldxc;
    zd* Qc;
    long ldqc;
    if (dt == FEAST_R64) {
      zd* xb = h->b_Xc.get<zd>((size_t)n * m0);
      real_to_complex(s, (const double*)X, ldx, xb, n, n, m0);
      Xc = xb;
      ldxc = n;
      Qc = h->b_Qc.get<zd>((size_t)n * m0);
      ldqc = n;
    } else {
      Xc = (const zd*)X;
      ldxc = ldx;
      Qc = (zd*)Q;
      ldqc = ldq;
    }
    long ldac = lda;
    const zd* Ac = (prec != FEAST_FP64) ? complex_A(h, dt, n, A, lda, &ldac) : nullptr;
    // Classic refinement until the FP64 residual stops shrinking: each step contracts the
    // error by about kappa(z_j I - A) times the products' relative accuracy (2^-24 FP32,
    // ~2^-16 bf16x3), so bf16x3 may need many more steps.
    st = filter_core(h, dt, n, m0, Xc, ldxc, Qc, ldqc, Ac, ldac, nullptr,
                     prec == FEAST_BF16X3_IR ? 30 : 10, true);
    if (st == 0 && dt == FEAST_R64) complex_to_real(s, Qc, n, (double*)Q, ldq, n, m0);
    h->timer.end_total(s);
    FEAST_HIP(hipStreamSynchronize(s));
    finish_timing(h);
    return st;
  } catch (const HipError& e) {
    return fail_hip(h, e);
  } catch (const std::bad_alloc&) {
    return FEAST_ERR_ALLOC;
  }
}

int feast_rayleigh_ritz(feast_handle h, feast_dtype dt, int n, const void* A, int lda, void* Q,
                        int ldq, int m0, double emin, double emax, double anorm, double* lambda,
                        double* res, int* m) {
  if (!h) return -1;
  if (dt != FEAST_R64 && dt != FEAST_C128) return -2;
  if (n < 1) return -3;
  if (!A) return -4;
  if (lda < n) return -5;
  if (!Q) return -6;
  if (ldq < n) return -7;
  if (m0 < 1 || m0 > n) return -8;
  if (!std::isfinite(emin)) return -9;
  if (!std::isfinite(emax) || !(emin < emax)) return -10;
  if (!(anorm > 0) || !std::isfinite(anorm)) return -11;
  if (!lambda) return -12;
  if (!res) return -13;
  if (!m) return -14;
  try {
    hipStream_t s = h->stream;
    h->timer.clear();
    h->timer.begin_total(s);
    long ldac;
    const zd* Ac = complex_A(h, dt, n, A, lda, &ldac);
    zd* Qc;
    long ldqc;
    if (dt == FEAST_R64) {
      Qc = h->b_Qc.get<zd>((size_t)n * m0);
      ldqc = n;
      real_to_complex(s, (const double*)Q, ldq, Qc, n, n, m0);
    } else {
      Qc = (zd*)Q;
      ldqc = ldq;
    }
    int st = rr_core(h, Ac, ldac, n, Qc, ldqc, m0, emin, emax, anorm, lambda, res, m);
    if (st == 0 && dt == FEAST_R64) complex_to_real(s, Qc, n, (double*)Q, ldq, n, m0);
    h->timer.end_total(s);
    FEAST_HIP(hipStreamSynchronize(s));
    finish_timing(h);
    return st;
  } catch (const HipError& e) {
    return fail_hip(h, e);
  } catch (const std::bad_alloc&) {
    return FEAST_ERR_ALLOC;
  }
}

}  // extern "C"

namespace {
// The FEAST loop of the Appendix on A (B == nullptr) or on the pencil (A, B): the filter is
// applied to B X (rho(B^{-1} A) X = sum_j omega_j (z_j B - A)^{-1} B X + adjoint terms),
// Rayleigh-Ritz B-orthonormalizes, residuals are ||A x - lambda B x||, and the filter value
// of a Ritz vector is mu_k = Re(x_k^H B rho x_k).  Arguments checked by the callers.
int solve_impl(feast_handle h, feast_dtype dt, int n, const void* A, int lda, const void* B,
               int ldb, double emin, double emax, const feast_opts* opt, const void* X0, void* X,
               int ldx, double* lambda, double* res, int* m, int* iters, double* trace) {
  const int m0 = opt->m0;
  h->counted.assign(m0, 0);
  h->last_filters = h->last_iters = h->last_count = 0;
  h->last_filter_cols = 0;
  h->last_max_res = 0;
  try {
    hipStream_t s = h->stream;
    h->timer.clear();
    h->timer.begin_total(s);
    long ldac = 0;
    const zd* Ac = nullptr;
    double anorm = 0;
    zd* Xw = h->b_X0c.get<zd>((size_t)n * m0);
    int st = solve_setup(h, dt, n, A, lda, emin, emax, opt, X0, ldx, &Ac, &ldac, &anorm, Xw,
                         B, ldb);
    if (st) {
      FEAST_HIP(hipStreamSynchronize(s));
      finish_timing(h);
      *iters = 0;
      *m = 0;
      return st;
    }
    if (opt->method != FEAST_METHOD_FEAST)
      return xr_solve(h, dt, n, Ac, ldac, anorm, emin, emax, opt, Xw, X, ldx, lambda, res, m,
                      iters, trace);
    zd* Qf = h->b_Qc.get<zd>((size_t)n * m0);
    PencilB pb;
    if (B) pb.B = complex_B(h, dt, n, B, ldb, &pb.ld);
    zd* BXf = B ? h->b_BXf.get<zd>((size_t)n * m0) : nullptr;
    // the filter's right-hand side for the block Xc: Xc itself, or B Xc for a pencil
    auto rhs = [&](const zd* Xc) -> const zd* {
      if (!B) return Xc;
      tall_product(h, n, m0, n, pb.B, pb.ld, Xc, n, BXf, n);
      return BXf;
    };
    st = FEAST_NOT_CONVERGED;
    int it = 0, prev_m = -1, mm = 0;
    // FP32 factors leave the filtered block's damped directions (|rho| far below the FP32
    // noise floor) as noise, which Rayleigh-Ritz turns into Ritz pairs inside I with large
    // residuals; the filter-value test rejects them, so FP32_IR always applies it.
    const bool spur = opt->spurious != 0 || opt->prec != FEAST_FP64;
    h->mu.assign(m0, 0.0);
    const bool mixed = opt->prec != FEAST_FP64;
    zd* Reig = mixed ? h->b_Reig.get<zd>((size_t)n * m0) : nullptr;
    RitzInfo ri{Reig, nullptr};
    int fs = filter_core(h, dt, n, m0, rhs(Xw), n, Qf, n, Ac, ldac, nullptr,
                         opt->refine_max);  // step 1 of the first iteration
    if (fs) {
      st = fs;
      it = 1;
    }
    for (it = 1; fs == 0 && it <= opt->max_iter; ++it) {
      int rs = rr_core(h, Ac, ldac, n, Qf, n, m0, emin, emax, anorm, lambda, res, &mm,
                       Reig, false, pb);  // step 2
      std::swap(Xw, Qf);  // Ritz vectors become the next block
      ri.lam = (const double*)h->b_lam.p;
      if (rs) {
        finish_timing(h);
        st = rs;
        break;
      }
      const bool plain = spur && plain_step3_converged(lambda, res, m0, emin, emax, opt->tol,
                                                       m0, it);
      bool partial = false;  // this application has filtered columns [plo, phi) only
      int plo = 0, phi = m0;
      const zd* bxp = nullptr;
      if (plain) {
        scalar_filter_mu(h, (const double*)h->b_lam.p, m0);
      } else if (spur) {  // the next step 1 gives mu_k = Re(x_k^H rho(A) x_k)
        const zd* bx = rhs(Xw);
        // Step 3 reads mu_k only for the Ritz pairs inside I (indices [lo, hi): lambda is in
        // ascending order).  When every pair counted at the previous iteration now has a
        // residual at or below tol, this application is likely the last one: filter those
        // columns first, and the others only if step 3 does not stop.  Every column of an
        // application is filtered independently, so the result is the same either way.
        int lo = 0, hi = m0, conv = 0;
        while (lo < m0 && !(lambda[lo] > emin)) ++lo;
        hi = lo;
        while (hi < m0 && lambda[hi] < emax) conv += (res[hi++] <= opt->tol);
        partial = (g_split_filter.load(std::memory_order_relaxed) != 0 ||
                   (prev_m > 0 && conv >= prev_m)) &&
                  hi > lo && hi - lo < m0;
        plo = lo;
        phi = hi;
        bxp = bx;
        const int c0 = partial ? lo : 0, nc0 = partial ? hi - lo : m0;
        RitzInfo rs0{mixed ? Reig + (size_t)c0 * n : nullptr, ri.lam ? ri.lam + c0 : nullptr};
        fs = filter_core(h, dt, n, nc0, bx + (size_t)c0 * n, n, Qf + (size_t)c0 * n, n, Ac, ldac,
                         mixed ? &rs0 : nullptr);
        if (fs) {
          st = fs;
          break;
        }
        // outside [lo, hi) a partial application leaves the scalar filter rho(lambda_k)
        if (partial) scalar_filter_mu(h, (const double*)h->b_lam.p, m0);
        double* dmu = h->b_mu.get<double>(m0);
        coldot_re(s, bx + (size_t)c0 * n, n, Qf + (size_t)c0 * n, n, n, nc0, dmu);
        FEAST_HIP(hipMemcpyAsync(h->mu.data() + c0, dmu, sizeof(double) * nc0,
                                 hipMemcpyDeviceToHost, s));
        FEAST_HIP(hipStreamSynchronize(s));
      }
      finish_timing(h);
      double r = 0;  // step 3
      int cnt = 0;
      h->counted.assign(m0, 0);
      for (int k = 0; k < m0; ++k) {
        if (!(lambda[k] > emin && lambda[k] < emax)) continue;
        if (spur && !plain && !(h->mu[k] > 0.5)) continue;
        h->counted[k] = 1;
        cnt++;
        r = std::max(r, res[k]);
      }
      mm = cnt;
      h->last_max_res = r;
      if (trace) trace[it - 1] = r;
      if (mm == 0) {
        if (prev_m == 0) {
          st = FEAST_NO_EIGENVALUES;
          break;
        }
      } else if (mm >= m0 && it >= 2) {
        st = FEAST_M0_TOO_SMALL;
        break;
      } else if (r <= opt->tol) {
        st = FEAST_OK;
        break;
      }
      prev_m = mm;
      if (partial) {  // step 3 did not stop: the other columns of this application
        for (int part = 0; part < 2 && fs == 0; ++part) {
          const int c0 = part ? phi : 0, ncol = part ? m0 - phi : plo;
          if (ncol <= 0) continue;
          RitzInfo rs1{mixed ? Reig + (size_t)c0 * n : nullptr, ri.lam ? ri.lam + c0 : nullptr};
          fs = filter_core(h, dt, n, ncol, bxp + (size_t)c0 * n, n, Qf + (size_t)c0 * n, n, Ac,
                           ldac, mixed ? &rs1 : nullptr, 0, false, false);
        }
        if (fs) {
          st = fs;
          break;
        }
      }
      if (!spur && it < opt->max_iter) {
        fs = filter_core(h, dt, n, m0, rhs(Xw), n, Qf, n, Ac, ldac,
                         mixed ? &ri : nullptr);  // step 1 of the next iteration
        if (fs) {
          st = fs;
          break;
        }
      }
    }
    if (it > opt->max_iter) it = opt->max_iter;
    *iters = it;
    *m = mm;
    h->last_iters = it;
    h->last_count = mm;
    if (dt == FEAST_R64) complex_to_real(s, Xw, n, (double*)X, ldx, n, m0);
    else copy_matrix(s, Xw, n, (zd*)X, ldx, n, m0);
    h->timer.end_total(s);
    FEAST_HIP(hipStreamSynchronize(s));
    finish_timing(h);
    return st;
  } catch (const HipError& e) {
    return fail_hip(h, e);
  } catch (const std::bad_alloc&) {
    return FEAST_ERR_ALLOC;
  }
}
}  // namespace

extern "C" {

int feast_solve(feast_handle h, feast_dtype dt, int n, const void* A, int lda, double emin,
                double emax, const feast_opts* opt, const void* X0, void* X, int ldx,
                double* lambda, double* res, int* m, int* iters, double* trace) {
  if (!h) return -1;
  if (dt != FEAST_R64 && dt != FEAST_C128) return -2;
  if (n < 1) return -3;
  if (!A) return -4;
  if (lda < n) return -5;
  if (!std::isfinite(emin)) return -6;
  if (!std::isfinite(emax) || !(emin < emax)) return -7;
  if (!opt || opt->n_c < 1 || opt->n_c > 128 || opt->m0 < 1 || opt->m0 > n ||
      opt->max_iter < 1 || !(opt->tol > 0) ||
      (opt->prec != FEAST_FP64 && opt->prec != FEAST_FP32_IR &&
       opt->prec != FEAST_BF16X3_IR) ||
      (opt->prec != FEAST_FP64 && opt->refine_max < 0) ||
      (opt->method != FEAST_METHOD_FEAST && opt->method != FEAST_METHOD_XFEAST &&
       opt->method != FEAST_METHOD_RFEAST) ||
      (opt->method != FEAST_METHOD_FEAST &&
       (opt->expand < 1 || (long)opt->expand * opt->m0 > n)))
    return -8;
  if (!X) return -10;
  if (ldx < n) return -11;
  if (!lambda) return -12;
  if (!res) return -13;
  if (!m) return -14;
  if (!iters) return -15;
  return solve_impl(h, dt, n, A, lda, nullptr, 0, emin, emax, opt, X0, X, ldx, lambda, res, m,
                    iters, trace);
}

int feast_solve_gen(feast_handle h, feast_dtype dt, int n, const void* A, int lda, const void* B,
                    int ldb, double emin, double emax, const feast_opts* opt, const void* X0,
                    void* X, int ldx, double* lambda, double* res, int* m, int* iters,
                    double* trace) {
  if (!h) return -1;
  if (dt != FEAST_R64 && dt != FEAST_C128) return -2;
  if (n < 1) return -3;
  if (!A) return -4;
  if (lda < n) return -5;
  if (!B) return -6;
  if (ldb < n) return -7;
  if (!std::isfinite(emin)) return -8;
  if (!std::isfinite(emax) || !(emin < emax)) return -9;
  if (!opt || opt->n_c < 1 || opt->n_c > 128 || opt->m0 < 1 || opt->m0 > n ||
      opt->max_iter < 1 || !(opt->tol > 0) || opt->prec != FEAST_FP64 ||
      opt->method != FEAST_METHOD_FEAST)
    return -10;
  if (!X) return -12;
  if (ldx < n) return -13;
  if (!lambda) return -14;
  if (!res) return -15;
  if (!m) return -16;
  if (!iters) return -17;
  return solve_impl(h, dt, n, A, lda, B, ldb, emin, emax, opt, X0, X, ldx, lambda, res, m, iters,
                    trace);
}

int feast_filter_apply_gen(feast_handle h, feast_dtype dt, int n, const void* A, int lda,
                           const void* B, int ldb, double emin, double emax, int n_c,
                           feast_precision prec, const void* X, int ldx, int m0, void* Q,
                           int ldq) {
  if (!h) return -1;
  if (dt != FEAST_R64 && dt != FEAST_C128) return -2;
  if (n < 1) return -3;
  if (!A) return -4;
  if (lda < n) return -5;
  if (!B) return -6;
  if (ldb < n) return -7;
  if (!std::isfinite(emin)) return -8;
  if (!std::isfinite(emax) || !(emin < emax)) return -9;
  if (n_c < 1 || n_c > 128) return -10;
  if (prec != FEAST_FP64) return -11;
  if (!X) return -12;
  if (ldx < n) return -13;
  if (m0 < 1 || m0 > n) return -14;
  if (!Q || Q == X) return -15;
  if (ldq < n) return -16;
  try {
    hipStream_t s = h->stream;
    h->timer.clear();
    h->timer.begin_total(s);
    int st = ensure_factors(h, dt, n, A, lda, emin, emax, n_c, prec, B, ldb);
    if (st) {
      finish_timing(h);
      return st;
    }
    const zd* Xc = (const zd*)X;
    long ldxc = ldx;
    if (dt == FEAST_R64) {
      zd* xb = h->b_Xc.get<zd>((size_t)n * m0);
      real_to_complex(s, (const double*)X, ldx, xb, n, n, m0);
      Xc = xb;
      ldxc = n;
    }
    long ldbc = 0;
    const zd* Bc = complex_B(h, dt, n, B, ldb, &ldbc);
    zd* BX = h->b_BXf.get<zd>((size_t)n * m0);
    tall_product(h, n, m0, n, Bc, ldbc, Xc, ldxc, BX, n);
    zd* Qc = (dt == FEAST_R64) ? h->b_Qc.get<zd>((size_t)n * m0) : (zd*)Q;
    long ldqc = (dt == FEAST_R64) ? n : ldq;
    st = filter_core(h, dt, n, m0, BX, n, Qc, ldqc);
    if (st == 0 && dt == FEAST_R64) complex_to_real(s, Qc, n, (double*)Q, ldq, n, m0);
    h->timer.end_total(s);
    FEAST_HIP(hipStreamSynchronize(s));
    finish_timing(h);
    return st;
  } catch (const HipError& e) {
    return fail_hip(h, e);
  } catch (const std::bad_alloc&) {
    return FEAST_ERR_ALLOC;
  }
}

int feast_solve_batched(feast_handle h, feast_dtype dt, int nprob, const feast_problem* probs,
                        const feast_opts* opt, int nstreams) {
  if (!h) return -1;
  if (dt != FEAST_R64 && dt != FEAST_C128) return -2;
  if (nprob < 0) return -3;
  if (nprob > 0 && !probs) return -4;
  if (!opt) return -5;
  if (nstreams < 1 || nstreams > 32) return -6;
  if (nprob == 0) return 0;
  try {
    FEAST_HIP(hipSetDevice(h->device));
    while ((int)h->workers.size() < nstreams) {
      hipStream_t st;
      FEAST_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      feast_handle w = nullptr;
      int rc = feast_create(&w, st);
      if (rc) {
        (void)hipStreamDestroy(st);
        return rc;
      }
      w->prof.on = h->prof.on;
      h->workers.push_back(w);
      h->worker_streams.push_back(st);
    }
    // Inputs written on the caller's stream before this call come first: every worker stream
    // waits for an event recorded on it before its first launch.
    hipEvent_t ready = nullptr;
    FEAST_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    struct EvGuard {
      hipEvent_t e;
      ~EvGuard() { (void)hipEventDestroy(e); }
    } ready_guard{ready};
    FEAST_HIP(hipEventRecord(ready, h->stream));
    for (int wi = 0; wi < nstreams; ++wi)
      FEAST_HIP(hipStreamWaitEvent(h->worker_streams[wi], ready, 0));
    std::vector<int> order(nprob);
    for (int i = 0; i < nprob; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      return (double)probs[a].n * probs[a].n * probs[a].n >
             (double)probs[b].n * probs[b].n * probs[b].n;
    });
    std::atomic<int> next(0);
    const int dev = h->device;
    auto work = [&](int wi) {
      (void)hipSetDevice(dev);
      feast_ctx* wh = h->workers[wi];
      for (int k = next.fetch_add(1); k < nprob; k = next.fetch_add(1)) {
        const feast_problem& p = probs[order[k]];
        feast_opts o = *opt;
        o.m0 = p.m0;
        o.anorm = p.anorm;
        int st = -7;
        if (p.lambda && p.res && p.m && p.iters)
          st = feast_solve(wh, dt, p.n, p.A, p.lda, p.emin, p.emax, &o, p.X0, p.X, p.ldx,
                           p.lambda, p.res, p.m, p.iters, p.trace);
        if (p.mu)
          for (int q = 0; q < p.m0; ++q) p.mu[q] = q < (int)wh->mu.size() ? wh->mu[q] : 0.0;
        if (p.info || p.counted) feast_get_solve_info(wh, p.info, p.counted, p.m0);
        if (p.status) *p.status = st;
      }
    };
    std::vector<std::thread> threads;
    for (int wi = 0; wi < nstreams; ++wi) threads.emplace_back(work, wi);
    for (auto& t : threads) t.join();
    int bad = 0;
    for (int i = 0; i < nprob; ++i)
      if (!probs[i].status || *probs[i].status != FEAST_OK) bad++;
    return bad;
  } catch (const HipError& e) {
    return fail_hip(h, e);
  }
}

int feast_get_solve_info(feast_handle h, feast_solve_info* info, int* counted, int m0) {
  if (!h) return -1;
  if (counted && m0 < 0) return -4;
  if (info) {
    info->iters = h->last_iters;
    info->filter_applications = h->last_filters;
    info->filter_columns = h->last_filter_cols;
    info->counted = h->last_count;
    info->max_res = h->last_max_res;
    info->time_ms = h->timer.ms[P_TOTAL];
  }
  if (counted)
    for (int k = 0; k < m0; ++k) counted[k] = k < (int)h->counted.size() ? h->counted[k] : 0;
  return h->last_count;
}

int feast_tune_split_filter(int mode) {
  if (mode != 0 && mode != 1) return -1;
  g_split_filter.store(mode);
  return 0;
}

int feast_get_filter_values(feast_handle h, double* mu, int m0) {
  if (!h || !mu) return 0;
  int k = std::min(m0, (int)h->mu.size());
  for (int i = 0; i < k; ++i) mu[i] = h->mu[i];
  return k;
}

int feast_get_timings(feast_handle h, double* out, int count) {
  if (!h || !out) return 0;
  int k = std::min(count, 6);
  for (int i = 0; i < k; ++i) out[i] = h->timer.ms[i];
  return k;
}

int feast_set_profiling(feast_handle h, int on) {
  if (!h) return -1;
  for (feast_ctx* w : h->workers) feast_set_profiling(w, on);
  h->prof.on = (on != 0);
  for (int c = 0; c < NCLASS; ++c) {
    h->prof.ms[c] = 0;
    h->prof.flops[c] = 0;
    h->prof.launches[c] = 0;
  }
  return 0;
}

int feast_get_kernel_stats(feast_handle h, int kclass, double* total_ms, long long* launches,
                           double* dense_flops) {
  if (!h) return -1;
  if (kclass < 0 || kclass >= NCLASS) return -2;
  double ms = h->prof.ms[kclass], fl = h->prof.flops[kclass];
  long long nl = h->prof.launches[kclass];
  for (feast_ctx* w : h->workers) {
    ms += w->prof.ms[kclass];
    fl += w->prof.flops[kclass];
    nl += w->prof.launches[kclass];
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = nl;
  if (dense_flops) *dense_flops = fl;
  return 0;
}

}  // extern "C"
