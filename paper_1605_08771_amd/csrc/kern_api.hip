// Exported building blocks (include/feast_kernels.h) for kernel-level parity tests.
#include <vector>

#include "../../include/feast_kernels.h"
#include "common.h"
#include "kernels.h"

using namespace feast;

namespace {
int pick_np(int n, int prec) {  // the padding the solver uses (a multiple of the sweep block)
  const int nbt = sweep_block(n, prec == 0 ? 0 : 1);
  return (n + nbt - 1) / nbt * nbt;
}

// Device scratch of one call, freed on every path out of it (hipFree waits for the device).
struct DevMem {
  void* p = nullptr;
  explicit DevMem(size_t bytes) {
    if (bytes) FEAST_HIP(hipMalloc(&p, bytes));
  }
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  template <typename T>
  T* as() const {
    return (T*)p;
  }
};
}  // namespace

extern "C" int feast_kern_gemm(int prec, int opA, int opB, int M, int N, int K,
                               const double* alpha, const void* A, long lda, const void* B,
                               long ldb, const double* beta, void* C, long ldc,
                               void* hip_stream) {
  if (prec < 0 || prec > 3) return -1;
  if (opA < 0 || opA > 2) return -2;
  if (opB < 0 || opB > 2) return -3;
  if (M < 0) return -4;
  if (N < 0) return -5;
  if (K < 0) return -6;
  if (!alpha) return -7;
  if (!A && K > 0) return -8;
  if (lda < (opA == OP_N ? M : K) || lda < 1) return -9;
  if (!B && K > 0) return -10;
  if (ldb < (opB == OP_N ? K : N) || ldb < 1) return -11;
  if (!beta) return -12;
  if (!C) return -13;
  if (ldc < M || ldc < 1) return -14;
  try {
    hipStream_t s = (hipStream_t)hip_stream;
    if (prec == 0 || prec == 3) {
      Z3mScope z3(prec == 3);
      zgemm(s, opA, opB, M, N, K, zmake(alpha[0], alpha[1]), (const zd*)A, lda, (const zd*)B, ldb,
            zmake(beta[0], beta[1]), (zd*)C, ldc);
    } else {
      SplitBf16Scope split(prec == 2);
      cgemm(s, opA, opB, M, N, K, make_float2((float)alpha[0], (float)alpha[1]), (const zf*)A,
            lda, (const zf*)B, ldb, make_float2((float)beta[0], (float)beta[1]), (zf*)C, ldc);
    }
  } catch (const HipError&) {
    return -101;
  }
  return 0;
}

extern "C" int feast_kern_lu(int prec, const void* A, int lda, int n, int nc, const double* z,
                             void* LU, int* perm, int* np_out, void* hip_stream) {
  const bool column_steps = prec >= 0 && (prec & 8);
  if (column_steps) prec &= 7;
  if (prec < 0 || prec > 2) return -1;
  if (n < 1) return -4;
  if (!A) return -2;
  if (lda < n) return -3;
  if (nc < 1) return -5;
  if (!z) return -6;
  const int np = pick_np(n, prec);
  if (np_out) *np_out = np;
  if (!LU) return 0;
  if (!perm) return -8;
  try {
    hipStream_t s = (hipStream_t)hip_stream;
    DevMem zbuf(sizeof(zd) * nc), wbuf(lu_work_bytes(np, nc));
    zd* zdev = zbuf.as<zd>();
    FEAST_HIP(hipMemcpyAsync(zdev, z, sizeof(zd) * nc, hipMemcpyHostToDevice, s));
    LuWork w;
    lu_work_carve(w, wbuf.p, np, nc);
    w.column_steps = column_steps;
    if (prec == 0) {
      shift_matrices(s, A, lda, 0, n, np, zdev, nc, (zd*)LU, w.flag);
      lu_factor_f64(s, (zd*)LU, np, nc, w);
    } else {
      SplitBf16Scope split(prec == 2);
      shift_matrices_f32(s, A, lda, 0, n, np, zdev, nc, (zf*)LU, w.flag);
      lu_factor_f32(s, (zf*)LU, np, nc, w);
    }
    int flag = 0;
    FEAST_HIP(hipMemcpyAsync(perm, w.perm, sizeof(int) * (size_t)nc * np, hipMemcpyDeviceToDevice, s));
    FEAST_HIP(hipMemcpyAsync(&flag, w.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    FEAST_HIP(hipStreamSynchronize(s));
    return flag ? 6 : 0;
  } catch (const HipError&) {
    return -101;
  }
}

extern "C" int feast_kern_sweeps(int prec, int n, int nc, int m0, int sides, const void* LU,
                                 void* invL, void* invU, int compute_inverses, void* B, void* Z,
                                 int* np_out, int* nbt_out, void* hip_stream) {
  if (prec < 0 || prec > 2) return -1;
  if (n < 1) return -2;
  if (nc < 1) return -3;
  if (m0 < 1) return -4;
  if (sides != 1 && sides != 2) return -5;
  const int cls = prec == 0 ? 0 : 1;
  const int nbt = sweep_block(n, cls);
  const int np = (n + nbt - 1) / nbt * nbt;
  if (np_out) *np_out = np;
  if (nbt_out) *nbt_out = nbt;
  if (!LU) return 0;
  if (!invL || !invU) return -6;
  if (!B || !Z || B == Z) return -7;
  try {
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t esz = prec == 0 ? sizeof(zd) : sizeof(zf);
    DevMem tbuf(compute_inverses ? esz * (size_t)np * nbt : 0);
    void* tmp = tbuf.p;
    if (prec == 0) {
      if (compute_inverses)
        tri_inverse_blocks_f64(s, (const zd*)LU, np, nc, nbt, (zd*)invL, (zd*)invU, (zd*)tmp);
      solve_sweeps_f64(s, (const zd*)LU, (const zd*)invL, (const zd*)invU, np, nc, nbt, sides, m0,
                       (zd*)B, (zd*)Z);
    } else {
      SplitBf16Scope split(prec == 2);
      if (compute_inverses)
        tri_inverse_blocks_f32(s, (const zf*)LU, np, nc, nbt, (zf*)invL, (zf*)invU, (zf*)tmp);
      solve_sweeps_f32(s, (const zf*)LU, (const zf*)invL, (const zf*)invU, np, nc, nbt, sides, m0,
                       (zf*)B, (zf*)Z);
    }
    FEAST_HIP(hipStreamSynchronize(s));
    return 0;
  } catch (const HipError&) {
    return -101;
  }
}

extern "C" int feast_tune_sweep_block(int nbt) { return set_sweep_block_override(nbt); }

extern "C" int feast_kern_jacobi(const void* H, int m, double* d, void* W, void* hip_stream) {
  if (!H) return -1;
  if (m < 1) return -2;
  if (!d) return -3;
  if (!W) return -4;
  try {
    hipStream_t s = (hipStream_t)hip_stream;
    const int mp = jacobi_order(m);
    DevMem hbuf(sizeof(zd) * (size_t)m * m), vbuf(sizeof(zd) * (size_t)mp * mp),
        wbuf(sizeof(zd) * jacobi_work(mp)), dbuf(sizeof(double) * mp), fbuf(256),
        rbuf(sizeof(int) * mp);
    zd* Hc = hbuf.as<zd>();
    zd* V = vbuf.as<zd>();
    copy_matrix(s, (const zd*)H, m, Hc, m, m, m);
    int sweeps = jacobi_eigh(s, Hc, m, dbuf.as<double>(), V, wbuf.as<zd>(), fbuf.as<int>(), 60,
                             nullptr, mp);
    sort_eigen(s, dbuf.as<double>(), V, m, mp, d, (zd*)W, rbuf.as<int>());
    FEAST_HIP(hipStreamSynchronize(s));
    return sweeps;
  } catch (const HipError&) {
    return -101;
  }
}
