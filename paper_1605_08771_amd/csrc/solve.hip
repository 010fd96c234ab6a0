// Multi-right-hand-side triangular solves with the node factors, and the weighted
// accumulation of eq. (contour_int_quad).
//
// For every node j (P_j M_j = L_j U_j) and complex Hermitian A two systems share the
// factors (Sec. 1 quadrature folded onto the upper half circle):
//   side 0:  Y_j  = (z_j I - A)^{-1} X      = U^{-1} L^{-1} P X
//   side 1:  Y'_j = (conj z_j I - A)^{-1} X = M_j^{-H} X = P^T L^{-H} U^{-H} X.
// A real symmetric A needs side 0 only (Y'_j = conj Y_j).
//
// Block sweeps of height nbt: the diagonal blocks are applied through their explicit
// inverses (computed once per factorization), the off-diagonal blocks through one GEMM per
// block step, so every flop of the sweep runs on the matrix cores.  U^H and L^H are never
// formed: the GEMM reads U and L with a conjugate-transpose operand.
#include <atomic>

#include "common.h"
#include "kernels.h"
#include "sweep_tune.h"

namespace feast {

namespace {

template <typename T>
struct V2;
template <>
struct V2<double> {
  typedef double2 t;
};
template <>
struct V2<float> {
  typedef float2 t;
};

constexpr int TB = 64;  // base block of the triangular inverses

// Inverse of one 64x64 diagonal block: which == 0 -> unit lower L, which == 1 -> upper U.
template <typename T>
__global__ __launch_bounds__(256) void tri_inv64_kernel(const typename V2<T>::t* __restrict__ LU,
                                                        int np, int nbt,
                                                        typename V2<T>::t* __restrict__ invL,
                                                        typename V2<T>::t* __restrict__ invU) {
  typedef typename V2<T>::t v2;
  __shared__ v2 Tm[TB][TB + 1];
  __shared__ v2 X[TB][TB + 1];
  const int q = blockIdx.x, node = blockIdx.y, which = blockIdx.z;
  const int t = threadIdx.x;
  LU += (long)node * np * np;
  const int R = q * TB;
  for (int e = t; e < TB * TB; e += 256) {
    int r = e % TB, c = e / TB;
    Tm[r][c] = LU[R + r + (long)(R + c) * np];
    X[r][c] = v2{T(r == c ? 1 : 0), T(0)};
  }
  __syncthreads();
  if (which == 0) {
    for (int r = 0; r < TB - 1; ++r) {  // X = L^{-1}: forward, unit diagonal
      int rows = TB - 1 - r;
      for (int e = t; e < rows * (r + 1); e += 256) {
        int i = r + 1 + e % rows, c = e / rows;  // only columns c <= r are nonzero in row r
        v2 l = Tm[i][r], x = X[r][c];
        X[i][c].x -= l.x * x.x - l.y * x.y;
        X[i][c].y -= l.x * x.y + l.y * x.x;
      }
      __syncthreads();
    }
  } else {
    for (int r = TB - 1; r >= 0; --r) {  // X = U^{-1}: backward
      if (t < TB - r) {                 // row r is nonzero for columns c >= r
        int c = r + t;
        v2 d = Tm[r][r], x = X[r][c];
        // x / d with Smith scaling
        v2 o;
        if (fabs(d.x) >= fabs(d.y)) {
          T s = d.y / d.x, den = d.x + d.y * s;
          o.x = (x.x + x.y * s) / den;
          o.y = (x.y - x.x * s) / den;
        } else {
          T s = d.x / d.y, den = d.y + d.x * s;
          o.x = (x.x * s + x.y) / den;
          o.y = (x.y * s - x.x) / den;
        }
        X[r][c] = o;
      }
      __syncthreads();
      int cols = TB - r;
      for (int e = t; e < r * cols; e += 256) {
        int i = e % r, c = r + e / r;
        v2 u = Tm[i][r], x = X[r][c];
        X[i][c].x -= u.x * x.x - u.y * x.y;
        X[i][c].y -= u.x * x.y + u.y * x.x;
      }
      __syncthreads();
    }
  }
  v2* out = (which == 0 ? invL : invU) + (long)node * np * nbt;
  const int b = R / nbt, o = R % nbt;
  out += (long)b * nbt * nbt + o + (long)o * nbt;
  for (int e = t; e < TB * TB; e += 256) {
    int r = e % TB, c = e / TB;
    out[r + (long)c * nbt] = X[r][c];
  }
}

template <typename T>
__global__ void gather_kernel(const zd* __restrict__ X, long ldx, int n, int np, int m0, int nc,
                              int sides, const int* __restrict__ perm,
                              typename V2<T>::t* __restrict__ B) {
  typedef typename V2<T>::t v2;
  long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  long per = (long)np * m0;
  if (idx >= per * nc * sides) return;
  long blk = idx / per, e = idx % per;
  int node = (int)(blk / sides), side = (int)(blk % sides);
  int r = (int)(e % np), c = (int)(e / np);
  v2 out = {T(0), T(0)};
  if (r < n) {
    int src = (side == 0) ? perm[(long)node * np + r] : r;
    if (src < n) {  // a padded row can only move up after an exact zero pivot (reported)
      zd x = X[src + (long)c * ldx];
      out.x = (T)x.x;
      out.y = (T)x.y;
    }
  }
  B[idx] = out;
}

__global__ void accumulate_kernel(const zd* __restrict__ Y, int n, int np, int m0, int nc,
                                  int sides, const zd* __restrict__ omega,
                                  const int* __restrict__ pinv, zd* __restrict__ Q, long ldq) {
  long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)n * m0) return;
  int i = (int)(idx % n), c = (int)(idx / n);
  long per = (long)np * m0;
  double re = 0, im = 0;
  for (int j = 0; j < nc; ++j) {
    zd w = omega[j];
    const zd* y0 = Y + (long)j * sides * per;
    zd a = y0[i + (long)c * np];
    if (sides == 2) {
      zd b = y0[per + pinv[(long)j * np + i] + (long)c * np];
      re += w.x * a.x - w.y * a.y + w.x * b.x + w.y * b.y;  // w a + conj(w) b
      im += w.x * a.y + w.y * a.x + w.x * b.y - w.y * b.x;
    } else {
      re += 2.0 * (w.x * a.x - w.y * a.y);  // 2 Re(w a)
    }
  }
  Q[i + (long)c * ldq] = zmake(re, im);
}

template <typename T>
void gemm_t(hipStream_t s, int opA, int opB, int M, int N, int K, double ar, const typename V2<T>::t* A,
            long lda, const typename V2<T>::t* B, long ldb, double br, typename V2<T>::t* C, long ldc,
            const Batch& bt);
template <>
void gemm_t<double>(hipStream_t s, int opA, int opB, int M, int N, int K, double ar, const zd* A,
                    long lda, const zd* B, long ldb, double br, zd* C, long ldc, const Batch& bt) {
  zgemm(s, opA, opB, M, N, K, zmake(ar, 0), A, lda, B, ldb, zmake(br, 0), C, ldc, bt);
}
template <>
void gemm_t<float>(hipStream_t s, int opA, int opB, int M, int N, int K, double ar, const zf* A,
                   long lda, const zf* B, long ldb, double br, zf* C, long ldc, const Batch& bt) {
  cgemm(s, opA, opB, M, N, K, make_float2((float)ar, 0), A, lda, B, ldb, make_float2((float)br, 0),
        C, ldc, bt);
}

template <typename T>
void tri_inverse(hipStream_t s, const typename V2<T>::t* LU, int np, int nc, int nbt,
                 typename V2<T>::t* invL, typename V2<T>::t* invU, typename V2<T>::t* tmp) {
  typedef typename V2<T>::t v2;
  const size_t invbytes = sizeof(v2) * (size_t)nc * np * nbt;
  fill_zero(s, invL, invbytes);
  fill_zero(s, invU, invbytes);
  hipLaunchKernelGGL((tri_inv64_kernel<T>), dim3(np / TB, nc, 2), dim3(256), 0, s, LU, np, nbt,
                     invL, invU);
  FEAST_LAUNCH_CHECK();
  const int nblk = np / nbt;
  for (int sz = TB; 2 * sz <= nbt; sz *= 2) {
    const int ppb = nbt / (2 * sz);  // pairs per nbt block
    for (int nd = 0; nd < nc; ++nd) {
      const v2* F = LU + (long)nd * np * np;
      v2* iL = invL + (long)nd * np * nbt;
      v2* iU = invU + (long)nd * np * nbt;
      Batch bF;  // factor sub-blocks: pair (b1 within nbt block, b2 = nbt block)
      bF.n1 = ppb;
      bF.n2 = nblk;
      bF.sA1 = 2L * sz * (np + 1);
      bF.sA2 = (long)nbt * (np + 1);
      bF.sB1 = 2L * sz * (nbt + 1);
      bF.sB2 = (long)nbt * nbt;
      bF.sC1 = (long)sz * sz;
      bF.sC2 = (long)ppb * sz * sz;
      Batch bI;  // inverse sub-blocks x tmp -> inverse sub-blocks
      bI.n1 = ppb;
      bI.n2 = nblk;
      bI.sA1 = 2L * sz * (nbt + 1);
      bI.sA2 = (long)nbt * nbt;
      bI.sB1 = (long)sz * sz;
      bI.sB2 = (long)ppb * sz * sz;
      bI.sC1 = 2L * sz * (nbt + 1);
      bI.sC2 = (long)nbt * nbt;
      // lower: [[A,0],[C,D]]^{-1} = [[iA,0],[-iD C iA, iD]]
      gemm_t<T>(s, OP_N, OP_N, sz, sz, sz, 1.0, F + sz, np, iL, nbt, 0.0, tmp, sz, bF);
      gemm_t<T>(s, OP_N, OP_N, sz, sz, sz, -1.0, iL + sz + (long)sz * nbt, nbt, tmp, sz, 0.0,
                iL + sz, nbt, bI);
      // upper: [[A,B],[0,D]]^{-1} = [[iA, -iA B iD],[0, iD]]
      gemm_t<T>(s, OP_N, OP_N, sz, sz, sz, 1.0, F + (long)sz * np, np,
                iU + sz + (long)sz * nbt, nbt, 0.0, tmp, sz, bF);
      gemm_t<T>(s, OP_N, OP_N, sz, sz, sz, -1.0, iU, nbt, tmp, sz, 0.0, iU + (long)sz * nbt, nbt,
                bI);
    }
  }
}

template <typename T>
void gemm_pair_t(hipStream_t s, int op0, int op1, int M, int N, int K, double ar,
                 const typename V2<T>::t* const A[2], const long lda[2],
                 const typename V2<T>::t* const B[2], const long ldb[2], double br,
                 typename V2<T>::t* const C[2], const long ldc[2], const Batch& bt);
template <>
void gemm_pair_t<double>(hipStream_t s, int op0, int op1, int M, int N, int K, double ar,
                         const zd* const A[2], const long lda[2], const zd* const B[2],
                         const long ldb[2], double br, zd* const C[2], const long ldc[2],
                         const Batch& bt) {
  zgemm_pair(s, op0, op1, OP_N, M, N, K, zmake(ar, 0), A, lda, B, ldb, zmake(br, 0), C, ldc, bt);
}
template <>
void gemm_pair_t<float>(hipStream_t s, int op0, int op1, int M, int N, int K, double ar,
                        const zf* const A[2], const long lda[2], const zf* const B[2],
                        const long ldb[2], double br, zf* const C[2], const long ldc[2],
                        const Batch& bt) {
  cgemm_pair(s, op0, op1, OP_N, M, N, K, make_float2((float)ar, 0), A, lda, B, ldb,
             make_float2((float)br, 0), C, ldc, bt);
}

// Block sweeps for all (node, side) systems; both sides of a block step share one launch.
template <typename T>
void sweeps(hipStream_t s, const typename V2<T>::t* LU, const typename V2<T>::t* invL,
            const typename V2<T>::t* invU, int np, int nc, int nbt, int sides, int m0,
            typename V2<T>::t* B, typename V2<T>::t* Z) {
  typedef typename V2<T>::t v2;
  const int nblk = np / nbt;
  const long per = (long)np * m0;
  Batch bi;  // inverse blocks x right-hand sides, over nodes
  bi.n1 = nc;
  bi.sA1 = (long)np * nbt;
  bi.sB1 = bi.sC1 = sides * per;
  Batch bg = bi;  // factor blocks x right-hand sides, over nodes
  bg.sA1 = (long)np * np;
  Batch bl = bi, bu = bi;  // the inverse blocks are lower (L, U^H) or upper (U, L^H)
  bl.tri = 1;
  bu.tri = 2;
  const long ldn[2] = {np, np}, ldb[2] = {nbt, nbt};
  v2* Bs[2] = {B, B + per};
  v2* Zs[2] = {Z, Z + per};
  // lower sweep: side 0 with L, side 1 with U^H (solution into Z)
  for (int k = 0; k < nblk; ++k) {
    const int r0 = k * nbt;
    const v2* iA[2] = {invL + (long)k * nbt * nbt, invU + (long)k * nbt * nbt};
    const v2* rhs[2] = {Bs[0] + r0, Bs[1] + r0};
    v2* out[2] = {Zs[0] + r0, Zs[1] + r0};
    if (sides == 2)
      gemm_pair_t<T>(s, OP_N, OP_C, nbt, m0, nbt, 1.0, iA, ldb, rhs, ldn, 0.0, out, ldn, bl);
    else
      gemm_t<T>(s, OP_N, OP_N, nbt, m0, nbt, 1.0, iA[0], nbt, rhs[0], np, 0.0, out[0], np, bl);
    const int rest = np - r0 - nbt;
    if (rest > 0) {
      const v2* T2[2] = {LU + (r0 + nbt) + (long)r0 * np, LU + r0 + (long)(r0 + nbt) * np};
      const v2* zin[2] = {Zs[0] + r0, Zs[1] + r0};
      v2* upd[2] = {Bs[0] + r0 + nbt, Bs[1] + r0 + nbt};
      if (sides == 2)
        gemm_pair_t<T>(s, OP_N, OP_C, rest, m0, nbt, -1.0, T2, ldn, zin, ldn, 1.0, upd, ldn, bg);
      else
        gemm_t<T>(s, OP_N, OP_N, rest, m0, nbt, -1.0, T2[0], np, zin[0], np, 1.0, upd[0], np,
                  bg);
    }
  }
  // upper sweep: side 0 with U, side 1 with L^H; right-hand side Z, solution into B
  for (int k = nblk - 1; k >= 0; --k) {
    const int r0 = k * nbt;
    const v2* iA[2] = {invU + (long)k * nbt * nbt, invL + (long)k * nbt * nbt};
    const v2* rhs[2] = {Zs[0] + r0, Zs[1] + r0};
    v2* out[2] = {Bs[0] + r0, Bs[1] + r0};
    if (sides == 2)
      gemm_pair_t<T>(s, OP_N, OP_C, nbt, m0, nbt, 1.0, iA, ldb, rhs, ldn, 0.0, out, ldn, bu);
    else
      gemm_t<T>(s, OP_N, OP_N, nbt, m0, nbt, 1.0, iA[0], nbt, rhs[0], np, 0.0, out[0], np, bu);
    if (r0 > 0) {
      const v2* T2[2] = {LU + (long)r0 * np, LU + r0};
      const v2* yin[2] = {Bs[0] + r0, Bs[1] + r0};
      v2* upd[2] = {Zs[0], Zs[1]};
      if (sides == 2)
        gemm_pair_t<T>(s, OP_N, OP_C, r0, m0, nbt, -1.0, T2, ldn, yin, ldn, 1.0, upd, ldn, bg);
      else
        gemm_t<T>(s, OP_N, OP_N, r0, m0, nbt, -1.0, T2[0], np, yin[0], np, 1.0, upd[0], np, bg);
    }
  }
}

}  // namespace

void tri_inverse_blocks_f64(hipStream_t s, const zd* LU, int np, int nc, int nbt, zd* invL,
                            zd* invU, zd* tmp) {
  tri_inverse<double>(s, LU, np, nc, nbt, invL, invU, tmp);
}
void tri_inverse_blocks_f32(hipStream_t s, const zf* LU, int np, int nc, int nbt, zf* invL,
                            zf* invU, zf* tmp) {
  tri_inverse<float>(s, LU, np, nc, nbt, invL, invU, tmp);
}

void gather_rhs(hipStream_t s, const zd* X, long ldx, int n, int np, int m0, int nc, int sides,
                const int* perm, zd* B) {
  long tot = (long)np * m0 * nc * sides;
  hipLaunchKernelGGL((gather_kernel<double>), dim3((tot + 255) / 256), dim3(256), 0, s, X, ldx, n,
                     np, m0, nc, sides, perm, B);
  FEAST_LAUNCH_CHECK();
}
void gather_rhs_f32(hipStream_t s, const zd* X, long ldx, int n, int np, int m0, int nc,
                    int sides, const int* perm, zf* B) {
  long tot = (long)np * m0 * nc * sides;
  hipLaunchKernelGGL((gather_kernel<float>), dim3((tot + 255) / 256), dim3(256), 0, s, X, ldx, n,
                     np, m0, nc, sides, perm, B);
  FEAST_LAUNCH_CHECK();
}

namespace {
std::atomic<int> g_sweep_override{0};
}

// The tuned table (sweep_tune.h, written by the package's autotune module from measured
// solves), unless the process-wide override is set.  Rows are ordered by n_max within a
// precision class; orders beyond the last row take the largest height the FP64 residual
// floor allows.  A row holds for a range of orders measured at one of them, so the height is
// halved (down to 64) while padding n to a multiple of it would add more than n / 8 rows.
int sweep_block(int n, int prec_class) {
  const int o = g_sweep_override.load(std::memory_order_relaxed);
  if (o > 0) return o;
  int nbt = 512;
  for (const SweepTuneRow& r : kSweepTune)
    if (r.prec_class == prec_class && n <= r.n_max) {
      nbt = r.nbt;
      break;
    }
  while (nbt > 64 && 8L * ((n + nbt - 1) / nbt * nbt - n) > n) nbt /= 2;
  return nbt;
}

int set_sweep_block_override(int nbt) {
  if (nbt != 0 && nbt != 64 && nbt != 128 && nbt != 256 && nbt != 512) return -1;
  g_sweep_override.store(nbt, std::memory_order_relaxed);
  return 0;
}

void solve_sweeps_f64(hipStream_t s, const zd* LU, const zd* invL, const zd* invU, int np,
                      int nc, int nbt, int sides, int m0, zd* B, zd* Y) {
  sweeps<double>(s, LU, invL, invU, np, nc, nbt, sides, m0, B, Y);
}
void solve_sweeps_f32(hipStream_t s, const zf* LU, const zf* invL, const zf* invU, int np,
                      int nc, int nbt, int sides, int m0, zf* B, zf* Y) {
  sweeps<float>(s, LU, invL, invU, np, nc, nbt, sides, m0, B, Y);
}

void accumulate(hipStream_t s, const zd* Y, int n, int np, int m0, int nc, int sides,
                const zd* omega_dev, const int* pinv, zd* Q, long ldq) {
  long tot = (long)n * m0;
  hipLaunchKernelGGL(accumulate_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, Y, n, np, m0,
                     nc, sides, omega_dev, pinv, Q, ldq);
  FEAST_LAUNCH_CHECK();
}

}  // namespace feast
