// Batched complex GEMM on CDNA4 matrix cores (FP64 v_mfma_f64_16x16x4f64, FP32
// v_mfma_f32_16x16x4f32), C = alpha op(A) op(B) + beta C with op in {N, T, C}.
//
// Complex products are decomposed into four real MFMAs per 16x16x4 step
// (re*re, -im*im into the real accumulator; re*im, im*re into the imaginary one), so
// every MFMA flop is a useful flop of the 8-flop complex multiply-add.
//
// Tiling: 256 threads = 4 wave64s in a 2x2 grid, workgroup tile 64x64 complex outputs,
// K-tile 16 complex, double-buffered LDS (operands are staged k-major so that lanes 0..15
// of an MFMA fetch read 16 consecutive entries).  Each wave owns 32x32 outputs (2x2 MFMA
// blocks).  The MFMA is fed with op(B)^T as its first operand and op(A)^T as its second,
// so it produces C^T: the lane index then runs along the rows of the column-major C and
// the epilogue stores 16 consecutive rows per lane group.
//
// Batching: two nested strided batch dimensions (blockIdx.y, blockIdx.z) with their own
// element strides for A, B and C; split-K reductions and per-node/per-block batches are
// both expressed this way.
#include "common.h"
#include "kernels.h"

namespace feast {

thread_local GemmProfiler* g_gemm_prof = nullptr;

namespace {

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;

template <typename T>
struct CT;
template <>
struct CT<double> {
  typedef double2 v2;
  typedef d4 acc;
};
template <>
struct CT<float> {
  typedef float2 v2;
  typedef f4 acc;
};

__device__ inline d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// Row of the 16x16 MFMA result held by lane l in accumulator register v.
template <typename T>
__device__ inline int mfma_row(int l, int v);
template <>
__device__ inline int mfma_row<double>(int l, int v) { return (l >> 4) + 4 * v; }
template <>
__device__ inline int mfma_row<float>(int l, int v) { return 4 * (l >> 4) + v; }

// Guarded load of one complex entry, conjugated when CONJ.
template <typename v2, bool CONJ>
__device__ __forceinline__ v2 ldc_(const v2* p, bool ok) {
  v2 v;
  if (ok) {
    v = *p;
  } else {
    v.x = 0;
    v.y = 0;
  }
  if (CONJ) v.y = -v.y;
  return v;
}

template <typename T, int OPA, int OPB>
__global__ __launch_bounds__(NT) void gemm_kernel(int M, int N, int K,
                                                  typename CT<T>::v2 alpha,
                                                  typename CT<T>::v2 beta,
                                                  const typename CT<T>::v2* __restrict__ A,
                                                  long lda, long sA1, long sA2,
                                                  const typename CT<T>::v2* __restrict__ B,
                                                  long ldb, long sB1, long sB2,
                                                  typename CT<T>::v2* __restrict__ C, long ldc,
                                                  long sC1, long sC2, int tilesM, int splitk) {
  typedef typename CT<T>::v2 v2;
  typedef typename CT<T>::acc accv;
  __shared__ v2 As[2][BK][BM];
  __shared__ v2 Bs[2][BK][BN];

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int tile = blockIdx.x;
  const int i0 = (tile % tilesM) * BM, j0 = (tile / tilesM) * BN;
  A += blockIdx.z * sA2;
  B += blockIdx.z * sB2;
  C += blockIdx.y * sC1 + blockIdx.z * sC2;
  if (splitk == 0) {
    A += blockIdx.y * sA1;
    B += blockIdx.y * sB1;
  } else {  // blockIdx.y selects a K chunk; partial products go to separate C slices
    const long kb = (long)blockIdx.y * splitk;
    K = (K - kb < splitk) ? (int)(K - kb) : splitk;
    A += (OPA == OP_N) ? kb * lda : kb;
    B += (OPB == OP_N) ? kb : kb * ldb;
  }

  const v2 zero = {T(0), T(0)};
  v2 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;

#define FEAST_LOAD_A(R, DST)                                                  \
  {                                                                           \
    if (OPA == OP_N) {                                                        \
      int i = t & 63, k = (t >> 6) + 4 * (R);                                 \
      int gi = i0 + i, gk = k0 + k;                                           \
      DST = (gi < M && gk < K) ? A[gi + (long)gk * lda] : zero;               \
    } else {                                                                  \
      int k = t & 15, i = (t >> 4) + 16 * (R);                                \
      int gi = i0 + i, gk = k0 + k;                                           \
      DST = ldc_<v2, OPA == OP_C>(A + gk + (long)gi * lda, gi < M && gk < K);       \
    }                                                                         \
  }
#define FEAST_LOAD_B(R, DST)                                                  \
  {                                                                           \
    if (OPB == OP_N) {                                                        \
      int k = t & 15, j = (t >> 4) + 16 * (R);                                \
      int gj = j0 + j, gk = k0 + k;                                           \
      DST = (gj < N && gk < K) ? B[gk + (long)gj * ldb] : zero;               \
    } else {                                                                  \
      int j = t & 63, k = (t >> 6) + 4 * (R);                                 \
      int gj = j0 + j, gk = k0 + k;                                           \
      DST = ldc_<v2, OPB == OP_C>(B + gj + (long)gk * ldb, gj < N && gk < K);       \
    }                                                                         \
  }
#define FEAST_LOAD_TILE(K0)                                                   \
  {                                                                           \
    const int k0 = (K0);                                                      \
    FEAST_LOAD_A(0, ra0) FEAST_LOAD_A(1, ra1) FEAST_LOAD_A(2, ra2) FEAST_LOAD_A(3, ra3) \
    FEAST_LOAD_B(0, rb0) FEAST_LOAD_B(1, rb1) FEAST_LOAD_B(2, rb2) FEAST_LOAD_B(3, rb3) \
  }
#define FEAST_STORE_AB(R, SA, SB)                                             \
  {                                                                           \
    if (OPA == OP_N) As[buf_][(t >> 6) + 4 * (R)][t & 63] = SA;               \
    else As[buf_][t & 15][(t >> 4) + 16 * (R)] = SA;                          \
    if (OPB == OP_N) Bs[buf_][t & 15][(t >> 4) + 16 * (R)] = SB;              \
    else Bs[buf_][(t >> 6) + 4 * (R)][t & 63] = SB;                           \
  }
#define FEAST_STORE_TILE(BUF)                                                 \
  {                                                                           \
    const int buf_ = (BUF);                                                   \
    FEAST_STORE_AB(0, ra0, rb0) FEAST_STORE_AB(1, ra1, rb1)                   \
    FEAST_STORE_AB(2, ra2, rb2) FEAST_STORE_AB(3, ra3, rb3)                   \
  }

  accv accr[2][2], acci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      accr[a][b] = accv{T(0), T(0), T(0), T(0)};
      acci[a][b] = accv{T(0), T(0), T(0), T(0)};
    }

  const int nkt = (K + BK - 1) / BK;
  if (nkt > 0) {
    FEAST_LOAD_TILE(0)
    FEAST_STORE_TILE(0)
  }
  __syncthreads();
  for (int kt = 0; kt < nkt; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nkt) FEAST_LOAD_TILE((kt + 1) * BK)
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kidx = kk * 4 + (lane >> 4);
      v2 fa[2], fb[2];
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) fa[mb] = As[buf][kidx][wm * 32 + mb * 16 + (lane & 15)];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) fb[nb] = Bs[buf][kidx][wn * 32 + nb * 16 + (lane & 15)];
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          accr[mb][nb] = mfma(fb[nb].x, fa[mb].x, accr[mb][nb]);
          accr[mb][nb] = mfma(-fb[nb].y, fa[mb].y, accr[mb][nb]);
          acci[mb][nb] = mfma(fb[nb].x, fa[mb].y, acci[mb][nb]);
          acci[mb][nb] = mfma(fb[nb].y, fa[mb].x, acci[mb][nb]);
        }
    }
    if (kt + 1 < nkt) FEAST_STORE_TILE(buf ^ 1)
    __syncthreads();
  }

  const bool beta_zero = (beta.x == T(0) && beta.y == T(0));
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int i = i0 + wm * 32 + mb * 16 + (lane & 15);
        int j = j0 + wn * 32 + nb * 16 + mfma_row<T>(lane, v);
        if (i < M && j < N) {
          T re = accr[mb][nb][v], im = acci[mb][nb][v];
          v2 out;
          out.x = alpha.x * re - alpha.y * im;
          out.y = alpha.x * im + alpha.y * re;
          if (!beta_zero) {
            v2 c = C[i + (long)j * ldc];
            out.x += beta.x * c.x - beta.y * c.y;
            out.y += beta.x * c.y + beta.y * c.x;
          }
          C[i + (long)j * ldc] = out;
        }
      }
#undef FEAST_LOAD_A
#undef FEAST_LOAD_B
#undef FEAST_LOAD_TILE
#undef FEAST_STORE_AB
#undef FEAST_STORE_TILE
}

template <typename T, int OPA, int OPB>
void launch(hipStream_t s, int M, int N, int K, typename CT<T>::v2 alpha,
            const typename CT<T>::v2* A, long lda, const typename CT<T>::v2* B, long ldb,
            typename CT<T>::v2 beta, typename CT<T>::v2* C, long ldc, const Batch& bt) {
  int tm = (M + BM - 1) / BM, tn = (N + BN - 1) / BN;
  dim3 grid(tm * tn, bt.n1, bt.n2);
  hipLaunchKernelGGL((gemm_kernel<T, OPA, OPB>), grid, dim3(NT), 0, s, M, N, K, alpha, beta, A,
                     lda, bt.sA1, bt.sA2, B, ldb, bt.sB1, bt.sB2, C, ldc, bt.sC1, bt.sC2, tm,
                     bt.splitk);
}

template <typename T>
void dispatch(hipStream_t s, int opA, int opB, int M, int N, int K, typename CT<T>::v2 alpha,
              const typename CT<T>::v2* A, long lda, const typename CT<T>::v2* B, long ldb,
              typename CT<T>::v2 beta, typename CT<T>::v2* C, long ldc, const Batch& bt) {
  if (M <= 0 || N <= 0 || bt.n1 <= 0 || bt.n2 <= 0) return;
  GemmProfiler* prof = g_gemm_prof;
  const double flops = 8.0 * M * N * (double)(K > 0 ? K : 0) *
                       (bt.splitk > 0 ? 1.0 : (double)bt.n1) * bt.n2;
#define FEAST_G(a, b)                                                                \
  if (opA == a && opB == b) {                                                       \
    if (prof) prof->begin(s);                                                       \
    launch<T, a, b>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);           \
    FEAST_LAUNCH_CHECK();                                                           \
    if (prof) prof->end(s, flops);                                                  \
    return;                                                                         \
  }
  FEAST_G(OP_N, OP_N) FEAST_G(OP_N, OP_T) FEAST_G(OP_N, OP_C)
  FEAST_G(OP_T, OP_N) FEAST_G(OP_T, OP_T) FEAST_G(OP_T, OP_C)
  FEAST_G(OP_C, OP_N) FEAST_G(OP_C, OP_T) FEAST_G(OP_C, OP_C)
#undef FEAST_G
}

}  // namespace

void zgemm(hipStream_t s, int opA, int opB, int M, int N, int K, zd alpha, const zd* A, long lda,
           const zd* B, long ldb, zd beta, zd* C, long ldc, const Batch& bt) {
  dispatch<double>(s, opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
}

void cgemm(hipStream_t s, int opA, int opB, int M, int N, int K, zf alpha, const zf* A, long lda,
           const zf* B, long ldb, zf beta, zf* C, long ldc, const Batch& bt) {
  dispatch<float>(s, opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
}

}  // namespace feast
