// Batched complex GEMM on CDNA4 matrix cores (FP64 v_mfma_f64_16x16x4f64, FP32
// v_mfma_f32_16x16x4f32), C = alpha op(A) op(B) + beta C with op in {N, T, C}.
//
// Complex products are decomposed into four real MFMAs per 16x16x4 step
// (re*re, -im*im into the real accumulator; re*im, im*re into the imaginary one), so
// every MFMA flop is a useful flop of the 8-flop complex multiply-add.
//
// Tiling: 256 threads = 4 wave64s in a 2x2 grid, workgroup tile 64x64 complex outputs,
// double-buffered LDS, one register set of staged operands: the global loads of K-tile kt+1
// are in flight while K-tile kt is multiplied, and the other resident workgroups cover the
// rest of their latency.  Occupancy is what hides it (measured against two register sets with
// loads two K-tiles ahead at fewer waves): FP32 tiles (K-tile 16, about 120 VGPRs, 33 KB of
// LDS) run four waves per SIMD, 2-9 % faster on the hot shapes than three; four-product FP64
// tiles (K-tile 8, about 140 VGPRs, 33 KB) three, 2-4 % faster than two with a 16-deep K-tile;
// three-product FP64 tiles (K-tile 16, about 180 VGPRs: a third accumulator set) two, where a
// K-tile of 8 was 3 % slower.  Interior tiles whose K is a multiple of the K-tile load without
// bounds tests.  Within a
// 4-deep k step the MFMAs are issued so that eight independent accumulators separate the two
// products that feed the same one.  Operands are staged k-major so that lanes 0..15
// of an MFMA fetch read 16 consecutive entries; LDS rows are padded by one entry so that
// the transposing stores (k contiguous in HBM, k-major in LDS) hit 16 distinct banks.
// Each wave owns 32x32 outputs (2x2 MFMA blocks).  The MFMA is fed with op(B)^T as its
// first operand and op(A)^T as its second, so it produces C^T: the lane index then runs
// along the rows of the column-major C and the epilogue stores 16 consecutive rows per lane
// group.
//
// Scheduling: the linear workgroup id is remapped so that each of the 8 XCDs receives a
// contiguous range of output tiles, ordered with the N tiles of one M row adjacent: tiles
// that read the same rows of op(A) run on the same XCD and share its L2.
//
// Batching: two nested strided batch dimensions with their own element strides, and up to
// two independent problems (own A/B/C pointers, leading dimensions and op(A)) with the same
// M, N, K in one launch; split-K reductions are a batch dimension over K chunks.
#include <algorithm>
#include <atomic>

#include "common.h"
#include "kernels.h"

namespace feast {

thread_local GemmProfiler* g_gemm_prof = nullptr;
thread_local bool g_split_bf16 = false;
thread_local bool g_z3m = false;

namespace {

constexpr int BM = 64, BN = 64, NT = 256, PAD = 1;

// FEAST_GEMM_3M = 1: FP32 complex products as three real matrix-core products (Gauss's
// method: 3 MFMAs per 16x16x4 complex step instead of 4, a quarter less matrix-core work; the
// imaginary part is formed as a difference, with a normwise error bound a small multiple of
// the four-product one).  0: the four-product form.  FP64 products use the three-product form
// only inside a Z3mScope (the caller decides where its accuracy suffices).
#ifndef FEAST_GEMM_3M
#define FEAST_GEMM_3M 1
#endif


// bk: K-tile depth (complex entries) of the staged operand tiles, by precision and product
// form (a 32-deep FP32 tile needs 248-255 VGPRs and twice the LDS, and measured 8-13 % slower
// on the hot shapes).  waves: waves per SIMD the kernel is compiled for (the register budget:
// 128 VGPRs at four, 168 at three, 256 at two).
template <typename T>
struct CT;
template <>
struct CT<double> {
  typedef double2 v2;
  typedef d4 acc;
  static constexpr int bk(bool g3) { return g3 ? 16 : 8; }
  static constexpr int waves(bool g3) { return g3 ? 2 : 3; }
};
template <>
struct CT<float> {
  typedef float2 v2;
  typedef f4 acc;
  static constexpr int bk(bool) { return 16; }
  static constexpr int waves(bool) { return 4; }
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

template <typename v2>
struct Args {
  int M, N, K, tilesM, tilesN, n1, n2, splitk, tri;
  v2 alpha, beta;
  const v2* A[2];
  const v2* B[2];
  v2* C[2];
  long lda[2], ldb[2], ldc[2];
  long sA1, sA2, sB1, sB2, sC1, sC2;
};

// One output tile of one problem, op(A) = OPA.  (i0, j0) is the tile origin.
template <typename T, int OPA, int OPB, bool G3>
__device__ __forceinline__ void gemm_tile(const Args<typename CT<T>::v2>& a, int prob, int b1,
                                          int b2, int i0, int j0,
                                          typename CT<T>::v2 (*As)[CT<T>::bk(G3)][BM + PAD],
                                          typename CT<T>::v2 (*Bs)[CT<T>::bk(G3)][BN + PAD]) {
  typedef typename CT<T>::v2 v2;
  typedef typename CT<T>::acc accv;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int M = a.M, N = a.N;
  int K = a.K;
  const long lda = a.lda[prob], ldb = a.ldb[prob], ldc = a.ldc[prob];
  const v2* A = a.A[prob] + b2 * a.sA2;
  const v2* B = a.B[prob] + b2 * a.sB2;
  v2* C = a.C[prob] + b1 * a.sC1 + b2 * a.sC2;
  if (a.splitk == 0) {
    A += b1 * a.sA1;
    B += b1 * a.sB1;
  } else {  // b1 selects a K chunk; partial products go to separate C slices
    const long kb = (long)b1 * a.splitk;
    K = (K - kb < a.splitk) ? (int)(K - kb) : a.splitk;
    A += (OPA == OP_N) ? kb * lda : kb;
    B += (OPB == OP_N) ? kb : kb * ldb;
  }
  if (a.tri != 0) {  // op(A) triangular (square): only the K range of its nonzero part
    const int kb = (a.tri == 2) ? i0 : 0;
    const int ke = (a.tri == 1) ? min(K, i0 + BM) : K;
    A += (OPA == OP_N) ? (long)kb * lda : kb;
    B += (OPB == OP_N) ? kb : (long)kb * ldb;
    K = ke - kb;
  }

  // Each thread stages NL entries of each operand per K-tile: along the rows (64 per K column)
  // when the rows are contiguous in storage, along K (BK per row) when K is.
  constexpr int BK = CT<T>::bk(G3), NL = BK / 4, KR = NT / BK;
  v2 ra[NL], rb[NL];

// G: bounds tests needed (false only for interior tiles whose K is a multiple of BK, where
// every staged entry lies inside the operands; the loaded values are the same either way).
#define FEAST_LOAD_A(R, DST, G)                                                      \
  {                                                                                  \
    if (OPA == OP_N) {                                                               \
      int i = t & 63, k = (t >> 6) + 4 * (R);                                        \
      int gi = i0 + i, gk = k0 + k;                                                  \
      DST = ldc_<v2, false>(A + gi + (long)gk * lda, !(G) || (gi < M && gk < K));    \
    } else {                                                                         \
      int k = t % BK, i = t / BK + KR * (R);                                         \
      int gi = i0 + i, gk = k0 + k;                                                  \
      DST = ldc_<v2, OPA == OP_C>(A + gk + (long)gi * lda,                           \
                                  !(G) || (gi < M && gk < K));                       \
    }                                                                                \
  }
#define FEAST_LOAD_B(R, DST, G)                                                      \
  {                                                                                  \
    if (OPB == OP_N) {                                                               \
      int k = t % BK, j = t / BK + KR * (R);                                         \
      int gj = j0 + j, gk = k0 + k;                                                  \
      DST = ldc_<v2, false>(B + gk + (long)gj * ldb, !(G) || (gj < N && gk < K));    \
    } else {                                                                         \
      int j = t & 63, k = (t >> 6) + 4 * (R);                                        \
      int gj = j0 + j, gk = k0 + k;                                                  \
      DST = ldc_<v2, OPB == OP_C>(B + gj + (long)gk * ldb,                           \
                                  !(G) || (gj < N && gk < K));                       \
    }                                                                                \
  }
#define FEAST_LOAD_TILE_INTO(K0, RA, RB, G)                                          \
  {                                                                                  \
    const int k0 = (K0);                                                             \
    _Pragma("unroll") for (int r_ = 0; r_ < NL; ++r_) FEAST_LOAD_A(r_, RA[r_], G)     \
    _Pragma("unroll") for (int r_ = 0; r_ < NL; ++r_) FEAST_LOAD_B(r_, RB[r_], G)     \
  }
#define FEAST_STORE_AB(R, SA, SB)                                                    \
  {                                                                                  \
    if (OPA == OP_N) As[buf_][(t >> 6) + 4 * (R)][t & 63] = SA;                      \
    else As[buf_][t % BK][t / BK + KR * (R)] = SA;                                   \
    if (OPB == OP_N) Bs[buf_][t % BK][t / BK + KR * (R)] = SB;                       \
    else Bs[buf_][(t >> 6) + 4 * (R)][t & 63] = SB;                                  \
  }
#define FEAST_STORE_TILE_FROM(BUF, RA, RB)                                           \
  {                                                                                  \
    const int buf_ = (BUF);                                                          \
    _Pragma("unroll") for (int r_ = 0; r_ < NL; ++r_) FEAST_STORE_AB(r_, RA[r_], RB[r_]) \
  }
  // G3 (FP32): three real products per complex one (Gauss): p1 = re re, p2 = im im,
  // p3 = (re + im)(re + im); the epilogue forms re = p1 - p2, im = p3 - p1 - p2.
#define FEAST_COMPUTE(BUF, CHK)                                                       \
  if constexpr (G3) {                                                                 \
      const int buf = (BUF);                                                          \
      _Pragma("unroll") for (int kk = 0; kk < BK / 4; ++kk) {                         \
        const int kidx = kk * 4 + (lane >> 4);                                        \
        v2 fa[2], fb[2];                                                              \
        T sa[2], sb[2];                                                               \
        _Pragma("unroll") for (int mb = 0; mb < 2; ++mb) {                            \
          fa[mb] = As[buf][kidx][wm * 32 + mb * 16 + (lane & 15)];                    \
          sa[mb] = fa[mb].x + fa[mb].y;                                               \
        }                                                                             \
        _Pragma("unroll") for (int nb = 0; nb < 2; ++nb) {                            \
          fb[nb] = Bs[buf][kidx][wn * 32 + nb * 16 + (lane & 15)];                    \
          sb[nb] = fb[nb].x + fb[nb].y;                                               \
        }                                                                             \
        _Pragma("unroll") for (int mb = 0; mb < 2; ++mb)                              \
          _Pragma("unroll") for (int nb = 0; nb < 2; ++nb) {                          \
            if ((CHK) && !live[mb][nb]) continue;                                     \
            accr[mb][nb] = mfma(fb[nb].x, fa[mb].x, accr[mb][nb]);                    \
            acci[mb][nb] = mfma(fb[nb].y, fa[mb].y, acci[mb][nb]);                    \
          }                                                                           \
        _Pragma("unroll") for (int mb = 0; mb < 2; ++mb)                              \
          _Pragma("unroll") for (int nb = 0; nb < 2; ++nb) {                          \
            if ((CHK) && !live[mb][nb]) continue;                                     \
            accs[mb][nb] = mfma(sb[nb], sa[mb], accs[mb][nb]);                        \
          }                                                                           \
      }                                                                               \
  } else {                                                                            \
      const int buf = (BUF);                                                          \
      _Pragma("unroll") for (int kk = 0; kk < BK / 4; ++kk) {                         \
        const int kidx = kk * 4 + (lane >> 4);                                        \
        v2 fa[2], fb[2];                                                              \
        _Pragma("unroll") for (int mb = 0; mb < 2; ++mb)                              \
          fa[mb] = As[buf][kidx][wm * 32 + mb * 16 + (lane & 15)];                    \
        _Pragma("unroll") for (int nb = 0; nb < 2; ++nb)                              \
          fb[nb] = Bs[buf][kidx][wn * 32 + nb * 16 + (lane & 15)];                    \
        _Pragma("unroll") for (int mb = 0; mb < 2; ++mb)                              \
          _Pragma("unroll") for (int nb = 0; nb < 2; ++nb) {                          \
            if ((CHK) && !live[mb][nb]) continue;                                     \
            accr[mb][nb] = mfma(fb[nb].x, fa[mb].x, accr[mb][nb]);                    \
            acci[mb][nb] = mfma(fb[nb].x, fa[mb].y, acci[mb][nb]);                    \
          }                                                                           \
        _Pragma("unroll") for (int mb = 0; mb < 2; ++mb)                              \
          _Pragma("unroll") for (int nb = 0; nb < 2; ++nb) {                          \
            if ((CHK) && !live[mb][nb]) continue;                                     \
            accr[mb][nb] = mfma(-fb[nb].y, fa[mb].y, accr[mb][nb]);                   \
            acci[mb][nb] = mfma(fb[nb].y, fa[mb].x, acci[mb][nb]);                    \
          }                                                                           \
      }                                                                               \
  }
  accv accr[2][2], acci[2][2], accs[2][2];
  // A 16 x 16 output block that lies entirely past M or N has nothing to compute; the test
  // is uniform over the wave, so skipping its MFMAs frees the matrix core for other waves.
  bool live[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      accr[p][q] = accv{T(0), T(0), T(0), T(0)};
      acci[p][q] = accv{T(0), T(0), T(0), T(0)};
      accs[p][q] = accv{T(0), T(0), T(0), T(0)};
      live[p][q] = (i0 + wm * 32 + p * 16 < M) && (j0 + wn * 32 + q * 16 < N);
    }

  const int nkt = (K + BK - 1) / BK;
  const bool interior = i0 + BM <= M && j0 + BN <= N;
  // Loads of K-tile kt+1 are in flight while K-tile kt is multiplied; the other resident
  // workgroups cover the rest of their latency.
  if (nkt > 0) {
    FEAST_LOAD_TILE_INTO(0, ra, rb, true)
    FEAST_STORE_TILE_FROM(0, ra, rb)
  }
  __syncthreads();
#define FEAST_KLOOP(CHK, G)                                                          \
  for (int kt = 0; kt < nkt; ++kt) {                                                 \
    const int cur = kt & 1;                                                          \
    if (kt + 1 < nkt) FEAST_LOAD_TILE_INTO((kt + 1) * BK, ra, rb, G)                 \
    FEAST_COMPUTE(cur, CHK)                                                          \
    if (kt + 1 < nkt) FEAST_STORE_TILE_FROM(cur ^ 1, ra, rb)                         \
    __syncthreads();                                                                 \
  }
  // The branch is uniform over the workgroup (it depends on the tile origin and K only), so
  // every loop sees the same barriers; only ragged edge tiles pay for the per-block tests.
  if (interior && K % BK == 0) {
    FEAST_KLOOP(0, false)
  } else if (interior) {
    FEAST_KLOOP(0, true)
  } else {
    FEAST_KLOOP(1, true)
  }
#undef FEAST_KLOOP
#undef FEAST_LOAD_A
#undef FEAST_LOAD_B
#undef FEAST_LOAD_TILE_INTO
#undef FEAST_COMPUTE
#undef FEAST_STORE_AB
#undef FEAST_STORE_TILE_FROM

  const v2 alpha = a.alpha, beta = a.beta;
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
          if constexpr (G3) {
            const T p1 = re, p2 = im;
            re = p1 - p2;
            im = accs[mb][nb][v] - p1 - p2;
          }
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
}

template <typename T, int OPA0, int OPA1, int OPB, bool G3>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(CT<T>::waves(G3)))) void gemm_kernel(const Args<typename CT<T>::v2> a) {
  typedef typename CT<T>::v2 v2;
  __shared__ v2 As[2][CT<T>::bk(G3)][BM + PAD];
  __shared__ v2 Bs[2][CT<T>::bk(G3)][BN + PAD];
  // XCD-aware order: linear id L runs on XCD L % 8; each XCD gets a contiguous range.
  const long per = (long)a.tilesM * a.tilesN;
  const long total = (long)gridDim.x * gridDim.y * gridDim.z;
  const long L = blockIdx.x + (long)gridDim.x * (blockIdx.y + (long)gridDim.y * blockIdx.z);
  const int x = (int)(L & 7);
  long start = 0;
  for (int q = 0; q < x; ++q) start += (total - q + 7) / 8;
  const long g = start + (L >> 3);
  // lower triangular op(A): the longest K ranges (last tile rows) are handed out first
  const int tile = (a.tri == 1) ? (int)(per - 1 - g % per) : (int)(g % per);
  long rest = g / per;
  const int b1 = (int)(rest % a.n1);
  rest /= a.n1;
  const int b2 = (int)(rest % a.n2);
  const int prob = (int)(rest / a.n2);
  const int i0 = (tile / a.tilesN) * BM, j0 = (tile % a.tilesN) * BN;
  if constexpr (OPA0 == OPA1) {
    gemm_tile<T, OPA0, OPB, G3>(a, prob, b1, b2, i0, j0, As, Bs);
  } else {
    if (prob == 0) gemm_tile<T, OPA0, OPB, G3>(a, 0, b1, b2, i0, j0, As, Bs);
    else gemm_tile<T, OPA1, OPB, G3>(a, 1, b1, b2, i0, j0, As, Bs);
  }
}

template <typename T, int OPA0, int OPA1, int OPB>
void launch(hipStream_t s, const Args<typename CT<T>::v2>& a, int nprob) {
  dim3 grid(a.tilesM * a.tilesN, a.n1, a.n2 * nprob);
  if constexpr (sizeof(T) == 4) {
    hipLaunchKernelGGL((gemm_kernel<T, OPA0, OPA1, OPB, (bool)FEAST_GEMM_3M>), grid, dim3(NT), 0,
                       s, a);
  } else if (g_z3m) {
    hipLaunchKernelGGL((gemm_kernel<T, OPA0, OPA1, OPB, true>), grid, dim3(NT), 0, s, a);
  } else {
    hipLaunchKernelGGL((gemm_kernel<T, OPA0, OPA1, OPB, false>), grid, dim3(NT), 0, s, a);
  }
}

template <typename T>
void dispatch(hipStream_t s, const int* opA, int nprob, int opB,
              const Args<typename CT<T>::v2>& a) {
  GemmProfiler* prof = g_gemm_prof;
  const double flops = 8.0 * a.M * a.N * (double)(a.K > 0 ? a.K : 0) *
                       (a.splitk > 0 ? 1.0 : (double)a.n1) * a.n2 * nprob;
  const int o0 = opA[0], o1 = (nprob == 2) ? opA[1] : opA[0];
  bool done = false;
  if (prof) prof->begin(s);
#define FEAST_G(x, y, b)                                         \
  if (!done && o0 == x && o1 == y && opB == b) {                 \
    launch<T, x, y, b>(s, a, nprob);                             \
    done = true;                                                 \
  }
  FEAST_G(OP_N, OP_N, OP_N) FEAST_G(OP_N, OP_N, OP_T) FEAST_G(OP_N, OP_N, OP_C)
  FEAST_G(OP_T, OP_T, OP_N) FEAST_G(OP_T, OP_T, OP_T) FEAST_G(OP_T, OP_T, OP_C)
  FEAST_G(OP_C, OP_C, OP_N) FEAST_G(OP_C, OP_C, OP_T) FEAST_G(OP_C, OP_C, OP_C)
  FEAST_G(OP_N, OP_C, OP_N)
#undef FEAST_G
  if (!done) throw HipError{hipErrorInvalidValue, "gemm: unsupported op combination"};
  FEAST_LAUNCH_CHECK();
  if (prof) prof->end(s, flops);
}

// ---- bf16x3: FP32 complex operands split into bf16 hi + lo -------------------------------
// Each FP32 value x is stored as hi = bf16(x) and lo = bf16(x - hi) (round to nearest even);
// a real product is hi*hi + hi*lo + lo*hi (the lo*lo term, ~2^-16 relative, is dropped) on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  Per 32-deep step a 16x16 complex block
// takes 12 of these MFMAs: real part re*re - im*im and imaginary part re*im + im*re, each
// real product three-fold.  LDS holds four bf16 planes (re hi, re lo, im hi, im lo) per
// operand with the 32 k values of a row contiguous, in 16-byte chunks whose position is
// XOR-swizzled by (row >> 2) so that the 16 rows one MFMA operand read touches hit distinct
// banks.  Operand roles and the C^T epilogue are those of gemm_tile above; the MFMA result
// layout is the FP32 one (row 4 (l >> 4) + v).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int XBK = 32;

__device__ __forceinline__ unsigned bf16_rne_bits(float x) {  // finite x
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

// 8 consecutive-k complex values -> four 16-byte chunks (re hi, re lo, im hi, im lo).
__device__ __forceinline__ void split8(const float2 (&v)[8], uint4 (&o)[4]) {
  unsigned rh[8], rl[8], ih[8], il[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    unsigned h = bf16_rne_bits(v[e].x);
    rh[e] = h;
    rl[e] = bf16_rne_bits(v[e].x - __uint_as_float(h << 16));
    h = bf16_rne_bits(v[e].y);
    ih[e] = h;
    il[e] = bf16_rne_bits(v[e].y - __uint_as_float(h << 16));
  }
  o[0] = make_uint4(rh[0] | (rh[1] << 16), rh[2] | (rh[3] << 16), rh[4] | (rh[5] << 16),
                    rh[6] | (rh[7] << 16));
  o[1] = make_uint4(rl[0] | (rl[1] << 16), rl[2] | (rl[3] << 16), rl[4] | (rl[5] << 16),
                    rl[6] | (rl[7] << 16));
  o[2] = make_uint4(ih[0] | (ih[1] << 16), ih[2] | (ih[3] << 16), ih[4] | (ih[5] << 16),
                    ih[6] | (ih[7] << 16));
  o[3] = make_uint4(il[0] | (il[1] << 16), il[2] | (il[3] << 16), il[4] | (il[5] << 16),
                    il[6] | (il[7] << 16));
}

// LDS tile: [plane 4][row 64][chunk 4] of uint4 (8 bf16); chunk position swizzled by row.
__device__ __forceinline__ int xoff(int plane, int row, int chunk) {
  return (plane * 64 + row) * 4 + (chunk ^ ((row >> 2) & 3));
}

// One thread's share of an operand tile: 8 consecutive k values of one row (row = the M
// index of op(A) or the N index of op(B)); KCONTIG: k is the contiguous storage direction.
template <bool KCONTIG, bool CONJ>
__device__ __forceinline__ void xload(const float2* P, long ld, int row0, int k0, int nrow, int K,
                                      int t, float2 (&v)[8], int& row, int& chunk) {
  if (KCONTIG) {  // element (r, k) at P[k + r ld]: four threads cover the 32 k of a row
    row = t >> 2;
    chunk = t & 3;
  } else {        // element (r, k) at P[r + k ld]: lanes run along the rows
    row = t & 63;
    chunk = t >> 6;
  }
  const int gr = row0 + row;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int gk = k0 + chunk * 8 + e;
    float2 x = make_float2(0.f, 0.f);
    if (gr < nrow && gk < K) x = KCONTIG ? P[gk + (long)gr * ld] : P[gr + (long)gk * ld];
    if (CONJ) x.y = -x.y;
    v[e] = x;
  }
}

template <int OPA, int OPB>
__device__ __forceinline__ void gemmx_tile(const Args<float2>& a, int prob, int b1, int b2, int i0,
                                           int j0, uint4* As, uint4* Bs) {
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int M = a.M, N = a.N;
  int K = a.K;
  const long lda = a.lda[prob], ldb = a.ldb[prob], ldc = a.ldc[prob];
  const float2* A = a.A[prob] + b2 * a.sA2;
  const float2* B = a.B[prob] + b2 * a.sB2;
  float2* C = a.C[prob] + b1 * a.sC1 + b2 * a.sC2;
  if (a.splitk == 0) {
    A += b1 * a.sA1;
    B += b1 * a.sB1;
  } else {
    const long kb = (long)b1 * a.splitk;
    K = (K - kb < a.splitk) ? (int)(K - kb) : a.splitk;
    A += (OPA == OP_N) ? kb * lda : kb;
    B += (OPB == OP_N) ? kb : kb * ldb;
  }
  if (a.tri != 0) {  // op(A) triangular (square): only the K range of its nonzero part
    const int kb = (a.tri == 2) ? i0 : 0;
    const int ke = (a.tri == 1) ? min(K, i0 + BM) : K;
    A += (OPA == OP_N) ? (long)kb * lda : kb;
    B += (OPB == OP_N) ? kb : (long)kb * ldb;
    K = ke - kb;
  }
  constexpr bool AK = (OPA != OP_N), BK_ = (OPB == OP_N);  // k contiguous in storage
  constexpr int TILE = 4 * 64 * 4;                          // uint4 per operand tile

  f4 acc_rr[2][2], acc_ii[2][2], acc_im[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      acc_rr[p][q] = f4{0, 0, 0, 0};
      acc_ii[p][q] = f4{0, 0, 0, 0};
      acc_im[p][q] = f4{0, 0, 0, 0};
    }

  float2 pa[8], pb[8], qa[8], qb[8];
  int ra_row, ra_ch, rb_row, rb_ch;
#define FEAST_XLOAD(KT, VA, VB)                                                          \
  {                                                                                      \
    xload<AK, OPA == OP_C>(A, lda, i0, (KT) * XBK, M, K, t, VA, ra_row, ra_ch);          \
    xload<BK_, OPB == OP_C>(B, ldb, j0, (KT) * XBK, N, K, t, VB, rb_row, rb_ch);         \
  }
#define FEAST_XSTORE(BUF, VA, VB)                                                        \
  {                                                                                      \
    uint4 oa[4], ob[4];                                                                  \
    split8(VA, oa);                                                                      \
    split8(VB, ob);                                                                      \
    uint4* sa = As + (BUF) * TILE;                                                       \
    uint4* sb = Bs + (BUF) * TILE;                                                       \
    _Pragma("unroll") for (int pl = 0; pl < 4; ++pl) {                                   \
      sa[xoff(pl, ra_row, ra_ch)] = oa[pl];                                              \
      sb[xoff(pl, rb_row, rb_ch)] = ob[pl];                                              \
    }                                                                                    \
  }
#define FEAST_XCOMPUTE(BUF)                                                              \
  {                                                                                      \
    const uint4* sa = As + (BUF) * TILE;                                                 \
    const uint4* sb = Bs + (BUF) * TILE;                                                 \
    const int ch = lane >> 4;                                                            \
    bf16x8 fa[2][4], fb[2][4];                                                           \
    _Pragma("unroll") for (int q = 0; q < 2; ++q)                                        \
      _Pragma("unroll") for (int pl = 0; pl < 4; ++pl) {                                 \
        uint4 x = sa[xoff(pl, wm * 32 + q * 16 + (lane & 15), ch)];                      \
        uint4 y = sb[xoff(pl, wn * 32 + q * 16 + (lane & 15), ch)];                      \
        fa[q][pl] = __builtin_bit_cast(bf16x8, x);                                       \
        fb[q][pl] = __builtin_bit_cast(bf16x8, y);                                       \
      }                                                                                  \
    _Pragma("unroll") for (int mb = 0; mb < 2; ++mb)                                     \
      _Pragma("unroll") for (int nb = 0; nb < 2; ++nb) {                                 \
        f4 rr = acc_rr[mb][nb], ii = acc_ii[mb][nb], im = acc_im[mb][nb];                \
        rr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[nb][0], fa[mb][0], rr, 0, 0, 0); \
        ii = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[nb][2], fa[mb][2], ii, 0, 0, 0); \
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[nb][2], fa[mb][0], im, 0, 0, 0); \
        rr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[nb][0], fa[mb][1], rr, 0, 0, 0); \
        ii = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[nb][2], fa[mb][3], ii, 0, 0, 0); \
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[nb][2], fa[mb][1], im, 0, 0, 0); \
        rr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[nb][1], fa[mb][0], rr, 0, 0, 0); \
        ii = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[nb][3], fa[mb][2], ii, 0, 0, 0); \
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[nb][3], fa[mb][0], im, 0, 0, 0); \
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[nb][0], fa[mb][2], im, 0, 0, 0); \
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[nb][0], fa[mb][3], im, 0, 0, 0); \
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[nb][1], fa[mb][2], im, 0, 0, 0); \
        acc_rr[mb][nb] = rr;                                                             \
        acc_ii[mb][nb] = ii;                                                             \
        acc_im[mb][nb] = im;                                                             \
      }                                                                                  \
  }

  // prefetch distance two: the loads of K-tile kt+2 are in flight while kt is multiplied
  const int nkt = (K + XBK - 1) / XBK;
  if (nkt > 0) {
    FEAST_XLOAD(0, pa, pb)
    FEAST_XSTORE(0, pa, pb)
  }
  if (nkt > 1) FEAST_XLOAD(1, qa, qb)
  __syncthreads();
  for (int kt = 0; kt < nkt; kt += 2) {
    if (kt + 2 < nkt) FEAST_XLOAD(kt + 2, pa, pb)
    FEAST_XCOMPUTE(0)
    if (kt + 1 < nkt) FEAST_XSTORE(1, qa, qb)
    __syncthreads();
    if (kt + 1 >= nkt) break;
    if (kt + 3 < nkt) FEAST_XLOAD(kt + 3, qa, qb)
    FEAST_XCOMPUTE(1)
    if (kt + 2 < nkt) FEAST_XSTORE(0, pa, pb)
    __syncthreads();
  }
#undef FEAST_XLOAD
#undef FEAST_XSTORE
#undef FEAST_XCOMPUTE

  const float2 alpha = a.alpha, beta = a.beta;
  const bool beta_zero = (beta.x == 0.f && beta.y == 0.f);
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int i = i0 + wm * 32 + mb * 16 + (lane & 15);
        int j = j0 + wn * 32 + nb * 16 + 4 * (lane >> 4) + v;
        if (i < M && j < N) {
          float re = acc_rr[mb][nb][v] - acc_ii[mb][nb][v], im = acc_im[mb][nb][v];
          float2 out;
          out.x = alpha.x * re - alpha.y * im;
          out.y = alpha.x * im + alpha.y * re;
          if (!beta_zero) {
            float2 c = C[i + (long)j * ldc];
            out.x += beta.x * c.x - beta.y * c.y;
            out.y += beta.x * c.y + beta.y * c.x;
          }
          C[i + (long)j * ldc] = out;
        }
      }
}

template <int OPA0, int OPA1, int OPB>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void gemmx_kernel(
    const Args<float2> a) {
  __shared__ uint4 As[2 * 4 * 64 * 4];
  __shared__ uint4 Bs[2 * 4 * 64 * 4];
  const long per = (long)a.tilesM * a.tilesN;
  const long total = (long)gridDim.x * gridDim.y * gridDim.z;
  const long L = blockIdx.x + (long)gridDim.x * (blockIdx.y + (long)gridDim.y * blockIdx.z);
  const int x = (int)(L & 7);
  long start = 0;
  for (int q = 0; q < x; ++q) start += (total - q + 7) / 8;
  const long g = start + (L >> 3);
  // lower triangular op(A): the longest K ranges (last tile rows) are handed out first
  const int tile = (a.tri == 1) ? (int)(per - 1 - g % per) : (int)(g % per);
  long rest = g / per;
  const int b1 = (int)(rest % a.n1);
  rest /= a.n1;
  const int b2 = (int)(rest % a.n2);
  const int prob = (int)(rest / a.n2);
  const int i0 = (tile / a.tilesN) * BM, j0 = (tile % a.tilesN) * BN;
  if constexpr (OPA0 == OPA1) {
    gemmx_tile<OPA0, OPB>(a, prob, b1, b2, i0, j0, As, Bs);
  } else {
    if (prob == 0) gemmx_tile<OPA0, OPB>(a, 0, b1, b2, i0, j0, As, Bs);
    else gemmx_tile<OPA1, OPB>(a, 1, b1, b2, i0, j0, As, Bs);
  }
}

void dispatchx(hipStream_t s, const int* opA, int nprob, int opB, const Args<float2>& a) {
  GemmProfiler* prof = g_gemm_prof;
  const double flops = 8.0 * a.M * a.N * (double)(a.K > 0 ? a.K : 0) *
                       (a.splitk > 0 ? 1.0 : (double)a.n1) * a.n2 * nprob;
  const int o0 = opA[0], o1 = (nprob == 2) ? opA[1] : opA[0];
  bool done = false;
  dim3 grid(a.tilesM * a.tilesN, a.n1, a.n2 * nprob);
  if (prof) prof->begin(s);
#define FEAST_GX(x, y, b)                                                         \
  if (!done && o0 == x && o1 == y && opB == b) {                                  \
    hipLaunchKernelGGL((gemmx_kernel<x, y, b>), grid, dim3(NT), 0, s, a);         \
    done = true;                                                                  \
  }
  FEAST_GX(OP_N, OP_N, OP_N) FEAST_GX(OP_N, OP_N, OP_T) FEAST_GX(OP_N, OP_N, OP_C)
  FEAST_GX(OP_T, OP_T, OP_N) FEAST_GX(OP_T, OP_T, OP_T) FEAST_GX(OP_T, OP_T, OP_C)
  FEAST_GX(OP_C, OP_C, OP_N) FEAST_GX(OP_C, OP_C, OP_T) FEAST_GX(OP_C, OP_C, OP_C)
  FEAST_GX(OP_N, OP_C, OP_N)
#undef FEAST_GX
  if (!done) throw HipError{hipErrorInvalidValue, "gemm bf16x3: unsupported op combination"};
  FEAST_LAUNCH_CHECK();
  if (prof) prof->end(s, flops);
}

template <typename v2>
Args<v2> make_args(int M, int N, int K, v2 alpha, v2 beta, const Batch& bt) {
  if (bt.tri < 0 || bt.tri > 2 || (bt.tri != 0 && (M != K || bt.splitk != 0)))
    throw HipError{hipErrorInvalidValue, "gemm: a triangular op(A) must be square, no split-K"};
  Args<v2> a;
  a.M = M;
  a.N = N;
  a.K = K;
  a.tilesM = (M + BM - 1) / BM;
  a.tilesN = (N + BN - 1) / BN;
  a.n1 = bt.n1;
  a.n2 = bt.n2;
  a.splitk = bt.splitk;
  a.tri = bt.tri;
  a.alpha = alpha;
  a.beta = beta;
  a.sA1 = bt.sA1;
  a.sA2 = bt.sA2;
  a.sB1 = bt.sB1;
  a.sB2 = bt.sB2;
  a.sC1 = bt.sC1;
  a.sC2 = bt.sC2;
  return a;
}

template <typename T>
void gemm1(hipStream_t s, int opA, int opB, int M, int N, int K, typename CT<T>::v2 alpha,
           const typename CT<T>::v2* A, long lda, const typename CT<T>::v2* B, long ldb,
           typename CT<T>::v2 beta, typename CT<T>::v2* C, long ldc, const Batch& bt) {
  if (M <= 0 || N <= 0 || bt.n1 <= 0 || bt.n2 <= 0) return;
  auto a = make_args(M, N, K, alpha, beta, bt);
  a.A[0] = a.A[1] = A;
  a.B[0] = a.B[1] = B;
  a.C[0] = a.C[1] = C;
  a.lda[0] = a.lda[1] = lda;
  a.ldb[0] = a.ldb[1] = ldb;
  a.ldc[0] = a.ldc[1] = ldc;
  int ops[1] = {opA};
  if constexpr (sizeof(T) == 4) {
    if (g_split_bf16) {
      dispatchx(s, ops, 1, opB, a);
      return;
    }
  }
  dispatch<T>(s, ops, 1, opB, a);
}

template <typename T>
void gemm2(hipStream_t s, int opA0, int opA1, int opB, int M, int N, int K,
           typename CT<T>::v2 alpha, const typename CT<T>::v2* const A[2], const long lda[2],
           const typename CT<T>::v2* const B[2], const long ldb[2], typename CT<T>::v2 beta,
           typename CT<T>::v2* const C[2], const long ldc[2], const Batch& bt) {
  if (M <= 0 || N <= 0 || bt.n1 <= 0 || bt.n2 <= 0) return;
  auto a = make_args(M, N, K, alpha, beta, bt);
  for (int p = 0; p < 2; ++p) {
    a.A[p] = A[p];
    a.B[p] = B[p];
    a.C[p] = C[p];
    a.lda[p] = lda[p];
    a.ldb[p] = ldb[p];
    a.ldc[p] = ldc[p];
  }
  int ops[2] = {opA0, opA1};
  if constexpr (sizeof(T) == 4) {
    if (g_split_bf16) {
      dispatchx(s, ops, 2, opB, a);
      return;
    }
  }
  dispatch<T>(s, ops, 2, opB, a);
}

}  // namespace

void zgemm(hipStream_t s, int opA, int opB, int M, int N, int K, zd alpha, const zd* A, long lda,
           const zd* B, long ldb, zd beta, zd* C, long ldc, const Batch& bt) {
  gemm1<double>(s, opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
}
void cgemm(hipStream_t s, int opA, int opB, int M, int N, int K, zf alpha, const zf* A, long lda,
           const zf* B, long ldb, zf beta, zf* C, long ldc, const Batch& bt) {
  gemm1<float>(s, opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
}
namespace {
__global__ __launch_bounds__(256) void sum_partials_kernel(const zd* part, int nparts, int M,
                                                           long len, zd* C, long ldc) {
  const long i = blockIdx.x * 256L + threadIdx.x;
  if (i >= len) return;
  zd acc = part[i];
  for (int p = 1; p < nparts; ++p) acc = zadd(acc, part[(long)p * len + i]);
  C[(i % M) + (i / M) * ldc] = acc;
}

// Workgroups of the FP64 op(N, N) GEMM kernel resident on the current device at once, for
// the product form that runs (g3: three real products, which holds fewer per CU).
int zgemm_resident_tiles(bool g3) {
  static std::atomic<int> cache[64][2];
  int dev = 0;
  FEAST_HIP(hipGetDevice(&dev));
  std::atomic<int>* c = (dev >= 0 && dev < 64) ? &cache[dev][g3 ? 1 : 0] : nullptr;
  if (c && c->load() > 0) return c->load();
  int cus = 0, per_cu = 0;
  FEAST_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const void* k = g3 ? reinterpret_cast<const void*>(&gemm_kernel<double, OP_N, OP_N, OP_N, true>)
                     : reinterpret_cast<const void*>(&gemm_kernel<double, OP_N, OP_N, OP_N, false>);
  FEAST_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, NT, 0));
  const int r = std::max(1, cus * std::max(1, per_cu));
  if (c) c->store(r);
  return r;
}
}  // namespace

int zgemm_kchunks(int M, int N, int K) {
  if (M <= 0 || N <= 0 || K < 512) return 1;
  const long tiles = (long)((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  const long slots = zgemm_resident_tiles(g_z3m);
  // Cost model: rounds of resident workgroups times the K length each one runs.  A split
  // is taken only when it saves at least 3 % (the partial sums cost a pass over C).
  int best = 1;
  double best_cost = (double)((tiles + slots - 1) / slots) * K;
  for (int nk = 2; nk <= 8; ++nk) {
    const int chunk = (K + nk - 1) / nk;
    if (chunk < 256) break;
    const double cost = (double)((tiles * nk + slots - 1) / slots) * chunk;
    if (cost < 0.97 * best_cost) {
      best = nk;
      best_cost = cost;
    }
  }
  return best;
}

void zgemm_nn_split(hipStream_t s, int M, int N, int K, const zd* A, long lda, const zd* B,
                    long ldb, zd* C, long ldc, int nchunk, zd* part) {
  const zd one = zmake(1, 0), zero = zmake(0, 0);
  if (nchunk <= 1) {
    zgemm(s, OP_N, OP_N, M, N, K, one, A, lda, B, ldb, zero, C, ldc);
    return;
  }
  if (M <= 0 || N <= 0) return;
  Batch b;
  b.n1 = nchunk;
  b.splitk = (K + nchunk - 1) / nchunk;
  b.sC1 = (long)M * N;
  zgemm(s, OP_N, OP_N, M, N, K, one, A, lda, B, ldb, zero, part, M, b);
  const long len = (long)M * N;
  hipLaunchKernelGGL(sum_partials_kernel, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s,
                     part, nchunk, M, len, C, ldc);
  FEAST_LAUNCH_CHECK();
}

void zgemm_pair(hipStream_t s, int opA0, int opA1, int opB, int M, int N, int K, zd alpha,
                const zd* const A[2], const long lda[2], const zd* const B[2], const long ldb[2],
                zd beta, zd* const C[2], const long ldc[2], const Batch& bt) {
  gemm2<double>(s, opA0, opA1, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
}
void cgemm_pair(hipStream_t s, int opA0, int opA1, int opB, int M, int N, int K, zf alpha,
                const zf* const A[2], const long lda[2], const zf* const B[2], const long ldb[2],
                zf beta, zf* const C[2], const long ldc[2], const Batch& bt) {
  gemm2<float>(s, opA0, opA1, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bt);
}

}  // namespace feast
