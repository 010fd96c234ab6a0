// Kernels of the expanded-subspace variants (Sec. 2, Method 1 "XFEAST" and Method 2
// "RFEAST"): unit scaling of the basis columns, the truncated Gram basis T = V_keep S^{-1}
// of the orthogonalization by the Gram matrix, and gathers of the selected Ritz pairs.
#include "common.h"
#include "kernels.h"

namespace feast {

namespace {

inline dim3 grid1(long n) { return dim3((unsigned)((n + 255) / 256)); }

// One workgroup per column: B[:, k] /= ||B[:, k]||_2 (a zero column stays zero).
__global__ __launch_bounds__(256) void normalize_columns_kernel(zd* __restrict__ B, long ldb,
                                                                int n) {
  __shared__ double sh[256];
  zd* col = B + (long)blockIdx.x * ldb;
  double s = 0;
  for (int i = threadIdx.x; i < n; i += 256) {
    zd v = col[i];
    s += v.x * v.x + v.y * v.y;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double nrm = sqrt(sh[0]);
  const double sc = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    zd v = col[i];
    col[i] = zmake(v.x * sc, v.y * sc);
  }
}

// T[:, j] = V[:, keep[j]] / sqrt(d[keep[j]])  (T: k x r, ld k; V: ld ldv).
__global__ void gram_basis_kernel(const double* __restrict__ d, const zd* __restrict__ V, long ldv,
                                  const int* __restrict__ keep, int k, int r, zd* __restrict__ T) {
  long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)k * r) return;
  int i = (int)(idx % k), j = (int)(idx / k);
  int src = keep[j];
  double sc = 1.0 / sqrt(d[src]);
  zd v = V[i + (long)src * ldv];
  T[idx] = zmake(v.x * sc, v.y * sc);
}

// dst[:, a] = src[:, idx[a]], a < cnt (rows < n).
__global__ void gather_columns_kernel(const zd* __restrict__ src, long lds,
                                      const int* __restrict__ idx, int n, int cnt,
                                      zd* __restrict__ dst, long ldd) {
  long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)n * cnt) return;
  int i = (int)(e % n), a = (int)(e / n);
  dst[i + (long)a * ldd] = src[i + (long)idx[a] * lds];
}

__global__ void gather_values_kernel(const double* __restrict__ src, const int* __restrict__ idx,
                                     int cnt, double* __restrict__ dst) {
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a < cnt) dst[a] = src[idx[a]];
}

}  // namespace

void normalize_columns(hipStream_t s, zd* B, long ldb, int n, int k) {
  if (k <= 0 || n <= 0) return;
  hipLaunchKernelGGL(normalize_columns_kernel, dim3(k), dim3(256), 0, s, B, ldb, n);
  FEAST_LAUNCH_CHECK();
}

void gram_basis(hipStream_t s, const double* d, const zd* V, long ldv, const int* keep, int k,
                int r, zd* T) {
  if (k <= 0 || r <= 0) return;
  hipLaunchKernelGGL(gram_basis_kernel, grid1((long)k * r), dim3(256), 0, s, d, V, ldv, keep, k, r,
                     T);
  FEAST_LAUNCH_CHECK();
}

void gather_columns(hipStream_t s, const zd* src, long lds, const int* idx, int n, int cnt, zd* dst,
                    long ldd) {
  if (cnt <= 0 || n <= 0) return;
  hipLaunchKernelGGL(gather_columns_kernel, grid1((long)n * cnt), dim3(256), 0, s, src, lds, idx, n,
                     cnt, dst, ldd);
  FEAST_LAUNCH_CHECK();
}

void gather_values(hipStream_t s, const double* src, const int* idx, int cnt, double* dst) {
  if (cnt <= 0) return;
  hipLaunchKernelGGL(gather_values_kernel, grid1(cnt), dim3(256), 0, s, src, idx, cnt, dst);
  FEAST_LAUNCH_CHECK();
}

}  // namespace feast
