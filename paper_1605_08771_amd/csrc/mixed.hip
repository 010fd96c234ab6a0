// Mixed-precision filter application: FP32 complex factors and triangular sweeps on the FP32
// matrix cores, FP64 residuals, updates and accumulation (precision is not discussed by the
// paper; the filter is its Sec. 1 eq. contour_int_quad).
//
// Two ways to reach FP64 accuracy from FP32 solves:
//  * classic iterative refinement: Y <- Y + M^{-1}(X - M Y) with X - M Y = X - z Y + A Y
//    formed in FP64 (one FP64 product of A with all n_c * sides solution blocks per step);
//  * Ritz-seeded correction (inside the FEAST loop, iteration >= 2): X holds Ritz vectors
//    with Ritz values Lambda and FP64 residual R = A X - X Lambda from the last
//    Rayleigh-Ritz step.  Y0 = X (z - Lambda)^{-1} has residual X - M Y0 = R (z - Lambda)^{-1}
//    exactly, so Y = Y0 + M^{-1}[R (z - Lambda)^{-1}] needs no product with A, and summing
//    the quadrature gives Q = X diag(rho(Lambda)) + sum_j (omega_j D_j + conj(omega_j) D'_j):
//    the FP64 scalar filter of the Ritz values plus FP32-solved corrections whose size is the
//    current FEAST residual.
#include "common.h"
#include "kernels.h"

namespace feast {

namespace {

inline dim3 grid1(long n) { return dim3((unsigned)((n + 255) / 256)); }

// B[j][s][r, c] = (R[src, c] / (zz - lam_c)) in FP32, src = perm_j[r] (side 0) or r (side 1),
// zz = z_j (side 0) or conj(z_j) (side 1).
__global__ void seeded_rhs_kernel(const zd* __restrict__ R, long ldr, const double* __restrict__ lam,
                                  const zd* __restrict__ z, const int* __restrict__ perm, int n,
                                  int np, int m0, int nc, int sides, zf* __restrict__ B) {
  long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  long per = (long)np * m0;
  if (idx >= per * nc * sides) return;
  long blk = idx / per, e = idx % per;
  int node = (int)(blk / sides), side = (int)(blk % sides);
  int r = (int)(e % np), c = (int)(e / np);
  zf out = make_float2(0.f, 0.f);
  if (r < n) {
    int src = (side == 0) ? perm[(long)node * np + r] : r;
    if (src < n) {
      zd zz = z[node];
      if (side == 1) zz.y = -zz.y;
      zd d = zmake(zz.x - lam[c], zz.y);
      zd v = zdiv(R[src + (long)c * ldr], d);
      out = make_float2((float)v.x, (float)v.y);
    }
  }
  B[idx] = out;
}

// rho[c] = sum_j 2 Re(omega_j / (z_j - lam_c)), the quadrature filter at the Ritz values.
__global__ void rho_kernel(const double* lam, const zd* z, const zd* omega, int nc, int m0,
                           double* rho) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m0) return;
  double s = 0;
  for (int j = 0; j < nc; ++j) {
    zd q = zdiv(omega[j], zmake(z[j].x - lam[c], z[j].y));
    s += 2.0 * q.x;
  }
  rho[c] = s;
}

// Q = X diag(rho) (if X) + sum_j omega_j D0_j + conj(omega_j) P_j^T D1_j (sides 2) or
// + sum_j 2 Re(omega_j D0_j) (sides 1); D in FP32, accumulation in FP64.
__global__ void accumulate_mixed_kernel(const zd* __restrict__ X, long ldx,
                                        const double* __restrict__ rho, const zf* __restrict__ D,
                                        int n, int np, int m0, int nc, int sides,
                                        const zd* __restrict__ omega, const int* __restrict__ pinv,
                                        zd* __restrict__ Q, long ldq) {
  long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)n * m0) return;
  int i = (int)(idx % n), c = (int)(idx / n);
  long per = (long)np * m0;
  double re = 0, im = 0;
  if (X) {
    zd x = X[i + (long)c * ldx];
    re = x.x * rho[c];
    im = x.y * rho[c];
  }
  for (int j = 0; j < nc; ++j) {
    zd w = omega[j];
    const zf* d0 = D + (long)j * sides * per;
    zf a = d0[i + (long)c * np];
    if (sides == 2) {
      zf b = d0[per + pinv[(long)j * np + i] + (long)c * np];
      re += w.x * a.x - w.y * a.y + w.x * b.x + w.y * b.y;
      im += w.x * a.y + w.y * a.x + w.x * b.y - w.y * b.x;
    } else {
      re += 2.0 * (w.x * a.x - w.y * a.y);
    }
  }
  Q[i + (long)c * ldq] = zmake(re, im);
}

// Y64[j][s][i, c] (=, or += when add) D32[j][s][i', c], i' = pinv_j[i] for side 1 else i.
__global__ void unpermute_kernel(const zf* __restrict__ D, const int* __restrict__ pinv, int n,
                                 int np, int m0, int nc, int sides, int add, zd* __restrict__ Y) {
  long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  long per = (long)np * m0;
  if (idx >= per * nc * sides) return;
  long blk = idx / per, e = idx % per;
  int node = (int)(blk / sides), side = (int)(blk % sides);
  int i = (int)(e % np), c = (int)(e / np);
  zd v = zmake(0, 0);
  if (i < n) {
    int src = (side == 1) ? pinv[(long)node * np + i] : i;
    zf d = D[blk * per + src + (long)c * np];
    v = zmake(d.x, d.y);
  }
  if (add) {
    zd y = Y[idx];
    v = zadd(y, v);
  }
  Y[idx] = v;
}

// B32[j][s][r, c] = R[src, c] with R = X - zz Y + AY (FP64) at row src = perm_j[r] (side 0)
// or r (side 1).  Y, AY: [nc][sides] blocks of np x m0 in original row order.
// rmax (optional): the largest |R| entry over all systems, accumulated as the bit pattern of
// a non-negative double (whose unsigned order is its numeric order); zeroed by the caller.
__global__ __launch_bounds__(256) void refine_rhs_kernel(
    const zd* __restrict__ X, long ldx, const zd* __restrict__ Y, const zd* __restrict__ AY,
    const zd* __restrict__ z, const int* __restrict__ perm, int n, int np, int m0, int nc,
    int sides, zf* __restrict__ B, unsigned long long* rmax) {
  __shared__ double sm[256];
  long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  long per = (long)np * m0;
  double mag = 0.0;
  if (idx < per * nc * sides) {
    long blk = idx / per, e = idx % per;
    int node = (int)(blk / sides), side = (int)(blk % sides);
    int r = (int)(e % np), c = (int)(e / np);
    zf out = make_float2(0.f, 0.f);
    if (r < n) {
      int src = (side == 0) ? perm[(long)node * np + r] : r;
      if (src < n) {
        zd zz = z[node];
        if (side == 1) zz.y = -zz.y;
        long o = blk * per + src + (long)c * np;
        zd y = Y[o];
        zd v = zadd(zsub(X[src + (long)c * ldx], zmul(zz, y)), AY[o]);
        out = make_float2((float)v.x, (float)v.y);
        mag = sqrt(v.x * v.x + v.y * v.y);
        if (!(mag <= 1.79e308)) mag = 1.79e308;  // non-finite: largest finite value
      }
    }
    B[idx] = out;
  }
  if (!rmax) return;  // uniform over the grid
  sm[threadIdx.x] = mag;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(rmax, (unsigned long long)__double_as_longlong(sm[0]));
}

__global__ void zero_u64_kernel(unsigned long long* p) { p[0] = 0ull; }

// Q = sum_j omega_j Y0_j + conj(omega_j) Y1_j (both in original row order), or 2 Re(.)
__global__ void accumulate_plain_kernel(const zd* __restrict__ Y, int n, int np, int m0, int nc,
                                        int sides, const zd* __restrict__ omega,
                                        zd* __restrict__ Q, long ldq) {
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
      zd b = y0[per + i + (long)c * np];
      re += w.x * a.x - w.y * a.y + w.x * b.x + w.y * b.y;
      im += w.x * a.y + w.y * a.x + w.x * b.y - w.y * b.x;
    } else {
      re += 2.0 * (w.x * a.x - w.y * a.y);
    }
  }
  Q[i + (long)c * ldq] = zmake(re, im);
}

}  // namespace

void seeded_rhs(hipStream_t s, const zd* R, long ldr, const double* lam, const zd* z,
                const int* perm, int n, int np, int m0, int nc, int sides, zf* B) {
  long tot = (long)np * m0 * nc * sides;
  hipLaunchKernelGGL(seeded_rhs_kernel, grid1(tot), dim3(256), 0, s, R, ldr, lam, z, perm, n, np,
                     m0, nc, sides, B);
  FEAST_LAUNCH_CHECK();
}

void filter_values(hipStream_t s, const double* lam, const zd* z, const zd* omega, int nc, int m0,
                   double* rho) {
  hipLaunchKernelGGL(rho_kernel, grid1(m0), dim3(256), 0, s, lam, z, omega, nc, m0, rho);
  FEAST_LAUNCH_CHECK();
}

void accumulate_mixed(hipStream_t s, const zd* X, long ldx, const double* rho, const zf* D, int n,
                      int np, int m0, int nc, int sides, const zd* omega, const int* pinv, zd* Q,
                      long ldq) {
  hipLaunchKernelGGL(accumulate_mixed_kernel, grid1((long)n * m0), dim3(256), 0, s, X, ldx, rho, D,
                     n, np, m0, nc, sides, omega, pinv, Q, ldq);
  FEAST_LAUNCH_CHECK();
}

void unpermute_to64(hipStream_t s, const zf* D, const int* pinv, int n, int np, int m0, int nc,
                    int sides, int add, zd* Y) {
  long tot = (long)np * m0 * nc * sides;
  hipLaunchKernelGGL(unpermute_kernel, grid1(tot), dim3(256), 0, s, D, pinv, n, np, m0, nc, sides,
                     add, Y);
  FEAST_LAUNCH_CHECK();
}

void refine_rhs(hipStream_t s, const zd* X, long ldx, const zd* Y, const zd* AY, const zd* z,
                const int* perm, int n, int np, int m0, int nc, int sides, zf* B,
                unsigned long long* rmax) {
  long tot = (long)np * m0 * nc * sides;
  if (rmax) {
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, s, rmax);
    FEAST_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(refine_rhs_kernel, grid1(tot), dim3(256), 0, s, X, ldx, Y, AY, z, perm, n, np,
                     m0, nc, sides, B, rmax);
  FEAST_LAUNCH_CHECK();
}

void accumulate_plain(hipStream_t s, const zd* Y, int n, int np, int m0, int nc, int sides,
                      const zd* omega, zd* Q, long ldq) {
  hipLaunchKernelGGL(accumulate_plain_kernel, grid1((long)n * m0), dim3(256), 0, s, Y, n, np, m0, nc,
                     sides, omega, Q, ldq);
  FEAST_LAUNCH_CHECK();
}

}  // namespace feast
