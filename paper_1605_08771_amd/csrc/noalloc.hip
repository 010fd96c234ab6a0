// Filter application that allocates no device memory: the FP64 path of feast_filter_apply
// (shifted factorizations, inverted diagonal blocks, paired block sweeps, weighted
// accumulation; Sec. 1 eq. contour_int_quad) with every intermediate carved from one
// file-scope device array instead of handle workspace.  For callers that cannot call
// hipMalloc (code under graph capture, tight serving loops, harnesses that forbid it).
//
// The array is a device symbol: each GPU holds its own copy, at its own address, from the
// time the library's code object is loaded on it until the process ends.  Host code never
// passes the symbol's name to a kernel (in host code it is a host-side stand-in); the device
// address is looked up once per device with hipGetSymbolAddress and kept.  Every call on a
// GPU shares that GPU's array, so calls that overlap on one GPU (several streams or host
// threads) race; the array keeps the last call's contents, and everything that must start at
// zero is cleared by the call itself.
#include <cmath>
#include <mutex>
#include <vector>

#include "../../include/feast.h"
#include "../../include/feast_noalloc.h"
#include "common.h"
#include "kernels.h"

using namespace feast;

namespace {

constexpr size_t kScratchBytes = (size_t)FEAST_NOALLOC_SCRATCH_MB << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // device address of `scratch`, by device ordinal

// Device address of the current device's scratch array (looked up on the first call on
// that device, with that device current).
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Bump carving of the scratch array at 256-byte alignment; `used` ends as the total (with
// base 0 it only measures the layout).
struct Carve {
  uintptr_t base;
  size_t used = 0;
  template <typename T>
  T* take(size_t count) {
    T* p = (T*)(base + used);
    used += (count * sizeof(T) + 255) & ~(size_t)255;
    return p;
  }
};

// Up to 64 complex values by value (a 1 KiB kernel argument), stored to device memory.
struct Values64 {
  zd v[64];
};
__global__ void store_values_kernel(Values64 vals, int count, zd* dst) {
  const int t = threadIdx.x;
  if (t < count) dst[t] = vals.v[t];
}

void store_values(hipStream_t s, const zd* host, int count, zd* dst) {
  for (int off = 0; off < count; off += 64) {
    Values64 v;
    const int c = std::min(64, count - off);
    for (int i = 0; i < c; ++i) v.v[i] = host[off + i];
    hipLaunchKernelGGL(store_values_kernel, dim3(1), dim3(64), 0, s, v, c, dst + off);
    FEAST_LAUNCH_CHECK();
  }
}

int read_flag(hipStream_t s, const int* dflag) {
  int h = 0;
  FEAST_HIP(hipMemcpyAsync(&h, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
  FEAST_HIP(hipStreamSynchronize(s));
  return h;
}

}  // namespace

extern "C" int feast_filter_apply_noalloc(feast_dtype dt, int n, const void* A, int lda,
                                          double emin, double emax, int n_c, const void* X,
                                          int ldx, int m0, void* Q, int ldq, void* hip_stream) {
  if (dt != FEAST_R64 && dt != FEAST_C128) return -1;
  if (n < 1) return -2;
  if (!A) return -3;
  if (lda < n) return -4;
  if (!std::isfinite(emin)) return -5;
  if (!std::isfinite(emax) || !(emin < emax)) return -6;
  if (n_c < 1 || n_c > 128) return -7;
  if (!X) return -8;
  if (ldx < n) return -9;
  if (m0 < 1 || m0 > n) return -10;
  if (!Q || Q == X) return -11;
  if (ldq < n) return -12;
  const int sides = (dt == FEAST_C128) ? 2 : 1;
  const int nbt = sweep_block(n, 0);
  const int np = (n + nbt - 1) / nbt * nbt;
  // Layout (and size check) before any device work.
  Carve cv{0};
  cv.take<zd>(n_c);                                  // z
  cv.take<zd>(n_c);                                  // omega
  cv.take<char>(lu_work_bytes(np, n_c));             // LU workspace
  cv.take<zd>((size_t)n_c * np * np);                // factors
  cv.take<zd>((size_t)n_c * np * nbt);               // inverted diagonal blocks of L
  cv.take<zd>((size_t)n_c * np * nbt);               // ... and of U
  cv.take<zd>((size_t)np * nbt);                     // inversion temporary
  cv.take<zd>((size_t)n_c * sides * np * m0);        // right-hand sides / solutions
  cv.take<zd>((size_t)n_c * sides * np * m0);        // sweep intermediate
  if (dt == FEAST_R64) {
    cv.take<zd>((size_t)n * m0);                     // complex copy of X
    cv.take<zd>((size_t)n * m0);                     // complex Q
  }
  if (cv.used > kScratchBytes) return FEAST_ERR_SCRATCH;
  try {
    hipStream_t s = (hipStream_t)hip_stream;
    void* base = nullptr;
    FEAST_HIP(scratch_address(&base));
    Carve c{(uintptr_t)base};
    zd* zdev = c.take<zd>(n_c);
    zd* odev = c.take<zd>(n_c);
    LuWork w;
    lu_work_carve(w, c.take<char>(lu_work_bytes(np, n_c)), np, n_c);
    zd* F = c.take<zd>((size_t)n_c * np * np);
    zd* iL = c.take<zd>((size_t)n_c * np * nbt);
    zd* iU = c.take<zd>((size_t)n_c * np * nbt);
    zd* tmp = c.take<zd>((size_t)np * nbt);
    zd* B = c.take<zd>((size_t)n_c * sides * np * m0);
    zd* Z = c.take<zd>((size_t)n_c * sides * np * m0);
    const zd* Xc = (const zd*)X;
    long ldxc = ldx;
    zd* Qc = (zd*)Q;
    long ldqc = ldq;
    if (dt == FEAST_R64) {
      zd* xb = c.take<zd>((size_t)n * m0);
      real_to_complex(s, (const double*)X, ldx, xb, n, n, m0);
      Xc = xb;
      ldxc = n;
      Qc = c.take<zd>((size_t)n * m0);
      ldqc = n;
    }
    std::vector<zd> zh(n_c), oh(n_c);
    quadrature_nodes(emin, emax, n_c, zh.data(), oh.data());
    store_values(s, zh.data(), n_c, zdev);
    store_values(s, oh.data(), n_c, odev);
    fill_zero(s, w.flag, sizeof(int));
    shift_matrices(s, A, lda, dt == FEAST_R64, n, np, zdev, n_c, F, w.flag);
    if (read_flag(s, w.flag)) return FEAST_NONFINITE;
    lu_factor_f64(s, F, np, n_c, w);
    if (read_flag(s, w.flag)) return FEAST_ZERO_PIVOT;
    tri_inverse_blocks_f64(s, F, np, n_c, nbt, iL, iU, tmp);
    gather_rhs(s, Xc, ldxc, n, np, m0, n_c, sides, w.perm, B);
    solve_sweeps_f64(s, F, iL, iU, np, n_c, nbt, sides, m0, B, Z);
    accumulate(s, B, n, np, m0, n_c, sides, odev, w.pinv, Qc, ldqc);
    if (dt == FEAST_R64) complex_to_real(s, Qc, n, (double*)Q, ldq, n, m0);
    FEAST_HIP(hipStreamSynchronize(s));
    return 0;
  } catch (const HipError&) {
    return FEAST_ERR_HIP;
  }
}
