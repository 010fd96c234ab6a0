// Shared device/host helpers of the FEAST MI355X library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

namespace feast {

// Interleaved complex values, (re, im) pairs as in std::complex / numpy complex128.
typedef double2 zd;
typedef float2 zf;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

enum Op { OP_N = 0, OP_T = 1, OP_C = 2 };

__host__ __device__ inline zd zmake(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline zd zadd(zd a, zd b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline zd zsub(zd a, zd b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline zd zmul(zd a, zd b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline zd zconj(zd a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline zd zscale(zd a, double s) { return make_double2(a.x * s, a.y * s); }
__host__ __device__ inline double zabs2(zd a) { return a.x * a.x + a.y * a.y; }
// a * conj(b)
__host__ __device__ inline zd zmulc(zd a, zd b) {
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// Division by Smith's scaling (avoids overflow in |b|^2 for large entries).
__host__ __device__ inline zd zdiv(zd a, zd b) {
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  } else {
    double r = b.x / b.y, d = b.y + b.x * r;
    return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
  }
}

struct HipError {
  hipError_t err;
  const char* what;
};

}  // namespace feast

#define FEAST_HIP(call)                                       \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) throw ::feast::HipError{e_, #call}; \
  } while (0)

#define FEAST_LAUNCH_CHECK() FEAST_HIP(hipGetLastError())
