// Rayleigh-Ritz building blocks (Appendix, FEAST step 2; residuals of step 3):
//   Cholesky-QR orthonormalisation of the filtered block (G = Q^H Q = R^H R, Q <- Q R^{-1}),
//   block-pair parallel-order two-sided Jacobi for the m0 x m0 reduced matrix, eigenpair sort,
//   and the residual norms ||A x_k - lambda_k x_k||.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace feast {

namespace {

__global__ void reduce_herm_kernel(const zd* __restrict__ part, int nparts, int m,
                                   zd* __restrict__ G, int ldg) {
  long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)m * m) return;
  int i = (int)(idx % m), j = (int)(idx / m);
  if (i > j) return;
  const long mm = (long)m * m;
  double ar = 0, ai = 0, br = 0, bi = 0;
  for (int p = 0; p < nparts; ++p) {
    zd a = part[p * mm + i + (long)j * m];
    zd b = part[p * mm + j + (long)i * m];
    ar += a.x;
    ai += a.y;
    br += b.x;
    bi += b.y;
  }
  // (S + S^H)/2 at (i, j) and its conjugate at (j, i)
  double re = 0.5 * (ar + br), im = 0.5 * (ai - bi);
  if (i == j) im = 0.0;
  G[i + (long)j * ldg] = zmake(re, im);
  G[j + (long)i * ldg] = zmake(re, -im);
}

constexpr int CB = 64;

// Unblocked upper Cholesky of the b x b diagonal block at G (ld) in LDS.
__global__ __launch_bounds__(256) void chol_diag_kernel(zd* G, int ld, int b, int* flag) {
  __shared__ zd S[CB][CB + 1];
  const int t = threadIdx.x;
  for (int e = t; e < b * b; e += 256) {
    int r = e % b, c = e / b;
    S[r][c] = G[r + (long)c * ld];
  }
  __syncthreads();
  for (int j = 0; j < b; ++j) {
    double d = S[j][j].x;
    bool bad = !(d > 0.0);
    double rjj = bad ? 1.0 : sqrt(d);
    __syncthreads();
    if (t == 0) {
      if (bad && flag) atomicOr(flag, 1);
      S[j][j] = zmake(rjj, 0.0);
    }
    for (int c = j + 1 + t; c < b; c += 256) S[j][c] = zscale(S[j][c], 1.0 / rjj);
    __syncthreads();
    // trailing: S[i][c] -= conj(S[j][i]) S[j][c] for j < i <= c
    int rest = b - j - 1;
    for (int e = t; e < rest * rest; e += 256) {
      int i = j + 1 + e % rest, c = j + 1 + e / rest;
      if (i <= c) {
        zd u = S[j][i], v = S[j][c];
        S[i][c] = zsub(S[i][c], zmake(u.x * v.x + u.y * v.y, u.x * v.y - u.y * v.x));
      }
    }
    __syncthreads();
  }
  for (int e = t; e < b * b; e += 256) {
    int r = e % b, c = e / b;
    G[r + (long)c * ld] = (r <= c) ? S[r][c] : zmake(0, 0);
  }
}

// X = R11^{-H} X for a 64-column chunk: R11 (b x b upper) at R, X (b x ncols) at X.
__global__ __launch_bounds__(256) void chol_rowpanel_kernel(const zd* R, int ld, int b, zd* X,
                                                            int ncols) {
  __shared__ zd Rs[CB][CB + 1];
  __shared__ zd Xs[CB][CB + 1];
  const int t = threadIdx.x;
  const int c0 = blockIdx.x * 64;
  for (int e = t; e < b * b; e += 256) {
    int r = e % b, c = e / b;
    Rs[r][c] = R[r + (long)c * ld];
  }
  for (int e = t; e < b * 64; e += 256) {
    int r = e % b, c = e / b;
    Xs[r][c] = (c0 + c < ncols) ? X[r + (long)(c0 + c) * ld] : zmake(0, 0);
  }
  __syncthreads();
  // solve R11^H Y = X: forward, row r: y_r = (x_r - sum_{i<r} conj(R[i][r]) y_i) / R[r][r]
  for (int r = 0; r < b; ++r) {
    if (t < 64) Xs[r][t] = zscale(Xs[r][t], 1.0 / Rs[r][r].x);
    __syncthreads();
    int rows = b - r - 1;
    for (int e = t; e < rows * 64; e += 256) {
      int i = r + 1 + e % rows, c = e / rows;
      zd u = Rs[r][i], y = Xs[r][c];  // conj(u) * y
      Xs[i][c] = zsub(Xs[i][c], zmake(u.x * y.x + u.y * y.y, u.x * y.y - u.y * y.x));
    }
    __syncthreads();
  }
  for (int e = t; e < b * 64; e += 256) {
    int r = e % b, c = e / b;
    if (c0 + c < ncols) X[r + (long)(c0 + c) * ld] = Xs[r][c];
  }
}

// Inverses of the diagonal blocks of the m x m upper R, one workgroup per block: block j
// (b = min(64, m - 64 j) rows from row 64 j) into the same position of out (identity-padded
// in LDS).
__global__ __launch_bounds__(256) void upper_inv_small_kernel(const zd* R, int ldr, int m, zd* out,
                                                              int ldo) {
  __shared__ zd Tm[CB][CB + 1];
  __shared__ zd X[CB][CB + 1];
  const int t = threadIdx.x;
  const int j0 = blockIdx.x * CB;
  const int b = (m - j0 < CB) ? m - j0 : CB;
  R += j0 + (long)j0 * ldr;
  out += j0 + (long)j0 * ldo;
  for (int e = t; e < CB * CB; e += 256) {
    int r = e % CB, c = e / CB;
    Tm[r][c] = (r < b && c < b) ? R[r + (long)c * ldr] : zmake(r == c ? 1 : 0, 0);
    X[r][c] = zmake(r == c ? 1 : 0, 0);
  }
  __syncthreads();
  for (int r = CB - 1; r >= 0; --r) {
    if (t < CB - r) {
      int c = r + t;
      X[r][c] = zdiv(X[r][c], Tm[r][r]);
    }
    __syncthreads();
    int cols = CB - r;
    for (int e = t; e < r * cols; e += 256) {
      int i = e % r, c = r + e / r;
      X[i][c] = zsub(X[i][c], zmul(Tm[i][r], X[r][c]));
    }
    __syncthreads();
  }
  for (int e = t; e < b * b; e += 256) {
    int r = e % b, c = e / b;
    out[r + (long)c * ldo] = X[r][c];
  }
}

// ---- Jacobi ---------------------------------------------------------------------------
struct Rot {
  bool active;
  double c, s, t, a;
  zd e;  // e^{-i phi}, phi = arg(h_pq)
};

// 1/d for finite d != 0: the hardware estimate refined by two Newton steps (each squares the
// relative error), so the result is within a few ulp.
__device__ inline double rcp_acc(double d) {
  double x = __builtin_amdgcn_rcp(d);
  x = fma(x, fma(-d, x, 1.0), x);
  x = fma(x, fma(-d, x, 1.0), x);
  return x;
}

// The rotation G = [[c, s], [-s e, c e]] that zeroes h_pq of the 2 x 2 Hermitian block
// [[hpp, hpq], [conj(hpq), hqq]] (t = s / c, the smaller root of t^2 + 2 tau t - 1 = 0 with
// tau = (hqq - hpp) / (2 |hpq|)); c = (1 + t^2)^{-1/2}, s = t c, e = conj(hpq) / |hpq|.
// A rotation is skipped when |h_pq| <= max(1e-17 sqrt(|h_pp h_qq|), tol), tol = eps ||H||_F:
// forming the reduced matrix already perturbs every entry by about eps ||H||, so rotating
// smaller entries only chases rounding noise.  The tests are taken on squares and the
// quotients through reciprocal square roots, which keeps the latency of the serial part of a
// round short; every quantity stays within a few ulp, so G is unitary to a few ulp.
__device__ inline Rot make_rot(double hpp, double hqq, zd hpq, double tol) {
  Rot r;
  const double a2 = hpq.x * hpq.x + hpq.y * hpq.y;
  r.active = !(a2 == 0.0 || a2 <= 1e-34 * fabs(hpp * hqq) || a2 <= tol * tol);
  if (!r.active) {
    r.a = sqrt(a2);
    r.c = 1;
    r.s = 0;
    r.t = 0;
    r.e = zmake(1, 0);
    return r;
  }
  const double ra = rsqrt(a2);
  r.a = a2 * ra;
  r.e = zmake(hpq.x * ra, -hpq.y * ra);
  const double tau = 0.5 * (hqq - hpp) * ra;
  const double u = fma(tau, tau, 1.0);
  const double tt = copysign(rcp_acc(fabs(tau) + u * rsqrt(u)), tau);
  r.t = tt;
  r.c = rsqrt(fma(tt, tt, 1.0));
  r.s = tt * r.c;
  return r;
}

// Pair a of round t in the round-robin ("circle") ordering of mp indices.
__device__ inline void pair_of(int a, int t, int mp, int& p, int& q) {
  auto f = [&](int i) { return i == 0 ? 0 : ((i - 1 + t) % (mp - 1)) + 1; };
  int x = f(a), y = f(mp - 1 - a);
  p = x < y ? x : y;
  q = x < y ? y : x;
}

// Block-pair ordering.  The mp indices form nb = mp / JB blocks of JB; an outer round pairs
// the blocks by the same round-robin ordering (nb / 2 disjoint pairs P = I u J of JP = 2 JB
// indices), and for each pair one workgroup runs parallel rounds of plane rotations over the
// JP x JP diagonal tile H[P, P] in LDS, accumulating them into the unitary U_P.  A second
// kernel then applies the outer round's block-diagonal transformation to the rest:
// H[P, Q] <- U_P^H H[P, Q] U_Q (P != Q) and V[:, Q] <- V[:, Q] U_Q.  nb - 1 outer rounds are one
// sweep, in which every index pair (p, q) is rotated once (pairs inside a block in the first
// outer round, cross pairs when their blocks meet), as in the cyclic element ordering, but
// with nb - 1 dependent launch pairs instead of mp - 1.
constexpr int JB = 16;
constexpr int JP = 2 * JB;

// Global index of local index l (0..JP-1) of block pair (I, J).
__device__ inline int pair_index(int l, int I, int J) { return l < JB ? I * JB + l : J * JB + l - JB; }

// Outer round 0 of a sweep runs the full inner sweep (all JP (JP - 1) / 2 local pairs, so every
// within-block pair is rotated once per sweep); later outer rounds rotate only the JB^2
// cross pairs (p in I, q in J), in JB rounds pairing I[i] with J[(i + k) mod JB].
__global__ __launch_bounds__(256) void jacobi_inner_kernel(zd* __restrict__ H, int mp, int round,
                                                           zd* __restrict__ Ubuf,
                                                           const double* __restrict__ tolp) {
  __shared__ zd Hs[JP][JP + 1];
  __shared__ zd Us[JP][JP + 1];
  __shared__ double rc[JB], rsn[JB], rt[JB], ra[JB];
  __shared__ zd re[JB];
  __shared__ int rp[JB], rq[JB], ract[JB];
  const int t = threadIdx.x;
  const int nb = mp / JB;
  int I, J;
  pair_of(blockIdx.x, round, nb, I, J);
  const double tol = tolp[0];
  for (int e = t; e < JP * JP; e += 256) {
    int r = e % JP, c = e / JP;
    Hs[r][c] = H[pair_index(r, I, J) + (long)pair_index(c, I, J) * mp];
    Us[r][c] = zmake(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const bool full = (round == 0);
  const int nrounds = full ? JP - 1 : JB;
  for (int it = 0; it < nrounds; ++it) {
    if (t < JB) {
      int p, q;
      if (full) {
        pair_of(t, it, JP, p, q);
      } else {
        p = t;
        q = JB + (t + it) % JB;
      }
      Rot r = make_rot(Hs[p][p].x, Hs[q][q].x, Hs[p][q], tol);
      rc[t] = r.c;
      rsn[t] = r.s;
      rt[t] = r.t;
      ra[t] = r.a;
      re[t] = r.e;
      rp[t] = p;
      rq[t] = q;
      ract[t] = r.active;
    }
    __syncthreads();
    {  // H <- G^H H G on the 2 x 2 sub-blocks (rotation pairs a, b): each entry once
      const int a = t % JB, b = t / JB;
      const int pa = rp[a], qa = rq[a], pb = rp[b], qb = rq[b];
      zd b00 = Hs[pa][pb], b01 = Hs[pa][qb], b10 = Hs[qa][pb], b11 = Hs[qa][qb];
      zd ga11 = zmake(rc[a], 0), ga12 = zmake(rsn[a], 0);
      zd ga21 = zscale(re[a], -rsn[a]), ga22 = zscale(re[a], rc[a]);
      zd y00 = zadd(zmul(zconj(ga11), b00), zmul(zconj(ga21), b10));
      zd y01 = zadd(zmul(zconj(ga11), b01), zmul(zconj(ga21), b11));
      zd y10 = zadd(zmul(zconj(ga12), b00), zmul(zconj(ga22), b10));
      zd y11 = zadd(zmul(zconj(ga12), b01), zmul(zconj(ga22), b11));
      zd gb11 = zmake(rc[b], 0), gb12 = zmake(rsn[b], 0);
      zd gb21 = zscale(re[b], -rsn[b]), gb22 = zscale(re[b], rc[b]);
      zd x00 = zadd(zmul(y00, gb11), zmul(y01, gb21));
      zd x01 = zadd(zmul(y00, gb12), zmul(y01, gb22));
      zd x10 = zadd(zmul(y10, gb11), zmul(y11, gb21));
      zd x11 = zadd(zmul(y10, gb12), zmul(y11, gb22));
      if (a == b && ract[a]) {
        x00 = zmake(b00.x - rt[a] * ra[a], 0);
        x11 = zmake(b11.x + rt[a] * ra[a], 0);
        x01 = zmake(0, 0);
        x10 = zmake(0, 0);
      }
      Hs[pa][pb] = x00;
      Hs[pa][qb] = x01;
      Hs[qa][pb] = x10;
      Hs[qa][qb] = x11;
    }
    for (int e = t; e < JP * JB; e += 256) {  // U <- U G: row i, rotation b
      const int i = e % JP, b = e / JP;
      const int pb = rp[b], qb = rq[b];
      zd gb11 = zmake(rc[b], 0), gb12 = zmake(rsn[b], 0);
      zd gb21 = zscale(re[b], -rsn[b]), gb22 = zscale(re[b], rc[b]);
      zd u0 = Us[i][pb], u1 = Us[i][qb];
      Us[i][pb] = zadd(zmul(u0, gb11), zmul(u1, gb21));
      Us[i][qb] = zadd(zmul(u0, gb12), zmul(u1, gb22));
    }
    __syncthreads();
  }
  zd* U = Ubuf + (long)blockIdx.x * JP * JP;
  for (int e = t; e < JP * JP; e += 256) {
    int r = e % JP, c = e / JP;
    H[pair_index(r, I, J) + (long)pair_index(c, I, J) * mp] = Hs[r][c];
    U[e] = Us[r][c];
  }
}

// grid (npair, npair + mp / JP), 1024 threads (one output entry each).  y < npair: H tiles
// P = y < Q = x: X = U_P^H H[P, Q] U_Q is written to H[P, Q] and X^H to H[Q, P] (the
// transformed matrix stays exactly Hermitian; blocks with y >= x return at once).
// y >= npair: V rows JP (y - npair) .. + JP - 1 against column pair Q = x.
__global__ __launch_bounds__(1024) void jacobi_apply_kernel(zd* __restrict__ H, zd* __restrict__ V,
                                                            int mp, int round,
                                                            const zd* __restrict__ Ubuf) {
  __shared__ zd Ts[JP][JP + 1];
  __shared__ zd Uq[JP][JP + 1];
  __shared__ zd Up[JP][JP + 1];
  const int t = threadIdx.x;
  const int nb = mp / JB, npair = nb / 2;
  const int x = blockIdx.x, y = blockIdx.y;
  const bool isH = y < npair;
  if (isH && y >= x) return;  // diagonal tiles: inner kernel; lower tiles: mirrored below
  int Iq, Jq, Ip = 0, Jp = 0;
  pair_of(x, round, nb, Iq, Jq);
  if (isH) pair_of(y, round, nb, Ip, Jp);
  zd* M = isH ? H : V;
  const int r0 = (y - npair) * JP;
  const int c = t % JP, r = t / JP;
  const int gc = pair_index(c, Iq, Jq);
  const int gr = isH ? pair_index(r, Ip, Jp) : r0 + r;
  Ts[r][c] = M[gr + (long)gc * mp];
  Uq[r][c] = Ubuf[(long)x * JP * JP + r + c * JP];
  if (isH) Up[r][c] = Ubuf[(long)y * JP * JP + r + c * JP];
  __syncthreads();
  zd acc = zmake(0, 0);
#pragma unroll 8
  for (int j = 0; j < JP; ++j) acc = zadd(acc, zmul(Ts[r][j], Uq[j][c]));
  if (isH) {
    __syncthreads();
    Ts[r][c] = acc;
    __syncthreads();
    acc = zmake(0, 0);
#pragma unroll 8
    for (int j = 0; j < JP; ++j) acc = zadd(acc, zmul(zconj(Up[j][r]), Ts[j][c]));
    H[gc + (long)gr * mp] = zconj(acc);
  }
  M[gr + (long)gc * mp] = acc;
}

__global__ void jacobi_check_kernel(const zd* __restrict__ H, int mp, const double* __restrict__ tolp,
                                    int* flag) {
  long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)mp * mp) return;
  int p = (int)(idx % mp), q = (int)(idx / mp);
  if (p >= q) return;
  zd hpq = H[p + (long)q * mp];
  double a = sqrt(hpq.x * hpq.x + hpq.y * hpq.y);
  double hpp = H[p + (long)p * mp].x, hqq = H[q + (long)q * mp].x;
  if (!(a == 0.0 || a <= 1e-17 * sqrt(fabs(hpp * hqq)) || a <= tolp[1])) atomicOr(flag, 1);
}

// tol[0] = eps ||H||_F (rotation floor) and tol[1] = 4 eps ||H||_F (convergence test) over the
// m x m input, in two deterministic stages (64 partial sums).  Each outer round transforms
// every entry by 32-term block products, which leaves rounding noise of about eps ||H|| in the
// off-diagonal part: a sweep still rotates entries down to that level, but convergence is
// declared once none exceeds a few times it, which the noise cannot keep from happening.
__global__ __launch_bounds__(256) void fro_partial_kernel(const zd* __restrict__ H, long count,
                                                          double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < count; i += 256L * gridDim.x) {
    zd v = H[i];
    s += v.x * v.x + v.y * v.y;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void fro_final_kernel(const double* __restrict__ part, int nparts, double* tol) {
  if (threadIdx.x == 0) {
    double s = 0;
    for (int i = 0; i < nparts; ++i) s += part[i];
    tol[0] = 2.220446049250313e-16 * sqrt(s);
    tol[1] = 4.0 * tol[0];
  }
}

__global__ void jacobi_init_kernel(const zd* __restrict__ H, int m, int mp, zd* __restrict__ A,
                                   zd* __restrict__ V) {
  long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)mp * mp) return;
  int i = (int)(idx % mp), j = (int)(idx / mp);
  zd v;
  if (i < m && j < m) v = H[i + (long)j * m];
  else v = zmake(i == j ? 1e100 : 0.0, 0.0);  // padded index: decoupled, sorts last
  A[idx] = v;
  V[idx] = zmake(i == j ? 1.0 : 0.0, 0.0);
}

__global__ void diag_kernel(const zd* H, int mp, double* d) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < mp) d[i] = H[i + (long)i * mp].x;
}

__global__ void rank_kernel(const double* d, int mp, int* rank) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= mp) return;
  double di = d[i];
  int r = 0;
  for (int j = 0; j < mp; ++j) {
    double dj = d[j];
    if (dj < di || (dj == di && j < i)) r++;
  }
  rank[i] = r;
}

__global__ void sort_copy_kernel(const double* d, const zd* V, const int* rank, int m, int mp,
                                 double* lam, zd* W) {
  long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)m * mp) return;
  int i = (int)(idx % m), src = (int)(idx / m);
  int r = rank[src];
  if (r >= m) return;
  W[i + (long)r * m] = V[i + (long)src * mp];
  if (i == 0) lam[r] = d[src];
}

__global__ __launch_bounds__(256) void residual_kernel(const zd* __restrict__ AX, long ldax,
                                                       const zd* __restrict__ X, long ldx,
                                                       const double* __restrict__ lam, int n,
                                                       double anorm, double* res) {
  __shared__ double sh[256];
  const int k = blockIdx.x;
  const double l = lam[k];
  double s = 0;
  for (int i = threadIdx.x; i < n; i += 256) {
    zd a = AX[i + (long)k * ldax], x = X[i + (long)k * ldx];
    double rr = a.x - l * x.x, ri = a.y - l * x.y;
    s += rr * rr + ri * ri;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) res[k] = sqrt(sh[0]) / anorm;
}

__global__ __launch_bounds__(256) void coldot_kernel(const zd* __restrict__ X, long ldx,
                                                     const zd* __restrict__ Y, long ldy, int n,
                                                     double* out) {
  __shared__ double sh[256];
  const int k = blockIdx.x;
  double s = 0;
  for (int i = threadIdx.x; i < n; i += 256) {
    zd a = X[i + (long)k * ldx], b = Y[i + (long)k * ldy];
    s += a.x * b.x + a.y * b.y;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = sh[0];
}

__global__ void ritz_residual_kernel(const zd* AX, long ldax, const zd* X, long ldx,
                                     const double* lam, int n, int m0, zd* R) {
  long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)n * m0) return;
  int i = (int)(idx % n), k = (int)(idx / n);
  zd a = AX[i + (long)k * ldax], x = X[i + (long)k * ldx];
  R[i + (long)k * n] = zmake(a.x - lam[k] * x.x, a.y - lam[k] * x.y);
}

__global__ void copy_kernel(const zd* src, long lds, zd* dst, long ldd, int rows, int cols) {
  long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)rows * cols) return;
  int i = (int)(idx % rows), j = (int)(idx / rows);
  dst[i + (long)j * ldd] = src[i + (long)j * lds];
}
__global__ void r2c_kernel(const double* src, long lds, zd* dst, long ldd, int rows, int cols) {
  long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)rows * cols) return;
  int i = (int)(idx % rows), j = (int)(idx / rows);
  dst[i + (long)j * ldd] = zmake(src[i + (long)j * lds], 0.0);
}
__global__ void c2r_kernel(const zd* src, long lds, double* dst, long ldd, int rows, int cols) {
  long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)rows * cols) return;
  int i = (int)(idx % rows), j = (int)(idx / rows);
  dst[i + (long)j * ldd] = src[i + (long)j * lds].x;
}
__global__ void nonfinite_kernel(const zd* a, long ld, int rows, int cols, int* flag) {
  long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)rows * cols) return;
  int i = (int)(idx % rows), j = (int)(idx / rows);
  zd v = a[i + (long)j * ld];
  if (!isfinite(v.x) || !isfinite(v.y)) atomicOr(flag, 1);
}

__global__ void diag_real_kernel(const zd* G, int m, int ldg, double* diag) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) diag[k] = G[k + (long)k * ldg].x;
}
__global__ void add_diag_kernel(zd* G, int m, int ldg, double sigma) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) G[k + (long)k * ldg].x += sigma;
}

__device__ inline unsigned long long splitmix64(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
__device__ inline double u01(unsigned long long x) {  // (0, 1]
  return ((x >> 11) + 1.0) * (1.0 / 9007199254740992.0);
}
__global__ void gaussian_kernel(void* X, long ldx, int rows, int cols, int is_real,
                                unsigned long long seed) {
  long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)rows * cols) return;
  int i = (int)(idx % rows), j = (int)(idx / rows);
  unsigned long long h = splitmix64(seed ^ splitmix64((unsigned long long)idx));
  double u1 = u01(h), u2 = u01(splitmix64(h));
  double rad = sqrt(-2.0 * log(u1)), ang = 6.283185307179586 * u2;
  if (is_real) ((double*)X)[i + (long)j * ldx] = rad * cos(ang);
  else ((zd*)X)[i + (long)j * ldx] = zmake(rad * cos(ang), rad * sin(ang));
}

__global__ __launch_bounds__(256) void vec_norm_kernel(const zd* v, int n, double* out) {
  __shared__ double sh[256];
  double s = 0;
  for (int i = threadIdx.x; i < n; i += 256) s += zabs2(v[i]);
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sqrt(sh[0]);
}
__global__ void vec_scale_kernel(const zd* w, int n, const double* nrm, zd* v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double s = nrm[0] > 0 ? 1.0 / nrm[0] : 0.0;
  if (i < n) v[i] = zscale(w[i], s);
}

inline dim3 grid1(long n) { return dim3((unsigned)((n + 255) / 256)); }

// Zero fill of `words` 32-bit words then `tail` bytes (grid-stride, 16-byte stores when the
// buffer allows them).  A kernel rather than hipMemsetAsync, so that clearing flags and
// scratch stays an ordinary kernel node if a caller records the work into a HIP graph.
__global__ void zero_fill_kernel(void* p, size_t bytes) {
  const size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  char* c = (char*)p;
  size_t head = 0;
  if (((uintptr_t)c & 15) == 0) {
    const size_t n16 = bytes / 16;
    uint4* q = (uint4*)c;
    for (size_t i = tid; i < n16; i += stride) q[i] = make_uint4(0, 0, 0, 0);
    head = n16 * 16;
  }
  for (size_t i = head + tid; i < bytes; i += stride) c[i] = 0;
}

}  // namespace

void reduce_partials_hermitian(hipStream_t s, const zd* part, int nparts, int m, zd* G, int ldg) {
  hipLaunchKernelGGL(reduce_herm_kernel, grid1((long)m * m), dim3(256), 0, s, part, nparts, m, G,
                     ldg);
  FEAST_LAUNCH_CHECK();
}

void cholesky_upper(hipStream_t s, zd* G, int m, int ldg, int* flag, zd* tmp) {
  (void)tmp;
  for (int k = 0; k < m; k += CB) {
    int b = (m - k < CB) ? m - k : CB;
    zd* Gkk = G + k + (long)k * ldg;
    hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(256), 0, s, Gkk, ldg, b, flag);
    FEAST_LAUNCH_CHECK();
    int rest = m - k - b;
    if (rest > 0) {
      zd* G12 = G + k + (long)(k + b) * ldg;
      hipLaunchKernelGGL(chol_rowpanel_kernel, dim3((rest + 63) / 64), dim3(256), 0, s, Gkk, ldg,
                         b, G12, rest);
      FEAST_LAUNCH_CHECK();
      zgemm(s, OP_C, OP_N, rest, rest, b, zmake(-1, 0), G12, ldg, G12, ldg, zmake(1, 0),
            G + (k + b) + (long)(k + b) * ldg, ldg);
    }
  }
}

void upper_inverse(hipStream_t s, const zd* R, int m, int ldr, zd* Rinv, int ldi, zd* tmp) {
  // Rinv must be zero on entry.  Block columns of 64: Rinv_jj = R_jj^{-1} (all diagonal
  // blocks in one launch); Rinv[0:j, j] = -Rinv[0:j, 0:j] (R[0:j, j] Rinv_jj).
  hipLaunchKernelGGL(upper_inv_small_kernel, dim3((m + CB - 1) / CB), dim3(256), 0, s, R, ldr, m,
                     Rinv, ldi);
  FEAST_LAUNCH_CHECK();
  for (int j = 0; j < m; j += CB) {
    int b = (m - j < CB) ? m - j : CB;
    if (j > 0) {
      zgemm(s, OP_N, OP_N, j, b, b, zmake(1, 0), R + (long)j * ldr, ldr, Rinv + j + (long)j * ldi,
            ldi, zmake(0, 0), tmp, j);
      zgemm(s, OP_N, OP_N, j, b, j, zmake(-1, 0), Rinv, ldi, tmp, j, zmake(0, 0),
            Rinv + (long)j * ldi, ldi);
    }
  }
}

__global__ void zero_int_kernel(int* p) { p[0] = 0; }
// One sweep (nb - 1 outer rounds of an inner kernel and an apply kernel, in place) followed
// by the convergence check, either launched directly or recorded into a graph by stream
// capture.
static void jacobi_sweep_launches(hipStream_t s, zd* A, zd* V, zd* Ubuf, int mp, int* dflag,
                                  const double* tolp) {
  const int nb = mp / JB, npair = nb / 2;
  for (int r = 0; r < nb - 1; ++r) {
    hipLaunchKernelGGL(jacobi_inner_kernel, dim3(npair), dim3(256), 0, s, A, mp, r, Ubuf, tolp);
    hipLaunchKernelGGL(jacobi_apply_kernel, dim3(npair, npair + mp / JP), dim3(1024), 0, s, A, V,
                       mp, r, (const zd*)Ubuf);
  }
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, s, dflag);
  hipLaunchKernelGGL(jacobi_check_kernel, grid1((long)mp * mp), dim3(256), 0, s, A, mp, tolp,
                     dflag);
}

JacobiGraph::~JacobiGraph() {
  if (exec) (void)hipGraphExecDestroy((hipGraphExec_t)exec);
  if (graph) (void)hipGraphDestroy((hipGraph_t)graph);
}

int jacobi_eigh(hipStream_t s, zd* H, int m, double* d, zd* V, zd* work, int* dflag,
                int max_sweeps, JacobiGraph* cache, int mp) {
  // work: jacobi_work(mp) complex: the working matrix (mp^2), the outer round's block-pair
  // unitaries (mp / JP of JP x JP), then 64 partial sums and tol as doubles; V is mp x mp.
  if (mp < jacobi_order(m) || mp % JP)
    throw HipError{hipErrorInvalidValue, "jacobi_eigh: padded order must be a multiple of 32 >= m"};
  zd* A0 = work;
  zd* Ubuf = work + (long)mp * mp;
  double* dwork = (double*)(Ubuf + (long)mp * JP);
  double* tolp = dwork + 64;
  hipLaunchKernelGGL(jacobi_init_kernel, grid1((long)mp * mp), dim3(256), 0, s, H, m, mp, A0, V);
  hipLaunchKernelGGL(fro_partial_kernel, dim3(64), dim3(256), 0, s, H, (long)m * m, dwork);
  hipLaunchKernelGGL(fro_final_kernel, dim3(1), dim3(64), 0, s, dwork, 64, tolp);
  FEAST_LAUNCH_CHECK();
  hipGraphExec_t exec = nullptr;
  if (cache && s) {  // the legacy null stream cannot be captured
    if (!(cache->exec && cache->mp == mp && cache->A0 == A0 && cache->V == V &&
          cache->flag == dflag)) {
      if (cache->exec) FEAST_HIP(hipGraphExecDestroy((hipGraphExec_t)cache->exec));
      if (cache->graph) FEAST_HIP(hipGraphDestroy((hipGraph_t)cache->graph));
      cache->exec = cache->graph = nullptr;
      hipGraph_t g = nullptr;
      FEAST_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      jacobi_sweep_launches(s, A0, V, Ubuf, mp, dflag, tolp);
      FEAST_HIP(hipStreamEndCapture(s, &g));
      hipGraphExec_t ge = nullptr;
      FEAST_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
      cache->graph = g;
      cache->exec = ge;
      cache->mp = mp;
      cache->A0 = A0;
      cache->V = V;
      cache->flag = dflag;
    }
    exec = (hipGraphExec_t)cache->exec;
  }
  int sweeps = 0;
  bool converged = false;
  for (; sweeps < max_sweeps && !converged; ++sweeps) {
    if (exec) FEAST_HIP(hipGraphLaunch(exec, s));
    else jacobi_sweep_launches(s, A0, V, Ubuf, mp, dflag, tolp);
    FEAST_LAUNCH_CHECK();
    int h = 0;
    FEAST_HIP(hipMemcpyAsync(&h, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
    FEAST_HIP(hipStreamSynchronize(s));
    converged = (h == 0);
  }
  hipLaunchKernelGGL(diag_kernel, grid1(mp), dim3(256), 0, s, A0, mp, d);
  FEAST_LAUNCH_CHECK();
  return converged ? sweeps : -1;
}

void sort_eigen(hipStream_t s, const double* d, const zd* V, int m, int mp, double* lam, zd* W,
                int* rank) {
  hipLaunchKernelGGL(rank_kernel, grid1(mp), dim3(256), 0, s, d, mp, rank);
  FEAST_LAUNCH_CHECK();
  hipLaunchKernelGGL(sort_copy_kernel, grid1((long)m * mp), dim3(256), 0, s, d, V, rank, m, mp,
                     lam, W);
  FEAST_LAUNCH_CHECK();
}

void residual_norms(hipStream_t s, const zd* AX, long ldax, const zd* X, long ldx,
                    const double* lam, int n, int m0, double anorm, double* res) {
  hipLaunchKernelGGL(residual_kernel, dim3(m0), dim3(256), 0, s, AX, ldax, X, ldx, lam, n, anorm,
                     res);
  FEAST_LAUNCH_CHECK();
}

void coldot_re(hipStream_t s, const zd* X, long ldx, const zd* Y, long ldy, int n, int m0,
               double* out) {
  hipLaunchKernelGGL(coldot_kernel, dim3(m0), dim3(256), 0, s, X, ldx, Y, ldy, n, out);
  FEAST_LAUNCH_CHECK();
}

void ritz_residual(hipStream_t s, const zd* AX, long ldax, const zd* X, long ldx,
                   const double* lam, int n, int m0, zd* R) {
  hipLaunchKernelGGL(ritz_residual_kernel, grid1((long)n * m0), dim3(256), 0, s, AX, ldax, X, ldx,
                     lam, n, m0, R);
  FEAST_LAUNCH_CHECK();
}

void copy_matrix(hipStream_t s, const zd* src, long lds, zd* dst, long ldd, int rows, int cols) {
  hipLaunchKernelGGL(copy_kernel, grid1((long)rows * cols), dim3(256), 0, s, src, lds, dst, ldd,
                     rows, cols);
  FEAST_LAUNCH_CHECK();
}
void real_to_complex(hipStream_t s, const double* src, long lds, zd* dst, long ldd, int rows,
                     int cols) {
  hipLaunchKernelGGL(r2c_kernel, grid1((long)rows * cols), dim3(256), 0, s, src, lds, dst, ldd,
                     rows, cols);
  FEAST_LAUNCH_CHECK();
}
void complex_to_real(hipStream_t s, const zd* src, long lds, double* dst, long ldd, int rows,
                     int cols) {
  hipLaunchKernelGGL(c2r_kernel, grid1((long)rows * cols), dim3(256), 0, s, src, lds, dst, ldd,
                     rows, cols);
  FEAST_LAUNCH_CHECK();
}
void fill_zero(hipStream_t s, void* p, size_t bytes) {
  if (bytes == 0) return;
  const size_t n16 = bytes / 16 + 1;
  const unsigned blocks = (unsigned)std::min<size_t>((n16 + 255) / 256, 8192);
  hipLaunchKernelGGL(zero_fill_kernel, dim3(blocks), dim3(256), 0, s, p, bytes);
  FEAST_LAUNCH_CHECK();
}

void diag_real(hipStream_t s, const zd* G, int m, int ldg, double* diag) {
  hipLaunchKernelGGL(diag_real_kernel, grid1(m), dim3(256), 0, s, G, m, ldg, diag);
  FEAST_LAUNCH_CHECK();
}
void add_diag(hipStream_t s, zd* G, int m, int ldg, double sigma) {
  hipLaunchKernelGGL(add_diag_kernel, grid1(m), dim3(256), 0, s, G, m, ldg, sigma);
  FEAST_LAUNCH_CHECK();
}
void gaussian_fill(hipStream_t s, void* X, long ldx, int rows, int cols, int is_real,
                   unsigned long long seed) {
  hipLaunchKernelGGL(gaussian_kernel, grid1((long)rows * cols), dim3(256), 0, s, X, ldx, rows, cols,
                     is_real, seed);
  FEAST_LAUNCH_CHECK();
}
double norm2_estimate(hipStream_t s, const zd* A, long lda, int n, int iters, zd* work,
                      double* dnorm) {
  zd* v = work;
  zd* w = work + n;
  gaussian_fill(s, v, n, n, 1, 0, 0x5EEDull);
  for (int it = 0; it < iters; ++it) {
    hipLaunchKernelGGL(vec_norm_kernel, dim3(1), dim3(256), 0, s, v, n, dnorm);
    hipLaunchKernelGGL(vec_scale_kernel, grid1(n), dim3(256), 0, s, v, n, dnorm, v);
    zgemm(s, OP_N, OP_N, n, 1, n, zmake(1, 0), A, lda, v, n, zmake(0, 0), w, n);
    std::swap(v, w);
  }
  hipLaunchKernelGGL(vec_norm_kernel, dim3(1), dim3(256), 0, s, v, n, dnorm);
  FEAST_LAUNCH_CHECK();
  double h = 0;
  FEAST_HIP(hipMemcpyAsync(&h, dnorm, sizeof(double), hipMemcpyDeviceToHost, s));
  FEAST_HIP(hipStreamSynchronize(s));
  return h;
}

int nonfinite_check(hipStream_t s, const zd* a, long ld, int rows, int cols, int* dflag) {
  fill_zero(s, dflag, sizeof(int));
  hipLaunchKernelGGL(nonfinite_kernel, grid1((long)rows * cols), dim3(256), 0, s, a, ld, rows, cols,
                     dflag);
  FEAST_LAUNCH_CHECK();
  int h = 0;
  FEAST_HIP(hipMemcpyAsync(&h, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
  FEAST_HIP(hipStreamSynchronize(s));
  return h;
}

}  // namespace feast
