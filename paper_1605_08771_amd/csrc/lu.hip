// Batched complex LU with partial pivoting of the shifted matrices M_j = z_j I - A, one per
// quadrature node (the "linear system solver" of Sec. 1, eq. contour_int_quad; the nodes are
// independent, so all n_c factorizations advance together in every launch).
//
// Blocked right-looking LU, panel width 64:
//   panel: one launch per column (one per group of PG columns while at most 1024 (FP64) or
//          2048 (FP32) rows remain).  Rows are never moved inside the panel ("implicit"
//          pivoting): each launch reduces the per-workgroup pivot candidates of the previous
//          launch, reads the pivot row, and eliminates every other active row, then leaves
//          the candidates of the next column.  The pivot row is read-only in that launch, so
//          workgroups never race.  The column steps update only the columns of their group
//          of PG; at the end of a group one launch applies the group's rank-PG update to the
//          panel's later columns and a second one writes the group's rows of U there.
//   swaps: the panel's pivot rows are moved to the top with the fewest row moves (at most
//          2 x 64 rows, LAPACK swap order) over all columns, and the permutation is updated;
//   U12:   L11^{-1} A12 as one matrix-core product with the explicit inverse of the unit-lower
//          64x64 L11 (formed once per panel in LDS);
//   A22 -= L21 U12 on the matrix cores (batched complex GEMM).
#include "common.h"
#include "kernels.h"

namespace feast {

namespace {

constexpr int NBP = 64;   // panel width
constexpr int NSUB = 8;   // panels per outer panel (trailing updates contract over NSUB * NBP)
constexpr int RPW = 256;  // rows per workgroup in the panel kernels
#ifndef FEAST_LU_PG
#define FEAST_LU_PG 16
#endif
constexpr int PG = FEAST_LU_PG;  // panel columns per group of column steps

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

template <typename v2>
__device__ inline v2 cmul(v2 a, v2 b) {
  v2 r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename v2>
__device__ inline v2 crecip(v2 a) {  // 1 / a with Smith scaling
  v2 r;
  if (fabs(a.x) >= fabs(a.y)) {
    auto q = a.y / a.x, d = a.x + a.y * q;
    r.x = 1 / d;
    r.y = -q / d;
  } else {
    auto q = a.x / a.y, d = a.y + a.x * q;
    r.x = q / d;
    r.y = -1 / d;
  }
  return r;
}

// M_j = z_j B - A (B == nullptr: B = I); A and B real (is_real) or complex.  *flag is set
// when a shifted entry is not finite in T (NaN/Inf in A or B, or beyond the FP32 range).
template <typename T>
__global__ void shift_kernel(const void* __restrict__ A, long lda, const void* __restrict__ B,
                             long ldb, int is_real, int n, int np, const zd* __restrict__ z,
                             int nc, typename V2<T>::t* __restrict__ M, int* flag) {
  typedef typename V2<T>::t v2;
  long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  long total = (long)np * np;
  if (idx >= total) return;
  int i = (int)(idx % np), c = (int)(idx / np);
  double ar = 0, ai = 0, br = (i == c) ? 1.0 : 0.0, bi = 0;
  bool inside = (i < n && c < n);
  if (inside) {
    if (is_real) {
      ar = ((const double*)A)[i + (long)c * lda];
      if (B) br = ((const double*)B)[i + (long)c * ldb];
    } else {
      zd a = ((const zd*)A)[i + (long)c * lda];
      ar = a.x;
      ai = a.y;
      if (B) {
        zd b = ((const zd*)B)[i + (long)c * ldb];
        br = b.x;
        bi = b.y;
      }
    }
  }
  for (int j = 0; j < nc; ++j) {
    v2 out;
    if (inside) {
      double re = z[j].x * br - z[j].y * bi - ar, im = z[j].x * bi + z[j].y * br - ai;
      out.x = (T)re;
      out.y = (T)im;
      if (!isfinite(out.x) || !isfinite(out.y)) atomicOr(flag, 1);
    } else {
      out.x = (T)(i == c ? 1.0 : 0.0);
      out.y = (T)0;
    }
    M[(long)j * total + idx] = out;
  }
}

__device__ inline void argmax_merge(double& v, int& r, double v2_, int r2) {
  if (v2_ > v || (v2_ == v && r2 < r)) {
    v = v2_;
    r = r2;
  }
}

// Block-wide (value, row) max reduction; result valid in thread 0.
__device__ inline void block_argmax(double& v, int& r, double* sv, int* sr) {
  const int t = threadIdx.x;
  sv[t] = v;
  sr[t] = r;
  __syncthreads();
  for (int s = RPW / 2; s > 0; s >>= 1) {
    if (t < s) {
      double ov = sv[t + s];
      int orow = sr[t + s];
      double cv = sv[t];
      int cr = sr[t];
      argmax_merge(cv, cr, ov, orow);
      sv[t] = cv;
      sr[t] = cr;
    }
    __syncthreads();
  }
  v = sv[0];
  r = sr[0];
}

template <typename T>
__global__ __launch_bounds__(RPW) void panel_search_kernel(const typename V2<T>::t* __restrict__ M,
                                                           int np, int k, double* pval,
                                                           int* prow, int maxwg) {
  __shared__ double sv[RPW];
  __shared__ int sr[RPW];
  const int node = blockIdx.y;
  M += (long)node * np * np;
  int row = k + blockIdx.x * RPW + threadIdx.x;
  double v = -1.0;
  int r = 0x7fffffff;
  if (row < np) {
    auto a = M[row + (long)k * np];
    v = (double)a.x * a.x + (double)a.y * a.y;
    r = row;
  }
  block_argmax(v, r, sv, sr);
  if (threadIdx.x == 0) {
    pval[node * maxwg + blockIdx.x] = v;
    prow[node * maxwg + blockIdx.x] = r;
  }
}

template <typename T>
__global__ __launch_bounds__(RPW) void panel_step_kernel(
    typename V2<T>::t* __restrict__ M, int np, int k, int w, int jj, int gend, int nwg,
    int maxwg, const double* __restrict__ pval_in, const int* __restrict__ prow_in,
    double* pval_out, int* prow_out, int* retired, int* pivrows, int* flag) {
  typedef typename V2<T>::t v2;
  __shared__ double sv[RPW];
  __shared__ int sr[RPW];
  __shared__ v2 upiv[NBP];
  __shared__ int s_p;
  __shared__ v2 s_rinv;
  __shared__ int s_zero;
  const int node = blockIdx.y;
  const int t = threadIdx.x;
  M += (long)node * np * np;
  retired += node * np;
  const int c = k + jj;
  const int stamp = k + 1;

  // pivot of column c from the candidates left by the previous launch
  {
    double v = -1.0;
    int r = 0x7fffffff;
    for (int q = t; q < nwg; q += RPW)
      argmax_merge(v, r, pval_in[node * maxwg + q], prow_in[node * maxwg + q]);
    block_argmax(v, r, sv, sr);
    if (t == 0) {
      bool bad = !(v > 0.0) || r < k || r >= np;  // zero column or non-finite candidates
      s_p = bad ? c : r;
      s_zero = bad;
    }
    __syncthreads();
  }
  const int p = s_p;
  const int width = gend - jj;  // columns c .. k+gend-1 (the rest of this column's group)
  if (t < width) upiv[t] = M[p + (long)(c + t) * np];
  __syncthreads();
  if (t == 0) {
    s_rinv = s_zero ? v2{0, 0} : crecip(upiv[0]);
    if (s_zero && flag) atomicCAS(flag, 0, c + 1);
  }
  __syncthreads();
  const v2 rinv = s_rinv;

  int row = k + blockIdx.x * RPW + t;
  double cand = -1.0;
  int crow = 0x7fffffff;
  if (row < np) {
    if (row == p) {
      retired[row] = stamp;
      pivrows[node * NBP + jj] = p;
    } else if (retired[row] != stamp) {
      v2 a = M[row + (long)c * np];
      v2 l = cmul(a, rinv);
      M[row + (long)c * np] = l;
      for (int q = 1; q < width; ++q) {
        v2 m = M[row + (long)(c + q) * np];
        v2 u = upiv[q];
        m.x -= l.x * u.x - l.y * u.y;
        m.y -= l.x * u.y + l.y * u.x;
        M[row + (long)(c + q) * np] = m;
        if (q == 1) {
          cand = (double)m.x * m.x + (double)m.y * m.y;
          crow = row;
        }
      }
    }
  }
  if (jj + 1 < gend) {  // at a group's last column the group update leaves the candidates
    block_argmax(cand, crow, sv, sr);
    if (t == 0) {
      pval_out[node * maxwg + blockIdx.x] = cand;
      prow_out[node * maxwg + blockIdx.x] = crow;
    }
  }
}

// Rows of U of the group's pivots in the panel columns k+gend .. k+w-1 (nu of them) into Us:
// forward substitution with the unit-lower PG x PG block of the group's multipliers, from
// the pivot rows as the column steps left them (updated by earlier groups only).
template <typename T>
__device__ void group_u_rows(const typename V2<T>::t* __restrict__ M, int np, int k, int g0,
                             int ng, int gend, int nu, const int* __restrict__ prows,
                             typename V2<T>::t (*Ls)[PG], typename V2<T>::t (*Us)[NBP]) {
  typedef typename V2<T>::t v2;
  const int t = threadIdx.x;
  for (int e = t; e < ng * ng; e += RPW) {
    const int j = e % ng, i = e / ng;
    Ls[j][i] = M[prows[j] + (long)(k + g0 + i) * np];
  }
  for (int e = t; e < ng * nu; e += RPW) {
    const int j = e % ng, q = e / ng;
    Us[j][q] = M[prows[j] + (long)(k + gend + q) * np];
  }
  __syncthreads();
  if (t < nu) {
    for (int j = 1; j < ng; ++j) {
      v2 u = Us[j][t];
      for (int i = 0; i < j; ++i) {
        const v2 l = Ls[j][i], v = Us[i][t];
        u.x -= l.x * v.x - l.y * v.y;
        u.y -= l.x * v.y + l.y * v.x;
      }
      Us[j][t] = u;
    }
  }
  __syncthreads();
}

// End of a group of column steps (columns k+g0 .. k+gend-1): every active row (not a pivot
// of this panel) gets M[r, c] -= sum_i L[r, k+g0+i] U[i, c] over the later panel columns
// c >= k+gend, then the workgroup leaves its pivot candidates for column k+gend.  The pivot
// rows themselves are left as they are (other workgroups read them here); the next launch
// writes their U values.
template <typename T>
__global__ __launch_bounds__(RPW) void panel_group_kernel(
    typename V2<T>::t* __restrict__ M, int np, int k, int w, int g0, int gend, int maxwg,
    double* pval_out, int* prow_out, const int* __restrict__ retired,
    const int* __restrict__ pivrows) {
  typedef typename V2<T>::t v2;
  __shared__ v2 Ls[PG][PG];
  __shared__ v2 Us[PG][NBP];
  __shared__ int sp[PG];
  __shared__ double sv[RPW];
  __shared__ int sr[RPW];
  const int node = blockIdx.y;
  const int t = threadIdx.x;
  M += (long)node * np * np;
  retired += node * np;
  const int ng = gend - g0, nu = w - gend;
  if (t < ng) sp[t] = pivrows[node * NBP + g0 + t];
  __syncthreads();
  group_u_rows<T>(M, np, k, g0, ng, gend, nu, sp, Ls, Us);
  const int row = k + blockIdx.x * RPW + t;
  double cand = -1.0;
  int crow = 0x7fffffff;
  if (row < np && retired[row] != k + 1) {
    v2 l[PG];
#pragma unroll
    for (int i = 0; i < PG; ++i)
      l[i] = (i < ng) ? M[row + (long)(k + g0 + i) * np] : v2{0, 0};
    for (int q = 0; q < nu; ++q) {
      v2 m = M[row + (long)(k + gend + q) * np];
#pragma unroll
      for (int i = 0; i < PG; ++i) {
        const v2 u = Us[i][q];
        m.x -= l[i].x * u.x - l[i].y * u.y;
        m.y -= l[i].x * u.y + l[i].y * u.x;
      }
      M[row + (long)(k + gend + q) * np] = m;
      if (q == 0) {
        cand = (double)m.x * m.x + (double)m.y * m.y;
        crow = row;
      }
    }
  }
  block_argmax(cand, crow, sv, sr);
  if (t == 0) {
    pval_out[node * maxwg + blockIdx.x] = cand;
    prow_out[node * maxwg + blockIdx.x] = crow;
  }
}

// One workgroup per node: the group's pivot rows get their rows of U in the later panel
// columns (the same forward substitution as panel_group_kernel).
template <typename T>
__global__ __launch_bounds__(RPW) void panel_group_pivots_kernel(
    typename V2<T>::t* __restrict__ M, int np, int k, int w, int g0, int gend,
    const int* __restrict__ pivrows) {
  typedef typename V2<T>::t v2;
  __shared__ v2 Ls[PG][PG];
  __shared__ v2 Us[PG][NBP];
  __shared__ int sp[PG];
  const int node = blockIdx.y;
  const int t = threadIdx.x;
  M += (long)node * np * np;
  const int ng = gend - g0, nu = w - gend;
  if (t < ng) sp[t] = pivrows[node * NBP + g0 + t];
  __syncthreads();
  group_u_rows<T>(M, np, k, g0, ng, gend, nu, sp, Ls, Us);
  for (int e = t; e < ng * nu; e += RPW) {
    const int j = e % ng, q = e / ng;
    M[sp[j] + (long)(k + gend + q) * np] = Us[j][q];
  }
}

// Short panels (at most GT * R rows from the panel start down): one workgroup per node runs
// all column steps of a group in one launch, its rows of the group's columns held in
// registers (thread t owns rows k + t + i GT, i < R).  The arithmetic and the pivot choice
// (largest |.|^2, ties to the lower row) are those of panel_step_kernel, so the factors are
// the same; a group costs one launch instead of one per column.  Per column each wave reduces
// its candidates with lane shuffles and leaves its best row's group values in LDS; after one
// barrier every thread reduces the per-wave candidates itself and reads the pivot row from
// the winning wave's slot.  The slots alternate between columns, so that one barrier per
// column orders every LDS write after the reads of two columns before.
template <typename T>
struct ShortPanel;
template <>
struct ShortPanel<float> {
  static constexpr int R = 2;
};
template <>
struct ShortPanel<double> {
  static constexpr int R = 1;
};
constexpr int GT = 1024;     // threads of the short-panel kernel
constexpr int GW = GT / 64;  // its waves

template <typename T>
__global__ __launch_bounds__(GT) void panel_group_short_kernel(
    typename V2<T>::t* __restrict__ M, int np, int k, int g0, int gend, int* __restrict__ retired,
    int* __restrict__ pivrows, int* flag) {
  typedef typename V2<T>::t v2;
  constexpr int R = ShortPanel<T>::R;
  __shared__ double sv[2][GW];
  __shared__ int sr[2][GW];
  __shared__ v2 srow[2][GW][PG];  // each wave's best row in the group's columns
  __shared__ v2 zrow[PG];         // pivot row after an exactly zero column
  const int node = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  M += (long)node * np * np;
  retired += node * np;
  const int stamp = k + 1;
  const int ng = gend - g0;
  v2 x[R][PG];
  bool act[R];
  int row[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    row[i] = k + t + i * GT;
    const bool ok = row[i] < np;
    act[i] = ok && retired[row[i]] != stamp;
#pragma unroll
    for (int q = 0; q < PG; ++q)
      x[i][q] = (ok && q < ng) ? M[row[i] + (long)(k + g0 + q) * np] : v2{0, 0};
  }
  for (int j = 0; j < ng; ++j) {
    const int b = j & 1;
    double v = -1.0;
    int r = 0x7fffffff;
    v2 xj[R];  // column j of the owned rows
#pragma unroll
    for (int i = 0; i < R; ++i) {
      xj[i] = x[i][0];
#pragma unroll
      for (int q = 1; q < PG; ++q)
        if (q == j) xj[i] = x[i][q];
      if (act[i]) argmax_merge(v, r, (double)xj[i].x * xj[i].x + (double)xj[i].y * xj[i].y, row[i]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(v, off);
      const int orow = __shfl_xor(r, off);
      argmax_merge(v, r, ov, orow);
    }
#pragma unroll
    for (int i = 0; i < R; ++i)
      if (act[i] && row[i] == r) {
#pragma unroll
        for (int q = 0; q < PG; ++q) srow[b][wave][q] = x[i][q];
      }
    if (lane == 0) {
      sv[b][wave] = v;
      sr[b][wave] = r;
    }
    __syncthreads();
    // every wave reduces the GW per-wave candidates itself: lane l < GW takes wave l's, then
    // lane shuffles (the merge order does not matter: larger value, then lower row)
    double bv = -1.0;
    int br = 0x7fffffff;
    if (lane < GW) {
      bv = sv[b][lane];
      br = sr[b][lane];
    }
#pragma unroll
    for (int off = GW / 2; off > 0; off >>= 1) {
      const double ov = __shfl_xor(bv, off);
      const int orow = __shfl_xor(br, off);
      argmax_merge(bv, br, ov, orow);
    }
    bv = __shfl(bv, 0);
    br = __shfl(br, 0);
    // the winning wave holds the pivot row in its slot: rows k + t + i GT sit in wave
    // ((br - k) mod GT) / 64
    const int bw = (br >= k && br < np) ? ((br - k) % GT) >> 6 : 0;
    const int c = k + g0 + j;
    const bool bad = !(bv > 0.0) || br < k || br >= np;  // zero column or non-finite values
    const int p = bad ? c : br;
    const v2* u = srow[b][bw];
    if (bad) {  // uniform: the pivot row is row c, owned by thread c - k
      if (t == c - k) {
#pragma unroll
        for (int q = 0; q < PG; ++q) zrow[q] = x[0][q];
      }
      __syncthreads();
      u = zrow;
    }
    const v2 rinv = bad ? v2{0, 0} : crecip(u[j]);
    if (t == 0) {
      pivrows[node * NBP + g0 + j] = p;
      if (bad && flag) atomicCAS(flag, 0, c + 1);
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      if (row[i] == p) {
        act[i] = false;
        retired[p] = stamp;
      }
      if (act[i]) {
        const v2 l = cmul(xj[i], rinv);
#pragma unroll
        for (int q = 0; q < PG; ++q) {
          if (q == j) x[i][q] = l;
          if (q > j && q < ng) {
            const v2 uq = u[q];
            x[i][q].x -= l.x * uq.x - l.y * uq.y;
            x[i][q].y -= l.x * uq.y + l.y * uq.x;
          }
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < R; ++i) {
#pragma unroll
    for (int q = 0; q < PG; ++q)
      if (row[i] < np && q < ng) M[row[i] + (long)(k + g0 + q) * np] = x[i][q];
  }
}

// One workgroup per node: the LAPACK-order swap sequence of the panel, simulated on the set
// of affected positions (the panel's top rows and the pivot rows below them), gives a list
// of row moves (dst <- src) and the same moves applied to perm.  Slots: position k + i is
// slot i (i < w); the pivot rows below the panel get slots w, w+1, ...
__global__ __launch_bounds__(128) void panel_moves_kernel(int np, int k, int w,
                                                          const int* pivrows, int* moves,
                                                          int* perm) {
  __shared__ int slot_pos[2 * NBP];   // position held by each slot
  __shared__ int content[2 * NBP];    // original slot whose row sits at this slot now
  __shared__ int where_[2 * NBP];     // current slot of each original slot
  __shared__ int srcp[2 * NBP];
  __shared__ int pslot[NBP];
  __shared__ int s_cnt;
  const int node = blockIdx.x;
  const int t = threadIdx.x;
  const int* pr = pivrows + node * NBP;
  int* pm = perm + (long)node * np;
  if (t == 0) {
    int cnt = w;
    for (int jj = 0; jj < w; ++jj) {
      int p = pr[jj];
      if (p >= k + w) {
        slot_pos[cnt] = p;
        pslot[jj] = cnt++;
      } else {
        pslot[jj] = p - k;
      }
    }
    s_cnt = cnt;
  }
  __syncthreads();
  const int cnt = s_cnt;
  if (t < w) slot_pos[t] = k + t;
  if (t < cnt) {
    content[t] = t;
    where_[t] = t;
  }
  __syncthreads();
  if (t == 0) {
    for (int jj = 0; jj < w; ++jj) {
      int src = pslot[jj];
      if (src < 0 || src >= cnt) continue;  // only after a reported zero pivot
      int q = where_[src];
      int a = content[jj], b = content[q];
      content[jj] = b;
      content[q] = a;
      where_[b] = jj;
      where_[a] = q;
    }
  }
  __syncthreads();
  int* mv = moves + node * (4 * NBP + 1);
  if (t < cnt) srcp[t] = pm[slot_pos[content[t]]];
  __syncthreads();
  if (t < cnt) {
    mv[1 + 2 * t] = slot_pos[t];
    mv[2 + 2 * t] = slot_pos[content[t]];
    pm[slot_pos[t]] = srcp[t];
  }
  if (t == 0) mv[0] = cnt;
}

constexpr int SWAP_COLS = 32;
template <typename T>
__global__ __launch_bounds__(256) void laswp_kernel(typename V2<T>::t* __restrict__ M, int np,
                                                   const int* moves) {
  typedef typename V2<T>::t v2;
  const int node = blockIdx.y;
  M += (long)node * np * np;
  const int* mv = moves + node * (4 * NBP + 1);
  const int nm = mv[0];
  const int a = threadIdx.x & 127, half = threadIdx.x >> 7;
  const int c0 = blockIdx.x * SWAP_COLS;
  v2 vals[SWAP_COLS / 2];
  int dst = 0, src = 0;
  if (a < nm) {
    dst = mv[1 + 2 * a];
    src = mv[2 + 2 * a];
#pragma unroll
    for (int q = 0; q < SWAP_COLS / 2; ++q) {
      int c = c0 + half + 2 * q;
      if (c < np) vals[q] = M[src + (long)c * np];
    }
  }
  __syncthreads();
  if (a < nm) {
#pragma unroll
    for (int q = 0; q < SWAP_COLS / 2; ++q) {
      int c = c0 + half + 2 * q;
      if (c < np) M[dst + (long)c * np] = vals[q];
    }
  }
}

// Inverse of the unit-lower w x w diagonal block L11 of the panel at column k (w <= 64) for
// every node (one workgroup per node), into Linv (64 x 64 per node, ld 64; identity past w):
// forward substitution on the identity in LDS.
template <typename T>
__global__ __launch_bounds__(256) void l11_inverse_kernel(const typename V2<T>::t* __restrict__ M,
                                                          int np, int k, int w,
                                                          typename V2<T>::t* __restrict__ Linv) {
  typedef typename V2<T>::t v2;
  __shared__ v2 L[NBP][NBP + 1];
  __shared__ v2 X[NBP][NBP + 1];
  const int node = blockIdx.x;
  const int t = threadIdx.x;
  M += (long)node * np * np;
  for (int e = t; e < NBP * NBP; e += 256) {
    const int r = e % NBP, c = e / NBP;
    L[r][c] = (r < w && c < w && r > c) ? M[k + r + (long)(k + c) * np] : v2{0, 0};
    X[r][c] = v2{T(r == c ? 1 : 0), T(0)};
  }
  __syncthreads();
  for (int r = 0; r < NBP - 1; ++r) {  // row i -= L[i][r] * row r, for i > r (columns c <= r)
    const int rows = NBP - 1 - r;
    for (int e = t; e < rows * (r + 1); e += 256) {
      const int i = r + 1 + e % rows, c = e / rows;
      const v2 l = L[i][r], x = X[r][c];
      X[i][c].x -= l.x * x.x - l.y * x.y;
      X[i][c].y -= l.x * x.y + l.y * x.x;
    }
    __syncthreads();
  }
  v2* out = Linv + (long)node * NBP * NBP;
  for (int e = t; e < NBP * NBP; e += 256) out[e] = X[e % NBP][e / NBP];
}

// Staging copy of the panel's rows k .. k+w-1 of columns c0 .. c1-1 into U (ld 64 per node).
template <typename T>
__global__ void rows_copy_kernel(const typename V2<T>::t* __restrict__ M, int np, int k, int w,
                                 int c0, int c1, typename V2<T>::t* __restrict__ U) {
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long cols = c1 - c0;
  if (idx >= (long)NBP * cols) return;
  const int node = blockIdx.y;
  const int r = (int)(idx % NBP), c = (int)(idx / NBP);
  if (r >= w) return;
  U[(long)node * NBP * np + r + (long)c * NBP] = M[(long)node * np * np + k + r + (c0 + c) * (long)np];
}

__global__ void perm_init_kernel(int* perm, int np, int nc) {
  long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx < (long)np * nc) perm[idx] = (int)(idx % np);
}
__global__ void perm_invert_kernel(const int* perm, int* pinv, int np, int nc) {
  long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx < (long)np * nc) {
    long node = idx / np;
    pinv[node * np + perm[idx]] = (int)(idx % np);
  }
}

// C = ar op(A) op(B) + br C in the factor precision.
template <typename T>
void gemm_t(hipStream_t s, int opA, int opB, int M, int N, int K, double ar,
            const typename V2<T>::t* A, long lda, const typename V2<T>::t* B, long ldb, double br,
            typename V2<T>::t* C, long ldc, const Batch& bt) {
  if constexpr (sizeof(T) == 8)
    zgemm(s, opA, opB, M, N, K, zmake(ar, 0), A, lda, B, ldb, zmake(br, 0), C, ldc, bt);
  else
    cgemm(s, opA, opB, M, N, K, make_float2((float)ar, 0), A, lda, B, ldb,
          make_float2((float)br, 0), C, ldc, bt);
}

// M[r0:r0+rows, c0:c0+cols] -= M[r0:r0+rows, k:k+kw] * M[k:k+kw, c0:c0+cols] for every node.
template <typename T>
void gemm_update(hipStream_t s, typename V2<T>::t* M, int np, int nc, int r0, int rows, int c0,
                 int cols, int k, int kw);
template <>
void gemm_update<double>(hipStream_t s, zd* M, int np, int nc, int r0, int rows, int c0, int cols,
                         int k, int kw) {
  Batch b;
  b.n1 = nc;
  b.sA1 = b.sB1 = b.sC1 = (long)np * np;
  zgemm(s, OP_N, OP_N, rows, cols, kw, zmake(-1, 0), M + r0 + (long)k * np, np,
        M + k + (long)c0 * np, np, zmake(1, 0), M + r0 + (long)c0 * np, np, b);
}
template <>
void gemm_update<float>(hipStream_t s, zf* M, int np, int nc, int r0, int rows, int c0, int cols,
                        int k, int kw) {
  Batch b;
  b.n1 = nc;
  b.sA1 = b.sB1 = b.sC1 = (long)np * np;
  cgemm(s, OP_N, OP_N, rows, cols, kw, make_float2(-1, 0), M + r0 + (long)k * np, np,
        M + k + (long)c0 * np, np, make_float2(1, 0), M + r0 + (long)c0 * np, np, b);
}

template <typename T>
void lu_factor(hipStream_t s, typename V2<T>::t* M, int np, int nc, LuWork& w) {
  const int maxwg = (np + RPW - 1) / RPW;
  fill_zero(s, w.retired, sizeof(int) * (size_t)nc * np);
  fill_zero(s, w.flag, sizeof(int));
  {
    long tot = (long)np * nc;
    hipLaunchKernelGGL(perm_init_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, w.perm, np, nc);
    FEAST_LAUNCH_CHECK();
  }
  // Factor one 64-wide panel starting at column kp (pivot search, implicit-pivoting column
  // steps, row moves applied across all columns).
  auto factor_panel = [&](int kp, int width) {
    const int nwg = (np - kp + RPW - 1) / RPW;
    const bool short_panel = !w.column_steps && np - kp <= GT * ShortPanel<T>::R;
    double* pv[2] = {w.pval, w.pval + nc * maxwg};
    int* pr[2] = {w.prow, w.prow + nc * maxwg};
    if (!short_panel) {
      hipLaunchKernelGGL((panel_search_kernel<T>), dim3(nwg, nc), dim3(RPW), 0, s, M, np, kp,
                         pv[0], pr[0], maxwg);
      FEAST_LAUNCH_CHECK();
    }
    for (int g0 = 0; g0 < width; g0 += PG) {
      const int gend = std::min(width, g0 + PG);
      if (short_panel) {
        hipLaunchKernelGGL((panel_group_short_kernel<T>), dim3(nc), dim3(GT), 0, s, M, np, kp,
                           g0, gend, w.retired, w.pivrows, w.flag);
        FEAST_LAUNCH_CHECK();
      } else {
        for (int jj = g0; jj < gend; ++jj) {
          hipLaunchKernelGGL((panel_step_kernel<T>), dim3(nwg, nc), dim3(RPW), 0, s, M, np, kp,
                             width, jj, gend, nwg, maxwg, pv[jj & 1], pr[jj & 1],
                             pv[(jj + 1) & 1], pr[(jj + 1) & 1], w.retired, w.pivrows, w.flag);
          FEAST_LAUNCH_CHECK();
        }
      }
      if (gend < width) {  // later panel columns: the group's rank-PG update, then its U rows
        hipLaunchKernelGGL((panel_group_kernel<T>), dim3(nwg, nc), dim3(RPW), 0, s, M, np, kp,
                           width, g0, gend, maxwg, pv[gend & 1], pr[gend & 1], w.retired,
                           w.pivrows);
        FEAST_LAUNCH_CHECK();
        hipLaunchKernelGGL((panel_group_pivots_kernel<T>), dim3(1, nc), dim3(RPW), 0, s, M, np,
                           kp, width, g0, gend, w.pivrows);
        FEAST_LAUNCH_CHECK();
      }
    }
    hipLaunchKernelGGL(panel_moves_kernel, dim3(nc), dim3(128), 0, s, np, kp, width, w.pivrows,
                       w.moves, w.perm);
    FEAST_LAUNCH_CHECK();
    hipLaunchKernelGGL((laswp_kernel<T>), dim3((np + SWAP_COLS - 1) / SWAP_COLS, nc), dim3(256),
                       0, s, M, np, w.moves);
    FEAST_LAUNCH_CHECK();
  };
  // U12 = L11^{-1} M[kp:kp+width, c0:c1] with the unit-lower diagonal block of panel kp: the
  // block's explicit inverse (computed once per panel, l11_inverse) times a staging copy of the
  // rows, one matrix-core product over all nodes.
  typedef typename V2<T>::t v2;
  v2* u12 = (v2*)w.u12;
  // inverse of sub-panel q's L11 (q < NSUB within the current outer panel)
  auto linv = [&](int q) { return (v2*)w.linv + (long)q * nc * NBP * NBP; };
  auto l11_inverse = [&](int q, int kp, int width) {
    hipLaunchKernelGGL((l11_inverse_kernel<T>), dim3(nc), dim3(256), 0, s, M, np, kp, width,
                       linv(q));
    FEAST_LAUNCH_CHECK();
  };
  auto trsm = [&](int q, int kp, int width, int c0, int c1) {
    const long tot = (long)NBP * (c1 - c0);
    hipLaunchKernelGGL((rows_copy_kernel<T>), dim3((unsigned)((tot + 255) / 256), nc), dim3(256),
                       0, s, M, np, kp, width, c0, c1, u12);
    FEAST_LAUNCH_CHECK();
    Batch b;
    b.n1 = nc;
    b.sA1 = (long)NBP * NBP;
    b.sB1 = (long)NBP * np;
    b.sC1 = (long)np * np;
    gemm_t<T>(s, OP_N, OP_N, width, c1 - c0, width, 1.0, linv(q), NBP, u12, NBP, 0.0,
              M + kp + (long)c0 * np, np, b);
  };
  // Outer panels of NSUB 64-wide sub-panels: the trailing update then contracts over
  // NSUB * 64 columns at once (1 / NSUB of the read-modify-write traffic of 64-deep updates).
  // Inside an outer panel the sub-panels are factored right-looking over the panel's own
  // columns; the panel's block rows of U for the trailing columns follow by block forward
  // substitution.
  for (int k = 0; k < np; k += NSUB * NBP) {
    int kw[NSUB];
    int W = 0;
    for (int q = 0; q < NSUB; ++q) {
      kw[q] = std::max(0, std::min(NBP, np - k - W));
      W += kw[q];
    }
    for (int q = 0, kq = k; q < NSUB && kw[q] > 0; kq += kw[q], ++q) {
      factor_panel(kq, kw[q]);
      const int e = kq + kw[q];  // first column of the outer panel not yet factored
      if (e < np) l11_inverse(q, kq, kw[q]);
      if (e < k + W) {
        trsm(q, kq, kw[q], e, k + W);
        gemm_update<T>(s, M, np, nc, e, np - e, e, k + W - e, kq, kw[q]);
      }
    }
    const int c = k + W;
    if (c < np) {
      for (int q = 0, kq = k; q < NSUB && kw[q] > 0; kq += kw[q], ++q) {
        trsm(q, kq, kw[q], c, np);
        const int e = kq + kw[q];
        if (e < c) gemm_update<T>(s, M, np, nc, e, c - e, c, np - c, kq, kw[q]);
      }
      gemm_update<T>(s, M, np, nc, c, np - c, c, np - c, k, W);
    }
  }
  long tot = (long)np * nc;
  hipLaunchKernelGGL(perm_invert_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, w.perm, w.pinv,
                     np, nc);
  FEAST_LAUNCH_CHECK();
}

}  // namespace

size_t lu_work_bytes(int np, int nc) {
  const int maxwg = (np + RPW - 1) / RPW;
  size_t b = 0;
  b += sizeof(int) * (size_t)nc * np;           // retired
  b += sizeof(double) * 2 * (size_t)nc * maxwg;  // pval
  b += sizeof(int) * 2 * (size_t)nc * maxwg;     // prow
  b += sizeof(int) * (size_t)nc * NBP;           // pivrows
  b += sizeof(int) * (size_t)nc * (4 * NBP + 1); // moves
  b += 2 * sizeof(int) * (size_t)nc * np;        // perm, pinv
  b += 256;                                      // flag
  b += sizeof(double2) * (size_t)nc * NSUB * NBP * NBP;  // L11 inverses (FP64 size)
  b += sizeof(double2) * (size_t)nc * NBP * np;  // U12 staging
  return b + 10 * 256;                           // alignment slack
}

void lu_work_carve(LuWork& w, void* base, int np, int nc) {
  const int maxwg = (np + RPW - 1) / RPW;
  char* p = (char*)base;
  auto take = [&](size_t bytes) {
    char* r = p;
    p += (bytes + 255) & ~(size_t)255;
    return (void*)r;
  };
  w.pval = (double*)take(sizeof(double) * 2 * (size_t)nc * maxwg);
  w.retired = (int*)take(sizeof(int) * (size_t)nc * np);
  w.prow = (int*)take(sizeof(int) * 2 * (size_t)nc * maxwg);
  w.pivrows = (int*)take(sizeof(int) * (size_t)nc * NBP);
  w.moves = (int*)take(sizeof(int) * (size_t)nc * (4 * NBP + 1));
  w.perm = (int*)take(sizeof(int) * (size_t)nc * np);
  w.pinv = (int*)take(sizeof(int) * (size_t)nc * np);
  w.flag = (int*)take(256);
  w.linv = take(sizeof(double2) * (size_t)nc * NSUB * NBP * NBP);
  w.u12 = take(sizeof(double2) * (size_t)nc * NBP * np);
}

void shift_matrices(hipStream_t s, const void* A, long lda, int is_real, int n, int np,
                    const zd* z_dev, int nc, zd* M, int* flag, const void* B, long ldb) {
  long tot = (long)np * np;
  hipLaunchKernelGGL((shift_kernel<double>), dim3((tot + 255) / 256), dim3(256), 0, s, A, lda, B,
                     ldb, is_real, n, np, z_dev, nc, M, flag);
  FEAST_LAUNCH_CHECK();
}
void shift_matrices_f32(hipStream_t s, const void* A, long lda, int is_real, int n, int np,
                        const zd* z_dev, int nc, zf* M, int* flag, const void* B, long ldb) {
  long tot = (long)np * np;
  hipLaunchKernelGGL((shift_kernel<float>), dim3((tot + 255) / 256), dim3(256), 0, s, A, lda, B,
                     ldb, is_real, n, np, z_dev, nc, M, flag);
  FEAST_LAUNCH_CHECK();
}

void lu_factor_f64(hipStream_t s, zd* M, int np, int nc, LuWork& w) { lu_factor<double>(s, M, np, nc, w); }
void lu_factor_f32(hipStream_t s, zf* M, int np, int nc, LuWork& w) { lu_factor<float>(s, M, np, nc, w); }

}  // namespace feast
