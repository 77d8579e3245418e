// Dense FP64 linear algebra on gfx950 for the refinement pre-computation
// (Algorithm 1 steps 1-4) and the Woodbury solve:
//  * row interpolative decomposition (Definition 3.1) of a tall sketch:
//    skeleton rows by tournament selection (blockwise pivoted Gram-Schmidt,
//    then among the survivors), or by one cooperative kernel with a grid
//    barrier per pivot for wide sketches; interpolation P = C C_J^{-1};
//  * tall-skinny products A^T B (W = I + R X, z = R y), Y -= X W;
//  * Gauss-Jordan inverse with partial pivoting of the small Woodbury
//    operator W (always FP64);
//  * blocked right-looking LU without pivoting of A_pp with the trailing
//    update on the FP64 matrix cores, and blocked triangular solves.
#include <hip/hip_cooperative_groups.h>

#include "dev_gj.h"
#include "dev_reduce.h"
#include "kernels.h"

namespace cg = cooperative_groups;

namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));
inline unsigned blocks(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// ================================================================ row ID
struct RowIdArgs {
  const double* Y;
  int64_t m;
  int ncols;
  double tol2;         // tol^2 (squared row norms are compared)
  int kmax;
  int rows_per;        // rows owned by one workgroup
  int lds_rows;        // 1 if the owned rows live in LDS
  double* Yw;          // global working copy (used when lds_rows == 0)
  int* J;
  double* C;           // m x kmax row-major
  double* slot_norm;   // 2 * G
  int64_t* slot_idx;   // 2 * G
  double* slot_vec;    // 2 * G * ncols
  int* out_k;
};

__device__ __forceinline__ bool better(double v1, int64_t i1, double v2, int64_t i2) {
  if (i1 < 0) return false;
  if (i2 < 0) return true;
  return (v1 > v2) || (v1 == v2 && i1 < i2);
}

__global__ __launch_bounds__(256) void rowid_kernel(RowIdArgs a) {
  extern __shared__ double sh[];
  cg::grid_group grid = cg::this_grid();
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int NC = a.ncols;
  const int64_t r0 = (int64_t)g * a.rows_per;
  const int nloc = (int)max<int64_t>(0, min<int64_t>(a.rows_per, a.m - r0));
  const int stride = a.lds_rows ? NC + 1 : NC;
  double* rows = a.lds_rows ? sh : a.Yw + r0 * NC;
  double* q = sh + (a.lds_rows ? (size_t)a.rows_per * (NC + 1) : 0);
  double* rn = q + NC;                 // rows_per squared norms (-1 = selected)
  double* redv = rn + a.rows_per;      // 256
  int64_t* redi = (int64_t*)(redv + 256);  // 256
  int* redb = (int*)(redi + 256);      // 256

  for (int idx = tid; idx < nloc * NC; idx += 256) {
    const int i = idx / NC, c = idx - i * NC;
    rows[i * stride + c] = a.Y[(r0 + i) * NC + c];
  }
  __syncthreads();
  for (int i = tid; i < nloc; i += 256) {
    double s = 0;
    for (int c = 0; c < NC; ++c) s += rows[i * stride + c] * rows[i * stride + c];
    rn[i] = s;
  }
  __syncthreads();
  double nrm0 = 0.0;
  int k = 0;
  for (int step = 0; step < a.kmax; ++step) {
    // ---- local argmax
    double bv = -1.0;
    int64_t bi = -1;
    for (int i = tid; i < nloc; i += 256)
      if (rn[i] >= 0.0 && better(rn[i], r0 + i, bv, bi)) { bv = rn[i]; bi = r0 + i; }
    redv[tid] = bv;
    redi[tid] = bi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w && better(redv[tid + w], redi[tid + w], redv[tid], redi[tid])) {
        redv[tid] = redv[tid + w];
        redi[tid] = redi[tid + w];
      }
      __syncthreads();
    }
    const int par = step & 1;
    const int64_t lbest = redi[0];
    if (tid == 0) {
      a.slot_norm[par * G + g] = redv[0];
      a.slot_idx[par * G + g] = lbest;
    }
    for (int c = tid; c < NC; c += 256)
      a.slot_vec[((size_t)par * G + g) * NC + c] = (lbest >= 0) ? rows[(lbest - r0) * stride + c] : 0.0;
    __threadfence();
    grid.sync();
    // ---- global argmax (identical in every workgroup)
    bv = -1.0;
    bi = -1;
    int bb = -1;
    for (int s = tid; s < G; s += 256) {
      const double v = a.slot_norm[par * G + s];
      const int64_t i = a.slot_idx[par * G + s];
      if (better(v, i, bv, bi)) { bv = v; bi = i; bb = s; }
    }
    __syncthreads();
    redv[tid] = bv;
    redi[tid] = bi;
    redb[tid] = bb;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w && better(redv[tid + w], redi[tid + w], redv[tid], redi[tid])) {
        redv[tid] = redv[tid + w];
        redi[tid] = redi[tid + w];
        redb[tid] = redb[tid + w];
      }
      __syncthreads();
    }
    const double gv = redv[0];
    const int64_t gi = redi[0];
    const int gb = redb[0];
    if (step == 0) nrm0 = gv;
    if (gi < 0 || !(gv > a.tol2 * nrm0) || !(gv > 0.0)) break;
    for (int c = tid; c < NC; c += 256) q[c] = a.slot_vec[((size_t)par * G + gb) * NC + c];
    __syncthreads();
    if (tid == 0) {
      double s = 0;
      for (int c = 0; c < NC; ++c) s += q[c] * q[c];
      redv[0] = 1.0 / sqrt(s);
    }
    __syncthreads();
    const double inv = redv[0];
    for (int c = tid; c < NC; c += 256) q[c] *= inv;
    __syncthreads();
    if (g == 0 && tid == 0) a.J[step] = (int)gi;
    // ---- project every owned row against q (two passes) and record the coefficient
    for (int i = tid; i < nloc; i += 256) {
      double* row = rows + (size_t)i * stride;
      double cf = 0;
      for (int pass = 0; pass < 2; ++pass) {
        double d = 0;
        for (int c = 0; c < NC; ++c) d += row[c] * q[c];
        for (int c = 0; c < NC; ++c) row[c] -= d * q[c];
        cf += d;
      }
      a.C[(r0 + i) * a.kmax + step] = cf;
      if (rn[i] >= 0.0) {
        double s = 0;
        for (int c = 0; c < NC; ++c) s += row[c] * row[c];
        rn[i] = (r0 + i == gi) ? -1.0 : s;
      }
    }
    __syncthreads();
    k = step + 1;
  }
  if (g == 0 && tid == 0) *a.out_k = k;
}

// ------------------------------------------- row ID by tournament selection
// For sketches of at most 64 columns.  Stage 0 cuts the rows into blocks of
// 512; every block runs pivoted Gram-Schmidt on its rows (one row in the
// registers of each thread) and keeps the rows whose residual norm exceeds
// the threshold tol * (largest row norm of the whole sketch), at most kmax
// of them.  Each later stage does the same on the concatenated selections of
// the previous one until one block is left; its selections, in order, are
// the skeleton rows J.  Selection needs residual norms only to choose
// pivots, so one projection pass per pivot suffices there; the basis Q of
// Y(J, :) and the coefficients C = Y Q^T of every row follow with full
// accuracy, and the largest residual |y_i - C_i Q| certifies the result (the
// caller falls back to the one-pass kernel above if a row was missed).
constexpr int SEL_ROWS = 512;
constexpr int SEL_NC = 64;

// Largest squared row norm of Y (m x nc, row-major), as ordered bits.
__global__ __launch_bounds__(256) void rowid_maxnorm_kernel(const double* __restrict__ Y, int64_t m, int nc,
                                                            unsigned long long* __restrict__ out) {
  double best = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
    double s = 0.0;
    for (int c = 0; c < nc; ++c) s += Y[i * nc + c] * Y[i * nc + c];
    best = fmax(best, s);
  }
  best = wave_max_nonneg(best);
  if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(best));
}

__global__ __launch_bounds__(SEL_ROWS) void rowid_select_kernel(const double* __restrict__ Y, int64_t m, int nc,
                                                                const int* __restrict__ prev_idx,
                                                                const int* __restrict__ prev_cnt, int nprev, int kmax,
                                                                double tol2,
                                                                const unsigned long long* __restrict__ nrm0,
                                                                int* __restrict__ out_idx, int* __restrict__ out_cnt) {
  __shared__ double q[SEL_NC];
  __shared__ double wkey[SEL_ROWS / 64];
  __shared__ int pref[1025];
  const int b = blockIdx.x, t = threadIdx.x, lane = t & 63, w = t >> 6;
  const double thresh = tol2 * __longlong_as_double((long long)*nrm0);
  // ---- candidate of this thread
  int idx = -1;
  if (!prev_idx) {
    const int64_t i = (int64_t)b * SEL_ROWS + t;
    idx = i < m ? (int)i : -1;
  } else {
    for (int u = t; u < nprev; u += SEL_ROWS) pref[u + 1] = prev_cnt[u];
    __syncthreads();
    if (t == 0) {
      pref[0] = 0;
      for (int u = 1; u <= nprev; ++u) pref[u] += pref[u - 1];
    }
    __syncthreads();
    const int pos = b * SEL_ROWS + t;
    if (pos < pref[nprev]) {
      int lo = 0, hi = nprev - 1;  // last u with pref[u] <= pos
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pref[mid] <= pos) lo = mid; else hi = mid - 1;
      }
      idx = prev_idx[lo * kmax + (pos - pref[lo])];
    }
  }
  double y[SEL_NC];
  double rn = -1.0;
  if (idx >= 0) {
    rn = 0.0;
#pragma unroll
    for (int c = 0; c < SEL_NC; ++c) {
      y[c] = c < nc ? Y[(int64_t)idx * nc + c] : 0.0;
      rn += y[c] * y[c];
    }
  } else {
#pragma unroll
    for (int c = 0; c < SEL_NC; ++c) y[c] = 0.0;
  }
  int k = 0;
  for (; k < kmax; ++k) {
    // ---- pivot: largest residual norm among the candidates
    const double key = wave_max_nonneg(pivot_key_bits<9>(rn, t, rn >= 0.0));
    if (lane == 0) wkey[w] = key;
    __syncthreads();
    double bk = wkey[0];
#pragma unroll
    for (int u = 1; u < SEL_ROWS / 64; ++u) bk = fmax(bk, wkey[u]);
    // the pivot's squared norm (the key, to 2^-43 relative) decides the stop;
    // every thread holds the same key, so the decision is uniform
    if (!(bk > thresh) || !(bk >= 2.2250738585072014e-308)) break;
    const int p = pivot_key_index<9>(bk);
    if (t == p) {
      const double inv = 1.0 / sqrt(rn);
#pragma unroll
      for (int c = 0; c < SEL_NC; ++c) q[c] = y[c] * inv;
      out_idx[b * kmax + k] = idx;
      rn = -1.0;
    }
    __syncthreads();
    // ---- project this candidate against q (one pass) and renew its norm
    if (rn >= 0.0) {
      double d = 0.0;
#pragma unroll
      for (int c = 0; c < SEL_NC; ++c) d += y[c] * q[c];
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < SEL_NC; ++c) {
        y[c] -= d * q[c];
        s += y[c] * y[c];
      }
      rn = s;
    }
  }
  if (t == 0) out_cnt[b] = k;
}

// Orthonormal rows Q (k x nc) of Y(J, :) in pivot order: classical
// Gram-Schmidt with one reorthogonalization, one wave (thread u computes the
// coefficient on q_u, thread c updates column c; every sum in four
// independent partial sums).  k <= 64, nc a multiple of 4.
// The selected rows J (idx[0..*kp)) are copied to Jout and orthonormalized
// in order into Q (k x nc, row-major); k is read on the device.
__global__ __launch_bounds__(64) void rowid_basis_kernel(const double* __restrict__ Y, int nc,
                                                         const int* __restrict__ J, const int* __restrict__ kp,
                                                         int* __restrict__ Jout, double* __restrict__ Q) {
  __shared__ double qs[64][SEL_NC + 1];
  __shared__ double v[SEL_NC], d[64];
  const int c = threadIdx.x;
  const int k = *kp;
  if (c < k) Jout[c] = J[c];
  for (int s = 0; s < k; ++s) {
    if (c < nc) v[c] = Y[(int64_t)J[s] * nc + c];
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
      if (c < s) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        for (int u = 0; u < nc; u += 4) {
          a0 += v[u] * qs[c][u];
          a1 += v[u + 1] * qs[c][u + 1];
          a2 += v[u + 2] * qs[c][u + 2];
          a3 += v[u + 3] * qs[c][u + 3];
        }
        d[c] = (a0 + a1) + (a2 + a3);
      }
      __syncthreads();
      if (c < nc) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int u = 0;
        for (; u + 4 <= s; u += 4) {
          a0 += d[u] * qs[u][c];
          a1 += d[u + 1] * qs[u + 1][c];
          a2 += d[u + 2] * qs[u + 2][c];
          a3 += d[u + 3] * qs[u + 3][c];
        }
        for (; u < s; ++u) a0 += d[u] * qs[u][c];
        v[c] -= (a0 + a1) + (a2 + a3);
      }
      __syncthreads();
    }
    double n0 = 0.0, n1 = 0.0, n2a = 0.0, n3 = 0.0;
    for (int u = 0; u < nc; u += 4) {
      n0 += v[u] * v[u];
      n1 += v[u + 1] * v[u + 1];
      n2a += v[u + 2] * v[u + 2];
      n3 += v[u + 3] * v[u + 3];
    }
    const double n2 = (n0 + n1) + (n2a + n3);
    const double inv = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
    if (c < nc) {
      qs[s][c] = v[c] * inv;
      Q[s * nc + c] = v[c] * inv;
    }
    __syncthreads();
  }
}

// C(i, t) = <y_i, q_t> (row-major, ld kmax) for every row, and the largest
// squared residual |y_i - C_i Q|^2 (ordered bits) in *maxres.  Four threads
// per row (RCW columns each; 64 rows per workgroup): each projection's dot
// product is four partial sums per thread, added over the thread's quad by
// DPP (every lane of the quad gets the same bits), then the quad's columns
// are updated.  Q is staged in LDS with the four column slices of a row
// RCQ doubles apart (2 mod 16), so that the quad's reads hit disjoint banks.
constexpr int RC4 = 4, RCW = SEL_NC / RC4, RCQ = RCW + 2;
static_assert(RCW % 4 == 0 && RCQ % 16 == 2, "row-coefficient layout");
__device__ __forceinline__ double quad_sum(double t) {
  t += dpp_f64<0xB1, 0xf>(t);   // quad_perm [1,0,3,2]
  return t + dpp_f64<0x4E, 0xf>(t);   // quad_perm [2,3,0,1]
}
__global__ __launch_bounds__(256) void rowid_coef_kernel(const double* __restrict__ Y, int64_t m, int nc,
                                                         const double* __restrict__ Q, const int* __restrict__ kp,
                                                         int kmax, double* __restrict__ C,
                                                         unsigned long long* __restrict__ maxres) {
  extern __shared__ double qs[];  // k x (RC4 RCQ): column c of q_s at s RC4 RCQ + (c / RCW) RCQ + c % RCW
  const int k = *kp;
  if (k == 0) return;
  for (int u = threadIdx.x; u < k * SEL_NC; u += 256) {
    const int s = u / SEL_NC, c = u - s * SEL_NC;
    qs[s * (RC4 * RCQ) + (c / RCW) * RCQ + c % RCW] = c < nc ? Q[s * nc + c] : 0.0;
  }
  __syncthreads();
  const int h = threadIdx.x & (RC4 - 1);
  const int64_t i = (int64_t)blockIdx.x * (256 / RC4) + (threadIdx.x >> 2);
  const bool valid = i < m;
  double y[RCW];
#pragma unroll
  for (int c = 0; c < RCW; ++c) {
    const int col = h * RCW + c;
    y[c] = (valid && col < nc) ? Y[i * nc + col] : 0.0;
  }
  for (int s = 0; s < k; ++s) {
    const double* qv = qs + s * (RC4 * RCQ) + h * RCQ;
    double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
#pragma unroll
    for (int c = 0; c < RCW; c += 4) {
      d0 = fma(y[c], qv[c], d0);
      d1 = fma(y[c + 1], qv[c + 1], d1);
      d2 = fma(y[c + 2], qv[c + 2], d2);
      d3 = fma(y[c + 3], qv[c + 3], d3);
    }
    const double d = quad_sum((d0 + d1) + (d2 + d3));
    if (valid && h == 0) C[i * kmax + s] = d;
#pragma unroll
    for (int c = 0; c < RCW; ++c) y[c] -= d * qv[c];
  }
  double r0 = 0.0, r1 = 0.0;
#pragma unroll
  for (int c = 0; c < RCW; c += 2) {
    r0 = fma(y[c], y[c], r0);
    r1 = fma(y[c + 1], y[c + 1], r1);
  }
  double res = quad_sum(r0 + r1);
  for (int off = 32; off > 0; off >>= 1) res = fmax(res, __shfl_xor(res, off));
  if ((threadIdx.x & 63) == 0) atomicMax(maxres, (unsigned long long)__double_as_longlong(res));
}

// C_J(s, t) = C(J[s], t) is lower triangular (row J[s] has no component on
// q_t for t > s).  cj_inv_kernel writes Inv = C_J^{-1} (k x k, row-major,
// lower triangular); rowid_interp_kernel forms P(i, :) = C(i, 0:k) Inv and
// writes it to L(pos[i], col0 + t).  Skeleton rows then get exact unit rows.
__global__ __launch_bounds__(256) void cj_inv_kernel(const double* __restrict__ C, int kmax, int k,
                                                     const int* __restrict__ J, double* __restrict__ inv) {
  extern __shared__ double x[];  // k x k row-major: x[s * k + t] = Inv(s, t)
  const int t = threadIdx.x;
  for (int idx = t; idx < k * k; idx += blockDim.x) x[idx] = 0.0;
  __syncthreads();
  if (t < k) {
    // column t of Inv: C_J x = e_t, forward substitution over s >= t
    for (int s = t; s < k; ++s) {
      double v = (s == t) ? 1.0 : 0.0;
      const double* cs = C + (int64_t)J[s] * kmax;
      for (int u = t; u < s; ++u) v -= cs[u] * x[u * k + t];
      x[s * k + t] = v / cs[s];
    }
  }
  __syncthreads();
  for (int idx = t; idx < k * k; idx += blockDim.x) inv[idx] = x[idx];
}

__global__ __launch_bounds__(256) void rowid_interp_kernel(const double* __restrict__ C, int64_t m, int kmax, int k,
                                                           const double* __restrict__ inv,
                                                           const int* __restrict__ pos, double* __restrict__ L,
                                                           int64_t ldL, int col0) {
  extern __shared__ double iv[];  // k x k
  for (int idx = threadIdx.x; idx < k * k; idx += 256) iv[idx] = inv[idx];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  const double* ci = C + i * kmax;
  const int64_t row = pos ? pos[i] : i;
  for (int t = 0; t < k; ++t) {
    double v = 0.0;
    for (int s = t; s < k; ++s) v += ci[s] * iv[s * k + t];
    L[row + (int64_t)(col0 + t) * ldL] = v;
  }
}

__global__ void rowid_unit_rows_kernel(int k, const int* __restrict__ J, const int* __restrict__ pos,
                                       double* __restrict__ L, int64_t ldL, int col0) {
  const int s = blockIdx.x;
  const int64_t row = pos ? pos[J[s]] : J[s];
  for (int t = threadIdx.x; t < k; t += blockDim.x) L[row + (int64_t)(col0 + t) * ldL] = (t == s) ? 1.0 : 0.0;
}

// ================================================================ A^T B
// Split over row ranges (one workgroup each); per 48 x 48 output tile every
// thread keeps a 3 x 3 block (rows ti + 16 x, columns tj + 16 y) in
// registers while chunks of 32 rows of A and B pass through LDS.
constexpr int TN_CH = 32;  // rows per LDS chunk
constexpr int TN_T = 48;   // output tile edge

__global__ __launch_bounds__(256) void gemm_tn_part_kernel(const double* __restrict__ A, int64_t lda,
                                                           const double* __restrict__ B, int64_t ldb, int64_t M,
                                                           int ka, int kb, int64_t rows_per,
                                                           double* __restrict__ part) {
  __shared__ double As[TN_CH][TN_T + 1];
  __shared__ double Bs[TN_CH][TN_T + 1];
  const int tid = threadIdx.x, ti = tid & 15, tj = tid >> 4;
  const int64_t e0 = (int64_t)blockIdx.x * rows_per;
  const int64_t e1 = min(M, e0 + rows_per);
  const int nout = ka * kb;
  double* pb = part + (int64_t)blockIdx.x * nout;
  for (int ia0 = 0; ia0 < ka; ia0 += TN_T)
    for (int ib0 = 0; ib0 < kb; ib0 += TN_T) {
      double acc[3][3];
#pragma unroll
      for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y) acc[x][y] = 0.0;
      for (int64_t c0 = e0; c0 < e1; c0 += TN_CH) {
        const int cnt = (int)min<int64_t>(TN_CH, e1 - c0);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < TN_CH * TN_T / 256; ++u) {
          const int idx = tid + 256 * u, r = idx & (TN_CH - 1), c = idx / TN_CH;
          As[r][c] = (r < cnt && ia0 + c < ka) ? A[c0 + r + (int64_t)(ia0 + c) * lda] : 0.0;
          Bs[r][c] = (r < cnt && ib0 + c < kb) ? B[c0 + r + (int64_t)(ib0 + c) * ldb] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int r = 0; r < TN_CH; ++r) {
          double av[3], bv[3];
#pragma unroll
          for (int x = 0; x < 3; ++x) av[x] = As[r][ti + 16 * x];
#pragma unroll
          for (int y = 0; y < 3; ++y) bv[y] = Bs[r][tj + 16 * y];
#pragma unroll
          for (int x = 0; x < 3; ++x)
#pragma unroll
            for (int y = 0; y < 3; ++y) acc[x][y] += av[x] * bv[y];
        }
      }
#pragma unroll
      for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y) {
          const int ia = ia0 + ti + 16 * x, ib = ib0 + tj + 16 * y;
          if (ia < ka && ib < kb) pb[ia + ib * ka] = acc[x][y];
        }
    }
}

// One right-hand side (kb = 1): grid (nparts, ceil(ka / 4)); wave w of block
// (p, y) forms the partial dot product of column 4 y + w of A with x over the
// rows of part p, every lane's loads independent of the others.
__global__ __launch_bounds__(256) void gemv_tn_part_kernel(const double* __restrict__ A, int64_t lda,
                                                           const double* __restrict__ x, int64_t M, int ka,
                                                           int64_t rows_per, double* __restrict__ part) {
  const int lane = threadIdx.x & 63, ia = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (ia >= ka) return;
  const int64_t e0 = (int64_t)blockIdx.x * rows_per;
  const int64_t e1 = min(M, e0 + rows_per);
  const double* a = A + (int64_t)ia * lda;
  double s0 = 0.0, s1 = 0.0;
  int64_t r = e0 + lane;
  for (; r + 64 < e1; r += 128) {
    s0 = fma(a[r], x[r], s0);
    s1 = fma(a[r + 64], x[r + 64], s1);
  }
  if (r < e1) s0 = fma(a[r], x[r], s0);
  double v = s0 + s1;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (lane == 0) part[(int64_t)blockIdx.x * ka + ia] = v;
}

// One wave per output entry: the nparts partials in a fixed order (lane
// strides, then a butterfly), plus the identity if asked.
__global__ __launch_bounds__(256) void gemm_tn_reduce_kernel(const double* __restrict__ part, int nparts, int ka,
                                                             int kb, double* __restrict__ C, int64_t ldc, int ident) {
  const int lane = threadIdx.x & 63;
  const int o = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (o >= ka * kb) return;
  double s = 0;
  for (int p = lane; p < nparts; p += 64) s += part[(int64_t)p * ka * kb + o];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) {
    const int ia = o % ka, ib = o / ka;
    if (ident && ia == ib) s += 1.0;
    C[ia + (int64_t)ib * ldc] = s;
  }
}

// Row ranges of 64 rows (two LDS chunks), up to 1024 of them: the products
// here are short and wide (M ~ 10^4 - 10^5 rows, k < 100 columns), so the
// part count sets the parallelism; the reduction reads nparts k^2 partials.
int gemm_tn_nparts(int64_t M) {
  int64_t p = (M + 63) / 64;
  return (int)(p < 1 ? 1 : (p > 1024 ? 1024 : p));
}

// ================================================================ Y -= X W
__global__ __launch_bounds__(256) void sub_xw_kernel(const double* __restrict__ X, int64_t ldx, int64_t M, int k,
                                                     const double* __restrict__ W, double* __restrict__ Y,
                                                     int64_t ldy, int nrhs) {
  extern __shared__ double ws[];  // k x nrhs
  for (int idx = threadIdx.x; idx < k * nrhs; idx += 256) ws[idx] = W[idx];
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= M) return;
  for (int c = 0; c < nrhs; ++c) {
    double s = 0;
    for (int j = 0; j < k; ++j) s += X[e + (int64_t)j * ldx] * ws[j + c * k];
    Y[e + (int64_t)c * ldy] -= s;
  }
}

// y -= X (W^-1 z) in one launch: every block stages W^-1 (k x k) and z in
// LDS, forms w = W^-1 z there (the same sums as small_gemm_kernel), then
// subtracts X w from its rows as sub_xw_kernel does.
__global__ __launch_bounds__(256) void woodbury_sub_kernel(const double* __restrict__ X, int64_t ldx, int64_t M, int k,
                                                           const double* __restrict__ Wi,
                                                           const double* __restrict__ z, double* __restrict__ Y,
                                                           int64_t ldy, int nrhs) {
  extern __shared__ double sm[];
  double* sW = sm;               // k x k
  double* sz = sW + k * k;       // k x nrhs
  double* ws = sz + k * nrhs;    // k x nrhs
  for (int idx = threadIdx.x; idx < k * k; idx += 256) sW[idx] = Wi[idx];
  for (int idx = threadIdx.x; idx < k * nrhs; idx += 256) sz[idx] = z[idx];
  __syncthreads();
  for (int idx = threadIdx.x; idx < k * nrhs; idx += 256) {
    const int i = idx % k, c = idx / k;
    double s = 0;
    for (int j = 0; j < k; ++j) s += sW[i + j * k] * sz[j + c * k];
    ws[idx] = s;
  }
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= M) return;
  for (int c = 0; c < nrhs; ++c) {
    double s = 0;
    for (int j = 0; j < k; ++j) s += X[e + (int64_t)j * ldx] * ws[j + c * k];
    Y[e + (int64_t)c * ldy] -= s;
  }
}

// ================================================================ small inverse
// Gauss-Jordan with partial pivoting, one workgroup, matrix in global memory
// (k x k, ld = k), inverse built in `inv` then copied back.
// In-place inverse of W (k x k, k <= 64) by the register Gauss-Jordan.
__global__ __launch_bounds__(256) void small_inverse64_kernel(double* __restrict__ A, int k, int* __restrict__ info) {
  __shared__ Gj64Scratch S;
  double a[16];
  int q, rot;
  gj64_load(A, k, k, a);
  if (!reg_gj64(a, k, S, q, rot)) {
    if (threadIdx.x == 0) *info = 1;
    return;
  }
  gj64_store(a, k, q, rot, S.piv, A, k);
  if (threadIdx.x == 0) *info = 0;
}

__global__ __launch_bounds__(256) void small_inverse_kernel(double* __restrict__ A, double* __restrict__ inv, int k,
                                                            int* __restrict__ info) {
  __shared__ double rv[256];
  __shared__ int ri[256];
  __shared__ double pivrow_scale;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < k * k; idx += 256) inv[idx] = ((idx % k) == (idx / k)) ? 1.0 : 0.0;
  if (tid == 0) *info = 0;
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    double bv = -1.0;
    int bi = -1;
    for (int i = j + tid; i < k; i += 256) {
      const double v = fabs(A[i + j * k]);
      if (v > bv) { bv = v; bi = i; }
    }
    rv[tid] = bv;
    ri[tid] = bi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w && (rv[tid + w] > rv[tid] || (rv[tid + w] == rv[tid] && ri[tid + w] >= 0 && ri[tid + w] < ri[tid]))) {
        rv[tid] = rv[tid + w];
        ri[tid] = ri[tid + w];
      }
      __syncthreads();
    }
    const int p = ri[0];
    const double pv = rv[0];
    if (!(pv > 0.0) || !isfinite(pv) || p < 0) {
      if (tid == 0) *info = j + 1;
      return;
    }
    if (p != j)
      for (int c = tid; c < k; c += 256) {
        double t = A[j + c * k]; A[j + c * k] = A[p + c * k]; A[p + c * k] = t;
        t = inv[j + c * k]; inv[j + c * k] = inv[p + c * k]; inv[p + c * k] = t;
      }
    __syncthreads();
    if (tid == 0) pivrow_scale = 1.0 / A[j + j * k];
    __syncthreads();
    const double sc = pivrow_scale;
    for (int c = tid; c < k; c += 256) {
      A[j + c * k] *= sc;
      inv[j + c * k] *= sc;
    }
    __syncthreads();
    // eliminate column j from every other row
    for (int idx = tid; idx < k * k; idx += 256) {
      const int i = idx % k, c = idx / k;
      if (i == j) continue;
      const double f = A[i + j * k];
      if (c != j) A[i + c * k] -= f * A[j + c * k];
      inv[i + c * k] -= f * inv[j + c * k];
    }
    __syncthreads();
    for (int i = tid; i < k; i += 256)
      if (i != j) A[i + j * k] = 0.0;
    __syncthreads();
  }
  for (int idx = tid; idx < k * k; idx += 256) A[idx] = inv[idx];
}

__global__ __launch_bounds__(256) void small_gemm_kernel(const double* __restrict__ Wi, int k,
                                                         const double* __restrict__ z, int nrhs,
                                                         double* __restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= k) return;
  double s = 0;
  for (int j = 0; j < k; ++j) s += Wi[i + j * k] * z[j + c * k];
  out[i + c * k] = s;
}

// ================================================================ LU (no pivoting)
constexpr int LU_NB = 64;

// Largest |multiplier| seen by a wavefront, folded into *mult (the bits of a
// non-negative double order as the double does); NaN counts as infinity.
__device__ void lu_note_mult(double m, unsigned long long* mult) {
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0 && m > 0.0) atomicMax(mult, (unsigned long long)__double_as_longlong(m));
}

// Block 0: factor A11 and write it back; blocks 1..nrt: L21 tiles; the rest:
// U12 tiles.  Every block factors A11 in LDS from the same input.  Blocks 0
// .. nrt fold the largest |multiplier| (entry of L) they produce into *mult.
__global__ __launch_bounds__(256) void lu_panel_kernel(double* __restrict__ A, int64_t n, int64_t ld, int64_t K0,
                                                       int nrt, int* __restrict__ info,
                                                       unsigned long long* __restrict__ mult) {
  __shared__ double D[LU_NB][LU_NB + 1];
  __shared__ double T[LU_NB][LU_NB + 1];
  const int tid = threadIdx.x;
  const int nb = (int)min<int64_t>(LU_NB, n - K0);
  for (int idx = tid; idx < nb * nb; idx += 256) {
    const int r = idx % nb, c = idx / nb;
    D[r][c] = A[K0 + r + (K0 + c) * ld];
  }
  __syncthreads();
  double mmax = 0.0;
  for (int j = 0; j < nb; ++j) {
    const double pv = D[j][j];
    if (!(fabs(pv) > 0.0) || !isfinite(pv)) {
      if (blockIdx.x == 0 && tid == 0 && *info == 0) *info = (int)(K0 + j + 1);
      return;
    }
    for (int i = j + 1 + tid; i < nb; i += 256) {
      const double l = D[i][j] / pv;
      D[i][j] = l;
      mmax = fabs(l) <= mmax ? mmax : (isnan(l) ? INFINITY : fabs(l));
    }
    __syncthreads();
    const int rem = nb - j - 1;
    for (int idx = tid; idx < rem * rem; idx += 256) {
      const int i = j + 1 + idx % rem, c = j + 1 + idx / rem;
      D[i][c] -= D[i][j] * D[j][c];
    }
    __syncthreads();
  }
  const int b = blockIdx.x;
  if (b == 0) {
    for (int idx = tid; idx < nb * nb; idx += 256) {
      const int r = idx % nb, c = idx / nb;
      A[K0 + r + (K0 + c) * ld] = D[r][c];
    }
    lu_note_mult(mmax, mult);
    return;
  }
  const int64_t start = K0 + nb;
  if (b <= nrt) {
    // L21 tile: rows start + (b-1)*64 .. ; solve X U11 = A21 (row-wise)
    const int64_t rbase = start + (int64_t)(b - 1) * LU_NB;
    const int rows = (int)min<int64_t>(LU_NB, n - rbase);
    for (int idx = tid; idx < rows * nb; idx += 256) {
      const int r = idx % rows, c = idx / rows;
      T[r][c] = A[rbase + r + (K0 + c) * ld];
    }
    __syncthreads();
    double lm = 0.0;
    if (tid < rows) {
      for (int c = 0; c < nb; ++c) {
        double v = T[tid][c];
        for (int t = 0; t < c; ++t) v -= T[tid][t] * D[t][c];
        const double l = v / D[c][c];
        T[tid][c] = l;
        lm = fabs(l) <= lm ? lm : (isnan(l) ? INFINITY : fabs(l));
      }
    }
    __syncthreads();
    for (int idx = tid; idx < rows * nb; idx += 256) {
      const int r = idx % rows, c = idx / rows;
      A[rbase + r + (K0 + c) * ld] = T[r][c];
    }
    lu_note_mult(lm, mult);
  } else {
    // U12 tile: cols start + (b-1-nrt)*64 ..; solve L11 Y = A12 (unit lower)
    const int64_t cbase = start + (int64_t)(b - 1 - nrt) * LU_NB;
    const int cols = (int)min<int64_t>(LU_NB, n - cbase);
    for (int idx = tid; idx < nb * cols; idx += 256) {
      const int r = idx % nb, c = idx / nb;
      T[r][c] = A[K0 + r + (cbase + c) * ld];
    }
    __syncthreads();
    if (tid < cols) {
      for (int r = 0; r < nb; ++r) {
        double v = T[r][tid];
        for (int t = 0; t < r; ++t) v -= D[r][t] * T[t][tid];
        T[r][tid] = v;
      }
    }
    __syncthreads();
    for (int idx = tid; idx < nb * cols; idx += 256) {
      const int r = idx % nb, c = idx / nb;
      A[K0 + r + (cbase + c) * ld] = T[r][c];
    }
  }
}

// C -= A B, 64 x 64 tile per workgroup, FP64 MFMA 16x16x4.
__global__ __launch_bounds__(256) void gemm_nn_sub_kernel(const double* __restrict__ A, int64_t lda,
                                                          const double* __restrict__ B, int64_t ldb,
                                                          double* __restrict__ C, int64_t ldc, int64_t m, int64_t n,
                                                          int64_t kk) {
  __shared__ double As[16][64 + 1];  // [k][row]
  __shared__ double Bs[16][64 + 1];  // [k][col]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i16 = lane & 15, k4 = lane >> 4;
  const int wr = wave & 1, wc = wave >> 1;
  const int64_t row0 = (int64_t)blockIdx.x * 64, col0 = (int64_t)blockIdx.y * 64;
  double4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (double4_t){0.0, 0.0, 0.0, 0.0};
  for (int64_t k0 = 0; k0 < kk; k0 += 16) {
    __syncthreads();
    for (int idx = tid; idx < 64 * 16; idx += 256) {
      const int r = idx & 63, kc = idx >> 6;
      const int64_t gr = row0 + r, gk = k0 + kc;
      As[kc][r] = (gr < m && gk < kk) ? A[gr + gk * lda] : 0.0;
      const int kc2 = idx & 15, c = idx >> 4;
      const int64_t gc = col0 + c, gk2 = k0 + kc2;
      Bs[kc2][c] = (gc < n && gk2 < kk) ? B[gk2 + gc * ldb] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[ks * 4 + k4][wr * 32 + i * 16 + i16];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[ks * 4 + k4][wc * 32 + j * 16 + i16];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // item r of lane l holds D[l / 16 + 4 r][l % 16]
        const int64_t gr = row0 + wr * 32 + i * 16 + k4 + 4 * r;
        const int64_t gc = col0 + wc * 32 + j * 16 + i16;
        if (gr < m && gc < n) C[gr + gc * ldc] -= acc[i][j][r];
      }
}

// C -= A X for few columns (GEMV-like): thread per row.
__global__ __launch_bounds__(256) void gemv_sub_kernel(const double* __restrict__ A, int64_t lda,
                                                       const double* __restrict__ X, int64_t ldx,
                                                       double* __restrict__ C, int64_t ldc, int64_t m, int64_t kk,
                                                       int nrhs) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= m) return;
  double s = 0;
  const double* x = X + (int64_t)c * ldx;
#pragma unroll 4
  for (int64_t t = 0; t < kk; ++t) s += A[i + t * lda] * x[t];
  C[i + (int64_t)c * ldc] -= s;
}

constexpr int TS_NB = 128;

// In-place triangular solve on one diagonal block (rows b0 .. b0+nbs) of the
// packed LU: lower = unit lower (forward), else upper (backward).
__global__ __launch_bounds__(256) void trsv_diag_kernel(const double* __restrict__ LU, int64_t ld, int64_t b0,
                                                        int nbs, double* __restrict__ B, int64_t ldb, int lower) {
  __shared__ double x[TS_NB];
  const int c = blockIdx.x;  // right-hand side
  double* b = B + (int64_t)c * ldb + b0;
  for (int i = threadIdx.x; i < nbs; i += 256) x[i] = b[i];
  __syncthreads();
  if (lower) {
    for (int j = 0; j < nbs; ++j) {
      const double xj = x[j];
      for (int i = j + 1 + threadIdx.x; i < nbs; i += 256) x[i] -= LU[b0 + i + (b0 + j) * ld] * xj;
      __syncthreads();
    }
  } else {
    for (int j = nbs - 1; j >= 0; --j) {
      if (threadIdx.x == 0) x[j] /= LU[b0 + j + (b0 + j) * ld];
      __syncthreads();
      const double xj = x[j];
      for (int i = threadIdx.x; i < j; i += 256) x[i] -= LU[b0 + i + (b0 + j) * ld] * xj;
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < nbs; i += 256) b[i] = x[i];
}

}  // namespace

// ------------------------------------------------------------------ launchers
static size_t rowid_sel_bytes(int64_t m, int ncols, int kmax) {
  const int64_t nb = (m + SEL_ROWS - 1) / SEL_ROWS;
  return 2 * sizeof(unsigned long long) + 2 * sizeof(int) * (size_t)nb * (kmax + 1) +
         sizeof(double) * (size_t)kmax * ncols + 1024;
}

size_t rowid_work_bytes(int64_t m, int ncols, int kmax, int ngroups) {
  return sizeof(double) * (size_t)(2 * ngroups) + sizeof(int64_t) * (size_t)(2 * ngroups) +
         sizeof(double) * (size_t)(2 * ngroups) * ncols + sizeof(double) * (size_t)m * ncols + 1024 +
         rowid_sel_bytes(m, ncols, kmax);
}

static int rowid_cooperative(rw_ctx* ctx, const double* Y, int64_t m, int ncols, double tol, int kmax, int* J,
                             double* C, void* work, hipStream_t s) {
  if (m <= 0) return 0;
  const int ncu = ctx->n_cu > 0 ? ctx->n_cu : 256;
  // rows per workgroup: keep them in LDS when they fit (<= 120 KiB of rows)
  const int64_t lds_budget = 120 * 1024;
  int64_t rows_per = (m + ncu - 1) / ncu;
  if (rows_per < 32) rows_per = 32;
  int G = (int)((m + rows_per - 1) / rows_per);
  const bool lds_rows = rows_per * (ncols + 1) * 8 <= lds_budget;
  const size_t extra = sizeof(double) * ((size_t)ncols + rows_per + 256) + sizeof(int64_t) * 256 + sizeof(int) * 256;
  const size_t shmem = (lds_rows ? sizeof(double) * rows_per * (ncols + 1) : 0) + extra;
  char* w = (char*)work;
  RowIdArgs a{};
  a.Y = Y;
  a.m = m;
  a.ncols = ncols;
  a.tol2 = tol * tol;
  a.kmax = kmax;
  a.rows_per = (int)rows_per;
  a.lds_rows = lds_rows ? 1 : 0;
  a.slot_norm = (double*)w; w += sizeof(double) * 2 * G;
  a.slot_idx = (int64_t*)w; w += sizeof(int64_t) * 2 * G;
  a.slot_vec = (double*)w; w += sizeof(double) * 2 * G * ncols;
  a.Yw = (double*)w; w += sizeof(double) * m * ncols;
  a.J = J;
  a.C = C;
  int* dk = (int*)ctx->d_sync;
  a.out_k = dk;
  if (!lds_rows) HIP_CHECK(hipMemcpyAsync(a.Yw, Y, sizeof(double) * m * ncols, hipMemcpyDeviceToDevice, s));
  void* args[] = {&a};
  func_lds_at_least((const void*)rowid_kernel, (int)shmem);
  {
    KernelTimer kt("rowid_kernel", 6.0 * (double)m * ncols * kmax, 0.0, s);
    HIP_CHECK(hipLaunchCooperativeKernel((const void*)rowid_kernel, dim3(G), dim3(256), args, shmem, s));
  }
  KERNEL_CHECK("rowid");
  int k = 0;
  HIP_CHECK(hipMemcpyAsync(&k, dk, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  return k;
}

bool launch_rowid_enqueue(rw_ctx* ctx, const double* Y, int64_t m, int ncols, double tol, int kmax, int* J,
                          double* C, void* work, int* res_k, unsigned long long* res_m, hipStream_t s) {
  const int64_t nb0 = (m + SEL_ROWS - 1) / SEL_ROWS;
  if (m <= 0 || ncols > SEL_NC || ncols % 4 != 0 || kmax > 64 || nb0 > 1024) return false;
  // the selection buffers sit behind the cooperative kernel's share of `work`
  char* w = (char*)work + (rowid_work_bytes(m, ncols, kmax, std::max(256, ctx->n_cu)) - rowid_sel_bytes(m, ncols, kmax));
  w = (char*)(((uintptr_t)w + 255) & ~(uintptr_t)255);
  unsigned long long* dmax = (unsigned long long*)w;  // [0] max row norm^2, [1] max residual^2
  int* idx[2] = {(int*)(dmax + 2), (int*)(dmax + 2) + nb0 * kmax};
  int* cnt[2] = {idx[1] + nb0 * kmax, idx[1] + nb0 * kmax + nb0};
  double* Q = (double*)(((uintptr_t)(cnt[1] + nb0) + 15) & ~(uintptr_t)15);
  KernelTimer kt("rowid_select_kernel", 0.0, 0.0, s);
  HIP_CHECK(hipMemsetAsync(dmax, 0, 2 * sizeof(unsigned long long), s));
  hipLaunchKernelGGL(rowid_maxnorm_kernel, dim3((unsigned)std::min<int64_t>(1024, blocks(m))), dim3(256), 0, s, Y, m,
                     ncols, dmax);
  KERNEL_CHECK("rowid_maxnorm");
  int64_t nb = nb0;
  int cur = 0;
  hipLaunchKernelGGL(rowid_select_kernel, dim3((unsigned)nb), dim3(SEL_ROWS), 0, s, Y, m, ncols, (const int*)nullptr,
                     (const int*)nullptr, 0, kmax, tol * tol, dmax, idx[cur], cnt[cur]);
  KERNEL_CHECK("rowid_select");
  while (nb > 1) {
    const int64_t nb2 = (nb * kmax + SEL_ROWS - 1) / SEL_ROWS;
    hipLaunchKernelGGL(rowid_select_kernel, dim3((unsigned)nb2), dim3(SEL_ROWS), 0, s, Y, m, ncols, idx[cur], cnt[cur],
                       (int)nb, kmax, tol * tol, dmax, idx[1 - cur], cnt[1 - cur]);
    KERNEL_CHECK("rowid_select");
    cur = 1 - cur;
    nb = nb2;
  }
  // basis and coefficients read the selected count on the device
  hipLaunchKernelGGL(rowid_basis_kernel, dim3(1), dim3(64), 0, s, Y, ncols, idx[cur], cnt[cur], J, Q);
  KERNEL_CHECK("rowid_basis");
  hipLaunchKernelGGL(rowid_coef_kernel, dim3((unsigned)((m + 256 / RC4 - 1) / (256 / RC4))), dim3(256),
                     sizeof(double) * kmax * RC4 * RCQ, s, Y, m, ncols, Q, cnt[cur], kmax, C, dmax + 1);
  KERNEL_CHECK("rowid_coef");
  HIP_CHECK(hipMemcpyAsync(res_k, cnt[cur], sizeof(int), hipMemcpyDeviceToDevice, s));
  HIP_CHECK(hipMemcpyAsync(res_m, dmax, 2 * sizeof(unsigned long long), hipMemcpyDeviceToDevice, s));
  return true;
}

bool rowid_certified(int k, int kmax, double tol, const unsigned long long* hm) {
  // every row within 10 tol of span(Y(J, :)) relative to the largest row;
  // k == kmax sends the caller to a wider sketch anyway
  const double n0 = __builtin_bit_cast(double, hm[0]), res = __builtin_bit_cast(double, hm[1]);
  return k >= kmax || res <= 100.0 * tol * tol * n0;
}

int launch_rowid(rw_ctx* ctx, const double* Y, int64_t m, int ncols, double tol, int kmax, int* J, double* C,
                 void* work, hipStream_t s) {
  if (m <= 0) return 0;
  DBuf<char> res(ctx, 256);
  int* rk = (int*)res.p;
  unsigned long long* rm = (unsigned long long*)(res.p + 64);
  if (!launch_rowid_enqueue(ctx, Y, m, ncols, tol, kmax, J, C, work, rk, rm, s))
    return rowid_cooperative(ctx, Y, m, ncols, tol, kmax, J, C, work, s);
  int k = 0;
  unsigned long long hm[2] = {0, 0};
  HIP_CHECK(hipMemcpyAsync(&k, rk, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(hm, rm, sizeof(hm), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  if (!rowid_certified(k, kmax, tol, hm)) return rowid_cooperative(ctx, Y, m, ncols, tol, kmax, J, C, work, s);
  return k;
}

int launch_rowid_fallback(rw_ctx* ctx, const double* Y, int64_t m, int ncols, double tol, int kmax, int* J, double* C,
                          void* work, hipStream_t s) {
  return rowid_cooperative(ctx, Y, m, ncols, tol, kmax, J, C, work, s);
}

void launch_rowid_interp(const double* C, int64_t m, int kmax, int k, const int* J, const int* pos, double* L,
                         int64_t ldL, int col0, double* inv_work, hipStream_t s) {
  if (k <= 0 || m <= 0) return;
  if (k > 128) RW_THROW(RW_EINVAL, "row ID rank above 128");
  const size_t sh = sizeof(double) * k * k;
  func_lds_at_least((const void*)cj_inv_kernel, (int)sh);
  func_lds_at_least((const void*)rowid_interp_kernel, (int)sh);
  hipLaunchKernelGGL(cj_inv_kernel, dim3(1), dim3(128), sh, s, C, kmax, k, J, inv_work);
  KERNEL_CHECK("cj_inv");
  hipLaunchKernelGGL(rowid_interp_kernel, dim3(blocks(m)), dim3(256), sh, s, C, m, kmax, k, inv_work, pos, L, ldL,
                     col0);
  KERNEL_CHECK("rowid_interp");
  hipLaunchKernelGGL(rowid_unit_rows_kernel, dim3(k), dim3(64), 0, s, k, J, pos, L, ldL, col0);
  KERNEL_CHECK("rowid_unit_rows");
}

size_t gemm_tn_part_doubles(int64_t M, int ka, int kb) { return (size_t)gemm_tn_nparts(M) * ka * kb; }

void launch_gemm_tn(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M, int ka, int kb, double* C,
                    int64_t ldc, bool add_identity, double* part, hipStream_t s) {
  if (ka <= 0 || kb <= 0) return;
  const int np = gemm_tn_nparts(M);
  const int64_t rows_per = (M + np - 1) / np;
  if (kb == 1)
    hipLaunchKernelGGL(gemv_tn_part_kernel, dim3(np, (ka + 3) / 4), dim3(256), 0, s, A, lda, B, M, ka, rows_per,
                       part);
  else
    hipLaunchKernelGGL(gemm_tn_part_kernel, dim3(np), dim3(256), 0, s, A, lda, B, ldb, M, ka, kb, rows_per, part);
  KERNEL_CHECK("gemm_tn_part");
  hipLaunchKernelGGL(gemm_tn_reduce_kernel, dim3(blocks((int64_t)ka * kb, 4)), dim3(256), 0, s, part, np, ka, kb, C,
                     ldc, add_identity ? 1 : 0);
  KERNEL_CHECK("gemm_tn_reduce");
}

void launch_sub_xw(const double* X, int64_t ldx, int64_t M, int k, const double* W, double* Y, int64_t ldy, int nrhs,
                   hipStream_t s) {
  if (k <= 0 || M <= 0 || nrhs <= 0) return;
  // W (k x nrhs) is staged in LDS: as many columns per launch as 150 KB hold
  const int per = (int)std::min<int64_t>(nrhs, (150 * 1024) / (sizeof(double) * k));
  if (per < 1) RW_THROW(RW_EINVAL, "Woodbury rank too large for one column in LDS");
  func_lds_at_least((const void*)sub_xw_kernel, (int)(sizeof(double) * k * per));
  for (int c0 = 0; c0 < nrhs; c0 += per) {
    const int nc = std::min(per, nrhs - c0);
    hipLaunchKernelGGL(sub_xw_kernel, dim3(blocks(M)), dim3(256), sizeof(double) * k * nc, s, X, ldx, M, k,
                       W + (size_t)c0 * k, Y + (size_t)c0 * ldy, ldy, nc);
    KERNEL_CHECK("sub_xw");
  }
}

bool launch_woodbury_sub(const double* X, int64_t ldx, int64_t M, int k, const double* Winv, const double* z,
                         double* Y, int64_t ldy, int nrhs, hipStream_t s) {
  if (k <= 0 || M <= 0) return true;
  const size_t sh = sizeof(double) * ((size_t)k * k + 2 * (size_t)k * nrhs);
  if (sh > 150 * 1024) return false;
  func_lds_at_least((const void*)woodbury_sub_kernel, (int)sh);
  hipLaunchKernelGGL(woodbury_sub_kernel, dim3(blocks(M)), dim3(256), sh, s, X, ldx, M, k, Winv, z, Y, ldy, nrhs);
  KERNEL_CHECK("woodbury_sub");
  return true;
}

void launch_small_inverse(double* W, int k, int* info, hipStream_t s) {
  // in place for k <= 64; else built in the k*k doubles that follow W
  if (k <= GN)
    hipLaunchKernelGGL(small_inverse64_kernel, dim3(1), dim3(256), 0, s, W, k, info);
  else
    hipLaunchKernelGGL(small_inverse_kernel, dim3(1), dim3(256), 0, s, W, W + (size_t)k * k, k, info);
  KERNEL_CHECK("small_inverse");
}

void launch_small_gemm(const double* Winv, int k, const double* z, int nrhs, double* out, hipStream_t s) {
  if (k <= 0) return;
  hipLaunchKernelGGL(small_gemm_kernel, dim3(blocks(k), nrhs), dim3(256), 0, s, Winv, k, z, nrhs, out);
  KERNEL_CHECK("small_gemm");
}

void launch_gemm_nn_sub(const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc, int64_t m,
                        int64_t n, int64_t kk, hipStream_t s) {
  if (m <= 0 || n <= 0 || kk <= 0) return;
  if (n <= 8) {
    hipLaunchKernelGGL(gemv_sub_kernel, dim3(blocks(m), (unsigned)n), dim3(256), 0, s, A, lda, B, ldb, C, ldc, m, kk,
                       (int)n);
    KERNEL_CHECK("gemv_sub");
    return;
  }
  dim3 grid((unsigned)((m + 63) / 64), (unsigned)((n + 63) / 64));
  hipLaunchKernelGGL(gemm_nn_sub_kernel, grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, m, n, kk);
  KERNEL_CHECK("gemm_nn_sub");
}

void launch_lu_nopiv(double* A, int64_t n, int64_t ld, int* info, unsigned long long* mult, hipStream_t s) {
  HIP_CHECK(hipMemsetAsync(info, 0, sizeof(int), s));
  HIP_CHECK(hipMemsetAsync(mult, 0, sizeof(unsigned long long), s));
  for (int64_t K0 = 0; K0 < n; K0 += LU_NB) {
    const int nb = (int)std::min<int64_t>(LU_NB, n - K0);
    const int64_t rest = n - K0 - nb;
    const int nrt = (int)((rest + LU_NB - 1) / LU_NB);
    hipLaunchKernelGGL(lu_panel_kernel, dim3(1 + 2 * nrt), dim3(256), 0, s, A, n, ld, K0, nrt, info, mult);
    KERNEL_CHECK("lu_panel");
    if (rest > 0)
      launch_gemm_nn_sub(A + (K0 + nb) + K0 * ld, ld, A + K0 + (K0 + nb) * ld, ld, A + (K0 + nb) + (K0 + nb) * ld, ld,
                         rest, rest, nb, s);
  }
}

void launch_lu_solve(const double* LU, int64_t n, int64_t ld, double* B, int64_t ldb, int nrhs, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return;
  for (int64_t b0 = 0; b0 < n; b0 += TS_NB) {
    const int nbs = (int)std::min<int64_t>(TS_NB, n - b0);
    hipLaunchKernelGGL(trsv_diag_kernel, dim3(nrhs), dim3(256), 0, s, LU, ld, b0, nbs, B, ldb, 1);
    KERNEL_CHECK("trsv_lower");
    const int64_t rest = n - b0 - nbs;
    if (rest > 0) launch_gemm_nn_sub(LU + b0 + nbs + b0 * ld, ld, B + b0, ldb, B + b0 + nbs, ldb, rest, nrhs, nbs, s);
  }
  const int64_t nblk = (n + TS_NB - 1) / TS_NB;
  for (int64_t bi = nblk - 1; bi >= 0; --bi) {
    const int64_t b0 = bi * TS_NB;
    const int nbs = (int)std::min<int64_t>(TS_NB, n - b0);
    hipLaunchKernelGGL(trsv_diag_kernel, dim3(nrhs), dim3(256), 0, s, LU, ld, b0, nbs, B, ldb, 0);
    KERNEL_CHECK("trsv_upper");
    if (b0 > 0) launch_gemm_nn_sub(LU + b0 * ld, ld, B + b0, ldb, B, ldb, b0, nrhs, nbs, s);
  }
}
