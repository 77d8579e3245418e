// Register-resident Gauss-Jordan inverse with partial pivoting for blocks of
// at most 64 unknowns, one workgroup of 256 threads (shared by the HBS node
// factorization and the Woodbury operator).
#pragma once

#include "dev_reduce.h"

// Lane l owns row l of the block, wave h the 16 columns 16 h .. 16 h + 15
// (a[16]).  Step j pivots on column j among the rows not yet used, without
// moving rows: the owner wave of column j keeps it in a[0] by shifting its
// registers down by one in each of its updates (the new column j goes to
// a[15]); the result is (P A)^-1, row j stored in row p_j, so
// A^-1(j, p_c) = B(p_j, c), which gj64_store writes out.  The pivot search
// stays inside the owner wave (DPP maximum of pivot keys); the owner's
// column goes through LDS, and every wave reads its segment of the pivot row
// from its own lane p (readlane), so a step needs one barrier: the column
// and key slots alternate, and a slot is rewritten two steps later, after
// every wave has passed the barrier of the step in between.
constexpr int GN = 64;

struct Gj64Scratch {
  double colv[2][GN];
  double key[2];
  int piv[GN];
};

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane), hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ inline bool reg_gj64(double (&a)[16], int n, Gj64Scratch& S, int& myq, int& rot) {
  const int tid = threadIdx.x, r = tid & 63;
  const int h = __builtin_amdgcn_readfirstlane(tid >> 6);
  bool used = r >= n;
  myq = -1;
  for (int j = 0; j < n; ++j) {
    const int b = j & 1;
    const bool own = h == (j >> 4);  // wave-uniform
    if (own) {
      S.colv[b][r] = a[0];
      const double k = wave_max_nonneg(pivot_key_bits<6>(a[0], r, !used));
      if (r == 0) S.key[b] = k;
    }
    __syncthreads();
    const int p = __builtin_amdgcn_readfirstlane(pivot_key_index<6>(S.key[b]));
    const double piv = S.colv[b][p];
    if (!(fabs(piv) > 0.0) || !isfinite(piv)) {
      __syncthreads();
      return false;
    }
    if (tid == 0) S.piv[j] = p;
    const double pinv = 1.0 / piv;
    const double f = S.colv[b][r] * pinv;
    double pr[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) pr[c] = readlane_f64(a[c], p);
    if (r == p) {
      used = true;
      myq = j;
    }
    if (own) {
      if (r == p) {
#pragma unroll
        for (int c = 0; c < 15; ++c) a[c] = a[c + 1] * pinv;
        a[15] = pinv;
      } else {
#pragma unroll
        for (int c = 0; c < 15; ++c) a[c] = a[c + 1] - f * pr[c + 1];
        a[15] = -f;
      }
    } else {
      if (r == p) {
#pragma unroll
        for (int c = 0; c < 16; ++c) a[c] *= pinv;
      } else {
#pragma unroll
        for (int c = 0; c < 16; ++c) a[c] -= f * pr[c];
      }
    }
  }
  __syncthreads();   // S.piv complete for gj64_store
  rot = min(max(n - 16 * h, 0), 16) & 15;
  return true;
}

// Registers of reg_gj64 from / to a column-major n x n block (ld).
__device__ __forceinline__ void gj64_load(const double* M, int ld, int n, double (&a)[16]) {
  const int r = threadIdx.x & 63, h = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int col = 16 * h + c;
    a[c] = (r < n && col < n) ? M[r + (int64_t)col * ld] : 0.0;
  }
}
__device__ __forceinline__ void gj64_store(const double (&a)[16], int n, int q, int rot, const int* piv, double* M,
                                           int ld) {
  const int r = threadIdx.x & 63, h = threadIdx.x >> 6;
  if (r < n) {
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int col = 16 * h + ((c + rot) & 15);
      if (col < n) M[q + (int64_t)piv[col] * ld] = a[c];
    }
  }
}

