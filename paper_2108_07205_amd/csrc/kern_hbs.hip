// HBS inverse apply: level sweeps over packed generators (Algorithm 1, solve
// step 1, the A_oo^{-1} block; also Algorithm 1 pre-computation step 3 with
// many right-hand sides).
//
// The apply is a batch of small GEMVs per tree level and is bound by the
// generator bytes streamed from HBM.  Each node's generator block
// (column-major, R rows x C columns) is cut into slabs of 64 rows; one
// workgroup takes one slab: lane l owns row l of the slab, the four waves
// split the C columns into quarters, and every lane keeps 16 independent
// loads in flight (each wave-wide load reads 64 consecutive rows of one
// column).  The node's input slice is staged in LDS (broadcast reads) and
// the four partial sums are added through LDS.  Up to 8 right-hand sides
// share one pass over the generators.
#include "kernels.h"
#include "hbs_dev.h"

namespace {

// BF16 generator entry (the high half of an FP32 word), widened on load.
struct bf16s {
  uint16_t u;
  __device__ __forceinline__ operator double() const { return (double)__uint_as_float((unsigned)u << 16); }
};

constexpr int kThreads = 256;
constexpr int kRows = 64;    // rows per workgroup (one per lane)
constexpr int kUnroll = 16;  // loads in flight per lane
constexpr int kMfmaMin = 40;    // right-hand sides from which the FP64 slab product runs on MFMA (measured crossover)
constexpr int kMfmaMin32 = 16;  // the same for FP32 and BF16 generators (FP32 accumulation)
template <typename T>
constexpr int mfma_min() { return sizeof(T) < 8 ? kMfmaMin32 : kMfmaMin; }

// The first kUnroll entries of row `row` in the column quarter w of M (R x
// C, ld R), loaded before the input slice is staged so that the two loads'
// latencies overlap (slab_gemv takes them as its first chunk).
template <typename T>
__device__ __forceinline__ void slab_prefetch(const T* __restrict__ M, int R, int C, int row, int w,
                                              double (&m0)[kUnroll]) {
  const int c0 = (w * C) >> 2, c1 = ((w + 1) * C) >> 2;
  if (row >= R || c0 + kUnroll > c1) return;
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) m0[u] = (double)M[row + (int64_t)(c0 + u) * R];
}

// acc = rows `row` of M (R x C, ld R) times xs (C x RB, row-major in LDS),
// over the column quarter w of the four waves; m0: slab_prefetch's chunk.
template <typename T, int RB>
__device__ __forceinline__ void slab_gemv(const T* __restrict__ M, int R, int C, int row, const double* xs, int w,
                                          const double (&m0)[kUnroll], double (&acc)[RB]) {
#pragma unroll
  for (int c = 0; c < RB; ++c) acc[c] = 0.0;
  if (row >= R) return;
  const int c0 = (w * C) >> 2, c1 = ((w + 1) * C) >> 2;
  const T* mp = M + row;
  int col = c0;
  if (col + kUnroll <= c1) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
#pragma unroll
      for (int c = 0; c < RB; ++c) acc[c] += m0[u] * xs[(col + u) * RB + c];
    col += kUnroll;
  }
  for (; col + kUnroll <= c1; col += kUnroll) {
    double m[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) m[u] = (double)mp[(int64_t)(col + u) * R];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
#pragma unroll
      for (int c = 0; c < RB; ++c) acc[c] += m[u] * xs[(col + u) * RB + c];
  }
  for (; col < c1; ++col) {
    const double m = (double)mp[(int64_t)col * R];
#pragma unroll
    for (int c = 0; c < RB; ++c) acc[c] += m * xs[col * RB + c];
  }
}

// Sum of the four waves' partial results for right-hand side c of this lane.
template <int RB>
__device__ __forceinline__ double slab_sum(const double* red, int c, int lane) {
  return (red[(0 * RB + c) * kRows + lane] + red[(1 * RB + c) * kRows + lane]) +
         (red[(2 * RB + c) * kRows + lane] + red[(3 * RB + c) * kRows + lane]);
}

// grid (nodes x rbmax, ceil(nrhs / RB)).  [bhat; gb] = [F*; G] b per node.
template <typename T, int RB>
__global__ __launch_bounds__(kThreads) void hbs_up_kernel(
    int rbmax, const int* __restrict__ nin, const int* __restrict__ kk, const int64_t* __restrict__ in_off,
    const int64_t* __restrict__ kout_off, const int64_t* __restrict__ up_off, const T* __restrict__ gen,
    const double* __restrict__ in, int64_t ld_in, double* __restrict__ bhat, int64_t ld_bhat,
    double* __restrict__ gb, int64_t ld_gb, int nrhs, int xs_len) {
  extern __shared__ double sm[];
  const int j = blockIdx.x / rbmax, rb = blockIdx.x - j * rbmax;
  const int n = nin[j], k = kk[j], R = k + n;
  if (rb * kRows >= R) return;  // whole workgroup
  const int r0 = blockIdx.y * RB, nr = min(RB, nrhs - r0);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  double* xs = sm;
  double* red = sm + xs_len;
  const int64_t io = in_off[j];
  const int row = rb * kRows + lane;
  const T* Mj = gen + up_off[j];
  double m0[kUnroll];
  slab_prefetch<T>(Mj, R, n, row, w, m0);
  for (int idx = tid; idx < n * RB; idx += kThreads) {
    const int col = idx / RB, c = idx - col * RB;
    xs[idx] = (c < nr) ? in[io + col + (int64_t)(r0 + c) * ld_in] : 0.0;
  }
  __syncthreads();
  double acc[RB];
  slab_gemv<T, RB>(Mj, R, n, row, xs, w, m0, acc);
#pragma unroll
  for (int c = 0; c < RB; ++c) red[(w * RB + c) * kRows + lane] = acc[c];
  __syncthreads();
  if (row < R) {
    const int64_t ko = kout_off[j];
    for (int c = w; c < nr; c += 4) {
      const double v = slab_sum<RB>(red, c, lane);
      if (row < k) bhat[ko + row + (int64_t)(r0 + c) * ld_bhat] = v;
      else gb[io + (row - k) + (int64_t)(r0 + c) * ld_gb] = v;
    }
  }
}

// grid (nodes x rbmax, ceil(nrhs / RB)).  out = E xhat + gb per node.
template <typename T, int RB>
__global__ __launch_bounds__(kThreads) void hbs_down_kernel(
    int rbmax, const int* __restrict__ nin, const int* __restrict__ kk, const int64_t* __restrict__ in_off,
    const int64_t* __restrict__ kout_off, const int64_t* __restrict__ e_off, const T* __restrict__ gen,
    const double* __restrict__ xhat, int64_t ld_xh, const double* __restrict__ gb, int64_t ld_gb,
    double* __restrict__ out, int64_t ld_out, int nrhs, int xs_len) {
  extern __shared__ double sm[];
  const int j = blockIdx.x / rbmax, rb = blockIdx.x - j * rbmax;
  const int n = nin[j], k = kk[j];
  if (rb * kRows >= n) return;  // whole workgroup
  const int r0 = blockIdx.y * RB, nr = min(RB, nrhs - r0);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  double* xs = sm;
  double* red = sm + xs_len;
  const int64_t io = in_off[j], ko = kout_off[j];
  const int row = rb * kRows + lane;
  const T* Ej = gen + e_off[j];
  double m0[kUnroll];
  slab_prefetch<T>(Ej, n, k, row, w, m0);
  for (int idx = tid; idx < k * RB; idx += kThreads) {
    const int col = idx / RB, c = idx - col * RB;
    xs[idx] = (c < nr) ? xhat[ko + col + (int64_t)(r0 + c) * ld_xh] : 0.0;
  }
  __syncthreads();
  double acc[RB];
  slab_gemv<T, RB>(Ej, n, k, row, xs, w, m0, acc);
#pragma unroll
  for (int c = 0; c < RB; ++c) red[(w * RB + c) * kRows + lane] = acc[c];
  __syncthreads();
  if (row < n)
    for (int c = w; c < nr; c += 4)
      out[io + row + (int64_t)(r0 + c) * ld_out] =
          slab_sum<RB>(red, c, lane) + gb[io + row + (int64_t)(r0 + c) * ld_gb];
}

// grid (ceil(nmax / 64), ceil(nrhs / RB)).  out = G_root in; the root size
// is n_dev[0] when n_dev is given (at most nmax), else nmax.
template <int RB>
__global__ __launch_bounds__(kThreads) void hbs_root_kernel(int nmax, const int* __restrict__ n_dev,
                                                            const double* __restrict__ G,
                                                            const double* __restrict__ in, int64_t ld_in,
                                                            double* __restrict__ out, int64_t ld_out, int nrhs) {
  extern __shared__ double sm[];
  const int n = n_dev ? min(*n_dev, nmax) : nmax;
  if (blockIdx.x * kRows >= n) return;  // whole workgroup
  const int r0 = blockIdx.y * RB, nr = min(RB, nrhs - r0);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  double* xs = sm;
  double* red = sm + nmax * RB;
  const int row = blockIdx.x * kRows + lane;
  double m0[kUnroll];
  slab_prefetch<double>(G, n, n, row, w, m0);
  for (int idx = tid; idx < n * RB; idx += kThreads) {
    const int col = idx / RB, c = idx - col * RB;
    xs[idx] = (c < nr) ? in[col + (int64_t)(r0 + c) * ld_in] : 0.0;
  }
  __syncthreads();
  double acc[RB];
  slab_gemv<double, RB>(G, n, n, row, xs, w, m0, acc);
#pragma unroll
  for (int c = 0; c < RB; ++c) red[(w * RB + c) * kRows + lane] = acc[c];
  __syncthreads();
  if (row < n)
    for (int c = w; c < nr; c += 4) out[row + (int64_t)(r0 + c) * ld_out] = slab_sum<RB>(red, c, lane);
}


// ------------------------------------------- many right-hand sides (MFMA)
// For 40 or more right-hand sides the slab product is a small GEMM: out
// (64 rows x 64 RHS) = M(slab rows, :) X(:, 64 RHS).  Wave w owns row block w
// (16 rows) and the four 16-column blocks of the RHS; the A fragments come
// straight from the column-major generators (16 consecutive rows per column),
// the B tile (16 input rows x 64 RHS) is staged in LDS per chunk of the
// contraction, and the FP64 matrix cores accumulate.
typedef double double4_t __attribute__((ext_vector_type(4)));
constexpr int kMR = 64;  // right-hand sides per pass

template <typename T, typename Load, typename Emit>
__device__ __forceinline__ void slab_mfma(const T* __restrict__ M, int R, int C, int slab, int r0, int nr,
                                          double (*Bs)[kMR + 2], Load load, Emit emit) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, i16 = lane & 15, k4 = lane >> 4;
  const int arow = slab * kRows + w * 16 + i16;
  const bool aval = arow < R;
  const T* mp = M + (aval ? arow : 0);
  double4_t acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = (double4_t){0.0, 0.0, 0.0, 0.0};
  // this thread's share of a chunk: A fragments of the four k-steps, and B
  // elements (input row c0 + (e & 15), right-hand side e >> 4 for
  // e = tid + 256 u), read along input rows
  double an[4], bn[4];
  auto fetch = [&](int c0) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int kc = c0 + ks * 4 + k4;
      an[ks] = (aval && kc < C) ? (double)mp[(int64_t)kc * R] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + kThreads * u, kk = e & 15, c = e >> 4;
      bn[u] = (c0 + kk < C && c < nr) ? load(c0 + kk, r0 + c) : 0.0;
    }
  };
  if (C > 0) fetch(0);
  for (int c0 = 0; c0 < C; c0 += 16) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + kThreads * u;
      Bs[e & 15][e >> 4] = bn[u];
    }
    double a[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) a[ks] = an[ks];
    __syncthreads();
    if (c0 + 16 < C) fetch(c0 + 16);  // in flight during this chunk's products
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
        acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks], Bs[ks * 4 + k4][cb * 16 + i16], acc[cb], 0, 0, 0);
  }
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      // v_mfma_f64_16x16x4f64: item r of lane l holds D[l / 16 + 4 r][l % 16]
      const int row = slab * kRows + w * 16 + k4 + 4 * r, c = cb * 16 + i16;
      if (row < R && c < nr) emit(row, r0 + c, acc[cb][r]);
    }
}

// FP32 generators on the FP32 matrix cores (v_mfma_f32_16x16x4f32, FP32
// accumulation): the same tiling as slab_mfma, the input tile rounded to
// FP32 as it is staged; the products return to the FP64 vectors.  This is
// the mixed-precision apply; FP64 iterative refinement recovers the digits.
typedef float float4_t __attribute__((ext_vector_type(4)));

template <typename Load, typename Emit>
__device__ __forceinline__ void slab_mfma_f32(const float* __restrict__ M, int R, int C, int slab, int r0, int nr,
                                              float (*Bs)[kMR + 4], Load load, Emit emit) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, i16 = lane & 15, k4 = lane >> 4;
  const int arow = slab * kRows + w * 16 + i16;
  const bool aval = arow < R;
  const float* mp = M + (aval ? arow : 0);
  float4_t acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = (float4_t){0.f, 0.f, 0.f, 0.f};
  float an[4], bn[4];
  auto fetch = [&](int c0) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int kc = c0 + ks * 4 + k4;
      an[ks] = (aval && kc < C) ? mp[(int64_t)kc * R] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + kThreads * u, kk = e & 15, c = e >> 4;
      bn[u] = (c0 + kk < C && c < nr) ? (float)load(c0 + kk, r0 + c) : 0.f;
    }
  };
  if (C > 0) fetch(0);
  for (int c0 = 0; c0 < C; c0 += 16) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + kThreads * u;
      Bs[e & 15][e >> 4] = bn[u];
    }
    float a[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) a[ks] = an[ks];
    __syncthreads();
    if (c0 + 16 < C) fetch(c0 + 16);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ks], Bs[ks * 4 + k4][cb * 16 + i16], acc[cb], 0, 0, 0);
  }
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      // v_mfma_f32_16x16x4f32: item r of lane l holds D[4 (l / 16) + r][l % 16]
      const int row = slab * kRows + w * 16 + 4 * k4 + r, c = cb * 16 + i16;
      if (row < R && c < nr) emit(row, r0 + c, (double)acc[cb][r]);
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void hbs_up_mfma_kernel(
    int rbmax, const int* __restrict__ nin, const int* __restrict__ kk, const int64_t* __restrict__ in_off,
    const int64_t* __restrict__ kout_off, const int64_t* __restrict__ up_off, const T* __restrict__ gen,
    const double* __restrict__ in, int64_t ld_in, double* __restrict__ bhat, int64_t ld_bhat,
    double* __restrict__ gb, int64_t ld_gb, int nrhs) {
  __shared__ double Bs[16][kMR + 2];
  const int j = blockIdx.x / rbmax, rb = blockIdx.x - j * rbmax;
  const int n = nin[j], k = kk[j], R = k + n;
  if (rb * kRows >= R) return;
  const int r0 = blockIdx.y * kMR, nr = min(kMR, nrhs - r0);
  const int64_t io = in_off[j], ko = kout_off[j];
  slab_mfma<T>(
      gen + up_off[j], R, n, rb, r0, nr, Bs, [&](int col, int c) { return in[io + col + (int64_t)c * ld_in]; },
      [&](int row, int c, double v) {
        if (row < k) bhat[ko + row + (int64_t)c * ld_bhat] = v;
        else gb[io + (row - k) + (int64_t)c * ld_gb] = v;
      });
}

template <typename T>
__global__ __launch_bounds__(kThreads) void hbs_down_mfma_kernel(
    int rbmax, const int* __restrict__ nin, const int* __restrict__ kk, const int64_t* __restrict__ in_off,
    const int64_t* __restrict__ kout_off, const int64_t* __restrict__ e_off, const T* __restrict__ gen,
    const double* __restrict__ xhat, int64_t ld_xh, const double* __restrict__ gb, int64_t ld_gb,
    double* __restrict__ out, int64_t ld_out, int nrhs) {
  __shared__ double Bs[16][kMR + 2];
  const int j = blockIdx.x / rbmax, rb = blockIdx.x - j * rbmax;
  const int n = nin[j], k = kk[j];
  if (rb * kRows >= n) return;
  const int r0 = blockIdx.y * kMR, nr = min(kMR, nrhs - r0);
  const int64_t io = in_off[j], ko = kout_off[j];
  slab_mfma<T>(
      gen + e_off[j], n, k, rb, r0, nr, Bs, [&](int col, int c) { return xhat[ko + col + (int64_t)c * ld_xh]; },
      [&](int row, int c, double v) {
        out[io + row + (int64_t)c * ld_out] = v + gb[io + row + (int64_t)c * ld_gb];
      });
}

// BF16 generators on the BF16 matrix cores (v_mfma_f32_16x16x16bf16_1k, FP32
// accumulation).  The input tile is split into a high and a low BF16 part
// (x = hi + lo to about 16 bits) and both are multiplied, so only the
// generators carry BF16 rounding.  Lane l supplies A(l % 16, 4 (l / 16) + t)
// and B(4 (l / 16) + t, l % 16), t = 0..3; item r of the result is
// D(4 (l / 16) + r, l % 16) (both checked with an in-bounds probe).
typedef short short4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

template <typename Load, typename Emit>
__device__ __forceinline__ void slab_mfma_bf16(const uint16_t* __restrict__ M, int R, int C, int slab, int r0, int nr,
                                               short (*Bh)[kMR + 8], short (*Bl)[kMR + 8], Load load, Emit emit) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, i16 = lane & 15, k4 = lane >> 4;
  const int arow = slab * kRows + w * 16 + i16;
  const bool aval = arow < R;
  const uint16_t* mp = M + (aval ? arow : 0);
  float4_t acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = (float4_t){0.f, 0.f, 0.f, 0.f};
  for (int c0 = 0; c0 < C; c0 += 16) {
    short4_t a;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int kc = c0 + 4 * k4 + t;
      a[t] = (aval && kc < C) ? (short)mp[(int64_t)kc * R] : (short)0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + kThreads * u, kk = e & 15, c = e >> 4;
      const float v = (c0 + kk < C && c < nr) ? (float)load(c0 + kk, r0 + c) : 0.f;
      const short hi = bf16_rne(v);
      Bh[kk][c] = hi;
      Bl[kk][c] = bf16_rne(v - __uint_as_float((unsigned)(unsigned short)hi << 16));
    }
    __syncthreads();
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      short4_t bh, bl;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        bh[t] = Bh[4 * k4 + t][cb * 16 + i16];
        bl[t] = Bl[4 * k4 + t][cb * 16 + i16];
      }
      acc[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bh, acc[cb], 0, 0, 0);
      acc[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bl, acc[cb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = slab * kRows + w * 16 + 4 * k4 + r, c = cb * 16 + i16;
      if (row < R && c < nr) emit(row, r0 + c, (double)acc[cb][r]);
    }
}

__global__ __launch_bounds__(kThreads) void hbs_up_mfma16_kernel(
    int rbmax, const int* __restrict__ nin, const int* __restrict__ kk, const int64_t* __restrict__ in_off,
    const int64_t* __restrict__ kout_off, const int64_t* __restrict__ up_off, const uint16_t* __restrict__ gen,
    const double* __restrict__ in, int64_t ld_in, double* __restrict__ bhat, int64_t ld_bhat,
    double* __restrict__ gb, int64_t ld_gb, int nrhs) {
  __shared__ short Bh[16][kMR + 8], Bl[16][kMR + 8];
  const int j = blockIdx.x / rbmax, rb = blockIdx.x - j * rbmax;
  const int n = nin[j], k = kk[j], R = k + n;
  if (rb * kRows >= R) return;
  const int r0 = blockIdx.y * kMR, nr = min(kMR, nrhs - r0);
  const int64_t io = in_off[j], ko = kout_off[j];
  slab_mfma_bf16(
      gen + up_off[j], R, n, rb, r0, nr, Bh, Bl, [&](int col, int c) { return in[io + col + (int64_t)c * ld_in]; },
      [&](int row, int c, double v) {
        if (row < k) bhat[ko + row + (int64_t)c * ld_bhat] = v;
        else gb[io + (row - k) + (int64_t)c * ld_gb] = v;
      });
}

__global__ __launch_bounds__(kThreads) void hbs_down_mfma16_kernel(
    int rbmax, const int* __restrict__ nin, const int* __restrict__ kk, const int64_t* __restrict__ in_off,
    const int64_t* __restrict__ kout_off, const int64_t* __restrict__ e_off, const uint16_t* __restrict__ gen,
    const double* __restrict__ xhat, int64_t ld_xh, const double* __restrict__ gb, int64_t ld_gb,
    double* __restrict__ out, int64_t ld_out, int nrhs) {
  __shared__ short Bh[16][kMR + 8], Bl[16][kMR + 8];
  const int j = blockIdx.x / rbmax, rb = blockIdx.x - j * rbmax;
  const int n = nin[j], k = kk[j];
  if (rb * kRows >= n) return;
  const int r0 = blockIdx.y * kMR, nr = min(kMR, nrhs - r0);
  const int64_t io = in_off[j], ko = kout_off[j];
  slab_mfma_bf16(
      gen + e_off[j], n, k, rb, r0, nr, Bh, Bl, [&](int col, int c) { return xhat[ko + col + (int64_t)c * ld_xh]; },
      [&](int row, int c, double v) {
        out[io + row + (int64_t)c * ld_out] = v + gb[io + row + (int64_t)c * ld_gb];
      });
}

__global__ __launch_bounds__(kThreads) void hbs_up_mfma32_kernel(
    int rbmax, const int* __restrict__ nin, const int* __restrict__ kk, const int64_t* __restrict__ in_off,
    const int64_t* __restrict__ kout_off, const int64_t* __restrict__ up_off, const float* __restrict__ gen,
    const double* __restrict__ in, int64_t ld_in, double* __restrict__ bhat, int64_t ld_bhat,
    double* __restrict__ gb, int64_t ld_gb, int nrhs) {
  __shared__ float Bs[16][kMR + 4];
  const int j = blockIdx.x / rbmax, rb = blockIdx.x - j * rbmax;
  const int n = nin[j], k = kk[j], R = k + n;
  if (rb * kRows >= R) return;
  const int r0 = blockIdx.y * kMR, nr = min(kMR, nrhs - r0);
  const int64_t io = in_off[j], ko = kout_off[j];
  slab_mfma_f32(
      gen + up_off[j], R, n, rb, r0, nr, Bs, [&](int col, int c) { return in[io + col + (int64_t)c * ld_in]; },
      [&](int row, int c, double v) {
        if (row < k) bhat[ko + row + (int64_t)c * ld_bhat] = v;
        else gb[io + (row - k) + (int64_t)c * ld_gb] = v;
      });
}

__global__ __launch_bounds__(kThreads) void hbs_down_mfma32_kernel(
    int rbmax, const int* __restrict__ nin, const int* __restrict__ kk, const int64_t* __restrict__ in_off,
    const int64_t* __restrict__ kout_off, const int64_t* __restrict__ e_off, const float* __restrict__ gen,
    const double* __restrict__ xhat, int64_t ld_xh, const double* __restrict__ gb, int64_t ld_gb,
    double* __restrict__ out, int64_t ld_out, int nrhs) {
  __shared__ float Bs[16][kMR + 4];
  const int j = blockIdx.x / rbmax, rb = blockIdx.x - j * rbmax;
  const int n = nin[j], k = kk[j];
  if (rb * kRows >= n) return;
  const int r0 = blockIdx.y * kMR, nr = min(kMR, nrhs - r0);
  const int64_t io = in_off[j], ko = kout_off[j];
  slab_mfma_f32(
      gen + e_off[j], n, k, rb, r0, nr, Bs, [&](int col, int c) { return xhat[ko + col + (int64_t)c * ld_xh]; },
      [&](int row, int c, double v) {
        out[io + row + (int64_t)c * ld_out] = v + gb[io + row + (int64_t)c * ld_gb];
      });
}

__global__ __launch_bounds__(kThreads) void hbs_root_mfma_kernel(int nmax, const int* __restrict__ n_dev,
                                                                 const double* __restrict__ G,
                                                                 const double* __restrict__ in, int64_t ld_in,
                                                                 double* __restrict__ out, int64_t ld_out, int nrhs) {
  __shared__ double Bs[16][kMR + 2];
  const int n = n_dev ? min(*n_dev, nmax) : nmax;
  if (blockIdx.x * kRows >= n) return;
  const int r0 = blockIdx.y * kMR, nr = min(kMR, nrhs - r0);
  slab_mfma<double>(
      G, n, n, blockIdx.x, r0, nr, Bs, [&](int col, int c) { return in[col + (int64_t)c * ld_in]; },
      [&](int row, int c, double v) { out[row + (int64_t)c * ld_out] = v; });
}

// ------------------------------------------ one right-hand side (split)
// With one right-hand side every level is a batch of small GEMVs whose time
// is the latency of the loads, not their bytes.  Each workgroup therefore
// takes one slab of 64 rows and one split of at most kSplit columns of a
// node's block: lane l owns row l, wave w columns 16 w .. 16 w + 15 of the
// split, so every lane issues its loads in one round.  The split's partial
// product goes to a partial vector of its own; the kernel that consumes the
// vector sums the partials while it stages its input, so no separate
// reduction runs and no atomics are needed.  A partial vector is written
// for every split of every row of every node (zeros where a node has fewer
// columns than the level's splits), so the consumer can sum them all.
constexpr int kSplit = 64;

// Partial vectors: part p of element i at base[p * stride + i].
struct Parts {
  const double* base;
  int64_t stride;
  int np;
};

// Sum of the partials of element i: up to 16 loads issued at once (one
// memory round trip), then a fixed-order sum.
__device__ __forceinline__ double parts_sum(const Parts& P, int64_t i) {
  double t[16];
#pragma unroll
  for (int p = 0; p < 16; ++p) t[p] = p < P.np ? P.base[(int64_t)p * P.stride + i] : 0.0;
  double v = ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7])) +
             (((t[8] + t[9]) + (t[10] + t[11])) + ((t[12] + t[13]) + (t[14] + t[15])));
  for (int p = 16; p < P.np; ++p) v += P.base[(int64_t)p * P.stride + i];
  return v;
}

// Loads of this lane (row `row` of M, R x C, ld R; columns of wave w in the
// split starting at c0), issued before the input is staged.
template <typename T>
__device__ __forceinline__ void split_load(const T* __restrict__ M, int R, int C, int row, int c0, int w,
                                           double (&m)[16]) {
  const int cw = c0 + 16 * w;
  const bool rv = row < R;
#pragma unroll
  for (int u = 0; u < 16; ++u) m[u] = (rv && cw + u < C) ? (double)M[row + (int64_t)(cw + u) * R] : 0.0;
}

// This wave's part of the dot product (four independent sums), the four
// waves' parts added through LDS; every lane of wave 0 returns its row's sum.
__device__ __forceinline__ double split_dot(const double (&m)[16], const double* xs, int w, double* red) {
  const int lane = threadIdx.x & 63;
  const double* x = xs + 16 * w;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
  for (int u = 0; u < 16; u += 4) {
    a0 = fma(m[u], x[u], a0);
    a1 = fma(m[u + 1], x[u + 1], a1);
    a2 = fma(m[u + 2], x[u + 2], a2);
    a3 = fma(m[u + 3], x[u + 3], a3);
  }
  red[w * 64 + lane] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  return (red[lane] + red[64 + lane]) + (red[128 + lane] + red[192 + lane]);
}

// grid (nodes * rbmax * ns).  [bhat; gb] partials = [F*; G](:, split) b(split).
template <typename T>
__global__ __launch_bounds__(kThreads) void hbs_up1_kernel(int rbmax, int ns, const int* __restrict__ nin,
                                                           const int* __restrict__ kk,
                                                           const int64_t* __restrict__ in_off,
                                                           const int64_t* __restrict__ kout_off,
                                                           const int64_t* __restrict__ up_off,
                                                           const T* __restrict__ gen, Parts in, double* __restrict__ bhat,
                                                           int64_t bstride, double* __restrict__ gb,
                                                           int64_t gstride) {
  __shared__ double xs[kSplit];
  __shared__ double red[4 * 64];
  const int b = blockIdx.x;
  const int j = b / (rbmax * ns), rem = b - j * rbmax * ns, rb = rem / ns, sp = rem - rb * ns;
  const int n = nin[j], k = kk[j], R = k + n;
  if (rb * kRows >= R) return;  // whole workgroup
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int row = rb * kRows + lane, c0 = sp * kSplit;
  double m[16];
  split_load<T>(gen + up_off[j], R, n, row, c0, w, m);
  const int64_t io = in_off[j];
  if (tid < kSplit) xs[tid] = c0 + tid < n ? parts_sum(in, io + c0 + tid) : 0.0;
  __syncthreads();
  const double v = split_dot(m, xs, w, red);
  if (w == 0 && row < R) {
    if (row < k) bhat[(int64_t)sp * bstride + kout_off[j] + row] = v;
    else gb[(int64_t)sp * gstride + io + (row - k)] = v;
  }
}

// grid (nodes * rbmax * ns).  out partials = E(:, split) xhat(split) (+ gb in split 0).
template <typename T>
__global__ __launch_bounds__(kThreads) void hbs_down1_kernel(int rbmax, int ns, const int* __restrict__ nin,
                                                             const int* __restrict__ kk,
                                                             const int64_t* __restrict__ in_off,
                                                             const int64_t* __restrict__ kout_off,
                                                             const int64_t* __restrict__ e_off,
                                                             const T* __restrict__ gen, Parts xhat, Parts gb,
                                                             double* __restrict__ out, int64_t ostride) {
  __shared__ double xs[kSplit];
  __shared__ double red[4 * 64];
  const int b = blockIdx.x;
  const int j = b / (rbmax * ns), rem = b - j * rbmax * ns, rb = rem / ns, sp = rem - rb * ns;
  const int n = nin[j], k = kk[j];
  if (rb * kRows >= n) return;  // whole workgroup
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int row = rb * kRows + lane, c0 = sp * kSplit;
  double m[16];
  split_load<T>(gen + e_off[j], n, k, row, c0, w, m);
  const int64_t io = in_off[j];
  double g = 0.0;
  if (sp == 0 && w == 0 && row < n) g = parts_sum(gb, io + row);
  if (tid < kSplit) xs[tid] = c0 + tid < k ? parts_sum(xhat, kout_off[j] + c0 + tid) : 0.0;
  __syncthreads();
  const double v = split_dot(m, xs, w, red);
  if (w == 0 && row < n) out[(int64_t)sp * ostride + io + row] = v + g;
}

// grid (rbmax * ns).  out partials = G_root(:, split) in(split); the root
// size is n_dev[0] when n_dev is given (at most nmax), else nmax.
__global__ __launch_bounds__(kThreads) void hbs_root1_kernel(int nmax, int ns, const int* __restrict__ n_dev,
                                                             const double* __restrict__ G, Parts in,
                                                             double* __restrict__ out, int64_t ostride) {
  __shared__ double xs[kSplit];
  __shared__ double red[4 * 64];
  const int n = n_dev ? min(*n_dev, nmax) : nmax;
  const int rb = blockIdx.x / ns, sp = blockIdx.x - rb * ns;
  if (rb * kRows >= n) return;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int row = rb * kRows + lane, c0 = sp * kSplit;
  double m[16];
  split_load<double>(G, n, n, row, c0, w, m);
  if (tid < kSplit) xs[tid] = c0 + tid < n ? parts_sum(in, c0 + tid) : 0.0;
  __syncthreads();
  const double v = split_dot(m, xs, w, red);
  if (w == 0 && row < n) out[(int64_t)sp * ostride + row] = v;
}

// x = sum of the partials (a leaf level whose E has more than kSplit columns).
__global__ __launch_bounds__(kThreads) void parts_reduce_kernel(Parts in, int64_t n, double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) x[i] = parts_sum(in, i);
}

inline size_t slab_lds(int xs_len, int rb) {
  const size_t b = sizeof(double) * ((size_t)xs_len + 4 * (size_t)rb * kRows);
  if (b > 64 * 1024) RW_THROW(RW_EINVAL, "HBS node too large for the apply kernels");
  return b;
}

template <typename T, int RB>
void up_launch(const HbsLevelDev& L, const T* gen, const double* in, int64_t ld_in, double* bhat, int64_t ld_bhat,
               double* gb, int64_t ld_gb, int nrhs, hipStream_t s) {
  const int rbmax = (L.max_k + L.max_nin + kRows - 1) / kRows;
  const int xs_len = L.max_nin * RB;
  dim3 grid(L.nnodes * rbmax, (nrhs + RB - 1) / RB);
  hipLaunchKernelGGL((hbs_up_kernel<T, RB>), grid, dim3(kThreads), slab_lds(xs_len, RB), s, rbmax, L.nin, L.k,
                     L.in_off, L.kout_off, L.up_off, gen, in, ld_in, bhat, ld_bhat, gb, ld_gb, nrhs, xs_len);
}

template <typename T>
void up_impl(const HbsLevelDev& L, const T* gen, const double* in, int64_t ld_in, double* bhat,
             int64_t ld_bhat, double* gb, int64_t ld_gb, int nrhs, int mfma_from, hipStream_t s) {
  if (!L.nnodes || nrhs <= 0) return;
  if (mfma_from <= 0) mfma_from = mfma_min<T>();
  // generators streamed once per pass of up to 8 right-hand sides
  const double passes = nrhs == 1 ? 1.0 : (nrhs < mfma_from ? (nrhs + 7) / 8 : (nrhs + kMR - 1) / kMR);
  KernelTimer kt("hbs_up_kernel", 2.0 * L.up_entries * nrhs, sizeof(T) * (double)L.up_entries * passes, s);
  if (nrhs == 1) {
    up_launch<T, 1>(L, gen, in, ld_in, bhat, ld_bhat, gb, ld_gb, nrhs, s);
  } else if (nrhs < mfma_from) {
    up_launch<T, 8>(L, gen, in, ld_in, bhat, ld_bhat, gb, ld_gb, nrhs, s);
  } else {
    const int rbmax = (L.max_k + L.max_nin + kRows - 1) / kRows;
    const dim3 grid(L.nnodes * rbmax, (nrhs + kMR - 1) / kMR);
    if constexpr (sizeof(T) == 4)
      hipLaunchKernelGGL(hbs_up_mfma32_kernel, grid, dim3(kThreads), 0, s, rbmax, L.nin, L.k, L.in_off, L.kout_off,
                         L.up_off, (const float*)gen, in, ld_in, bhat, ld_bhat, gb, ld_gb, nrhs);
    else if constexpr (sizeof(T) == 2)
      hipLaunchKernelGGL(hbs_up_mfma16_kernel, grid, dim3(kThreads), 0, s, rbmax, L.nin, L.k, L.in_off, L.kout_off,
                         L.up_off, (const uint16_t*)gen, in, ld_in, bhat, ld_bhat, gb, ld_gb, nrhs);
    else
      hipLaunchKernelGGL((hbs_up_mfma_kernel<T>), grid, dim3(kThreads), 0, s, rbmax, L.nin, L.k, L.in_off, L.kout_off,
                         L.up_off, gen, in, ld_in, bhat, ld_bhat, gb, ld_gb, nrhs);
  }
  KERNEL_CHECK("hbs_up");
}

template <typename T, int RB>
void down_launch(const HbsLevelDev& L, const T* gen, const double* xhat, int64_t ld_xh, const double* gb,
                 int64_t ld_gb, double* out, int64_t ld_out, int nrhs, hipStream_t s) {
  const int rbmax = (L.max_nin + kRows - 1) / kRows;
  const int xs_len = (L.max_k > 0 ? L.max_k : 1) * RB;
  dim3 grid(L.nnodes * rbmax, (nrhs + RB - 1) / RB);
  hipLaunchKernelGGL((hbs_down_kernel<T, RB>), grid, dim3(kThreads), slab_lds(xs_len, RB), s, rbmax, L.nin, L.k,
                     L.in_off, L.kout_off, L.e_off, gen, xhat, ld_xh, gb, ld_gb, out, ld_out, nrhs, xs_len);
}

template <typename T>
void down_impl(const HbsLevelDev& L, const T* gen, const double* xhat, int64_t ld_xh, const double* gb,
               int64_t ld_gb, double* out, int64_t ld_out, int nrhs, int mfma_from, hipStream_t s) {
  if (!L.nnodes || nrhs <= 0) return;
  if (mfma_from <= 0) mfma_from = mfma_min<T>();
  const double passes = nrhs == 1 ? 1.0 : (nrhs < mfma_from ? (nrhs + 7) / 8 : (nrhs + kMR - 1) / kMR);
  KernelTimer kt("hbs_down_kernel", 2.0 * L.e_entries * nrhs, sizeof(T) * (double)L.e_entries * passes, s);
  if (nrhs == 1) {
    down_launch<T, 1>(L, gen, xhat, ld_xh, gb, ld_gb, out, ld_out, nrhs, s);
  } else if (nrhs < mfma_from) {
    down_launch<T, 8>(L, gen, xhat, ld_xh, gb, ld_gb, out, ld_out, nrhs, s);
  } else {
    const int rbmax = (L.max_nin + kRows - 1) / kRows;
    const dim3 grid(L.nnodes * rbmax, (nrhs + kMR - 1) / kMR);
    if constexpr (sizeof(T) == 4)
      hipLaunchKernelGGL(hbs_down_mfma32_kernel, grid, dim3(kThreads), 0, s, rbmax, L.nin, L.k, L.in_off, L.kout_off,
                         L.e_off, (const float*)gen, xhat, ld_xh, gb, ld_gb, out, ld_out, nrhs);
    else if constexpr (sizeof(T) == 2)
      hipLaunchKernelGGL(hbs_down_mfma16_kernel, grid, dim3(kThreads), 0, s, rbmax, L.nin, L.k, L.in_off,
                         L.kout_off, L.e_off, (const uint16_t*)gen, xhat, ld_xh, gb, ld_gb, out, ld_out, nrhs);
    else
      hipLaunchKernelGGL((hbs_down_mfma_kernel<T>), grid, dim3(kThreads), 0, s, rbmax, L.nin, L.k, L.in_off,
                         L.kout_off, L.e_off, gen, xhat, ld_xh, gb, ld_gb, out, ld_out, nrhs);
  }
  KERNEL_CHECK("hbs_down");
}

}  // namespace

int hbs_split_count(int ncols) { return ncols <= 0 ? 1 : (ncols + kSplit - 1) / kSplit; }

namespace {
template <typename T>
void up1_impl(const HbsLevelDev& L, const T* gen, const double* in, int64_t in_stride, int in_np, double* bhat,
              int64_t bstride, double* gb, int64_t gstride, hipStream_t s) {
  if (!L.nnodes) return;
  const int rbmax = (L.max_k + L.max_nin + kRows - 1) / kRows, ns = hbs_split_count(L.max_nin);
  KernelTimer kt("hbs_up_kernel", 2.0 * L.up_entries, sizeof(T) * (double)L.up_entries, s);
  hipLaunchKernelGGL((hbs_up1_kernel<T>), dim3(L.nnodes * rbmax * ns), dim3(kThreads), 0, s, rbmax, ns, L.nin, L.k,
                     L.in_off, L.kout_off, L.up_off, gen, Parts{in, in_stride, in_np}, bhat, bstride, gb, gstride);
  KERNEL_CHECK("hbs_up1");
}
template <typename T>
void down1_impl(const HbsLevelDev& L, const T* gen, const double* xh, int64_t xstride, int xnp, const double* gb,
                int64_t gstride, int gnp, double* out, int64_t ostride, hipStream_t s) {
  if (!L.nnodes) return;
  const int rbmax = (L.max_nin + kRows - 1) / kRows, ns = hbs_split_count(L.max_k);
  KernelTimer kt("hbs_down_kernel", 2.0 * L.e_entries, sizeof(T) * (double)L.e_entries, s);
  hipLaunchKernelGGL((hbs_down1_kernel<T>), dim3(L.nnodes * rbmax * ns), dim3(kThreads), 0, s, rbmax, ns, L.nin,
                     L.k, L.in_off, L.kout_off, L.e_off, gen, Parts{xh, xstride, xnp}, Parts{gb, gstride, gnp}, out,
                     ostride);
  KERNEL_CHECK("hbs_down1");
}
}  // namespace

void launch_hbs_up1(const HbsLevelDev& L, const double* gen, const float* gen32, const double* in, int64_t in_stride,
                    int in_np, double* bhat, int64_t bstride, double* gb, int64_t gstride, hipStream_t s,
                    const uint16_t* gen16) {
  if (gen16) up1_impl<bf16s>(L, (const bf16s*)gen16, in, in_stride, in_np, bhat, bstride, gb, gstride, s);
  else if (gen32) up1_impl<float>(L, gen32, in, in_stride, in_np, bhat, bstride, gb, gstride, s);
  else up1_impl<double>(L, gen, in, in_stride, in_np, bhat, bstride, gb, gstride, s);
}
void launch_hbs_down1(const HbsLevelDev& L, const double* gen, const float* gen32, const double* xh, int64_t xstride,
                      int xnp, const double* gb, int64_t gstride, int gnp, double* out, int64_t ostride,
                      hipStream_t s, const uint16_t* gen16) {
  if (gen16) down1_impl<bf16s>(L, (const bf16s*)gen16, xh, xstride, xnp, gb, gstride, gnp, out, ostride, s);
  else if (gen32) down1_impl<float>(L, gen32, xh, xstride, xnp, gb, gstride, gnp, out, ostride, s);
  else down1_impl<double>(L, gen, xh, xstride, xnp, gb, gstride, gnp, out, ostride, s);
}
void launch_hbs_up_bf16(const HbsLevelDev& L, const uint16_t* gen, const double* in, int64_t ld_in, double* bhat,
                        int64_t ld_bhat, double* gb, int64_t ld_gb, int nrhs, hipStream_t s, int mfma_from) {
  up_impl<bf16s>(L, (const bf16s*)gen, in, ld_in, bhat, ld_bhat, gb, ld_gb, nrhs, mfma_from, s);
}
void launch_hbs_down_bf16(const HbsLevelDev& L, const uint16_t* gen, const double* xhat, int64_t ld_xh,
                          const double* gb, int64_t ld_gb, double* out, int64_t ld_out, int nrhs, hipStream_t s,
                          int mfma_from) {
  down_impl<bf16s>(L, (const bf16s*)gen, xhat, ld_xh, gb, ld_gb, out, ld_out, nrhs, mfma_from, s);
}
void launch_hbs_root1(int nroot, const int* d_nroot, const double* G, const double* in, int64_t in_stride, int in_np,
                      double* out, int64_t ostride, hipStream_t s) {
  if (nroot <= 0) return;
  const int rbmax = (nroot + kRows - 1) / kRows, ns = hbs_split_count(nroot);
  hipLaunchKernelGGL(hbs_root1_kernel, dim3(rbmax * ns), dim3(kThreads), 0, s, nroot, ns, d_nroot, G,
                     Parts{in, in_stride, in_np}, out, ostride);
  KERNEL_CHECK("hbs_root1");
}
void launch_parts_reduce(const double* in, int64_t stride, int np, int64_t n, double* x, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(parts_reduce_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                     Parts{in, stride, np}, n, x);
  KERNEL_CHECK("parts_reduce");
}

double hbs_gen_passes(int nrhs, bool narrow) {
  if (nrhs <= 1) return 1.0;
  return nrhs < (narrow ? kMfmaMin32 : kMfmaMin) ? (double)((nrhs + 7) / 8) : (double)((nrhs + kMR - 1) / kMR);
}

void launch_hbs_up(const HbsLevelDev& L, const double* gen, const double* in, int64_t ld_in, double* bhat,
                   int64_t ld_bhat, double* gb, int64_t ld_gb, int nrhs, hipStream_t s, int mfma_from) {
  up_impl<double>(L, gen, in, ld_in, bhat, ld_bhat, gb, ld_gb, nrhs, mfma_from, s);
}
void launch_hbs_up_f32(const HbsLevelDev& L, const float* gen, const double* in, int64_t ld_in,
                       double* bhat, int64_t ld_bhat, double* gb, int64_t ld_gb, int nrhs, hipStream_t s,
                       int mfma_from) {
  up_impl<float>(L, gen, in, ld_in, bhat, ld_bhat, gb, ld_gb, nrhs, mfma_from, s);
}
void launch_hbs_down(const HbsLevelDev& L, const double* gen, const double* xhat, int64_t ld_xh,
                     const double* gb, int64_t ld_gb, double* out, int64_t ld_out, int nrhs, hipStream_t s,
                     int mfma_from) {
  down_impl<double>(L, gen, xhat, ld_xh, gb, ld_gb, out, ld_out, nrhs, mfma_from, s);
}
void launch_hbs_down_f32(const HbsLevelDev& L, const float* gen, const double* xhat, int64_t ld_xh,
                         const double* gb, int64_t ld_gb, double* out, int64_t ld_out, int nrhs,
                         hipStream_t s, int mfma_from) {
  down_impl<float>(L, gen, xhat, ld_xh, gb, ld_gb, out, ld_out, nrhs, mfma_from, s);
}
void launch_hbs_root(int nroot, const int* d_nroot, const double* G, const double* in, int64_t ld_in, double* out,
                     int64_t ld_out, int nrhs, hipStream_t s, int mfma_from) {
  if (nroot <= 0 || nrhs <= 0) return;
  const int nb = (nroot + kRows - 1) / kRows;
  if (mfma_from <= 0) mfma_from = kMfmaMin;
  if (nrhs >= mfma_from) {
    hipLaunchKernelGGL(hbs_root_mfma_kernel, dim3(nb, (nrhs + kMR - 1) / kMR), dim3(kThreads), 0, s, nroot, d_nroot,
                       G, in, ld_in, out, ld_out, nrhs);
  } else if (nrhs == 1) {
    hipLaunchKernelGGL((hbs_root_kernel<1>), dim3(nb, 1), dim3(kThreads), slab_lds(nroot * 1, 1), s, nroot, d_nroot,
                       G, in, ld_in, out, ld_out, nrhs);
  } else {
    hipLaunchKernelGGL((hbs_root_kernel<8>), dim3(nb, (nrhs + 7) / 8), dim3(kThreads), slab_lds(nroot * 8, 8), s,
                       nroot, d_nroot, G, in, ld_in, out, ld_out, nrhs);
  }
  KERNEL_CHECK("hbs_root");
}
