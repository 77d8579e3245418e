// HBS inverse apply: level sweeps over packed generators (Algorithm 1, solve
// step 1, the A_oo^{-1} block; also Algorithm 1 pre-computation step 3 with
// many right-hand sides).
//
// Per node the generators are streamed once per right-hand-side chunk:
// [F*; G] is stored column-major with (k + nin) rows, so thread `row` reads
// consecutive addresses for consecutive rows (coalesced) while the node's
// input is staged in LDS; E likewise with nin rows.  One workgroup per node.
#include "kernels.h"

namespace {

constexpr int kThreads = 256;
constexpr int kRB = 8;  // right-hand sides per pass

template <typename T>
__global__ __launch_bounds__(kThreads) void hbs_up_kernel(
    const int* __restrict__ nin, const int* __restrict__ kk, const int64_t* __restrict__ in_off,
    const int64_t* __restrict__ kout_off, const int64_t* __restrict__ up_off, const T* __restrict__ gen,
    const double* __restrict__ in, int64_t ld_in, double* __restrict__ bhat, int64_t ld_bhat,
    double* __restrict__ gb, int64_t ld_gb, int nrhs) {
  extern __shared__ double sb[];
  const int j = blockIdx.x;
  const int r0 = blockIdx.y * kRB;
  const int nr = min(kRB, nrhs - r0);
  const int n = nin[j], k = kk[j];
  const int64_t io = in_off[j];
  for (int idx = threadIdx.x; idx < n * kRB; idx += kThreads) {
    const int c = idx / n, i = idx - c * n;
    sb[idx] = (c < nr) ? in[io + i + (int64_t)(r0 + c) * ld_in] : 0.0;
  }
  __syncthreads();
  const T* M = gen + up_off[j];
  const int rows = k + n;
  const int64_t ko = kout_off[j];
  for (int row = threadIdx.x; row < rows; row += kThreads) {
    double acc[kRB];
#pragma unroll
    for (int c = 0; c < kRB; ++c) acc[c] = 0.0;
    const T* mp = M + row;
#pragma unroll 4
    for (int col = 0; col < n; ++col) {
      const double m = (double)mp[(int64_t)col * rows];
#pragma unroll
      for (int c = 0; c < kRB; ++c) acc[c] += m * sb[c * n + col];
    }
    if (row < k) {
      for (int c = 0; c < nr; ++c) bhat[ko + row + (int64_t)(r0 + c) * ld_bhat] = acc[c];
    } else {
      for (int c = 0; c < nr; ++c) gb[io + (row - k) + (int64_t)(r0 + c) * ld_gb] = acc[c];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void hbs_down_kernel(
    const int* __restrict__ nin, const int* __restrict__ kk, const int64_t* __restrict__ in_off,
    const int64_t* __restrict__ kout_off, const int64_t* __restrict__ e_off, const T* __restrict__ gen,
    const double* __restrict__ xhat, int64_t ld_xh, const double* __restrict__ gb, int64_t ld_gb,
    double* __restrict__ out, int64_t ld_out, int nrhs) {
  extern __shared__ double sx[];
  const int j = blockIdx.x;
  const int r0 = blockIdx.y * kRB;
  const int nr = min(kRB, nrhs - r0);
  const int n = nin[j], k = kk[j];
  const int64_t io = in_off[j], ko = kout_off[j];
  for (int idx = threadIdx.x; idx < k * kRB; idx += kThreads) {
    const int c = idx / k, i = idx - c * k;
    sx[idx] = (c < nr) ? xhat[ko + i + (int64_t)(r0 + c) * ld_xh] : 0.0;
  }
  __syncthreads();
  const T* E = gen + e_off[j];
  for (int row = threadIdx.x; row < n; row += kThreads) {
    double acc[kRB];
#pragma unroll
    for (int c = 0; c < kRB; ++c) acc[c] = (c < nr) ? gb[io + row + (int64_t)(r0 + c) * ld_gb] : 0.0;
    const T* ep = E + row;
#pragma unroll 4
    for (int col = 0; col < k; ++col) {
      const double e = (double)ep[(int64_t)col * n];
#pragma unroll
      for (int c = 0; c < kRB; ++c) acc[c] += e * sx[c * k + col];
    }
    for (int c = 0; c < nr; ++c) out[io + row + (int64_t)(r0 + c) * ld_out] = acc[c];
  }
}

__global__ __launch_bounds__(kThreads) void hbs_root_kernel(int n, const double* __restrict__ G,
                                                            const double* __restrict__ in, int64_t ld_in,
                                                            double* __restrict__ out, int64_t ld_out,
                                                            int nrhs) {
  extern __shared__ double sb[];
  const int r0 = blockIdx.y * kRB;
  const int nr = min(kRB, nrhs - r0);
  for (int idx = threadIdx.x; idx < n * kRB; idx += kThreads) {
    const int c = idx / n, i = idx - c * n;
    sb[idx] = (c < nr) ? in[i + (int64_t)(r0 + c) * ld_in] : 0.0;
  }
  __syncthreads();
  for (int row = blockIdx.x * kThreads + threadIdx.x; row < n; row += gridDim.x * kThreads) {
    double acc[kRB];
#pragma unroll
    for (int c = 0; c < kRB; ++c) acc[c] = 0.0;
    for (int col = 0; col < n; ++col) {
      const double g = G[row + (int64_t)col * n];
#pragma unroll
      for (int c = 0; c < kRB; ++c) acc[c] += g * sb[c * n + col];
    }
    for (int c = 0; c < nr; ++c) out[row + (int64_t)(r0 + c) * ld_out] = acc[c];
  }
}

template <typename T>
void up_impl(const HbsLevelDev& L, const T* gen, const double* in, int64_t ld_in, double* bhat,
             int64_t ld_bhat, double* gb, int64_t ld_gb, int nrhs, hipStream_t s) {
  if (!L.nnodes || nrhs <= 0) return;
  dim3 grid(L.nnodes, (nrhs + kRB - 1) / kRB);
  const size_t sh = sizeof(double) * L.max_nin * kRB;
  // generators streamed once per pass of kRB right-hand sides
  const double passes = (nrhs + kRB - 1) / kRB;
  KernelTimer kt("hbs_up_kernel", 2.0 * L.up_entries * nrhs, sizeof(T) * (double)L.up_entries * passes);
  hipLaunchKernelGGL(hbs_up_kernel<T>, grid, dim3(kThreads), sh, s, L.nin, L.k, L.in_off, L.kout_off,
                     L.up_off, gen, in, ld_in, bhat, ld_bhat, gb, ld_gb, nrhs);
  KERNEL_CHECK("hbs_up");
}

template <typename T>
void down_impl(const HbsLevelDev& L, const T* gen, const double* xhat, int64_t ld_xh, const double* gb,
               int64_t ld_gb, double* out, int64_t ld_out, int nrhs, hipStream_t s) {
  if (!L.nnodes || nrhs <= 0) return;
  dim3 grid(L.nnodes, (nrhs + kRB - 1) / kRB);
  const size_t sh = sizeof(double) * (L.max_k > 0 ? L.max_k : 1) * kRB;
  const double passes = (nrhs + kRB - 1) / kRB;
  KernelTimer kt("hbs_down_kernel", 2.0 * L.e_entries * nrhs, sizeof(T) * (double)L.e_entries * passes);
  hipLaunchKernelGGL(hbs_down_kernel<T>, grid, dim3(kThreads), sh, s, L.nin, L.k, L.in_off, L.kout_off,
                     L.e_off, gen, xhat, ld_xh, gb, ld_gb, out, ld_out, nrhs);
  KERNEL_CHECK("hbs_down");
}

}  // namespace

void launch_hbs_up(const HbsLevelDev& L, const double* gen, const double* in, int64_t ld_in, double* bhat,
                   int64_t ld_bhat, double* gb, int64_t ld_gb, int nrhs, hipStream_t s) {
  up_impl<double>(L, gen, in, ld_in, bhat, ld_bhat, gb, ld_gb, nrhs, s);
}
void launch_hbs_up_f32(const HbsLevelDev& L, const float* gen, const double* in, int64_t ld_in,
                       double* bhat, int64_t ld_bhat, double* gb, int64_t ld_gb, int nrhs, hipStream_t s) {
  up_impl<float>(L, gen, in, ld_in, bhat, ld_bhat, gb, ld_gb, nrhs, s);
}
void launch_hbs_down(const HbsLevelDev& L, const double* gen, const double* xhat, int64_t ld_xh,
                     const double* gb, int64_t ld_gb, double* out, int64_t ld_out, int nrhs, hipStream_t s) {
  down_impl<double>(L, gen, xhat, ld_xh, gb, ld_gb, out, ld_out, nrhs, s);
}
void launch_hbs_down_f32(const HbsLevelDev& L, const float* gen, const double* xhat, int64_t ld_xh,
                         const double* gb, int64_t ld_gb, double* out, int64_t ld_out, int nrhs,
                         hipStream_t s) {
  down_impl<float>(L, gen, xhat, ld_xh, gb, ld_gb, out, ld_out, nrhs, s);
}
void launch_hbs_root(int nroot, const double* G, const double* in, int64_t ld_in, double* out,
                     int64_t ld_out, int nrhs, hipStream_t s) {
  if (nroot <= 0 || nrhs <= 0) return;
  dim3 grid((nroot + kThreads - 1) / kThreads, (nrhs + kRB - 1) / kRB);
  hipLaunchKernelGGL(hbs_root_kernel, grid, dim3(kThreads), sizeof(double) * nroot * kRB, s, nroot, G, in,
                     ld_in, out, ld_out, nrhs);
  KERNEL_CHECK("hbs_root");
}
