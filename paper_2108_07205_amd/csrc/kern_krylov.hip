// Vector kernels of the preconditioned GMRES driver (Sec. 4): scaling of the
// new Arnoldi vector by the inverse of a norm that stays on the device, and
// a scaled copy.  The inner products and the Gram-Schmidt updates reuse the
// A^T B and Y -= X W kernels of kern_la.hip.
#include "kernels.h"

namespace {

constexpr int kT = 256;

// v = w / sqrt(nrm2[0]); w and v may alias.  A zero norm (an exact
// breakdown) leaves v = 0, which the driver's Hessenberg entry then shows.
__global__ __launch_bounds__(kT) void scale_rsqrt_kernel(const double* __restrict__ w, int64_t n,
                                                         const double* __restrict__ nrm2, double* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  const double s = nrm2[0] > 0.0 ? 1.0 / sqrt(nrm2[0]) : 0.0;
  if (i < n) v[i] = w[i] * s;
}

// y = a x
__global__ __launch_bounds__(kT) void scale_copy_kernel(const double* __restrict__ x, int64_t n, double a,
                                                        double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

unsigned nblk(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

}  // namespace

void launch_scale_rsqrt(const double* w, int64_t n, const double* nrm2, double* v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(scale_rsqrt_kernel, dim3(nblk(n)), dim3(kT), 0, s, w, n, nrm2, v);
  KERNEL_CHECK("scale_rsqrt");
}

void launch_scale_copy(const double* x, int64_t n, double a, double* y, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(scale_copy_kernel, dim3(nblk(n)), dim3(kT), 0, s, x, n, a, y);
  KERNEL_CHECK("scale_copy");
}
