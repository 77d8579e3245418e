// Wave-level maximum of non-negative doubles by DPP row shifts and row
// broadcasts (no LDS round trips), shared by the pivot searches of the
// Gauss-Jordan and row-ID kernels.
#pragma once

#include <hip/hip_runtime.h>

// 64-bit DPP move of v (lanes without a source read 0).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Maximum over the wave of non-negative doubles; lane 63 collects it through
// row_shr 1/2/4/8 and row_bcast 15/31, and it is returned in every lane.
__device__ __forceinline__ double wave_max_nonneg(double v) {
  v = fmax(v, dpp_f64<0x111, 0xf>(v));  // row_shr:1
  v = fmax(v, dpp_f64<0x112, 0xf>(v));  // row_shr:2
  v = fmax(v, dpp_f64<0x114, 0xf>(v));  // row_shr:4
  v = fmax(v, dpp_f64<0x118, 0xf>(v));  // row_shr:8
  v = fmax(v, dpp_f64<0x142, 0xa>(v));  // row_bcast:15
  v = fmax(v, dpp_f64<0x143, 0xc>(v));  // row_bcast:31
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// 1 / x for a finite, normal, nonzero x to within an ulp or two: hardware
// reciprocal and two Newton steps (a shorter dependency chain than the
// correctly rounded division).
__device__ __forceinline__ double recip_nr2(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * (2.0 - x * y);
  return y * (2.0 - x * y);
}

// Pivot key: the non-negative magnitude v with its `bits` lowest mantissa
// bits replaced by (2^bits - 1 - i), so that the largest key belongs to the
// largest v (to 2^(bits-52) relative) and, among equal magnitudes, to the
// lowest index i < 2^bits.  Unusable entries get 0; non-finite magnitudes
// get the largest finite double, so that they are picked (and reported).
template <int BITS>
__device__ __forceinline__ double pivot_key_bits(double v, int i, bool usable) {
  if (!usable) return 0.0;
  const double m = isfinite(v) ? fabs(v) : 1.7976931348623157e308;
  constexpr unsigned long long mask = (1ull << BITS) - 1;
  const unsigned long long b = ((unsigned long long)__double_as_longlong(m) & ~mask) | (unsigned)(mask - i);
  return __longlong_as_double((long long)b);
}
// The same key, branch-free (formed, then selected), for callers whose
// straight-line step should stay one block the scheduler can interleave.
template <int BITS>
__device__ __forceinline__ double pivot_key_bits_sel(double v, int i, bool usable) {
  const double m = isfinite(v) ? fabs(v) : 1.7976931348623157e308;
  constexpr unsigned long long mask = (1ull << BITS) - 1;
  const unsigned long long b = ((unsigned long long)__double_as_longlong(m) & ~mask) | (unsigned)(mask - i);
  return usable ? __longlong_as_double((long long)b) : 0.0;
}
template <int BITS>
__device__ __forceinline__ int pivot_key_index(double key) {
  constexpr unsigned long long mask = (1ull << BITS) - 1;
  return (int)(mask - ((unsigned long long)__double_as_longlong(key) & mask));
}
