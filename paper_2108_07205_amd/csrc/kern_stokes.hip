// Kernels that generate entries of the Stokes Nystrom operator on the fly
// (Sec. 2: A = -1/2 I + D + N with
//   D(x, y) = (1/pi) (r r^T / r^2) (r . n_y / r^2),  r = x - y,
//   N(x, y) = n_x n_y^T, weights w_j folded into the source side).
//
//  * residual r = g - A tau on one discretization (FP64 VALU: one division
//    and ~12 FMAs per 2x2 block and right-hand side);
//  * Stokeslet boundary data (eq. stokeslet, mu = 1);
//  * dense assembly of A(targets, sources);
//  * skeleton rows R of the update matrix Q (uniform row-ID format);
//  * the random sketch Y = A(tgt, src) Omega of the off-diagonal blocks of Q,
//    with the kernel tile generated in registers and contracted on the FP64
//    matrix cores (v_mfma_f64_16x16x4f64); Omega = +-1 from a counter-based
//    hash (SplitMix64 finalizer), so it is never stored.
#include "kernels.h"

namespace {

constexpr double kInvPi = 0.31830988618379067154;

// ---------------------------------------------------------------- residual
constexpr int RT = 128;  // targets per block
constexpr int RRB = 4;   // right-hand sides per pass
constexpr int RT1 = 4;   // targets per thread of the one-right-hand-side kernel

int resid_splits(int64_t n, int nrhs) {
  if (n <= 0 || nrhs <= 0) return 1;
  if (nrhs == 1) {
    // scalar-broadcast kernel: 256 RT1 targets per workgroup; about 8 waves per SIMD
    const int64_t tb = (n + 256 * RT1 - 1) / (256 * RT1);
    int64_t s = (2048 + tb - 1) / tb;
    s = s < 1 ? 1 : (s > 64 ? 64 : s);
    const int64_t maxs = (n + 63) / 64;   // at least 64 sources per split
    return (int)(s > maxs ? maxs : s);
  }
  const int64_t tb = (n + RT - 1) / RT;
  const int64_t chunks = (nrhs + RRB - 1) / RRB;
  int64_t s = (2048 + tb * chunks - 1) / (tb * chunks);
  s = s < 1 ? 1 : (s > 32 ? 32 : s);
  const int64_t maxs = (n + RT - 1) / RT;  // at least one source tile per split
  if (s > maxs) s = maxs;
  return (int)(s < 1 ? 1 : s);
}

// 1 / x (x > 0) to within an ulp or two: hardware reciprocal and two Newton
// steps (cheaper than the correctly rounded division).
__device__ __forceinline__ double rcp_nr2(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * (2.0 - x * y);
  return y * (2.0 - x * y);
}

// The same by one third-order step: with e = 1 - x y0, 1 / x = y0 (1 + e +
// e^2 + ...), so y0 + y0 (e + e^2) leaves a relative error of e^3 plus
// rounding (three operations instead of four).
__device__ __forceinline__ double rcp_nr3(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, y, 1.0);
  return fma(y, fma(e, e, e), y);
}

// grid (ceil(n / RT), ceil(nrhs / RB), nsplit).  Thread: one target node;
// sources of this split staged RT at a time in LDS as (x, y), (n w / pi) and
// (tau_x, tau_y) pairs.
template <int RB>
__global__ __launch_bounds__(RT) void resid_tiles_kernel(const NodeRec* __restrict__ nd, int64_t n,
                                                         const double* __restrict__ tau, int nrhs, int nsplit,
                                                         double* __restrict__ part) {
  __shared__ double2 sp[RT], sn[RT], st[RB][RT];
  const int64_t t = (int64_t)blockIdx.x * RT + threadIdx.x;
  const int r0 = blockIdx.y * RB;
  const int nr = min(RB, nrhs - r0);
  const int z = blockIdx.z;
  const int64_t chunk = (n + nsplit - 1) / nsplit;
  const int64_t s0 = z * chunk, s1 = min(n, s0 + chunk);
  const int64_t ld = 2 * n;
  double xi = 0, yi = 0;
  if (t < n) { xi = nd[t].x; yi = nd[t].y; }
  double ax[RB], ay[RB];
#pragma unroll
  for (int c = 0; c < RB; ++c) { ax[c] = 0; ay[c] = 0; }
  for (int64_t b0 = s0; b0 < s1; b0 += RT) {
    const int64_t sj = b0 + threadIdx.x;
    __syncthreads();
    if (sj < s1) {
      const NodeRec q = nd[sj];
      sp[threadIdx.x] = make_double2(q.x, q.y);
      sn[threadIdx.x] = make_double2(q.nx * q.w * kInvPi, q.ny * q.w * kInvPi);
#pragma unroll
      for (int c = 0; c < RB; ++c)
        st[c][threadIdx.x] = (c < nr) ? make_double2(tau[2 * sj + (int64_t)(r0 + c) * ld],
                                                     tau[2 * sj + 1 + (int64_t)(r0 + c) * ld])
                                      : make_double2(0.0, 0.0);
    } else {
      sp[threadIdx.x] = make_double2(1e300, 1e300);  // far away; zero weight
      sn[threadIdx.x] = make_double2(0.0, 0.0);
#pragma unroll
      for (int c = 0; c < RB; ++c) st[c][threadIdx.x] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int cnt = (int)min<int64_t>(RT, s1 - b0);
#pragma unroll 4
    for (int s = 0; s < cnt; ++s) {
      const double2 p = sp[s], nw = sn[s];
      const double rx = xi - p.x, ry = yi - p.y;
      const double r2 = rx * rx + ry * ry;
      const double inv = r2 > 0.0 ? rcp_nr2(r2) : 0.0;  // r = 0 only on the diagonal
      const double cf = (rx * nw.x + ry * nw.y) * inv * inv;
#pragma unroll
      for (int c = 0; c < RB; ++c) {
        const double2 tv = st[c][s];
        const double d = cf * (rx * tv.x + ry * tv.y);
        ax[c] += d * rx;
        ay[c] += d * ry;
      }
    }
  }
  if (t < n)
    for (int c = 0; c < nr; ++c) {
      double* p = part + ((int64_t)z * nrhs + r0 + c) * ld;
      p[2 * t] = ax[c];
      p[2 * t + 1] = ay[c];
    }
}

// Sum over a workgroup of 256 threads in a fixed order (butterfly within
// each wave, then the four wave sums in order), returned to thread 0.
__device__ __forceinline__ double block_sum256(double v, double* red4) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red4[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red4[0] + red4[1]) + (red4[2] + red4[3]);
}

// Partial sums of s_N[c] = sum_j w_j n_j . tau_j (the rank-one nullspace
// term) over the 256 nodes of block b: fpart[c * nb + b].
__device__ __forceinline__ double flux_term(const NodeRec& q, const double* tc, int64_t j) {
  return q.w * (q.nx * tc[2 * j] + q.ny * tc[2 * j + 1]);
}
__global__ __launch_bounds__(256) void flux_part_kernel(const NodeRec* __restrict__ nd, int64_t n,
                                                        const double* __restrict__ tau,
                                                        double* __restrict__ fpart) {
  __shared__ double red4[4];
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  const double v = j < n ? flux_term(nd[j], tau + (int64_t)c * 2 * n, j) : 0.0;
  const double t = block_sum256(v, red4);
  if (threadIdx.x == 0) fpart[(int64_t)c * gridDim.x + blockIdx.x] = t;
}

// One right-hand side: the sources packed as (x, y, n_x w / pi, n_y w / pi,
// tau_x, tau_y, 0, 0), so that a source index that is the same in every lane
// turns into scalar loads of one 64-byte record per source: the kernel's
// inner loop then reads no LDS and runs at the FP64 instruction rate.
constexpr int RPK = 8;   // doubles per packed source
// Also writes the flux partial of its block (fpart[blockIdx.x]).
__global__ __launch_bounds__(256) void resid_pack_kernel(const NodeRec* __restrict__ nd, int64_t n,
                                                         const double* __restrict__ tau, double* __restrict__ pk,
                                                         double* __restrict__ fpart) {
  __shared__ double red4[4];
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double fl = 0.0;
  if (j < n) {
    const NodeRec q = nd[j];
    double* o = pk + j * RPK;
    o[0] = q.x;
    o[1] = q.y;
    o[2] = q.nx * q.w * kInvPi;
    o[3] = q.ny * q.w * kInvPi;
    o[4] = tau[2 * j];
    o[5] = tau[2 * j + 1];
    o[6] = 0.0;
    o[7] = 0.0;
    fl = flux_term(q, tau, j);
  }
  const double t = block_sum256(fl, red4);
  if (threadIdx.x == 0) fpart[blockIdx.x] = t;
}

// grid (ceil(n / (256 RT1)), 1, nsplit): thread = RT1 targets (256 apart),
// sources of the split in order (the same index in every lane, so each
// source record is one scalar load shared by the RT1 targets).
__global__ __launch_bounds__(256) void resid_scalar_kernel(const NodeRec* __restrict__ nd, int64_t n,
                                                           const double* __restrict__ pk, int nsplit,
                                                           double* __restrict__ part) {
  const int64_t t0 = (int64_t)blockIdx.x * 256 * RT1 + threadIdx.x;
  const int z = blockIdx.z;
  const int64_t chunk = (n + nsplit - 1) / nsplit;
  const int64_t s0 = z * chunk, s1 = min(n, s0 + chunk);
  double xi[RT1], yi[RT1], ax[RT1], ay[RT1];
#pragma unroll
  for (int u = 0; u < RT1; ++u) {
    const int64_t t = t0 + 256 * u;
    xi[u] = t < n ? nd[t].x : 0.0;
    yi[u] = t < n ? nd[t].y : 0.0;
    ax[u] = ay[u] = 0.0;
  }
  // r = 0 only on the diagonal: |r|^2 carries kR2Floor, which keeps 1 / r^4
  // finite there (the zero r . n makes the term vanish) and moves no other
  // |r|^2 above 1e-35 by a relative 1e-25
  constexpr double kR2Floor = 1e-60;
  auto r2f = [](double rx, double ry) { return fma(rx, rx, fma(ry, ry, kR2Floor)); };
  auto term = [&](int u, const double* q, double rx, double ry, double inv) {
    const double cf = (rx * q[2] + ry * q[3]) * inv * inv;
    const double d = cf * (rx * q[4] + ry * q[5]);
    ax[u] += d * rx;
    ay[u] += d * ry;
  };
  int64_t sj = s0;
  // four sources per reciprocal: 1 / (a b c d) and products give the four
  // 1 / r^2 (r^2 within [1e-60, 1e60], so the product stays in range)
  for (; sj + 4 <= s1; sj += 4) {
    const double* q0 = pk + sj * RPK;
    const double* q1 = q0 + RPK;
    const double* q2 = q1 + RPK;
    const double* q3 = q2 + RPK;
#pragma unroll
    for (int u = 0; u < RT1; ++u) {
      const double x0 = xi[u] - q0[0], y0 = yi[u] - q0[1], x1 = xi[u] - q1[0], y1 = yi[u] - q1[1];
      const double x2 = xi[u] - q2[0], y2 = yi[u] - q2[1], x3 = xi[u] - q3[0], y3 = yi[u] - q3[1];
      const double a = r2f(x0, y0), b = r2f(x1, y1), c = r2f(x2, y2), d = r2f(x3, y3);
      const double ab = a * b, cd = c * d;
      const double y = rcp_nr3(ab * cd);
      const double yab = y * cd, ycd = y * ab;
      term(u, q0, x0, y0, b * yab);
      term(u, q1, x1, y1, a * yab);
      term(u, q2, x2, y2, d * ycd);
      term(u, q3, x3, y3, c * ycd);
    }
  }
  for (; sj < s1; ++sj) {
    const double* q = pk + sj * RPK;
#pragma unroll
    for (int u = 0; u < RT1; ++u) {
      const double rx = xi[u] - q[0], ry = yi[u] - q[1];
      term(u, q, rx, ry, rcp_nr3(r2f(rx, ry)));
    }
  }
  double* p = part + (int64_t)z * 2 * n;
#pragma unroll
  for (int u = 0; u < RT1; ++u) {
    const int64_t t = t0 + 256 * u;
    if (t < n) {
      p[2 * t] = ax[u];
      p[2 * t + 1] = ay[u];
    }
  }
}

// grid (nb = ceil(n / 256), nrhs), 1024 threads: four quarters of 256
// threads, one target node per thread; quarter h sums the split partials
// z = h, h + 4, ... of the block's 256 targets (eight loads in flight), and
// quarter 0 adds the four sums in a fixed order and finishes.  s_N[c] is the
// sum of the nb flux partials, taken in the same order by every wave of
// quarter 0; with npart, block b also writes the partial sums of |r|^2 and
// |g|^2 over its nodes to npart[2 (c nb + b)] and npart[2 (c nb + b) + 1].
constexpr int RFQ = 4;   // quarters (threads per target)
__global__ __launch_bounds__(256 * RFQ) void resid_finalize_kernel(const NodeRec* __restrict__ nd, int64_t n,
                                                                   const double* __restrict__ g,
                                                                   const double* __restrict__ tau, int nrhs,
                                                                   int nsplit, const double* __restrict__ part,
                                                                   const double* __restrict__ fpart,
                                                                   double* __restrict__ r,
                                                                   double* __restrict__ npart) {
  __shared__ double2 qs[RFQ - 1][256];
  __shared__ double red4[2][4];
  const int tq = threadIdx.x & 255;
  const int h = __builtin_amdgcn_readfirstlane(threadIdx.x >> 8);
  const int64_t i = (int64_t)blockIdx.x * 256 + tq;
  const int c = blockIdx.y, nb = gridDim.x;
  const int64_t ld = 2 * n;
  // this quarter's splits: eight independent sums (z / RFQ mod 8), added
  // pairwise in a fixed order
  double sx = 0.0, sy = 0.0;
  if (i < n) {
    constexpr int U = 8;
    double px[U] = {}, py[U] = {};
    const double2* p2 = reinterpret_cast<const double2*>(part + (int64_t)c * ld) + i;
    const int64_t zst = (int64_t)nrhs * n;   // split stride in double2
    int z = h;
    for (; z + RFQ * (U - 1) < nsplit; z += RFQ * U) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double2 v = p2[(int64_t)(z + RFQ * u) * zst];
        px[u] += v.x;
        py[u] += v.y;
      }
    }
    for (int u = 0; z < nsplit; z += RFQ, ++u) {
      const double2 v = p2[(int64_t)z * zst];
      px[u] += v.x;
      py[u] += v.y;
    }
#pragma unroll
    for (int w = U / 2; w > 0; w >>= 1)
#pragma unroll
      for (int u = 0; u < w; ++u) {
        px[u] += px[u + w];
        py[u] += py[u + w];
      }
    sx = px[0];
    sy = py[0];
  }
  if (h > 0) qs[h - 1][tq] = make_double2(sx, sy);
  __syncthreads();
  double r2 = 0.0, g2 = 0.0;
  if (h == 0) {
    // s_N: lane l sums the partials b = l (mod 64) in order, then a
    // butterfly over the wave; every wave of quarter 0 takes the same steps,
    // so all hold the same value
    double sN = 0.0;
    for (int b = threadIdx.x & 63; b < nb; b += 64) sN += fpart[(int64_t)c * nb + b];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sN += __shfl_xor(sN, o);
    if (i < n) {
      const NodeRec q = nd[i];
      const double tx = tau[2 * i + (int64_t)c * ld], ty = tau[2 * i + 1 + (int64_t)c * ld];
      // self block without its nullspace part (added through s_N below)
      const double a00 = q.s00 - q.w * q.nx * q.nx, a01 = q.s01 - q.w * q.nx * q.ny, a11 = q.s11 - q.w * q.ny * q.ny;
      double ax = a00 * tx + a01 * ty + q.nx * sN;
      double ay = a01 * tx + a11 * ty + q.ny * sN;
      const double2 q1 = qs[0][tq], q2 = qs[1][tq], q3 = qs[2][tq];
      ax += (sx + q1.x) + (q2.x + q3.x);
      ay += (sy + q1.y) + (q2.y + q3.y);
      const double gx = g[2 * i + (int64_t)c * ld], gy = g[2 * i + 1 + (int64_t)c * ld];
      const double rx = gx - ax, ry = gy - ay;
      r[2 * i + (int64_t)c * ld] = rx;
      r[2 * i + 1 + (int64_t)c * ld] = ry;
      r2 = rx * rx + ry * ry;
      g2 = gx * gx + gy * gy;
    }
  }
  if (npart) {   // uniform
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      r2 += __shfl_xor(r2, o);
      g2 += __shfl_xor(g2, o);
    }
    if (h == 0 && (threadIdx.x & 63) == 0) {
      red4[0][threadIdx.x >> 6] = r2;
      red4[1][threadIdx.x >> 6] = g2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      npart[2 * ((int64_t)c * nb + blockIdx.x)] = (red4[0][0] + red4[0][1]) + (red4[0][2] + red4[0][3]);
      npart[2 * ((int64_t)c * nb + blockIdx.x) + 1] = (red4[1][0] + red4[1][1]) + (red4[1][2] + red4[1][3]);
    }
  }
}

// grid (nrhs), one wave: norms[c] = sum_b npart[2 (c nb + b)] (|r_c|^2),
// norms[nrhs + c] = the same for |g_c|^2.
__global__ __launch_bounds__(64) void resid_norms_kernel(const double* __restrict__ npart, int nb, int nrhs,
                                                         double* __restrict__ norms) {
  const int c = blockIdx.x, lane = threadIdx.x;
  double sr = 0.0, sg = 0.0;
  for (int b = lane; b < nb; b += 64) {
    sr += npart[2 * ((int64_t)c * nb + b)];
    sg += npart[2 * ((int64_t)c * nb + b) + 1];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sr += __shfl_xor(sr, o);
    sg += __shfl_xor(sg, o);
  }
  if (lane == 0) {
    norms[c] = sr;
    norms[nrhs + c] = sg;
  }
}

// ------------------------------------------- residual, far clusters by expansion
// The sources are cut into clusters of RC_CS consecutive nodes (arcs of the
// curve, since a discretization stores its panels in curve order).  A group
// of RC_TG consecutive targets (one wave), inside a circle of radius R_t
// about c_t, takes a cluster (radius R_s about c_s) whose centre is at least
// RC_RATIO R_s + R_t from c_t through the cluster's multipole expansion,
// every other cluster pair by pair (as resid_scalar_kernel).  The expansion comes from the
// complex form of the double layer D of Sec. 2 (source zeta with normal nu,
// weight w, density mu; target z):
//   D mu = (w / 4 pi) [ nu mu / r + 2 Re(conj(nu) mu) / conj(r)
//                       + r conj(nu mu) / conj(r)^2 ],   r = z - zeta,
// with Z = z - c_s, t = zeta - c_s, s = t / R_s and W = R_s / Z (|s| <= 1):
//   sum_j D_j mu_j = iz G(W) + conj(iz E(W)) + Z conj(iz^2 F(W)),  iz = 1 / Z,
//   G_p = sum_j a_j s_j^p,   F_p = (p + 1) G_p,
//   E_q = sum_j b_j s_j^q - q a_j conj(s_j) s_j^(q - 1),
//   a_j = w_j nu_j mu_j / (4 pi),   b_j = w_j Re(conj(nu_j) mu_j) / (2 pi),
// the geometric series of 1 / (Z - t) and 1 / (Z - t)^2 in t / Z.  The far
// test keeps |W| <= 1 / RC_RATIO = 1/3 at every target of the group; each
// far cluster keeps the powers up to the smallest P (at most RC_P = 40) for
// which the dropped terms stay below 1e-17 of the cluster's sum_j |a_j| /
// |Z| (the squared series, with its factor p + 1, included).
constexpr int RC_CS = 256;       // nodes per source cluster (one packing workgroup)
constexpr int RC_P = 40;         // highest power kept
constexpr int RC_NP = RC_P + 1;
constexpr double RC_RATIO = 3.0;
constexpr int RC_REC = 256;      // doubles per cluster record: c_x, c_y, R, 0, then (G_p, F_p, E_p), p = 0..RC_P
constexpr int RC_PG = (RC_NP + 3) / 4;   // groups of four powers in the coefficient sums
constexpr int64_t RC_MIN_N = 4096;   // RW_RESID_AUTO: expansions from this many nodes
static_assert(4 + 6 * RC_NP <= RC_REC, "cluster record too small");

__device__ __forceinline__ double2 cmul2(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Wave-wide min / max / sum by butterfly (every lane holds the result).
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
// A double that is the same in every lane, moved to scalar registers (so that
// branches on it and addresses from it are scalar).
__device__ __forceinline__ double uniform_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

constexpr int RC_CZ = 4;                             // power slices per cluster
constexpr int RC_PGZ = (RC_PG + RC_CZ - 1) / RC_CZ;  // groups of four powers per slice
constexpr int RC_SGZ = 256 / RC_PGZ;                 // source groups per slice
constexpr int RC_NPZ = 4 * RC_PGZ;                   // powers per slice
constexpr int RC_GEO = 8;    // doubles per compact cluster record: c_x, c_y, R, x0, x1, y0, y1, 0
constexpr int RC_L2 = 8;     // first-level clusters per second-level cluster
constexpr int RC_CC = 8;     // right-hand sides per workgroup of the coefficient kernels
constexpr int64_t RC_L2_MIN_N = 32768;   // second-level clusters from this many nodes

// Shared memory of the coefficient sums of one cluster slice.
struct ClusterSums {
  double2 sa[RC_CS], sas[RC_CS], ss[RC_CS];   // a_j, a_j conj(s_j), s_j
  double sb[RC_CS];                           // b_j
  double2 gpart[RC_SGZ][RC_NPZ], epart[RC_SGZ][RC_NPZ];
  double2 gred[RC_NPZ][16], ered[RC_NPZ][16];
};

// Stage source tid's a_j, b_j and s_j (t_j = zeta_j - c, s_j = t_j / R)
// from its packed record q (x, y, n_x w / pi, n_y w / pi, tau_x, tau_y):
// a_j = w nu mu / (4 pi), b_j = w Re(conj(nu) mu) / (2 pi); q = nullptr
// stages a zero source.
__device__ __forceinline__ void cluster_stage(ClusterSums& S, const double* q, double cx, double cy, double R) {
  const int tid = threadIdx.x;
  double2 a = make_double2(0.0, 0.0), sv = make_double2(0.0, 0.0);
  double bj = 0.0;
  if (q) {
    a = make_double2(0.25 * (q[2] * q[4] - q[3] * q[5]), 0.25 * (q[2] * q[5] + q[3] * q[4]));
    bj = 0.5 * (q[2] * q[4] + q[3] * q[5]);
    sv = make_double2((q[0] - cx) / R, (q[1] - cy) / R);
  }
  S.sa[tid] = a;
  S.ss[tid] = sv;
  S.sas[tid] = cmul2(a, make_double2(sv.x, -sv.y));
  S.sb[tid] = bj;
}

// The sums G_p and E_p over the RC_CS staged sources for the powers of slice
// z (p = 4 z RC_PGZ + tid for tid < RC_NPZ, valid while p <= RC_P), in a
// fixed order.  Thread (pgl, g): powers p = 4 pg .. 4 pg + 3 (pg = z RC_PGZ +
// pgl) of the sources g, g + RC_SGZ, ... (one binary powering per source,
// then three products); then 16 partial sums per power and their sum.  Call
// after the staging is visible to the block; every thread must call it.
__device__ void cluster_power_sums(ClusterSums& S, int z, double2& Gout, double2& Eout) {
  const int tid = threadIdx.x;
  const int pg0 = z * RC_PGZ;
  if (tid < RC_PGZ * RC_SGZ) {
    const int pgl = tid / RC_SGZ, g = tid % RC_SGZ, p0 = 4 * (pg0 + pgl);
    double2 G[4], E[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) G[u] = E[u] = make_double2(0.0, 0.0);
    if (p0 <= RC_P) {
      for (int k = g; k < RC_CS; k += RC_SGZ) {
        const double2 sv = S.ss[k], a = S.sa[k], as = S.sas[k];
        const double bj = S.sb[k];
        // prev = s^(p0 - 1) (1 for p0 = 0, where it is multiplied by p = 0)
        double2 prev = make_double2(1.0, 0.0), base = sv;
        for (int m = p0 > 0 ? p0 - 1 : 0; m; m >>= 1) {
          if (m & 1) prev = cmul2(prev, base);
          base = cmul2(base, base);
        }
        double2 cur = p0 > 0 ? cmul2(prev, sv) : make_double2(1.0, 0.0);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double pp = (double)(p0 + u);
          G[u].x = fma(a.x, cur.x, fma(-a.y, cur.y, G[u].x));
          G[u].y = fma(a.x, cur.y, fma(a.y, cur.x, G[u].y));
          const double2 t = cmul2(as, prev);
          E[u].x = fma(bj, cur.x, fma(-pp, t.x, E[u].x));
          E[u].y = fma(bj, cur.y, fma(-pp, t.y, E[u].y));
          prev = cur;
          cur = cmul2(cur, sv);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      S.gpart[g][4 * pgl + u] = G[u];
      S.epart[g][4 * pgl + u] = E[u];
    }
  }
  __syncthreads();
  if (tid < RC_NPZ * 16) {
    const int pl = tid / 16, h = tid % 16;
    double2 G = make_double2(0.0, 0.0), E = make_double2(0.0, 0.0);
    for (int g = h; g < RC_SGZ; g += 16) {
      G.x += S.gpart[g][pl].x;
      G.y += S.gpart[g][pl].y;
      E.x += S.epart[g][pl].x;
      E.y += S.epart[g][pl].y;
    }
    S.gred[pl][h] = G;
    S.ered[pl][h] = E;
  }
  __syncthreads();
  Gout = Eout = make_double2(0.0, 0.0);
  if (tid < RC_NPZ) {
    double2 G = S.gred[tid][0], E = S.ered[tid][0];
    for (int h = 1; h < 16; ++h) {
      G.x += S.gred[tid][h].x;
      G.y += S.gred[tid][h].y;
      E.x += S.ered[tid][h].x;
      E.y += S.ered[tid][h].y;
    }
    Gout = G;
    Eout = E;
  }
}

// grid (ceil(n / RC_CS), ceil(nrhs / RC_CC), RC_CZ), 256 threads.  Block
// (b, y, z): the coefficients of cluster b for the powers of slice z, for
// columns c = y RC_CC .. y RC_CC + RC_CC - 1 in turn (the cluster's geometry
// found once); slice 0 also packs the sources (the RPK format of resid_scalar_kernel, at
// pk + (c n + j) RPK), writes the flux partial of its nodes to fpart[c nb + b]
// and the record's centre and radius, also to the compact geo + (c nb + b)
// RC_GEO (c_x, c_y, R and the bounding box) that the evaluation scans.
// Record: rec + (c nb + b) RC_REC.
__global__ __launch_bounds__(256) void resid_clusters_kernel(const NodeRec* __restrict__ nd, int64_t n, int nrhs,
                                                             const double* __restrict__ tau, double* __restrict__ pk,
                                                             double* __restrict__ fpart, double* __restrict__ rec,
                                                             double* __restrict__ geo) {
  __shared__ double red4[4];
  __shared__ double wred[4][4];
  __shared__ ClusterSums S;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int b = blockIdx.x, nb = gridDim.x, z = blockIdx.z;
  const int c0 = blockIdx.y * RC_CC, c1 = min(nrhs, c0 + RC_CC);
  const int64_t j = (int64_t)b * RC_CS + tid;
  const bool ok = j < n;
  NodeRec q{};
  if (ok) q = nd[j];
  // bounding box of the cluster, its centre and radius (the same for every column)
  {
    const double v0 = wave_min(ok ? q.x : INFINITY), v1 = wave_max(ok ? q.x : -INFINITY);
    const double v2 = wave_min(ok ? q.y : INFINITY), v3 = wave_max(ok ? q.y : -INFINITY);
    if (lane == 0) { wred[wv][0] = v0; wred[wv][1] = v1; wred[wv][2] = v2; wred[wv][3] = v3; }
  }
  __syncthreads();
  const double x0 = fmin(fmin(wred[0][0], wred[1][0]), fmin(wred[2][0], wred[3][0]));
  const double x1 = fmax(fmax(wred[0][1], wred[1][1]), fmax(wred[2][1], wred[3][1]));
  const double y0 = fmin(fmin(wred[0][2], wred[1][2]), fmin(wred[2][2], wred[3][2]));
  const double y1 = fmax(fmax(wred[0][3], wred[1][3]), fmax(wred[2][3], wred[3][3]));
  const double cx = 0.5 * (x0 + x1), cy = 0.5 * (y0 + y1);
  const double ex = q.x - cx, ey = q.y - cy;
  const double d2 = wave_max(ok ? ex * ex + ey * ey : 0.0);
  __syncthreads();
  if (lane == 0) wred[wv][0] = d2;
  __syncthreads();
  // R > 0 even for a cluster of one point (its s_j are then 0 and only the
  // p = 0 terms remain)
  const double R = fmax(sqrt(fmax(fmax(wred[0][0], wred[1][0]), fmax(wred[2][0], wred[3][0]))), 1e-300);
  for (int c = c0; c < c1; ++c) {
    const double* tc = tau + (int64_t)c * 2 * n;
    double tx = 0.0, ty = 0.0;
    if (ok) {
      tx = tc[2 * j];
      ty = tc[2 * j + 1];
    }
    const double qr[6] = {q.x, q.y, q.nx * q.w * kInvPi, q.ny * q.w * kInvPi, tx, ty};
    if (z == 0) {   // uniform
      double fl = 0.0;
      if (ok) {
        double* o = pk + ((int64_t)c * n + j) * RPK;
#pragma unroll
        for (int e = 0; e < 6; ++e) o[e] = qr[e];
        o[6] = 0.0;
        o[7] = 0.0;
        fl = flux_term(q, tc, j);
      }
      const double fsum = block_sum256(fl, red4);
      if (tid == 0) fpart[(int64_t)c * nb + b] = fsum;
    }
    __syncthreads();   // the previous column's sums have read the staging
    cluster_stage(S, ok ? qr : nullptr, cx, cy, R);
    __syncthreads();
    double2 G, E;
    cluster_power_sums(S, z, G, E);
    double* r = rec + ((int64_t)c * nb + b) * RC_REC;
    const int p = 4 * z * RC_PGZ + tid;
    if (tid < RC_NPZ && p <= RC_P) {
      double* o = r + 4 + 6 * p;
      o[0] = G.x;
      o[1] = G.y;
      o[2] = (p + 1) * G.x;
      o[3] = (p + 1) * G.y;
      o[4] = E.x;
      o[5] = E.y;
    } else if (tid == 64 && z == 0) {
      r[0] = cx;
      r[1] = cy;
      r[2] = R;
      r[3] = 0.0;
      double* gc = geo + ((int64_t)c * nb + b) * RC_GEO;
      const double gv[RC_GEO] = {cx, cy, R, x0, x1, y0, y1, 0.0};
#pragma unroll
      for (int e = 0; e < RC_GEO; ++e) gc[e] = gv[e];
    }
  }
}

// Second-level cluster b2 (first-level clusters RC_L2 b2 .. RC_L2 b2 +
// RC_L2 - 1): centre at the middle of the union of their bounding boxes, and
// a radius that bounds every node's distance from it (the largest of
// |c_1 - c_2| + R_1 over its clusters; at least the true radius, so the far
// test and the truncation bound hold).
__device__ __forceinline__ void l2_geometry(const double* geo1c, int nb1, int b2, double& cx, double& cy, double& R) {
  double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
  const int e1 = min(nb1, RC_L2 * (b2 + 1));
  for (int b1 = RC_L2 * b2; b1 < e1; ++b1) {
    const double* g = geo1c + (int64_t)b1 * RC_GEO;
    x0 = fmin(x0, g[3]);
    x1 = fmax(x1, g[4]);
    y0 = fmin(y0, g[5]);
    y1 = fmax(y1, g[6]);
  }
  cx = 0.5 * (x0 + x1);
  cy = 0.5 * (y0 + y1);
  R = 1e-300;
  for (int b1 = RC_L2 * b2; b1 < e1; ++b1) {
    const double* g = geo1c + (int64_t)b1 * RC_GEO;
    R = fmax(R, sqrt((g[0] - cx) * (g[0] - cx) + (g[1] - cy) * (g[1] - cy)) + g[2]);
  }
}

// grid (nb2 RC_L2, ceil(nrhs / RC_CC), RC_CZ), 256 threads: block (b2 RC_L2 +
// u, y, z) sums the powers of slice z over first-level cluster RC_L2 b2 + u
// (packed sources of each column c = y RC_CC ..) about second-level cluster
// b2's centre, into
// part2 + ((c nb2 + b2) RC_L2 + u) 4 RC_NP (G_p, E_p; zero for a cluster
// past the end).
__global__ __launch_bounds__(256) void resid_clusters2_kernel(int64_t n, int nrhs, const double* __restrict__ pk,
                                                              const double* __restrict__ geo1, int nb1, int nb2,
                                                              double* __restrict__ part2) {
  __shared__ ClusterSums S;
  const int tid = threadIdx.x;
  const int b2 = blockIdx.x / RC_L2, u = blockIdx.x % RC_L2, z = blockIdx.z;
  const int c0 = blockIdx.y * RC_CC, c1 = min(nrhs, c0 + RC_CC);
  const int b1 = RC_L2 * b2 + u;
  double cx, cy, R;
  l2_geometry(geo1 + (int64_t)c0 * nb1 * RC_GEO, nb1, b2, cx, cy, R);
  const int64_t j = (int64_t)b1 * RC_CS + tid;
  for (int c = c0; c < c1; ++c) {
    __syncthreads();   // the previous column's sums have read the staging
    cluster_stage(S, (b1 < nb1 && j < n) ? pk + ((int64_t)c * n + j) * RPK : nullptr, cx, cy, R);
    __syncthreads();
    double2 G, E;
    cluster_power_sums(S, z, G, E);
    const int p = 4 * z * RC_PGZ + tid;
    if (tid < RC_NPZ && p <= RC_P) {
      double* o = part2 + (((int64_t)c * nb2 + b2) * RC_L2 + u) * 4 * RC_NP + 4 * p;
      o[0] = G.x;
      o[1] = G.y;
      o[2] = E.x;
      o[3] = E.y;
    }
  }
}

// grid (nb2, nrhs), 64 threads: second-level records from the RC_L2 partial
// sums (fixed order), rec2 + (c nb2 + b2) RC_REC and geo2 + (c nb2 + b2) RC_GEO.
__global__ __launch_bounds__(64) void resid_clusters2_sum_kernel(const double* __restrict__ geo1, int nb1, int nb2,
                                                                 const double* __restrict__ part2,
                                                                 double* __restrict__ rec2, double* __restrict__ geo2) {
  const int b2 = blockIdx.x, c = blockIdx.y, lane = threadIdx.x;
  double* r = rec2 + ((int64_t)c * nb2 + b2) * RC_REC;
  const double* pp = part2 + ((int64_t)c * nb2 + b2) * RC_L2 * 4 * RC_NP;
  if (lane <= RC_P) {
    const int p = lane;
    double g0 = 0.0, g1 = 0.0, e0 = 0.0, e1 = 0.0;
    for (int u = 0; u < RC_L2; ++u) {
      const double* o = pp + (int64_t)u * 4 * RC_NP + 4 * p;
      g0 += o[0];
      g1 += o[1];
      e0 += o[2];
      e1 += o[3];
    }
    double* o = r + 4 + 6 * p;
    o[0] = g0;
    o[1] = g1;
    o[2] = (p + 1) * g0;
    o[3] = (p + 1) * g1;
    o[4] = e0;
    o[5] = e1;
  }
  if (lane == 63) {
    double cx, cy, R;
    l2_geometry(geo1 + (int64_t)c * nb1 * RC_GEO, nb1, b2, cx, cy, R);
    r[0] = cx;
    r[1] = cy;
    r[2] = R;
    r[3] = 0.0;
    double* gc = geo2 + ((int64_t)c * nb2 + b2) * RC_GEO;
    const double gv[RC_GEO] = {cx, cy, R, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < RC_GEO; ++e) gc[e] = gv[e];
  }
}

// grid (ceil(n / (4 RC_TG)), nrhs, nnear + nfar), 256 threads: wave w of
// block x takes the target group 4 x + w, RC_TG = 128 consecutive nodes, two
// per lane (64 apart), so that every source record or coefficient the wave
// loads serves two targets.  Half a cluster summed pair by pair (a "near"
// unit) costs about as much as eight clusters taken by expansion ("far"
// units), so the work of a group is cut into items of similar cost: item
// z < nnear takes the near units of rank z, z + nnear, ... among the group's
// near ones, item nnear + z' the far units of rank z', z' + nfar, ... (with
// nnear = 0 the single item takes every unit).  The near / far test runs for
// 64 clusters at once (one per lane) and its ballot is walked bit by bit.
// Each item writes the double-layer sum of its units (the pair i = j
// contributes 0) to part[((z nrhs + c) n + i) 2 + {0, 1}], as
// resid_scalar_kernel does.
constexpr int RC_TG = 128;   // targets per group (a wave)
template <bool TWO>   // second-level clusters (ncl2 > 0)
__global__ __launch_bounds__(256) void resid_far_eval_kernel(const NodeRec* __restrict__ nd, int64_t n,
                                                             const double* __restrict__ pk,
                                                             const double* __restrict__ rec,
                                                             const double* __restrict__ geo, int ncl,
                                                             const double* __restrict__ rec2,
                                                             const double* __restrict__ geo2, int ncl2, int nnear,
                                                             int nfar, double* __restrict__ part) {
  const int c = blockIdx.y, nrhs = gridDim.y, z = blockIdx.z;
  const int lane = threadIdx.x & 63;
  const int64_t g0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * RC_TG;
  if (g0 >= n) return;   // the whole wave
  double xi[2], yi[2], ax[2] = {0.0, 0.0}, ay[2] = {0.0, 0.0};
  bool ok[2];
  double bx0 = INFINITY, bx1 = -INFINITY, by0 = INFINITY, by1 = -INFINITY;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int64_t i = g0 + lane + 64 * u;
    ok[u] = i < n;
    xi[u] = ok[u] ? nd[i].x : 0.0;
    yi[u] = ok[u] ? nd[i].y : 0.0;
    if (ok[u]) {
      bx0 = fmin(bx0, xi[u]);
      bx1 = fmax(bx1, xi[u]);
      by0 = fmin(by0, yi[u]);
      by1 = fmax(by1, yi[u]);
    }
  }
  // the group's circle (centre of its bounding box)
  const double tcx = uniform_d(0.5 * (wave_min(bx0) + wave_max(bx1)));
  const double tcy = uniform_d(0.5 * (wave_min(by0) + wave_max(by1)));
  double e2 = 0.0;
#pragma unroll
  for (int u = 0; u < 2; ++u)
    if (ok[u]) e2 = fmax(e2, (xi[u] - tcx) * (xi[u] - tcx) + (yi[u] - tcy) * (yi[u] - tcy));
  const double rt = uniform_d(sqrt(wave_max(e2)));
  constexpr double kR2Floor = 1e-60;   // as resid_scalar_kernel: keeps the pair i = j finite (and zero)
  auto r2f = [](double rx, double ry) { return fma(rx, rx, fma(ry, ry, kR2Floor)); };
  auto term = [&](int u, const double* q, double rx, double ry, double inv) {
    const double cf = (rx * q[2] + ry * q[3]) * inv * inv;
    const double d = cf * (rx * q[4] + ry * q[5]);
    ax[u] += d * rx;
    ay[u] += d * ry;
  };
  const double* pkc = pk + (int64_t)c * n * RPK;
  // this wave's slice of the near-source staging: positions, n w / pi, tau
  __shared__ double2 stage[4][3][128];
  double2(*sp)[128] = stage[threadIdx.x >> 6];
  // kind of work this item takes (0 near, 1 far, 2 both), its slot among
  // the items of that kind and their count
  const int kind = nnear == 0 ? 2 : (z < nnear ? 0 : 1);
  const int slot = kind == 0 ? z : (nnear == 0 ? z : z - nnear);
  const int nslot = kind == 0 ? nnear : nfar;
  int rank = 0;   // units of this item's kind met so far (a near cluster is two units of RC_CS / 2 sources)
  int next = kind == 2 ? 0 : slot;   // rank of the next unit this item takes
  const int step_r = kind == 2 ? 1 : nslot;
  auto take = [&]() __attribute__((always_inline)) {
    const bool t = rank == next;
    if (t) next += step_r;
    ++rank;
    return t;
  };
  // ---- a cluster (record cr, centre (cx, cy), radius R) by its expansion
  auto eval_far = [&](const double* cr, double cx, double cy, double R) __attribute__((always_inline)) {
    // rho = R / (|c_t - c_s| - R_t) >= |W| at every target of the group;
    // the terms after p = P sum to at most (P + 2) rho^(P + 1) / (1 - rho)^2
    // of the cluster's scale, and P is the smallest that keeps this below
    // 1e-17 (P + 2 <= 42 in the bound; one term more for the float logs)
    const double dx = tcx - cx, dy = tcy - cy;
    const double rho = R / (sqrt(dx * dx + dy * dy) - rt);
    const float l2r = __log2f((float)rho), l2q = __log2f((float)(1.0 - rho));
    const float pf = (-56.5f + 2.0f * l2q - 5.4f) / l2r;   // log2(1e-17) = -56.47
    const int pe = pf >= (float)RC_P ? RC_P : (pf > 0.0f ? (int)pf + 1 : 1);
    const int P = __builtin_amdgcn_readfirstlane(pe < RC_P ? pe : RC_P);
    double2 Zt[2], iz[2], W[2], G[2], F[2], E[2];
    const double* co = cr + 4 + 6 * P;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      Zt[u] = make_double2(xi[u] - cx, yi[u] - cy);
      const double in2 = 1.0 / fma(Zt[u].x, Zt[u].x, Zt[u].y * Zt[u].y);
      iz[u] = make_double2(Zt[u].x * in2, -Zt[u].y * in2);
      W[u] = make_double2(R * iz[u].x, R * iz[u].y);
      G[u] = make_double2(co[0], co[1]);
      F[u] = make_double2(co[2], co[3]);
      E[u] = make_double2(co[4], co[5]);
    }
    auto step = [&](const double* cp) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const double2 w = W[u];
        G[u] = make_double2(fma(G[u].x, w.x, fma(-G[u].y, w.y, cp[0])), fma(G[u].x, w.y, fma(G[u].y, w.x, cp[1])));
        F[u] = make_double2(fma(F[u].x, w.x, fma(-F[u].y, w.y, cp[2])), fma(F[u].x, w.y, fma(F[u].y, w.x, cp[3])));
        E[u] = make_double2(fma(E[u].x, w.x, fma(-E[u].y, w.y, cp[4])), fma(E[u].x, w.y, fma(E[u].y, w.x, cp[5])));
      }
    };
    int p = P - 1;
    for (; p >= 3; p -= 4) {
      const double* cp = cr + 4 + 6 * p;
      step(cp);
      step(cp - 6);
      step(cp - 12);
      step(cp - 18);
    }
    for (; p >= 0; --p) step(cr + 4 + 6 * p);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const double2 u1 = cmul2(iz[u], G[u]);
      const double2 u2 = cmul2(iz[u], E[u]);
      const double2 f2 = cmul2(cmul2(iz[u], iz[u]), F[u]);
      // Z conj(f2)
      const double2 u3 = make_double2(Zt[u].x * f2.x + Zt[u].y * f2.y, Zt[u].y * f2.x - Zt[u].x * f2.y);
      ax[u] += u1.x + u2.x + u3.x;
      ay[u] += u1.y - u2.y + u3.y;
    }
  };
  // ---- halves h0 (and h1) of first-level cluster s1 pair by pair, staged
  // in this wave's LDS slice 128 at a time (coalesced loads), then read
  // with the same address in every lane (broadcast)
  auto eval_near = [&](int s1, int h0, int h1) __attribute__((always_inline)) {
    const int64_t c0 = (int64_t)s1 * RC_CS;
    const int64_t j0 = min(n, c0 + (int64_t)h0 * (RC_CS / 2));
    const int64_t j1 = min(n, c0 + (int64_t)((h1 >= 0 ? h1 : h0) + 1) * (RC_CS / 2));
    for (int64_t b0 = j0; b0 < j1; b0 += 128) {
      const int cnt = (int)min<int64_t>(128, j1 - b0);
      __builtin_amdgcn_wave_barrier();   // the previous chunk's reads are issued
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int t = lane + 64 * h;
        if (t < cnt) {
          const double* q = pkc + (b0 + t) * RPK;
          sp[0][t] = make_double2(q[0], q[1]);
          sp[1][t] = make_double2(q[2], q[3]);
          sp[2][t] = make_double2(q[4], q[5]);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      auto terml = [&](int u, double2 nw, double2 tv, double rx, double ry, double inv) {
        const double cf = (rx * nw.x + ry * nw.y) * inv * inv;
        const double d = cf * (rx * tv.x + ry * tv.y);
        ax[u] += d * rx;
        ay[u] += d * ry;
      };
      int t = 0;
      for (; t + 4 <= cnt; t += 4) {
        const double2 p0 = sp[0][t], p1 = sp[0][t + 1], p2 = sp[0][t + 2], p3 = sp[0][t + 3];
        const double2 n0 = sp[1][t], n1 = sp[1][t + 1], n2 = sp[1][t + 2], n3 = sp[1][t + 3];
        const double2 v0 = sp[2][t], v1 = sp[2][t + 1], v2 = sp[2][t + 2], v3 = sp[2][t + 3];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const double rx0 = xi[u] - p0.x, ry0 = yi[u] - p0.y, rx1 = xi[u] - p1.x, ry1 = yi[u] - p1.y;
          const double rx2 = xi[u] - p2.x, ry2 = yi[u] - p2.y, rx3 = xi[u] - p3.x, ry3 = yi[u] - p3.y;
          const double a = r2f(rx0, ry0), bb = r2f(rx1, ry1), cc = r2f(rx2, ry2), d = r2f(rx3, ry3);
          const double ab = a * bb, cd = cc * d;
          const double y = rcp_nr3(ab * cd);
          const double yab = y * cd, ycd = y * ab;
          terml(u, n0, v0, rx0, ry0, bb * yab);
          terml(u, n1, v1, rx1, ry1, a * yab);
          terml(u, n2, v2, rx2, ry2, d * ycd);
          terml(u, n3, v3, rx3, ry3, cc * ycd);
        }
      }
      for (; t < cnt; ++t) {
        const double2 p0 = sp[0][t], n0 = sp[1][t], v0 = sp[2][t];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const double rx = xi[u] - p0.x, ry = yi[u] - p0.y;
          terml(u, n0, v0, rx, ry, rcp_nr3(r2f(rx, ry)));
        }
      }
    }
  };
  // near / far test of a cluster against the group's circle
  auto is_far = [&](double gx, double gy, double gr) __attribute__((always_inline)) {
    const double dx = tcx - gx, dy = tcy - gy, lim = RC_RATIO * gr + rt;
    return dx * dx + dy * dy >= lim * lim;
  };
  // ---- the clusters, tested 64 at a time (one per lane) and walked bit by
  // bit; with second-level clusters, a far one is one far unit and a near
  // one has its first-level clusters tested and walked the same way.  One
  // place below takes every unit: a far cluster (either level) is one far
  // unit, a near first-level cluster two near units.
  if constexpr (!TWO) {
    // one level: the clusters of this item's kind only, each met once
    for (int base = 0; base < ncl; base += 64) {
      const int sl = base + lane;
      double gx = 0.0, gy = 0.0, gr = 0.0;
      bool far_l = false;
      if (sl < ncl) {
        const double* gc = geo + ((int64_t)c * ncl + sl) * RC_GEO;
        gx = gc[0];
        gy = gc[1];
        gr = gc[2];
        far_l = is_far(gx, gy, gr);
      }
      const uint64_t fm = __ballot(sl < ncl && far_l);
      const uint64_t vm = __ballot(sl < ncl);
      uint64_t m = kind == 0 ? (vm & ~fm) : (kind == 1 ? fm : vm);
      while (m) {
        const int b = __builtin_ctzll(m);
        m &= m - 1;
        const int s1 = base + b;
        const bool far = (fm >> b) & 1;
        // the units of this cluster that are this item's (near halves 0 / 1)
        int h0 = -1, h1 = -1;
        if (take()) h0 = 0;
        if (!far && take()) (h0 < 0 ? h0 : h1) = 1;
        if (h0 < 0) continue;
        if (far)
          eval_far(rec + ((int64_t)c * ncl + s1) * RC_REC, __shfl(gx, b), __shfl(gy, b), __shfl(gr, b));
        else
          eval_near(s1, h0, h1);
      }
    }
  } else {
    const int ntop = TWO ? ncl2 : ncl;
    const double* geot = TWO ? geo2 + (int64_t)c * ncl2 * RC_GEO : geo + (int64_t)c * ncl * RC_GEO;
    for (int base = 0; base < ntop; base += 64) {
      const int sl = base + lane;
      double gx = 0.0, gy = 0.0, gr = 0.0;
      bool far_l = false;
      if (sl < ntop) {
        const double* gc = geot + (int64_t)sl * RC_GEO;
        gx = gc[0];
        gy = gc[1];
        gr = gc[2];
        far_l = is_far(gx, gy, gr);
      }
      const uint64_t fm = __ballot(sl < ntop && far_l);
      uint64_t m = __ballot(sl < ntop);
      if (!TWO && kind == 0) m &= ~fm;   // near items meet no far unit at one level
      if (!TWO && kind == 1) m &= fm;
      uint64_t cm = 0, fm1 = 0;   // first-level clusters of the near second-level cluster cs2 still to walk
      int cs2 = 0;
      double hx = 0.0, hy = 0.0, hr = 0.0;
      for (;;) {
        int s1;
        bool far;
        double cx, cy, R;
        const double* cr;
        if (TWO && cm) {
          const int k = __builtin_ctzll(cm);
          cm &= cm - 1;
          s1 = RC_L2 * cs2 + k;
          far = (fm1 >> k) & 1;
          cx = __shfl(hx, k);
          cy = __shfl(hy, k);
          R = __shfl(hr, k);
          cr = rec + ((int64_t)c * ncl + s1) * RC_REC;
        } else if (m) {
          const int b = __builtin_ctzll(m);
          m &= m - 1;
          const int st = base + b;
          far = (fm >> b) & 1;
          if (TWO && !far) {
            // its first-level clusters, lane k taking cluster RC_L2 st + k
            const int k1 = RC_L2 * st + (lane & (RC_L2 - 1));
            const bool v1 = lane < RC_L2 && k1 < ncl;
            bool f1 = false;
            hx = hy = hr = 0.0;
            if (v1) {
              const double* gc = geo + ((int64_t)c * ncl + k1) * RC_GEO;
              hx = gc[0];
              hy = gc[1];
              hr = gc[2];
              f1 = is_far(hx, hy, hr);
            }
            fm1 = __ballot(v1 && f1);
            cm = __ballot(v1);
            cs2 = st;
            continue;
          }
          s1 = st;
          cx = __shfl(gx, b);
          cy = __shfl(gy, b);
          R = __shfl(gr, b);
          cr = TWO ? rec2 + ((int64_t)c * ncl2 + st) * RC_REC : rec + ((int64_t)c * ncl + st) * RC_REC;
        } else {
          break;
        }
        if (far) {
          if (kind != 0 && take()) eval_far(cr, cx, cy, R);
        } else if (kind != 1) {
          int h0 = -1, h1 = -1;
          if (take()) h0 = 0;
          if (take()) (h0 < 0 ? h0 : h1) = 1;
          if (h0 >= 0) eval_near(s1, h0, h1);
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 2; ++u)
    if (ok[u]) {
      double* p = part + (((int64_t)z * nrhs + c) * n + g0 + lane + 64 * u) * 2;
      p[0] = ax[u];
      p[1] = ay[u];
    }
}

// ---------------------------------------------------------------- RHS
__global__ __launch_bounds__(256) void stokeslet_kernel(const NodeRec* __restrict__ nd, int64_t n,
                                                        const double* __restrict__ zf, int n_src,
                                                        double* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double x = nd[i].x, y = nd[i].y;
  double ux = 0, uy = 0;
  for (int m = 0; m < n_src; ++m) {
    const double rx = x - zf[4 * m], ry = y - zf[4 * m + 1];
    const double fx = zf[4 * m + 2], fy = zf[4 * m + 3];
    const double r2 = rx * rx + ry * ry;
    const double lg = -0.5 * log(r2);
    const double rf = (rx * fx + ry * fy) / r2;
    ux += lg * fx + rf * rx;
    uy += lg * fy + rf * ry;
  }
  const double s = 0.25 * kInvPi;
  g[2 * i] = s * ux;
  g[2 * i + 1] = s * uy;
}

// ---------------------------------------------------------------- assembly
__device__ __forceinline__ void a_block(const NodeRec& t, const NodeRec& q, double B[4]) {
  const double rx = t.x - q.x, ry = t.y - q.y;
  const double r2 = rx * rx + ry * ry;
  const double cf = (rx * q.nx + ry * q.ny) * q.w * kInvPi / (r2 * r2);
  B[0] = cf * rx * rx + q.w * t.nx * q.nx;
  B[1] = cf * rx * ry + q.w * t.nx * q.ny;
  B[2] = cf * ry * rx + q.w * t.ny * q.nx;
  B[3] = cf * ry * ry + q.w * t.ny * q.ny;
}

__global__ __launch_bounds__(256) void assemble_kernel(const NodeRec* __restrict__ tgt, int64_t nt,
                                                       const NodeRec* __restrict__ src, int64_t ns, int same,
                                                       double* __restrict__ A, int64_t ld) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= nt) return;
  double B[4];
  if (same && i == j) {
    const NodeRec q = src[j];
    B[0] = q.s00; B[1] = q.s01; B[2] = q.s01; B[3] = q.s11;
  } else {
    a_block(tgt[i], src[j], B);
  }
  A[2 * i + (2 * j) * ld] = B[0];
  A[2 * i + 1 + (2 * j) * ld] = B[2];
  A[2 * i + (2 * j + 1) * ld] = B[1];
  A[2 * i + 1 + (2 * j + 1) * ld] = B[3];
}

// R rows.  mode 0 (k skeleton rows): row = [0 at kept, -A(t, cut) at cut | A(t, p)]
//          mode 1 (p skeleton rows): row = [A(t, kept) at kept, 0 at cut | 0]
// ref_kind[o] = 0 kept, 1 cut.
__global__ __launch_bounds__(256) void r_rows_kernel(const NodeRec* __restrict__ tnodes,
                                                     const int* __restrict__ skel, const NodeRec* __restrict__ ref,
                                                     const int* __restrict__ ref_kind, int64_t n_o,
                                                     const NodeRec* __restrict__ pn, int64_t n_p, int mode,
                                                     double* __restrict__ R, int64_t ldR) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int a = blockIdx.y;
  if (e >= 2 * (n_o + n_p)) return;
  const int sd = skel[a];
  const NodeRec t = tnodes[sd >> 1];
  const int c = sd & 1;
  double v = 0.0;
  double B[4];
  if (e < 2 * n_o) {
    const int64_t o = e >> 1;
    const int d = (int)(e & 1);
    const int kind = ref_kind[o];
    if (mode == 0 && kind == 1) { a_block(t, ref[o], B); v = -B[c * 2 + d]; }
    if (mode == 1 && kind == 0) { a_block(t, ref[o], B); v = B[c * 2 + d]; }
  } else if (mode == 0) {
    const int64_t q = (e - 2 * n_o) >> 1;
    const int d = (int)(e & 1);
    a_block(t, pn[q], B);
    v = B[c * 2 + d];
  }
  R[(int64_t)a * ldR + e] = v;
}

// ---------------------------------------------------------------- sketch
typedef double double4_t __attribute__((ext_vector_type(4)));

struct SegArgs {
  const NodeRec* src[2];
  int64_t ns[2];
  double sign[2];
  int64_t orow[2];
  int nseg;
};

// 64 random signs of Omega row `row`, columns 64 g .. 64 g + 63 (bit c & 63
// of the result is column c): SplitMix64 finalizer of a counter, so Omega is
// never stored and any kernel can regenerate any entry.
__device__ __forceinline__ uint64_t omega_bits(uint64_t seed, int64_t row, int g) {
  uint64_t z = seed ^ ((uint64_t)row * 0x9E3779B97F4A7C15ull) ^ ((uint64_t)(g + 1) * 0xD1B54A32D192ED03ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// 1 / x for x > 0: hardware reciprocal and one Newton step (the sketch only
// has to represent the block to well below the interpolation tolerance).
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  return y * (2.0 - x * y);
}

// grid (ceil(2 nt / 64), nsplit), 256 threads.  One workgroup: 64 target rows
// (32 nodes) x 16 NC sketch columns over its split of the sources.  Per chunk
// of 8 source nodes (16 unknowns) the threads write the A tile (thread t: the
// 2x2 kernel block of target node t / 8 and source node t % 8) and the
// Omega tile (+-1) to LDS; then wave w multiplies its 16 rows by all NC
// column blocks on the FP64 matrix cores.  LDS is double-buffered, so one
// barrier per chunk suffices.
template <int NC>
__global__ __launch_bounds__(256) void sketch_kernel(const NodeRec* __restrict__ tgt, int64_t nt, SegArgs sa,
                                                     uint64_t seed, int col_off, int nsplit, double* __restrict__ out) {
  constexpr int NCOL = 16 * NC;
  __shared__ double As[2][16][64 + 2];    // [source unknown][target row]
  __shared__ double Bs[2][16][NCOL + 2];  // [source unknown][column]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i16 = lane & 15, k4 = lane >> 4;
  const int64_t tb = blockIdx.x;
  const int z = blockIdx.y;
  // this thread's target node (A tile) and Omega slot (B tile)
  const int tn = tid >> 3, sn = tid & 7;
  const int64_t tgi = tb * 32 + tn;
  const bool tval = tgi < nt;
  const NodeRec tr = tgt[tval ? tgi : 0];
  const int kb = tid >> 4, gcol = tid & 15;
  const int64_t ntot = sa.ns[0] + (sa.nseg > 1 ? sa.ns[1] : 0);
  const int64_t nchunk_all = (ntot + 7) / 8;
  const int64_t per = (nchunk_all + nsplit - 1) / nsplit;
  const int64_t c0 = z * per, c1 = min(nchunk_all, c0 + per);
  const int grp = (col_off >> 6);
  double4_t acc[NC];
#pragma unroll
  for (int cb = 0; cb < NC; ++cb) acc[cb] = (double4_t){0.0, 0.0, 0.0, 0.0};
  auto src_of = [&](int64_t gs, int& sg, int64_t& li) {
    sg = (gs < sa.ns[0]) ? 0 : 1;
    li = sg ? gs - sa.ns[0] : gs;
  };
  for (int64_t ch = c0; ch < c1; ++ch) {
    const int buf = (int)(ch & 1);
    // ---- A tile: 2x2 block of (target node tn, source node sn)
    {
      const int64_t gs = ch * 8 + sn;
      double b00 = 0, b01 = 0, b10 = 0, b11 = 0;
      if (gs < ntot && tval) {
        int sg;
        int64_t li;
        src_of(gs, sg, li);
        const NodeRec q = sa.src[sg][li];
        const double sgn = sa.sign[sg];
        const double rx = tr.x - q.x, ry = tr.y - q.y;
        const double r2 = rx * rx + ry * ry;
        const double cf = sgn * q.w * kInvPi * (rx * q.nx + ry * q.ny) * rcp_nr(r2 * r2);
        const double nw = sgn * q.w;
        b00 = cf * rx * rx + nw * tr.nx * q.nx;
        b01 = cf * rx * ry + nw * tr.nx * q.ny;
        b10 = cf * ry * rx + nw * tr.ny * q.nx;
        b11 = cf * ry * ry + nw * tr.ny * q.ny;
      }
      As[buf][2 * sn][2 * tn] = b00;
      As[buf][2 * sn + 1][2 * tn] = b01;
      As[buf][2 * sn][2 * tn + 1] = b10;
      As[buf][2 * sn + 1][2 * tn + 1] = b11;
    }
    // ---- Omega tile: source unknown kb, columns gcol + 16 cb
    {
      const int64_t gs = ch * 8 + (kb >> 1);
      uint64_t bits = 0;
      bool ok = gs < ntot;
      if (ok) {
        int sg;
        int64_t li;
        src_of(gs, sg, li);
        bits = omega_bits(seed, sa.orow[sg] + 2 * li + (kb & 1), grp);
      }
#pragma unroll
      for (int cb = 0; cb < NC; ++cb) {
        const int bit = ((col_off & 63) + cb * 16 + gcol) & 63;
        Bs[buf][kb][cb * 16 + gcol] = ok ? (((bits >> bit) & 1ull) ? -1.0 : 1.0) : 0.0;
      }
    }
    __syncthreads();
    // ---- wave: rows 16 wave .. + 15, all column blocks, K = 16
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const double a = As[buf][ks * 4 + k4][wave * 16 + i16];
#pragma unroll
      for (int cb = 0; cb < NC; ++cb) {
        const double bb = Bs[buf][ks * 4 + k4][cb * 16 + i16];
        acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc[cb], 0, 0, 0);
      }
    }
  }
  // ---- this split's partial sums (rows x NCOL, row-major)
  const int64_t rows_tot = 2 * nt;
  double* o = out + (int64_t)z * rows_tot * NCOL;
#pragma unroll
  for (int cb = 0; cb < NC; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      // v_mfma_f64_16x16x4f64: item r of lane l holds D[l / 16 + 4 r][l % 16]
      const int64_t grow = tb * 64 + wave * 16 + k4 + 4 * r;
      if (grow < rows_tot) o[grow * NCOL + cb * 16 + i16] = acc[cb][r];
    }
}

// Y(:, col_off .. col_off + w) = sum over splits of part[z] (rows x w, row-major)
__global__ __launch_bounds__(256) void sum_parts_kernel(const double* __restrict__ part, int nsplit, int64_t rows,
                                                        int w, double* __restrict__ Y, int ldY, int col_off) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t len = rows * w;
  if (i >= len) return;
  // four independent sums (z mod 4), so that four loads are in flight at a
  // time, combined in a fixed order
  double sv[4] = {0.0, 0.0, 0.0, 0.0};
  int z = 0;
  for (; z + 4 <= nsplit; z += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) sv[u] += part[(int64_t)(z + u) * len + i];
  }
  for (int u = 0; z < nsplit; ++z, ++u) sv[u] += part[(int64_t)z * len + i];
  const double s = (sv[0] + sv[1]) + (sv[2] + sv[3]);
  const int64_t r = i / w;
  const int c = (int)(i - r * w);
  Y[r * ldY + col_off + c] = s;
}

int sketch_splits(int64_t nt, int64_t nsrc) {
  if (nt <= 0) return 1;   // no targets (a near set can be empty): no splits to size
  const int64_t rb = (2 * nt + 63) / 64;
  int64_t s = (2048 + rb - 1) / rb;
  const int64_t pairs = (nsrc + 1) / 2;
  const int64_t maxs = pairs / 16 > 0 ? pairs / 16 : 1;
  if (s > maxs) s = maxs;
  if (s > 64) s = 64;
  return (int)(s < 1 ? 1 : s);
}

// ---------------------------------------------------------------- orderings
// grid (ceil(max(n_new, n_ref) / 256), nrhs): thread i moves refined node i
// to its extended position, and zeroes reference node i if the refinement
// cut it (ref_kind 1).  The two sets are disjoint and together cover the
// extended vector, so no separate clearing runs.
__global__ __launch_bounds__(256) void to_ext_kernel(const double* __restrict__ g, int64_t ld_g, int64_t n_new,
                                                     const int* __restrict__ new2ext,
                                                     const int* __restrict__ ref_kind, int64_t n_ref,
                                                     double* __restrict__ ext, int64_t ld_ext) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (i < n_new) {
    const int64_t e = new2ext[i];
    ext[2 * e + c * ld_ext] = g[2 * i + c * ld_g];
    ext[2 * e + 1 + c * ld_ext] = g[2 * i + 1 + c * ld_g];
  }
  if (i < n_ref && ref_kind[i] == 1) {
    ext[2 * i + c * ld_ext] = 0.0;
    ext[2 * i + 1 + c * ld_ext] = 0.0;
  }
}

__global__ __launch_bounds__(256) void from_ext_kernel(const double* __restrict__ ext, int64_t ld_ext,
                                                       int64_t n_new, const int* __restrict__ new2ext,
                                                       double* __restrict__ out, int64_t ld_out, int acc) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n_new) return;
  const int64_t e = new2ext[i];
  const double vx = ext[2 * e + c * ld_ext], vy = ext[2 * e + 1 + c * ld_ext];
  if (acc) {
    out[2 * i + c * ld_out] += vx;
    out[2 * i + 1 + c * ld_out] += vy;
  } else {
    out[2 * i + c * ld_out] = vx;
    out[2 * i + 1 + c * ld_out] = vy;
  }
}

__global__ __launch_bounds__(256) void gather_nodes_kernel(const NodeRec* __restrict__ src, const int* __restrict__ idx,
                                                           int64_t n, NodeRec* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[idx[i]];
}

inline unsigned blocks(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

// Items per target group of the cluster-expansion residual: about 6000 waves
// in all, at most 32 (a little over half of them near); with one item, near
// and far clusters in the same one.
static void far_items(int64_t n, int nrhs, int* nnear, int* nfar) {
  const int64_t waves = ((n + RC_TG - 1) / RC_TG) * nrhs;
  int64_t it = (6000 + waves - 1) / waves;
  it = it < 1 ? 1 : (it > 32 ? 32 : it);
  if (it == 1) {
    *nnear = 0;
    *nfar = 1;
  } else {
    const int64_t nn = (it * 11 + 19) / 20;   // 55 % near, rounded up, and at least one far item
    *nnear = (int)(nn < it ? nn : it - 1);
    *nfar = (int)it - *nnear;
  }
}
static int far_splits(int64_t n, int nrhs) {
  int a, b;
  far_items(n, nrhs, &a, &b);
  return a + b;
}

bool resid_far_on(int mode, int64_t n) { return mode == RW_RESID_EXPAND || (mode == RW_RESID_AUTO && n >= RC_MIN_N); }

// workspace of one call: split partials (nsplit x nrhs x 2n), flux partials
// (nrhs x nb), norm partials (2 x nrhs x nb), packed sources (RPK x n, one
// right-hand side; RPK x n x nrhs with the cluster expansions) and, with
// those, the cluster records (RC_REC x nb x nrhs); the larger of the two forms
static size_t resid_call_doubles(int64_t n, int nrhs) {
  const int64_t nb = blocks(n);
  const size_t pairs =
      (size_t)resid_splits(n, nrhs) * nrhs * 2 * n + (size_t)(3 * nb * nrhs) + (nrhs == 1 ? (size_t)RPK * n : 0);
  const int64_t nb2 = n >= RC_L2_MIN_N ? (nb + RC_L2 - 1) / RC_L2 : 0;
  const size_t far = (size_t)far_splits(n, nrhs) * nrhs * 2 * n + (size_t)(3 * nb * nrhs) +
                     (size_t)RPK * n * nrhs + (size_t)(RC_REC + RC_GEO) * nb * nrhs +
                     (size_t)(RC_REC + RC_GEO + RC_L2 * 4 * RC_NP) * nb2 * nrhs;
  return pairs > far ? pairs : far;
}

// The split counts shrink as columns are added, so one call's workspace is
// not monotone in nrhs (the one-column kernel takes up to 64 splits, four
// columns 13 at 20224 nodes): the largest over 1..nrhs columns, so that a
// workspace sized for nrhs serves every smaller count.
size_t resid_part_doubles(int64_t n, int nrhs) {
  if (n <= 0 || nrhs <= 0) return 0;
  size_t m = 0;
  for (int c = 1; c <= nrhs; ++c) {
    const size_t v = resid_call_doubles(n, c);
    if (v > m) m = v;
  }
  return m;
}

void launch_residual(const NodeRec* nodes, int64_t n, const double* g, const double* tau, double* r, int nrhs,
                     double* part, double* norms, hipStream_t s, int mode) {
  if (n <= 0 || nrhs <= 0) return;
  const bool far = resid_far_on(mode, n);
  const int ns = far ? far_splits(n, nrhs) : resid_splits(n, nrhs);
  const int nb = (int)blocks(n);
  double* fpart = part + (size_t)ns * nrhs * 2 * n;
  double* npart = fpart + (size_t)nb * nrhs;
  if (far) {
    double* pk = npart + (size_t)2 * nb * nrhs;
    double* rec = pk + (size_t)RPK * n * nrhs;
    double* geo = rec + (size_t)RC_REC * nb * nrhs;
    const int nb2 = n >= RC_L2_MIN_N ? (nb + RC_L2 - 1) / RC_L2 : 0;
    double* rec2 = geo + (size_t)RC_GEO * nb * nrhs;
    double* geo2 = rec2 + (size_t)RC_REC * nb2 * nrhs;
    double* part2 = geo2 + (size_t)RC_GEO * nb2 * nrhs;
    KernelTimer kt("resid_far_eval_kernel", 0.0, 0.0, s);
    const unsigned ncc = (unsigned)((nrhs + RC_CC - 1) / RC_CC);
    hipLaunchKernelGGL(resid_clusters_kernel, dim3(nb, ncc, RC_CZ), dim3(256), 0, s, nodes, n, nrhs, tau, pk, fpart,
                       rec, geo);
    if (nb2 > 0) {
      hipLaunchKernelGGL(resid_clusters2_kernel, dim3(nb2 * RC_L2, ncc, RC_CZ), dim3(256), 0, s, n, nrhs, pk, geo, nb,
                         nb2, part2);
      hipLaunchKernelGGL(resid_clusters2_sum_kernel, dim3(nb2, nrhs), dim3(64), 0, s, geo, nb, nb2, part2, rec2, geo2);
    }
    int nnear, nfar;
    far_items(n, nrhs, &nnear, &nfar);
    if (nb2 > 0)
      hipLaunchKernelGGL(resid_far_eval_kernel<true>, dim3(blocks(n, 4 * RC_TG), nrhs, ns), dim3(256), 0, s, nodes, n,
                         pk, rec, geo, nb, rec2, geo2, nb2, nnear, nfar, part);
    else
      hipLaunchKernelGGL(resid_far_eval_kernel<false>, dim3(blocks(n, 4 * RC_TG), nrhs, ns), dim3(256), 0, s, nodes, n,
                         pk, rec, geo, nb, rec2, geo2, nb2, nnear, nfar, part);
    KERNEL_CHECK("resid_far_eval");
  } else {
    // algorithmic work: 12 flops per 2x2 block (r, r^2, r.n, 1/r^2 scaling) + 6 per
    // block and right-hand side; the division counts as one flop
    KernelTimer kt("resid_tiles_kernel", (double)n * n * (12.0 + 6.0 * nrhs), 0.0, s);
    if (nrhs == 1) {
      double* pk = npart + (size_t)2 * nb * nrhs;
      hipLaunchKernelGGL(resid_pack_kernel, dim3(nb), dim3(256), 0, s, nodes, n, tau, pk, fpart);
      hipLaunchKernelGGL(resid_scalar_kernel, dim3(blocks(n, 256 * RT1), 1, ns), dim3(256), 0, s, nodes, n, pk, ns,
                         part);
    } else {
      hipLaunchKernelGGL(flux_part_kernel, dim3(nb, nrhs), dim3(256), 0, s, nodes, n, tau, fpart);
      hipLaunchKernelGGL(resid_tiles_kernel<RRB>, dim3(blocks(n, RT), (nrhs + RRB - 1) / RRB, ns), dim3(RT), 0, s,
                         nodes, n, tau, nrhs, ns, part);
    }
    KERNEL_CHECK("resid_tiles");
  }
  hipLaunchKernelGGL(resid_finalize_kernel, dim3(nb, nrhs), dim3(256 * RFQ), 0, s, nodes, n, g, tau, nrhs, ns, part, fpart,
                     r, norms ? npart : (double*)nullptr);
  KERNEL_CHECK("resid_finalize");
  if (norms) {
    hipLaunchKernelGGL(resid_norms_kernel, dim3(nrhs), dim3(64), 0, s, npart, nb, nrhs, norms);
    KERNEL_CHECK("resid_norms");
  }
}

void launch_stokeslet_rhs(const NodeRec* nodes, int64_t n, const double* zf, int n_src, double* g,
                          hipStream_t s) {
  hipLaunchKernelGGL(stokeslet_kernel, dim3(blocks(n)), dim3(256), 0, s, nodes, n, zf, n_src, g);
  KERNEL_CHECK("stokeslet_rhs");
}

void launch_assemble(const NodeRec* tgt, int64_t nt, const NodeRec* src, int64_t ns, bool same, double* A,
                     int64_t ld, hipStream_t s) {
  if (nt <= 0 || ns <= 0) return;
  hipLaunchKernelGGL(assemble_kernel, dim3(blocks(nt), (unsigned)ns), dim3(256), 0, s, tgt, nt, src, ns,
                     same ? 1 : 0, A, ld);
  KERNEL_CHECK("assemble");
}

void launch_r_rows(const NodeRec* tnodes, const int* skel_dof, int nrows, const NodeRec* ref_nodes,
                   const int* ref_kind, int64_t n_o, const NodeRec* pnodes, int64_t n_p, int mode, double* R,
                   int64_t ldR, hipStream_t s) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL(r_rows_kernel, dim3(blocks(2 * (n_o + n_p)), nrows), dim3(256), 0, s, tnodes, skel_dof,
                     ref_nodes, ref_kind, n_o, pnodes, n_p, mode, R, ldR);
  KERNEL_CHECK("r_rows");
}

size_t sketch_part_doubles(int64_t nt, int64_t nsrc) { return (size_t)sketch_splits(nt, nsrc) * 2 * nt * 64; }

void launch_sketch(const NodeRec* tgt, int64_t nt, const SketchSeg* segs, int nseg, int ncols, uint64_t seed,
                   double* Y, double* part, hipStream_t s) {
  if (nt <= 0) return;
  if (ncols != 32 && ncols != 64 && ncols != 96 && ncols != 128)
    RW_THROW(RW_EINVAL, "sketch_cols must be 32, 64, 96 or 128");
  SegArgs sa{};
  sa.nseg = nseg;
  int64_t nsrc = 0;
  for (int i = 0; i < nseg && i < 2; ++i) {
    sa.src[i] = segs[i].src;
    sa.ns[i] = segs[i].ns;
    sa.sign[i] = segs[i].sign;
    sa.orow[i] = segs[i].omega_row0;
    nsrc += segs[i].ns;
  }
  if (nseg < 2) { sa.src[1] = segs[0].src; sa.ns[1] = 0; }
  const int64_t rows = 2 * nt;
  if (nsrc == 0) {
    HIP_CHECK(hipMemsetAsync(Y, 0, sizeof(double) * rows * ncols, s));
    return;
  }
  const int ns = sketch_splits(nt, nsrc);
  dim3 grid((unsigned)((rows + 63) / 64), ns);
  // passes of 64 columns (32 for the remainder): the 64-wide tile keeps the
  // accumulators in registers without spilling
  for (int off = 0; off < ncols;) {
    const int w = (ncols - off >= 64) ? 64 : 32;
    KernelTimer kt("sketch_kernel", 2.0 * rows * 2.0 * nsrc * w, 0.0, s);
    if (w == 64)
      hipLaunchKernelGGL(sketch_kernel<4>, grid, dim3(256), 0, s, tgt, nt, sa, seed, off, ns, part);
    else
      hipLaunchKernelGGL(sketch_kernel<2>, grid, dim3(256), 0, s, tgt, nt, sa, seed, off, ns, part);
    KERNEL_CHECK("sketch");
    hipLaunchKernelGGL(sum_parts_kernel, dim3(blocks(rows * w)), dim3(256), 0, s, part, ns, rows, w, Y, ncols, off);
    KERNEL_CHECK("sketch_sum");
    off += w;
  }
}

void launch_to_ext(const double* g, int64_t ld_g, int64_t n_new, const int* new2ext, const int* ref_kind,
                   int64_t n_ref, double* ext, int64_t ld_ext, int nrhs, hipStream_t s) {
  const int64_t n = n_new > n_ref ? n_new : n_ref;
  if (n <= 0 || nrhs <= 0) return;
  hipLaunchKernelGGL(to_ext_kernel, dim3(blocks(n), nrhs), dim3(256), 0, s, g, ld_g, n_new, new2ext, ref_kind, n_ref,
                     ext, ld_ext);
  KERNEL_CHECK("to_ext");
}

void launch_from_ext(const double* ext, int64_t ld_ext, int64_t n_new, const int* new2ext, double* out,
                     int64_t ld_out, int nrhs, bool accumulate, hipStream_t s) {
  hipLaunchKernelGGL(from_ext_kernel, dim3(blocks(n_new), nrhs), dim3(256), 0, s, ext, ld_ext, n_new, new2ext,
                     out, ld_out, accumulate ? 1 : 0);
  KERNEL_CHECK("from_ext");
}

// grid ceil(n / 256): node t of panel t / q, whose parameter interval is
// (pan[2 (t / q)], pan[2 (t / q) + 1]); the node record of the star curve
// gamma(theta) = (1 + a cos(m theta)) (cos theta, sin theta) at the
// Gauss-Legendre point j = t % q (position, outward normal, weight
// w_GL (dtheta / 2) |gamma'| and the self block, Sec. 2.1).
__global__ __launch_bounds__(256) void discretize_kernel(const double* __restrict__ pan, int64_t n, int q,
                                                         GlRule gl, double a, int m, NodeRec* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  const int64_t p = t / q;
  const int j = (int)(t - p * q);
  const double ta = pan[2 * p], tb = pan[2 * p + 1];
  const double half = 0.5 * (tb - ta), mid = 0.5 * (tb + ta);
  const double th = mid + half * gl.s[j];
  double s, c, smt, cmt;
  sincos(th, &s, &c);
  sincos(m * th, &smt, &cmt);
  const double r = 1.0 + a * cmt;
  const double r1 = -a * m * smt;
  const double r2 = -a * m * m * cmt;
  const double x1 = r1 * c - r * s, y1 = r1 * s + r * c;                                   // gamma'
  const double x2 = r2 * c - 2.0 * r1 * s - r * c, y2 = r2 * s + 2.0 * r1 * c - r * s;    // gamma''
  const double sp = sqrt(x1 * x1 + y1 * y1);
  const double tx = x1 / sp, ty = y1 / sp;
  const double nx = ty, ny = -tx;
  const double kap = (x1 * y2 - y1 * x2) / (sp * sp * sp);
  const double w = gl.w[j] * half * sp;
  const double dl = -kap / (2.0 * M_PI);
  NodeRec o;
  o.x = r * c;
  o.y = r * s;
  o.nx = nx;
  o.ny = ny;
  o.w = w;
  o.s00 = -0.5 + w * (dl * tx * tx + nx * nx);
  o.s01 = w * (dl * tx * ty + nx * ny);
  o.s11 = -0.5 + w * (dl * ty * ty + ny * ny);
  out[t] = o;
}

void launch_discretize(const double* pan, int64_t n_panels, int q, const GlRule& gl, double a, int m, NodeRec* out,
                       hipStream_t s) {
  const int64_t n = n_panels * q;
  if (n <= 0) return;
  if (q < 1 || q > GlRule::kMax) RW_THROW(RW_EINVAL, "panel order outside 1..32");
  hipLaunchKernelGGL(discretize_kernel, dim3(blocks(n)), dim3(256), 0, s, pan, n, q, gl, a, m, out);
  KERNEL_CHECK("discretize");
}

void launch_gather_nodes(const NodeRec* src, const int* idx, int64_t n, NodeRec* dst, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(gather_nodes_kernel, dim3(blocks(n)), dim3(256), 0, s, src, idx, n, dst);
  KERNEL_CHECK("gather_nodes");
}
