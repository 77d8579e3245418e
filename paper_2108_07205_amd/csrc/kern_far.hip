// Far field of the Q sketches (Sec. 3.3, Fig. 3): the refined arc Gamma_r lies
// in a circle of radius rho about c.  Kept nodes farther than FAR_RATIO rho
// from c see the arc's sources (cut and added nodes) through a multipole
// expansion about c, and the added nodes see the kept sources beyond that
// radius through a local expansion about c; only the kept nodes inside it are
// summed directly (by the exact sketch kernel, elsewhere).
//
// Both expansions come from the complex form of the double-layer block of A
// (source tau with normal nu, weight w, density mu = mu1 + i mu2; target z,
// r = z - tau; velocity u = u1 + i u2):
//   D mu = (w / 4 pi) [ nu mu / r + 2 Re(conj(nu) mu) / conj(r)
//                       + r conj(nu) conj(mu) / conj(r)^2 ],
//   N mu = n(z) w Re(conj(nu) mu)            (the rank-one nullspace term),
// with r = rho (zeta - t), zeta = (z - c) / rho, t = (tau - c) / rho and the
// geometric series of 1 / (zeta - t) and 1 / conj(zeta - t)^2 in t / zeta
// (multipole, |zeta| > |t|) or zeta / t (local, |zeta| < |t|).  With
// FAR_RATIO = 2.5 and FAR_P = 40 terms the truncation is below 1e-15 relative.
#include <cmath>

#include "kernels.h"

namespace {

constexpr double kInv4Pi = 0.079577471545947667884;
constexpr int FAR_ROWS = 4 * FAR_P + 1;   // A_p, B_p, C_p, D_p (p < FAR_P), then S
constexpr int FC_CHUNK = 16;              // sources per LDS chunk of the coefficient kernel
constexpr int FE_COLS = 16;               // sketch columns per evaluation workgroup

struct FarSegArgs {
  const NodeRec* src[2];
  int64_t ns[2];
  double sign[2];
  int64_t orow[2];
};

struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cplx cconj(cplx a) { return {a.re, -a.im}; }
__device__ __forceinline__ cplx cinv(cplx a) {
  const double d = 1.0 / (a.re * a.re + a.im * a.im);
  return {a.re * d, -a.im * d};
}

// Same counter-based +-1 generator as the exact sketch (bit j & 63 of the
// word of Omega row `row`, column group j >> 6; set bit = -1).
__device__ __forceinline__ uint64_t far_omega_bits(uint64_t seed, int64_t row, int g) {
  uint64_t z = seed ^ ((uint64_t)row * 0x9E3779B97F4A7C15ull) ^ ((uint64_t)(g + 1) * 0xD1B54A32D192ED03ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// grid (nsplit, ceil(ncols / 64)), 256 threads.  Partial expansion
// coefficients of this split's sources for sketch columns 64 gy .. 64 gy + 63:
// part[z][row * ncols + j] (complex), rows A_p, B_p, C_p, D_p, S.
// Per chunk of 16 sources the source factors (powers of t) go to LDS; thread
// (rg = tid / 64, j = tid % 64) then accumulates rows p = rg, rg + 4, ...
// of all four families and, for rg = 0, S.
template <bool LOCAL>
__global__ __launch_bounds__(256) void far_coef_kernel(FarSegArgs sa, double cx, double cy, double inv_rho,
                                                       uint64_t seed, int ncols, int nsplit, double2* __restrict__ part) {
  __shared__ double2 ea[FC_CHUNK][FAR_P], eb[FC_CHUNK][FAR_P], ec[FC_CHUNK][FAR_P], ed[FC_CHUNK][FAR_P];
  __shared__ double snx[FC_CHUNK], sny[FC_CHUNK], sw[FC_CHUNK];   // unit normal, signed weight
  __shared__ uint64_t om[FC_CHUNK][2];
  const int tid = threadIdx.x, jl = tid & 63, rg = tid >> 6;
  const int gy = blockIdx.y, z = blockIdx.x;
  const int j = 64 * gy + jl;
  const int64_t ntot = sa.ns[0] + sa.ns[1];
  const int64_t per = (ntot + nsplit - 1) / nsplit;
  const int64_t s0 = z * per, s1 = min(ntot, s0 + per);
  constexpr int NR = FAR_P / 4;
  cplx A[NR], B[NR], C[NR], D[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) A[q] = B[q] = C[q] = D[q] = {0.0, 0.0};
  double S = 0.0;
  for (int64_t cb = s0; cb < s1; cb += FC_CHUNK) {
    // ---- source factors: thread (s = tid / 16, q = tid % 16) stores p = q, q + 16, ...
    {
      const int sl = tid >> 4, q = tid & 15;
      const int64_t gs = cb + sl;
      if (gs < s1) {
        const int sg = gs < sa.ns[0] ? 0 : 1;
        const int64_t li = sg ? gs - sa.ns[0] : gs;
        const NodeRec nd = sa.src[sg][li];
        const double wq = sa.sign[sg] * nd.w;
        const cplx nu = {nd.nx, nd.ny};
        const cplx t = {(nd.x - cx) * inv_rho, (nd.y - cy) * inv_rho};
        const cplx wnu = {wq * nu.re, wq * nu.im};
        const cplx wnub = {wq * nu.re, -wq * nu.im};
        // multipole: a = w nu t^p, b = 2 w conj(t)^p, c = (p+1) w conj(nu) conj(t)^p, d = c t
        // local:     a = w nu / t^(p+1), b = 2 w / conj(t)^(p+1), c = (p+1) w conj(nu) / conj(t)^(p+2), d = c t
        const cplx base = LOCAL ? cinv(t) : t;
        cplx pw = LOCAL ? base : cplx{1.0, 0.0};   // t^p or t^-(p+1)
        for (int p = 0; p < FAR_P; ++p) {
          if ((p & 15) == q) {
            const cplx pb = cconj(pw);
            const cplx a = cmul(wnu, pw);
            const cplx b = {2.0 * wq * pb.re, 2.0 * wq * pb.im};
            cplx c = cmul(wnub, pb);
            if (LOCAL) c = cmul(c, cconj(base));     // one more conj(t)^-1
            c.re *= (p + 1);
            c.im *= (p + 1);
            const cplx d = cmul(c, t);
            ea[sl][p] = make_double2(a.re, a.im);
            eb[sl][p] = make_double2(b.re, b.im);
            ec[sl][p] = make_double2(c.re, c.im);
            ed[sl][p] = make_double2(d.re, d.im);
          }
          pw = cmul(pw, base);
        }
        if (q == 0) {
          snx[sl] = nu.re;
          sny[sl] = nu.im;
          sw[sl] = wq;
          const int64_t row = sa.orow[sg] + 2 * li;
          om[sl][0] = far_omega_bits(seed, row, gy);
          om[sl][1] = far_omega_bits(seed, row + 1, gy);
        }
      } else if (q == 0) {
        snx[sl] = sny[sl] = sw[sl] = 0.0;
        om[sl][0] = om[sl][1] = 0;
#pragma unroll 1
        for (int p = 0; p < FAR_P; ++p)
          ea[sl][p] = eb[sl][p] = ec[sl][p] = ed[sl][p] = make_double2(0.0, 0.0);
      }
    }
    __syncthreads();
    // ---- accumulate: mu = mu1 + i mu2 with mu1, mu2 = +-1 from Omega;
    // Re(conj(nu) mu) = nx mu1 + ny mu2 with the unit normal
#pragma unroll 2
    for (int sl = 0; sl < FC_CHUNK; ++sl) {
      const double m1 = ((om[sl][0] >> jl) & 1ull) ? -1.0 : 1.0;
      const double m2 = ((om[sl][1] >> jl) & 1ull) ? -1.0 : 1.0;
      const double re_u = snx[sl] * m1 + sny[sl] * m2;
      if (rg == 0) S += sw[sl] * re_u;
#pragma unroll
      for (int qq = 0; qq < NR; ++qq) {
        const int p = rg + 4 * qq;
        const double2 a = ea[sl][p], b = eb[sl][p], c = ec[sl][p], d = ed[sl][p];
        A[qq].re += a.x * m1 - a.y * m2;   // a (m1 + i m2)
        A[qq].im += a.x * m2 + a.y * m1;
        B[qq].re += b.x * re_u;            // b Re(conj(nu) mu)
        B[qq].im += b.y * re_u;
        C[qq].re += c.x * m1 + c.y * m2;   // c (m1 - i m2)
        C[qq].im += c.y * m1 - c.x * m2;
        D[qq].re += d.x * m1 + d.y * m2;
        D[qq].im += d.y * m1 - d.x * m2;
      }
    }
    __syncthreads();
  }
  if (j < ncols) {
    double2* o = part + (int64_t)z * FAR_ROWS * ncols;
#pragma unroll
    for (int qq = 0; qq < NR; ++qq) {
      const int p = rg + 4 * qq;
      o[(int64_t)(0 * FAR_P + p) * ncols + j] = make_double2(A[qq].re, A[qq].im);
      o[(int64_t)(1 * FAR_P + p) * ncols + j] = make_double2(B[qq].re, B[qq].im);
      o[(int64_t)(2 * FAR_P + p) * ncols + j] = make_double2(C[qq].re, C[qq].im);
      o[(int64_t)(3 * FAR_P + p) * ncols + j] = make_double2(D[qq].re, D[qq].im);
    }
    if (rg == 0) o[(int64_t)(4 * FAR_P) * ncols + j] = make_double2(S, 0.0);
  }
}

__global__ __launch_bounds__(256) void far_coef_sum_kernel(const double2* __restrict__ part, int nsplit, int64_t len,
                                                           double2* __restrict__ coef) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= len) return;
  // four independent sums (z mod 4), so that four loads are in flight at a
  // time, combined in a fixed order
  double re[4] = {0.0, 0.0, 0.0, 0.0}, im[4] = {0.0, 0.0, 0.0, 0.0};
  int z = 0;
  for (; z + 4 <= nsplit; z += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double2 v = part[(int64_t)(z + u) * len + i];
      re[u] += v.x;
      im[u] += v.y;
    }
  }
  for (int u = 0; z < nsplit; ++z, ++u) {
    const double2 v = part[(int64_t)z * len + i];
    re[u] += v.x;
    im[u] += v.y;
  }
  coef[i] = make_double2((re[0] + re[1]) + (re[2] + re[3]), (im[0] + im[1]) + (im[2] + im[3]));
}

// grid (ceil(nt / 256), ncols / 16), 256 threads: thread = target node,
// 16 sketch columns; coefficients of those columns staged in LDS.  Rows
// 2 pos[i], 2 pos[i] + 1 of Y (row-major, ncols) get the expansion's velocity
// (pos = nullptr: pos[i] = i); accumulate adds to Y.
template <bool LOCAL>
__global__ __launch_bounds__(256) void far_eval_kernel(const NodeRec* __restrict__ tgt, int64_t nt,
                                                       const int* __restrict__ pos, double cx, double cy,
                                                       double inv_rho, const double2* __restrict__ coef, int ncols,
                                                       int accumulate, double* __restrict__ Y) {
  __shared__ double2 cf[FAR_ROWS][FE_COLS];
  const int tid = threadIdx.x;
  const int j0 = blockIdx.y * FE_COLS;
  for (int idx = tid; idx < FAR_ROWS * FE_COLS; idx += 256) {
    const int r = idx / FE_COLS, jj = idx - r * FE_COLS;
    cf[r][jj] = coef[(int64_t)r * ncols + j0 + jj];
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + tid;
  if (i >= nt) return;
  const NodeRec nd = tgt[i];
  const cplx zt = {(nd.x - cx) * inv_rho, (nd.y - cy) * inv_rho};
  cplx acc[FE_COLS];
#pragma unroll
  for (int jj = 0; jj < FE_COLS; ++jj) acc[jj] = {0.0, 0.0};
  // multipole: u = sum_p A_p zeta^-(p+1) + B_p conj(zeta)^-(p+1) + (zeta C_p - D_p) conj(zeta)^-(p+2)
  // local:     u = sum_p -A_p zeta^p - B_p conj(zeta)^p + (zeta C_p - D_p) conj(zeta)^p
  const cplx base = LOCAL ? zt : cinv(zt);
  cplx pw = LOCAL ? cplx{1.0, 0.0} : base;
  const cplx bconj = cconj(base);
  for (int p = 0; p < FAR_P; ++p) {
    const cplx pb = cconj(pw);
    const cplx pc = LOCAL ? pb : cmul(pb, bconj);
    const cplx zpc = cmul(zt, pc);
#pragma unroll
    for (int jj = 0; jj < FE_COLS; ++jj) {
      const double2 a = cf[0 * FAR_P + p][jj], b = cf[1 * FAR_P + p][jj];
      const double2 c = cf[2 * FAR_P + p][jj], d = cf[3 * FAR_P + p][jj];
      const double sa = LOCAL ? -1.0 : 1.0;
      acc[jj].re += sa * (a.x * pw.re - a.y * pw.im) + sa * (b.x * pb.re - b.y * pb.im) +
                    (c.x * zpc.re - c.y * zpc.im) - (d.x * pc.re - d.y * pc.im);
      acc[jj].im += sa * (a.x * pw.im + a.y * pw.re) + sa * (b.x * pb.im + b.y * pb.re) +
                    (c.x * zpc.im + c.y * zpc.re) - (d.x * pc.im + d.y * pc.re);
    }
    pw = cmul(pw, base);
  }
  const double sc = kInv4Pi * inv_rho;
  const int64_t row = 2 * (pos ? (int64_t)pos[i] : i);
  double* y0 = Y + row * ncols + j0;
  double* y1 = y0 + ncols;
#pragma unroll
  for (int jj = 0; jj < FE_COLS; ++jj) {
    const double s = cf[4 * FAR_P][jj].x;
    const double u1 = sc * acc[jj].re + nd.nx * s;
    const double u2 = sc * acc[jj].im + nd.ny * s;
    if (accumulate) {
      y0[jj] += u1;
      y1[jj] += u2;
    } else {
      y0[jj] = u1;
      y1[jj] = u2;
    }
  }
}

// Y rows 2 pos[i], 2 pos[i] + 1 <- rows 2 i, 2 i + 1 of Yc (both row-major, ncols).
__global__ __launch_bounds__(256) void scatter_rows_kernel(const double* __restrict__ Yc, int64_t n,
                                                           const int* __restrict__ pos, int ncols,
                                                           double* __restrict__ Y) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = 2 * n * ncols;
  if (idx >= total) return;
  const int64_t r = idx / ncols, j = idx - r * ncols;
  const int64_t i = r >> 1;
  Y[(2 * (int64_t)pos[i] + (r & 1)) * ncols + j] = Yc[idx];
}

unsigned nblocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

size_t far_part_elems(int ncols, int nsplit) { return (size_t)nsplit * FAR_ROWS * ncols; }

void launch_far_sketch(const SketchSeg* segs, int nseg, const NodeRec* tgt, int64_t nt, const int* pos, bool local,
                       double cx, double cy, double rho, int ncols, uint64_t seed, bool accumulate, double* Y,
                       double2* part, int nsplit, double2* coef, hipStream_t s) {
  if (nt <= 0) return;
  if (ncols % FE_COLS != 0 || ncols > 128) RW_THROW(RW_EINVAL, "far-field sketch: ncols must be a multiple of 16, <= 128");
  if (!(rho > 0.0)) RW_THROW(RW_EINVAL, "far-field sketch: circle radius must be positive");
  FarSegArgs sa{};
  for (int i = 0; i < 2; ++i) {
    const bool on = i < nseg;
    sa.src[i] = on ? segs[i].src : segs[0].src;
    sa.ns[i] = on ? segs[i].ns : 0;
    sa.sign[i] = on ? segs[i].sign : 0.0;
    sa.orow[i] = on ? segs[i].omega_row0 : 0;
  }
  const double inv_rho = 1.0 / rho;
  const int64_t len = (int64_t)FAR_ROWS * ncols;
  {
    KernelTimer kt("far_coef_kernel", 0.0, 0.0, s);
    const dim3 grid((unsigned)nsplit, (unsigned)((ncols + 63) / 64));
    if (local)
      hipLaunchKernelGGL(far_coef_kernel<true>, grid, dim3(256), 0, s, sa, cx, cy, inv_rho, seed, ncols, nsplit, part);
    else
      hipLaunchKernelGGL(far_coef_kernel<false>, grid, dim3(256), 0, s, sa, cx, cy, inv_rho, seed, ncols, nsplit, part);
    KERNEL_CHECK("far_coef");
    hipLaunchKernelGGL(far_coef_sum_kernel, dim3(nblocks(len)), dim3(256), 0, s, part, nsplit, len, coef);
    KERNEL_CHECK("far_coef_sum");
  }
  KernelTimer kt("far_eval_kernel", 0.0, 0.0, s);
  const dim3 grid(nblocks(nt), (unsigned)(ncols / FE_COLS));
  if (local)
    hipLaunchKernelGGL(far_eval_kernel<true>, grid, dim3(256), 0, s, tgt, nt, pos, cx, cy, inv_rho, coef, ncols,
                       accumulate ? 1 : 0, Y);
  else
    hipLaunchKernelGGL(far_eval_kernel<false>, grid, dim3(256), 0, s, tgt, nt, pos, cx, cy, inv_rho, coef, ncols,
                       accumulate ? 1 : 0, Y);
  KERNEL_CHECK("far_eval");
}

void launch_scatter_rows(const double* Yc, int64_t n, const int* pos, int ncols, double* Y, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(scatter_rows_kernel, dim3(nblocks(2 * n * ncols)), dim3(256), 0, s, Yc, n, pos, ncols, Y);
  KERNEL_CHECK("scatter_rows");
}
