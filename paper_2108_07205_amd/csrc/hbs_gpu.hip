// HBS inverse in HBM: upload of a host-built inverse, the level-sweep apply,
// and the batched GPU build used per refinement for A_pp (Algorithm 1,
// pre-computation step 2: an approximate inverse of A_pp from a fast direct
// solver, used when the added node count is large).
//
// GPU build, per tree level (leaves to root), one workgroup per node:
//  1. sketch: Y = M Omega (m x 96) of the node's off-diagonal block row
//     (row ID) and block column (column ID), where M holds the exact kernel
//     entries to the nodes inside the node's proxy circle and, for everything
//     outside it, 48 proxy points on that circle (Stokeslet and double-layer
//     columns / double-layer rows) plus the rank-one nullspace column / flux
//     row; Omega = +-1 from a counter-based hash.  Entries are generated on the
//     fly, never stored.
//  2. row ID of each sketch by pivoted Gram-Schmidt over rows held in
//     registers (one projection per step); the node rank is the larger of
//     the two tolerance ranks.
//  3. interpolation matrices U, V and the skeleton lists (the parent's
//     candidate rows / columns).
//  4. node inverse: D (leaf block, or [[D^_a, A(Jr_a, Jc_b)], [A(Jr_b, Jc_a),
//     D^_b]]), D^ = (V* D^-1 U)^-1, E = D^-1 U D^, F* = D^ V* D^-1,
//     G = D^-1 - D^-1 U D^ V* D^-1; the root stores G_root = D_root^-1.
#include <algorithm>
#include <type_traits>
#include <cmath>
#include <utility>

#include "dev_gj.h"
#include "dev_reduce.h"
#include "hbs_dev.h"

namespace {

constexpr double kInvPi = 0.31830988618379067154;
constexpr int SK_R = 96;       // sketch columns per node
constexpr int SK_KCAP = 88;    // largest node rank (sketch columns minus oversampling)
constexpr int SK_NP = 48;      // proxy points
constexpr double SK_RATIO = 2.0;
constexpr int INV_LDS_N = 128; // node blocks up to this size are inverted in LDS
constexpr int INV_LDS_BYTES = 150 * 1024;

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

struct GNode {
  int64_t n0, n1;       // node range
  double cx, cy, rp;    // proxy circle
  int m;                // candidate count (rows = columns = node input size)
  int k;                // rank (after the ID)
  int64_t cand_off;     // offset in the level's candidate arrays (= input offset)
  int64_t uv_off;       // U / V slot (m x k, column-major)
  int64_t dhat_off;     // D^ (k x k) of this node
  int64_t ws_off;       // inverse workspace
  int64_t up_off, e_off;
};

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// A = -1/2 I + D + N block for target t and source s (w_s folded in).
__device__ __forceinline__ void a_blk(const NodeRec& t, const NodeRec& s, bool self, double B[4]) {
  if (self) { B[0] = s.s00; B[1] = s.s01; B[2] = s.s01; B[3] = s.s11; return; }
  const double rx = t.x - s.x, ry = t.y - s.y;
  const double r2 = rx * rx + ry * ry;
  const double cf = (rx * s.nx + ry * s.ny) * s.w * kInvPi / (r2 * r2);
  B[0] = cf * rx * rx + s.w * t.nx * s.nx;
  B[1] = cf * rx * ry + s.w * t.nx * s.ny;
  B[2] = cf * ry * rx + s.w * t.ny * s.nx;
  B[3] = cf * ry * ry + s.w * t.ny * s.ny;
}

// ---------------------------------------------------------------- 0. proxy circles
// One workgroup per node record g = 1 .. 2^(L+1) - 1 (level l at
// [2^l, 2^(l+1))): the centroid (cx, cy) of the node's points [n0, n1) and
// the proxy radius rp = SK_RATIO max |x_i - c|, by block sums and maxima in
// a fixed order.
__global__ __launch_bounds__(256) void node_geom_kernel(GNode* __restrict__ dg, const NodeRec* __restrict__ nd) {
  __shared__ double red[3][4];
  GNode& g = dg[blockIdx.x + 1];
  const int64_t n0 = g.n0, n1 = g.n1;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double sx = 0.0, sy = 0.0;
  for (int64_t i = n0 + tid; i < n1; i += 256) {
    sx += nd[i].x;
    sy += nd[i].y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sx += __shfl_xor(sx, o);
    sy += __shfl_xor(sy, o);
  }
  if (lane == 0) { red[0][w] = sx; red[1][w] = sy; }
  __syncthreads();
  const double inv = 1.0 / (double)(n1 - n0);
  const double cx = ((red[0][0] + red[0][1]) + (red[0][2] + red[0][3])) * inv;
  const double cy = ((red[1][0] + red[1][1]) + (red[1][2] + red[1][3])) * inv;
  double r2 = 0.0;
  for (int64_t i = n0 + tid; i < n1; i += 256) {
    const double dx = nd[i].x - cx, dy = nd[i].y - cy;
    r2 = fmax(r2, dx * dx + dy * dy);
  }
  r2 = wave_max_nonneg(r2);
  if (lane == 0) red[2][w] = r2;
  __syncthreads();
  if (tid == 0) {
    g.cx = cx;
    g.cy = cy;
    g.rp = SK_RATIO * sqrt(fmax(fmax(red[2][0], red[2][1]), fmax(red[2][2], red[2][3])));
  }
}

// ---------------------------------------------------------------- 1. sketch
// grid (nodes, 2): side 0 = row sketch of candr, side 1 = column sketch of candc.
// thread t: candidate row (t & 127) of the current pass, columns 48*(t >> 7) ..
// grid (nodes, 2, nsplit): split z handles nodes [z N / nsplit, (z+1) N / nsplit);
// the last split also adds the proxy and nullspace entities.  Partial sums go
// to part[z] (same layout as S), summed by node_sketch_sum_kernel.
__global__ __launch_bounds__(256) void node_sketch_kernel(const GNode* __restrict__ gn, const int* __restrict__ candr,
                                                          const int* __restrict__ candc,
                                                          const NodeRec* __restrict__ nd, int64_t N, uint64_t seed,
                                                          int64_t part_stride, double* __restrict__ Sr,
                                                          double* __restrict__ Sc, int mlo, int mhi) {
  __shared__ NodeRec snd[256];
  const GNode g = gn[blockIdx.x];
  if (g.m <= mlo || g.m > mhi) return;   // node handled by another launch
  const int side = blockIdx.y;
  const int z = blockIdx.z, nz = gridDim.z;
  const int* cand = (side == 0 ? candr : candc) + g.cand_off;
  double* S = (side == 0 ? Sr : Sc) + g.cand_off * SK_R + (int64_t)z * part_stride;
  const int64_t j_lo = (z * N) / nz, j_hi = ((z + 1) * N) / nz;
  const bool last = (z == nz - 1);
  const int half = threadIdx.x >> 7, ri = threadIdx.x & 127;
  const double rp2 = g.rp * g.rp;
  const double wp = 2.0 * M_PI * g.rp / SK_NP;
  const uint64_t base = seed * 0x9E3779B97F4A7C15ull;
  for (int row0 = 0; row0 < g.m; row0 += 128) {
    const int i = row0 + ri;
    const bool valid = i < g.m;
    const int dof = cand[valid ? i : 0];
    const NodeRec a = nd[dof >> 1];
    const int ca = dof & 1;
    double acc[48];
#pragma unroll
    for (int c = 0; c < 48; ++c) acc[c] = 0.0;
    // Entities: near nodes (2 entries each), then -- if any node lies outside
    // the proxy circle -- the proxy points (side 0: 4 entries, side 1: 2) and
    // the nullspace column / flux row (1 entry).  Each entry e with Omega row
    // `pos` is folded into the 48 accumulators by one shared loop.
    // the proxies stand for every node outside the circle: does one exist?
    bool any_far = false;
    if (last) {
      for (int64_t j0 = 0; j0 < N && !any_far; j0 += 256) {
        const int64_t jj = j0 + threadIdx.x;
        int far = 0;
        if (jj < N && !(jj >= g.n0 && jj < g.n1)) {
          const double dx = nd[jj].x - g.cx, dy = nd[jj].y - g.cy;
          far = dx * dx + dy * dy >= rp2;
        }
        any_far = __syncthreads_or(far) != 0;
      }
    }
    const int64_t n_ent = last ? N + SK_NP + 1 : j_hi;
    for (int64_t j = j_lo; j < n_ent; ++j) {
      if (j < j_hi && ((j - j_lo) & 255) == 0) {
        // stage the next 256 nodes of this split through LDS
        __syncthreads();
        const int64_t jj = j + threadIdx.x;
        if (jj < j_hi) snd[threadIdx.x] = nd[jj];
        __syncthreads();
      }
      if (j >= j_hi && j < N) { j = N - 1; continue; }   // jump to the proxies
      double e[4];
      int64_t pos0 = 0;
      int cnt = 0;
      if (j < N) {
        if (j >= g.n0 && j < g.n1) continue;
        const NodeRec q = snd[(j - j_lo) & 255];
        const double dx = q.x - g.cx, dy = q.y - g.cy;
        if (dx * dx + dy * dy >= rp2) continue;
        double B[4];
        if (side == 0) {
          a_blk(a, q, false, B);                 // A(a, j)
          e[0] = B[ca * 2 + 0];
          e[1] = B[ca * 2 + 1];
        } else {
          a_blk(q, a, false, B);                 // A(j, a)
          e[0] = B[0 * 2 + ca];
          e[1] = B[1 * 2 + ca];
        }
        pos0 = 2 * j;
        cnt = 2;
      } else if (!any_far) {
        break;
      } else if (j < N + SK_NP) {
        const int l = (int)(j - N);
        const double th = 2.0 * M_PI * l / SK_NP;
        const double ux = cos(th), uy = sin(th);
        const double px = g.cx + g.rp * ux, py = g.cy + g.rp * uy;
        if (side == 0) {
          const double rx = a.x - px, ry = a.y - py, r2 = rx * rx + ry * ry;
          const double lg = -0.125 * kInvPi * log(r2), b = 0.25 * kInvPi / r2;
          const double rc = ca ? ry : rx;
          const double cf = (rx * ux + ry * uy) * kInvPi / (r2 * r2) * wp;
          e[0] = (ca == 0 ? lg : 0.0) + b * rc * rx;   // Stokeslet, source comp 0
          e[1] = (ca == 1 ? lg : 0.0) + b * rc * ry;   // Stokeslet, source comp 1
          e[2] = cf * rc * rx;                          // double layer (radial normal)
          e[3] = cf * rc * ry;
          cnt = 4;
        } else {
          const double rx = px - a.x, ry = py - a.y, r2 = rx * rx + ry * ry;
          const double cf = (rx * a.nx + ry * a.ny) * a.w * kInvPi / (r2 * r2);
          const double rd = ca ? ry : rx;
          e[0] = cf * rx * rd;                          // target comp 0 at the proxy
          e[1] = cf * ry * rd;                          // target comp 1
          cnt = 2;
        }
        pos0 = 2 * N + 4 * (int64_t)l;
      } else {
        e[0] = (side == 0) ? (ca ? a.ny : a.nx) : a.w * (ca ? a.ny : a.nx);
        pos0 = 2 * N + 4 * (int64_t)SK_NP;
        cnt = 1;
      }
      for (int t = 0; t < cnt; ++t) {
        const double v = e[t];
        const uint64_t key = base ^ ((uint64_t)(pos0 + t) * 0xD1B54A32D192ED03ull);
        const uint64_t h0 = mix64(key);
        const uint64_t h1 = mix64(key ^ 0x5851F42D4C957F2Dull);
        // columns 48*half .. 48*half+47 of the 96-bit sign pattern (h0 | h1)
        const uint64_t lo = half ? ((h0 >> 48) | (h1 << 16)) : h0;
        const uint64_t hi = half ? (h1 >> 48) : 0;
        (void)hi;
#pragma unroll
        for (int c = 0; c < 48; ++c) acc[c] += ((lo >> c) & 1) ? -v : v;
      }
    }
    if (valid)
#pragma unroll
      for (int c = 0; c < 48; ++c) S[(int64_t)i * SK_R + half * 48 + c] = acc[c];
  }
}

// MFMA form of the node sketch (same Y = M Omega, same entities and Omega
// rows), for nodes of at most 64 RBW candidate rows.  grid (nodes, 2).
// Near nodes are found pass by pass (2048 nodes per pass, compacted in index
// order by a block prefix sum, so the summation order is fixed); entity
// columns are taken 16 at a time: the threads write the A tile (thread t:
// column t % 16, rows t / 16 + 16 u) and the +-1 Omega tile to LDS, then wave
// w accumulates its row blocks w, w + 4, ... times the six 16-column blocks
// of the sketch on the FP64 matrix cores.
typedef double double4_t __attribute__((ext_vector_type(4)));
constexpr int NSK_PASS = 2048;

// 96 signs of Omega row pos (bit c of (lo, hi) is column c).
__device__ __forceinline__ void sketch_signs(uint64_t base, int64_t pos, uint64_t& lo, uint64_t& hi) {
  const uint64_t key = base ^ ((uint64_t)pos * 0xD1B54A32D192ED03ull);
  lo = mix64(key);
  hi = mix64(key ^ 0x5851F42D4C957F2Dull);
}

template <int RBW>
__global__ __launch_bounds__(256) void node_sketch_mfma_kernel(const GNode* __restrict__ gn,
                                                               const int* __restrict__ candr,
                                                               const int* __restrict__ candc,
                                                               const NodeRec* __restrict__ nd, int64_t N,
                                                               uint64_t seed, int64_t part_stride,
                                                               double* __restrict__ Sr, double* __restrict__ Sc,
                                                               int mlo, int mhi) {
  constexpr int MR = 64 * RBW;  // row capacity
  __shared__ NodeRec rn[MR];
  __shared__ int rc[MR];
  __shared__ int nlist[NSK_PASS];
  __shared__ int wsum[257];
  __shared__ double As[16][MR + 2];
  __shared__ double Bs[16][SK_R + 2];
  const GNode g = gn[blockIdx.x];
  if (g.m <= mlo || g.m > mhi) return;   // node handled by another launch
  const int side = blockIdx.y, m = g.m;
  const int z = blockIdx.z, nz = gridDim.z;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, i16 = lane & 15, k4 = lane >> 4;
  const int* cand = (side == 0 ? candr : candc) + g.cand_off;
  double* S = (side == 0 ? Sr : Sc) + g.cand_off * SK_R + (int64_t)z * part_stride;
  const double rp2 = g.rp * g.rp;
  const double wp = 2.0 * M_PI * g.rp / SK_NP;
  const uint64_t base = seed * 0x9E3779B97F4A7C15ull;
  for (int i = tid; i < m; i += 256) {
    const int dof = cand[i];
    rn[i] = nd[dof >> 1];
    rc[i] = dof & 1;
  }
  double4_t acc[RBW][6];
#pragma unroll
  for (int u = 0; u < RBW; ++u)
#pragma unroll
    for (int cb = 0; cb < 6; ++cb) acc[u][cb] = (double4_t){0.0, 0.0, 0.0, 0.0};
  const int nrb = (m + 15) >> 4;
  // one chunk of 16 entity columns: kind 0 = near node dofs (nlist[c0 / 2 ..]),
  // 1 = proxy columns c0 .., 2 = the nullspace column
  auto chunk = [&](int kind, int c0, int ncols) {
    const int col = tid & 15;
    const bool cval = col < ncols;
    // entity of this column
    NodeRec q{};
    int comp = 0, pl = 0, kd = 0;
    int64_t pos = 0;
    double px = 0, py = 0, ux = 0, uy = 0;
    if (cval) {
      if (kind == 0) {
        const int j = nlist[(c0 + col) >> 1];
        comp = (c0 + col) & 1;
        q = nd[j];
        pos = 2 * (int64_t)j + comp;
      } else if (kind == 1) {
        const int u = c0 + col;
        const int per = side == 0 ? 4 : 2;
        pl = u / per;
        kd = u - pl * per;
        const double th = 2.0 * M_PI * pl / SK_NP;
        ux = cos(th);
        uy = sin(th);
        px = g.cx + g.rp * ux;
        py = g.cy + g.rp * uy;
        pos = 2 * N + 4 * (int64_t)pl + kd;
      } else {
        pos = 2 * N + 4 * (int64_t)SK_NP;
      }
    }
    for (int i = tid >> 4; i < nrb * 16; i += 16) {
      double v = 0.0;
      if (cval && i < m) {
        const NodeRec& a = rn[i];
        const int ca = rc[i];
        if (kind == 0) {
          double B[4];
          if (side == 0) {
            a_blk(a, q, false, B);  // A(a, j)
            v = B[ca * 2 + comp];
          } else {
            a_blk(q, a, false, B);  // A(j, a)
            v = B[comp * 2 + ca];
          }
        } else if (kind == 1) {
          if (side == 0) {
            const double rx = a.x - px, ry = a.y - py, r2 = rx * rx + ry * ry;
            const double rcv = ca ? ry : rx;
            if (kd < 2) {  // Stokeslet, source component kd
              v = ((ca == kd) ? -0.125 * kInvPi * log(r2) : 0.0) + 0.25 * kInvPi / r2 * rcv * (kd ? ry : rx);
            } else {       // double layer with the radial normal
              const double cf = (rx * ux + ry * uy) * kInvPi / (r2 * r2) * wp;
              v = cf * rcv * (kd == 3 ? ry : rx);
            }
          } else {
            const double rx = px - a.x, ry = py - a.y, r2 = rx * rx + ry * ry;
            const double cf = (rx * a.nx + ry * a.ny) * a.w * kInvPi / (r2 * r2);
            v = cf * (kd ? ry : rx) * (ca ? ry : rx);
          }
        } else {
          v = (side == 0) ? (ca ? a.ny : a.nx) : a.w * (ca ? a.ny : a.nx);
        }
      }
      As[col][i] = v;
    }
    {
      const int bc = tid >> 4, gcol = tid & 15;  // column bc of the chunk, sketch columns gcol + 16 cb
      uint64_t lo = 0, hi = 0;
      const bool ok = bc < ncols;
      if (ok) {
        int64_t bpos;
        if (kind == 0) bpos = 2 * (int64_t)nlist[(c0 + bc) >> 1] + ((c0 + bc) & 1);
        else if (kind == 1) {
          const int per = side == 0 ? 4 : 2;
          const int u = c0 + bc, l = u / per;
          bpos = 2 * N + 4 * (int64_t)l + (u - l * per);
        } else bpos = 2 * N + 4 * (int64_t)SK_NP;
        sketch_signs(base, bpos, lo, hi);
      }
#pragma unroll
      for (int cb = 0; cb < 6; ++cb) {
        const int c = cb * 16 + gcol;
        const uint64_t bit = c < 64 ? (lo >> c) & 1ull : (hi >> (c - 64)) & 1ull;
        Bs[bc][c] = ok ? (bit ? -1.0 : 1.0) : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      double bv[6];
#pragma unroll
      for (int cb = 0; cb < 6; ++cb) bv[cb] = Bs[ks * 4 + k4][cb * 16 + i16];
#pragma unroll
      for (int u = 0; u < RBW; ++u) {
        const int rb = wave + 4 * u;
        if (rb < nrb) {
          const double a = As[ks * 4 + k4][rb * 16 + i16];
#pragma unroll
          for (int cb = 0; cb < 6; ++cb) acc[u][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv[cb], acc[u][cb], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  };
  // ---- near nodes of the whole arc, pass by pass; the 16-column chunks of
  // each pass's near list, then the proxy chunks and the nullspace column,
  // are dealt round-robin over the splits, so every split does the same work
  int chunk_no = 0;   // running chunk number (near chunks of all passes, then the far chunks)
  int farl_any = 0;
  for (int64_t p0 = 0; p0 < N; p0 += NSK_PASS) {
    const int64_t p1 = min(N, p0 + NSK_PASS);
    const int per = NSK_PASS / 256;
    int cntl = 0, farl = 0;
    int loc[NSK_PASS / 256];
#pragma unroll
    for (int u = 0; u < NSK_PASS / 256; ++u) {
      const int64_t j = p0 + tid * per + u;
      loc[u] = 0;
      if (j < p1 && !(j >= g.n0 && j < g.n1)) {
        const double dx = nd[j].x - g.cx, dy = nd[j].y - g.cy;
        if (dx * dx + dy * dy < rp2) { loc[u] = 1; ++cntl; } else farl = 1;
      }
    }
    // exclusive prefix of the per-thread counts: wave scan, then the 4 wave totals
    int incl = cntl;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(incl, o);
      if (lane >= o) incl += v;
    }
    if (lane == 63) wsum[wave] = incl;
    farl_any |= __syncthreads_or(farl);
    int wbase = 0;
#pragma unroll
    for (int w2 = 0; w2 < 4; ++w2) wbase += (w2 < wave) ? wsum[w2] : 0;
    const int nnear = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    int o = wbase + incl - cntl;
#pragma unroll
    for (int u = 0; u < NSK_PASS / 256; ++u)
      if (loc[u]) nlist[o++] = (int)(p0 + tid * per + u);
    __syncthreads();
    for (int c0 = 0; c0 < 2 * nnear; c0 += 16, ++chunk_no)
      if (chunk_no % nz == z) chunk(0, c0, min(16, 2 * nnear - c0));
    __syncthreads();   // nlist and wsum are rewritten by the next pass
  }
  // ---- proxies and the nullspace column stand for the far nodes, if any
  if (farl_any) {
    const int npc = SK_NP * (side == 0 ? 4 : 2);
    for (int c0 = 0; c0 < npc; c0 += 16, ++chunk_no)
      if (chunk_no % nz == z) chunk(1, c0, min(16, npc - c0));
    if (chunk_no % nz == z) chunk(2, 0, 1);
    ++chunk_no;
  }
  // ---- write the sketch rows (m x SK_R, row-major)
#pragma unroll
  for (int u = 0; u < RBW; ++u) {
    const int rb = wave + 4 * u;
#pragma unroll
    for (int cb = 0; cb < 6; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // v_mfma_f64_16x16x4f64: item r of lane l holds D[l / 16 + 4 r][l % 16]
        const int row = rb * 16 + k4 + 4 * r;
        if (rb < nrb && row < m) S[(int64_t)row * SK_R + cb * 16 + i16] = acc[u][cb][r];
      }
  }
}

// grid (ceil(len / 256), 2): y = 0 sums the row-sketch partials, y = 1 the column ones.
__global__ __launch_bounds__(256) void node_sketch_sum_kernel(const double* __restrict__ part_r,
                                                              const double* __restrict__ part_c, int nsplit,
                                                              int64_t len, int64_t stride, double* __restrict__ Sr,
                                                              double* __restrict__ Sc) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= len) return;
  const double* part = blockIdx.y ? part_c : part_r;
  // four independent sums (z mod 4), so that four loads are in flight at a
  // time, combined in a fixed order
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  int z = 0;
  for (; z + 4 <= nsplit; z += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] += part[i + (int64_t)(z + u) * stride];
  }
  for (int u = 0; z < nsplit; ++z, ++u) v[u] += part[i + (int64_t)z * stride];
  (blockIdx.y ? Sc : Sr)[i] = (v[0] + v[1]) + (v[2] + v[3]);
}

// ---------------------------------------------------------------- 2. row ID
// (value, index) maximum over a wavefront; ties go to the lower index, index
// -1 marks an empty slot.
__device__ __forceinline__ void wave_argmax(double& v, int& i) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double v2 = __shfl_xor(v, off);
    const int i2 = __shfl_xor(i, off);
    if (i2 >= 0 && (i < 0 || v2 > v || (v2 == v && i2 < i))) { v = v2; i = i2; }
  }
}

// Sum over the TPR (2 or 4) consecutive lanes that hold one sketch row, by
// DPP quad permutations; every lane of the group gets the same bits.
template <int TPR>
__device__ __forceinline__ double row_group_sum(double t) {
  t += dpp_f64<0xB1, 0xf>(t);                          // quad_perm [1,0,3,2]
  if constexpr (TPR == 4) t += dpp_f64<0x4E, 0xf>(t);  // quad_perm [2,3,0,1]
  return t;
}

// Dot product of CPT-vectors with four independent partial sums.
template <int CPT>
__device__ __forceinline__ double dot_by4(const double (&a)[CPT], const double (&b)[CPT]) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
  for (int c = 0; c < CPT; c += 4) {
    s0 = fma(a[c], b[c], s0);
    s1 = fma(a[c + 1], b[c + 1], s1);
    s2 = fma(a[c + 2], b[c + 2], s2);
    s3 = fma(a[c + 3], b[c + 3], s3);
  }
  return (s0 + s1) + (s2 + s3);
}

// Pivoted Gram-Schmidt on one node side: sketch row i lives in the registers
// of the TPR threads TPR i .. TPR i + TPR - 1 (SK_R / TPR columns each), and
// every step projects the remaining rows on the new direction once.  The
// computed quantities satisfy Y = C Q^T + R exactly up to the rounding of
// each update, whether or not Q stays orthogonal to working precision, and
// the rank test recomputes the residual row norms, so the interpolation
// error stays bounded by the residual rows without a second pass.
// Outputs piv[SK_KCAP], C (m x SK_KCAP row-major at cand_off*SK_KCAP),
// info[0] = tolerance rank, info[1] = steps.
// The node's rank is the larger of the two sides' tolerance ranks, so a side
// needs steps up to the other side's rank: each side publishes its rank in
// pub (tagged with the level) as soon as it is known and stops once it has
// taken as many steps as both ranks.  While the other side's rank is not in
// (that side may not be running yet) it goes on, up to kmax steps, so the
// node's rank never depends on the order in which the two sides run.
// The pivot keys and the pivot vector alternate between two LDS slots, so a
// step needs two barriers: a slot is written again two steps later, after
// every thread has passed the first barrier of the step in between.
// The pivot vector's TPR slices of SK_R / TPR entries lie ID_QST(TPR)
// doubles apart, a stride of 2 (mod 16) doubles, so that the lanes of a wave
// reading the same pair of entries of the TPR slices hit disjoint LDS banks.
constexpr int ID_NT = 512;
__host__ __device__ constexpr int ID_QST(int tpr) { return SK_R / tpr + (18 - (SK_R / tpr) % 16) % 16; }
struct IdScratch {
  double q[2][4 * ID_QST(4)];
  double rv[2][ID_NT / 64];
  int other[2];
};

template <int TPR>
__device__ __forceinline__ void node_id_body(const GNode& g, const double* __restrict__ S, double tol2, int* pv,
                                             double* __restrict__ C, int* __restrict__ inf, long long* mine,
                                             long long* theirs, long long tag, IdScratch& L) {
  constexpr int NW = ID_NT / 64, CPT = SK_R / TPR, QST = ID_QST(TPR);
  static_assert(CPT % 4 == 0, "four partial sums per dot product");
  static_assert(QST % 16 == 2 && TPR * QST <= 4 * ID_QST(4), "pivot vector slices");
  const int m = g.m, tid = threadIdx.x;
  const int i = tid / TPR, h = tid % TPR;
  const bool valid = i < m;
  double y[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) y[c] = valid ? S[(int64_t)i * SK_R + h * CPT + c] : 0.0;
  double nrm = row_group_sum<TPR>(dot_by4<CPT>(y, y));
  bool sel = !valid;
  double n0 = 0;
  int rank = -1, step = 0;
  const int kmax = min(SK_KCAP, m);
  // the other side's published rank, loaded one step ahead of its use
  long long seen = 0;
  if (tid == 0) seen = __hip_atomic_load(theirs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (; step < kmax; ++step) {
    const int b = step & 1;
    // pivot: DPP maximum of the keys of the unselected rows (the key carries
    // the squared norm to 2^-43 relative, enough for the rank decision)
    const double key = wave_max_nonneg(pivot_key_bits<9>(nrm, i, !sel));
    if ((tid & 63) == 0) L.rv[b][tid >> 6] = key;
    if (tid == 0) {
      L.other[b] = (seen >> 8) == tag ? (int)(seen & 255) : -1;
      seen = __hip_atomic_load(theirs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    double v = L.rv[b][0];
#pragma unroll
    for (int w = 1; w < NW; ++w) v = fmax(v, L.rv[b][w]);
    const int p = v > 0.0 ? pivot_key_index<9>(v) : -1;
    if (step == 0) n0 = v;
    if (rank < 0 && !(v > tol2 * n0)) {
      rank = step;
      if (tid == 0) __hip_atomic_store(mine, (tag << 8) | rank, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const int other = L.other[b];
    if (rank >= 0 && other >= 0 && step >= max(rank, other)) break;
    if (p < 0 || !(v >= 2.2250738585072014e-308)) break;
    if (i == p) {
      const double inv = 1.0 / sqrt(nrm);
#pragma unroll
      for (int c = 0; c < CPT; ++c) L.q[b][h * QST + c] = y[c] * inv;
    }
    if (tid == 0) pv[step] = p;
    __syncthreads();
    double qr[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) qr[c] = L.q[b][h * QST + c];
    const double cf = row_group_sum<TPR>(dot_by4<CPT>(y, qr));
#pragma unroll
    for (int c = 0; c < CPT; ++c) y[c] = fma(-cf, qr[c], y[c]);
    if (valid && h == 0) C[(int64_t)i * SK_KCAP + step] = cf;
    if (i == p) sel = true;
    nrm = row_group_sum<TPR>(dot_by4<CPT>(y, y));
  }
  if (tid == 0) {
    inf[0] = rank < 0 ? step : rank;
    inf[1] = step;
  }
}

// grid (nodes, 2), ID_NT threads: y = 0 the row side, y = 1 the column side.
// ---------------------------------------------------------------- 2b. level plan
// One wave: the ID ranks of level l (info: row rank, row steps,
// column rank, column steps per node) give each node's rank k (the larger
// tolerance rank, at most the smaller step count) and, by prefix sums in
// node order, its U / V, D^, workspace and generator offsets; the skeleton
// positions in the parent's candidate list (ppos); the parent level's
// candidate counts m and offsets.  cnt[0] (generator entries used) advances
// by the level's total.  fail[1]: a rank reached the sketch size, or a side
// stopped before the larger tolerance rank (cannot happen: each side runs
// until it has seen both ranks, or to the end of its candidates); fail[2]:
// an offset passed its buffer bound.
__device__ __forceinline__ long long wave_incl_scan(long long v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const long long u = __shfl_up(v, o);
    if (lane >= o) v += u;
  }
  return v;
}

// Run by one wave (lane = 0 .. 63) of the level's last ID workgroup.
__device__ void level_plan_wave(GNode* gl, int nn, const int* info, GNode* gpar, int64_t* ppos, int64_t* cnt,
                                int64_t gen_cap, int64_t ws_cap, int* fail, int lane) {
  long long base[5] = {0, 0, 0, (long long)cnt[0], 0};   // U/V, D^, workspace, generators, skeleton positions
  for (int j0 = 0; j0 < nn; j0 += 64) {
    const int j = j0 + lane;
    const bool v = j < nn;
    long long m = 0, k = 0;
    if (v) {
      m = gl[j].m;
      const int kr = info[4 * j], sr = info[4 * j + 1], kc = info[4 * j + 2], sc = info[4 * j + 3];
      k = min(max(kr, kc), min(sr, sc));
      if (max(kr, kc) >= SK_KCAP || k < max(kr, kc)) fail[1] = 1;
    }
    const long long q[5] = {m * k, k * k, 3 * m * m + 2 * m * k + 2 * k * k, (k + m) * m + m * k, k};
    long long ex[5], tot[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) {
      const long long in = wave_incl_scan(q[t], lane);
      ex[t] = base[t] + in - q[t];
      tot[t] = __shfl(in, 63);
    }
    const long long k_next = __shfl_down(k, 1);
    if (v) {
      GNode& g = gl[j];
      g.k = (int)k;
      g.uv_off = ex[0];
      g.dhat_off = ex[1];
      g.ws_off = ex[2];
      g.up_off = ex[3];
      g.e_off = ex[3] + (k + m) * m;
      ppos[j] = ex[4];
      if ((j & 1) == 0) {
        gpar[j >> 1].m = (int)(k + k_next);
        gpar[j >> 1].cand_off = ex[4];
      }
    }
#pragma unroll
    for (int t = 0; t < 5; ++t) base[t] += tot[t];
  }
  if (lane == 0) {
    cnt[0] = base[3];
    if (base[3] > gen_cap || base[2] > ws_cap) fail[2] = 1;
  }
}

// Nodes of at most 128 candidates take four threads per row, larger ones (up
// to 256) two.  pub: 2 slots per node, zero at the start of the build; tag:
// a positive number unique to the level.  The workgroup that finishes last
// (a device-scope counter, done, zero at the start of the build, counts the
// finished workgroups after each has fenced its results) runs the level plan
// below on its first wave, so that the plan needs no launch of its own.
__global__ __launch_bounds__(ID_NT) void node_id_kernel(GNode* gl, const double* __restrict__ Sr,
                                                        const double* __restrict__ Sc, double tol2,
                                                        int* __restrict__ piv, double* __restrict__ Cr,
                                                        double* __restrict__ Cc, int* info,
                                                        long long* __restrict__ pub, long long tag,
                                                        GNode* gpar, int64_t* ppos, int64_t* cnt, int64_t gen_cap,
                                                        int64_t ws_cap, int* fail,
                                                        unsigned long long* __restrict__ done) {
  __shared__ IdScratch L;
  __shared__ int last;
  const GNode g = gl[blockIdx.x];
  const int side = blockIdx.y;
  const double* S = (side == 0 ? Sr : Sc) + g.cand_off * SK_R;
  double* C = (side == 0 ? Cr : Cc) + g.cand_off * SK_KCAP;
  int* pv = piv + ((int64_t)blockIdx.x * 2 + side) * SK_KCAP;
  int* inf = info + (blockIdx.x * 2 + side) * 2;
  long long* mine = pub + blockIdx.x * 2 + side;
  long long* theirs = pub + blockIdx.x * 2 + (1 - side);
  if (g.m <= 128)
    node_id_body<4>(g, S, tol2, pv, C, inf, mine, theirs, tag, L);
  else
    node_id_body<2>(g, S, tol2, pv, C, inf, mine, theirs, tag, L);
  // thread 0 wrote this workgroup's info; release it, then count
  if (threadIdx.x == 0) {
    __threadfence();
    last = atomicAdd(done, 1ull) == 2ull * gridDim.x - 1;
  }
  __syncthreads();
  if (last && threadIdx.x < 64) {   // uniform per workgroup
    __threadfence();   // acquire the other workgroups' info
    level_plan_wave(gl, gridDim.x, info, gpar, ppos, cnt, gen_cap, ws_cap, fail, threadIdx.x);
  }
}

// ---------------------------------------------------------------- 2c. apply descriptors
// Once per build, over the node records 1 .. 2^(L+1) - 1 (level l at
// [2^l, 2^(l+1))): level l's input sizes and ranks go to ints[2^(l+1) - 4 ..]
// (nin, then k), its input offsets, skeleton offsets (ppos), [F*; G] and E
// offsets to offs[2^(l+2) - 8 ..]; the root size to ints[2^(L+2) - 4].  A
// failed build leaves every size zero, so that applies do nothing.
__global__ __launch_bounds__(256) void apply_desc_kernel(const GNode* __restrict__ dg,
                                                         const int64_t* __restrict__ ppos, int L,
                                                         const int* __restrict__ fail, int* __restrict__ ints,
                                                         int64_t* __restrict__ offs) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x + 1;
  if (g >= (int64_t(2) << L)) return;
  const bool bad = (fail[0] | fail[1] | fail[2]) != 0;
  const GNode r = dg[g];
  if (g == 1) {
    ints[(int64_t(4) << L) - 4] = bad ? 0 : r.m;
    return;
  }
  const int l = 63 - __clzll((unsigned long long)g);
  const int64_t nn = int64_t(1) << l, j = g - nn;
  int* ii = ints + 2 * nn - 4;
  int64_t* oo = offs + 4 * nn - 8;
  ii[j] = bad ? 0 : r.m;
  ii[nn + j] = bad ? 0 : r.k;
  oo[j] = r.cand_off;
  oo[nn + j] = ppos[g];
  oo[2 * nn + j] = r.up_off;
  oo[3 * nn + j] = r.e_off;
}

// ---------------------------------------------------------------- 3. interpolation
// grid (nodes, 2).  P = C(:, 0:k) C_J^{-1} -> U (side 0) or V (side 1), m x k
// column-major; the skeleton dofs go to the parent's candidate list.  C_J
// (the pivot rows of the Gram-Schmidt coefficients) is lower triangular: its
// rows are staged in LDS, and its inverse is formed row by row in registers
// (interp_inverse).  The product then gives each thread the C row of its
// candidate and a stripe of SK_KCAP / TPR columns in registers, reading the
// rows of the inverse from LDS as broadcasts.  The skeleton rows get the
// identity rows directly.
constexpr int IV_LD = SK_KCAP;

// Inv = C_J^{-1}, k <= SK_KCAP, by forward substitution along the rows of
// C_J with two threads per column t: thread 2 t + hh holds Inv(u, t) for
// u = 4 w + 2 hh + e (e = 0, 1) in x[2 w + e], so every row step reads the
// row of C_J (cj, ld SK_KCAP, zero above the diagonal) as pairs at static
// offsets and sums over the entries of Inv computed so far (the others are
// still zero).  The pair of threads adds its two partial sums by DPP, and the
// owner of Inv(srow, t) stores it.  dinv: reciprocals of the diagonal.
// Output: Inv in iv (row-major, ld IV_LD), columns t < k.
template <int SROW>
__device__ __forceinline__ void interp_inverse_row(double (&x)[SK_KCAP / 2], const double* cj, const double* dinv,
                                                   int t, int hh) {
  const double* cs = cj + SROW * SK_KCAP + 2 * hh;
  double s0 = 0.0, s1 = 0.0;
#pragma unroll
  for (int w = 0; 4 * w < SROW; ++w) {
    const double2 c2 = *reinterpret_cast<const double2*>(cs + 4 * w);
    s0 = fma(c2.x, x[2 * w], s0);
    s1 = fma(c2.y, x[2 * w + 1], s1);
  }
  const double sum = row_group_sum<2>(s0 + s1);
  const double val = ((SROW == t ? 1.0 : 0.0) - sum) * dinv[SROW];
  if (hh == ((SROW >> 1) & 1)) x[2 * (SROW >> 2) + (SROW & 1)] = val;
}

template <int... R>
__device__ __forceinline__ void interp_inverse_rows(std::integer_sequence<int, R...>, double (&x)[SK_KCAP / 2],
                                                    const double* cj, const double* dinv, int k, int t, int hh) {
  ((R < k ? interp_inverse_row<R>(x, cj, dinv, t, hh) : void()), ...);
}

__device__ __forceinline__ void interp_inverse(const double* cj, const double* dinv, int k, double* iv) {
  constexpr int NX = SK_KCAP / 2;
  static_assert(SK_KCAP % 4 == 0, "pairs of pairs of rows");
  const int t = threadIdx.x >> 1, hh = threadIdx.x & 1;
  double x[NX];
#pragma unroll
  for (int e = 0; e < NX; ++e) x[e] = 0.0;
  interp_inverse_rows(std::make_integer_sequence<int, SK_KCAP>{}, x, cj, dinv, k, t, hh);
  if (t < k) {
#pragma unroll
    for (int w = 0; w < NX / 2; ++w)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int u = 4 * w + 2 * hh + e;
        if (u < k) iv[u * IV_LD + t] = x[2 * w + e];
      }
  }
}

template <int TPR>
__device__ __forceinline__ void interp_product(const double* __restrict__ C, const double* iv, const int* pstep,
                                               int m, int k, double* __restrict__ P) {
  constexpr int CPT = SK_KCAP / TPR;
  static_assert(SK_KCAP % (2 * TPR) == 0, "stripes of whole double pairs");
  const int i = threadIdx.x / TPR, h = threadIdx.x % TPR;
  if (i >= m) return;
  const int c0 = h * CPT;
  const int ps = pstep[i];
  double v[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) v[c] = 0.0;
  if (ps < 0) {
    const double* ci = C + (int64_t)i * SK_KCAP;
    double a = ci[0];
    for (int srow = 0; srow < k; ++srow) {
      const double an = srow + 1 < k ? ci[srow + 1] : 0.0;
      const double* ir = iv + srow * IV_LD + c0;
#pragma unroll
      for (int c = 0; c < CPT; ++c) v[c] = fma(a, ir[c], v[c]);
      a = an;
    }
  } else {
#pragma unroll
    for (int c = 0; c < CPT; ++c) v[c] = (c0 + c == ps) ? 1.0 : 0.0;
  }
#pragma unroll
  for (int c = 0; c < CPT; ++c)
    if (c0 + c < k) P[i + (int64_t)(c0 + c) * m] = v[c];
}

__global__ __launch_bounds__(256) void node_interp_kernel(const GNode* __restrict__ gn,
                                                              const int* __restrict__ candr,
                                                              const int* __restrict__ candc,
                                                              const int* __restrict__ piv,
                                                              const double* __restrict__ Cr,
                                                              const double* __restrict__ Cc, double* __restrict__ U,
                                                              double* __restrict__ V,
                                                              const int64_t* __restrict__ par_pos,
                                                              int* __restrict__ pcandr, int* __restrict__ pcandc) {
  extern __shared__ double lds[];  // cj[s * SK_KCAP + u] = C_J(s, u); iv[u * IV_LD + t] = Inv(u, t)
  __shared__ int pstep[256];       // skeleton step of each candidate, -1 for the others
  __shared__ double dinv[SK_KCAP];
  const GNode g = gn[blockIdx.x];
  const int side = blockIdx.y;
  const int k = g.k, m = g.m, tid = threadIdx.x;
  const int* pv = piv + ((int64_t)blockIdx.x * 2 + side) * SK_KCAP;
  const double* C = (side == 0 ? Cr : Cc) + g.cand_off * SK_KCAP;
  double* P = (side == 0 ? U : V) + g.uv_off;
  double* cj = lds;
  double* iv = lds + SK_KCAP * SK_KCAP;
  for (int idx = tid; idx < k * SK_KCAP; idx += 256) {
    const int srow = idx / SK_KCAP, u = idx - srow * SK_KCAP;
    const double c = (u <= srow) ? C[(int64_t)pv[srow] * SK_KCAP + u] : 0.0;
    cj[idx] = c;
    iv[idx] = 0.0;
    if (u == srow) dinv[srow] = 1.0 / c;
  }
  pstep[tid] = -1;
  __syncthreads();
  if (tid < k) pstep[pv[tid]] = tid;
  interp_inverse(cj, dinv, k, iv);
  __syncthreads();
  if (m <= 64)
    interp_product<4>(C, iv, pstep, m, k, P);
  else if (m <= 128)
    interp_product<2>(C, iv, pstep, m, k, P);
  else
    interp_product<1>(C, iv, pstep, m, k, P);
  if (par_pos) {
    const int* cand = (side == 0 ? candr : candc) + g.cand_off;
    int* pc = (side == 0 ? pcandr : pcandc) + par_pos[blockIdx.x];
    for (int srow = tid; srow < k; srow += 256) pc[srow] = cand[pv[srow]];
  }
}

// ---------------------------------------------------------------- 4. inverse
// One workgroup of 256 threads: in-place Gauss-Jordan inverse with partial
// pivoting of A (n x n, ld n, n <= 256; LDS or global): the pivot row is
// scaled, every other row is eliminated with the pivot column's entry replaced
// by the running inverse, and the recorded row interchanges are undone as
// column interchanges at the end.  Rows are owned by threads (two per row when
// n <= 128), so no index division is needed.  perm: n ints of scratch; f: n
// doubles of scratch.  Returns false on a zero / non-finite pivot.
__device__ bool wg_inverse_inplace(double* A, int n, int* perm, double* f, double* rv, int* ri) {
  const int tid = threadIdx.x;
  const bool two = n <= 128;
  const int row = two ? (tid & 127) : tid;
  const int half = two ? (tid >> 7) : 0;
  const int cw = two ? (n + 1) / 2 : n;
  const int c0 = half * cw, c1 = min(n, c0 + cw);
  for (int j = 0; j < n; ++j) {
    if (tid < 64) {
      double bv = -1.0;
      int bi = -1;
      for (int i = j + tid; i < n; i += 64) {
        const double v = fabs(A[i + j * n]);
        if (v > bv || bi < 0) { bv = v; bi = i; }
      }
      wave_argmax(bv, bi);
      if (tid == 0) { rv[0] = bv; ri[0] = bi; }
    }
    __syncthreads();
    const int p = ri[0];
    const double pabs = rv[0];
    if (p < 0 || !(pabs > 0.0) || !isfinite(pabs)) return false;
    if (tid == 0) perm[j] = p;
    if (p != j)
      for (int c = tid; c < n; c += 256) {
        const double t = A[j + c * n];
        A[j + c * n] = A[p + c * n];
        A[p + c * n] = t;
      }
    __syncthreads();
    const double pinv = 1.0 / A[j + j * n];
    if (tid < n) f[tid] = (tid == j) ? 0.0 : A[tid + j * n];
    __syncthreads();
    for (int c = tid; c < n; c += 256) A[j + c * n] = (c == j) ? pinv : A[j + c * n] * pinv;
    __syncthreads();
    if (row < n && row != j) {
      const double fr = f[row];
      for (int c = c0; c < c1; ++c)
        A[row + c * n] = (c == j) ? -fr * pinv : A[row + c * n] - fr * A[j + c * n];
    }
    __syncthreads();
  }
  for (int j = n - 1; j >= 0; --j) {
    const int p = perm[j];
    if (p != j)
      for (int i = tid; i < n; i += 256) {
        const double t = A[i + j * n];
        A[i + j * n] = A[i + p * n];
        A[i + p * n] = t;
      }
    __syncthreads();
  }
  return true;
}

// C (m x n, ldc) = alpha op(A) op(B) + beta C, all column-major, one
// workgroup of 256 threads; output (i, j) walks the tile without division and
// the inner loop keeps eight independent loads in flight.
__device__ void wg_gemm(bool ta, bool tb, int m, int n, int k, double alpha, const double* __restrict__ A, int lda,
                        const double* __restrict__ B, int ldb, double beta, double* __restrict__ C, int ldc) {
  if (m > 0 && n > 0) {
    int i = threadIdx.x % m, j = threadIdx.x / m;
    const int di = 256 % m, dj = 256 / m;
    const int64_t sa = ta ? 1 : lda, sb = tb ? ldb : 1;     // stride along the inner index
    for (; j < n;) {
      const double* a = ta ? A + (int64_t)i * lda : A + i;
      const double* b = tb ? B + j : B + (int64_t)j * ldb;
      double s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0, s6 = 0, s7 = 0;
      int l = 0;
      for (; l + 8 <= k; l += 8) {
        s0 += a[(l + 0) * sa] * b[(l + 0) * sb];
        s1 += a[(l + 1) * sa] * b[(l + 1) * sb];
        s2 += a[(l + 2) * sa] * b[(l + 2) * sb];
        s3 += a[(l + 3) * sa] * b[(l + 3) * sb];
        s4 += a[(l + 4) * sa] * b[(l + 4) * sb];
        s5 += a[(l + 5) * sa] * b[(l + 5) * sb];
        s6 += a[(l + 6) * sa] * b[(l + 6) * sb];
        s7 += a[(l + 7) * sa] * b[(l + 7) * sb];
      }
      for (; l < k; ++l) s0 += a[l * sa] * b[l * sb];
      const double sum = ((s0 + s1) + (s2 + s3)) + ((s4 + s5) + (s6 + s7));
      C[i + (int64_t)j * ldc] = alpha * sum + (beta == 0.0 ? 0.0 : beta * C[i + (int64_t)j * ldc]);
      i += di;
      j += dj;
      if (i >= m) { i -= m; ++j; }
    }
  }
  __syncthreads();
}

// ------------------------------------------- 4b. register-resident node factorization
// Fast path for node blocks of at most FN = 128 unknowns (every leaf of 64
// nodes and every parent whose children have ranks summing to <= 128).
// Thread t of the 256 owns row (t & 127) of the block and the 64 columns
// 64 (t >> 7) .. + 63 in registers.  Gauss-Jordan with partial pivoting runs
// without moving rows: step j picks pivot row p_j among the rows not yet used
// and applies the in-place exchange update with (p_j, j), which is the
// diagonal-pivot update of the row-permuted matrix P A.  The registers then
// hold (P A)^-1 = A^-1 P^T with row j stored in row p_j, so
// A^-1(j, p_c) = B(p_j, c): the result is scattered to HBM once at the end.
constexpr int FN = 128;
constexpr int GM_KC = 16;  // K chunk of the tiled workgroup GEMM

struct GjScratch {
  double colv[2][FN];  // column j of the current step (double-buffered)
  double key[2][FN];   // pivot keys (pivot_key_bits)
  double prow[2][FN];  // pivot row
  int piv[FN];         // pivot row of each step
};

struct GemmScratch {
  double As[GM_KC][FN + 1];
  double Bs[GM_KC][FN + 1];
};

// In-place Gauss-Jordan inverse of the n x n block held as described above
// (n <= FN; rows >= n and columns >= n must hold zeros).  Registers are never
// indexed dynamically: the half of the columns that holds the current pivot
// column j keeps it in a[0], because that half's update shifts its registers
// down by one (a[c] <- updated a[c + 1], the new column j into a[63]).  On
// return, register c of half h holds column 64 h + ((c + rot) & 63), myq is
// the step at which this thread's row was the pivot (-1 for rows >= n) and
// S.piv[j] the pivot row of step j.  Returns false (uniformly) on a zero or
// non-finite pivot.
__device__ bool reg_gauss_jordan(double (&a)[64], int n, GjScratch& S, int& myq, int& rot) {
  const int tid = threadIdx.x, r = tid & (FN - 1), lane = tid & 63;
  const int h = __builtin_amdgcn_readfirstlane(tid >> 7);
  bool used = r >= n;
  myq = -1;
  for (int j = 0; j < n; ++j) {
    const int b = j & 1;
    const bool own = h == (j >> 6);  // wave-uniform
    if (own) {
      S.colv[b][r] = a[0];
      S.key[b][r] = pivot_key_bits<7>(a[0], r, !used);
    }
    __syncthreads();
    // every wave finds the same pivot (same data, same reduction)
    const double kmax = wave_max_nonneg(fmax(S.key[b][lane], S.key[b][lane + 64]));
    const int p = pivot_key_index<7>(kmax);
    const double piv = S.colv[b][p];
    if (!(fabs(piv) > 0.0) || !isfinite(piv)) return false;
    if (r == p) {
      used = true;
      myq = j;
#pragma unroll
      for (int c = 0; c < 64; ++c) S.prow[b][64 * h + c] = a[c];  // register order of this half
    }
    if (tid == 0) S.piv[j] = p;
    __syncthreads();
    const double pinv = 1.0 / piv;
    const double* pr = &S.prow[b][64 * h];
    if (own) {
      if (r == p) {
#pragma unroll
        for (int c = 0; c < 63; ++c) a[c] = a[c + 1] * pinv;
        a[63] = pinv;
      } else {
        // rows >= n hold zeros and stay zero
        const double f = S.colv[b][r] * pinv;
#pragma unroll
        for (int c = 0; c < 63; ++c) a[c] = a[c + 1] - f * pr[c + 1];
        a[63] = -f;
      }
    } else {
      if (r == p) {
#pragma unroll
        for (int c = 0; c < 64; ++c) a[c] *= pinv;
      } else {
        const double f = S.colv[b][r] * pinv;
#pragma unroll
        for (int c = 0; c < 64; ++c) a[c] -= f * pr[c];
      }
    }
  }
  rot = (h == 0 ? min(n, 64) : max(0, n - 64)) & 63;
  return true;
}

// C (m x n, ldc) = alpha op(A) op(B) + C0 (m x n, ldc0; none when null), all
// column-major, m, n <= FN, any K.  256 threads as a 16 x 16 grid; thread
// (ti, tj) owns rows ti + 16 a (a < MA) and columns tj + 16 b (b < NB); K is
// staged through LDS in chunks of GM_KC (zero-padded past m, n and K).
template <int MA, int NB>
__device__ void wg_gemm_tile(bool ta, bool tb, int m, int n, int K, double alpha, const double* __restrict__ A,
                             int lda, const double* __restrict__ B, int ldb, const double* C0, int ldc0,
                             double* C, int ldc, GemmScratch& S) {
  constexpr int PER = GM_KC * FN / 256;  // staged elements per thread and operand
  const int tid = threadIdx.x, ti = tid & 15, tj = tid >> 4;
  double acc[MA][NB];
#pragma unroll
  for (int x = 0; x < MA; ++x)
#pragma unroll
    for (int y = 0; y < NB; ++y) acc[x][y] = 0.0;
  // element u of this thread's share of a chunk: (row or column, k) pair
  auto a_rk = [&](int u, int& row, int& kc) {
    const int idx = tid + 256 * u;
    if (ta) { kc = idx & (GM_KC - 1); row = idx >> 4; } else { row = idx & (FN - 1); kc = idx >> 7; }
  };
  auto b_ck = [&](int u, int& col, int& kb) {
    const int idx = tid + 256 * u;
    if (tb) { col = idx & (FN - 1); kb = idx >> 7; } else { kb = idx & (GM_KC - 1); col = idx >> 4; }
  };
  double pa[PER], pb[PER];
  auto fetch = [&](int k0) {
    const int kn = min(GM_KC, K - k0);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      int row, kc, col, kb;
      a_rk(u, row, kc);
      b_ck(u, col, kb);
      pa[u] = (row < m && kc < kn) ? (ta ? A[(k0 + kc) + (int64_t)row * lda] : A[row + (int64_t)(k0 + kc) * lda]) : 0.0;
      pb[u] = (col < n && kb < kn) ? (tb ? B[col + (int64_t)(k0 + kb) * ldb] : B[(k0 + kb) + (int64_t)col * ldb]) : 0.0;
    }
  };
  if (K > 0) fetch(0);
  for (int k0 = 0; k0 < K; k0 += GM_KC) {
    const int kn = min(GM_KC, K - k0);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      int row, kc, col, kb;
      a_rk(u, row, kc);
      b_ck(u, col, kb);
      S.As[kc][row] = pa[u];
      S.Bs[kb][col] = pb[u];
    }
    __syncthreads();
    if (k0 + GM_KC < K) fetch(k0 + GM_KC);  // in flight during this chunk's products
    for (int kc = 0; kc < kn; ++kc) {
      double av[MA], bv[NB];
#pragma unroll
      for (int x = 0; x < MA; ++x) av[x] = S.As[kc][ti + 16 * x];
#pragma unroll
      for (int y = 0; y < NB; ++y) bv[y] = S.Bs[kc][tj + 16 * y];
#pragma unroll
      for (int x = 0; x < MA; ++x)
#pragma unroll
        for (int y = 0; y < NB; ++y) acc[x][y] += av[x] * bv[y];
    }
  }
#pragma unroll
  for (int x = 0; x < MA; ++x)
#pragma unroll
    for (int y = 0; y < NB; ++y) {
      const int row = ti + 16 * x, col = tj + 16 * y;
      if (row < m && col < n)
        C[row + (int64_t)col * ldc] = alpha * acc[x][y] + (C0 ? C0[row + (int64_t)col * ldc0] : 0.0);
    }
  __syncthreads();
}

__device__ void wg_gemm_small(bool ta, bool tb, int m, int n, int K, double alpha, const double* A, int lda,
                              const double* B, int ldb, const double* C0, int ldc0, double* C, int ldc,
                              GemmScratch& S) {
  if (m <= 0 || n <= 0) return;
  const bool m8 = m > 64, n8 = n > 64;
  if (!m8 && !n8) wg_gemm_tile<4, 4>(ta, tb, m, n, K, alpha, A, lda, B, ldb, C0, ldc0, C, ldc, S);
  else if (!m8) wg_gemm_tile<4, 8>(ta, tb, m, n, K, alpha, A, lda, B, ldb, C0, ldc0, C, ldc, S);
  else if (!n8) wg_gemm_tile<8, 4>(ta, tb, m, n, K, alpha, A, lda, B, ldb, C0, ldc0, C, ldc, S);
  else wg_gemm_tile<8, 8>(ta, tb, m, n, K, alpha, A, lda, B, ldb, C0, ldc0, C, ldc, S);
}

// One entry of the A = -1/2 I + D + N block: row component ti of target t,
// column component sj of source s.
__device__ __forceinline__ double a_entry(const NodeRec& t, const NodeRec& s, bool self, int ti, int sj) {
  if (self) return (ti == 0) ? (sj == 0 ? s.s00 : s.s01) : (sj == 0 ? s.s01 : s.s11);
  const double rx = t.x - s.x, ry = t.y - s.y;
  const double r2 = rx * rx + ry * ry;
  const double cf = (rx * s.nx + ry * s.ny) * s.w * kInvPi / (r2 * r2);
  const double rt = ti ? ry : rx, rs = sj ? ry : rx;
  const double nt = ti ? t.ny : t.nx, ns = sj ? s.ny : s.nx;
  return cf * rt * rs + s.w * nt * ns;
}

// a_entry with the target given by its position and normal.
__device__ __forceinline__ double a_entry_xy(double tx, double ty, double tnx, double tny, const NodeRec& s, bool self,
                                             int ti, int sj) {
  if (self) return (ti == 0) ? (sj == 0 ? s.s00 : s.s01) : (sj == 0 ? s.s01 : s.s11);
  const double rx = tx - s.x, ry = ty - s.y;
  const double r2 = rx * rx + ry * ry;
  const double cf = (rx * s.nx + ry * s.ny) * s.w * kInvPi / (r2 * r2);
  const double rt = ti ? ry : rx, rs = sj ? ry : rx;
  const double nt = ti ? tny : tnx, ns = sj ? s.ny : s.nx;
  return cf * rt * rs + s.w * nt * ns;
}

// ------------------------------------------------- 4a. bordered factorization
// One Gauss-Jordan inversion per node of the bordered matrix
//   M = [[D, U], [V*, 0]]   ((n + k) x (n + k)),
// whose inverse, by the block inverse with Schur complement -V* D^-1 U, is
//   M^-1 = [[G, E], [F*, -D^]]
// with D^ = (V* D^-1 U)^-1, E = D^-1 U D^, F* = D^ V* D^-1 and
// G = D^-1 - D^-1 U D^ V* D^-1: every generator of the node in one pass,
// without D^-1 or the products ever leaving the registers.  The root (k = 0)
// gets D^-1 = G_root.
// grid (nodes), BWV * 64 threads; n + k <= BT.  Lane l holds rows l, l + 64,
// l + 128 (sub-rows s), wave w the BC columns BC w .. BC w + BC - 1
// (a[s][c]).  Partial pivoting by rows, which are never moved, so the result
// is (P M)^-1 with row j stored in row p_j; the column steps are blocked by
// the BC columns of a wave (the scheme is described at the sweep below).
constexpr int BT = 192;        // largest bordered size
constexpr int BWV = 12;        // waves
constexpr int BC = BT / BWV;   // columns per wave
constexpr int BS = BT / 64;    // sub-rows per lane
static_assert(BC == 16 && BS == 3, "the column switches and pivot-row branches below are written for 16 x 3");

struct BorderScratch {
  double pan[2][BT][BC + 1];   // transformed panel of the block (alternating slots)
  double rows[BWV][BC][BC + 1];   // per wave: its columns of the block's pivot rows (rows padded
                                  // so that the lanes storing different pivot rows hit different banks)
  double pinv[BT];             // 1 / pivot of each step
  int piv[BT];                 // pivot row of each step
  int bad;                     // a panel met a zero or non-finite pivot
};

__global__ __launch_bounds__(BWV * 64) void node_factor_bordered_kernel(
    const GNode* __restrict__ gn, const GNode* __restrict__ gch, int is_leaf, int is_root,
    const int* __restrict__ candr, const int* __restrict__ candc, const NodeRec* __restrict__ nd,
    const double* __restrict__ U, const double* __restrict__ V, const double* __restrict__ dhat_ch,
    double* __restrict__ dhat, double* __restrict__ ws, double* __restrict__ gen, double* __restrict__ groot,
    int* __restrict__ fail) {
  __shared__ BorderScratch S;
  const GNode g = gn[blockIdx.x];
  const int n = g.m, k = is_root ? 0 : g.k, T = n + k;
  if (T > BT) return;   // node taken by the block-inverse kernels
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int* cr = candr + g.cand_off;
  const int* cc = candc + g.cand_off;
  const double* Un = U + g.uv_off;
  const double* Vn = V + g.uv_off;
  int ka = 0, kb = 0;
  const double *Da = nullptr, *Db = nullptr;
  if (!is_leaf) {
    const GNode ca = gch[2 * blockIdx.x], cbn = gch[2 * blockIdx.x + 1];
    ka = ca.k;
    kb = cbn.k;
    Da = dhat_ch + ca.dhat_off;
    Db = dhat_ch + cbn.dhat_off;
  }
  // ---- M assembled straight into the registers: lane l, wave w hold rows
  // l + 64 s, columns BC w + c (the children's D^ blocks, kernel entries
  // between the candidates, U and V* on the border); one sub-row at a time,
  // the column records read per entry (wave-uniform, from the cache)
  double a[BS][BC];
#pragma unroll
  for (int sr = 0; sr < BS; ++sr) {
    const int row = lane + 64 * sr;
    const int rd = row < n ? cr[row] : 0;
    const NodeRec& t = nd[rd >> 1];
    const double tx = t.x, ty = t.y, tnx = t.nx, tny = t.ny;
#pragma unroll
    for (int c = 0; c < BC; ++c) {
      const int col = BC * w + c;   // wave-uniform
      double v = 0.0;
      if (row < n && col < n) {
        if (!is_leaf && row < ka && col < ka) v = Da[row + col * ka];
        else if (!is_leaf && row >= ka && col >= ka) v = Db[(row - ka) + (col - ka) * kb];
        else {
          const int cb = cc[col];
          v = a_entry_xy(tx, ty, tnx, tny, nd[cb >> 1], is_leaf && (rd >> 1) == (cb >> 1), rd & 1, cb & 1);
        }
      } else if (row < n && col < T) {
        v = Un[row + (int64_t)(col - n) * n];
      } else if (row < T && col < n) {
        v = Vn[col + (int64_t)(row - n) * n];
      }
      a[sr][c] = v;
    }
  }
  // Blocked Gauss-Jordan: block bj is the 16 columns of wave bj.  That wave
  // runs the 16 steps on its own columns alone (pivot search by DPP, pivot
  // row by readlane: no barrier), the new inverse column replacing the
  // eliminated one in place; its columns then hold E(:, I), the block's
  // row operations E = E_15 ... E_0 restricted to the pivot rows I.  After
  // one barrier every other wave's columns take
  //   A <- A + (E(:, I) - I(:, I)) A(I, :),
  // a rank-16 update (the next block's columns first, on the matrix cores).  Pivot rows are not scaled during the sweep (a later
  // elimination with an unscaled pivot row gives the same result for the
  // other rows, and the pivot row stays piv times its scaled form), so each
  // row is divided by its own pivot once at the end.
  if (tid == 0) S.bad = 0;
  bool used[BS];
  int myq[BS];
  double rinv[BS];
#pragma unroll
  for (int sr = 0; sr < BS; ++sr) {
    used[sr] = lane + 64 * sr >= T;
    myq[sr] = -1;
    rinv[sr] = 0.0;
  }
  const int nbk = (T + BC - 1) / BC;
  for (int bj = 0; bj < nbk; ++bj) {
    const int j0 = bj * BC, nb = min(BC, T - j0), slot = bj & 1;
    if (w == bj) {
      // ---- panel: nb steps on this wave's columns
      bool ok = true;
      // pivot key of the step's column: the first one here, the next one
      // inside each step, right after that column is eliminated, so that its
      // search overlaps the step's other column updates
      auto col_key = [&](int c) __attribute__((always_inline)) {
        double km = 0.0;
#pragma unroll
        for (int sr = 0; sr < BS; ++sr) km = fmax(km, pivot_key_bits_sel<8>(a[sr][c], lane + 64 * sr, !used[sr]));
        return wave_max_nonneg(km);
      };
      double kmax = col_key(0);
#pragma unroll
      for (int c = 0; c < BC; ++c) {
        if (c < nb && ok) {
          const int p = __builtin_amdgcn_readfirstlane(pivot_key_index<8>(kmax));
          const int ps = p >> 6, pl = p & 63;
          // pivot row by readlane from its (wave-uniform) row slot: one
          // branch instead of a register select per column
          double pr[BC];
          if (ps == 0) {
#pragma unroll
            for (int cc = 0; cc < BC; ++cc) pr[cc] = readlane_f64(a[0][cc], pl);
          } else if (ps == 1) {
#pragma unroll
            for (int cc = 0; cc < BC; ++cc) pr[cc] = readlane_f64(a[1][cc], pl);
          } else {
#pragma unroll
            for (int cc = 0; cc < BC; ++cc) pr[cc] = readlane_f64(a[2][cc], pl);
          }
          const double piv = pr[c];
          if (!(fabs(piv) >= 2.2250738585072014e-308) || !isfinite(piv)) {
            ok = false;
            if (lane == 0) S.bad = 1;
          } else {
            const double pinv = recip_nr2(piv);
            bool isp[BS];
            double f[BS];
#pragma unroll
            for (int sr = 0; sr < BS; ++sr) {
              isp[sr] = lane + 64 * sr == p;
              f[sr] = isp[sr] ? 0.0 : a[sr][c] * pinv;
              used[sr] = used[sr] || isp[sr];
            }
            if (c + 1 < BC) {
#pragma unroll
              for (int sr = 0; sr < BS; ++sr) a[sr][c + 1] -= f[sr] * pr[c + 1];
              kmax = col_key(c + 1);
            }
#pragma unroll
            for (int sr = 0; sr < BS; ++sr) {
#pragma unroll
              for (int cc = 0; cc < BC; ++cc)
                if (cc != c + 1) a[sr][cc] -= f[sr] * pr[cc];
              a[sr][c] = isp[sr] ? 1.0 : -f[sr];
            }
            // wave-uniform values: every lane stores the same words (no
            // branch, so the step stays one block for the scheduler)
            S.piv[j0 + c] = p;
            S.pinv[j0 + c] = pinv;
          }
        }
      }
      // publish the transformed panel E(:, I) of the block
#pragma unroll
      for (int sr = 0; sr < BS; ++sr)
#pragma unroll
        for (int cc = 0; cc < BC; ++cc) S.pan[slot][lane + 64 * sr][cc] = a[sr][cc];
      __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();
    if (S.bad) {
      if (tid == 0) atomicExch(fail, 1);
      return;   // uniform
    }
    // the block's pivot rows: used, step and 1 / pivot of this lane's rows
    int tt[BS];
#pragma unroll
    for (int sr = 0; sr < BS; ++sr) tt[sr] = -1;
    for (int t = 0; t < nb; ++t) {
      const int pt = S.piv[j0 + t];
#pragma unroll
      for (int sr = 0; sr < BS; ++sr)
        if (lane + 64 * sr == pt) {
          tt[sr] = t;
          used[sr] = true;
          myq[sr] = j0 + t;
          rinv[sr] = S.pinv[j0 + t];
        }
    }
    // rank-nb update of this wave's columns by the block's row operations
    auto update = [&]() __attribute__((always_inline)) {
      // this wave's columns of the pivot rows, before the update
#pragma unroll
      for (int sr = 0; sr < BS; ++sr)
        if (tt[sr] >= 0) {
#pragma unroll
          for (int cc = 0; cc < BC; ++cc) S.rows[w][tt[sr]][cc] = a[sr][cc];
        }
      __builtin_amdgcn_wave_barrier();
      // software-pipelined over half rows of 8 columns: the LDS reads of the
      // next half (and of the next step's coefficients) are issued before
      // the current half's FMAs, so that one wave running alone does not
      // wait for each read
      constexpr int H = BC / 2;
      auto coef = [&](int t, double (&cf)[BS]) __attribute__((always_inline)) {
#pragma unroll
        for (int sr = 0; sr < BS; ++sr) cf[sr] = S.pan[slot][lane + 64 * sr][t] - (tt[sr] == t ? 1.0 : 0.0);
      };
      double r0[H], r1[H], cf[BS], cfn[BS];
#pragma unroll
      for (int x = 0; x < H; ++x) r0[x] = S.rows[w][0][x];
      coef(0, cf);
      for (int t = 0; t < nb; ++t) {
#pragma unroll
        for (int x = 0; x < H; ++x) r1[x] = S.rows[w][t][H + x];
#pragma unroll
        for (int sr = 0; sr < BS; ++sr)
#pragma unroll
          for (int x = 0; x < H; ++x) a[sr][x] += cf[sr] * r0[x];
        const int tn = min(t + 1, nb - 1);
#pragma unroll
        for (int x = 0; x < H; ++x) r0[x] = S.rows[w][tn][x];
        coef(tn, cfn);
#pragma unroll
        for (int sr = 0; sr < BS; ++sr)
#pragma unroll
          for (int x = 0; x < H; ++x) a[sr][H + x] += cf[sr] * r1[x];
#pragma unroll
        for (int sr = 0; sr < BS; ++sr) cf[sr] = cfn[sr];
      }
      __builtin_amdgcn_wave_barrier();
    };
    // The next panel's columns (wave bj + 1) are updated first, by every
    // wave at once on the matrix cores: wave v forms rows 16 v .. 16 v + 15
    // of (E(:, I) - I(:, I)) A(I, columns of wave bj + 1), a 16 x 16 x nb
    // product (four v_mfma_f64_16x16x4f64), into the other panel slot, which
    // nobody uses until that wave publishes its own panel.  That wave adds
    // the product to its columns and factors its panel at raised priority,
    // while the other waves update their own columns (the panel steps read
    // no LDS).  Waves whose columns all lie beyond T have nothing to update.
    const int nx = bj + 1;
    if (nx < BWV && BC * nx < T) {   // uniform
      if (w == nx) {
#pragma unroll
        for (int sr = 0; sr < BS; ++sr)
          if (tt[sr] >= 0) {
#pragma unroll
            for (int cc = 0; cc < BC; ++cc) S.rows[w][tt[sr]][cc] = a[sr][cc];
          }
      }
      __syncthreads();
      double(*dl)[BC + 1] = S.pan[slot ^ 1];
      const int i16 = lane & 15, k4 = lane >> 4, row = 16 * w + i16;
      double4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        // A(i, t) = coefficient of row 16 w + i for step t; B(t, j) = pivot
        // row of step t in column j of wave nx (zero past the block's nb steps)
        const int t = 4 * kb + k4;
        const bool in = t < nb;
        const double av = in ? S.pan[slot][row][t] - (S.piv[j0 + t] == row ? 1.0 : 0.0) : 0.0;
        const double bv = in ? S.rows[nx][t][i16] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
      }
      // item r of lane l holds row 16 w + l / 16 + 4 r, column l % 16
#pragma unroll
      for (int r = 0; r < 4; ++r) dl[16 * w + k4 + 4 * r][i16] = acc[r];
      __syncthreads();
      if (w == nx) {
        __builtin_amdgcn_s_setprio(3);
#pragma unroll
        for (int sr = 0; sr < BS; ++sr)
#pragma unroll
          for (int cc = 0; cc < BC; ++cc) a[sr][cc] += dl[lane + 64 * sr][cc];
      }
    }
    if (w != bj && w != nx && BC * w < T) update();
  }
#pragma unroll
  for (int sr = 0; sr < BS; ++sr)
#pragma unroll
    for (int c = 0; c < BC; ++c) a[sr][c] *= rinv[sr];
  __syncthreads();   // S.piv complete
  // ---- M^-1(q, piv[col]) = a: route the blocks to G_root or [F*; G], E, D^
  double* up = gen + g.up_off;
  double* E = gen + g.e_off;
  double* Dh = dhat + g.dhat_off;
  const int ld_up = k + n;
#pragma unroll
  for (int sr = 0; sr < BS; ++sr) {
    const int i = myq[sr];
    if (lane + 64 * sr >= T || i < 0) continue;
#pragma unroll
    for (int c = 0; c < BC; ++c) {
      const int col = BC * w + c;
      if (col >= T) continue;
      const int jo = S.piv[col];
      const double v = a[sr][c];
      if (is_root) groot[i + (int64_t)jo * n] = v;
      else if (i < n && jo < n) up[(k + i) + (int64_t)jo * ld_up] = v;
      else if (jo < n) up[(i - n) + (int64_t)jo * ld_up] = v;
      else if (i < n) E[i + (int64_t)(jo - n) * n] = v;
      else Dh[(i - n) + (int64_t)(jo - n) * k] = -v;
    }
  }
}

// grid (nodes), nodes of at most FN unknowns.  Same inputs and outputs as
// node_inverse_kernel: D assembled straight into registers, D^-1 by the
// register Gauss-Jordan, then with W = ws + ws_off holding
// [D^-1 (n x n) | D^-1 U (n x k) | V* D^-1 (k x n) | V* D^-1 U (k x k)]:
// D^ = (V* D^-1 U)^-1, E = D^-1 U D^, F* = D^ V* D^-1, G = D^-1 - E V* D^-1.
__global__ __launch_bounds__(256) void node_factor_kernel(const GNode* __restrict__ gn, const GNode* __restrict__ gch,
                                                          int is_leaf, int is_root, const int* __restrict__ candr,
                                                          const int* __restrict__ candc,
                                                          const NodeRec* __restrict__ nd, const double* __restrict__ U,
                                                          const double* __restrict__ V,
                                                          const double* __restrict__ dhat_ch, double* __restrict__ dhat,
                                                          double* __restrict__ ws, double* __restrict__ gen,
                                                          double* __restrict__ groot, int* __restrict__ fail,
                                                          int mlo, int mhi) {
  __shared__ GjScratch gs;
  __shared__ Gj64Scratch g64;
  __shared__ GemmScratch ms;
  const GNode g = gn[blockIdx.x];
  if (g.m <= mlo || g.m > mhi) return;   // node handled by another launch
  if (g.m + (is_root ? 0 : g.k) <= BT) return;   // taken by the bordered factorization
  const int n = g.m, k = g.k, tid = threadIdx.x, r = tid & (FN - 1);
  const int h = __builtin_amdgcn_readfirstlane(tid >> 7);
  const int* cr = candr + g.cand_off;
  const int* cc = candc + g.cand_off;
  // ---- assemble D (column-major, in the workspace slot of D^-1), then
  // each thread takes its row segment into registers
  double* Dw = ws + g.ws_off;
  if (is_leaf) {
    for (int idx = tid; idx < n * n; idx += 256) {
      const int i = idx % n, j = idx / n;
      const int ra = cr[i], cb = cc[j];
      Dw[idx] = a_entry(nd[ra >> 1], nd[cb >> 1], (ra >> 1) == (cb >> 1), ra & 1, cb & 1);
    }
  } else {
    const GNode ca = gch[2 * blockIdx.x], cbn = gch[2 * blockIdx.x + 1];
    const int ka = ca.k, kb = cbn.k;
    const double* Da = dhat_ch + ca.dhat_off;
    const double* Db = dhat_ch + cbn.dhat_off;
    for (int idx = tid; idx < n * n; idx += 256) {
      const int i = idx % n, j = idx / n;
      double v;
      if (i < ka && j < ka) v = Da[i + j * ka];
      else if (i >= ka && j >= ka) v = Db[(i - ka) + (j - ka) * kb];
      else {
        const int ra = cr[i], cb = cc[j];
        v = a_entry(nd[ra >> 1], nd[cb >> 1], false, ra & 1, cb & 1);
      }
      Dw[idx] = v;
    }
  }
  __syncthreads();
  double* Dinv = is_root ? groot : ws + g.ws_off;  // Dinv == Dw except at the root
  int q, rot;
  // split of the 2 x 2 block inverse: the children's skeletons for a parent
  const int n1 = is_leaf ? (n + 1) / 2 : gch[2 * blockIdx.x].k, n2 = n - n1;
  if (n <= GN) {
    double a16[16];
    gj64_load(Dw, n, n, a16);
    if (!reg_gj64(a16, n, g64, q, rot)) {
      if (tid == 0) atomicExch(fail, 1);
      return;
    }
    gj64_store(a16, n, q, rot, g64.piv, Dinv, n);
  } else if (n1 > 0 && n2 > 0 && n1 <= GN && n2 <= GN) {
    // D = [[A, B], [C, E]]: A^-1 and the Schur complement E - C A^-1 B
    // inverted in registers, the rest by workgroup GEMMs
    double* Ai = ws + g.ws_off + (int64_t)n * n;  // n1 x n1
    double* Xb = Ai + (int64_t)n1 * n1;            // n1 x n2: A^-1 B
    double* Yb = Xb + (int64_t)n1 * n2;            // n2 x n1: C A^-1
    double* Si = Yb + (int64_t)n2 * n1;            // n2 x n2: (E - C A^-1 B)^-1
    double* Tb = Si + (int64_t)n2 * n2;            // n1 x n2: A^-1 B Si
    const double* Bb = Dw + (int64_t)n1 * n;
    const double* Cb = Dw + n1;
    const double* Eb = Dw + n1 + (int64_t)n1 * n;
    {
      double a16[16];
      gj64_load(Dw, n, n1, a16);
      if (!reg_gj64(a16, n1, g64, q, rot)) {
        if (tid == 0) atomicExch(fail, 1);
        return;
      }
      gj64_store(a16, n1, q, rot, g64.piv, Ai, n1);
    }
    __syncthreads();
    wg_gemm_small(false, false, n1, n2, n1, 1.0, Ai, n1, Bb, n, nullptr, 0, Xb, n1, ms);
    wg_gemm_small(false, false, n2, n1, n1, 1.0, Cb, n, Ai, n1, nullptr, 0, Yb, n2, ms);
    wg_gemm_small(false, false, n2, n2, n1, -1.0, Cb, n, Xb, n1, Eb, n, Si, n2, ms);
    {
      double a16[16];
      gj64_load(Si, n2, n2, a16);
      if (!reg_gj64(a16, n2, g64, q, rot)) {
        if (tid == 0) atomicExch(fail, 1);
        return;
      }
      gj64_store(a16, n2, q, rot, g64.piv, Si, n2);
    }
    __syncthreads();
    // D^-1 = [[A^-1 + T Y, -T], [-Si Y, Si]], T = X Si (the blocks of D are
    // no longer read, so D^-1 may overwrite them)
    wg_gemm_small(false, false, n1, n2, n2, 1.0, Xb, n1, Si, n2, nullptr, 0, Tb, n1, ms);
    wg_gemm_small(false, false, n1, n1, n2, 1.0, Tb, n1, Yb, n2, Ai, n1, Dinv, n, ms);
    wg_gemm_small(false, false, n2, n1, n2, -1.0, Si, n2, Yb, n2, nullptr, 0, Dinv + n1, n, ms);
    for (int idx = tid; idx < n1 * n2; idx += 256) {
      const int i = idx % n1, jj = idx / n1;
      Dinv[i + (int64_t)(n1 + jj) * n] = -Tb[i + (int64_t)jj * n1];
    }
    for (int idx = tid; idx < n2 * n2; idx += 256) {
      const int i = idx % n2, jj = idx / n2;
      Dinv[n1 + i + (int64_t)(n1 + jj) * n] = Si[i + (int64_t)jj * n2];
    }
  } else {
    double a[64];
#pragma unroll
    for (int c = 0; c < 64; ++c) {
      const int col = 64 * h + c;
      a[c] = (r < n && col < n) ? Dw[r + (int64_t)col * n] : 0.0;
    }
    if (!reg_gauss_jordan(a, n, gs, q, rot)) {
      if (tid == 0) atomicExch(fail, 1);
      return;
    }
    if (r < n) {
#pragma unroll
      for (int c = 0; c < 64; ++c) {
        const int col = 64 * h + ((c + rot) & 63);
        if (col < n) Dinv[q + (int64_t)gs.piv[col] * n] = a[c];
      }
    }
  }
  __syncthreads();
  if (is_root) return;
  double* DU = Dinv + (int64_t)n * n;
  double* VD = DU + (int64_t)n * k;
  double* Sm = VD + (int64_t)k * n;
  const double* Un = U + g.uv_off;
  const double* Vn = V + g.uv_off;
  // op 0: D^-1 U;  op 1: V* D^-1;  op 2: V* D^-1 U  (one call site keeps the code small)
  for (int op = 0; op < 3; ++op) {
    const int mo = op == 0 ? n : k, no = op == 1 ? n : k;
    const double* A = op == 0 ? Dinv : (op == 1 ? Vn : VD);
    const double* B = op == 1 ? Dinv : Un;
    double* C = op == 0 ? DU : (op == 1 ? VD : Sm);
    wg_gemm_small(op == 1, false, mo, no, n, 1.0, A, op == 2 ? k : n, B, n, nullptr, 0, C, op == 0 ? n : k, ms);
  }
  // D^ = (V* D^-1 U)^-1, through the registers again
  double* Dh = dhat + g.dhat_off;
  if (k <= GN) {
    double a16[16];
    gj64_load(Sm, k, k, a16);
    if (!reg_gj64(a16, k, g64, q, rot)) {
      if (tid == 0) atomicExch(fail, 2);
      return;
    }
    gj64_store(a16, k, q, rot, g64.piv, Dh, k);
  } else {
    double a[64];
#pragma unroll
    for (int c = 0; c < 64; ++c) {
      const int col = 64 * h + c;
      a[c] = (r < k && col < k) ? Sm[r + (int64_t)col * k] : 0.0;
    }
    if (!reg_gauss_jordan(a, k, gs, q, rot)) {
      if (tid == 0) atomicExch(fail, 2);
      return;
    }
    if (r < k) {
#pragma unroll
      for (int c = 0; c < 64; ++c) {
        const int col = 64 * h + ((c + rot) & 63);
        if (col < k) Dh[q + (int64_t)gs.piv[col] * k] = a[c];
      }
    }
  }
  __syncthreads();
  double* up = gen + g.up_off;  // [F*; G], (k + n) x n
  double* E = gen + g.e_off;    // n x k
  const int rows = k + n;
  // op 0: E = D^-1 U D^;  op 1: F* = D^ V* D^-1;  op 2: G = D^-1 - E V* D^-1
  for (int op = 0; op < 3; ++op) {
    const int mo = op == 1 ? k : n, no = op == 0 ? k : n;
    const double* A = op == 0 ? DU : (op == 1 ? Dh : E);
    const double* B = op == 0 ? Dh : VD;
    double* C = op == 0 ? E : (op == 1 ? up : up + k);
    wg_gemm_small(false, false, mo, no, k, op == 2 ? -1.0 : 1.0, A, op == 1 ? k : n, B, k, op == 2 ? Dinv : nullptr,
                  n, C, op == 0 ? n : rows, ms);
  }
}

// grid (nodes).  leaf: D = A(candr, candc); parent: children's D^ on the
// diagonal, kernel blocks between the children's skeletons off it.
// root (is_root): writes D^-1 to G_root only.
__global__ __launch_bounds__(256) void node_inverse_kernel(const GNode* __restrict__ gn, const GNode* __restrict__ gch,
                                                           int is_leaf, int is_root, const int* __restrict__ candr,
                                                           const int* __restrict__ candc,
                                                           const NodeRec* __restrict__ nd, const double* __restrict__ U,
                                                           const double* __restrict__ V,
                                                           const double* __restrict__ dhat_ch, double* __restrict__ dhat,
                                                           double* __restrict__ ws, double* __restrict__ gen,
                                                           double* __restrict__ groot, int* __restrict__ fail,
                                                           int mlo, int mhi) {
  __shared__ double rv[4];
  __shared__ int ri[4];
  __shared__ int perm[256];
  __shared__ double fsc[256];
  extern __shared__ double sA[];       // n x n when the node fits in LDS, then k x k
  const GNode g = gn[blockIdx.x];
  if (g.m <= mlo || g.m > mhi) return;   // node handled by another launch
  if (g.m + (is_root ? 0 : g.k) <= BT) return;   // taken by the bordered factorization
  const int n = g.m, k = g.k, tid = threadIdx.x;
  const int* cr = candr + g.cand_off;
  const int* cc = candc + g.cand_off;
  const bool in_lds = n <= INV_LDS_N;
  double* Dm = in_lds ? sA : ws + g.ws_off;   // n x n; becomes D^-1 in place
  double* Inv = Dm;
  // assemble D
  if (is_leaf) {
    for (int idx = tid; idx < n * n; idx += 256) {
      const int i = idx % n, j = idx / n;
      const int ra = cr[i], cb = cc[j];
      double B[4];
      a_blk(nd[ra >> 1], nd[cb >> 1], (ra >> 1) == (cb >> 1), B);
      Dm[idx] = B[(ra & 1) * 2 + (cb & 1)];
    }
  } else {
    const GNode ca = gch[2 * blockIdx.x], cbn = gch[2 * blockIdx.x + 1];
    const int ka = ca.k, kb = cbn.k;
    const double* Da = dhat_ch + ca.dhat_off;
    const double* Db = dhat_ch + cbn.dhat_off;
    for (int idx = tid; idx < n * n; idx += 256) {
      const int i = idx % n, j = idx / n;
      double v;
      if (i < ka && j < ka) v = Da[i + j * ka];
      else if (i >= ka && j >= ka) v = Db[(i - ka) + (j - ka) * kb];
      else {
        const int ra = cr[i], cb = cc[j];
        double B[4];
        a_blk(nd[ra >> 1], nd[cb >> 1], false, B);
        v = B[(ra & 1) * 2 + (cb & 1)];
      }
      Dm[idx] = v;
    }
  }
  __syncthreads();
  if (!wg_inverse_inplace(Dm, n, perm, fsc, rv, ri)) {
    if (tid == 0) atomicExch(fail, 1);
    return;
  }
  if (is_root) {
    for (int idx = tid; idx < n * n; idx += 256) groot[idx] = Inv[idx];
    return;
  }
  const double* Un = U + g.uv_off;
  const double* Vn = V + g.uv_off;
  double* DinvU = ws + g.ws_off + (int64_t)n * n;  // n x k (after the global D slot)
  double* VtDinv = DinvU + (int64_t)n * k;     // k x n
  double* Sm = VtDinv + (int64_t)k * n;        // k x k
  // the k x k inverse goes to LDS behind D^-1 when both fit
  double* Si = (in_lds && (n * n + k * k) * 8 <= INV_LDS_BYTES) ? sA + n * n : Sm + (int64_t)k * k;
  wg_gemm(false, false, n, k, n, 1.0, Inv, n, Un, n, 0.0, DinvU, n);
  wg_gemm(true, false, k, n, n, 1.0, Vn, n, Inv, n, 0.0, VtDinv, k);
  wg_gemm(false, false, k, k, n, 1.0, VtDinv, k, Un, n, 0.0, Sm, k);
  for (int idx = tid; idx < k * k; idx += 256) Si[idx] = Sm[idx];
  __syncthreads();
  if (!wg_inverse_inplace(Si, k, perm, fsc, rv, ri)) {
    if (tid == 0) atomicExch(fail, 2);
    return;
  }
  double* up = gen + g.up_off;                 // (k + n) x n
  double* E = gen + g.e_off;                   // n x k
  const int rows = k + n;
  wg_gemm(false, false, n, k, k, 1.0, DinvU, n, Si, k, 0.0, E, n);
  wg_gemm(false, false, k, n, k, 1.0, Si, k, VtDinv, k, 0.0, up, rows);     // F* into rows 0..k-1
  for (int idx = tid; idx < n * n; idx += 256) {
    const int i = idx % n, j = idx / n;
    up[k + i + (int64_t)j * rows] = Inv[idx];
  }
  __syncthreads();
  wg_gemm(false, false, n, n, k, -1.0, E, n, VtDinv, k, 1.0, up + k, rows); // G = Inv - E V* D^-1
  for (int idx = tid; idx < k * k; idx += 256) dhat[g.dhat_off + idx] = Si[idx];
}

}  // namespace

// ================================================================== upload / apply
void hbs_upload(rw_ctx* ctx, const HbsInverse& H, int prec, HbsDev& w) {
  const bool with_f32 = prec == 1, with_bf16 = prec == 2;
  hipStream_t s = ctx->stream;
  w.ctx = ctx;
  w.L = H.L;
  w.nroot = H.nroot;
  w.lev.assign(w.L + 1, HbsLevelDev());
  w.S.assign(w.L + 2, 0);
  w.K.assign(w.L + 2, 0);
  std::vector<int> ints;
  std::vector<int64_t> offs;
  std::vector<double> gen;
  std::vector<size_t> int_base(w.L + 1), off_base(w.L + 1);
  for (int l = 1; l <= w.L; ++l) {
    const auto& nodes = H.lev[l];
    const int nn = (int)nodes.size();
    int_base[l] = ints.size();
    off_base[l] = offs.size();
    for (int j = 0; j < nn; ++j) ints.push_back(nodes[j].nin);
    for (int j = 0; j < nn; ++j) ints.push_back(nodes[j].k);
    int64_t in_off = 0, k_off = 0;
    std::vector<int64_t> io(nn), ko(nn), uo(nn), eo(nn);
    int max_nin = 0, max_k = 0;
    for (int j = 0; j < nn; ++j) {
      const HbsNodeGen& g = nodes[j];
      io[j] = in_off;
      ko[j] = k_off;
      in_off += g.nin;
      k_off += g.k;
      max_nin = std::max(max_nin, g.nin);
      max_k = std::max(max_k, g.k);
      uo[j] = (int64_t)gen.size();
      const int rows = g.k + g.nin;
      gen.resize(gen.size() + (size_t)rows * g.nin);
      double* up = gen.data() + uo[j];
      for (int c = 0; c < g.nin; ++c) {
        for (int r = 0; r < g.k; ++r) up[r + (size_t)c * rows] = g.Ft[r + (size_t)c * g.k];
        for (int r = 0; r < g.nin; ++r) up[g.k + r + (size_t)c * rows] = g.G[r + (size_t)c * g.nin];
      }
      eo[j] = (int64_t)gen.size();
      gen.insert(gen.end(), g.E.begin(), g.E.end());
    }
    offs.insert(offs.end(), io.begin(), io.end());
    offs.insert(offs.end(), ko.begin(), ko.end());
    offs.insert(offs.end(), uo.begin(), uo.end());
    offs.insert(offs.end(), eo.begin(), eo.end());
    HbsLevelDev& d = w.lev[l];
    d.nnodes = nn;
    d.max_nin = max_nin;
    d.max_k = max_k;
    d.S = in_off;
    d.K = k_off;
    for (int j = 0; j < nn; ++j) {
      d.up_entries += (int64_t)(nodes[j].k + nodes[j].nin) * nodes[j].nin;
      d.e_entries += (int64_t)nodes[j].nin * nodes[j].k;
    }
    w.S[l] = in_off;
    w.K[l] = k_off;
  }
  w.S[0] = w.nroot;
  w.d_ints.alloc(ctx, ints.size());
  w.d_ints.upload(ints.data(), ints.size(), s);
  w.d_offs.alloc(ctx, offs.size());
  w.d_offs.upload(offs.data(), offs.size(), s);
  w.gen.alloc(ctx, gen.size());
  w.gen.upload(gen.data(), gen.size(), s);
  if (with_f32) {
    std::vector<float> g32(gen.begin(), gen.end());
    w.gen32.alloc(ctx, g32.size());
    w.gen32.upload(g32.data(), g32.size(), s);
    HIP_CHECK(hipStreamSynchronize(s));
  }
  if (with_bf16) {
    // FP64 -> FP32 -> BF16, round to nearest even at each step
    std::vector<uint16_t> g16(gen.size());
    for (size_t i = 0; i < gen.size(); ++i) {
      const float f = (float)gen[i];
      uint32_t u;
      memcpy(&u, &f, 4);
      u += 0x7fffu + ((u >> 16) & 1u);
      g16[i] = (uint16_t)(u >> 16);
    }
    w.gen16.alloc(ctx, g16.size());
    w.gen16.upload(g16.data(), g16.size(), s);
    HIP_CHECK(hipStreamSynchronize(s));
  }
  w.groot.alloc(ctx, H.Groot.size());
  w.groot.upload(H.Groot.data(), H.Groot.size(), s);
  for (int l = 1; l <= w.L; ++l) {
    HbsLevelDev& d = w.lev[l];
    const int nn = d.nnodes;
    d.nin = w.d_ints.p + int_base[l];
    d.k = w.d_ints.p + int_base[l] + nn;
    d.in_off = w.d_offs.p + off_base[l];
    d.kout_off = w.d_offs.p + off_base[l] + nn;
    d.up_off = w.d_offs.p + off_base[l] + 2 * nn;
    d.e_off = w.d_offs.p + off_base[l] + 3 * nn;
  }
  HIP_CHECK(hipStreamSynchronize(s));
  w.entries = H.entries;
  w.max_rank = H.max_rank;
}

static void hbs_ensure_ws(const HbsDev& w, HbsWork& wk, int nrhs) {
  int64_t tot = 0;
  for (int l = 1; l <= w.L; ++l) tot += w.K[l] + w.S[l];
  for (int l = 0; l < w.L; ++l) tot += w.S[l];
  if (nrhs <= wk.ws_nrhs && tot == wk.ws_per_rhs && (int)wk.U.size() == w.L + 1) return;
  wk.ws.alloc(wk.ctx, (size_t)tot * nrhs);
  wk.ws_per_rhs = tot;
  wk.U.assign(w.L + 1, nullptr);
  wk.GB.assign(w.L + 1, nullptr);
  wk.X.assign(w.L + 1, nullptr);
  double* p = wk.ws.p;
  for (int l = 1; l <= w.L; ++l) { wk.U[l] = p; p += w.K[l] * nrhs; wk.GB[l] = p; p += w.S[l] * nrhs; }
  for (int l = 0; l < w.L; ++l) { wk.X[l] = p; p += w.S[l] * nrhs; }
  wk.ws_nrhs = nrhs;
}

int64_t hbs_ws1_plan(const HbsDev& w, double* base, HbsWs1& ws) {
  const int L = w.L;
  if (L > HBS_MAX_LEVELS) RW_THROW(RW_EINVAL, "HBS tree deeper than the one-RHS plan supports");
  for (int l = 0; l <= L + 1; ++l) ws.nsu[l] = 1;
  for (int l = 0; l <= L; ++l) ws.nsd[l] = 1;
  for (int l = 1; l <= L; ++l) {
    ws.nsu[l] = hbs_split_count(w.lev[l].max_nin);
    ws.nsd[l] = hbs_split_count(w.lev[l].max_k);
  }
  ws.nsr = hbs_split_count(w.nroot);
  int64_t off = 0;
  auto take = [&](int64_t n) {
    double* q = base ? base + off : nullptr;
    off += n;
    return q;
  };
  ws.X1[0] = take((int64_t)ws.nsr * w.S[0]);
  for (int l = 1; l <= L; ++l) {
    ws.U1[l] = take((int64_t)ws.nsu[l] * w.K[l]);
    ws.GB1[l] = take((int64_t)ws.nsu[l] * w.S[l]);
    ws.X1[l] = take((int64_t)ws.nsd[l] * w.S[l]);
  }
  return off;
}

// One right-hand side: level sweeps of split products whose partial vectors
// are summed by the next kernel (see kern_hbs.hip).  Every partial vector is
// written before it is read, so `base` needs no clearing.
void hbs_dev_apply1_at(const HbsDev& w, const double* b, double* x, int prec, double* base, hipStream_t s) {
  HbsWs1 ws;
  hbs_ws1_plan(w, base, ws);
  const int L = w.L;
  const float* g32 = prec == 1 ? w.gen32.p : nullptr;
  const uint16_t* g16 = prec == 2 ? w.gen16.p : nullptr;
  for (int l = L; l >= 1; --l) {
    const bool leaf = l == L;
    launch_hbs_up1(w.lev[l], w.gen.p, g32, leaf ? b : ws.U1[l + 1], leaf ? 0 : w.K[l + 1], leaf ? 1 : ws.nsu[l + 1],
                   ws.U1[l], w.K[l], ws.GB1[l], w.S[l], s, g16);
  }
  launch_hbs_root1(w.nroot, w.d_nroot, w.groot.p, ws.U1[1], w.K[1], ws.nsu[1], ws.X1[0], w.S[0], s);
  for (int l = 1; l <= L; ++l) {
    const int xnp = l == 1 ? ws.nsr : ws.nsd[l - 1];
    const bool direct = l == L && ws.nsd[L] == 1;
    launch_hbs_down1(w.lev[l], w.gen.p, g32, ws.X1[l - 1], w.S[l - 1], xnp, ws.GB1[l], w.S[l], ws.nsu[l],
                     direct ? x : ws.X1[l], w.S[l], s, g16);
  }
  if (ws.nsd[L] > 1) launch_parts_reduce(ws.X1[L], w.S[L], ws.nsd[L], w.S[L], x, s);
}

void hbs_dev_apply_ws(const HbsDev& w, HbsWork& wk, const double* b, int64_t ldb, double* x, int64_t ldx, int nrhs,
                      int prec, hipStream_t s, int mfma_from) {
  if (nrhs <= 0) return;
  if (!wk.ctx) wk.ctx = w.ctx;
  if ((prec == 1 && !w.gen32.p) || (prec == 2 && !w.gen16.p)) prec = 0;
  if (nrhs == 1) {
    HbsWs1 ws;
    const int64_t need = std::max<int64_t>(1, hbs_ws1_plan(w, nullptr, ws));
    if (!wk.ws1.p || wk.ws1_need != need) {
      wk.ws1.alloc(wk.ctx, (size_t)need);
      wk.ws1_need = need;
    }
    hbs_dev_apply1_at(w, b, x, prec, wk.ws1.p, s);
    return;
  }
  hbs_ensure_ws(w, wk, nrhs);
  const bool f32 = prec == 1, b16 = prec == 2;
  const int from64 = mfma_from > 0 ? mfma_from : w.mfma_from64, from32 = mfma_from > 0 ? mfma_from : w.mfma_from32,
            from16 = mfma_from > 0 ? mfma_from : w.mfma_from16;
  for (int l = w.L; l >= 1; --l) {
    const double* in = (l == w.L) ? b : wk.U[l + 1];
    const int64_t ldin = (l == w.L) ? ldb : w.K[l + 1];
    if (b16)
      launch_hbs_up_bf16(w.lev[l], w.gen16.p, in, ldin, wk.U[l], w.K[l], wk.GB[l], w.S[l], nrhs, s, from16);
    else if (f32)
      launch_hbs_up_f32(w.lev[l], w.gen32.p, in, ldin, wk.U[l], w.K[l], wk.GB[l], w.S[l], nrhs, s, from32);
    else
      launch_hbs_up(w.lev[l], w.gen.p, in, ldin, wk.U[l], w.K[l], wk.GB[l], w.S[l], nrhs, s, from64);
  }
  launch_hbs_root(w.nroot, w.d_nroot, w.groot.p, wk.U[1], w.K[1], wk.X[0], w.S[0], nrhs, s, from64);
  for (int l = 1; l <= w.L; ++l) {
    double* out = (l == w.L) ? x : wk.X[l];
    const int64_t ldout = (l == w.L) ? ldx : w.S[l];
    if (b16)
      launch_hbs_down_bf16(w.lev[l], w.gen16.p, wk.X[l - 1], w.S[l - 1], wk.GB[l], w.S[l], out, ldout, nrhs, s,
                           from16);
    else if (f32)
      launch_hbs_down_f32(w.lev[l], w.gen32.p, wk.X[l - 1], w.S[l - 1], wk.GB[l], w.S[l], out, ldout, nrhs, s,
                          from32);
    else
      launch_hbs_down(w.lev[l], w.gen.p, wk.X[l - 1], w.S[l - 1], wk.GB[l], w.S[l], out, ldout, nrhs, s, from64);
  }
}

void hbs_autotune(HbsDev& w, hipStream_t s) {
  const int64_t n = w.n_unknowns();
  if (n <= 0) return;
  constexpr int kCand[] = {16, 24, 32, 40, 48, 56, 64};
  constexpr int kMax = 64, kNever = 1 << 30;
  DBuf<double> b(w.ctx, (size_t)n * kMax), x(w.ctx, (size_t)n * kMax);
  HIP_CHECK(hipMemsetAsync(b.p, 0, sizeof(double) * n * kMax, s));
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  auto thr_of = [&](int prec) -> int& { return prec == 2 ? w.mfma_from16 : (prec == 1 ? w.mfma_from32 : w.mfma_from64); };
  auto timed = [&](int nrhs, int prec, int from) {
    int& thr = thr_of(prec);
    const int keep = thr;
    thr = from;
    hbs_dev_apply(w, b.p, n, x.p, n, nrhs, prec, s);   // warm-up (and workspace)
    HIP_CHECK(hipEventRecord(e0, s));
    for (int r = 0; r < 3; ++r) hbs_dev_apply(w, b.p, n, x.p, n, nrhs, prec, s);
    HIP_CHECK(hipEventRecord(e1, s));
    HIP_CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    thr = keep;
    return ms;
  };
  for (int prec = 0; prec < 3; ++prec) {
    if ((prec == 1 && !w.gen32.p) || (prec == 2 && !w.gen16.p)) continue;
    int from = kNever;
    for (int i = (int)(sizeof kCand / sizeof kCand[0]) - 1; i >= 0; --i) {
      const int c = kCand[i];
      if (timed(c, prec, 1) < timed(c, prec, kNever)) from = c;
      else break;
    }
    thr_of(prec) = from;
  }
  HIP_CHECK(hipEventDestroy(e0));
  HIP_CHECK(hipEventDestroy(e1));
}

void hbs_dev_apply(HbsDev& w, const double* b, int64_t ldb, double* x, int64_t ldx, int nrhs, int prec,
                   hipStream_t s) {
  hbs_dev_apply_ws(w, w.work, b, ldb, x, ldx, nrhs, prec, s);
}

void hbs_gpu_finish(HbsDev& w) {
  if (!w.fin.pending) return;
  w.fin.pending = false;
  const GNode* hG = (const GNode*)w.fin.rec;
  int hf[4];
  memcpy(hf, w.fin.ctl, sizeof hf);
  if (hf[1]) RW_THROW(RW_ESINGULAR, "HBS node rank reached the sketch size");
  if (hf[2]) RW_THROW(RW_ESINGULAR, "HBS generator bound exceeded");
  if (hf[0]) RW_THROW(RW_ESINGULAR, "singular block in the GPU HBS build (" + std::to_string(hf[0]) + ")");
  rw_ctx* ctx = w.ctx;
  w.entries = 0;
  w.max_rank = 0;
  for (int l = w.L; l >= 1; --l) {
    const int nn = 1 << l;
    const GNode* gl = hG + nn;
    HbsLevelDev& d = w.lev[l];
    d.up_entries = d.e_entries = 0;
    double fl = 0.0, by = 0.0;
    for (int j = 0; j < nn; ++j) {
      const GNode& g = gl[j];
      d.up_entries += (int64_t)(g.k + g.m) * g.m;
      d.e_entries += (int64_t)g.m * g.k;
      w.entries += 2 * (int64_t)g.m * g.k + (int64_t)g.m * g.m;
      w.max_rank = std::max(w.max_rank, g.k);
      // flops and bytes credited to the bordered kernel: only the nodes it
      // factors (larger ones go to the block-inverse kernels).  Bytes: the
      // (m + k)^2 generator entries written, U and V read, the children's
      // D^ read, one node record (64 B) and two candidate indices per row
      const double nm = g.m, kk2 = g.k;
      if (g.m + g.k <= BT) {
        fl += 2.0 * nm * nm * nm + 2.0 * (3.0 * nm * nm * kk2 + 3.0 * nm * kk2 * kk2) + 2.0 * kk2 * kk2 * kk2;
        double ch = 0.0;
        if (l < w.L) {
          const GNode* gc = hG + 2 * nn;
          ch = (double)gc[2 * j].k * gc[2 * j].k + (double)gc[2 * j + 1].k * gc[2 * j + 1].k;
        }
        by += 8.0 * (nm + kk2) * (nm + kk2) + 16.0 * nm * kk2 + 8.0 * ch + 72.0 * nm;
      }
    }
    const size_t fe = w.fin.fac_entry[l];
    if (fe != SIZE_MAX && fe < ctx->pending.size()) {
      ctx->pending[fe].flops = fl;
      ctx->pending[fe].bytes = by;
    }
  }
  const double nr = hG[1].m;
  w.entries += (int64_t)(nr * nr);
  const size_t fe = w.fin.fac_entry[0];
  if (fe != SIZE_MAX && fe < ctx->pending.size()) {
    const double ka = hG[2].k, kb = hG[3].k;
    ctx->pending[fe].flops = 2.0 * nr * nr * nr;
    ctx->pending[fe].bytes = 8.0 * nr * nr + 8.0 * (ka * ka + kb * kb) + 72.0 * nr;
  }
}

// ================================================================== GPU build
void hbs_gpu_build(rw_ctx* ctx, const NodeRec* d_nodes, int64_t n_nodes, int leaf_max, double tol, uint64_t seed,
                   HbsDev& w) {
  hipStream_t s = ctx->stream;
  const int64_t N = n_nodes;
  if (N < 2) RW_THROW(RW_EINVAL, "HBS build needs at least two nodes");
  int L = 1;
  while ((N >> L) > leaf_max) ++L;
  if (2 * ((N + (int64_t(1) << L) - 1) >> L) > 2 * leaf_max + 2) RW_THROW(RW_EINVAL, "leaf size");
  // ---- level plans (ranges, proxy circles)
  std::vector<std::vector<GNode>> G(L + 1);
  for (int l = 0; l <= L; ++l) {
    const int64_t nn = int64_t(1) << l;
    G[l].resize(nn);
    for (int64_t j = 0; j < nn; ++j) {
      GNode& g = G[l][j];
      memset(&g, 0, sizeof g);
      g.n0 = (j * N) >> l;
      g.n1 = ((j + 1) * N) >> l;
      if (l == L) g.m = (int)(2 * (g.n1 - g.n0));
    }
  }
  // ---- buffers sized by the bounds m <= max(2 leaf_max, 2 SK_KCAP), k <= SK_KCAP.
  // The node factorizations of level l run on the side stream while the
  // main stream goes on with the sketches and IDs of level l - 1, so every
  // buffer that a factorization reads (node records, candidate lists, U, V)
  // has a region per level; the sketch and ID buffers serve one level at a
  // time on the main stream.
  const int mmax = std::max(2 * leaf_max + 2, 2 * SK_KCAP);
  std::vector<int64_t> cand_base(L + 1), uv_base(L + 1, 0);
  int64_t cand_total = 0, uv_total = 0, cap_max = 0, gen_bound = 0, ws_bound = 0;
  for (int l = 0; l <= L; ++l) {
    const int64_t nn = int64_t(1) << l;
    const int64_t mb = (l == L) ? 2 * ((N + nn - 1) / nn) : 2 * SK_KCAP;
    cand_base[l] = cand_total;
    cand_total += nn * mb;
    if (l == 0) continue;
    uv_base[l] = uv_total;
    uv_total += nn * mb * SK_KCAP;
    cap_max = std::max(cap_max, nn * mb);
    gen_bound += nn * ((SK_KCAP + mb) * mb + mb * SK_KCAP);
    ws_bound = std::max(ws_bound, nn * (3 * mb * mb + 2 * mb * SK_KCAP + 2 * SK_KCAP * SK_KCAP));
  }
  ws_bound = std::max<int64_t>(ws_bound, 3 * (int64_t)mmax * mmax);
  DBuf<GNode> dg(ctx, (size_t)(int64_t(2) << L));   // level l at [2^l, 2^(l+1))
  DBuf<int> candr(ctx, cand_total), candc(ctx, cand_total);
  DBuf<double> Sr(ctx, cap_max * SK_R), Sc(ctx, cap_max * SK_R);
  DBuf<double> Cr(ctx, cap_max * SK_KCAP), Cc(ctx, cap_max * SK_KCAP);
  DBuf<int> piv(ctx, (size_t)(int64_t(2) << L) * SK_KCAP), info(ctx, (size_t)(int64_t(4) << L));
  // control words, cleared together: fail flags (4 ints), generator / spare
  // counters (2), the ID sides' published ranks (2 per node of a level), the
  // finished ID workgroups of each level (L + 1)
  DBuf<int64_t> ctl(ctx, (size_t)(4 + (int64_t(2) << L) + L + 1));
  int* const failp = (int*)ctl.p;
  int64_t* const cntp = ctl.p + 2;
  long long* const pubp = (long long*)(ctl.p + 4);
  unsigned long long* const donep = (unsigned long long*)(ctl.p + 4 + (int64_t(2) << L));
  DBuf<double> Ub(ctx, uv_total), Vb(ctx, uv_total);
  DBuf<double> dhA(ctx, (int64_t(1) << L) * SK_KCAP * SK_KCAP), dhB(ctx, (int64_t(1) << L) * SK_KCAP * SK_KCAP);
  DBuf<double> ws(ctx, ws_bound);
  DBuf<int64_t> dpar(ctx, (size_t)(int64_t(2) << L));  // level l at [2^l, 2^(l+1))
  // sketch partial sums: the largest (candidates x split count) of any level.
  // About 384 workgroups per level (1.5 per compute unit): all of them
  // resident beside the concurrent row-ID and factor kernels, each with
  // several chunks to spread its fixed cost (candidate records, near-node
  // scan, partial rows) over
  auto level_split = [&](int64_t nn) {
    int ns = (int)std::min<int64_t>(64, std::max<int64_t>(1, 384 / (2 * nn)));
    return (int)std::min<int64_t>(ns, std::max<int64_t>(1, N / 64));
  };
  int64_t part_len = 0;
  for (int l = 1; l <= L; ++l) {
    const int64_t nn = int64_t(1) << l;
    const int64_t mb = (l == L) ? 2 * ((N + nn - 1) / nn) : 2 * SK_KCAP;
    part_len = std::max(part_len, nn * mb * SK_R * level_split(nn));
  }
  DBuf<double> part_r(ctx, part_len), part_c(ctx, part_len);
  w.gen.alloc(ctx, gen_bound);
  w.groot.alloc(ctx, (size_t)(2 * SK_KCAP) * (2 * SK_KCAP));
  HIP_CHECK(hipMemsetAsync(ctl.p, 0, sizeof(int64_t) * ctl.n, s));
  // pinned staging: node records (level l at [2^l, 2^(l+1))) and the leaf candidate lists
  char* pin = (char*)ctx_hbs_pinned(ctx, sizeof(GNode) * (size_t)(int64_t(2) << L) + sizeof(int64_t) * 4 +
                                          sizeof(int) * (size_t)(2 * N));
  GNode* hG = (GNode*)pin;
  int64_t* hCtl = (int64_t*)(pin + sizeof(GNode) * (size_t)(int64_t(2) << L));
  int* hC = (int*)(hCtl + 4);
  // leaf records carry their counts and offsets; a parent's are set on the
  // device from its children's ranks (level_plan_wave)
  {
    int64_t off = 0;
    for (GNode& g : G[L]) { g.cand_off = off; off += g.m; }
    for (int l = 0; l <= L; ++l) memcpy(hG + (int64_t(1) << l), G[l].data(), sizeof(GNode) * G[l].size());
    memset(hG, 0, sizeof(GNode));
    HIP_CHECK(hipMemcpyAsync(dg.p, hG, sizeof(GNode) * (size_t)(int64_t(2) << L), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(node_geom_kernel, dim3((unsigned)((int64_t(2) << L) - 1)), dim3(256), 0, s, dg.p, d_nodes);
    KERNEL_CHECK("node_geom");
    for (int64_t d = 0; d < 2 * N; ++d) hC[d] = (int)d;
    HIP_CHECK(hipMemcpyAsync(candr.p + cand_base[L], hC, sizeof(int) * 2 * N, hipMemcpyHostToDevice, s));
    HIP_CHECK(hipMemcpyAsync(candc.p + cand_base[L], hC, sizeof(int) * 2 * N, hipMemcpyHostToDevice, s));
  }
  // the factor chain starts after everything enqueued so far; whatever way
  // this function ends, later work on the main stream waits for it
  const hipStream_t sf = ctx_side_stream(ctx);
  stream_after(ctx, sf, s, 0);
  struct SideJoin {
    rw_ctx* c;
    hipStream_t main, side;
    ~SideJoin() {
      if (main == side) return;
      hipEvent_t e = nullptr;
      try { e = ctx_order_event(c, 2); } catch (...) { return; }
      if (hipEventRecord(e, side) == hipSuccess) (void)hipStreamWaitEvent(main, e, 0);
    }
  } side_join{ctx, s, sf};
  w.ctx = ctx;
  w.L = L;
  w.lev.assign(L + 1, HbsLevelDev());
  w.S.assign(L + 2, 0);
  w.K.assign(L + 2, 0);
  double* dh_child = dhB.p;
  double* dh_cur = dhA.p;
  const size_t shi = 2 * sizeof(double) * SK_KCAP * SK_KCAP;
  func_lds_at_least((const void*)node_interp_kernel, (int)shi);
  const size_t shv = INV_LDS_BYTES;
  func_lds_at_least((const void*)node_inverse_kernel, (int)shv);
  constexpr int MANY = 1 << 30;
  // profiler entries of the factor launches (their flops are known once the ranks are read back)
  std::vector<size_t> fac_entry(L + 1, SIZE_MAX);
  auto factor_launch = [&](const GNode* gn, const GNode* gch, int nn, int is_leaf, int is_root, const int* cr,
                           const int* cc, const double* U, const double* V, double* groot, int mn_known, int mx_known,
                           int lvl, hipStream_t fs) {
    // nodes with n + k <= BT: bordered Gauss-Jordan; the others: block
    // inverse in registers (n <= FN) or LDS Gauss-Jordan, launched first on
    // the same stream (each kernel takes only its own nodes and returns at
    // once when it has none).  mn_known / mx_known: the smallest and largest
    // node input of the level when the host knows them (the leaves, whose
    // sizes can differ by one node), else -1
    const bool small = !is_root && (mn_known < 0 || mn_known <= FN);
    const bool large = !is_root && (mx_known < 0 || mx_known > FN);
    if (small) {
      KernelTimer kt("node_factor_kernel", 0.0, 0.0, fs);
      hipLaunchKernelGGL(node_factor_kernel, dim3(nn), dim3(256), 0, fs, gn, gch, is_leaf, is_root, cr, cc, d_nodes,
                         U, V, dh_child, dh_cur, ws.p, w.gen.p, groot, failp, 0, FN);
      KERNEL_CHECK("node_factor");
    }
    if (large) {
      KernelTimer kt("node_inverse_kernel", 0.0, 0.0, fs);
      hipLaunchKernelGGL(node_inverse_kernel, dim3(nn), dim3(256), shv, fs, gn, gch, is_leaf, is_root, cr, cc, d_nodes,
                         U, V, dh_child, dh_cur, ws.p, w.gen.p, groot, failp, FN, MANY);
      KERNEL_CHECK("node_inverse");
    }
    {
      KernelTimer kt("node_factor_bordered_kernel", 0.0, 0.0, fs);
      hipLaunchKernelGGL(node_factor_bordered_kernel, dim3(nn), dim3(BWV * 64), 0, fs, gn, gch, is_leaf, is_root, cr, cc,
                         d_nodes, U, V, dh_child, dh_cur, ws.p, w.gen.p, groot, failp);
      KERNEL_CHECK("node_factor_bordered");
    }
    if (ctx->prof && !ctx->pending.empty()) fac_entry[lvl] = ctx->pending.size() - 1;
    // the root block (n = k_1 + k_2 <= 2 SK_KCAP) always fits the bordered kernel
    static_assert(2 * SK_KCAP <= BT, "the root block fits the bordered factorization");
  };
  int mx_leaf = 0;
  for (const GNode& g : G[L]) mx_leaf = std::max(mx_leaf, g.m);
  for (int l = L; l >= 1; --l) {
    const int nn = 1 << l;
    const bool leaf = l == L;
    GNode* dgl = dg.p + nn;
    int* cr = candr.p + cand_base[l];
    int* cc = candc.p + cand_base[l];
    // host-known sizes at the leaves; bounds above them
    int mx = 0, mn = 1 << 30;
    int64_t off = 0;
    if (leaf) {
      for (const GNode& g : G[L]) { off += g.m; mx = std::max(mx, g.m); mn = std::min(mn, g.m); }
      if (mx > mmax) RW_THROW(RW_ESINGULAR, "HBS node input exceeds the sketch bound");
      if (mx > ID_NT / 2) RW_THROW(RW_EINVAL, "HBS leaf of more than 128 nodes");
    } else {
      off = (int64_t)nn * 2 * SK_KCAP;
    }
    const int nsplit = level_split(nn);
    const int64_t len = off * SK_R;
    {
      KernelTimer kt("node_sketch_kernel", 0.0, 0.0);
      const dim3 grid(nn, 2, nsplit);
      double* outr = part_r.p;
      double* outc = part_c.p;
      const uint64_t sd = seed + 7919ull * l;
      if (leaf && mx > 192) {
        hipLaunchKernelGGL(node_sketch_kernel, grid, dim3(256), 0, s, dgl, cr, cc, d_nodes, N, sd, len, part_r.p,
                           part_c.p, 0, MANY);
      } else {
        // each kernel takes the nodes of its size range (leaves can straddle 128)
        if (!leaf || mn <= 128)
          hipLaunchKernelGGL(node_sketch_mfma_kernel<2>, grid, dim3(256), 0, s, dgl, cr, cc, d_nodes, N, sd, len,
                             outr, outc, 0, 128);
        if (!leaf || mx > 128)
          hipLaunchKernelGGL(node_sketch_mfma_kernel<3>, grid, dim3(256), 0, s, dgl, cr, cc, d_nodes, N, sd, len,
                             outr, outc, 128, 192);
      }
      KERNEL_CHECK("node_sketch");
      hipLaunchKernelGGL(node_sketch_sum_kernel, dim3(nblk(len), 2), dim3(256), 0, s, part_r.p, part_c.p, nsplit, len,
                         len, Sr.p, Sc.p);
      KERNEL_CHECK("node_sketch_sum");
    }
    {
      KernelTimer kt_id("node_id_kernel", 0.0, 0.0);
      // the level plan runs in the last workgroup to finish
      hipLaunchKernelGGL(node_id_kernel, dim3(nn, 2), dim3(ID_NT), 0, s, dgl, Sr.p, Sc.p, tol * tol, piv.p, Cr.p,
                         Cc.p, info.p, pubp, (long long)(l + 1), dg.p + nn / 2, dpar.p + nn, cntp,
                         (int64_t)w.gen.n, (int64_t)ws.n, failp, donep + l);
      KERNEL_CHECK("node_id");
    }
    hipLaunchKernelGGL(node_interp_kernel, dim3(nn, 2), dim3(256), shi, s, dgl, cr, cc, piv.p, Cr.p, Cc.p,
                       Ub.p + uv_base[l], Vb.p + uv_base[l], dpar.p + nn, candr.p + cand_base[l - 1],
                       candc.p + cand_base[l - 1]);
    KERNEL_CHECK("node_interp");
    // ---- node factorizations of this level on the side stream, once the
    // interpolation matrices are in (the children's D^ come from the
    // previous level's launches on the same stream), while this stream goes
    // on with the next level's sketches and IDs; level 1, after which no ID
    // work is left, runs on this stream once the side stream is through
    const GNode* dch = leaf ? dgl : dg.p + 2 * nn;
    hipStream_t fs = sf;
    if (l > 1) stream_after(ctx, sf, s, 1);
    else { stream_after(ctx, s, sf, 1); fs = s; }
    factor_launch(dgl, dch, nn, leaf ? 1 : 0, 0, cr, cc, Ub.p + uv_base[l], Vb.p + uv_base[l], (double*)nullptr,
                  leaf ? mn : -1, leaf ? mx : -1, l, fs);
    std::swap(dh_child, dh_cur);
  }
  // ---- root (its record was completed by the level-1 plan)
  factor_launch(dg.p + 1, dg.p + 2, 1, 0, 1, candr.p + cand_base[0], candc.p + cand_base[0], Ub.p, Vb.p, w.groot.p,
                -1, -1, 0, s);
  // ---- apply descriptors on the device; the host keeps bounds of the
  // sizes, and the records and flags are read back without a wait
  w.d_ints.alloc(ctx, (size_t)((int64_t(4) << L) - 3));
  w.d_offs.alloc(ctx, (size_t)((int64_t(8) << L) - 8));
  hipLaunchKernelGGL(apply_desc_kernel, dim3(nblk((int64_t(2) << L) - 1)), dim3(256), 0, s, dg.p, dpar.p, L, failp,
                     w.d_ints.p, w.d_offs.p);
  KERNEL_CHECK("apply_desc");
  for (int l = 1; l <= L; ++l) {
    const int64_t nn = int64_t(1) << l;
    HbsLevelDev& d = w.lev[l];
    d.nnodes = (int)nn;
    d.max_nin = l == L ? mx_leaf : 2 * SK_KCAP;
    d.max_k = SK_KCAP;
    d.S = l == L ? 2 * N : nn * 2 * SK_KCAP;
    d.K = nn * SK_KCAP;
    d.up_entries = d.e_entries = 0;
    w.S[l] = d.S;
    w.K[l] = d.K;
    d.nin = w.d_ints.p + 2 * nn - 4;
    d.k = d.nin + nn;
    d.in_off = w.d_offs.p + 4 * nn - 8;
    d.kout_off = d.in_off + nn;
    d.up_off = d.in_off + 2 * nn;
    d.e_off = d.in_off + 3 * nn;
  }
  w.nroot = 2 * SK_KCAP;
  w.S[0] = w.nroot;
  w.d_nroot = w.d_ints.p + (int64_t(4) << L) - 4;
  w.entries = 0;
  w.max_rank = 0;
  HIP_CHECK(hipMemcpyAsync(hG, dg.p, sizeof(GNode) * (size_t)(int64_t(2) << L), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipMemcpyAsync(hCtl, ctl.p, sizeof(int64_t) * 4, hipMemcpyDeviceToHost, s));
  w.fin.pending = true;
  w.fin.rec = hG;
  w.fin.ctl = hCtl;
  w.fin.fac_entry = fac_entry;
}
