// Launchers of the gfx950 kernels of the refined-wall solver.  All device
// matrices are column-major unless stated; every launcher enqueues on the
// given stream and checks the launch.
#pragma once

#include "common.h"

// ---------------------------------------------------------------- HBS apply
// One tree level of packed HBS inverse generators (device arrays, per node).
struct HbsLevelDev {
  int nnodes = 0;
  int max_nin = 0, max_k = 0;
  int64_t S = 0;              // sum of input sizes (this level's vector length)
  int64_t K = 0;              // sum of skeleton sizes (parent level's vector length)
  const int* nin = nullptr;
  const int* k = nullptr;
  const int64_t* in_off = nullptr;    // node input offset in this level's vectors
  const int64_t* kout_off = nullptr;  // node skeleton offset in the parent level's vectors
  const int64_t* up_off = nullptr;    // offset of [F*; G] ((k + nin) x nin) in the generator array
  const int64_t* e_off = nullptr;     // offset of E (nin x k)
  int64_t up_entries = 0;             // sum over nodes of (k + nin) nin
  int64_t e_entries = 0;              // sum over nodes of nin k
};

// up: bhat = F* b (to the parent level's vector), gb = G b (this level).
// mfma_from: right-hand sides from which the matrix-core path is taken
// (<= 0: the built-in crossover; a wall measures its own at build time).
void launch_hbs_up(const HbsLevelDev& L, const double* gen, const double* in, int64_t ld_in,
                   double* bhat, int64_t ld_bhat, double* gb, int64_t ld_gb, int nrhs, hipStream_t s,
                   int mfma_from = 0);
void launch_hbs_up_f32(const HbsLevelDev& L, const float* gen, const double* in, int64_t ld_in,
                       double* bhat, int64_t ld_bhat, double* gb, int64_t ld_gb, int nrhs, hipStream_t s,
                       int mfma_from = 0);
// root: out = G_root in (nroot x nroot, ld nroot); with d_nroot the size is
// read on the device (at most nroot).
void launch_hbs_root(int nroot, const int* d_nroot, const double* G, const double* in, int64_t ld_in, double* out,
                     int64_t ld_out, int nrhs, hipStream_t s, int mfma_from = 0);
// down: out = E xhat + gb.
void launch_hbs_down(const HbsLevelDev& L, const double* gen, const double* xhat, int64_t ld_xh,
                     const double* gb, int64_t ld_gb, double* out, int64_t ld_out, int nrhs, hipStream_t s,
                     int mfma_from = 0);
void launch_hbs_down_f32(const HbsLevelDev& L, const float* gen, const double* xhat, int64_t ld_xh,
                         const double* gb, int64_t ld_gb, double* out, int64_t ld_out, int nrhs, hipStream_t s,
                         int mfma_from = 0);

// One right-hand side: every level's block products split over column
// ranges of hbs_split_count(columns) workgroups, each writing a partial
// vector (part p of element i at base[p * stride + i]); a consumer sums
// the np partials of its input while staging it.  gen32 (if not null) is
// the FP32 copy of the generators.
int hbs_split_count(int ncols);
void launch_hbs_up1(const HbsLevelDev& L, const double* gen, const float* gen32, const double* in, int64_t in_stride,
                    int in_np, double* bhat, int64_t bstride, double* gb, int64_t gstride, hipStream_t s,
                    const uint16_t* gen16 = nullptr);
void launch_hbs_down1(const HbsLevelDev& L, const double* gen, const float* gen32, const double* xh, int64_t xstride,
                      int xnp, const double* gb, int64_t gstride, int gnp, double* out, int64_t ostride,
                      hipStream_t s, const uint16_t* gen16 = nullptr);
// BF16 generators (uint16 words: the high halves of FP32 values), FP32
// accumulation on the matrix cores from mfma_from right-hand sides.
void launch_hbs_up_bf16(const HbsLevelDev& L, const uint16_t* gen, const double* in, int64_t ld_in, double* bhat,
                        int64_t ld_bhat, double* gb, int64_t ld_gb, int nrhs, hipStream_t s, int mfma_from = 0);
void launch_hbs_down_bf16(const HbsLevelDev& L, const uint16_t* gen, const double* xhat, int64_t ld_xh,
                          const double* gb, int64_t ld_gb, double* out, int64_t ld_out, int nrhs, hipStream_t s,
                          int mfma_from = 0);
void launch_hbs_root1(int nroot, const int* d_nroot, const double* G, const double* in, int64_t in_stride, int in_np,
                      double* out, int64_t ostride, hipStream_t s);
void launch_parts_reduce(const double* in, int64_t stride, int np, int64_t n, double* x, hipStream_t s);

// ----------------------------------------------------------- Stokes tiles
// r = g - A tau on one node set (exact Nystrom operator, tiles on the fly).
// part: workspace of resid_part_doubles(n, nrhs) doubles (non-decreasing in
// nrhs: a workspace sized for nrhs columns serves any smaller count).  norms (optional,
// 2 nrhs doubles): |r_c|^2 in norms[c], |g_c|^2 in norms[nrhs + c].
// mode (an rw_resid value): every pair of nodes summed directly, or node
// clusters far from a wave of targets through their multipole expansions
// (resid_far_on tells which one a call takes).
size_t resid_part_doubles(int64_t n, int nrhs);
bool resid_far_on(int mode, int64_t n);
void launch_residual(const NodeRec* nodes, int64_t n, const double* g, const double* tau, double* r,
                     int nrhs, double* part, double* norms, hipStream_t s, int mode);
// g = sum_m S(x_i, z_m) f_m at all nodes (z, f device arrays, n_src x 2 row-major)
void launch_stokeslet_rhs(const NodeRec* nodes, int64_t n, const double* zf, int n_src, double* g,
                          hipStream_t s);
// dense A(targets, sources) (2 nt x 2 ns, column-major, ld) for two node sets
// that are either identical (self blocks on the diagonal) or disjoint.
void launch_assemble(const NodeRec* tgt, int64_t nt, const NodeRec* src, int64_t ns, bool same,
                     double* A, int64_t ld, hipStream_t s);
// Rows of R = skeleton rows of Q (uniform ID format): see kern_stokes.hip.
void launch_r_rows(const NodeRec* tnodes, const int* skel_dof, int nrows, const NodeRec* ref_nodes,
                   const int* ref_kind, int64_t n_o, const NodeRec* pnodes, int64_t n_p, int mode,
                   double* R, int64_t ldR, hipStream_t s);
// Y(2 nt x ncols, row-major) = sum over source segments sign * A(tgt, seg) Omega(seg rows, :)
// with Omega = counter-based +-1 entries; MFMA FP64.
struct SketchSeg {
  const NodeRec* src;
  int64_t ns;
  double sign;
  int64_t omega_row0;   // first Omega row of this segment
};
size_t sketch_part_doubles(int64_t nt, int64_t nsrc);  // workspace of launch_sketch
void launch_sketch(const NodeRec* tgt, int64_t nt, const SketchSeg* segs, int nseg, int ncols,
                   uint64_t seed, double* Y, double* part, hipStream_t s);

// Far field of the Q sketches by expansions about the center c of a circle
// of radius rho around the refined arc: rows 2 pos[i], 2 pos[i] + 1 of Y
// (row-major, ncols) (+)= the sketch of the sources in segs evaluated at
// tgt[i] (pos = nullptr: pos[i] = i), with the same Omega as launch_sketch
// (same seed and Omega row offsets).  local = false: multipole expansion of
// sources within rho, targets beyond FAR_RATIO rho; local = true: local
// expansion of sources beyond FAR_RATIO rho, targets within rho.
// part: far_part_elems(ncols, nsplit), coef: far_part_elems(ncols, 1).
constexpr int FAR_P = 40;           // expansion terms
constexpr double FAR_RATIO = 2.5;   // near / far split radius over rho
size_t far_part_elems(int ncols, int nsplit);
void launch_far_sketch(const SketchSeg* segs, int nseg, const NodeRec* tgt, int64_t nt, const int* pos, bool local,
                       double cx, double cy, double rho, int ncols, uint64_t seed, bool accumulate, double* Y,
                       double2* part, int nsplit, double2* coef, hipStream_t s);
// Y rows 2 pos[i], 2 pos[i] + 1 <- rows 2 i, 2 i + 1 of Yc (row-major, ncols)
void launch_scatter_rows(const double* Yc, int64_t n, const int* pos, int ncols, double* Y, hipStream_t s);

// gather / scatter between refined order and extended order; to_ext also
// zeroes the extended entries of the cut reference nodes (ref_kind 1 of
// n_ref), so it writes every entry of the extended vector
void launch_to_ext(const double* g, int64_t ld_g, int64_t n_new, const int* new2ext, const int* ref_kind,
                   int64_t n_ref, double* ext, int64_t ld_ext, int nrhs, hipStream_t s);
void launch_from_ext(const double* ext, int64_t ld_ext, int64_t n_new, const int* new2ext, double* out,
                     int64_t ld_out, int nrhs, bool accumulate, hipStream_t s);
void launch_gather_nodes(const NodeRec* src, const int* idx, int64_t n, NodeRec* dst, hipStream_t s);
// Gauss-Legendre rule of a panel order up to kMax, passed by value to kernels
struct GlRule {
  static constexpr int kMax = 32;
  double s[kMax], w[kMax];
};
// node records of n_panels panels of q nodes on the star curve (a, m): panel
// i's parameter interval is (pan[2 i], pan[2 i + 1]) (device); out: n_panels q
void launch_discretize(const double* pan, int64_t n_panels, int q, const GlRule& gl, double a, int m, NodeRec* out,
                       hipStream_t s);

// ------------------------------------------------------- dense FP64 algebra
// cooperative row ID of Y (m x ncols, row-major): pivots J (k), coefficient
// matrix C (m x kmax, row-major) and k; then P = C C_J^{-1} written into
// L (column-major, ld) at rows pos[i], columns col0..col0+k.
struct RowIdResult {
  int k = 0;
};
size_t rowid_work_bytes(int64_t m, int ncols, int kmax, int ngroups);
int launch_rowid(rw_ctx* ctx, const double* Y, int64_t m, int ncols, double tol, int kmax, int* J,
                 double* C, void* work, hipStream_t s);   // returns k (synchronizes)
// The same without synchronizing: the tournament selection, basis and
// coefficients are enqueued, and k (int) and the squared largest row norm and
// residual (2 x u64, ordered bits) land in res_k / res_m (device).  Returns
// false, enqueueing nothing, where only the cooperative form applies.  Once
// the caller has read the results back, rowid_certified tells whether they
// stand; if not, launch_rowid_fallback redoes the ID (synchronizing).
bool launch_rowid_enqueue(rw_ctx* ctx, const double* Y, int64_t m, int ncols, double tol, int kmax, int* J,
                          double* C, void* work, int* res_k, unsigned long long* res_m, hipStream_t s);
bool rowid_certified(int k, int kmax, double tol, const unsigned long long* hm);
int launch_rowid_fallback(rw_ctx* ctx, const double* Y, int64_t m, int ncols, double tol, int kmax, int* J, double* C,
                          void* work, hipStream_t s);
void launch_rowid_interp(const double* C, int64_t m, int kmax, int k, const int* J, const int* pos,
                         double* L, int64_t ldL, int col0, double* inv_work /* k*k doubles */, hipStream_t s);
// C_out = A^T B for tall A (M x ka), B (M x kb), column-major; beta: C_out = beta*C_out + ...
size_t gemm_tn_part_doubles(int64_t M, int ka, int kb);
void launch_gemm_tn(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M, int ka,
                    int kb, double* C, int64_t ldc, bool add_identity, double* part, hipStream_t s);
// Y = Y - X W (X: M x k col-major, W: k x nrhs col-major ld=k)
void launch_sub_xw(const double* X, int64_t ldx, int64_t M, int k, const double* W, double* Y,
                   int64_t ldy, int nrhs, hipStream_t s);
// Krylov vectors: v = w / sqrt(nrm2[0]) (nrm2 on the device; w, v may alias),
// y = a x.
void launch_scale_rsqrt(const double* w, int64_t n, const double* nrm2, double* v, hipStream_t s);
void launch_scale_copy(const double* x, int64_t n, double a, double* y, hipStream_t s);
// in-place inverse of a small k x k matrix (Gauss-Jordan, partial pivoting);
// writes 0 / pivot index + 1 to *info (device int)
void launch_small_inverse(double* W, int k, int* info, hipStream_t s);
// out = Winv z (k x k times k x nrhs)
void launch_small_gemm(const double* Winv, int k, const double* z, int nrhs, double* out, hipStream_t s);
// Y = Y - X (Winv z) in one launch (Winv: k x k, z: k x nrhs, both col-major
// ld = k); false, with nothing launched, when W^-1 and z do not fit in LDS.
bool launch_woodbury_sub(const double* X, int64_t ldx, int64_t M, int k, const double* Winv, const double* z,
                         double* Y, int64_t ldy, int nrhs, hipStream_t s);

// unpivoted blocked LU of an n x n matrix (ld), in place; *info = first zero
// or non-finite pivot + 1 (0 if none); *mult = bits of the largest |entry of
// L| (a growth measure: partial pivoting would keep it <= 1)
void launch_lu_nopiv(double* A, int64_t n, int64_t ld, int* info, unsigned long long* mult, hipStream_t s);
// B = U^{-1} L^{-1} B (nrhs columns, ldb) with the factors of launch_lu_nopiv
void launch_lu_solve(const double* LU, int64_t n, int64_t ld, double* B, int64_t ldb, int nrhs,
                     hipStream_t s);
// C -= A B (m x kk times kk x n, all column-major)
void launch_gemm_nn_sub(const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
                        int64_t ldc, int64_t m, int64_t n, int64_t kk, hipStream_t s);
