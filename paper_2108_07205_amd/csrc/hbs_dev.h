// HBS compressed inverse resident in HBM, and its apply (level sweeps).
// Built either on the host (hbs_build.h, the static reference wall) or on
// the GPU per refinement (hbs_gpu_build, the refined arc's A_pp).
#pragma once

#include "hbs_build.h"
#include "kernels.h"

// Apply workspace of one HBS inverse for one stream of work: the level
// vectors of multi-RHS applies and the partial vectors of one-RHS applies,
// allocated from `ctx` on first use.  An HbsDev holds one for its own ctx;
// another ctx that applies the same (read-only) inverse on its own stream
// brings its own (ctx_hbs_work), so that concurrent applies do not share it.
struct HbsWork {
  rw_ctx* ctx = nullptr;
  DBuf<double> ws;
  int ws_nrhs = 0;
  int64_t ws_per_rhs = 0;        // doubles per right-hand side of ws (checked against the inverse)
  std::vector<double*> U, GB, X;
  DBuf<double> ws1;
  int64_t ws1_need = 0;          // doubles of the one-RHS plan that ws1 was sized for
};

struct HbsDev {
  rw_ctx* ctx = nullptr;
  int L = 0, nroot = 0;
  std::vector<HbsLevelDev> lev;  // index 1..L
  std::vector<int64_t> S, K;     // S[l]: level input length; K[l]: sum of skeleton sizes at level l
  DBuf<int> d_ints;              // nin / k per level
  DBuf<int64_t> d_offs;          // in_off / kout_off / up_off / e_off per level
  DBuf<double> gen;              // packed generators: [F*; G] ((k + nin) x nin) and E (nin x k) per node
  DBuf<float> gen32;             // FP32 copy (optional)
  DBuf<uint16_t> gen16;          // BF16 copy (optional; high halves of the FP32 words, rounded to nearest even)
  DBuf<double> groot;            // G_root (nroot x nroot)
  const int* d_nroot = nullptr;  // GPU build: the root size on the device (nroot is then a bound)
  int64_t entries = 0;           // sum of |E| + |F| + |G| + |G_root|
  int max_rank = 0;
  // right-hand sides from which multi-RHS applies take the matrix cores,
  // FP64 and FP32 generators (0: the built-in crossover; hbs_autotune
  // measures them for this inverse)
  int mfma_from64 = 0, mfma_from32 = 0, mfma_from16 = 0;
  HbsWork work;                  // apply workspace of the owning ctx
  // GPU build: node records and flags read back without a wait, checked by
  // hbs_gpu_finish (records: pinned host memory of the building context)
  struct Finish {
    bool pending = false;
    const void* rec = nullptr;
    const int64_t* ctl = nullptr;
    std::vector<size_t> fac_entry;
  } fin;
  int64_t n_unknowns() const { return lev.size() > 1 ? S[L] : 0; }
};

// Partial vectors of a one-RHS apply laid out from `base` (U1: bhat, GB1:
// G b, X1: down outputs, X1[0] the root's) with the split counts of each
// level; fixed-size, so that planning allocates nothing.
constexpr int HBS_MAX_LEVELS = 32;
struct HbsWs1 {
  double* U1[HBS_MAX_LEVELS + 1];
  double* GB1[HBS_MAX_LEVELS + 1];
  double* X1[HBS_MAX_LEVELS + 1];
  int nsu[HBS_MAX_LEVELS + 2];
  int nsd[HBS_MAX_LEVELS + 1];
  int nsr;
};
// Doubles the plan needs; with base != nullptr also fills ws.
int64_t hbs_ws1_plan(const HbsDev& w, double* base, HbsWs1& ws);
// One-RHS apply x = A^{-1} b with the partial vectors at `base` (at least
// hbs_ws1_plan doubles); allocates nothing.
void hbs_dev_apply1_at(const HbsDev& w, const double* b, double* x, int prec, double* base, hipStream_t s);

// Passes over the generators that one apply of nrhs right-hand sides makes
// (8 columns per pass on the vector path, 64 on the matrix cores: from 40
// columns with FP64 generators, from 16 with FP32 ones): the algorithmic
// generator bytes are passes * entries * width.
double hbs_gen_passes(int nrhs, bool f32 = false);

// Measure, on stream s, the apply of this inverse at 16..64 right-hand sides
// on the vector slab kernels and on the matrix cores, and keep for each
// generator precision the smallest count from which the matrix cores are
// faster at every larger measured count (never: a count above 64).
void hbs_autotune(HbsDev& w, hipStream_t s);

// Pack a host-built inverse into HBM.
// prec: RW_F64 (0), RW_F32 (1) or RW_BF16 (2): which narrow copy is added.
void hbs_upload(rw_ctx* ctx, const HbsInverse& H, int prec, HbsDev& out);
// x = A^{-1} b (b, x: n x nrhs column-major with leading dimensions ldb, ldx),
// enqueued on stream s (the caller's; the generators may have been built on
// another stream of the same device, ordered before s by the caller).
// prec: which generator copy is read (0 FP64, 1 FP32, 2 BF16; falls back to
// FP64 when the inverse has no such copy).
void hbs_dev_apply(HbsDev& h, const double* b, int64_t ldb, double* x, int64_t ldx, int nrhs, int prec,
                   hipStream_t s);
// The same with the workspace `wk` (its ctx allocates it on first use).
// mfma_from > 0 overrides the inverse's measured crossover to the matrix cores.
void hbs_dev_apply_ws(const HbsDev& h, HbsWork& wk, const double* b, int64_t ldb, double* x, int64_t ldx, int nrhs,
                      int prec, hipStream_t s, int mfma_from = 0);

// GPU build of the HBS inverse of the Nystrom matrix of one node set
// (contiguous arcs, balanced binary tree with leaves of at most leaf_max
// nodes).  d_nodes: device copy of h_nodes.  Same generator layout as
// hbs_upload; the level descriptors are written on the device, the host
// keeps bounds of the sizes (nroot, S, K, max_nin, max_k), and nothing waits
// for the device: the apply can be enqueued at once on the same stream (or
// after it).  hbs_gpu_finish, called once the stream has been synchronized,
// throws RW_ESINGULAR on a singular node block or a rank that exceeds the
// node sketch (the descriptors are then empty, so applies enqueued before
// give zeros) and fills the statistics.
void hbs_gpu_build(rw_ctx* ctx, const NodeRec* d_nodes, int64_t n_nodes, int leaf_max, double tol, uint64_t seed,
                   HbsDev& out);
void hbs_gpu_finish(HbsDev& w);
