// Shared definitions of the refined-wall library: error handling, the ctx
// object, device-memory accounting and the packed node record the kernels
// read.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <exception>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <unordered_map>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "rw.h"

struct RwError : std::runtime_error {
  int code;
  RwError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define RW_THROW(code, msg) throw RwError((code), (msg))
#define HIP_CHECK(x)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess)                                                              \
      throw RwError(RW_EDEVICE, std::string(#x) + " failed: " + hipGetErrorString(e_)); \
  } while (0)
#define KERNEL_CHECK(name)                                                             \
  do {                                                                                 \
    hipError_t e_ = hipGetLastError();                                                 \
    if (e_ != hipSuccess)                                                              \
      throw RwError(RW_EDEVICE, std::string("launch of ") + (name) + ": " + hipGetErrorString(e_)); \
  } while (0)

// One quadrature node of a discretization, as every kernel reads it.
// (x, y): position; (nx, ny): outward unit normal; w: quadrature weight;
// (s00, s01, s11): the symmetric 2x2 self block of A = -1/2 I + D + N at this
// node, -1/2 I + w (-(kappa / (2 pi)) t t^T + n n^T).
struct NodeRec {
  double x, y, nx, ny, w, s00, s01, s11;
};

// Accumulated time and algorithmic work of one step of the method.
struct PhaseStat {
  double ms = 0.0;
  int64_t calls = 0;
  double flops = 0.0;   // algorithmic floating-point operations
  double bytes = 0.0;   // algorithmic HBM bytes
};

struct AuxWorker;

struct HbsWork;

struct rw_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;   // 0 = unlimited (an aux ctx checks it against both ctxs' bytes)
  std::atomic<size_t> used{0};   // bytes held (in use + cached); written by the thread that drives this ctx
  // helper ctx on its own stream whose work one host worker thread runs
  // beside this ctx's inside a call (aux_fork / aux_join); owner: set on the helper
  rw_ctx* aux = nullptr;
  rw_ctx* owner = nullptr;
  AuxWorker* worker = nullptr;
  std::string err;
  rw_options opt{};
  int n_cu = 0;
  unsigned* d_sync = nullptr;   // grid-barrier / flag scratch owned by the ctx
  size_t sync_words = 0;
  // caching allocator: freed blocks are kept by size for reuse
  std::multimap<size_t, void*> cache;
  std::unordered_map<void*, size_t> live;   // block sizes of the allocations in use
  size_t cached = 0;
  // second stream for work that runs beside `stream` inside one call
  // (non-blocking, default priority; created on first use) and the
  // timing-free events that order the two
  hipStream_t side = nullptr;
  hipStream_t side2 = nullptr;   // a third one, used beside `side` (created on first use)
  std::vector<hipStream_t> bstreams;   // per-instance streams of rw_solve_batch (created on first use)
  std::vector<hipEvent_t> order_events;
  // pinned host staging for small per-call transfers (grow-only), and a
  // separate pinned area for small read-backs (a pageable one would keep
  // the HIP runtime busy, and the ctx's other thread waiting, until the copy)
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  void* rb = nullptr;
  size_t rb_bytes = 0;
  // pinned area of the GPU HBS build on this ctx (node records and candidate
  // lists going down, the records and flags coming back), used by nothing
  // else: the records stay there until the refinement is settled, which
  // happens before the next build on the ctx
  void* hbs_pin = nullptr;
  size_t hbs_pin_bytes = 0;
  // event after the last enqueued copy out of `pinned` (ctx_pinned waits
  // for it before handing the buffer out again)
  hipEvent_t pinned_ev = nullptr;
  bool pinned_ev_set = false;
  // the refinement whose end rw_refine did not wait for (at most one per
  // ctx; its device-side checks are still to be read), and the pinned word
  // its W pivot flag comes back to
  rw_refined* unsettled = nullptr;
  // apply workspaces of HBS inverses owned by other ctxs that this ctx
  // applies on its own stream (a wall's reference inverse used by a serving
  // slot), keyed by the inverse
  std::unordered_map<const void*, std::shared_ptr<HbsWork>> hbs_work;
  int* defer_pin = nullptr;
  // phase profiler (HIP events on `stream`)
  bool prof = false;
  struct Pending { std::string name; hipEvent_t a, b; double flops, bytes; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  std::map<std::string, PhaseStat> phases;
};

// Records a HIP event pair around a phase when the ctx profiler is on; the
// elapsed time is folded into ctx->phases at the next prof_flush().
// st: the stream the phase runs on (default: ctx->stream).
struct PhaseTimer {
  rw_ctx* ctx;
  rw_ctx::Pending p{};
  bool on;
  hipStream_t st;
  PhaseTimer(rw_ctx* c, const char* name, double flops = 0.0, double bytes = 0.0, hipStream_t stream = nullptr);
  ~PhaseTimer();
};
void prof_flush(rw_ctx* ctx);   // call after the stream has been synchronized

// The ctx of the C-ABI call in progress on this host thread (set on entry),
// so launchers can time their kernels when the ctx profiler is on.
rw_ctx* current_ctx();
void set_current_ctx(rw_ctx* ctx);

// Kernel-level timer: like PhaseTimer, keyed "k:<kernel>", on the current ctx.
struct KernelTimer {
  PhaseTimer* t = nullptr;
  KernelTimer(const char* name, double flops, double bytes, hipStream_t stream = nullptr);
  ~KernelTimer();
};

// The ctx's second stream, and its i-th ordering event (both created on
// first use and kept until the ctx is destroyed).
hipStream_t ctx_side_stream(rw_ctx* ctx);
hipStream_t ctx_side2_stream(rw_ctx* ctx);
hipEvent_t ctx_order_event(rw_ctx* ctx, int i);
// Pinned host staging of at least `bytes` (grow-only; growing first waits
// for the ctx's streams, so no copy from the old buffer is still in flight).
// It first waits for the copies marked by ctx_pinned_used, so that the
// host may overwrite the buffer.
void* ctx_pinned(rw_ctx* ctx, size_t bytes);
// Marks the copies enqueued on `s` so far as the last users of the staging
// buffer (the next ctx_pinned waits for them).
void ctx_pinned_used(rw_ctx* ctx, hipStream_t s);
// Allow kernel fn at least `bytes` of dynamic LDS on the current device
// (hipFuncSetAttribute once per kernel, device and larger size).
void func_lds_at_least(const void* fn, int bytes);
// Pinned read-back area of at least `bytes` (grow-only; its contents are
// valid until the next call that reads back on this ctx).
void* ctx_readback(rw_ctx* ctx, size_t bytes);
// The ctx's pinned area of the GPU HBS build (rw_ctx::hbs_pin), at least
// `bytes` (grow-only; growing waits for the ctx's stream first).
void* ctx_hbs_pinned(rw_ctx* ctx, size_t bytes);
// `waiter` waits for everything enqueued on `src` so far (event i).
void stream_after(rw_ctx* ctx, hipStream_t waiter, hipStream_t src, int i);

// Run fn(aux) on the helper ctx's worker thread, its stream ordered after
// everything enqueued on ctx->stream so far; aux_join waits for it, orders
// `into` (default ctx->stream) after the helper's stream and rethrows fn's
// error.  Between
// the two, the caller's thread may use ctx but not the helper, and fn may
// use the helper but not ctx.  AuxTask joins (ignoring errors) if the caller
// leaves early.  With the ctx's one_stream option, AuxTask runs fn(ctx) at
// once on the caller's thread and stream instead.
void aux_fork(rw_ctx* ctx, std::function<void(rw_ctx*)> fn);
void aux_join(rw_ctx* ctx, hipStream_t into = nullptr);
// Wake the helper's worker thread ahead of an aux_fork that follows shortly,
// so that the fork does not wait for the thread to wake (no-op with one_stream).
void aux_prewake(rw_ctx* ctx);
struct AuxTask {
  rw_ctx* ctx = nullptr;
  bool active = false;
  void fork(rw_ctx* c, std::function<void(rw_ctx*)> fn) {
    if (c->opt.one_stream) { fn(c); return; }
    aux_fork(c, std::move(fn));
    ctx = c;
    active = true;
  }
  void join(hipStream_t into = nullptr) { if (active) { active = false; aux_join(ctx, into); } }
  ~AuxTask() { if (active) { active = false; try { aux_join(ctx); } catch (...) {} } }
};

// Device allocation accounted against the ctx budget.
void* dev_alloc(rw_ctx* ctx, size_t bytes);
void dev_free(rw_ctx* ctx, void* p, size_t bytes);

template <class T>
struct DBuf {
  rw_ctx* ctx = nullptr;
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(rw_ctx* c, size_t count) { alloc(c, count); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept { *this = std::move(o); }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      release();
      ctx = o.ctx; p = o.p; n = o.n;
      o.p = nullptr; o.n = 0;
    }
    return *this;
  }
  ~DBuf() { release(); }
  void alloc(rw_ctx* c, size_t count) {
    release();
    ctx = c;
    n = count;
    p = count ? static_cast<T*>(dev_alloc(c, count * sizeof(T))) : nullptr;
  }
  // grow-only reuse
  void ensure(rw_ctx* c, size_t count) {
    if (count > n || !p) alloc(c, count);
  }
  void release() {
    if (p) dev_free(ctx, p, n * sizeof(T));
    p = nullptr;
    n = 0;
  }
  void upload(const T* h, size_t count, hipStream_t s) {
    if (count) HIP_CHECK(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
  }
  void download(T* h, size_t count, hipStream_t s) const {
    if (count) HIP_CHECK(hipMemcpyAsync(h, p, count * sizeof(T), hipMemcpyDeviceToHost, s));
  }
  size_t bytes() const { return n * sizeof(T); }
};

// Run f(i) for i in [0, n) on up to `threads` host threads.
void parallel_for(int64_t n, const std::function<void(int64_t)>& f, int threads = 0);

double wall_ms();
