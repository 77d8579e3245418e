// C ABI of the refined-wall solver (include/rw.h): objects, the static
// reference-wall build, Algorithm 1 pre-computation per refinement and the
// Woodbury solve with FP64 iterative refinement.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <memory>
#include <mutex>
#include <set>

#include "geometry.h"
#include "hbs_dev.h"

// ======================================================================== ctx
// Caching allocator: a freed block goes back to ctx->cache and is reused by a
// later request of at most its size and at least half of it, so the
// per-step refine / solve cycle does not call hipMalloc or hipFree once warm
// (hipMalloc also holds up kernel launches from the ctx's other thread).
// Requests are rounded up to size classes (256-byte multiples up to 64 KiB,
// then four classes per octave), so that the sizes of successive
// refinements, which differ by some percent, fall on the same few blocks.
// Bytes held by ctx and by the ctx that shares its budget (owner or helper).
static size_t budget_used(const rw_ctx* ctx) {
  const rw_ctx* other = ctx->owner ? ctx->owner : ctx->aux;
  return ctx->used.load() + (other ? other->used.load() : 0);
}

static size_t size_class(size_t b) {
  b = (b + 255) & ~size_t(255);
  if (b <= 65536) return b;
  const int e = 63 - __builtin_clzll((unsigned long long)b);
  const size_t base = size_t(1) << e, step = base / 4;
  return base + (b - base + step - 1) / step * step;
}

void* dev_alloc(rw_ctx* ctx, size_t bytes) {
  bytes = size_class(bytes);
  auto it = ctx->cache.lower_bound(bytes);
  if (it != ctx->cache.end() && it->first <= 2 * bytes) {
    void* p = it->second;
    ctx->cached -= it->first;
    ctx->live[p] = it->first;
    ctx->cache.erase(it);
    return p;
  }
  if (ctx->budget && budget_used(ctx) + bytes > ctx->budget) {
    // release cached blocks before giving up
    for (auto& kv : ctx->cache) { (void)hipFree(kv.second); ctx->used -= std::min(ctx->used.load(), kv.first); }
    ctx->cache.clear();
    ctx->cached = 0;
    if (budget_used(ctx) + bytes > ctx->budget)
      RW_THROW(RW_ENOMEM, "HBM budget exceeded: need " + std::to_string(budget_used(ctx) + bytes) + " bytes, budget " +
                              std::to_string(ctx->budget));
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    for (auto& kv : ctx->cache) { (void)hipFree(kv.second); ctx->used -= std::min(ctx->used.load(), kv.first); }
    ctx->cache.clear();
    ctx->cached = 0;
    e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      RW_THROW(RW_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
  }
  ctx->used += bytes;
  ctx->live[p] = bytes;
  return p;
}

// Blocks return to the cache at their full size; the callers' stream order
// makes reuse safe (work on a ctx's second stream is joined back into its
// main stream before the buffers it uses are released).
void dev_free(rw_ctx* ctx, void* p, size_t bytes) {
  if (!p) return;
  auto it = ctx->live.find(p);
  if (it != ctx->live.end()) {
    bytes = it->second;
    ctx->live.erase(it);
  } else {
    bytes = size_class(bytes);
  }
  ctx->cache.emplace(bytes, p);
  ctx->cached += bytes;
}

static void ctx_release_cache(rw_ctx* ctx) {
  for (auto& kv : ctx->cache) {
    (void)hipFree(kv.second);
    ctx->used -= std::min(ctx->used.load(), kv.first);
  }
  ctx->cache.clear();
  ctx->cached = 0;
}

PhaseTimer::PhaseTimer(rw_ctx* c, const char* name, double flops, double bytes, hipStream_t stream)
    : ctx(c), on(c && c->prof), st(stream ? stream : (c ? c->stream : nullptr)) {
  if (!on) return;
  p.name = name;
  p.flops = flops;
  p.bytes = bytes;
  for (int i = 0; i < 2; ++i) {
    hipEvent_t e;
    if (!ctx->event_pool.empty()) { e = ctx->event_pool.back(); ctx->event_pool.pop_back(); }
    else HIP_CHECK(hipEventCreate(&e));
    (i == 0 ? p.a : p.b) = e;
  }
  HIP_CHECK(hipEventRecord(p.a, st));
}

PhaseTimer::~PhaseTimer() {
  if (!on) return;
  if (hipEventRecord(p.b, st) == hipSuccess) ctx->pending.push_back(p);
}

void prof_flush(rw_ctx* ctx) {
  if (ctx->aux) {
    // the helper's phases (its worker is idle whenever the owner flushes)
    prof_flush(ctx->aux);
    for (auto& kv : ctx->aux->phases) {
      PhaseStat& st = ctx->phases[kv.first];
      st.ms += kv.second.ms;
      st.calls += kv.second.calls;
      st.flops += kv.second.flops;
      st.bytes += kv.second.bytes;
    }
    ctx->aux->phases.clear();
  }
  for (auto& q : ctx->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(q.b) == hipSuccess && hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) {
      PhaseStat& st = ctx->phases[q.name];
      st.ms += ms;
      st.calls += 1;
      st.flops += q.flops;
      st.bytes += q.bytes;
    }
    ctx->event_pool.push_back(q.a);
    ctx->event_pool.push_back(q.b);
  }
  ctx->pending.clear();
}

static thread_local rw_ctx* g_current_ctx = nullptr;
rw_ctx* current_ctx() { return g_current_ctx; }
void set_current_ctx(rw_ctx* ctx) { g_current_ctx = ctx; }

KernelTimer::KernelTimer(const char* name, double flops, double bytes, hipStream_t stream) {
  rw_ctx* c = g_current_ctx;
  if (c && c->prof) {
    std::string key = std::string("k:") + name;
    t = new PhaseTimer(c, key.c_str(), flops, bytes, stream);
  }
}
KernelTimer::~KernelTimer() { delete t; }

hipStream_t ctx_side_stream(rw_ctx* ctx) {
  if (ctx->opt.one_stream) return ctx->stream;
  if (!ctx->side) HIP_CHECK(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
  return ctx->side;
}

hipStream_t ctx_side2_stream(rw_ctx* ctx) {
  if (ctx->opt.one_stream) return ctx->stream;
  if (!ctx->side2) HIP_CHECK(hipStreamCreateWithFlags(&ctx->side2, hipStreamNonBlocking));
  return ctx->side2;
}

hipEvent_t ctx_order_event(rw_ctx* ctx, int i) {
  while ((int)ctx->order_events.size() <= i) {
    hipEvent_t e;
    HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ctx->order_events.push_back(e);
  }
  return ctx->order_events[i];
}

void* ctx_pinned(rw_ctx* ctx, size_t bytes) {
  if (ctx->pinned_ev_set) {
    HIP_CHECK(hipEventSynchronize(ctx->pinned_ev));
    ctx->pinned_ev_set = false;
  }
  if (bytes <= ctx->pinned_bytes) return ctx->pinned;
  const size_t old_bytes = ctx->pinned_bytes;
  if (ctx->pinned) {
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    if (ctx->side) HIP_CHECK(hipStreamSynchronize(ctx->side));
    (void)hipHostFree(ctx->pinned);
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
  }
  // pinning pages is slow (milliseconds for megabytes): start at 4 MiB and
  // at least double, so that growth is rare
  bytes = std::max<size_t>({bytes, size_t(4) << 20, 2 * old_bytes});
  HIP_CHECK(hipHostMalloc(&ctx->pinned, bytes, hipHostMallocDefault));
  ctx->pinned_bytes = bytes;
  return ctx->pinned;
}

void ctx_pinned_used(rw_ctx* ctx, hipStream_t s) {
  if (!ctx->pinned_ev) HIP_CHECK(hipEventCreateWithFlags(&ctx->pinned_ev, hipEventDisableTiming));
  HIP_CHECK(hipEventRecord(ctx->pinned_ev, s));
  ctx->pinned_ev_set = true;
}

void func_lds_at_least(const void* fn, int bytes) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, int> done;
  int dev = 0;
  HIP_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  int& cur = done[{fn, dev}];
  if (bytes <= cur) return;
  HIP_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  cur = bytes;
}

void* ctx_readback(rw_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->rb_bytes) return ctx->rb;
  if (ctx->rb) {
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    (void)hipHostFree(ctx->rb);
    ctx->rb = nullptr;
    ctx->rb_bytes = 0;
  }
  bytes = std::max<size_t>(bytes, 4096);
  HIP_CHECK(hipHostMalloc(&ctx->rb, bytes, hipHostMallocDefault));
  ctx->rb_bytes = bytes;
  return ctx->rb;
}

void* ctx_hbs_pinned(rw_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->hbs_pin_bytes) return ctx->hbs_pin;
  if (ctx->hbs_pin) {
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    (void)hipHostFree(ctx->hbs_pin);
    ctx->hbs_pin = nullptr;
    ctx->hbs_pin_bytes = 0;
  }
  bytes = std::max<size_t>(bytes, size_t(256) << 10);
  HIP_CHECK(hipHostMalloc(&ctx->hbs_pin, bytes, hipHostMallocDefault));
  ctx->hbs_pin_bytes = bytes;
  return ctx->hbs_pin;
}

void stream_after(rw_ctx* ctx, hipStream_t waiter, hipStream_t src, int i) {
  if (waiter == src) return;
  hipEvent_t e = ctx_order_event(ctx, i);
  HIP_CHECK(hipEventRecord(e, src));
  HIP_CHECK(hipStreamWaitEvent(waiter, e, 0));
}

// ------------------------------------------------------------ helper ctx
struct AuxWorker {
  std::thread th;
  std::mutex mu;
  std::condition_variable cv;
  std::function<void()> job;
  bool has_job = false, busy = false, stop = false;
  bool soon = false;                    // aux_prewake: a job is on its way
  std::atomic<bool> job_flag{false};    // has_job, readable without the lock
  std::exception_ptr err;
};

static void aux_loop(rw_ctx* aux, AuxWorker* wk) {
  for (;;) {
    std::function<void()> job;
    {
      std::unique_lock<std::mutex> lk(wk->mu);
      wk->cv.wait(lk, [&] { return wk->has_job || wk->stop || wk->soon; });
      if (!wk->has_job && wk->stop) return;
      if (!wk->has_job) {
        // a job is on its way: wait for it awake (a sleeping thread takes
        // tens of microseconds to wake), at most 2 ms, then sleep again
        wk->soon = false;
        lk.unlock();
        const auto until = std::chrono::steady_clock::now() + std::chrono::milliseconds(2);
        while (!wk->job_flag.load(std::memory_order_acquire) && std::chrono::steady_clock::now() < until)
          __builtin_ia32_pause();
        continue;
      }
      job = std::move(wk->job);
      wk->has_job = false;
      wk->job_flag.store(false, std::memory_order_relaxed);
    }
    std::exception_ptr e;
    set_current_ctx(aux);
    try {
      HIP_CHECK(hipSetDevice(aux->device));
      job();
    } catch (...) {
      e = std::current_exception();
    }
    set_current_ctx(nullptr);
    {
      std::lock_guard<std::mutex> lk(wk->mu);
      wk->err = e;
      wk->busy = false;
    }
    wk->cv.notify_all();
  }
}

static rw_ctx* ctx_aux(rw_ctx* ctx) {
  if (ctx->aux) return ctx->aux;
  std::unique_ptr<rw_ctx> a(new rw_ctx());
  a->device = ctx->device;
  a->budget = ctx->budget;
  a->owner = ctx;
  a->n_cu = ctx->n_cu;
  HIP_CHECK(hipStreamCreateWithFlags(&a->stream, hipStreamNonBlocking));
  std::unique_ptr<AuxWorker> wk(new AuxWorker());
  wk->th = std::thread(aux_loop, a.get(), wk.get());
  ctx->worker = wk.release();
  ctx->aux = a.release();
  return ctx->aux;
}

void aux_fork(rw_ctx* ctx, std::function<void(rw_ctx*)> fn) {
  rw_ctx* a = ctx_aux(ctx);
  a->opt = ctx->opt;
  a->prof = ctx->prof;
  stream_after(ctx, a->stream, ctx->stream, 3);
  AuxWorker* wk = ctx->worker;
  {
    std::lock_guard<std::mutex> lk(wk->mu);
    wk->job = [fn, a]() { fn(a); };
    wk->has_job = true;
    wk->busy = true;
    wk->job_flag.store(true, std::memory_order_release);
  }
  wk->cv.notify_all();
}

void aux_prewake(rw_ctx* ctx) {
  if (ctx->opt.one_stream) return;
  ctx_aux(ctx);
  AuxWorker* wk = ctx->worker;
  {
    std::lock_guard<std::mutex> lk(wk->mu);
    if (wk->has_job || wk->busy) return;
    wk->soon = true;
  }
  wk->cv.notify_all();
}

void aux_join(rw_ctx* ctx, hipStream_t into) {
  AuxWorker* wk = ctx->worker;
  if (!wk) return;
  std::exception_ptr e;
  {
    std::unique_lock<std::mutex> lk(wk->mu);
    wk->cv.wait(lk, [&] { return !wk->busy; });
    e = wk->err;
    wk->err = nullptr;
  }
  stream_after(ctx, into ? into : ctx->stream, ctx->aux->stream, 4);
  if (e) std::rethrow_exception(e);
}

static void ctx_destroy_aux(rw_ctx* ctx) {
  if (ctx->worker) {
    {
      std::lock_guard<std::mutex> lk(ctx->worker->mu);
      ctx->worker->stop = true;
    }
    ctx->worker->cv.notify_all();
    ctx->worker->th.join();
    delete ctx->worker;
    ctx->worker = nullptr;
  }
  if (rw_ctx* a = ctx->aux) {
    (void)hipStreamSynchronize(a->stream);
    ctx_release_cache(a);
    for (auto& q : a->pending) { (void)hipEventDestroy(q.a); (void)hipEventDestroy(q.b); }
    for (auto e : a->event_pool) (void)hipEventDestroy(e);
    for (auto e : a->order_events) (void)hipEventDestroy(e);
    if (a->side) (void)hipStreamDestroy(a->side);
    if (a->side2) (void)hipStreamDestroy(a->side2);
    if (a->pinned) (void)hipHostFree(a->pinned);
    if (a->rb) (void)hipHostFree(a->rb);
    if (a->hbs_pin) (void)hipHostFree(a->hbs_pin);
    (void)hipStreamDestroy(a->stream);
    delete a;
    ctx->aux = nullptr;
  }
}

// ------------------------------------------------ no-allocation scratch
// Device memory of rw_hbs_apply_noalloc: a file-scope array that each device
// holds from the library's load until the process ends.  Host code never
// uses the array's name as an address: rw_ctx_create looks up each device's
// copy once (hipGetSymbolAddress, with that device current) and keeps it.
constexpr int64_t NOALLOC_DOUBLES = int64_t(1) << 21;   // 16 MiB
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static double* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
static std::mutex g_scratch_mu;

// Address of this device's copy of `scratch` (device current); looked up once.
static double* noalloc_scratch(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) RW_THROW(RW_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    double* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      RW_THROW(RW_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}

namespace {
thread_local std::string g_create_err;

template <class F>
int guarded(rw_ctx* ctx, F&& f) {
  try {
    if (ctx) {
      ctx->err.clear();
      HIP_CHECK(hipSetDevice(ctx->device));
    }
    set_current_ctx(ctx);
    f();
    set_current_ctx(nullptr);
    return RW_OK;
  } catch (const RwError& e) {
    set_current_ctx(nullptr);
    if (ctx) ctx->err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->err = "host allocation failed";
    return RW_ENOMEM;
  } catch (const std::exception& e) {
    if (ctx) ctx->err = e.what();
    return RW_EDEVICE;
  }
}
}  // namespace

// Event handle that moves with its owner and is destroyed with it.
struct OwnedEvent {
  hipEvent_t e = nullptr;
  OwnedEvent() = default;
  OwnedEvent(const OwnedEvent&) = delete;
  OwnedEvent& operator=(const OwnedEvent&) = delete;
  OwnedEvent(OwnedEvent&& o) noexcept : e(o.e) { o.e = nullptr; }
  OwnedEvent& operator=(OwnedEvent&& o) noexcept {
    std::swap(e, o.e);
    return *this;
  }
  ~OwnedEvent() {
    if (e) (void)hipEventDestroy(e);
  }
};

// ======================================================================= wall
struct rw_wall {
  rw_ctx* ctx = nullptr;
  rw_curve curve{};
  int P = 0, q = 16, leaf = 64, precision = RW_F64;
  double tol = 1e-10;
  std::vector<double> gl_s, gl_w;
  Discretization disc;
  DBuf<NodeRec> d_nodes;
  HbsDev hbs;                             // A_oo^{-1}
  rw_wall_stats stats{};
  DBuf<double> bat_in, bat_out;           // rw_solve_batch: stacked A_oo^{-1} inputs / outputs
};

namespace {

// Bytes per generator entry that the solve's applies of the wall's inverse read.
double gen_width(const rw_wall* w) { return w->precision == RW_BF16 ? 2.0 : (w->precision == RW_F32 ? 4.0 : 8.0); }

// The apply workspace that ctx uses for the inverse h (h's own for its ctx).
HbsWork& ctx_hbs_work(rw_ctx* ctx, HbsDev& h) {
  if (ctx == h.ctx) return h.work;
  std::shared_ptr<HbsWork>& p = ctx->hbs_work[&h];
  if (!p) {
    p = std::make_shared<HbsWork>();
    p->ctx = ctx;
  }
  return *p;
}

// x = A_oo^{-1} b on ctx's stream, with ctx's workspace for the wall's inverse.
void hbs_apply(rw_wall* w, rw_ctx* ctx, const double* b, int64_t ldb, double* x, int64_t ldx, int nrhs, int prec) {
  hbs_dev_apply_ws(w->hbs, ctx_hbs_work(ctx, w->hbs), b, ldb, x, ldx, nrhs, prec, ctx->stream, ctx->opt.mfma_from);
}

void build_wall(rw_ctx* ctx, const rw_curve& cv, int P, int q, int leaf, double tol, int precision, rw_wall& w) {
  const double t0 = wall_ms();
  w.ctx = ctx;
  w.curve = cv;
  w.P = P;
  w.q = q;
  w.leaf = leaf;
  w.tol = tol;
  w.precision = precision;
  gauss_legendre(q, w.gl_s, w.gl_w);
  discretize(cv.a, cv.m, q, w.gl_s, w.gl_w, reference_panels(P), w.disc);
  HbsParams prm;
  prm.leaf_nodes = leaf;
  prm.tol = tol;
  prm.merge = ctx->opt.hbs_merge;
  HbsInverse H;
  hbs_build_inverse(w.disc.nodes, prm, H);
  const int tree_levels = H.L, tree_max_rank = H.max_rank;
  hbs_fold_top(H, 768);   // root block of at most 768 rows (4.7 MB): the 8-RHS root kernel stages it in 64 KB of LDS
  hipStream_t s = ctx->stream;
  w.d_nodes.alloc(ctx, w.disc.nodes.size());
  w.d_nodes.upload(w.disc.nodes.data(), w.disc.nodes.size(), s);
  hbs_upload(ctx, H, precision, w.hbs);
  // the multi-RHS apply's crossover to the matrix cores, measured on this inverse
  hbs_autotune(w.hbs, s);
  HIP_CHECK(hipStreamSynchronize(s));
  w.stats.n_nodes = (int64_t)w.disc.nodes.size();
  w.stats.n_levels = tree_levels;
  w.stats.max_rank = tree_max_rank;
  w.stats.gen_entries = H.entries;
  w.stats.gen_bytes_f64 = 8 * H.entries;
  w.stats.mfma_from_f64 = w.hbs.mfma_from64;
  w.stats.mfma_from_f32 = w.hbs.mfma_from32 ? w.hbs.mfma_from32 : w.hbs.mfma_from16;
  w.stats.t_build_ms = wall_ms() - t0;
}

}  // namespace

// =================================================================== refined
struct rw_refined {
  rw_wall* wall = nullptr;
  rw_ctx* ctx = nullptr;
  std::vector<int32_t> level_of_panel;
  double q_tol = 1e-10;                // row-ID tolerance of Q (rw_refine's q_tol or the wall's id_tol)
  Discretization disc;                 // refined panels I_n (their node records: d_p, d_new)
  int64_t No = 0, Nk = 0, Nc = 0, Np = 0, Nn = 0, Next = 0;
  DBuf<NodeRec> d_ext;                 // [reference nodes | added nodes]
  DBuf<NodeRec> d_new, d_k, d_c, d_p;
  DBuf<int> d_new2ext, d_ref_kind, d_pos_k, d_pos_p;
  int k_k = 0, k_p = 0, k = 0;
  DBuf<double> L, R, X, W;             // W: k x k inverse + k x k scratch
  DBuf<int> d_J;                       // J_k then J_p
  DBuf<double> App;                    // LU of A_pp (dense path)
  bool app_hbs_on = false;             // A_pp^{-1} by a GPU-built HBS inverse instead
  HbsDev app_hbs;
  // solve workspace
  DBuf<double> gext, y, z, wv, r, tmp, part, norms;
  int ws_nrhs = 0;
  rw_info info{};
  // rw_refine returns once the device work is enqueued: `done` marks its
  // end, `pending` that its device-side checks (W pivot flag, A_pp build
  // flags) are still to be read; their outcome then sticks to the handle
  OwnedEvent done;
  OwnedEvent app_ready;                // on the side stream once the A_pp inverse is built
  bool pending = false;
  DBuf<int> dinfo;                     // W pivot flag (device)
  DBuf<double> wpart;                  // split partial sums of R X
  // GMRES workspace (rw_solve with RW_SOLVE_GMRES): Arnoldi basis V (N x
  // (m + 1)), preconditioned directions Z (N x m), the new vector, a zero
  // vector, Gram-Schmidt coefficients and norms, partial sums, y
  DBuf<double> gv, gz, gw, gzero, gh, gpart, gy;
  int gm = 0;
  int fail_rc = RW_OK;
  std::string fail_msg;
};

namespace {

// Reads the device-side outcome of a refinement whose end rw_refine did not
// wait for: waits for its device work (at once if the stream has been
// synchronized past it), then checks the W pivot flag and the A_pp build's
// flags.  A failure sticks to the handle; it is thrown unless `quiet`.
void refined_settle(rw_refined* f, bool quiet = false) {
  if (f->pending) {
    f->pending = false;
    if (f->ctx->unsettled == f) f->ctx->unsettled = nullptr;
    try {
      HIP_CHECK(hipEventSynchronize(f->done.e));
      const int info = *f->ctx->defer_pin;
      if (info) RW_THROW(RW_ESINGULAR, "singular Woodbury operator W (pivot " + std::to_string(info) + ")");
      if (f->app_hbs_on) {
        hbs_gpu_finish(f->app_hbs);
        f->info.app_entries = f->app_hbs.entries;
        f->info.app_max_rank = f->app_hbs.max_rank;
      }
    } catch (const RwError& e) {
      f->fail_rc = e.code;
      f->fail_msg = e.what();
    } catch (...) {   // (also reached from rw_refined_free, which must not throw)
      f->fail_rc = RW_EDEVICE;
      f->fail_msg = "reading the refinement's device-side checks failed";
    }
  }
  if (f->fail_rc != RW_OK && !quiet) RW_THROW(f->fail_rc, f->fail_msg);
}

void refined_ensure_ws(rw_refined* f, int nrhs) {
  if (nrhs <= f->ws_nrhs) return;
  const int64_t M = 2 * f->Next;
  f->gext.alloc(f->ctx, (size_t)M * nrhs);
  f->y.alloc(f->ctx, (size_t)M * nrhs);
  f->z.alloc(f->ctx, (size_t)std::max(1, f->k) * nrhs);
  f->wv.alloc(f->ctx, (size_t)std::max(1, f->k) * nrhs);
  f->r.alloc(f->ctx, (size_t)2 * f->Nn * nrhs);
  f->tmp.alloc(f->ctx, (size_t)2 * f->Nn * nrhs);
  const size_t part = std::max(resid_part_doubles(f->Nn, nrhs),
                               gemm_tn_part_doubles(M, std::max(1, f->k), nrhs));
  f->part.alloc(f->ctx, part);
  f->norms.alloc(f->ctx, (size_t)2 * nrhs);
  f->ws_nrhs = nrhs;
}

// Woodbury apply in stages so that several instances can share the apply of
// the reference inverse: in: src -> gext (extended order); the A_oo^{-1}
// block of y = A~^{-1} gext (ref_apply); out: the A_pp^{-1} block of y, the
// correction y -= X W^{-1} R y and dst (+)= y in refined order.
void woodbury_in(rw_refined* f, const double* src, int nrhs, hipStream_t s = nullptr) {
  const int64_t M = 2 * f->Next;
  launch_to_ext(src, 2 * f->Nn, f->Nn, f->d_new2ext.p, f->d_ref_kind.p, f->No, f->gext.p, M, nrhs,
                s ? s : f->ctx->stream);
}

void woodbury_ref_apply(rw_refined* f, int nrhs) {
  rw_wall* w = f->wall;
  const int64_t M = 2 * f->Next;
  const double gb = gen_width(w) * w->stats.gen_entries;
  PhaseTimer t(f->ctx, "a6_hbs_apply", 2.0 * w->stats.gen_entries * nrhs,
               gb * hbs_gen_passes(nrhs, w->precision != RW_F64));
  hbs_apply(w, f->ctx, f->gext.p, M, f->y.p, M, nrhs, w->precision);
}

// The A_pp^{-1} block of y on stream s.
void woodbury_app_apply(rw_refined* f, int nrhs, hipStream_t s) {
  const int64_t M = 2 * f->Next, Mo = 2 * f->No;
  PhaseTimer t(f->ctx, "a6_app_solve", 2.0 * f->app_hbs.entries * nrhs, 8.0 * f->app_hbs.entries * hbs_gen_passes(nrhs),
               s);
  hbs_dev_apply(f->app_hbs, f->gext.p + Mo, M, f->y.p + Mo, M, nrhs, false, s);
}

// app_done: the A_pp^{-1} block of y is already in (woodbury_app_apply).
void woodbury_out(rw_refined* f, double* dst, int nrhs, bool accumulate, bool app_done = false,
                  hipStream_t s = nullptr) {
  if (!s) s = f->ctx->stream;
  const int64_t M = 2 * f->Next, Mo = 2 * f->No, Mp = 2 * f->Np;
  // the refinement's last products (X, W, A_pp^{-1}) come from the side
  // stream: with app_done the stream has joined it already
  if (!app_done) HIP_CHECK(hipStreamWaitEvent(s, f->done.e, 0));
  if (app_done) {
  } else if (f->Np > 0 && f->app_hbs_on) {
    woodbury_app_apply(f, nrhs, s);
  } else if (f->Np > 0) {
    PhaseTimer t(f->ctx, "a6_app_solve", 2.0 * (double)Mp * Mp * nrhs, 8.0 * (double)Mp * Mp * nrhs, s);
    HIP_CHECK(hipMemcpy2DAsync(f->y.p + Mo, sizeof(double) * M, f->gext.p + Mo, sizeof(double) * M,
                               sizeof(double) * Mp, nrhs, hipMemcpyDeviceToDevice, s));
    launch_lu_solve(f->App.p, Mp, Mp, f->y.p + Mo, M, nrhs, s);
  }
  if (f->k > 0) {
    // z = R y, w = W^{-1} z, y -= X w
    PhaseTimer t(f->ctx, "a7_woodbury", 4.0 * f->k * (double)M * nrhs, 16.0 * f->k * (double)M, s);
    launch_gemm_tn(f->R.p, M, f->y.p, M, M, f->k, nrhs, f->z.p, f->k, false, f->part.p, s);
    if (!launch_woodbury_sub(f->X.p, M, M, f->k, f->W.p, f->z.p, f->y.p, M, nrhs, s)) {
      launch_small_gemm(f->W.p, f->k, f->z.p, nrhs, f->wv.p, s);
      launch_sub_xw(f->X.p, M, M, f->k, f->wv.p, f->y.p, M, nrhs, s);
    }
  }
  launch_from_ext(f->y.p, M, f->Nn, f->d_new2ext.p, dst, 2 * f->Nn, nrhs, accumulate, s);
}

// dst (2 N_n x nrhs) = (A~ + L R)^{-1} src via eq. (wood); accumulate: dst += ...
// A~ is block diagonal, so the A_pp^{-1} block (GPU-built HBS) runs on the
// side stream while the reference inverse runs on the main one.
void woodbury_apply(rw_refined* f, const double* src, double* dst, int nrhs, bool accumulate) {
  woodbury_in(f, src, nrhs);
  const bool hbs_app = f->Np > 0 && f->app_hbs_on;
  bool side_busy = false;
  // Only for one right-hand side, and not with k_p = 1: the side stream's
  // A_pp^{-1} L_p uses the A_pp inverse's multi-column workspace (its
  // one-column one when k_p = 1), which this apply must not share while
  // that runs; other cases keep to the side stream, behind it
  if (hbs_app && f->app_ready.e && nrhs == 1 && f->k_p != 1) {
    const hipError_t q = hipEventQuery(f->done.e);
    if (q == hipErrorNotReady) (void)hipGetLastError();   // not an error: the side stream is still at work
    else HIP_CHECK(q);
    side_busy = q == hipErrorNotReady;
  }
  if (side_busy) {
    // the refinement's last part (X_p, W) still runs on the side stream:
    // the A_pp^{-1} block, which needs only the finished A_pp inverse, runs
    // on this stream after the reference block instead of queuing behind it
    woodbury_ref_apply(f, nrhs);
    HIP_CHECK(hipStreamWaitEvent(f->ctx->stream, f->app_ready.e, 0));
    woodbury_app_apply(f, nrhs, f->ctx->stream);
    HIP_CHECK(hipStreamWaitEvent(f->ctx->stream, f->done.e, 0));
    woodbury_out(f, dst, nrhs, accumulate, true);
    return;
  }
  const bool fork = hbs_app;
  if (fork) {
    rw_ctx* ctx = f->ctx;
    const hipStream_t side = ctx_side_stream(ctx);
    stream_after(ctx, side, ctx->stream, 5);
    woodbury_app_apply(f, nrhs, side);
    woodbury_ref_apply(f, nrhs);
    stream_after(ctx, ctx->stream, side, 6);
  } else {
    woodbury_ref_apply(f, nrhs);
  }
  woodbury_out(f, dst, nrhs, accumulate, fork);
}

void validate_selection(const rw_wall* w, const int32_t* ids, const int32_t* levels, int n_sel) {
  if (n_sel < 0) RW_THROW(RW_EINVAL, "n_sel < 0");
  if (n_sel > 0 && (!ids || !levels)) RW_THROW(RW_EINVAL, "null panel_ids or levels");
  std::set<int32_t> seen;
  for (int i = 0; i < n_sel; ++i) {
    if (ids[i] < 0 || ids[i] >= w->P) RW_THROW(RW_EINVAL, "panel id " + std::to_string(ids[i]) + " out of range");
    if (!seen.insert(ids[i]).second) RW_THROW(RW_EINVAL, "duplicate panel id " + std::to_string(ids[i]));
    if (levels[i] < 0 || levels[i] > 8) RW_THROW(RW_EINVAL, "level outside [0, 8]");
  }
}

// Largest |entry of L| accepted from the unpivoted dense LU of A_pp.  A_pp
// is a second-kind matrix (-1/2 I plus a smooth part), whose multipliers
// stay far below 1; a larger one means growth that partial pivoting would
// have avoided, and A_pp then goes to the HBS inverse, whose node blocks are
// factored with pivoting.
constexpr double kAppLuMultMax = 1e3;

// Algorithm 1, pre-computation step 2: an inverse of A_pp on ctx ax (its
// own stream): dense LU for few added points, else (or when the LU meets a
// zero pivot or a multiplier above kAppLuMultMax) the GPU-built HBS inverse.
void build_app_inverse(rw_wall* w, rw_refined& f, uint64_t seed, rw_ctx* ax) {
  hipStream_t s = ax->stream;
  const int64_t Mp = 2 * f.Np;
  if (f.app_hbs_on) {
    PhaseTimer t(ax, "a3_app_hbs_build", 0.0, 0.0);
    hbs_gpu_build(ax, f.d_p.p, f.Np, w->leaf, w->tol, seed, f.app_hbs);
    return;
  }
  DBuf<int> dinfo(ax, 4);   // pivot flag, then (8-byte aligned) the multiplier bits
  f.App.alloc(ax, (size_t)Mp * Mp);
  {
    PhaseTimer t(ax, "a3_app_assemble", 0.0, 8.0 * (double)Mp * Mp);
    launch_assemble(f.d_p.p, f.Np, f.d_p.p, f.Np, true, f.App.p, Mp, s);
  }
  // test hook: a zero first column, which the LU's pivot check must report
  if (ax->opt.test_singular == 2) HIP_CHECK(hipMemsetAsync(f.App.p, 0, sizeof(double) * Mp, s));
  {
    PhaseTimer t(ax, "a3_app_lu", 2.0 / 3.0 * (double)Mp * Mp * Mp, 0.0);
    launch_lu_nopiv(f.App.p, Mp, Mp, dinfo.p, (unsigned long long*)(dinfo.p + 2), s);
  }
  int hinfo[4] = {0, 0, 0, 0};
  HIP_CHECK(hipMemcpyAsync(hinfo, dinfo.p, sizeof(hinfo), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  unsigned long long bits = 0;
  memcpy(&bits, hinfo + 2, sizeof(bits));
  double mult = 0.0;
  memcpy(&mult, &bits, sizeof(mult));
  f.info.app_lu_mult = hinfo[0] ? INFINITY : mult;
  if (hinfo[0] == 0 && mult <= kAppLuMultMax) return;
  f.App = DBuf<double>();
  f.app_hbs_on = true;
  PhaseTimer t(ax, "a3_app_hbs_build", 0.0, 0.0);
  hbs_gpu_build(ax, f.d_p.p, f.Np, w->leaf, w->tol, seed, f.app_hbs);
}

// Algorithm 1 pre-computation for the refinement described by level_of_panel,
// on ctx (the wall's own, or another ctx of the same device that uses the
// wall's read-only data on its own stream).
void build_refined(rw_wall* w, rw_ctx* ctx, const std::vector<int32_t>& level_of_panel, rw_refined& f) {
  hipStream_t s = ctx->stream;
  const double t0 = wall_ms();
  // the previous refinement's checks are read first: its read-back word and
  // pinned staging are reused below (its outcome stays with its handle)
  if (ctx->unsettled) refined_settle(ctx->unsettled, true);
  if (!ctx->defer_pin) HIP_CHECK(hipHostMalloc((void**)&ctx->defer_pin, 64, hipHostMallocDefault));
  aux_prewake(ctx);   // a3 is handed to the helper once the added nodes are known
  f.wall = w;
  f.ctx = ctx;
  f.level_of_panel = level_of_panel;
  // ---- a1: geometry and index sets (Sec. 3.1)
  std::unique_ptr<PhaseTimer> t_geo(new PhaseTimer(ctx, "a1_geometry"));
  const int q = w->q;
  // only the added panels are new: kept nodes are the reference nodes
  f.disc.order = q;
  f.disc.panels = refined_panels(w->P, level_of_panel);
  f.disc.nodes.clear();
  // the added panels' parameter intervals; their nodes are formed on the device
  std::vector<double> added_iv;
  for (const Panel& p : f.disc.panels)
    if (p.added) { added_iv.push_back(p.ta); added_iv.push_back(p.tb); }
  f.No = (int64_t)w->disc.nodes.size();
  f.Nn = (int64_t)f.disc.panels.size() * q;
  f.Np = (int64_t)(added_iv.size() / 2) * q;
  int64_t n_cut_panels = 0;
  for (int i = 0; i < w->P; ++i) n_cut_panels += level_of_panel[i] >= 0;
  f.Nc = n_cut_panels * q;
  f.Nk = f.No - f.Nc;
  f.Next = f.No + f.Np;
  const int64_t M = 2 * f.Next, Mo = 2 * f.No, Mp = 2 * f.Np;
  // host arrays go to the device through the ctx's pinned staging buffer
  // (one region per array), so the copies are asynchronous and the host
  // vectors may go out of scope at once; the buffer is next handed out once
  // these copies have run (ctx_pinned_used)
  const size_t stage_bytes = sizeof(double) * added_iv.size() +
                             sizeof(int) * (f.Nn + f.No + 3 * f.Nk + 2 * f.Np + f.Nc + 4 * f.Nk) + 16 * 256;
  char* stage_base = (char*)ctx_pinned(ctx, stage_bytes);
  size_t stage_off = 0;
  auto up = [&](void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    char* st = stage_base + stage_off;
    stage_off = (stage_off + bytes + 255) & ~size_t(255);
    if (stage_off > stage_bytes) RW_THROW(RW_EDEVICE, "pinned staging overflow");
    memcpy(st, src, bytes);
    HIP_CHECK(hipMemcpyAsync(dst, st, bytes, hipMemcpyHostToDevice, s));
  };
  // the added nodes first: a3 needs only them, so it starts before the rest of a1
  f.d_p.alloc(ctx, f.Np);
  DBuf<double> d_iv;
  if (f.Np) {
    d_iv.alloc(ctx, added_iv.size());
    up(d_iv.p, added_iv.data(), sizeof(double) * added_iv.size());
    GlRule gl{};
    for (int j = 0; j < q; ++j) { gl.s[j] = w->gl_s[j]; gl.w[j] = w->gl_w[j]; }
    launch_discretize(d_iv.p, (int64_t)added_iv.size() / 2, q, gl, w->curve.a, w->curve.m, f.d_p.p, s);
  }
  // ---- a3: A_pp^{-1} (dense LU for few added points, else a GPU-built HBS
  // inverse) on the helper ctx, beside the rest of a1 and the compression of
  // Q on this stream
  f.app_hbs_on = f.Np > ctx->opt.app_dense_max_nodes;
  f.info.app_lu_mult = 0.0;
  AuxTask a3;
  if (f.Np > 0) {
    const uint64_t seed = ctx->opt.seed ^ 0x3C6EF372FE94F82Bull;
    a3.fork(ctx, [&f, w, seed](rw_ctx* ax) { build_app_inverse(w, f, seed, ax); });
  }
  std::vector<int> k_ref, c_ref, new2ext(f.Nn), ref_kind(f.No, 0);
  k_ref.reserve(f.Nk);
  c_ref.reserve(f.Nc);
  for (int i = 0; i < w->P; ++i)
    for (int j = 0; j < q; ++j) {
      if (level_of_panel[i] >= 0) { c_ref.push_back(i * q + j); ref_kind[i * q + j] = 1; }
      else k_ref.push_back(i * q + j);
    }
  {
    int64_t np = 0;
    for (size_t pi = 0; pi < f.disc.panels.size(); ++pi) {
      const Panel& p = f.disc.panels[pi];
      for (int j = 0; j < q; ++j) {
        const int64_t n = (int64_t)pi * q + j;
        new2ext[n] = p.added ? (int)(f.No + np++) : p.ref_id * q + j;
      }
    }
  }
  f.d_ext.alloc(ctx, f.Next);
  HIP_CHECK(hipMemcpyAsync(f.d_ext.p, w->d_nodes.p, sizeof(NodeRec) * f.No, hipMemcpyDeviceToDevice, s));
  if (f.Np)
    HIP_CHECK(hipMemcpyAsync(f.d_ext.p + f.No, f.d_p.p, sizeof(NodeRec) * f.Np, hipMemcpyDeviceToDevice, s));
  f.d_new2ext.alloc(ctx, f.Nn);
  up(f.d_new2ext.p, new2ext.data(), sizeof(int) * f.Nn);
  f.d_ref_kind.alloc(ctx, f.No);
  up(f.d_ref_kind.p, ref_kind.data(), sizeof(int) * f.No);
  f.d_new.alloc(ctx, f.Nn);
  launch_gather_nodes(f.d_ext.p, f.d_new2ext.p, f.Nn, f.d_new.p, s);
  std::vector<int> pos_k(2 * f.Nk), pos_p(2 * f.Np);
  for (int64_t a = 0; a < f.Nk; ++a) { pos_k[2 * a] = 2 * k_ref[a]; pos_k[2 * a + 1] = 2 * k_ref[a] + 1; }
  for (int64_t a = 0; a < f.Np; ++a) { pos_p[2 * a] = (int)(Mo + 2 * a); pos_p[2 * a + 1] = (int)(Mo + 2 * a + 1); }
  f.d_pos_k.alloc(ctx, pos_k.size());
  up(f.d_pos_k.p, pos_k.data(), sizeof(int) * pos_k.size());
  f.d_pos_p.alloc(ctx, pos_p.size());
  up(f.d_pos_p.p, pos_p.data(), sizeof(int) * pos_p.size());
  {
    DBuf<int> idx_k(ctx, std::max<size_t>(1, k_ref.size())), idx_c(ctx, std::max<size_t>(1, c_ref.size()));
    f.d_k.alloc(ctx, f.Nk);
    up(idx_k.p, k_ref.data(), sizeof(int) * k_ref.size());
    launch_gather_nodes(w->d_nodes.p, idx_k.p, f.Nk, f.d_k.p, s);
    f.d_c.alloc(ctx, f.Nc);
    up(idx_c.p, c_ref.data(), sizeof(int) * c_ref.size());
    launch_gather_nodes(w->d_nodes.p, idx_c.p, f.Nc, f.d_c.p, s);
  }
  ctx_pinned_used(ctx, s);
  t_geo.reset();
  f.k_k = f.k_p = f.k = 0;
  f.info.n_near = -1;
  if (f.Nc > 0) {
    // ---- a2: Q ~= L R by randomized row IDs of the k-rows [-A_kc A_kp] and p-rows A_pk
    int ncols = ctx->opt.sketch_cols;
    const double tol = f.q_tol;
    DBuf<char> dres(ctx, 256);   // ranks and certificates of the two row IDs
    DBuf<double> Yk, Yp, Ck, Cp, part, part_p, Ynear;
    DBuf<double2> fpart, fcoef, fpart_p, fcoef_p;
    DBuf<char> work, work_p;
    // the p-row sketch and row ID run on the side stream beside the k-row
    // ones (they share only the inputs enqueued so far on this stream)
    const hipStream_t sp = ctx_side_stream(ctx);
    DBuf<int> dJ(ctx, 256);
    // Sec. 3.3: a circle of radius rho about the refined arc Gamma_r (its
    // cut and added nodes) splits the kept nodes into near (within
    // FAR_RATIO rho: exact entries) and far (expansions about the center).
    // The arc is sampled at its cut nodes and at the end points of the
    // refined panels (the added nodes lie between them on the curve), and
    // rho is widened by a relative 1e-4 for the curve between samples
    const std::vector<NodeRec>& rn = w->disc.nodes;
    std::vector<double> ax, ay;
    for (int i : c_ref) { ax.push_back(rn[i].x); ay.push_back(rn[i].y); }
    const double hp = 2.0 * M_PI / w->P;
    for (int i = 0; i < w->P; ++i)
      if (level_of_panel[i] >= 0)
        for (const double th : {i * hp, (i + 1) * hp}) {
          const double r = 1.0 + w->curve.a * std::cos(w->curve.m * th);
          ax.push_back(r * std::cos(th));
          ay.push_back(r * std::sin(th));
        }
    double bx0 = 1e300, bx1 = -1e300, by0 = 1e300, by1 = -1e300;
    for (size_t i = 0; i < ax.size(); ++i) {
      bx0 = std::min(bx0, ax[i]); bx1 = std::max(bx1, ax[i]);
      by0 = std::min(by0, ay[i]); by1 = std::max(by1, ay[i]);
    }
    const double fcx = 0.5 * (bx0 + bx1), fcy = 0.5 * (by0 + by1);
    auto d2 = [&](const NodeRec& q) { return (q.x - fcx) * (q.x - fcx) + (q.y - fcy) * (q.y - fcy); };
    double rho2 = 0.0;
    for (size_t i = 0; i < ax.size(); ++i)
      rho2 = std::max(rho2, (ax[i] - fcx) * (ax[i] - fcx) + (ay[i] - fcy) * (ay[i] - fcy));
    const double rho = std::sqrt(rho2) * (1.0 + 1e-4), near2 = FAR_RATIO * FAR_RATIO * rho * rho;
    std::vector<int> near_a, far_a, near_ref, far_ref;
    near_a.reserve(f.Nk);
    far_a.reserve(f.Nk);
    near_ref.reserve(f.Nk);
    far_ref.reserve(f.Nk);
    for (int64_t a = 0; a < f.Nk; ++a) {
      const NodeRec& q = rn[k_ref[a]];
      const bool nr = d2(q) < near2;
      (nr ? near_a : far_a).push_back((int)a);
      (nr ? near_ref : far_ref).push_back(k_ref[a]);
    }
    const bool far_on = ctx->opt.far_field != 0 && rho > 0.0 && f.Np > 0 && 2 * (int64_t)near_a.size() <= f.Nk;
    const int64_t n_near = (int64_t)near_a.size(), n_far = (int64_t)far_a.size();
    DBuf<NodeRec> d_near, d_far;
    DBuf<int> d_near_pos, d_far_pos, d_idx;
    if (far_on) {
      f.info.n_near = n_near;
      d_near.alloc(ctx, std::max<int64_t>(1, n_near));
      d_far.alloc(ctx, std::max<int64_t>(1, n_far));
      d_near_pos.alloc(ctx, std::max<int64_t>(1, n_near));
      d_far_pos.alloc(ctx, std::max<int64_t>(1, n_far));
      d_idx.alloc(ctx, std::max<int64_t>(1, f.Nk));
      up(d_near_pos.p, near_a.data(), sizeof(int) * n_near);
      up(d_far_pos.p, far_a.data(), sizeof(int) * n_far);
      up(d_idx.p, near_ref.data(), sizeof(int) * n_near);
      up(d_idx.p + n_near, far_ref.data(), sizeof(int) * n_far);
      launch_gather_nodes(w->d_nodes.p, d_idx.p, n_near, d_near.p, s);
      launch_gather_nodes(w->d_nodes.p, d_idx.p + n_near, n_far, d_far.p, s);
    }
    for (;;) {
      const int kmax = ncols - 8;
      Yk.alloc(ctx, (size_t)2 * f.Nk * ncols);
      Yp.alloc(ctx, (size_t)2 * f.Np * ncols);
      stream_after(ctx, sp, s, 11);
      SketchSeg sk[2] = {{f.d_c.p, f.Nc, -1.0, 0}, {f.d_p.p, f.Np, 1.0, 2 * f.Nc}};
      const uint64_t seed_k = ctx->opt.seed, seed_p = ctx->opt.seed ^ 0xA5A5A5A5ull;
      if (far_on) {
        // k-rows: far rows by the multipole expansion of the arc's sources,
        // near rows exactly (compact, then scattered); p-rows: the near kept
        // sources exactly, the far ones by a local expansion (Omega rows of
        // the near list after those of all kept nodes, so none repeats)
        const int ns_k = (int)std::min<int64_t>(256, std::max<int64_t>(1, (f.Nc + f.Np) / 32));
        const int ns_p = (int)std::min<int64_t>(256, std::max<int64_t>(1, n_far / 32));
        part.alloc(ctx, std::max<size_t>(1, sketch_part_doubles(n_near, f.Nc + f.Np)));
        part_p.alloc(ctx, std::max<size_t>(1, sketch_part_doubles(f.Np, n_near)));
        Ynear.alloc(ctx, (size_t)std::max<int64_t>(1, 2 * n_near * ncols));
        fpart.alloc(ctx, far_part_elems(ncols, ns_k));
        fcoef.alloc(ctx, far_part_elems(ncols, 1));
        fpart_p.alloc(ctx, far_part_elems(ncols, ns_p));
        fcoef_p.alloc(ctx, far_part_elems(ncols, 1));
        const double fl = 2.0 * ncols * (2.0 * n_near * 2.0 * (f.Nc + f.Np) + 2.0 * f.Np * 2.0 * n_near) +
                          8.0 * 4.0 * FAR_P * ncols * ((f.Nc + f.Np) + n_far + n_far + f.Np);
        PhaseTimer t(ctx, "a2_sketch", fl, 8.0 * ncols * 2.0 * (f.Nk + f.Np));
        SketchSeg spn[1] = {{d_near.p, n_near, 1.0, 2 * f.Nk}};
        launch_sketch(f.d_p.p, f.Np, spn, 1, ncols, seed_p, Yp.p, part_p.p, sp);
        SketchSeg spf[1] = {{d_far.p, n_far, 1.0, 0}};
        if (n_far)
          launch_far_sketch(spf, 1, f.d_p.p, f.Np, nullptr, true, fcx, fcy, rho, ncols, seed_p, true, Yp.p,
                            fpart_p.p, ns_p, fcoef_p.p, sp);
        launch_far_sketch(sk, 2, d_far.p, n_far, d_far_pos.p, false, fcx, fcy, rho, ncols, seed_k, false, Yk.p,
                          fpart.p, ns_k, fcoef.p, s);
        launch_sketch(d_near.p, n_near, sk, 2, ncols, seed_k, Ynear.p, part.p, s);
        launch_scatter_rows(Ynear.p, n_near, d_near_pos.p, ncols, Yk.p, s);
      } else {
        part.alloc(ctx, sketch_part_doubles(f.Nk, f.Nc + f.Np));
        part_p.alloc(ctx, sketch_part_doubles(f.Np, f.Nk));
        const double fl = 2.0 * ncols * (2.0 * f.Nk * 2.0 * (f.Nc + f.Np) + 2.0 * f.Np * 2.0 * f.Nk);
        PhaseTimer t(ctx, "a2_sketch", fl, 8.0 * ncols * 2.0 * (f.Nk + f.Np));
        SketchSeg spk[1] = {{f.d_k.p, f.Nk, 1.0, 0}};
        launch_sketch(f.d_p.p, f.Np, spk, 1, ncols, seed_p, Yp.p, part_p.p, sp);
        launch_sketch(f.d_k.p, f.Nk, sk, 2, ncols, seed_k, Yk.p, part.p, s);
      }
      Ck.alloc(ctx, (size_t)2 * f.Nk * kmax);
      Cp.alloc(ctx, (size_t)2 * f.Np * kmax);
      const int ng = std::max(256, ctx->n_cu);
      work.alloc(ctx, std::max(rowid_work_bytes(2 * f.Nk, ncols, kmax, ng), rowid_work_bytes(2 * f.Np, ncols, kmax, ng)));
      work_p.alloc(ctx, rowid_work_bytes(2 * f.Np, ncols, kmax, ng));
      PhaseTimer t_id(ctx, "a2_row_id", 8.0 * ncols * 2.0 * (f.Nk + f.Np) * 40.0, 8.0 * ncols * 2.0 * (f.Nk + f.Np));
      // both row IDs enqueued (the p rows' on the side stream), one read-back
      // of their ranks and certificates once this stream has joined the side
      int* rk = (int*)dres.p;
      unsigned long long* rm = (unsigned long long*)(dres.p + 64);
      const bool qp = f.Np > 0 && launch_rowid_enqueue(ctx, Yp.p, 2 * f.Np, ncols, tol, kmax, dJ.p + 128, Cp.p,
                                                       work_p.p, rk + 1, rm + 2, sp);
      const bool qk = f.Nk > 0 && launch_rowid_enqueue(ctx, Yk.p, 2 * f.Nk, ncols, tol, kmax, dJ.p, Ck.p, work.p, rk,
                                                       rm, s);
      stream_after(ctx, s, sp, 12);
      char* rbk = (char*)ctx_readback(ctx, 64 + 4 * sizeof(unsigned long long));
      int* hk = (int*)rbk;
      unsigned long long* hm = (unsigned long long*)(rbk + 64);
      HIP_CHECK(hipMemcpyAsync(hk, rk, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
      HIP_CHECK(hipMemcpyAsync(hm, rm, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
      HIP_CHECK(hipStreamSynchronize(s));
      f.k_k = qk ? hk[0] : 0;
      f.k_p = qp ? hk[1] : 0;
      if (f.Nk > 0 && (!qk || !rowid_certified(f.k_k, kmax, tol, hm)))
        f.k_k = launch_rowid_fallback(ctx, Yk.p, 2 * f.Nk, ncols, tol, kmax, dJ.p, Ck.p, work.p, s);
      if (f.Np > 0 && (!qp || !rowid_certified(f.k_p, kmax, tol, hm + 2)))
        f.k_p = launch_rowid_fallback(ctx, Yp.p, 2 * f.Np, ncols, tol, kmax, dJ.p + 128, Cp.p, work.p, s);
      const bool full = (f.k_k >= kmax) || (f.k_p >= kmax);
      if (!full) break;
      if (ncols >= 128) RW_THROW(RW_ESINGULAR, "rank of the update matrix exceeds the largest sketch (128 columns)");
      ncols = (ncols < 64) ? 64 : (ncols < 96 ? 96 : 128);
    }
    f.k = f.k_k + f.k_p;
    const int kmax = ncols - 8;
    PhaseTimer t_lr(ctx, "a2_interp_rows", 0.0, 16.0 * f.k * (double)M);
    f.L.alloc(ctx, (size_t)M * f.k);
    HIP_CHECK(hipMemsetAsync(f.L.p, 0, sizeof(double) * M * f.k, s));
    DBuf<double> inv(ctx, (size_t)128 * 128);
    f.d_J.alloc(ctx, f.k);
    if (f.k_k) HIP_CHECK(hipMemcpyAsync(f.d_J.p, dJ.p, sizeof(int) * f.k_k, hipMemcpyDeviceToDevice, s));
    if (f.k_p) HIP_CHECK(hipMemcpyAsync(f.d_J.p + f.k_k, dJ.p + 128, sizeof(int) * f.k_p, hipMemcpyDeviceToDevice, s));
    launch_rowid_interp(Ck.p, 2 * f.Nk, kmax, f.k_k, f.d_J.p, f.d_pos_k.p, f.L.p, M, 0, inv.p, s);
    launch_rowid_interp(Cp.p, 2 * f.Np, kmax, f.k_p, f.d_J.p + f.k_k, f.d_pos_p.p, f.L.p, M, f.k_k, inv.p, s);
    // R: skeleton rows of Q (k rows on k points, then p rows)
    f.R.alloc(ctx, (size_t)f.k * M);
    launch_r_rows(f.d_k.p, f.d_J.p, f.k_k, w->d_nodes.p, f.d_ref_kind.p, f.No, f.d_p.p, f.Np, 0, f.R.p, M, s);
    launch_r_rows(f.d_p.p, f.d_J.p + f.k_k, f.k_p, w->d_nodes.p, f.d_ref_kind.p, f.No, f.d_p.p, f.Np, 1,
                  f.R.p + (size_t)f.k_k * M, M, s);
  }
  if (f.k > 0) {
    // ---- a4: X = A~^{-1} L; the A_oo^{-1} block needs only the reference inverse
    f.X.alloc(ctx, (size_t)M * f.k);
    HIP_CHECK(hipMemsetAsync(f.X.p, 0, sizeof(double) * M * f.k, s));
  }
  // the side stream's A_pp^{-1} block of X below needs L, R and the cleared X
  // from this stream, not the A_oo^{-1} block: it waits for this event only
  const hipEvent_t x_in = ctx_order_event(ctx, 8);
  HIP_CHECK(hipEventRecord(x_in, s));
  if (f.k > 0 && f.k_k) {
    PhaseTimer t_x(ctx, "a4_X", 2.0 * w->stats.gen_entries * f.k_k, 8.0 * w->stats.gen_entries * hbs_gen_passes(f.k_k));
    hbs_apply(w, ctx, f.L.p, M, f.X.p, M, f.k_k, false);
  }
  // ---- the rest (A_pp^{-1} block of X, W and its inverse) runs on the side
  // stream, behind the A_pp build and this stream's inputs to it (the A_pp^{-1}
  // block of X beside the A_oo^{-1} block, W behind both), so that the main
  // stream is free for the solve's A_oo^{-1} apply meanwhile; the solve joins
  // the side stream before the Woodbury correction
  if (f.k > 0) {
    f.W.alloc(ctx, (size_t)2 * f.k * f.k);
    f.wpart.alloc(ctx, gemm_tn_part_doubles(M, f.k, f.k));
    f.dinfo.alloc(ctx, 4);
  }
  const hipStream_t st = ctx_side_stream(ctx);
  struct SideDrain {   // on an error below, no side-stream work outlives the handle's buffers
    hipStream_t st;
    bool armed = true;
    ~SideDrain() { if (armed) (void)hipStreamSynchronize(st); }
  } drain{st};
  HIP_CHECK(hipStreamWaitEvent(st, x_in, 0));
  a3.join(st);
  if (f.Np > 0 && f.app_hbs_on) {
    if (!f.app_ready.e) HIP_CHECK(hipEventCreateWithFlags(&f.app_ready.e, hipEventDisableTiming));
    HIP_CHECK(hipEventRecord(f.app_ready.e, st));
  }
  if (f.k > 0) {
    if (f.k_p) {
      double* xp = f.X.p + Mo + (size_t)f.k_k * M;
      if (f.app_hbs_on) {
        PhaseTimer t_x(ctx, "a4_Xp", 2.0 * f.app_hbs.entries * f.k_p, 8.0 * f.app_hbs.entries * hbs_gen_passes(f.k_p),
                       st);
        hbs_dev_apply(f.app_hbs, f.L.p + Mo + (size_t)f.k_k * M, M, xp, M, f.k_p, false, st);
      } else {
        PhaseTimer t_x(ctx, "a4_Xp", 2.0 * (double)Mp * Mp * f.k_p, 8.0 * (double)Mp * Mp, st);
        HIP_CHECK(hipMemcpy2DAsync(xp, sizeof(double) * M, f.L.p + Mo + (size_t)f.k_k * M, sizeof(double) * M,
                                   sizeof(double) * Mp, f.k_p, hipMemcpyDeviceToDevice, st));
        launch_lu_solve(f.App.p, Mp, Mp, xp, M, f.k_p, st);
      }
    }
    // ---- a5: W = I + R X and its inverse (FP64), behind the A_oo^{-1} block of X
    stream_after(ctx, st, s, 7);
    PhaseTimer t_w(ctx, "a5_W", 2.0 * f.k * (double)f.k * M + 2.0 * (double)f.k * f.k * f.k, 16.0 * f.k * (double)M,
                   st);
    launch_gemm_tn(f.R.p, M, f.X.p, M, M, f.k, f.k, f.W.p, f.k, true, f.wpart.p, st);
    // test hook: a zero first column, which the inversion's pivot check must report
    if (ctx->opt.test_singular == 1) HIP_CHECK(hipMemsetAsync(f.W.p, 0, sizeof(double) * f.k, st));
    launch_small_inverse(f.W.p, f.k, f.dinfo.p + 1, st);
    HIP_CHECK(hipMemcpyAsync(ctx->defer_pin, f.dinfo.p + 1, sizeof(int), hipMemcpyDeviceToHost, st));
  } else {
    stream_after(ctx, st, s, 7);
    *ctx->defer_pin = 0;
  }
  // the W pivot flag and the A_pp build's flags and statistics (read back on
  // the helper's stream, which the side stream has waited for) are checked
  // once the side stream has passed this event: here under the profiler,
  // otherwise by the next call that uses the handle or the next refinement
  if (!f.done.e) HIP_CHECK(hipEventCreateWithFlags(&f.done.e, hipEventDisableTiming));
  HIP_CHECK(hipEventRecord(f.done.e, st));
  drain.armed = false;
  f.pending = true;
  if (ctx->prof) {
    refined_settle(&f);
    prof_flush(ctx);
  }
  f.info.n_k = f.Nk;
  f.info.n_c = f.Nc;
  f.info.n_p = f.Np;
  f.info.k_k = f.k_k;
  f.info.k_p = f.k_p;
  f.info.k = f.k;
  f.info.t_refine_ms = wall_ms() - t0;
  if (f.pending) ctx->unsettled = &f;
}

// ------------------------------------------------------------------ GMRES
// Restarted GMRES on the exact refined operator A_nn for one column (Sec. 4:
// the Woodbury solve of the extended system is the preconditioner; here it
// is applied on the right, so the residual GMRES minimizes is the true
// ||g - A_nn tau||).  Products A z come from the residual kernel (g = 0);
// Gram-Schmidt is applied twice per step (classical, on the device), and the
// host reads back one Hessenberg column per step for the Givens rotations.
// Returns the iterations taken; *rel: the final ||g - A tau|| / ||g||,
// *rel1: the residual estimate after the first step.
void gmres_ensure_ws(rw_refined* f, int m) {
  if (m <= f->gm) return;
  rw_ctx* ctx = f->ctx;
  const int64_t N = 2 * f->Nn;
  f->gv.alloc(ctx, (size_t)N * (m + 1));
  f->gz.alloc(ctx, (size_t)N * m);
  f->gw.alloc(ctx, (size_t)N);
  f->gzero.alloc(ctx, (size_t)N);
  HIP_CHECK(hipMemsetAsync(f->gzero.p, 0, sizeof(double) * N, ctx->stream));
  f->gh.alloc(ctx, (size_t)2 * (m + 1) + 8);
  f->gpart.alloc(ctx, gemm_tn_part_doubles(N, m + 1, 1));
  f->gy.alloc(ctx, (size_t)m);
  f->gm = m;
}

int gmres_column(rw_refined* f, const double* g, double* tau, double tol, int maxit, double* rel, double* rel1) {
  rw_ctx* ctx = f->ctx;
  hipStream_t s = ctx->stream;
  const rw_options& o = ctx->opt;
  const int m = o.gmres_restart;
  const bool precond = o.gmres_precond != 0;
  const int64_t N = 2 * f->Nn;
  gmres_ensure_ws(f, m);
  refined_ensure_ws(f, 1);
  double* V = f->gv.p;
  double* Z = f->gz.p;
  double* w = f->gw.p;
  double* h1 = f->gh.p;            // m + 1
  double* h2 = f->gh.p + (m + 1);  // m + 1
  double* nrm = f->gh.p + 2 * (m + 1);   // [0]: |w|^2, [1]: |g|^2, [2]: |r|^2
  double* hb = (double*)ctx_readback(ctx, sizeof(double) * (2 * (m + 1) + 8));
  auto matvec = [&](const double* z, double* out) {   // out = A z
    PhaseTimer t(ctx, "a8_residual", 26.0 * (double)f->Nn * f->Nn, 0.0);
    launch_residual(f->d_new.p, f->Nn, f->gzero.p, z, out, 1, f->part.p, nullptr, s, ctx->opt.resid_mode);
    launch_scale_copy(out, N, -1.0, out, s);
  };
  auto dot_to = [&](const double* a, const double* b, double* dst) {
    launch_gemm_tn(a, N, b, N, N, 1, 1, dst, 1, false, f->gpart.p, s);
  };
  // tau = 0, r = g
  HIP_CHECK(hipMemsetAsync(tau, 0, sizeof(double) * N, s));
  dot_to(g, g, nrm + 1);
  HIP_CHECK(hipMemcpyAsync(hb, nrm + 1, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_CHECK(hipStreamSynchronize(s));
  refined_settle(f);
  const double gn = std::sqrt(hb[0]);
  if (!(gn > 0.0)) {
    *rel = *rel1 = 0.0;
    return 0;
  }
  double beta = gn;
  launch_scale_rsqrt(g, N, nrm + 1, V, s);
  int it = 0;
  *rel1 = -1.0;
  std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), gam(m + 1);
  for (;;) {
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(gam.begin(), gam.end(), 0.0);
    gam[0] = beta;
    int j = 0;
    double est = beta;
    for (; j < m && it < maxit; ++j) {
      double* vj = V + (size_t)j * N;
      double* zj = Z + (size_t)j * N;
      if (precond) {
        woodbury_apply(f, vj, zj, 1, false);
      } else {
        HIP_CHECK(hipMemcpyAsync(zj, vj, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
      }
      matvec(zj, w);
      // two passes of classical Gram-Schmidt against v_0 .. v_j
      launch_gemm_tn(V, N, w, N, N, j + 1, 1, h1, j + 1, false, f->gpart.p, s);
      launch_sub_xw(V, N, N, j + 1, h1, w, N, 1, s);
      launch_gemm_tn(V, N, w, N, N, j + 1, 1, h2, j + 1, false, f->gpart.p, s);
      launch_sub_xw(V, N, N, j + 1, h2, w, N, 1, s);
      dot_to(w, w, nrm);
      launch_scale_rsqrt(w, N, nrm, V + (size_t)(j + 1) * N, s);
      HIP_CHECK(hipMemcpyAsync(hb, h1, sizeof(double) * (2 * (m + 1) + 1), hipMemcpyDeviceToHost, s));
      HIP_CHECK(hipStreamSynchronize(s));
      ++it;
      // Hessenberg column j, then the rotations of the previous columns and a new one
      double* hc = H.data() + (size_t)j * (m + 1);
      for (int i = 0; i <= j; ++i) hc[i] = hb[i] + hb[(m + 1) + i];
      hc[j + 1] = std::sqrt(std::max(0.0, hb[2 * (m + 1)]));
      for (int i = 0; i < j; ++i) {
        const double a = hc[i], b = hc[i + 1];
        hc[i] = cs[i] * a + sn[i] * b;
        hc[i + 1] = -sn[i] * a + cs[i] * b;
      }
      const double a = hc[j], b = hc[j + 1];
      const double r = std::hypot(a, b);
      cs[j] = r > 0 ? a / r : 1.0;
      sn[j] = r > 0 ? b / r : 0.0;
      hc[j] = r;
      hc[j + 1] = 0.0;
      gam[j + 1] = -sn[j] * gam[j];
      gam[j] = cs[j] * gam[j];
      est = std::fabs(gam[j + 1]);
      if (*rel1 < 0) *rel1 = est / gn;
      if (est <= tol * gn || !(r > 0)) {
        ++j;
        break;
      }
    }
    // y = H(0:j, 0:j)^{-1} gam(0:j); tau += Z y
    if (j > 0) {
      std::vector<double> y(j);
      for (int i = j - 1; i >= 0; --i) {
        double v = gam[i];
        for (int c = i + 1; c < j; ++c) v -= H[(size_t)c * (m + 1) + i] * y[c];
        y[i] = H[(size_t)i * (m + 1) + i] != 0.0 ? v / H[(size_t)i * (m + 1) + i] : 0.0;
      }
      double* hy = (double*)ctx_pinned(ctx, sizeof(double) * j);
      for (int i = 0; i < j; ++i) hy[i] = -y[i];
      HIP_CHECK(hipMemcpyAsync(f->gy.p, hy, sizeof(double) * j, hipMemcpyHostToDevice, s));
      ctx_pinned_used(ctx, s);
      launch_sub_xw(Z, N, N, j, f->gy.p, tau, N, 1, s);
    }
    // true residual r = g - A tau, its norm; restart from it if needed
    {
      PhaseTimer t(ctx, "a8_residual", 26.0 * (double)f->Nn * f->Nn, 0.0);
      launch_residual(f->d_new.p, f->Nn, g, tau, w, 1, f->part.p, nullptr, s, ctx->opt.resid_mode);
    }
    dot_to(w, w, nrm + 2);
    HIP_CHECK(hipMemcpyAsync(hb, nrm + 2, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    beta = std::sqrt(std::max(0.0, hb[0]));
    *rel = beta / gn;
    if (!(beta > tol * gn) || it >= maxit) break;
    launch_scale_rsqrt(w, N, nrm + 2, V, s);
  }
  return it;
}

void copy_nodes_out(const std::vector<NodeRec>& nd, double* xy, double* nrm, double* wts, int64_t* n_nodes) {
  if (!n_nodes) RW_THROW(RW_EINVAL, "n_nodes is null");
  const int64_t n = (int64_t)nd.size();
  if ((xy || nrm || wts) && *n_nodes < n) {
    *n_nodes = n;
    RW_THROW(RW_EINVAL, "node arrays too small");
  }
  for (int64_t i = 0; i < n && (xy || nrm || wts); ++i) {
    if (xy) { xy[2 * i] = nd[i].x; xy[2 * i + 1] = nd[i].y; }
    if (nrm) { nrm[2 * i] = nd[i].nx; nrm[2 * i + 1] = nd[i].ny; }
    if (wts) wts[i] = nd[i].w;
  }
  *n_nodes = n;
}

}  // namespace

// ================================================================ C ABI
extern "C" {

const char* rw_create_error(void) { return g_create_err.c_str(); }

int rw_ctx_create(rw_ctx** out, int device, void* hip_stream, size_t hbm_budget_bytes) {
  g_create_err.clear();
  if (!out) { g_create_err = "out is null"; return RW_EINVAL; }
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    g_create_err = "no HIP device available";
    return RW_EDEVICE;
  }
  if (device < 0 || device >= ndev) { g_create_err = "device index out of range"; return RW_EINVAL; }
  std::unique_ptr<rw_ctx> c(new rw_ctx());
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->budget = hbm_budget_bytes;
  c->opt.ir_tol = 1e-13;
  c->opt.ir_maxit = 6;
  c->opt.sketch_cols = 64;
  c->opt.seed = 0x5eedull;
  c->opt.app_dense_max_nodes = 1024;
  c->opt.far_field = 1;
  c->opt.test_singular = 0;
  c->opt.one_stream = 0;
  c->opt.resid_mode = RW_RESID_AUTO;
  c->opt.hbs_merge = 2;
  c->opt.solver = RW_SOLVE_IR;
  c->opt.gmres_restart = 30;
  c->opt.gmres_precond = 1;
  c->opt.mfma_from = 0;
  int rc = guarded(c.get(), [&]() {
    hipDeviceProp_t prop;
    HIP_CHECK(hipGetDeviceProperties(&prop, device));
    c->n_cu = prop.multiProcessorCount;
    c->sync_words = 256;
    c->d_sync = (unsigned*)dev_alloc(c.get(), sizeof(unsigned) * c->sync_words);
    HIP_CHECK(hipMemset(c->d_sync, 0, sizeof(unsigned) * c->sync_words));
    noalloc_scratch(device);   // this device's copy of the no-allocation scratch
  });
  if (rc != RW_OK) { g_create_err = c->err; return rc; }
  *out = c.release();
  return RW_OK;
}

void rw_ctx_destroy(rw_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->hbs_work.clear();   // workspaces from this ctx's allocator, released before its cache
  ctx_destroy_aux(ctx);
  if (ctx->d_sync) dev_free(ctx, ctx->d_sync, sizeof(unsigned) * ctx->sync_words);
  ctx_release_cache(ctx);
  for (auto& q : ctx->pending) { (void)hipEventDestroy(q.a); (void)hipEventDestroy(q.b); }
  for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
  for (auto e : ctx->order_events) (void)hipEventDestroy(e);
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  if (ctx->side2) (void)hipStreamDestroy(ctx->side2);
  for (auto st : ctx->bstreams) (void)hipStreamDestroy(st);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->rb) (void)hipHostFree(ctx->rb);
  if (ctx->hbs_pin) (void)hipHostFree(ctx->hbs_pin);
  if (ctx->pinned_ev) (void)hipEventDestroy(ctx->pinned_ev);
  if (ctx->defer_pin) (void)hipHostFree(ctx->defer_pin);
  delete ctx;
}

const char* rw_last_error(const rw_ctx* ctx) { return ctx ? ctx->err.c_str() : "null ctx"; }

int rw_set_options(rw_ctx* ctx, const rw_options* opt) {
  if (!ctx || !opt) return RW_EINVAL;
  return guarded(ctx, [&]() {
    if (!(opt->ir_tol >= 0) || opt->ir_maxit < 0 || opt->app_dense_max_nodes < 0)
      RW_THROW(RW_EINVAL, "bad refinement options");
    if (opt->test_singular < 0 || opt->test_singular > 2) RW_THROW(RW_EINVAL, "test_singular outside 0..2");
    if (opt->hbs_merge < 1 || opt->hbs_merge > 4) RW_THROW(RW_EINVAL, "hbs_merge outside 1..4");
    if (opt->solver != RW_SOLVE_IR && opt->solver != RW_SOLVE_GMRES) RW_THROW(RW_EINVAL, "unknown solver");
    if (opt->gmres_restart < 1 || opt->gmres_restart > 256) RW_THROW(RW_EINVAL, "gmres_restart outside 1..256");
    if (opt->mfma_from < 0) RW_THROW(RW_EINVAL, "mfma_from < 0");
    if (opt->one_stream != 0 && opt->one_stream != 1) RW_THROW(RW_EINVAL, "one_stream must be 0 or 1");
    if (opt->resid_mode < RW_RESID_AUTO || opt->resid_mode > RW_RESID_EXPAND) RW_THROW(RW_EINVAL, "unknown resid_mode");
    if (opt->sketch_cols != 32 && opt->sketch_cols != 64 && opt->sketch_cols != 96 && opt->sketch_cols != 128)
      RW_THROW(RW_EINVAL, "sketch_cols must be 32, 64, 96 or 128");
    ctx->opt = *opt;
  });
}

int rw_get_options(const rw_ctx* ctx, rw_options* opt) {
  if (!ctx || !opt) return RW_EINVAL;
  *opt = ctx->opt;
  return RW_OK;
}

size_t rw_ctx_bytes(const rw_ctx* ctx) { return ctx ? budget_used(ctx) : 0; }

int rw_ctx_trim(rw_ctx* ctx) {
  if (!ctx) return RW_EINVAL;
  return guarded(ctx, [&]() {
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    ctx_release_cache(ctx);
    if (ctx->aux) {
      HIP_CHECK(hipStreamSynchronize(ctx->aux->stream));
      ctx_release_cache(ctx->aux);
    }
  });
}

int rw_profile_enable(rw_ctx* ctx, int on) {
  if (!ctx) return RW_EINVAL;
  return guarded(ctx, [&]() {
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    prof_flush(ctx);
    ctx->prof = on != 0;
  });
}

int rw_profile_reset(rw_ctx* ctx) {
  if (!ctx) return RW_EINVAL;
  return guarded(ctx, [&]() {
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    prof_flush(ctx);
    ctx->phases.clear();
  });
}

int64_t rw_profile_json(rw_ctx* ctx, char* buf, int64_t len) {
  if (!ctx) return RW_EINVAL;
  std::string js = "{";
  bool first = true;
  (void)hipStreamSynchronize(ctx->stream);
  prof_flush(ctx);
  for (auto& kv : ctx->phases) {
    char tmp[512];
    snprintf(tmp, sizeof tmp, "%s\"%s\": {\"ms\": %.6f, \"calls\": %lld, \"flops\": %.6e, \"bytes\": %.6e}",
             first ? "" : ", ", kv.first.c_str(), kv.second.ms, (long long)kv.second.calls, kv.second.flops,
             kv.second.bytes);
    js += tmp;
    first = false;
  }
  js += "}";
  if (buf && len > 0) {
    const size_t n = std::min<size_t>(js.size(), (size_t)len - 1);
    memcpy(buf, js.data(), n);
    buf[n] = 0;
  }
  return (int64_t)js.size() + 1;
}

int rw_wall_build(rw_ctx* ctx, const rw_curve* curve, int32_t n_panels, int32_t order, int32_t leaf_nodes,
                  double id_tol, int32_t precision, rw_wall** out) {
  if (!ctx) return RW_EINVAL;
  return guarded(ctx, [&]() {
    if (!out || !curve) RW_THROW(RW_EINVAL, "null argument");
    *out = nullptr;
    if (order < 2 || order > 32) RW_THROW(RW_EINVAL, "order outside [2, 32]");
    if (n_panels < 2 || leaf_nodes < order || leaf_nodes % order) RW_THROW(RW_EINVAL, "bad panel / leaf sizes");
    if (!(id_tol > 0 && id_tol < 1)) RW_THROW(RW_EINVAL, "id_tol outside (0, 1)");
    if (precision != RW_F64 && precision != RW_F32 && precision != RW_BF16) RW_THROW(RW_EINVAL, "unknown precision");
    if (!(std::fabs(curve->a) < 1.0) || curve->m < 0) RW_THROW(RW_EINVAL, "curve must have |a| < 1, m >= 0");
    std::unique_ptr<rw_wall> w(new rw_wall());
    build_wall(ctx, *curve, n_panels, order, leaf_nodes, id_tol, precision, *w);
    *out = w.release();
  });
}

void rw_wall_free(rw_wall* w) {
  if (!w) return;
  (void)hipSetDevice(w->ctx->device);
  delete w;
}

int rw_wall_stats_get(const rw_wall* w, rw_wall_stats* st) {
  if (!w || !st) return RW_EINVAL;
  *st = w->stats;
  return RW_OK;
}

int rw_wall_nodes(const rw_wall* w, double* xy, double* nrm, double* wts, int64_t* n_nodes) {
  if (!w) return RW_EINVAL;
  return guarded(w->ctx, [&]() { copy_nodes_out(w->disc.nodes, xy, nrm, wts, n_nodes); });
}

int rw_hbs_apply(rw_wall* w, const double* b, int32_t nrhs, double* x) {
  if (!w) return RW_EINVAL;
  return guarded(w->ctx, [&]() {
    if (nrhs <= 0 || !b || !x) RW_THROW(RW_EINVAL, "bad arguments");
    const int64_t n2 = 2 * (int64_t)w->disc.nodes.size();
    hbs_apply(w, w->ctx, b, n2, x, n2, nrhs, w->precision);
    KERNEL_CHECK("hbs_apply");
  });
}

int rw_hbs_apply_noalloc(rw_wall* w, const double* b, double* x) {
  if (!w) return RW_EINVAL;
  rw_ctx* ctx = w->ctx;
  ctx->err.clear();
  try {
    if (!b || !x) RW_THROW(RW_EINVAL, "null b or x");
    HIP_CHECK(hipSetDevice(ctx->device));
    HbsWs1 plan;
    const int64_t need = hbs_ws1_plan(w->hbs, nullptr, plan);
    if (need > NOALLOC_DOUBLES)
      RW_THROW(RW_EINVAL, "the wall's one-RHS apply needs " + std::to_string(need) + " scratch doubles, above the " +
                              std::to_string(NOALLOC_DOUBLES) + " of rw_hbs_apply_noalloc");
    double* base = g_scratch_ptr[ctx->device];
    if (!base) RW_THROW(RW_EDEVICE, "no-allocation scratch not set up for this device");
    hbs_dev_apply1_at(w->hbs, b, x, w->precision, base, ctx->stream);
    KERNEL_CHECK("hbs_apply_noalloc");
    return RW_OK;
  } catch (const RwError& e) {
    ctx->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    ctx->err = e.what();
    return RW_EDEVICE;
  }
}

int rw_refine(rw_wall* w, const int32_t* ids, const int32_t* levels, int32_t n_sel, double q_tol,
              rw_refined** out) {
  if (!w) return RW_EINVAL;
  return guarded(w->ctx, [&]() {
    if (!out) RW_THROW(RW_EINVAL, "out is null");
    *out = nullptr;
    validate_selection(w, ids, levels, n_sel);
    if (!(q_tol < 1.0) || std::isnan(q_tol)) RW_THROW(RW_EINVAL, "q_tol must be below 1 (<= 0: the wall's id_tol)");
    std::vector<int32_t> lop(w->P, -1);
    for (int i = 0; i < n_sel; ++i) lop[ids[i]] = levels[i];
    std::unique_ptr<rw_refined> f(new rw_refined());
    f->q_tol = q_tol > 0 ? q_tol : w->tol;
    build_refined(w, w->ctx, lop, *f);
    *out = f.release();
  });
}

int rw_refine_on(rw_ctx* ctx, rw_wall* w, const int32_t* ids, const int32_t* levels, int32_t n_sel, double q_tol,
                 rw_refined** out) {
  if (!ctx || !w) return RW_EINVAL;
  return guarded(ctx, [&]() {
    if (!out) RW_THROW(RW_EINVAL, "out is null");
    *out = nullptr;
    if (ctx->device != w->ctx->device) RW_THROW(RW_EINVAL, "the ctx and the wall are on different devices");
    validate_selection(w, ids, levels, n_sel);
    if (!(q_tol < 1.0) || std::isnan(q_tol)) RW_THROW(RW_EINVAL, "q_tol must be below 1 (<= 0: the wall's id_tol)");
    std::vector<int32_t> lop(w->P, -1);
    for (int i = 0; i < n_sel; ++i) lop[ids[i]] = levels[i];
    std::unique_ptr<rw_refined> f(new rw_refined());
    f->q_tol = q_tol > 0 ? q_tol : w->tol;
    build_refined(w, ctx, lop, *f);
    *out = f.release();
  });
}

int rw_coarsen(rw_refined* f, const int32_t* ids, int32_t n_sel) {
  if (!f) return RW_EINVAL;
  return guarded(f->ctx, [&]() {
    if (n_sel < 0 || (n_sel > 0 && !ids)) RW_THROW(RW_EINVAL, "bad arguments");
    std::vector<int32_t> lop = f->level_of_panel;
    std::set<int32_t> seen;
    for (int i = 0; i < n_sel; ++i) {
      if (ids[i] < 0 || ids[i] >= f->wall->P || lop[ids[i]] < 0)
        RW_THROW(RW_EINVAL, "panel " + std::to_string(ids[i]) + " is not refined");
      if (!seen.insert(ids[i]).second) RW_THROW(RW_EINVAL, "duplicate panel id");
      lop[ids[i]] = -1;
    }
    std::unique_ptr<rw_refined> g(new rw_refined());
    g->q_tol = f->q_tol;
    build_refined(f->wall, f->ctx, lop, *g);
    std::swap(*f, *g);
    if (f->ctx->unsettled == g.get()) f->ctx->unsettled = f;
  });
}

void rw_refined_free(rw_refined* f) {
  if (!f) return;
  (void)hipSetDevice(f->ctx->device);
  refined_settle(f, true);
  delete f;
}

int rw_refined_info(const rw_refined* f, rw_info* info) {
  if (!f || !info) return RW_EINVAL;
  *info = f->info;
  return RW_OK;
}

int rw_nodes(const rw_refined* f, double* xy, double* nrm, double* wts, int64_t* n_nodes) {
  if (!f) return RW_EINVAL;
  return guarded(f->ctx, [&]() {
    // refined nodes in panel order (the device's node records of the refined discretization)
    std::vector<NodeRec> nd((size_t)f->Nn);
    if (f->Nn && (xy || nrm || wts)) {
      HIP_CHECK(hipMemcpyAsync(nd.data(), f->d_new.p, sizeof(NodeRec) * f->Nn, hipMemcpyDeviceToHost, f->ctx->stream));
      HIP_CHECK(hipStreamSynchronize(f->ctx->stream));
    }
    copy_nodes_out(nd, xy, nrm, wts, n_nodes);
  });
}

int rw_solve(rw_refined* f, const double* g, int32_t nrhs, double* tau, rw_solve_info* sinfo) {
  if (!f) return RW_EINVAL;
  if (sinfo) *sinfo = rw_solve_info{};
  int rc = guarded(f->ctx, [&]() {
    if (nrhs <= 0 || !g || !tau) RW_THROW(RW_EINVAL, "bad arguments");
    if (f->fail_rc != RW_OK) RW_THROW(f->fail_rc, f->fail_msg);
    const double t0 = wall_ms();
    hipStream_t s = f->ctx->stream;
    const rw_options& o = f->ctx->opt;
    if (o.solver == RW_SOLVE_GMRES) {
      const int64_t N = 2 * f->Nn;
      int its = 0;
      double worst = 0.0, worst1 = 0.0;
      for (int c = 0; c < nrhs; ++c) {
        double rel = 0.0, rel1 = 0.0;
        its += gmres_column(f, g + (size_t)c * N, tau + (size_t)c * N, o.ir_tol, std::max(1, o.ir_maxit), &rel,
                            &rel1);
        worst = std::max(worst, std::isfinite(rel) ? rel : INFINITY);
        worst1 = std::max(worst1, rel1);
      }
      prof_flush(f->ctx);
      f->info.ir_iters = its;
      f->info.resid = worst;
      f->info.t_solve_ms = wall_ms() - t0;
      if (sinfo) {
        sinfo->ir_iters = its;
        sinfo->k = f->k;
        sinfo->resid = worst;
        sinfo->resid_direct = worst1;
        sinfo->t_solve_ms = f->info.t_solve_ms;
      }
      if (!(worst <= o.ir_tol)) RW_THROW(RW_ENOCONV, "GMRES stopped at relative residual " + std::to_string(worst));
      return;
    }
    refined_ensure_ws(f, nrhs);
    woodbury_apply(f, g, tau, nrhs, false);
    int it = 0;
    double worst = 0;
    // read-back area: the latest norms, then those of the direct solution
    double* hn = (double*)ctx_readback(f->ctx, sizeof(double) * 4 * nrhs);
    double* hn0 = hn + 2 * nrhs;
    auto residual = [&]() {
      PhaseTimer t(f->ctx, "a8_residual", 26.0 * (double)f->Nn * f->Nn * nrhs, 0.0);
      launch_residual(f->d_new.p, f->Nn, g, tau, f->r.p, nrhs, f->part.p, f->norms.p, s, f->ctx->opt.resid_mode);
    };
    auto correct = [&]() {
      woodbury_apply(f, f->r.p, tau, nrhs, true);
      ++it;
      residual();
    };
    residual();
    // norms of the direct solution, copied out before a correction overwrites them
    HIP_CHECK(hipMemcpyAsync(hn0, f->norms.p, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, s));
    // the Woodbury solution takes at least one correction when refinement is
    // on: it is enqueued with its residual before anything is read back
    if (o.ir_maxit > 0) correct();
    for (;;) {
      HIP_CHECK(hipMemcpyAsync(hn, f->norms.p, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, s));
      HIP_CHECK(hipStreamSynchronize(s));
      // the refinement's own checks, if rw_refine returned before its end
      refined_settle(f);
      worst = 0;
      for (int c = 0; c < nrhs; ++c) {
        const double rel = hn[nrhs + c] > 0 ? std::sqrt(hn[c] / hn[nrhs + c]) : std::sqrt(hn[c]);
        worst = std::max(worst, std::isfinite(rel) ? rel : INFINITY);
      }
      if (worst <= o.ir_tol || it >= o.ir_maxit) break;
      correct();
    }
    prof_flush(f->ctx);
    f->info.ir_iters = it;
    f->info.resid = worst;
    f->info.t_solve_ms = wall_ms() - t0;
    if (sinfo) {
      double w0 = 0;
      for (int c = 0; c < nrhs; ++c) {
        const double rel = hn0[nrhs + c] > 0 ? std::sqrt(hn0[c] / hn0[nrhs + c]) : std::sqrt(hn0[c]);
        w0 = std::max(w0, std::isfinite(rel) ? rel : INFINITY);
      }
      sinfo->ir_iters = it;
      sinfo->k = f->k;
      sinfo->resid = worst;
      sinfo->resid_direct = w0;
      sinfo->t_solve_ms = f->info.t_solve_ms;
    }
    if (!(worst <= o.ir_tol) && o.ir_maxit > 0)
      RW_THROW(RW_ENOCONV, "refinement stopped at relative residual " + std::to_string(worst));
  });
  return rc;
}

namespace {

// Streams for the per-instance work of a batch (created on first use,
// non-blocking, default priority; destroyed with the ctx).
constexpr int BATCH_STREAMS = 4;
hipStream_t ctx_batch_stream(rw_ctx* ctx, int i) {
  if (ctx->opt.one_stream) return ctx->stream;
  if (ctx->bstreams.empty()) {
    ctx->bstreams.assign(BATCH_STREAMS, nullptr);
    for (auto& st : ctx->bstreams) HIP_CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  }
  return ctx->bstreams[i % BATCH_STREAMS];
}

// One sweep for several instances of one wall: each instance's Woodbury
// apply of src (eq. wood) followed by its exact residual r = g - A tau and
// the residual norms (into nrm, pinned host memory, 2 nrhs per instance).
// The reference-mesh parts of all applies are stacked into one multi-RHS
// apply of A_oo^{-1} on the ctx stream (the generators are streamed once
// for all of them); the per-instance work before and after it (extension,
// A_pp^{-1}, R y, W^{-1} z, X w, residual) runs on BATCH_STREAMS streams
// side by side, instance i on stream i mod BATCH_STREAMS.
void batch_sweep(rw_wall* w, const std::vector<rw_refined*>& fs, const std::vector<const double*>& src,
                 const std::vector<double*>& dst, const std::vector<const double*>& g, const std::vector<int>& nr,
                 bool accumulate, double* nrm) {
  rw_ctx* ctx = w->ctx;
  hipStream_t s = ctx->stream;
  const int64_t Mo = 2 * (int64_t)w->disc.nodes.size();
  const int nst = std::min<int>(BATCH_STREAMS, (int)fs.size());
  int64_t C = 0;
  for (size_t i = 0; i < fs.size(); ++i) C += nr[i];
  w->bat_in.ensure(ctx, (size_t)(Mo * C));
  w->bat_out.ensure(ctx, (size_t)(Mo * C));
  for (int q = 0; q < nst; ++q) stream_after(ctx, ctx_batch_stream(ctx, q), s, 10);
  int64_t c0 = 0;
  for (size_t i = 0; i < fs.size(); ++i) {
    const hipStream_t si = ctx_batch_stream(ctx, (int)i);
    const int64_t M = 2 * fs[i]->Next;
    woodbury_in(fs[i], src[i], nr[i], si);
    HIP_CHECK(hipMemcpy2DAsync(w->bat_in.p + c0 * Mo, sizeof(double) * Mo, fs[i]->gext.p, sizeof(double) * M,
                               sizeof(double) * Mo, nr[i], hipMemcpyDeviceToDevice, si));
    c0 += nr[i];
  }
  for (int q = 0; q < nst; ++q) stream_after(ctx, s, ctx_batch_stream(ctx, q), 11);
  {
    const double gb = gen_width(w) * w->stats.gen_entries;
    PhaseTimer t(ctx, "a6_hbs_apply", 2.0 * w->stats.gen_entries * C,
                 gb * hbs_gen_passes((int)C, w->precision != RW_F64));
    hbs_apply(w, ctx, w->bat_in.p, Mo, w->bat_out.p, Mo, (int)C, w->precision);
  }
  for (int q = 0; q < nst; ++q) stream_after(ctx, ctx_batch_stream(ctx, q), s, 12);
  c0 = 0;
  int64_t n0 = 0;
  for (size_t i = 0; i < fs.size(); ++i) {
    rw_refined* f = fs[i];
    const hipStream_t si = ctx_batch_stream(ctx, (int)i);
    const int64_t M = 2 * f->Next;
    HIP_CHECK(hipMemcpy2DAsync(f->y.p, sizeof(double) * M, w->bat_out.p + c0 * Mo, sizeof(double) * Mo,
                               sizeof(double) * Mo, nr[i], hipMemcpyDeviceToDevice, si));
    c0 += nr[i];
    woodbury_out(f, dst[i], nr[i], accumulate, false, si);
    {
      PhaseTimer t(ctx, "a8_residual", 26.0 * (double)f->Nn * f->Nn * nr[i], 0.0, si);
      launch_residual(f->d_new.p, f->Nn, g[i], dst[i], f->r.p, nr[i], f->part.p, f->norms.p, si, ctx->opt.resid_mode);
    }
    HIP_CHECK(hipMemcpyAsync(nrm + n0, f->norms.p, sizeof(double) * 2 * nr[i], hipMemcpyDeviceToHost, si));
    n0 += 2 * nr[i];
  }
  for (int q = 0; q < nst; ++q) stream_after(ctx, s, ctx_batch_stream(ctx, q), 13);
}

}  // namespace

int rw_solve_batch(rw_refined* const* inst, int32_t n_inst, const double* const* g, const int32_t* nrhs,
                   double* const* tau, rw_info* info) {
  if (!inst || n_inst <= 0 || !inst[0]) return RW_EINVAL;
  rw_refined* f0 = inst[0];
  return guarded(f0->ctx, [&]() {
    if (!g || !nrhs || !tau) RW_THROW(RW_EINVAL, "null array argument");
    rw_wall* w = f0->wall;
    std::set<const rw_refined*> seen;
    for (int i = 0; i < n_inst; ++i) {
      if (!inst[i] || inst[i]->wall != w) RW_THROW(RW_EINVAL, "instances must be refinements of one wall");
      if (inst[i]->ctx != w->ctx) RW_THROW(RW_EINVAL, "instances must be refined on the wall's ctx");
      if (!seen.insert(inst[i]).second) RW_THROW(RW_EINVAL, "an instance appears twice");
      if (nrhs[i] <= 0 || !g[i] || !tau[i]) RW_THROW(RW_EINVAL, "bad arguments of instance " + std::to_string(i));
    }
    const double t0 = wall_ms();
    hipStream_t s = f0->ctx->stream;
    const rw_options& o = f0->ctx->opt;
    std::vector<rw_refined*> fs(inst, inst + n_inst);
    std::vector<int> nr(nrhs, nrhs + n_inst);
    for (int i = 0; i < n_inst; ++i) refined_settle(fs[i]);
    for (int i = 0; i < n_inst; ++i) refined_ensure_ws(fs[i], nr[i]);
    int64_t tot_cols = 0;
    for (int i = 0; i < n_inst; ++i) tot_cols += nr[i];
    double* hn = (double*)ctx_readback(f0->ctx, sizeof(double) * 2 * tot_cols);
    std::vector<const double*> gv(g, g + n_inst);
    std::vector<double*> tv(tau, tau + n_inst);
    batch_sweep(w, fs, gv, tv, gv, nr, false, hn);
    std::vector<int> it(n_inst, 0);
    std::vector<double> worst(n_inst, 0.0);
    std::vector<char> active(n_inst, 1);
    std::vector<int> idx(n_inst);
    for (int i = 0; i < n_inst; ++i) idx[i] = i;
    for (;;) {
      HIP_CHECK(hipStreamSynchronize(s));
      // norms of the instances just swept (in the order they were passed)
      std::vector<rw_refined*> fa;
      std::vector<const double*> sa, ga;
      std::vector<double*> da;
      std::vector<int> na, ia;
      int64_t n0 = 0;
      for (int i : idx) {
        const double* hnv = hn + n0;
        n0 += 2 * nr[i];
        worst[i] = 0;
        for (int c = 0; c < nr[i]; ++c) {
          const double rel = hnv[nr[i] + c] > 0 ? std::sqrt(hnv[c] / hnv[nr[i] + c]) : std::sqrt(hnv[c]);
          worst[i] = std::max(worst[i], std::isfinite(rel) ? rel : INFINITY);
        }
        if (worst[i] <= o.ir_tol || it[i] >= o.ir_maxit) {
          active[i] = 0;
          continue;
        }
        fa.push_back(fs[i]);
        sa.push_back(fs[i]->r.p);
        da.push_back(tau[i]);
        ga.push_back(g[i]);
        na.push_back(nr[i]);
        ia.push_back(i);
        ++it[i];
      }
      if (fa.empty()) break;
      idx = ia;
      batch_sweep(w, fa, sa, da, ga, na, true, hn);
    }
    prof_flush(f0->ctx);
    const double tms = wall_ms() - t0;
    bool conv = true;
    for (int i = 0; i < n_inst; ++i) {
      fs[i]->info.ir_iters = it[i];
      fs[i]->info.resid = worst[i];
      fs[i]->info.t_solve_ms = tms;
      if (info) info[i] = fs[i]->info;
      if (!(worst[i] <= o.ir_tol) && o.ir_maxit > 0) conv = false;
    }
    if (!conv) RW_THROW(RW_ENOCONV, "refinement stopped above the tolerance for at least one instance");
  });
}

int rw_residual(rw_refined* f, const double* g, const double* tau, int32_t nrhs, double* r) {
  if (!f) return RW_EINVAL;
  return guarded(f->ctx, [&]() {
    if (nrhs <= 0 || !g || !tau || !r) RW_THROW(RW_EINVAL, "bad arguments");
    refined_settle(f);
    refined_ensure_ws(f, nrhs);
    launch_residual(f->d_new.p, f->Nn, g, tau, r, nrhs, f->part.p, nullptr, f->ctx->stream, f->ctx->opt.resid_mode);
  });
}

int rw_stokeslet_rhs(rw_refined* f, const double* z, const double* fv, int32_t n_src, double* g) {
  if (!f) return RW_EINVAL;
  return guarded(f->ctx, [&]() {
    if (n_src <= 0 || !z || !fv || !g) RW_THROW(RW_EINVAL, "bad arguments");
    std::vector<double> zf(4 * (size_t)n_src);
    for (int m = 0; m < n_src; ++m) {
      zf[4 * m] = z[2 * m];
      zf[4 * m + 1] = z[2 * m + 1];
      zf[4 * m + 2] = fv[2 * m];
      zf[4 * m + 3] = fv[2 * m + 1];
    }
    // through the pinned staging buffer: an upload from pageable memory would
    // wait for the work already on the stream (a refinement still running)
    hipStream_t s = f->ctx->stream;
    double* hz = (double*)ctx_pinned(f->ctx, sizeof(double) * zf.size());
    memcpy(hz, zf.data(), sizeof(double) * zf.size());
    DBuf<double> d(f->ctx, zf.size());
    HIP_CHECK(hipMemcpyAsync(d.p, hz, sizeof(double) * zf.size(), hipMemcpyHostToDevice, s));
    ctx_pinned_used(f->ctx, s);
    launch_stokeslet_rhs(f->d_new.p, f->Nn, d.p, n_src, g, s);
  });
}

}  // extern "C"
