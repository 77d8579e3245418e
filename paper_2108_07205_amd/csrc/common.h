// Shared definitions of the refined-wall library: error handling, the ctx
// object, device-memory accounting and the packed node record the kernels
// read.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <functional>
#include <map>
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

struct rw_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;   // 0 = unlimited
  size_t used = 0;     // bytes held (in use + cached)
  std::string err;
  rw_options opt{};
  int n_cu = 0;
  unsigned* d_sync = nullptr;   // grid-barrier / flag scratch owned by the ctx
  size_t sync_words = 0;
  // caching allocator: freed blocks are kept by size for reuse
  std::multimap<size_t, void*> cache;
  size_t cached = 0;
  // phase profiler (HIP events on `stream`)
  bool prof = false;
  struct Pending { std::string name; hipEvent_t a, b; double flops, bytes; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  std::map<std::string, PhaseStat> phases;
};

// Records a HIP event pair around a phase when the ctx profiler is on; the
// elapsed time is folded into ctx->phases at the next prof_flush().
struct PhaseTimer {
  rw_ctx* ctx;
  rw_ctx::Pending p{};
  bool on;
  PhaseTimer(rw_ctx* c, const char* name, double flops = 0.0, double bytes = 0.0);
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
  KernelTimer(const char* name, double flops, double bytes);
  ~KernelTimer();
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
