// Request server for refined-wall solves against one resident wall: the
// time-stepping workflow of Sec. 5.3 (every snapshot refines some panels of
// the same wall, reuses the precomputed reference inverse and solves),
// served to many independent requests.
//
// Each of `slots` worker threads owns a ctx with a stream of its own and
// runs whole requests on it (rw_refine_on, Stokeslet data, rw_solve), so the
// device work of up to `slots` requests overlaps on the GPU; the wall's
// reference inverse and node data stay resident and are only read.  A
// request leaves the queue as soon as a slot is free and the device memory
// it is estimated to need fits the budget next to the requests in flight
// (first come, first served: a request that does not fit yet holds the
// queue until memory frees up; one that could never fit is rejected at
// submission).  Requests of any refinement size and right-hand-side count
// join and leave independently.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include <hip/hip_runtime.h>

#include "rw.h"

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
  int64_t id = 0;
  std::vector<int32_t> ids, levels;
  std::vector<double> z, f;   // nrhs * n_src x 2
  int n_src = 0, nrhs = 0;
  int64_t n_nodes = 0;        // refined nodes N_n
  size_t bytes = 0;           // estimated device memory
  double t_submit = 0, t_start = 0, t_done = 0;
  bool done = false;
  rw_request_info info{};
  std::vector<double> tau;    // 2 N_n x nrhs
};

}  // namespace

struct rw_server {
  rw_wall* wall = nullptr;
  rw_ctx* wctx = nullptr;
  int device = 0;
  int32_t n_panels = 0, order = 16;
  size_t budget = 0, in_flight = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<int64_t, std::shared_ptr<Request>> all;
  int64_t next_id = 1;
  bool stop = false;
  struct Slot {
    rw_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    double* g_dev = nullptr;
    double* tau_dev = nullptr;
    size_t cap = 0;               // doubles of g_dev / tau_dev
    double* pin = nullptr;        // pinned host staging for tau
    std::thread th;
  };
  std::vector<std::unique_ptr<Slot>> slots;
  std::string err;
};

namespace {

// Device bytes a request is taken to need while it runs: Q's factors and
// sketches (~3 x 96 columns of the extended length), the added arc's HBS
// inverse and its build (~600 doubles per added unknown), and the solve's
// vectors (~12 per unknown and right-hand side), plus a fixed part.
size_t estimate_bytes(int64_t n_ref_nodes, int64_t n_added, int64_t n_cut, int nrhs) {
  const double next = 2.0 * (double)(n_ref_nodes + n_added);
  const double nn = 2.0 * (double)(n_ref_nodes - n_cut + n_added);
  const double b = 8.0 * (next * 3.0 * 96.0 + 2.0 * (double)n_added * 600.0 + nn * 12.0 * nrhs) + 64.0 * (1 << 20);
  return (size_t)b;
}

void run_request(rw_server* sv, rw_server::Slot& sl, Request& q) {
  rw_ctx* c = sl.ctx;
  rw_refined* ref = nullptr;
  int rc = rw_refine_on(c, sv->wall, q.ids.data(), q.levels.data(), (int32_t)q.ids.size(), 0.0, &ref);
  if (rc == RW_OK) {
    rw_info ri{};
    rw_refined_info(ref, &ri);
    const int64_t n2 = 2 * (ri.n_k + ri.n_p);
    const size_t need = (size_t)n2 * q.nrhs;
    if (need > sl.cap) {
      if (sl.g_dev) (void)hipFree(sl.g_dev);
      if (sl.tau_dev) (void)hipFree(sl.tau_dev);
      if (sl.pin) (void)hipHostFree(sl.pin);
      sl.g_dev = sl.tau_dev = sl.pin = nullptr;
      sl.cap = 0;
      if (hipMalloc((void**)&sl.g_dev, need * sizeof(double)) != hipSuccess ||
          hipMalloc((void**)&sl.tau_dev, need * sizeof(double)) != hipSuccess ||
          hipHostMalloc((void**)&sl.pin, need * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        rc = RW_ENOMEM;
      } else {
        sl.cap = need;
      }
    }
    for (int r = 0; rc == RW_OK && r < q.nrhs; ++r)
      rc = rw_stokeslet_rhs(ref, q.z.data() + (size_t)r * q.n_src * 2, q.f.data() + (size_t)r * q.n_src * 2,
                            q.n_src, sl.g_dev + (size_t)r * n2);
    rw_solve_info si{};
    if (rc == RW_OK) {
      rc = rw_solve(ref, sl.g_dev, q.nrhs, sl.tau_dev, &si);
      q.info.ir_iters = si.ir_iters;
      q.info.k = si.k;
      q.info.resid = si.resid;
    }
    if (rc == RW_OK || rc == RW_ENOCONV) {
      if (hipMemcpyAsync(sl.pin, sl.tau_dev, need * sizeof(double), hipMemcpyDeviceToHost, sl.stream) != hipSuccess ||
          hipStreamSynchronize(sl.stream) != hipSuccess) {
        (void)hipGetLastError();
        rc = RW_EDEVICE;
      } else {
        q.tau.assign(sl.pin, sl.pin + need);
      }
    }
    q.info.n_nodes = ri.n_k + ri.n_p;
  }
  if (rc != RW_OK) {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->err.empty()) sv->err = std::string("request ") + std::to_string(q.id) + ": " + rw_last_error(c);
  }
  if (ref) rw_refined_free(ref);
  q.info.status = rc;
}

void slot_loop(rw_server* sv, int s) {
  rw_server::Slot& sl = *sv->slots[s];
  (void)hipSetDevice(sv->device);
  for (;;) {
    std::shared_ptr<Request> q;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv_work.wait(lk, [&] {
        return sv->stop || (!sv->queue.empty() && sv->in_flight + sv->queue.front()->bytes <= sv->budget);
      });
      if (sv->queue.empty() || !(sv->in_flight + sv->queue.front()->bytes <= sv->budget)) {
        if (sv->stop) return;
        continue;
      }
      q = sv->queue.front();
      sv->queue.pop_front();
      sv->in_flight += q->bytes;
      q->t_start = now_ms();
    }
    // another slot may fit the next request too
    sv->cv_work.notify_all();
    run_request(sv, sl, *q);
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->in_flight -= q->bytes;
      q->t_done = now_ms();
      q->info.slot = s;
      q->info.t_queue_ms = q->t_start - q->t_submit;
      q->info.t_run_ms = q->t_done - q->t_start;
      q->done = true;
    }
    sv->cv_done.notify_all();
    sv->cv_work.notify_all();
  }
}

void server_teardown(rw_server* sv) {
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  for (auto& sl : sv->slots)
    if (sl->th.joinable()) sl->th.join();
  for (auto& sl : sv->slots) {
    if (sl->ctx) rw_ctx_destroy(sl->ctx);
    if (sl->g_dev) (void)hipFree(sl->g_dev);
    if (sl->tau_dev) (void)hipFree(sl->tau_dev);
    if (sl->pin) (void)hipHostFree(sl->pin);
    if (sl->stream) (void)hipStreamDestroy(sl->stream);
  }
  sv->slots.clear();
}

thread_local std::string g_server_err;

}  // namespace

extern "C" {

const char* rw_server_error(const rw_server* sv) { return sv ? sv->err.c_str() : g_server_err.c_str(); }

int rw_server_create(rw_ctx* ctx, rw_wall* wall, int32_t n_panels, int32_t slots, size_t hbm_budget_bytes,
                     rw_server** out) {
  g_server_err.clear();
  if (!ctx || !wall || !out || slots < 1 || slots > 16 || n_panels < 1) {
    g_server_err = "bad arguments (ctx, wall, n_panels >= 1, 1 <= slots <= 16)";
    return RW_EINVAL;
  }
  *out = nullptr;
  rw_wall_stats st{};
  if (rw_wall_stats_get(wall, &st) != RW_OK || st.n_nodes % n_panels) {
    g_server_err = "n_panels does not match the wall";
    return RW_EINVAL;
  }
  std::unique_ptr<rw_server> sv(new rw_server());
  sv->wall = wall;
  sv->wctx = ctx;
  sv->n_panels = n_panels;
  sv->order = (int32_t)(st.n_nodes / n_panels);
  sv->budget = hbm_budget_bytes ? hbm_budget_bytes : ~size_t(0);
  if (hipGetDevice(&sv->device) != hipSuccess) {
    g_server_err = "no current HIP device";
    return RW_EDEVICE;
  }
  rw_options opt{};
  rw_get_options(ctx, &opt);
  // several slots: each request on its slot's one stream, so that the slots
  // overlap on separate hardware queues instead of a request's side streams
  // sharing queues with the other slots' work
  if (slots > 1) opt.one_stream = 1;
  for (int s = 0; s < slots; ++s) {
    std::unique_ptr<rw_server::Slot> sl(new rw_server::Slot());
    if (hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      server_teardown(sv.get());
      g_server_err = "hipStreamCreate failed";
      return RW_EDEVICE;
    }
    const int rc = rw_ctx_create(&sl->ctx, sv->device, sl->stream, 0);
    if (rc != RW_OK) {
      g_server_err = rw_create_error();
      sv->slots.push_back(std::move(sl));
      server_teardown(sv.get());
      return rc;
    }
    rw_set_options(sl->ctx, &opt);
    sv->slots.push_back(std::move(sl));
  }
  for (int s = 0; s < slots; ++s) sv->slots[s]->th = std::thread(slot_loop, sv.get(), s);
  *out = sv.release();
  return RW_OK;
}

int rw_server_submit(rw_server* sv, const int32_t* panel_ids, const int32_t* levels, int32_t n_sel,
                     const double* z_host, const double* f_host, int32_t n_src, int32_t nrhs, int64_t* id) {
  if (!sv || !id || n_sel < 0 || (n_sel > 0 && (!panel_ids || !levels)) || n_src < 1 || nrhs < 1 || !z_host ||
      !f_host)
    return RW_EINVAL;
  std::shared_ptr<Request> q = std::make_shared<Request>();
  q->ids.assign(panel_ids, panel_ids + n_sel);
  q->levels.assign(levels, levels + n_sel);
  int64_t added = 0;
  for (int i = 0; i < n_sel; ++i) {
    if (panel_ids[i] < 0 || panel_ids[i] >= sv->n_panels || levels[i] < 0 || levels[i] > 8) return RW_EINVAL;
    added += (int64_t)sv->order << levels[i];
  }
  const int64_t n_ref = (int64_t)sv->n_panels * sv->order;
  q->n_nodes = n_ref - (int64_t)n_sel * sv->order + added;
  q->bytes = estimate_bytes(n_ref, added, (int64_t)n_sel * sv->order, nrhs);
  if (q->bytes > sv->budget) {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->err = "request needs about " + std::to_string(q->bytes >> 20) + " MiB, above the server's budget";
    return RW_ENOMEM;
  }
  q->z.assign(z_host, z_host + (size_t)2 * n_src * nrhs);
  q->f.assign(f_host, f_host + (size_t)2 * n_src * nrhs);
  q->n_src = n_src;
  q->nrhs = nrhs;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    q->id = sv->next_id++;
    q->t_submit = now_ms();
    sv->all[q->id] = q;
    sv->queue.push_back(q);
    *id = q->id;
  }
  sv->cv_work.notify_all();
  return RW_OK;
}

int rw_server_wait(rw_server* sv, int64_t id, double* tau_host, int64_t cap, rw_request_info* info) {
  if (!sv) return RW_EINVAL;
  std::shared_ptr<Request> q;
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->all.find(id);
    if (it == sv->all.end()) return RW_EINVAL;
    q = it->second;
    sv->cv_done.wait(lk, [&] { return q->done; });
    sv->all.erase(it);
  }
  if (info) *info = q->info;
  if (tau_host) {
    if (cap < (int64_t)q->tau.size()) return RW_EINVAL;
    std::copy(q->tau.begin(), q->tau.end(), tau_host);
  }
  return q->info.status;
}

void rw_server_destroy(rw_server* sv) {
  if (!sv) return;
  {
    // requests still queued or running finish first
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_done.wait(lk, [&] {
      for (auto& kv : sv->all)
        if (!kv.second->done) return false;
      return true;
    });
  }
  server_teardown(sv);
  delete sv;
}

}  // extern "C"
