// Reuse of refinements across time steps (Sec. 5.3: several snapshots can
// use the same refinement).  In a time-stepping loop the region to refine
// (the panels near a particle) moves little from one snapshot to the next.
// The cache keeps refinements of one wall, each with its factors (Q ~= L R,
// A_pp^{-1}, X, W^{-1}), and serves a request with any cached refinement
// that covers it: every requested panel refined at least as deep.  A miss
// refines the requested panels widened by `margin` panels on both sides of
// every contiguous run (at the run's deepest requested level), so that the
// next snapshots, whose regions have moved by less than the margin, hit.
// Nearby runs whose widened ranges touch merge into one refined region.
// Least recently used refinements are freed when the cache is full.
#include <algorithm>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "rw.h"

namespace {

struct Entry {
  rw_refined* ref = nullptr;
  std::map<int32_t, int32_t> level;   // refined panel -> level
  uint64_t last_use = 0;
};

}  // namespace

struct rw_refcache {
  rw_wall* wall = nullptr;
  int32_t n_panels = 0, capacity = 1, margin = 0;
  double q_tol = 0.0;
  std::vector<Entry> entries;
  uint64_t clock = 0;
  int64_t hits = 0, misses = 0;
  std::string err;
};

namespace {

bool covers(const Entry& e, const int32_t* ids, const int32_t* levels, int n) {
  for (int i = 0; i < n; ++i) {
    auto it = e.level.find(ids[i]);
    if (it == e.level.end() || it->second < levels[i]) return false;
  }
  return true;
}

// The requested panels widened by `margin` on both sides (cyclically), each
// at the deepest requested level within `margin` panels of it.
std::map<int32_t, int32_t> widen(const int32_t* ids, const int32_t* levels, int n, int P, int margin) {
  std::map<int32_t, int32_t> out;
  for (int i = 0; i < n; ++i)
    for (int d = -margin; d <= margin; ++d) {
      const int32_t p = (int32_t)(((int64_t)ids[i] + d) % P + P) % P;
      auto it = out.find(p);
      if (it == out.end() || it->second < levels[i]) out[p] = levels[i];
    }
  return out;
}

thread_local std::string g_cache_err;

}  // namespace

extern "C" {

const char* rw_refcache_error(const rw_refcache* c) { return c ? c->err.c_str() : g_cache_err.c_str(); }

int rw_refcache_create(rw_wall* wall, int32_t n_panels, int32_t capacity, int32_t margin, double q_tol,
                       rw_refcache** out) {
  g_cache_err.clear();
  if (!wall || !out || n_panels < 1 || capacity < 1 || margin < 0 || margin >= n_panels) {
    g_cache_err = "bad arguments (wall, n_panels >= 1, capacity >= 1, 0 <= margin < n_panels)";
    return RW_EINVAL;
  }
  std::unique_ptr<rw_refcache> c(new rw_refcache());
  c->wall = wall;
  c->n_panels = n_panels;
  c->capacity = capacity;
  c->margin = margin;
  c->q_tol = q_tol;
  *out = c.release();
  return RW_OK;
}

int rw_refcache_get(rw_refcache* c, const int32_t* ids, const int32_t* levels, int32_t n_sel, rw_refined** out,
                    int32_t* hit) {
  if (!c || !out || n_sel < 0 || (n_sel > 0 && (!ids || !levels))) return RW_EINVAL;
  for (int i = 0; i < n_sel; ++i)
    if (ids[i] < 0 || ids[i] >= c->n_panels || levels[i] < 0 || levels[i] > 8) {
      c->err = "panel id or level out of range";
      return RW_EINVAL;
    }
  *out = nullptr;
  ++c->clock;
  // the covering refinement refined least (fewest added nodes) serves it
  Entry* best = nullptr;
  int64_t best_nodes = 0;
  for (Entry& e : c->entries) {
    if (!covers(e, ids, levels, n_sel)) continue;
    int64_t added = 0;
    for (auto& kv : e.level) added += int64_t(1) << kv.second;
    if (!best || added < best_nodes) {
      best = &e;
      best_nodes = added;
    }
  }
  if (best) {
    best->last_use = c->clock;
    ++c->hits;
    *out = best->ref;
    if (hit) *hit = 1;
    return RW_OK;
  }
  ++c->misses;
  const std::map<int32_t, int32_t> lv = widen(ids, levels, n_sel, c->n_panels, c->margin);
  std::vector<int32_t> wi, wl;
  for (auto& kv : lv) {
    wi.push_back(kv.first);
    wl.push_back(kv.second);
  }
  if ((int)c->entries.size() >= c->capacity) {
    auto lru = std::min_element(c->entries.begin(), c->entries.end(),
                                [](const Entry& a, const Entry& b) { return a.last_use < b.last_use; });
    rw_refined_free(lru->ref);
    c->entries.erase(lru);
  }
  Entry e;
  const int rc = rw_refine(c->wall, wi.data(), wl.data(), (int32_t)wi.size(), c->q_tol, &e.ref);
  if (rc != RW_OK) {
    c->err = "refinement of the widened region failed";
    return rc;
  }
  e.level = lv;
  e.last_use = c->clock;
  c->entries.push_back(std::move(e));
  *out = c->entries.back().ref;
  if (hit) *hit = 0;
  return RW_OK;
}

int rw_refcache_panels(const rw_refcache* c, const rw_refined* ref, int32_t* ids, int32_t* levels, int32_t* n) {
  if (!c || !ref || !n) return RW_EINVAL;
  for (const Entry& e : c->entries) {
    if (e.ref != ref) continue;
    const int32_t cnt = (int32_t)e.level.size();
    if (ids && levels) {
      if (*n < cnt) {
        *n = cnt;
        return RW_EINVAL;
      }
      int i = 0;
      for (auto& kv : e.level) {
        ids[i] = kv.first;
        levels[i] = kv.second;
        ++i;
      }
    }
    *n = cnt;
    return RW_OK;
  }
  return RW_EINVAL;
}

void rw_refcache_stats(const rw_refcache* c, int64_t* hits, int64_t* misses, int32_t* held) {
  if (!c) return;
  if (hits) *hits = c->hits;
  if (misses) *misses = c->misses;
  if (held) *held = (int32_t)c->entries.size();
}

void rw_refcache_destroy(rw_refcache* c) {
  if (!c) return;
  for (Entry& e : c->entries) rw_refined_free(e.ref);
  delete c;
}

}  // extern "C"
