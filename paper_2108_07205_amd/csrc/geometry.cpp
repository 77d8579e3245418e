#include "geometry.h"

#include <atomic>
#include <chrono>
#include <exception>
#include <mutex>
#include <cmath>

void gauss_legendre(int q, std::vector<double>& s, std::vector<double>& w) {
  s.assign(q, 0.0);
  w.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    // Chebyshev-like initial guess for the i-th root (descending), refine by
    // Newton on the three-term recurrence.
    double x = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= q; ++k) {
        double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      if (q == 1) { p1 = x; p0 = 1.0; }
      dp = q * (x * p1 - p0) / (x * x - 1.0);
      double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) {
        // one more step for the derivative at the converged root
        p0 = 1.0; p1 = x;
        for (int k = 2; k <= q; ++k) {
          double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = pk;
        }
        dp = q * (x * p1 - p0) / (x * x - 1.0);
        break;
      }
    }
    s[q - 1 - i] = x;
    w[q - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
}

std::vector<Panel> reference_panels(int n_panels) {
  std::vector<Panel> p(n_panels);
  const double h = 2.0 * M_PI / n_panels;
  for (int i = 0; i < n_panels; ++i) p[i] = Panel{i * h, (i + 1) * h, i, 0};
  return p;
}

std::vector<Panel> refined_panels(int n_panels, const std::vector<int32_t>& level_of_panel) {
  std::vector<Panel> out;
  const double h = 2.0 * M_PI / n_panels;
  for (int i = 0; i < n_panels; ++i) {
    const double a = i * h, b = (i + 1) * h;
    const int lev = level_of_panel[i];
    if (lev < 0) {
      out.push_back(Panel{a, b, i, 0});
    } else {
      const int nch = 1 << lev;
      const double hc = (b - a) / nch;
      for (int j = 0; j < nch; ++j) out.push_back(Panel{a + j * hc, a + (j + 1) * hc, i, 1});
    }
  }
  return out;
}

// sin and cos of x for |x| < 1e-2 by their Taylor series (through x^9 and
// x^8: the first omitted terms are below 1e-26)
static inline void sincos_small(double x, double& s, double& c) {
  const double x2 = x * x;
  c = 1.0 + x2 * (-1.0 / 2 + x2 * (1.0 / 24 + x2 * (-1.0 / 720 + x2 * (1.0 / 40320))));
  s = x * (1.0 + x2 * (-1.0 / 6 + x2 * (1.0 / 120 + x2 * (-1.0 / 5040 + x2 * (1.0 / 362880)))));
}

// sin and cos of t = b + e given those of b (e = t - b, exact for t near b):
// angle addition with the small angle's by Taylor series, so that the
// library's sine and cosine are called per panel, not per node (within
// about one unit in the last place of direct evaluation)
static inline void sincos_near(double sb, double cb, double e, double& s, double& c) {
  double se, ce;
  if (std::fabs(e) < 1e-2) sincos_small(e, se, ce);
  else { se = std::sin(e); ce = std::cos(e); }
  c = std::fma(cb, ce, -(sb * se));
  s = std::fma(sb, ce, cb * se);
}

void discretize(double a, int m, int order, const std::vector<double>& gl_s,
                const std::vector<double>& gl_w, std::vector<Panel> panels, Discretization& out) {
  out.order = order;
  out.panels = std::move(panels);
  out.nodes.resize(out.panels.size() * order);
  for (size_t p = 0; p < out.panels.size(); ++p) {
    const double ta = out.panels[p].ta, tb = out.panels[p].tb;
    const double half = 0.5 * (tb - ta), mid = 0.5 * (tb + ta);
    const double smid = std::sin(mid), cmid = std::cos(mid);
    const double bm = m * mid, sbm = std::sin(bm), cbm = std::cos(bm);
    for (int j = 0; j < order; ++j) {
      const double th = mid + half * gl_s[j], tm = m * th;
      double s, c, smt, cmt;
      sincos_near(smid, cmid, th - mid, s, c);   // theta
      sincos_near(sbm, cbm, tm - bm, smt, cmt);  // m theta
      const double r = 1.0 + a * cmt;
      const double r1 = -a * m * smt;
      const double r2 = -a * m * m * cmt;
      const double x1 = r1 * c - r * s, y1 = r1 * s + r * c;                  // gamma'
      const double x2 = r2 * c - 2.0 * r1 * s - r * c, y2 = r2 * s + 2.0 * r1 * c - r * s;  // gamma''
      const double sp = std::sqrt(x1 * x1 + y1 * y1);
      const double tx = x1 / sp, ty = y1 / sp;
      const double nx = ty, ny = -tx;
      const double kap = (x1 * y2 - y1 * x2) / (sp * sp * sp);
      const double w = gl_w[j] * half * sp;
      const double dl = -kap / (2.0 * M_PI);
      NodeRec& nd = out.nodes[p * order + j];
      nd.x = r * c;
      nd.y = r * s;
      nd.nx = nx;
      nd.ny = ny;
      nd.w = w;
      nd.s00 = -0.5 + w * (dl * tx * tx + nx * nx);
      nd.s01 = w * (dl * tx * ty + nx * ny);
      nd.s11 = -0.5 + w * (dl * ty * ty + ny * ny);
    }
  }
}

void parallel_for(int64_t n, const std::function<void(int64_t)>& f, int threads) {
  if (n <= 0) return;
  if (threads <= 0) {
    unsigned hc = std::thread::hardware_concurrency();
    threads = hc ? (int)std::min<unsigned>(hc, 32u) : 4;
  }
  if (threads == 1 || n == 1) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int64_t> next{0};
  std::vector<std::thread> pool;
  std::exception_ptr eptr = nullptr;
  std::mutex emu;
  const int nt = (int)std::min<int64_t>(threads, n);
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&]() {
      for (;;) {
        int64_t i = next.fetch_add(1);
        if (i >= n) break;
        try {
          f(i);
        } catch (...) {
          std::lock_guard<std::mutex> lk(emu);
          if (!eptr) eptr = std::current_exception();
        }
      }
    });
  for (auto& th : pool) th.join();
  if (eptr) std::rethrow_exception(eptr);
}

double wall_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}
