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

void discretize(double a, int m, int order, const std::vector<double>& gl_s,
                const std::vector<double>& gl_w, std::vector<Panel> panels, Discretization& out) {
  out.order = order;
  out.panels = std::move(panels);
  out.nodes.resize(out.panels.size() * order);
  // theta_j = mid + d_j with d_j = half * s_j: cos / sin of theta_j and of
  // m theta_j by the angle-addition formulas from those of mid (per panel)
  // and of d_j (per panel width: refined children share it), so that the
  // trigonometric calls are per panel, not per node.  The results differ
  // from direct evaluation by a few units in the last place.
  std::vector<double> cd(order), sd(order), cmd(order), smd(order);
  double half_done = -1.0;
  for (size_t p = 0; p < out.panels.size(); ++p) {
    const double ta = out.panels[p].ta, tb = out.panels[p].tb;
    const double half = 0.5 * (tb - ta), mid = 0.5 * (tb + ta);
    if (!(std::fabs(half - half_done) <= 1e-15 * half)) {
      for (int j = 0; j < order; ++j) {
        const double d = half * gl_s[j];
        cd[j] = std::cos(d);
        sd[j] = std::sin(d);
        cmd[j] = std::cos(m * d);
        smd[j] = std::sin(m * d);
      }
      half_done = half;
    }
    const double cm = std::cos(mid), sm = std::sin(mid);
    const double cmm = std::cos(m * mid), smm = std::sin(m * mid);
    for (int j = 0; j < order; ++j) {
      const double c = cm * cd[j] - sm * sd[j], s = sm * cd[j] + cm * sd[j];
      const double cmt = cmm * cmd[j] - smm * smd[j], smt = smm * cmd[j] + cmm * smd[j];
      const double r = 1.0 + a * cmt;
      const double r1 = -a * m * smt;
      const double r2 = -a * m * m * cmt;
      const double x1 = r1 * c - r * s, y1 = r1 * s + r * c;                  // gamma'
      const double x2 = r2 * c - 2.0 * r1 * s - r * c, y2 = r2 * s + 2.0 * r1 * c - r * s;  // gamma''
      const double sp = std::sqrt(x1 * x1 + y1 * y1), isp = 1.0 / sp;
      const double tx = x1 * isp, ty = y1 * isp;
      const double nx = ty, ny = -tx;
      const double kap = (x1 * y2 - y1 * x2) * (isp * isp * isp);
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
