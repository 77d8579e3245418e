// Star-curve panel discretization and local refinement bookkeeping
// (Sec. 2.1 Nystrom discretization; Sec. 3.1 index sets I_k, I_c, I_p).
#pragma once

#include <cstdint>
#include <vector>

#include "common.h"

// Gauss-Legendre rule on [-1, 1] by Newton's method on P_q (Golub-Welsch
// would do as well); nodes ascending.
void gauss_legendre(int q, std::vector<double>& s, std::vector<double>& w);

struct Panel {
  double ta, tb;      // parameter interval
  int32_t ref_id;     // reference panel it lies in
  int32_t added;      // 1 if it is a child of a refined panel (I_p), else 0 (I_k)
};

struct Discretization {
  std::vector<Panel> panels;
  std::vector<NodeRec> nodes;   // order * panels.size() records
  int order = 16;
  int64_t n() const { return (int64_t)nodes.size(); }
};

// gamma(theta) = (1 + a cos(m theta)) (cos theta, sin theta): node records
// (position, outward normal, weight w = w_GL (dtheta/2) |gamma'|, self block).
void discretize(double a, int m, int order, const std::vector<double>& gl_s,
                const std::vector<double>& gl_w, std::vector<Panel> panels, Discretization& out);

std::vector<Panel> reference_panels(int n_panels);

// Refined panel list: each selected reference panel replaced by 2^level
// equal-parameter children, in parameter order.
std::vector<Panel> refined_panels(int n_panels, const std::vector<int32_t>& level_of_panel);
