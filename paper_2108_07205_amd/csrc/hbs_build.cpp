#include "hbs_build.h"

#include <algorithm>
#include <cmath>

#include "hostla.h"

namespace {

// 2x2 block of A = -1/2 I + D + N for target t and source s (w_s folded in).
inline void a_block(const NodeRec& t, const NodeRec& s, bool self, double B[4]) {
  if (self) {
    B[0] = s.s00; B[1] = s.s01; B[2] = s.s01; B[3] = s.s11;
    return;
  }
  const double rx = t.x - s.x, ry = t.y - s.y;
  const double r2 = rx * rx + ry * ry;
  const double c = (rx * s.nx + ry * s.ny) * s.w / (M_PI * r2 * r2);
  B[0] = c * rx * rx + s.w * t.nx * s.nx;
  B[1] = c * rx * ry + s.w * t.nx * s.ny;
  B[2] = c * ry * rx + s.w * t.ny * s.nx;
  B[3] = c * ry * ry + s.w * t.ny * s.ny;
}

inline double a_entry(const std::vector<NodeRec>& nd, int rdof, int cdof) {
  double B[4];
  const int i = rdof >> 1, j = cdof >> 1;
  a_block(nd[i], nd[j], i == j, B);
  return B[(rdof & 1) * 2 + (cdof & 1)];
}

// A(rows, cols) column-major (ld = rows.size()).
void a_sub(const std::vector<NodeRec>& nd, const std::vector<int>& rows, const std::vector<int>& cols,
           std::vector<double>& out) {
  const size_t m = rows.size();
  out.resize(m * cols.size());
  for (size_t c = 0; c < cols.size(); ++c)
    for (size_t r = 0; r < m; ++r) out[r + c * m] = a_entry(nd, rows[r], cols[c]);
}

struct CNode {
  int64_t n0 = 0, n1 = 0;  // node range [n0, n1)
  std::vector<int> candr, candc;
  int k = 0;
  std::vector<int> Jr, Jc;
  std::vector<double> U, V;  // m x k column-major
};

// Stokeslet S(x, p) (1/(4 pi)) (-log r I + r r^T / r^2), r = x - p.
inline void stokeslet(double rx, double ry, double S[4]) {
  const double r2 = rx * rx + ry * ry;
  const double a = -0.25 / M_PI * 0.5 * std::log(r2);
  const double b = 0.25 / M_PI / r2;
  S[0] = a + b * rx * rx;
  S[1] = b * rx * ry;
  S[2] = S[1];
  S[3] = a + b * ry * ry;
}

// Double layer D(x, y) with normal ny (unit weight), r = x - y.
inline void dlayer(double rx, double ry, double nx, double ny, double D[4]) {
  const double r2 = rx * rx + ry * ry;
  const double c = (rx * nx + ry * ny) / (M_PI * r2 * r2);
  D[0] = c * rx * rx;
  D[1] = c * rx * ry;
  D[2] = D[1];
  D[3] = c * ry * ry;
}

void compress_node(const std::vector<NodeRec>& nd, const HbsParams& prm, CNode& cn) {
  const int64_t N = (int64_t)nd.size();
  // proxy circle around the node's points
  double cx = 0, cy = 0;
  for (int64_t i = cn.n0; i < cn.n1; ++i) { cx += nd[i].x; cy += nd[i].y; }
  cx /= double(cn.n1 - cn.n0);
  cy /= double(cn.n1 - cn.n0);
  double R = 0;
  for (int64_t i = cn.n0; i < cn.n1; ++i) R = std::max(R, std::hypot(nd[i].x - cx, nd[i].y - cy));
  const double Rp = prm.proxy_ratio * R;
  std::vector<int> near;
  bool all_near = true;
  for (int64_t i = 0; i < N; ++i) {
    if (i >= cn.n0 && i < cn.n1) continue;
    if (std::hypot(nd[i].x - cx, nd[i].y - cy) < Rp) {
      near.push_back(2 * (int)i);
      near.push_back(2 * (int)i + 1);
    } else {
      all_near = false;
    }
  }
  const int np = all_near ? 0 : prm.n_proxy;
  std::vector<double> px(np), py(np), pnx(np), pny(np);
  for (int l = 0; l < np; ++l) {
    const double th = 2.0 * M_PI * l / np;
    pnx[l] = std::cos(th);
    pny[l] = std::sin(th);
    px[l] = cx + Rp * pnx[l];
    py[l] = cy + Rp * pny[l];
  }

  // ---- row ID: rows = candr, columns = [near | Stokeslet proxies | DLP proxies | n]
  const double wp = np ? 2.0 * M_PI * Rp / np : 0.0;  // proxy-circle quadrature weight
  const int m_r = (int)cn.candr.size();
  const int ncol = (int)near.size() + (np ? 4 * np + 1 : 0);
  std::vector<double> MrT((size_t)ncol * m_r);  // transposed: column i = row i of M_r
  for (int i = 0; i < m_r; ++i) {
    const int rd = cn.candr[i], a = rd >> 1, ca = rd & 1;
    double* col = MrT.data() + (size_t)i * ncol;
    for (size_t q = 0; q < near.size(); ++q) col[q] = a_entry(nd, rd, near[q]);
    if (np) {
      double* pc = col + near.size();
      for (int l = 0; l < np; ++l) {
        double S[4], D[4];
        const double rx = nd[a].x - px[l], ry = nd[a].y - py[l];
        stokeslet(rx, ry, S);
        dlayer(rx, ry, pnx[l], pny[l], D);
        pc[2 * l] = S[ca * 2 + 0];
        pc[2 * l + 1] = S[ca * 2 + 1];
        pc[2 * np + 2 * l] = wp * D[ca * 2 + 0];
        pc[2 * np + 2 * l + 1] = wp * D[ca * 2 + 1];
      }
      pc[4 * np] = ca ? nd[a].ny : nd[a].nx;
    }
  }
  // ---- column ID: columns = candc, rows = [near | DLP at proxies (2 comps) | flux]
  const int m_c = (int)cn.candc.size();
  const int nrow = (int)near.size() + (np ? 2 * np + 1 : 0);
  std::vector<double> Mc((size_t)nrow * m_c);
  for (int j = 0; j < m_c; ++j) {
    const int cd = cn.candc[j], b = cd >> 1, cb = cd & 1;
    double* col = Mc.data() + (size_t)j * nrow;
    for (size_t q = 0; q < near.size(); ++q) col[q] = a_entry(nd, near[q], cd);
    if (np) {
      double* pc = col + near.size();
      for (int l = 0; l < np; ++l) {
        double D[4];
        dlayer(px[l] - nd[b].x, py[l] - nd[b].y, nd[b].nx, nd[b].ny, D);
        pc[2 * l] = nd[b].w * D[0 * 2 + cb];
        pc[2 * l + 1] = nd[b].w * D[1 * 2 + cb];
      }
      pc[2 * np] = nd[b].w * (cb ? nd[b].ny : nd[b].nx);
    }
  }
  std::vector<double> MrT_keep = MrT, Mc_keep = Mc;
  Cpqr fr = hcpqr(ncol, m_r, MrT, prm.tol, 0);
  Cpqr fc = hcpqr(nrow, m_c, Mc, prm.tol, 0);
  int k = std::max(fr.k_tol, fc.k_tol);
  k = std::min(k, std::min(m_r, m_c));
  if (fr.steps < k) { MrT = MrT_keep; fr = hcpqr(ncol, m_r, MrT, prm.tol, k); }
  if (fc.steps < k) { Mc = Mc_keep; fc = hcpqr(nrow, m_c, Mc, prm.tol, k); }
  k = std::min(k, std::min(fr.steps, fc.steps));
  cn.k = k;
  auto interp = [&](const Cpqr& f, int m, std::vector<double>& P) {
    std::vector<double> T = cpqr_interp(f, m, k);
    P.assign((size_t)m * k, 0.0);
    for (int i = 0; i < k; ++i) P[f.perm[i] + (size_t)i * m] = 1.0;
    for (int q = 0; q < m - k; ++q)
      for (int i = 0; i < k; ++i) P[f.perm[k + q] + (size_t)i * m] = T[i + (size_t)q * k];
  };
  interp(fr, m_r, cn.U);
  interp(fc, m_c, cn.V);
  cn.Jr.resize(k);
  cn.Jc.resize(k);
  for (int i = 0; i < k; ++i) {
    cn.Jr[i] = cn.candr[fr.perm[i]];
    cn.Jc[i] = cn.candc[fc.perm[i]];
  }
}

}  // namespace

void hbs_build_inverse(const std::vector<NodeRec>& nd, const HbsParams& prm, HbsInverse& out) {
  const int64_t N = (int64_t)nd.size();
  if (prm.leaf_nodes < 1 || N < 2) RW_THROW(RW_EINVAL, "HBS tree needs at least two nodes");
  // 2^L leaves of floor or ceil(N / 2^L) <= leaf_nodes consecutive nodes:
  // node j of binary depth d covers [(j N) >> d, ((j + 1) N) >> d), so the
  // ranges nest whatever N
  int L = 1;
  while (((N + (int64_t(1) << L) - 1) >> L) > prm.leaf_nodes) ++L;
  if ((int64_t(1) << L) > N) RW_THROW(RW_EINVAL, "HBS leaves would be empty");
  if (prm.merge < 1 || prm.merge > 4) RW_THROW(RW_EINVAL, "HBS merge outside [1, 4]");
  // tree levels t = 0 (root) .. T (leaves) at binary depths dep[t]: a node
  // at level t covers N / 2^dep[t] nodes and has 2^(dep[t+1] - dep[t])
  // children, contiguous in node order
  std::vector<int> dep;
  for (int d = L;; d = std::max(0, d - prm.merge)) {
    dep.push_back(d);
    if (d == 0) break;
  }
  std::reverse(dep.begin(), dep.end());
  const int T = (int)dep.size() - 1;
  out = HbsInverse();
  out.L = T;
  out.lev.resize(T + 1);
  std::vector<std::vector<CNode>> cn(T + 1);
  auto nchild = [&](int t) { return t < T ? (1 << (dep[t + 1] - dep[t])) : 0; };

  // ---- compression, leaves to level 1
  for (int t = T; t >= 1; --t) {
    const int64_t cnt = int64_t(1) << dep[t];
    const int B = nchild(t);
    cn[t].resize(cnt);
    parallel_for(cnt, [&](int64_t j) {
      CNode& c = cn[t][j];
      c.n0 = (j * N) >> dep[t];
      c.n1 = ((j + 1) * N) >> dep[t];
      if (t == T) {
        for (int64_t d = 2 * c.n0; d < 2 * c.n1; ++d) c.candr.push_back((int)d);
        c.candc = c.candr;
      } else {
        for (int b = 0; b < B; ++b) {
          const CNode& ch = cn[t + 1][B * j + b];
          c.candr.insert(c.candr.end(), ch.Jr.begin(), ch.Jr.end());
          c.candc.insert(c.candc.end(), ch.Jc.begin(), ch.Jc.end());
        }
      }
      compress_node(nd, prm, c);
    }, prm.threads);
  }

  // ---- inverse, leaves to root
  std::vector<std::vector<std::vector<double>>> Dhat(T + 1);
  for (int t = T; t >= 0; --t) {
    const int64_t cnt = int64_t(1) << dep[t];
    const int B = nchild(t);
    if (t >= 1) out.lev[t].resize(cnt);
    Dhat[t].resize(cnt);
    parallel_for(cnt, [&](int64_t j) {
      std::vector<double> Dm;
      int n;
      if (t == T) {
        const CNode& c = cn[t][j];
        n = (int)c.candr.size();
        a_sub(nd, c.candr, c.candc, Dm);
      } else {
        // children's D^ on the diagonal, A(J_r(a), J_c(b)) off it
        std::vector<int> off(B + 1, 0);
        for (int b = 0; b < B; ++b) off[b + 1] = off[b] + cn[t + 1][B * j + b].k;
        n = off[B];
        Dm.assign((size_t)n * n, 0.0);
        for (int a = 0; a < B; ++a) {
          const CNode& ca = cn[t + 1][B * j + a];
          for (int b = 0; b < B; ++b) {
            const CNode& cb = cn[t + 1][B * j + b];
            if (a == b) {
              const std::vector<double>& Da = Dhat[t + 1][B * j + a];
              for (int c = 0; c < ca.k; ++c)
                for (int r = 0; r < ca.k; ++r) Dm[off[a] + r + (size_t)(off[a] + c) * n] = Da[r + (size_t)c * ca.k];
            } else {
              for (int c = 0; c < cb.k; ++c)
                for (int r = 0; r < ca.k; ++r)
                  Dm[off[a] + r + (size_t)(off[b] + c) * n] = a_entry(nd, ca.Jr[r], cb.Jc[c]);
            }
          }
        }
      }
      if (hinv(n, Dm.data(), n)) RW_THROW(RW_ESINGULAR, "singular diagonal block in the HBS inverse");
      if (t == 0) {
        out.nroot = n;
        out.Groot = std::move(Dm);
        return;
      }
      const CNode& c = cn[t][j];
      const int k = c.k;
      // DinvU (n x k), VtDinv (k x n)
      std::vector<double> DinvU((size_t)n * k), VtDinv((size_t)k * n), S((size_t)k * k);
      hgemm('N', 'N', n, k, n, 1.0, Dm.data(), n, c.U.data(), n, 0.0, DinvU.data(), n);
      hgemm('T', 'N', k, n, n, 1.0, c.V.data(), n, Dm.data(), n, 0.0, VtDinv.data(), k);
      hgemm('N', 'N', k, k, n, 1.0, VtDinv.data(), k, c.U.data(), n, 0.0, S.data(), k);
      if (k > 0 && hinv(k, S.data(), k)) RW_THROW(RW_ESINGULAR, "singular V* D^-1 U in the HBS inverse");
      HbsNodeGen& g = out.lev[t][j];
      g.nin = n;
      g.k = k;
      g.E.assign((size_t)n * k, 0.0);
      g.Ft.assign((size_t)k * n, 0.0);
      hgemm('N', 'N', n, k, k, 1.0, DinvU.data(), n, S.data(), k, 0.0, g.E.data(), n);
      hgemm('N', 'N', k, n, k, 1.0, S.data(), k, VtDinv.data(), k, 0.0, g.Ft.data(), k);
      g.G = Dm;
      hgemm('N', 'N', n, n, k, -1.0, g.E.data(), n, VtDinv.data(), k, 1.0, g.G.data(), n);
      Dhat[t][j] = std::move(S);
    }, prm.threads);
  }
  out.max_rank = 0;
  out.entries = (int64_t)out.nroot * out.nroot;
  for (int t = 1; t <= T; ++t)
    for (auto& g : out.lev[t]) {
      out.max_rank = std::max(out.max_rank, g.k);
      out.entries += (int64_t)g.E.size() + (int64_t)g.Ft.size() + (int64_t)g.G.size();
    }
}

bool hbs_fold_top(HbsInverse& H, int max_root) {
  if (H.L < 2) return false;
  const std::vector<HbsNodeGen>& top = H.lev[1];
  int n = 0;
  for (const HbsNodeGen& g : top) n += g.nin;
  if (n > max_root) return false;
  // T = blockdiag(E_1) G_root blockdiag(F*_1) + blockdiag(G_1): the map from
  // the inputs of the level-1 nodes to their down-sweep outputs
  const int nr = H.nroot;
  std::vector<double> GF((size_t)nr * n, 0.0);   // G_root blockdiag(F*_1): nr x n
  {
    int c0 = 0, k0 = 0;
    for (const HbsNodeGen& g : top) {
      // columns c0 .. c0 + nin of GF = G_root(:, k0 .. k0 + k) F*_j
      hgemm('N', 'N', nr, g.nin, g.k, 1.0, H.Groot.data() + (size_t)k0 * nr, nr, g.Ft.data(), g.k, 0.0,
            GF.data() + (size_t)c0 * nr, nr);
      c0 += g.nin;
      k0 += g.k;
    }
  }
  std::vector<double> T((size_t)n * n, 0.0);
  {
    int r0 = 0, k0 = 0;
    for (const HbsNodeGen& g : top) {
      // rows r0 .. r0 + nin of T = E_j GF(k0 .. k0 + k, :)
      hgemm('N', 'N', g.nin, n, g.k, 1.0, g.E.data(), g.nin, GF.data() + k0, nr, 0.0, T.data() + r0, n);
      for (int c = 0; c < g.nin; ++c)
        for (int r = 0; r < g.nin; ++r) T[r0 + r + (size_t)(r0 + c) * n] += g.G[r + (size_t)c * g.nin];
      r0 += g.nin;
      k0 += g.k;
    }
  }
  for (const HbsNodeGen& g : top) H.entries -= (int64_t)(g.E.size() + g.Ft.size() + g.G.size());
  H.entries += (int64_t)n * n - (int64_t)nr * nr;
  H.Groot = std::move(T);
  H.nroot = n;
  H.lev.erase(H.lev.begin() + 1);
  H.L -= 1;
  return true;
}
