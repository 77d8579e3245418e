#include "hostla.h"

#include <algorithm>
#include <cmath>

void hgemm(char ta, char tb, int m, int n, int k, double alpha, const double* A, int lda,
           const double* B, int ldb, double beta, double* C, int ldc) {
  for (int j = 0; j < n; ++j) {
    double* c = C + (size_t)j * ldc;
    if (beta == 0.0)
      for (int i = 0; i < m; ++i) c[i] = 0.0;
    else if (beta != 1.0)
      for (int i = 0; i < m; ++i) c[i] *= beta;
  }
  if (ta == 'N') {
    // c(:, j) += alpha * sum_l A(:, l) op(B)(l, j): unit-stride inner loop
    for (int j = 0; j < n; ++j) {
      double* c = C + (size_t)j * ldc;
      for (int l = 0; l < k; ++l) {
        const double b = alpha * (tb == 'N' ? B[l + (size_t)j * ldb] : B[j + (size_t)l * ldb]);
        if (b == 0.0) continue;
        const double* a = A + (size_t)l * lda;
        for (int i = 0; i < m; ++i) c[i] += a[i] * b;
      }
    }
  } else {
    // c(i, j) += alpha * dot(A(:, i), op(B)(:, j))
    std::vector<double> bcol(k);
    for (int j = 0; j < n; ++j) {
      for (int l = 0; l < k; ++l) bcol[l] = (tb == 'N' ? B[l + (size_t)j * ldb] : B[j + (size_t)l * ldb]);
      double* c = C + (size_t)j * ldc;
      for (int i = 0; i < m; ++i) {
        const double* a = A + (size_t)i * lda;
        double s = 0.0;
        for (int l = 0; l < k; ++l) s += a[l] * bcol[l];
        c[i] += alpha * s;
      }
    }
  }
}

int hlu(int n, double* A, int lda, int* piv) {
  for (int j = 0; j < n; ++j) {
    int p = j;
    double best = std::fabs(A[j + (size_t)j * lda]);
    for (int i = j + 1; i < n; ++i) {
      double v = std::fabs(A[i + (size_t)j * lda]);
      if (v > best) { best = v; p = i; }
    }
    piv[j] = p;
    if (!(best > 0.0) || !std::isfinite(best)) return j + 1;
    if (p != j)
      for (int c = 0; c < n; ++c) std::swap(A[j + (size_t)c * lda], A[p + (size_t)c * lda]);
    const double inv = 1.0 / A[j + (size_t)j * lda];
    for (int i = j + 1; i < n; ++i) A[i + (size_t)j * lda] *= inv;
    for (int c = j + 1; c < n; ++c) {
      const double u = A[j + (size_t)c * lda];
      if (u == 0.0) continue;
      double* col = A + (size_t)c * lda;
      const double* l = A + (size_t)j * lda;
      for (int i = j + 1; i < n; ++i) col[i] -= l[i] * u;
    }
  }
  return 0;
}

void hlu_solve(int n, int nrhs, const double* LU, int lda, const int* piv, double* B, int ldb) {
  for (int r = 0; r < nrhs; ++r) {
    double* b = B + (size_t)r * ldb;
    for (int j = 0; j < n; ++j)
      if (piv[j] != j) std::swap(b[j], b[piv[j]]);
    for (int j = 0; j < n; ++j) {
      const double v = b[j];
      if (v == 0.0) continue;
      const double* l = LU + (size_t)j * lda;
      for (int i = j + 1; i < n; ++i) b[i] -= l[i] * v;
    }
    for (int j = n - 1; j >= 0; --j) {
      b[j] /= LU[j + (size_t)j * lda];
      const double v = b[j];
      if (v == 0.0) continue;
      const double* u = LU + (size_t)j * lda;
      for (int i = 0; i < j; ++i) b[i] -= u[i] * v;
    }
  }
}

int hinv(int n, double* A, int lda) {
  std::vector<double> LU((size_t)n * n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) LU[i + (size_t)j * n] = A[i + (size_t)j * lda];
  std::vector<int> piv(n);
  int info = hlu(n, LU.data(), n, piv.data());
  if (info) return info;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) A[i + (size_t)j * lda] = (i == j) ? 1.0 : 0.0;
  hlu_solve(n, n, LU.data(), n, piv.data(), A, lda);
  return 0;
}

Cpqr hcpqr(int r, int c, std::vector<double>& A, double tol, int min_steps) {
  Cpqr f;
  f.perm.resize(c);
  for (int j = 0; j < c; ++j) f.perm[j] = j;
  const int kmax = std::min(r, c);
  std::vector<double> nrm(c), nrm0(c);
  for (int j = 0; j < c; ++j) {
    double s = 0.0;
    const double* col = A.data() + (size_t)j * r;
    for (int i = 0; i < r; ++i) s += col[i] * col[i];
    nrm[j] = nrm0[j] = std::sqrt(s);
  }
  double r00 = 0.0;
  bool rank_found = false;
  std::vector<double> v(r);
  int j = 0;
  for (; j < kmax; ++j) {
    int p = j;
    for (int i = j + 1; i < c; ++i)
      if (nrm[i] > nrm[p]) p = i;
    if (p != j) {
      std::swap_ranges(A.begin() + (size_t)j * r, A.begin() + (size_t)(j + 1) * r, A.begin() + (size_t)p * r);
      std::swap(nrm[j], nrm[p]);
      std::swap(nrm0[j], nrm0[p]);
      std::swap(f.perm[j], f.perm[p]);
    }
    double* aj = A.data() + (size_t)j * r;
    double s = 0.0;
    for (int i = j; i < r; ++i) s += aj[i] * aj[i];
    const double alpha_abs = std::sqrt(s);
    if (j == 0) r00 = alpha_abs;
    if (!rank_found && !(alpha_abs > tol * r00)) {
      rank_found = true;
      f.k_tol = j;
    }
    if (rank_found && j >= min_steps) break;
    if (alpha_abs == 0.0) {
      // remaining columns are exactly zero: no further pivot exists
      if (!rank_found) { rank_found = true; f.k_tol = j; }
      break;
    }
    const double alpha = (aj[j] > 0) ? -alpha_abs : alpha_abs;
    // v = a - alpha e_j, beta = 2 / (v^T v)
    for (int i = j; i < r; ++i) v[i] = aj[i];
    v[j] -= alpha;
    double vv = 0.0;
    for (int i = j; i < r; ++i) vv += v[i] * v[i];
    const double beta = (vv > 0) ? 2.0 / vv : 0.0;
    aj[j] = alpha;
    for (int i = j + 1; i < r; ++i) aj[i] = 0.0;
    for (int q = j + 1; q < c; ++q) {
      double* aq = A.data() + (size_t)q * r;
      double d = 0.0;
      for (int i = j; i < r; ++i) d += v[i] * aq[i];
      d *= beta;
      if (d != 0.0)
        for (int i = j; i < r; ++i) aq[i] -= d * v[i];
      // downdate the trailing norm; recompute when cancellation is severe
      const double t = std::fabs(aq[j]) / (nrm[q] > 0 ? nrm[q] : 1.0);
      double fac = 1.0 - t * t;
      fac = fac < 0 ? 0 : fac;
      const double ratio = nrm[q] / (nrm0[q] > 0 ? nrm0[q] : 1.0);
      if (fac * ratio * ratio < 1.5e-8) {
        double ss = 0.0;
        for (int i = j + 1; i < r; ++i) ss += aq[i] * aq[i];
        nrm[q] = nrm0[q] = std::sqrt(ss);
      } else {
        nrm[q] *= std::sqrt(fac);
      }
    }
    nrm[j] = 0.0;
  }
  if (!rank_found) f.k_tol = j;
  f.steps = j;
  f.R.assign((size_t)f.steps * c, 0.0);
  for (int q = 0; q < c; ++q)
    for (int i = 0; i < std::min(q + 1, f.steps); ++i) f.R[i + (size_t)q * f.steps] = A[i + (size_t)q * r];
  return f;
}

std::vector<double> cpqr_interp(const Cpqr& f, int c, int k) {
  const int ld = f.steps;
  std::vector<double> T((size_t)k * (c - k));
  for (int q = 0; q < c - k; ++q) {
    double* t = T.data() + (size_t)q * k;
    for (int i = 0; i < k; ++i) t[i] = f.R[i + (size_t)(k + q) * ld];
    for (int i = k - 1; i >= 0; --i) {
      t[i] /= f.R[i + (size_t)i * ld];
      const double v = t[i];
      for (int l = 0; l < i; ++l) t[l] -= f.R[l + (size_t)i * ld] * v;
    }
  }
  return T;
}
