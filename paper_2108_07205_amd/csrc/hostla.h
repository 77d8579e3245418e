// Small dense FP64 linear algebra on the host, column-major, for the static
// HBS build of the reference wall.
#pragma once

#include <vector>

// C = alpha op(A) op(B) + beta C, op = 'N' or 'T'.
void hgemm(char ta, char tb, int m, int n, int k, double alpha, const double* A, int lda,
           const double* B, int ldb, double beta, double* C, int ldc);

// In-place LU with partial pivoting.  Returns 0, or j+1 if pivot j is zero or
// not finite.
int hlu(int n, double* A, int lda, int* piv);
// Solve with the factors of hlu (B overwritten by the solution).
void hlu_solve(int n, int nrhs, const double* LU, int lda, const int* piv, double* B, int ldb);
// In-place inverse; returns hlu's code.
int hinv(int n, double* A, int lda);

// Householder QR with column pivoting of an r x c matrix (column-major,
// ld = r).  Runs until step j has |R_jj| <= tol |R_00| and j >= min_steps, or
// min(r, c) steps.  k_tol = number of steps before the tolerance test first
// failed (the numerical rank); steps = Householder steps actually taken.
struct Cpqr {
  int k_tol = 0;
  int steps = 0;
  std::vector<int> perm;      // column order
  std::vector<double> R;      // steps x c upper trapezoid, column-major, ld = steps
};
Cpqr hcpqr(int r, int c, std::vector<double>& A, double tol, int min_steps);

// Interpolation block T = R11^{-1} R12 (k x (c - k), column-major) from the
// first k pivoted columns of a Cpqr with steps >= k.
std::vector<double> cpqr_interp(const Cpqr& f, int c, int k);
