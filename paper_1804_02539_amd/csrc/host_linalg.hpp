// Small dense linear algebra for the host setup: Cholesky factorisation,
// triangular inverse, cyclic Jacobi eigen-decomposition of symmetric matrices,
// the symmetric-definite generalised eigenproblem, and a null-space basis from
// the eigen-decomposition of the Gram matrix.  Row-major storage throughout.
#pragma once

#include <algorithm>
#include <cmath>
#include <vector>

namespace igamg {

using Mat = std::vector<double>;  // row-major, size r*c

// In-place lower Cholesky A = L L^T (upper part left untouched). false if not SPD.
inline bool cholesky(Mat& A, int n) {
  for (int j = 0; j < n; ++j) {
    double s = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
    if (!(s > 0.0)) return false;
    double d = std::sqrt(s);
    A[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double v = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) v -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
      A[(size_t)i * n + j] = v / d;
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) A[(size_t)i * n + j] = 0.0;
  return true;
}

// Inverse of a lower-triangular L (returns lower-triangular W = L^{-1}).
inline Mat lower_inverse(const Mat& L, int n) {
  Mat W((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    W[(size_t)j * n + j] = 1.0 / L[(size_t)j * n + j];
    for (int i = j + 1; i < n; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += L[(size_t)i * n + k] * W[(size_t)k * n + j];
      W[(size_t)i * n + j] = -s / L[(size_t)i * n + i];
    }
  }
  return W;
}

// Symmetric eigen-decomposition A = V diag(lam) V^T by cyclic Jacobi rotations.
// V columns are eigenvectors (V row-major n x n), ascending eigenvalues.
inline void sym_eig(const Mat& Ain, int n, std::vector<double>& lam, Mat& V) {
  Mat A = Ain;
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double a = A[(size_t)i * n + j] * A[(size_t)i * n + j];
        tot += a;
        if (i != j) off += a;
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[(size_t)p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        double theta = 0.5 * (aqq - app) / apq;
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = c * akp - s * akq;
          A[(size_t)k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = c * apk - s * aqk;
          A[(size_t)q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * vkp - s * vkq;
          V[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  lam.resize(n);
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) {
    lam[i] = A[(size_t)i * n + i];
    ord[i] = i;
  }
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return lam[a] < lam[b]; });
  Mat V2((size_t)n * n);
  std::vector<double> l2(n);
  for (int j = 0; j < n; ++j) {
    l2[j] = lam[ord[j]];
    for (int i = 0; i < n; ++i) V2[(size_t)i * n + j] = V[(size_t)i * n + ord[j]];
  }
  lam.swap(l2);
  V.swap(V2);
}

// Generalised problem K v = lam M v (K symmetric, M SPD): returns V with
// V^T M V = I and V^T K V = diag(lam).
inline bool gen_sym_eig(const Mat& K, const Mat& M, int n, std::vector<double>& lam, Mat& V) {
  Mat L = M;
  if (!cholesky(L, n)) return false;
  Mat W = lower_inverse(L, n);                     // L^{-1}
  Mat T((size_t)n * n, 0.0), C((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)                       // T = L^{-1} K
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = 0; k <= i; ++k) s += W[(size_t)i * n + k] * K[(size_t)k * n + j];
      T[(size_t)i * n + j] = s;
    }
  for (int i = 0; i < n; ++i)                       // C = T L^{-T}
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = 0; k <= j; ++k) s += T[(size_t)i * n + k] * W[(size_t)j * n + k];
      C[(size_t)i * n + j] = s;
    }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      double a = 0.5 * (C[(size_t)i * n + j] + C[(size_t)j * n + i]);
      C[(size_t)i * n + j] = C[(size_t)j * n + i] = a;
    }
  Mat Y;
  sym_eig(C, n, lam, Y);
  V.assign((size_t)n * n, 0.0);                     // V = L^{-T} Y
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = i; k < n; ++k) s += W[(size_t)k * n + i] * Y[(size_t)k * n + j];
      V[(size_t)i * n + j] = s;
    }
  return true;
}

// Orthonormal basis (columns, m x k row-major) of {v in R^m : C v = 0} for C (r x m).
// Rows of C are normalised; directions whose singular value is below tol * max
// are treated as null directions.  Uses the eigen-decomposition of C^T C, whose
// rounding floor is ~1e-8 in singular-value terms, so tol must sit well above it
// (the constraint matrices used here have no singular value in [1e-13, 1e-3]).
inline Mat null_space(const Mat& Cin, int r, int m, int* kout, double tol = 1e-5) {
  Mat C = Cin;
  for (int i = 0; i < r; ++i) {
    double s = 0.0;
    for (int j = 0; j < m; ++j) s += C[(size_t)i * m + j] * C[(size_t)i * m + j];
    s = std::sqrt(s);
    if (s > 0)
      for (int j = 0; j < m; ++j) C[(size_t)i * m + j] /= s;
  }
  Mat G((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      double s = 0.0;
      for (int k = 0; k < r; ++k) s += C[(size_t)k * m + i] * C[(size_t)k * m + j];
      G[(size_t)i * m + j] = s;
    }
  std::vector<double> lam;
  Mat V;
  sym_eig(G, m, lam, V);
  double lmax = lam.empty() ? 0.0 : std::max(lam.back(), 0.0);
  // singular value s = sqrt(lam): null when sqrt(lam) <= tol * sqrt(lmax)
  std::vector<int> keep;
  for (int j = 0; j < m; ++j)
    if (r == 0 || lam[j] <= tol * tol * lmax) keep.push_back(j);
  int k = (int)keep.size();
  Mat Z((size_t)m * k, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < k; ++j) Z[(size_t)i * k + j] = V[(size_t)i * m + keep[j]];
  *kout = k;
  return Z;
}

}  // namespace igamg
