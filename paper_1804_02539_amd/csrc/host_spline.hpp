// Host-side univariate spline tools for the setup phase (Sec. 2: S_{p,h}(0,1)).
//
//  - open uniform knot vectors, span search, the non-zero B-splines of a span
//    and their derivatives by the triangular recurrence tables;
//  - Gauss-Legendre nodes by Newton iteration on the Legendre polynomial;
//  - univariate mass and stiffness matrices by Gauss quadrature;
//  - the embedding matrix between nested spaces by repeated single-knot
//    insertion (Boehm), one midpoint per span (the uniform refinement of Sec. 3);
//  - Bernstein polynomials for the Bezier geometry maps.
#pragma once

#include <cmath>
#include <stdexcept>
#include <vector>

namespace igamg {

struct Knots {
  int p = 0;
  int nel = 0;
  std::vector<double> t;  // open, uniform
  int n() const { return (int)t.size() - p - 1; }
};

inline Knots open_uniform(int p, int nel) {
  Knots k;
  k.p = p;
  k.nel = nel;
  for (int i = 0; i <= p; ++i) k.t.push_back(0.0);
  for (int i = 1; i < nel; ++i) k.t.push_back((double)i / nel);
  for (int i = 0; i <= p; ++i) k.t.push_back(1.0);
  return k;
}

// Index s with t[s] <= x < t[s+1], p <= s <= n-1 (x = 1 maps to the last span).
inline int find_span(const Knots& k, double x) {
  const int n = k.n();
  if (x >= k.t[n]) return n - 1;
  if (x <= k.t[k.p]) return k.p;
  int lo = k.p, hi = n;
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (x < k.t[mid]) hi = mid; else lo = mid;
  }
  return lo;
}

// ders[r][j] = r-th derivative of B_{s-p+j} at x, r = 0..nd, j = 0..p.
inline void span_ders(const Knots& k, int s, double x, int nd, std::vector<std::vector<double>>& ders) {
  const int p = k.p;
  const std::vector<double>& t = k.t;
  std::vector<std::vector<double>> ndu(p + 1, std::vector<double>(p + 1, 0.0));
  std::vector<double> left(p + 1), right(p + 1);
  ndu[0][0] = 1.0;
  for (int j = 1; j <= p; ++j) {
    left[j] = x - t[s + 1 - j];
    right[j] = t[s + j] - x;
    double saved = 0.0;
    for (int r = 0; r < j; ++r) {
      ndu[j][r] = right[r + 1] + left[j - r];
      double tmp = ndu[r][j - 1] / ndu[j][r];
      ndu[r][j] = saved + right[r + 1] * tmp;
      saved = left[j - r] * tmp;
    }
    ndu[j][j] = saved;
  }
  ders.assign(nd + 1, std::vector<double>(p + 1, 0.0));
  for (int j = 0; j <= p; ++j) ders[0][j] = ndu[j][p];
  std::vector<std::vector<double>> a(2, std::vector<double>(p + 1, 0.0));
  for (int r = 0; r <= p; ++r) {
    int s1 = 0, s2 = 1;
    a[0][0] = 1.0;
    for (int kk = 1; kk <= nd; ++kk) {
      double d = 0.0;
      int rk = r - kk, pk = p - kk;
      if (r >= kk) {
        a[s2][0] = a[s1][0] / ndu[pk + 1][rk];
        d = a[s2][0] * ndu[rk][pk];
      }
      int j1 = (rk >= -1) ? 1 : -rk;
      int j2 = (r - 1 <= pk) ? kk - 1 : p - r;
      for (int j = j1; j <= j2; ++j) {
        a[s2][j] = (a[s1][j] - a[s1][j - 1]) / ndu[pk + 1][rk + j];
        d += a[s2][j] * ndu[rk + j][pk];
      }
      if (r <= pk) {
        a[s2][kk] = -a[s1][kk - 1] / ndu[pk + 1][r];
        d += a[s2][kk] * ndu[r][pk];
      }
      ders[kk][r] = d;
      std::swap(s1, s2);
    }
  }
  double fac = p;
  for (int kk = 1; kk <= nd; ++kk) {
    for (int j = 0; j <= p; ++j) ders[kk][j] *= fac;
    fac *= (p - kk);
  }
}

// Gauss-Legendre nodes/weights on [a, b] (Newton on P_n from Chebyshev guesses).
inline void gauss_legendre(int n, double a, double b, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5));
    double pp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = 0.0;
      for (int j = 1; j <= n; ++j) {
        double p2 = p1;
        p1 = p0;
        p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
      }
      pp = n * (z * p0 - p1) / (z * z - 1.0);
      double dz = p0 / pp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = 0.0;
      for (int j = 1; j <= n; ++j) {
        double p2 = p1;
        p1 = p0;
        p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
      }
      pp = n * (z * p0 - p1) / (z * z - 1.0);
    }
    // ascending order
    x[n - 1 - i] = 0.5 * (b - a) * z + 0.5 * (b + a);
    w[n - 1 - i] = (b - a) / ((1.0 - z * z) * pp * pp);
  }
}

// Univariate mass and stiffness matrices (dense n x n, row-major), exact with p+1 points.
inline void mass_stiffness_1d(const Knots& k, std::vector<double>& M, std::vector<double>& K) {
  const int n = k.n(), p = k.p;
  M.assign((size_t)n * n, 0.0);
  K.assign((size_t)n * n, 0.0);
  std::vector<double> gx, gw;
  std::vector<std::vector<double>> ders;
  for (int e = 0; e < k.nel; ++e) {
    double a = (double)e / k.nel, b = (double)(e + 1) / k.nel;
    gauss_legendre(p + 1, a, b, gx, gw);
    for (int q = 0; q <= p; ++q) {
      int s = find_span(k, gx[q]);
      span_ders(k, s, gx[q], 1, ders);
      for (int i = 0; i <= p; ++i)
        for (int j = 0; j <= p; ++j) {
          int I = s - p + i, J = s - p + j;
          M[(size_t)I * n + J] += gw[q] * ders[0][i] * ders[0][j];
          K[(size_t)I * n + J] += gw[q] * ders[1][i] * ders[1][j];
        }
    }
  }
}

// Embedding S(coarse) -> S(fine) where fine = coarse with every span halved.
// Returns P (n_f x n_c, row-major): fine coefficients = P * coarse coefficients.
inline std::vector<double> refinement_matrix(int p, int nel_c) {
  Knots cur = open_uniform(p, nel_c);
  int n = cur.n();
  std::vector<double> P((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) P[(size_t)i * n + i] = 1.0;
  int rows = n;
  for (int e = 0; e < nel_c; ++e) {
    double xbar = (e + 0.5) / nel_c;
    // insert xbar into cur (one knot): Boehm's rule
    int s = find_span(cur, xbar);
    int m = cur.n();
    std::vector<double> Q((size_t)(m + 1) * n, 0.0);
    for (int i = 0; i <= m; ++i) {
      double alpha;
      if (i <= s - p) alpha = 1.0;
      else if (i >= s + 1) alpha = 0.0;
      else alpha = (xbar - cur.t[i]) / (cur.t[i + p] - cur.t[i]);
      for (int c = 0; c < n; ++c) {
        double v = 0.0;
        if (alpha != 0.0 && i < m) v += alpha * P[(size_t)i * n + c];
        if (alpha != 1.0 && i >= 1) v += (1.0 - alpha) * P[(size_t)(i - 1) * n + c];
        Q[(size_t)i * n + c] = v;
      }
    }
    cur.t.insert(cur.t.begin() + s + 1, xbar);
    P.swap(Q);
    rows = m + 1;
  }
  (void)rows;
  return P;  // (n_c + nel_c) x n_c
}

// Bernstein values/derivatives of degree g at x: out[0][i] values, out[1][i] derivatives.
inline void bernstein(int g, double x, double* val, double* der) {
  // values by the binomial formula, derivatives by g (B_{i-1,g-1} - B_{i,g-1})
  std::vector<double> lo(g + 1, 0.0);
  auto binom = [](int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
  };
  for (int i = 0; i <= g; ++i) val[i] = binom(g, i) * std::pow(x, i) * std::pow(1.0 - x, g - i);
  if (g == 0) {
    der[0] = 0.0;
    return;
  }
  for (int i = 0; i < g; ++i) lo[i] = binom(g - 1, i) * std::pow(x, i) * std::pow(1.0 - x, g - 1 - i);
  for (int i = 0; i <= g; ++i) {
    double a = (i >= 1) ? lo[i - 1] : 0.0;
    double b = (i <= g - 1) ? lo[i] : 0.0;
    der[i] = g * (a - b);
  }
}

}  // namespace igamg
