// Host-side univariate spline tools for the setup phase (Sec. 2: S_{p,h}(0,1)).
//
//  - open uniform knot vectors, span search, the non-zero B-splines of a span
//    and their derivatives (Cox-de Boor recursion, de Boor's derivative formula);
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
  std::vector<double> t;  // open: p+1 copies of each end, simple interior knots
  int n() const { return (int)t.size() - p - 1; }
  double lo(int e) const { return t[p + e]; }       // element e = [lo(e), hi(e)]
  double hi(int e) const { return t[p + e + 1]; }
};

// Open knot vector with the breakpoints 0 = brk[0] < ... < brk[nel] = 1 as
// simple interior knots (maximal smoothness C^{p-1}).
inline Knots open_knots(int p, const std::vector<double>& brk) {
  Knots k;
  k.p = p;
  k.nel = (int)brk.size() - 1;
  for (int i = 0; i < p; ++i) k.t.push_back(brk.front());
  k.t.insert(k.t.end(), brk.begin(), brk.end());
  for (int i = 0; i < p; ++i) k.t.push_back(brk.back());
  return k;
}

inline std::vector<double> uniform_breaks(int nel) {
  std::vector<double> b(nel + 1);
  for (int i = 0; i <= nel; ++i) b[i] = (double)i / nel;
  b[nel] = 1.0;
  return b;
}

// The breakpoints after one uniform refinement: the midpoint of every span.
inline std::vector<double> refine_breaks(const std::vector<double>& b) {
  std::vector<double> f;
  f.reserve(2 * b.size() - 1);
  for (size_t i = 0; i + 1 < b.size(); ++i) {
    f.push_back(b[i]);
    f.push_back(0.5 * (b[i] + b[i + 1]));
  }
  f.push_back(b.back());
  return f;
}

inline Knots open_uniform(int p, int nel) { return open_knots(p, uniform_breaks(nel)); }

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
//
// Values come from the Cox-de Boor recursion run over the degrees 0..p on the
// span s: tab[q][i] holds B_{s-q+i,q}(x), the q+1 functions of degree q that do
// not vanish there.  Derivatives use de Boor's derivative formula
//   B'_{g,q} = q B_{g,q-1} / (t_{g+q} - t_g) - q B_{g+1,q-1} / (t_{g+q+1} - t_{g+1}),
// applied r times to the unit coefficient vector of one degree-p function; the
// resulting combination of degree p-r functions is read from the table.
inline void span_ders(const Knots& k, int s, double x, int nd, std::vector<std::vector<double>>& ders) {
  const int p = k.p;
  const std::vector<double>& t = k.t;
  std::vector<std::vector<double>> tab(p + 1);
  tab[0].assign(1, 1.0);
  for (int q = 1; q <= p; ++q) {
    tab[q].assign(q + 1, 0.0);
    for (int i = 0; i <= q; ++i) {
      const int g = s - q + i;                       // B_{g,q}
      double v = 0.0;
      if (i >= 1) {                                  // B_{g,q-1} = tab[q-1][i-1]
        const double den = t[g + q] - t[g];
        if (den > 0.0) v += (x - t[g]) / den * tab[q - 1][i - 1];
      }
      if (i < q) {                                   // B_{g+1,q-1} = tab[q-1][i]
        const double den = t[g + q + 1] - t[g + 1];
        if (den > 0.0) v += (t[g + q + 1] - x) / den * tab[q - 1][i];
      }
      tab[q][i] = v;
    }
  }
  ders.assign(nd + 1, std::vector<double>(p + 1, 0.0));
  for (int j = 0; j <= p; ++j) ders[0][j] = tab[p][j];
  std::vector<double> c, cn;
  for (int j = 0; j <= p; ++j) {
    const int g0 = s - p + j;
    c.assign(1, 1.0);                                // c[m]: coefficient of B_{g0+m, p-r}
    for (int r = 1; r <= nd && r <= p; ++r) {
      const int q = p - r + 1;                       // degree being differentiated
      cn.assign(r + 1, 0.0);
      for (int m = 0; m < r; ++m) {
        const int g = g0 + m;
        const double d0 = t[g + q] - t[g];
        const double d1 = t[g + q + 1] - t[g + 1];
        if (d0 > 0.0) cn[m] += q * c[m] / d0;
        if (d1 > 0.0) cn[m + 1] -= q * c[m] / d1;
      }
      c.swap(cn);
      const int qd = p - r;
      double v = 0.0;
      for (int m = 0; m <= r; ++m) {
        const int i = g0 + m - s + qd;               // position of B_{g0+m,qd} in tab[qd]
        if (i >= 0 && i <= qd) v += c[m] * tab[qd][i];
      }
      ders[r][j] = v;
    }
  }
}

// Gauss-Legendre nodes and weights on [a, b]: Newton's method on the Legendre
// polynomial P_n, evaluated by its three-term recurrence, started from
// Tricomi's asymptotic guesses cos(pi (i + 3/4) / (n + 1/2)); the weights are
// 2 / ((1 - z^2) P_n'(z)^2), scaled to [a, b].
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
    gauss_legendre(p + 1, k.lo(e), k.hi(e), gx, gw);
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
// The midpoints are inserted one knot at a time by Boehm's rule.
inline std::vector<double> refinement_matrix(const Knots& coarse) {
  const int p = coarse.p, nel_c = coarse.nel;
  Knots cur = coarse;
  int n = cur.n();
  std::vector<double> P((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) P[(size_t)i * n + i] = 1.0;
  for (int e = 0; e < nel_c; ++e) {
    const double xbar = 0.5 * (coarse.lo(e) + coarse.hi(e));
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
  }
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
