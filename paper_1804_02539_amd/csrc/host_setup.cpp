// Host setup of the multigrid hierarchy: problem validation, the C0 dof maps
// (Sec. 2, the space V_l), the pieces of the additive smoother (Sec. 3),
// patch-wise Gauss assembly of the banded A_{l,k} (Sec. 4), the transfer
// tables (Sec. 3, P_l by knot insertion), the smoother factors and the coarse
// Cholesky factor (Sec. 4).
#include "host_setup.hpp"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <atomic>
#include <cmath>
#include <functional>
#include <map>
#include <mutex>
#include <numeric>
#include <thread>

#include "host_linalg.hpp"
#include "host_spline.hpp"
#include "igamg.h"

namespace igamg {

[[noreturn]] static void fail(int code, const std::string& m) { throw SetupError{code, m}; }

// ---------------------------------------------------------------------------
// problem
// ---------------------------------------------------------------------------
ProblemH read_problem(const void* cp) {
  const igamg_problem* P = static_cast<const igamg_problem*>(cp);
  if (!P) fail(IGAMG_EINVAL, "problem is NULL");
  ProblemH q;
  q.d = P->dim;
  q.p = P->degree;
  q.K = P->npatch;
  q.levels = P->levels;
  if (q.d != 2 && q.d != 3) fail(IGAMG_EINVAL, "dim must be 2 or 3");
  if (q.p < 1 || q.p > MAX_P) fail(IGAMG_EINVAL, "degree must be in 1..8");
  if (q.K < 1) fail(IGAMG_EINVAL, "npatch must be >= 1");
  if (q.levels < 2 || q.levels > 14) fail(IGAMG_EINVAL, "levels must be in 2..14");
  if (!P->nel0 || !P->geo_degree || !P->geo_ctrl || !P->bc || (P->nif > 0 && !P->iface))
    fail(IGAMG_EINVAL, "problem array is NULL");
  if (P->nif < 0) fail(IGAMG_EINVAL, "nif < 0");
  const int d = q.d;
  q.nel0.assign(P->nel0, P->nel0 + q.K * d);
  q.gdeg.assign(P->geo_degree, P->geo_degree + q.K * d);
  q.bc.assign(P->bc, P->bc + q.K * 2 * d);
  size_t pos = 0;
  for (int k = 0; k < q.K; ++k) {
    size_t npt = 1;
    for (int c = 0; c < d; ++c) {
      int e = q.nel0[k * d + c], g = q.gdeg[k * d + c];
      if (e < 1 || e > 4096) fail(IGAMG_EINVAL, "nel0 out of range");
      if (g < 1 || g > 12) fail(IGAMG_EINVAL, "geometry degree out of range 1..12");
      npt *= (size_t)(g + 1);
    }
    q.ctrl.emplace_back(P->geo_ctrl + pos, P->geo_ctrl + pos + npt * d);
    pos += npt * d;
    for (double v : q.ctrl.back())
      if (!std::isfinite(v)) fail(IGAMG_EINVAL, "non-finite control point");
  }
  q.brk0.assign((size_t)q.K * d, std::vector<double>());
  if (P->knots0) {
    size_t kp = 0;
    for (int k = 0; k < q.K; ++k)
      for (int c = 0; c < d; ++c) {
        const int e = q.nel0[k * d + c];
        std::vector<double> b(P->knots0 + kp, P->knots0 + kp + e + 1);
        kp += (size_t)e + 1;
        if (b.front() != 0.0 || b.back() != 1.0) fail(IGAMG_EINVAL, "knots0: breakpoints must run from 0 to 1");
        for (int i = 0; i < e; ++i)
          if (!std::isfinite(b[i + 1]) || !(b[i + 1] > b[i])) fail(IGAMG_EINVAL, "knots0: breakpoints must increase");
        q.brk0[(size_t)k * d + c] = std::move(b);
      }
  }
  for (int b : q.bc)
    if (b != 0 && b != 1) fail(IGAMG_EINVAL, "bc entries must be 0 or 1");
  for (int i = 0; i < P->nif; ++i) {
    std::array<int, 5> f;
    for (int j = 0; j < 5; ++j) f[j] = P->iface[5 * i + j];
    if (f[0] < 0 || f[0] >= q.K || f[2] < 0 || f[2] >= q.K) fail(IGAMG_ETOPO, "interface patch index out of range");
    if (f[1] < 0 || f[1] >= 2 * d || f[3] < 0 || f[3] >= 2 * d) fail(IGAMG_ETOPO, "interface side out of range");
    if (f[4] < 0 || f[4] > 7 || (d == 2 && (f[4] & 5))) fail(IGAMG_ETOPO, "bad interface orientation");
    if (f[0] == f[2] && f[1] == f[3]) fail(IGAMG_ETOPO, "interface joins a side to itself");
    q.iface.push_back(f);
  }
  return q;
}

// ---------------------------------------------------------------------------
// dof maps
// ---------------------------------------------------------------------------
static void tangential(int c, int t[2]) {
  int j = 0;
  for (int a = 0; a < 3; ++a)
    if (a != c) t[j++] = a;
}

// layer of side s of a patch with sizes n: positions ordered [j1][j0] (j0 fastest)
static std::vector<int64_t> side_layer(const std::array<int, 3>& n, int s) {
  int c = s / 2, end = s % 2, t[2];
  tangential(c, t);
  int64_t st[3] = {1, n[0], (int64_t)n[0] * n[1]};
  int64_t fix = end ? n[c] - 1 : 0;
  std::vector<int64_t> out;
  out.reserve((size_t)n[t[0]] * n[t[1]]);
  for (int j1 = 0; j1 < n[t[1]]; ++j1)
    for (int j0 = 0; j0 < n[t[0]]; ++j0) out.push_back(fix * st[c] + j0 * st[t[0]] + j1 * st[t[1]]);
  return out;
}

// Breakpoints of patch k in direction c on level l: uniform, or the given
// coarsest ones with every span halved l times (Sec. 3, uniform refinement).
static std::vector<double> level_breaks(const ProblemH& P, int k, int c, int l) {
  const auto& b0 = P.brk0[(size_t)k * P.d + c];
  if (b0.empty()) return uniform_breaks(P.nel0[k * P.d + c] << l);
  std::vector<double> b = b0;
  for (int i = 0; i < l; ++i) b = refine_breaks(b);
  return b;
}

static void make_level_dofs(const ProblemH& P, LevelH& L) {
  const int d = P.d, p = P.p, K = P.K;
  L.n.resize(K);
  L.nel.resize(K);
  L.off.resize(K);
  L.rows.resize(K);
  L.brk.assign((size_t)K * 3, std::vector<double>{0.0, 1.0});
  int64_t pos = 0;
  for (int k = 0; k < K; ++k) {
    for (int c = 0; c < 3; ++c) {
      if (c < d) {
        L.nel[k][c] = P.nel0[k * d + c] << L.l;
        L.n[k][c] = L.nel[k][c] + p;
        L.brk[(size_t)k * 3 + c] = level_breaks(P, k, c, L.l);
      } else {
        L.nel[k][c] = 1;
        L.n[k][c] = 1;
      }
    }
    L.rows[k] = (int64_t)L.n[k][0] * L.n[k][1] * L.n[k][2];
    L.off[k] = pos;
    pos += (L.rows[k] + ROW_ALIGN - 1) / ROW_ALIGN * ROW_ALIGN;
  }
  L.NL = pos;
  std::vector<int64_t> parent(L.NL);
  std::iota(parent.begin(), parent.end(), 0);
  auto find = [&](int64_t x) {
    int64_t r = x;
    while (parent[r] != r) r = parent[r];
    while (parent[x] != r) {
      int64_t nx = parent[x];
      parent[x] = r;
      x = nx;
    }
    return r;
  };
  std::vector<std::vector<char>> is_iface(K, std::vector<char>(2 * d, 0));
  for (const auto& f : P.iface) {
    const int a = f[0], sa = f[1], b = f[2], sb = f[3], o = f[4];
    is_iface[a][sa] = is_iface[b][sb] = 1;
    int ta[2], tb[2];
    tangential(sa / 2, ta);
    tangential(sb / 2, tb);
    const auto& na = L.n[a];
    const auto& nbs = L.n[b];
    const bool swap = (o & 1) != 0;
    // partner of t0 / t1 on side b
    int u_of_t0 = swap ? tb[1] : tb[0];
    int u_of_t1 = swap ? tb[0] : tb[1];
    if (na[ta[0]] != nbs[u_of_t0] || na[ta[1]] != nbs[u_of_t1])
      fail(IGAMG_ETOPO, "interface sides do not match (element counts differ)");
    // fully matching (Sec. 2): the breakpoints of paired directions agree,
    // read backwards where the orientation reverses the axis
    for (int j = 0; j < 2; ++j) {
      if (ta[j] >= d) continue;
      const auto& xa = L.brk[(size_t)a * 3 + ta[j]];
      const auto& xb = L.brk[(size_t)b * 3 + (j == 0 ? u_of_t0 : u_of_t1)];
      const bool rev = (o & (j == 0 ? 2 : 4)) != 0;
      for (size_t i = 0; i < xa.size(); ++i) {
        const double v = rev ? 1.0 - xb[xb.size() - 1 - i] : xb[i];
        if (std::fabs(xa[i] - v) > 1e-12) fail(IGAMG_ETOPO, "interface sides do not match (knot vectors differ)");
      }
    }
    std::vector<int64_t> la = side_layer(na, sa), lb = side_layer(nbs, sb);
    const int n0a = na[ta[0]], n1a = na[ta[1]], n0b = nbs[tb[0]];
    for (int j1 = 0; j1 < n1a; ++j1)
      for (int j0 = 0; j0 < n0a; ++j0) {
        int x0 = (o & 2) ? n0a - 1 - j0 : j0;  // index along the partner of t0
        int x1 = (o & 4) ? n1a - 1 - j1 : j1;  // index along the partner of t1
        int k0 = swap ? x1 : x0, k1 = swap ? x0 : x1;
        int64_t A = L.off[a] + la[(size_t)j1 * n0a + j0];
        int64_t B = L.off[b] + lb[(size_t)k1 * n0b + k0];
        int64_t ra = find(A), rb = find(B);
        if (ra != rb) parent[std::max(ra, rb)] = std::min(ra, rb);
      }
  }
  std::vector<char> dir_root(L.NL, 0);
  for (int k = 0; k < K; ++k)
    for (int s = 0; s < 2 * d; ++s)
      if (P.bc[k * 2 * d + s] == 1 && !is_iface[k][s])
        for (int64_t x : side_layer(L.n[k], s)) dir_root[find(L.off[k] + x)] = 1;
  L.gid.assign(L.NL, -1);
  std::vector<int64_t> num(L.NL, -1);
  int64_t N = 0;
  for (int k = 0; k < K; ++k)
    for (int64_t r = 0; r < L.rows[k]; ++r) {
      int64_t x = L.off[k] + r, root = find(x);
      if (dir_root[root]) continue;
      if (num[root] < 0) num[root] = N++;
      L.gid[x] = num[root];
    }
  L.N = N;
  L.gptr.assign(N + 1, 0);
  for (int64_t x = 0; x < L.NL; ++x)
    if (L.gid[x] >= 0) L.gptr[L.gid[x] + 1]++;
  for (int64_t g = 0; g < N; ++g) L.gptr[g + 1] += L.gptr[g];
  L.gidx.assign(L.gptr[N], 0);
  std::vector<int64_t> fill(L.gptr.begin(), L.gptr.end() - 1);
  for (int64_t x = 0; x < L.NL; ++x)
    if (L.gid[x] >= 0) L.gidx[fill[L.gid[x]]++] = x;
  L.isfree.assign(L.NL, 0);
  for (int64_t x = 0; x < L.NL; ++x) L.isfree[x] = L.gid[x] >= 0;
  L.bpatch.assign(L.NL / ROW_ALIGN, -1);
  for (int k = 0; k < K; ++k)
    for (int64_t b = L.off[k] / ROW_ALIGN; b * ROW_ALIGN < L.off[k] + L.rows[k]; ++b) L.bpatch[b] = k;
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
struct GeoEval {
  int d;
  std::array<int, 3> g{{0, 0, 0}};
  const double* ctrl;
  // tables of Bernstein values / derivatives at the points of each direction
  std::vector<double> bv[3], bd[3];
  int npts[3] = {1, 1, 1};
  void tables(int c, const std::vector<double>& x) {
    int gc = g[c];
    npts[c] = (int)x.size();
    bv[c].assign(x.size() * (gc + 1), 0.0);
    bd[c].assign(x.size() * (gc + 1), 0.0);
    for (size_t i = 0; i < x.size(); ++i) bernstein(gc, x[i], &bv[c][i * (gc + 1)], &bd[c][i * (gc + 1)]);
  }
  // map X and Jacobian J[i*3+j] = dG_i/dxi_j at point (q0, q1, q2)
  void eval(int q0, int q1, int q2, double X[3], double J[9]) const {
    for (int i = 0; i < 9; ++i) J[i] = 0.0;
    X[0] = X[1] = X[2] = 0.0;
    const int g0 = g[0] + 1, g1 = g[1] + 1, g2 = (d == 3) ? g[2] + 1 : 1;
    const double* v0 = &bv[0][(size_t)q0 * g0];
    const double* d0 = &bd[0][(size_t)q0 * g0];
    const double* v1 = &bv[1][(size_t)q1 * g1];
    const double* d1 = &bd[1][(size_t)q1 * g1];
    for (int a2 = 0; a2 < g2; ++a2) {
      double w2 = (d == 3) ? bv[2][(size_t)q2 * g2 + a2] : 1.0;
      double w2d = (d == 3) ? bd[2][(size_t)q2 * g2 + a2] : 0.0;
      for (int a1 = 0; a1 < g1; ++a1)
        for (int a0 = 0; a0 < g0; ++a0) {
          const double* cp = ctrl + ((size_t)(a2 * g1 + a1) * g0 + a0) * d;
          double b = v0[a0] * v1[a1] * w2;
          double b0 = d0[a0] * v1[a1] * w2;
          double b1 = v0[a0] * d1[a1] * w2;
          double b2 = v0[a0] * v1[a1] * w2d;
          for (int i = 0; i < d; ++i) {
            X[i] += cp[i] * b;
            J[i * 3 + 0] += cp[i] * b0;
            J[i * 3 + 1] += cp[i] * b1;
            if (d == 3) J[i * 3 + 2] += cp[i] * b2;
          }
        }
    }
  }
};

// |det J| J^{-1} J^{-T} (row-major d x d into G) and det J
static double metric(int d, const double J[9], double G[9]) {
  if (d == 2) {
    double a = J[0], b = J[1], c = J[3], e = J[4];
    double det = a * e - b * c;
    double inv[4] = {e / det, -b / det, -c / det, a / det};
    double ad = std::fabs(det);
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) G[i * 3 + j] = ad * (inv[i * 2 + 0] * inv[j * 2 + 0] + inv[i * 2 + 1] * inv[j * 2 + 1]);
    return det;
  }
  double inv[9];
  inv[0] = J[4] * J[8] - J[5] * J[7];
  inv[1] = J[2] * J[7] - J[1] * J[8];
  inv[2] = J[1] * J[5] - J[2] * J[4];
  inv[3] = J[5] * J[6] - J[3] * J[8];
  inv[4] = J[0] * J[8] - J[2] * J[6];
  inv[5] = J[2] * J[3] - J[0] * J[5];
  inv[6] = J[3] * J[7] - J[4] * J[6];
  inv[7] = J[1] * J[6] - J[0] * J[7];
  inv[8] = J[0] * J[4] - J[1] * J[3];
  double det = J[0] * inv[0] + J[1] * inv[3] + J[2] * inv[6];
  for (int i = 0; i < 9; ++i) inv[i] /= det;
  double ad = std::fabs(det);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += inv[i * 3 + k] * inv[j * 3 + k];
      G[i * 3 + j] = ad * s;
    }
  return det;
}

static GeoEval make_geo(const ProblemH& P, int k) {
  GeoEval ge;
  ge.d = P.d;
  for (int c = 0; c < P.d; ++c) ge.g[c] = P.gdeg[k * P.d + c];
  ge.ctrl = P.ctrl[k].data();
  return ge;
}

// Geometry scale: mean over (0,1)^d of |det J| tr(J^{-1} J^{-T}) / d (8-point Gauss).
static double patch_omega(const ProblemH& P, int k) {
  GeoEval ge = make_geo(P, k);
  std::vector<double> x, w;
  gauss_legendre(8, 0.0, 1.0, x, w);
  for (int c = 0; c < P.d; ++c) ge.tables(c, x);
  double s = 0.0;
  const int n2 = (P.d == 3) ? 8 : 1;
  for (int q2 = 0; q2 < n2; ++q2)
    for (int q1 = 0; q1 < 8; ++q1)
      for (int q0 = 0; q0 < 8; ++q0) {
        double X[3], J[9], G[9];
        ge.eval(q0, q1, q2, X, J);
        metric(P.d, J, G);
        double tr = 0.0;
        for (int c = 0; c < P.d; ++c) tr += G[c * 3 + c];
        double wt = w[q0] * w[q1] * ((P.d == 3) ? w[q2] : 1.0);
        s += wt * tr / P.d;
      }
  return s;
}

// ---------------------------------------------------------------------------
// patch assembly (sum-factorised over the tensor Gauss rule, row-based)
// ---------------------------------------------------------------------------
struct Quad1D {
  int nel = 1, nq = 1, pc = 0;
  std::vector<double> x, w;           // nel*nq points
  std::vector<double> val, der;       // [(e*nq + q)*(pc+1) + l]
};

static Quad1D quad_1d(int p, const std::vector<double>& brk, bool dummy) {
  Quad1D Q;
  if (dummy) {
    Q.x = {0.0};
    Q.w = {1.0};
    Q.val = {1.0};
    Q.der = {0.0};
    return Q;
  }
  const int nel = (int)brk.size() - 1;
  Q.nel = nel;
  Q.nq = p + 1;
  Q.pc = p;
  Knots kn = open_knots(p, brk);
  std::vector<double> gx, gw;
  std::vector<std::vector<double>> ders;
  Q.val.resize((size_t)nel * Q.nq * (p + 1));
  Q.der.resize((size_t)nel * Q.nq * (p + 1));
  for (int e = 0; e < nel; ++e) {
    gauss_legendre(Q.nq, kn.lo(e), kn.hi(e), gx, gw);
    for (int q = 0; q < Q.nq; ++q) {
      Q.x.push_back(gx[q]);
      Q.w.push_back(gw[q]);
      int s = find_span(kn, gx[q]);
      if (s - p != e) fail(IGAMG_EINVAL, "internal: span mismatch");
      span_ders(kn, s, gx[q], 1, ders);
      for (int l = 0; l <= p; ++l) {
        Q.val[((size_t)e * Q.nq + q) * (p + 1) + l] = ders[0][l];
        Q.der[((size_t)e * Q.nq + q) * (p + 1) + l] = ders[1][l];
      }
    }
  }
  return Q;
}

// Adds the patch matrix of patch k on level L into band[o*NL + off + row].
// Returns the min and max of det J met at the quadrature points.
static void assemble_patch(const ProblemH& P, const LevelH& L, int k, double* band, double dets[2]) {
  const int d = P.d, p = P.p;
  const auto& n = L.n[k];
  Quad1D Q[3];
  for (int c = 0; c < 3; ++c) Q[c] = quad_1d(p, L.brk[(size_t)k * 3 + c], c >= d);
  GeoEval ge = make_geo(P, k);
  for (int c = 0; c < d; ++c) ge.tables(c, Q[c].x);
  const int nb0 = 2 * p + 1, nb1 = 2 * p + 1, p2 = Q[2].pc, nb2 = 2 * p2 + 1;
  const int nq = p + 1, nq2 = Q[2].nq;
  const int Q0 = (int)Q[0].x.size(), Q1 = (int)Q[1].x.size();
  const int64_t NL = L.NL, off = L.off[k];
  const size_t t1sz = (size_t)nq2 * Q1 * n[0] * nb0;
  const size_t t2sz = (size_t)nq2 * n[1] * nb1 * n[0] * nb0;
  std::vector<double> Gs((size_t)nq2 * Q1 * Q0 * 9), T1(t1sz), T2(t2sz * 4);
  dets[0] = 1e300;
  dets[1] = -1e300;
  for (int e2 = 0; e2 < Q[2].nel; ++e2) {
    for (int q2l = 0; q2l < nq2; ++q2l) {
      const int q2 = e2 * nq2 + q2l;
      for (int q1 = 0; q1 < Q1; ++q1)
        for (int q0 = 0; q0 < Q0; ++q0) {
          double X[3], J[9], G[9];
          ge.eval(q0, q1, q2, X, J);
          double det = metric(d, J, G);
          dets[0] = std::min(dets[0], det);
          dets[1] = std::max(dets[1], det);
          double wt = Q[0].w[q0] * Q[1].w[q1] * Q[2].w[q2];
          double* g = &Gs[(((size_t)q2l * Q1 + q1) * Q0 + q0) * 9];
          for (int i = 0; i < 9; ++i) g[i] = G[i] * wt;
        }
    }
    std::fill(T2.begin(), T2.end(), 0.0);
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) {
        const int s[3] = {a == 0, a == 1, a == 2}, t[3] = {b == 0, b == 1, b == 2};
        const int grp = s[2] * 2 + t[2];      // step-3 group: derivative flags in direction 2
        double* T2g = &T2[grp * t2sz];
        // step 1: contract direction 0
        std::fill(T1.begin(), T1.end(), 0.0);
        const std::vector<double>& F0s = s[0] ? Q[0].der : Q[0].val;
        const std::vector<double>& F0t = t[0] ? Q[0].der : Q[0].val;
        for (int q2l = 0; q2l < nq2; ++q2l)
          for (int q1 = 0; q1 < Q1; ++q1) {
            double* t1 = &T1[((size_t)q2l * Q1 + q1) * n[0] * nb0];
            const double* gq = &Gs[((size_t)q2l * Q1 + q1) * Q0 * 9];
            for (int e0 = 0; e0 < Q[0].nel; ++e0)
              for (int q = 0; q < nq; ++q) {
                const double gv = gq[(size_t)(e0 * nq + q) * 9 + a * 3 + b];
                const double* fs = &F0s[((size_t)e0 * nq + q) * (p + 1)];
                const double* ft = &F0t[((size_t)e0 * nq + q) * (p + 1)];
                for (int l = 0; l <= p; ++l) {
                  double gl = gv * fs[l];
                  double* row = t1 + (size_t)(e0 + l) * nb0 + p - l;
                  for (int lp = 0; lp <= p; ++lp) row[lp] += gl * ft[lp];
                }
              }
          }
        // step 2: contract direction 1 into T2g[q2l][i1][o1][i0][o0]
        const std::vector<double>& F1s = s[1] ? Q[1].der : Q[1].val;
        const std::vector<double>& F1t = t[1] ? Q[1].der : Q[1].val;
        const size_t rowlen = (size_t)n[0] * nb0;
        for (int q2l = 0; q2l < nq2; ++q2l)
          for (int e1 = 0; e1 < Q[1].nel; ++e1)
            for (int q = 0; q < nq; ++q) {
              const int q1 = e1 * nq + q;
              const double* src = &T1[((size_t)q2l * Q1 + q1) * rowlen];
              const double* fs = &F1s[((size_t)e1 * nq + q) * (p + 1)];
              const double* ft = &F1t[((size_t)e1 * nq + q) * (p + 1)];
              for (int l = 0; l <= p; ++l)
                for (int lp = 0; lp <= p; ++lp) {
                  const double cf = fs[l] * ft[lp];
                  if (cf == 0.0) continue;
                  double* dst = &T2g[(((size_t)q2l * n[1] + e1 + l) * nb1 + (lp - l + p)) * rowlen];
                  for (size_t i = 0; i < rowlen; ++i) dst[i] += cf * src[i];
                }
            }
      }
    // step 3: contract direction 2 (per derivative-flag group) into the band
    for (int grp = 0; grp < 4; ++grp) {
      const int s2 = grp >> 1, t2 = grp & 1;
      if (d == 2 && grp != 0) continue;
      const double* T2g = &T2[grp * t2sz];
      const std::vector<double>& F2s = s2 ? Q[2].der : Q[2].val;
      const std::vector<double>& F2t = t2 ? Q[2].der : Q[2].val;
      for (int l = 0; l <= p2; ++l)
        for (int lp = 0; lp <= p2; ++lp) {
          const int i2 = e2 + l, o2 = lp - l + p2;
          for (int q2l = 0; q2l < nq2; ++q2l) {
            const double cf = F2s[((size_t)e2 * nq2 + q2l) * (p2 + 1) + l] *
                              F2t[((size_t)e2 * nq2 + q2l) * (p2 + 1) + lp];
            if (cf == 0.0) continue;
            for (int i1 = 0; i1 < n[1]; ++i1)
              for (int o1 = 0; o1 < nb1; ++o1) {
                const double* src = &T2g[(((size_t)q2l * n[1] + i1) * nb1 + o1) * n[0] * nb0];
                const int64_t rowbase = off + (int64_t)n[0] * (i1 + (int64_t)n[1] * i2);
                for (int o0 = 0; o0 < nb0; ++o0) {
                  const int64_t o = o0 + (int64_t)nb0 * (o1 + (int64_t)nb1 * o2);
                  double* bd = band + o * NL + rowbase;
                  for (int i0 = 0; i0 < n[0]; ++i0) bd[i0] += cf * src[(size_t)i0 * nb0 + o0];
                }
              }
          }
        }
    }
  }
  (void)nb2;
}

static void parallel_for(int n, const std::function<void(int)>& f) {
  int nt = std::max(1u, std::thread::hardware_concurrency());
  nt = std::min(nt, n);
  std::atomic<int> next(0);
  std::vector<std::thread> th;
  std::vector<SetupError> errs;
  std::mutex mtx;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      for (;;) {
        int i = next++;
        if (i >= n) break;
        try {
          f(i);
        } catch (const SetupError& e) {
          std::lock_guard<std::mutex> lk(mtx);
          errs.push_back(e);
        }
      }
    });
  for (auto& x : th) x.join();
  if (!errs.empty()) throw errs[0];
}

static void assemble_level(const ProblemH& P, LevelH& L) {
  const int d = P.d, p = P.p;
  L.nb = 1;
  for (int c = 0; c < d; ++c) L.nb *= 2 * p + 1;
  L.band.assign((size_t)L.nb * L.NL, 0.0);
  std::vector<double> dmin(P.K), dmax(P.K);
  parallel_for(P.K, [&](int k) {
    double dd[2];
    assemble_patch(P, L, k, L.band.data(), dd);
    dmin[k] = dd[0];
    dmax[k] = dd[1];
  });
  for (int k = 0; k < P.K; ++k)
    if (!(dmin[k] > 0.0 || dmax[k] < 0.0))
      fail(IGAMG_EGEOM, "patch " + std::to_string(k) + ": det J vanishes or changes sign");
  // eliminate Dirichlet rows and columns: zero every coupling that touches one
  const int nb0 = 2 * p + 1, nb1 = 2 * p + 1, p2 = (d == 3) ? p : 0, nb2 = 2 * p2 + 1;
  for (int k = 0; k < P.K; ++k) {
    const auto& n = L.n[k];
    for (int64_t r = 0; r < L.rows[k]; ++r) {
      const int64_t x = L.off[k] + r;
      const int i0 = (int)(r % n[0]), i1 = (int)((r / n[0]) % n[1]), i2 = (int)(r / ((int64_t)n[0] * n[1]));
      const bool rfree = L.gid[x] >= 0;
      for (int o2 = 0; o2 < nb2; ++o2)
        for (int o1 = 0; o1 < nb1; ++o1)
          for (int o0 = 0; o0 < nb0; ++o0) {
            const int j0 = i0 + o0 - p, j1 = i1 + o1 - p, j2 = i2 + o2 - p2;
            const int64_t o = o0 + (int64_t)nb0 * (o1 + (int64_t)nb1 * o2);
            double& v = L.band[o * L.NL + x];
            if (j0 < 0 || j0 >= n[0] || j1 < 0 || j1 >= n[1] || j2 < 0 || j2 >= n[2]) {
              v = 0.0;
              continue;
            }
            const int64_t y = L.off[k] + j0 + (int64_t)n[0] * (j1 + (int64_t)n[1] * j2);
            if (!rfree || L.gid[y] < 0) v = 0.0;
          }
    }
  }
}

void make_assembly_tables(const ProblemH& P, const LevelH& L, std::vector<AsmPatch>& pt, std::vector<double>& pool) {
  const int d = P.d, p = P.p;
  pt.assign(P.K, AsmPatch{});
  pool.clear();
  auto put = [&](const std::vector<double>& v) {
    const int64_t at = (int64_t)pool.size();
    pool.insert(pool.end(), v.begin(), v.end());
    return at;
  };
  for (int k = 0; k < P.K; ++k) {
    AsmPatch& a = pt[k];
    a.off = L.off[k];
    for (int c = 0; c < 3; ++c) {
      const bool dummy = c >= d;
      const Quad1D Q = quad_1d(p, L.brk[(size_t)k * 3 + c], dummy);
      a.n[c] = L.n[k][c];
      a.nel[c] = dummy ? 1 : L.nel[k][c];
      a.pc[c] = Q.pc;
      a.nq[c] = dummy ? 1 : Q.nq;
      a.g[c] = dummy ? 0 : P.gdeg[k * d + c];
      a.w[c] = put(Q.w);
      a.val[c] = put(Q.val);
      a.der[c] = put(Q.der);
      const int gc = a.g[c];
      std::vector<double> bv(Q.x.size() * (gc + 1), 1.0), bd(Q.x.size() * (gc + 1), 0.0);
      if (!dummy)
        for (size_t i = 0; i < Q.x.size(); ++i) bernstein(gc, Q.x[i], &bv[i * (gc + 1)], &bd[i * (gc + 1)]);
      a.gv[c] = put(bv);
      a.gd[c] = put(bd);
    }
    a.ctrl = put(P.ctrl[k]);
  }
}

// ---------------------------------------------------------------------------
// smoother pieces
// ---------------------------------------------------------------------------
struct OneD {
  int m = 0;
  Mat Mi, Ki, U;          // interior mass/stiffness, FD basis (columns)
  std::vector<double> mu;
};

// Mean physical length of each parameter direction: the average over (0,1)^d
// of |dG/dxi_c| (8-point Gauss).
static std::array<double, 3> patch_lengths(const ProblemH& P, int k) {
  GeoEval ge = make_geo(P, k);
  std::vector<double> x, w;
  gauss_legendre(8, 0.0, 1.0, x, w);
  for (int c = 0; c < P.d; ++c) ge.tables(c, x);
  std::array<double, 3> len{1.0, 1.0, 1.0};
  for (int c = 0; c < P.d; ++c) len[c] = 0.0;
  const int n2 = (P.d == 3) ? 8 : 1;
  for (int q2 = 0; q2 < n2; ++q2)
    for (int q1 = 0; q1 < 8; ++q1)
      for (int q0 = 0; q0 < 8; ++q0) {
        double X[3], J[9];
        ge.eval(q0, q1, q2, X, J);
        const double wt = w[q0] * w[q1] * ((P.d == 3) ? w[q2] : 1.0);
        for (int c = 0; c < P.d; ++c) {
          double s = 0.0;
          for (int i = 0; i < P.d; ++i) s += J[i * 3 + c] * J[i * 3 + c];
          len[c] += wt * std::sqrt(s);
        }
      }
  return len;
}

// Interior 1D space of S_{p,1/nel} (functions 1..n-2), the subspace of splines
// whose even derivatives of order 2l (1 <= l, 2l < p) vanish at both ends, its
// M-orthogonal complement, and the basis U = [M-orthonormal basis of the
// subspace, M-orthonormal eigenvectors of K on the complement] with
// mu = [sigma .., eigenvalues] (eigenvalues + sigma when s1_sigma: the
// operator K + sigma M on the complement).
static OneD one_d(int p, const std::vector<double>& brk, double sigma, bool s1_sigma) {
  OneD o;
  Knots kn = open_knots(p, brk);
  const int n = kn.n(), m = n - 2;
  o.m = m;
  Mat M, K;
  mass_stiffness_1d(kn, M, K);
  o.Mi.assign((size_t)m * m, 0.0);
  o.Ki.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      o.Mi[(size_t)i * m + j] = M[(size_t)(i + 1) * n + j + 1];
      o.Ki[(size_t)i * m + j] = K[(size_t)(i + 1) * n + j + 1];
    }
  if (m <= 0) return o;
  // constraint rows
  Mat C;
  int r = 0;
  std::vector<std::vector<double>> ders;
  for (int l = 1; 2 * l < p; ++l)
    for (int side = 0; side < 2; ++side) {
      double x = side ? 1.0 : 0.0;
      int s = find_span(kn, x);
      span_ders(kn, s, x, 2 * l, ders);
      std::vector<double> row(m, 0.0);
      for (int j = 0; j <= p; ++j) {
        int fn = s - p + j;
        if (fn >= 1 && fn <= n - 2) row[fn - 1] = ders[2 * l][j];
      }
      C.insert(C.end(), row.begin(), row.end());
      ++r;
    }
  int k0 = 0;
  Mat Z = null_space(C, r, m, &k0);
  o.U.assign((size_t)m * m, 0.0);
  o.mu.assign(m, 0.0);
  // U0 = Z L0^{-T}, Z^T M Z = L0 L0^T
  if (k0 > 0) {
    Mat G((size_t)k0 * k0, 0.0);
    for (int i = 0; i < k0; ++i)
      for (int j = 0; j < k0; ++j) {
        double s = 0.0;
        for (int a = 0; a < m; ++a)
          for (int b = 0; b < m; ++b) s += Z[(size_t)a * k0 + i] * o.Mi[(size_t)a * m + b] * Z[(size_t)b * k0 + j];
        G[(size_t)i * k0 + j] = s;
      }
    if (!cholesky(G, k0)) fail(IGAMG_ENOTSPD, "internal: mass matrix on subspace not SPD");
    Mat W = lower_inverse(G, k0);
    for (int a = 0; a < m; ++a)
      for (int j = 0; j < k0; ++j) {
        double s = 0.0;
        for (int i = 0; i < k0; ++i) s += Z[(size_t)a * k0 + i] * W[(size_t)j * k0 + i];
        o.U[(size_t)a * m + j] = s;
      }
    for (int j = 0; j < k0; ++j) o.mu[j] = sigma;
  }
  const int k1 = m - k0;
  if (k1 > 0) {
    Mat Y;
    if (k0 > 0) {
      Mat ZtM((size_t)k0 * m, 0.0);
      for (int i = 0; i < k0; ++i)
        for (int b = 0; b < m; ++b) {
          double s = 0.0;
          for (int a = 0; a < m; ++a) s += Z[(size_t)a * k0 + i] * o.Mi[(size_t)a * m + b];
          ZtM[(size_t)i * m + b] = s;
        }
      int ky = 0;
      Y = null_space(ZtM, k0, m, &ky);
      if (ky != k1) fail(IGAMG_EINVAL, "internal: complement dimension mismatch");
    } else {
      Y.assign((size_t)m * m, 0.0);
      for (int i = 0; i < m; ++i) Y[(size_t)i * m + i] = 1.0;
    }
    Mat KY((size_t)k1 * k1, 0.0), MY((size_t)k1 * k1, 0.0);
    for (int i = 0; i < k1; ++i)
      for (int j = 0; j < k1; ++j) {
        double sk = 0.0, sm = 0.0;
        for (int a = 0; a < m; ++a)
          for (int b = 0; b < m; ++b) {
            double yy = Y[(size_t)a * k1 + i] * Y[(size_t)b * k1 + j];
            sk += yy * o.Ki[(size_t)a * m + b];
            sm += yy * o.Mi[(size_t)a * m + b];
          }
        KY[(size_t)i * k1 + j] = sk;
        MY[(size_t)i * k1 + j] = sm;
      }
    std::vector<double> lam;
    Mat V;
    if (!gen_sym_eig(KY, MY, k1, lam, V)) fail(IGAMG_ENOTSPD, "internal: generalised eigenproblem");
    for (int a = 0; a < m; ++a)
      for (int j = 0; j < k1; ++j) {
        double s = 0.0;
        for (int i = 0; i < k1; ++i) s += Y[(size_t)a * k1 + i] * V[(size_t)i * k1 + j];
        o.U[(size_t)a * m + k0 + j] = s;
      }
    for (int j = 0; j < k1; ++j) o.mu[k0 + j] = lam[j] + (s1_sigma ? sigma : 0.0);
  }
  return o;
}

struct PieceH {
  int kind = 0;          // 0 interior, 1 face, 2 edge, 3 vertex
  int owner = 0;
  std::vector<int> bd, ft;                // boundary dirs, free dirs (owner)
  std::vector<int64_t> g;                 // global ids (owner order)
  int m[2] = {1, 1};
  std::vector<std::pair<int, std::vector<int>>> adj;
};

static int patch_of(const LevelH& L, int64_t x) {
  return (int)(std::upper_bound(L.off.begin(), L.off.end(), x) - L.off.begin()) - 1;
}

static std::vector<PieceH> make_pieces(const ProblemH& P, const LevelH& L) {
  const int d = P.d;
  std::vector<char> seen(L.N, 0);
  std::vector<PieceH> out;
  for (int k = 0; k < P.K; ++k) {
    const auto& n = L.n[k];
    for (int nb = 0; nb <= d; ++nb)
      for (int mask = 0; mask < (1 << d); ++mask) {
        if (__builtin_popcount(mask) != nb) continue;
        for (int ends = 0; ends < (1 << nb); ++ends) {
          int lo[3], hi[3];
          std::vector<int> bd, ft;
          int e = 0;
          for (int c = 0; c < 3; ++c) {
            if (c >= d) {
              lo[c] = 0;
              hi[c] = 1;
            } else if (mask & (1 << c)) {
              int end = (ends >> e++) & 1;
              lo[c] = end ? n[c] - 1 : 0;
              hi[c] = lo[c] + 1;
              bd.push_back(c);
            } else {
              lo[c] = 1;
              hi[c] = n[c] - 1;
              ft.push_back(c);
            }
          }
          if (hi[0] <= lo[0] || hi[1] <= lo[1] || hi[2] <= lo[2]) continue;
          PieceH pc;
          int nfree = 0, ndir = 0;
          for (int i2 = lo[2]; i2 < hi[2]; ++i2)
            for (int i1 = lo[1]; i1 < hi[1]; ++i1)
              for (int i0 = lo[0]; i0 < hi[0]; ++i0) {
                int64_t x = L.off[k] + i0 + (int64_t)n[0] * (i1 + (int64_t)n[1] * i2);
                int64_t g = L.gid[x];
                if (g < 0) ++ndir; else ++nfree;
                pc.g.push_back(g);
              }
          if (nfree == 0) continue;
          if (ndir > 0) fail(IGAMG_ETOPO, "internal: entity with mixed Dirichlet status");
          if (seen[pc.g[0]]) continue;
          for (int64_t g : pc.g) seen[g] = 1;
          pc.kind = (nb == 0) ? 0 : (d - nb == 0 ? 3 : (d - nb == 1 ? 2 : 1));
          pc.owner = k;
          pc.bd = bd;
          pc.ft = ft;
          for (size_t j = 0; j < ft.size() && j < 2; ++j) pc.m[j] = n[ft[j]] - 2;
          std::map<int, std::vector<int>> adj;
          for (int64_t c = L.gptr[pc.g[0]]; c < L.gptr[pc.g[0] + 1]; ++c) {
            int64_t x = L.gidx[c];
            int kk = patch_of(L, x);
            int64_t r = x - L.off[kk];
            const auto& nn = L.n[kk];
            int idx[3] = {(int)(r % nn[0]), (int)((r / nn[0]) % nn[1]), (int)(r / ((int64_t)nn[0] * nn[1]))};
            std::vector<int> b;
            for (int c2 = 0; c2 < d; ++c2)
              if (idx[c2] == 0 || idx[c2] == nn[c2] - 1) b.push_back(c2);
            adj[kk] = b;
          }
          for (auto& kv : adj) pc.adj.push_back(kv);
          out.push_back(std::move(pc));
        }
      }
  }
  for (int64_t g = 0; g < L.N; ++g)
    if (!seen[g]) fail(IGAMG_ETOPO, "internal: dof outside every piece");
  return out;
}

// L^{-1} = W^T W (W = the inverse Cholesky factor) of an SPD m x m matrix,
// written to pool[at .. at + m*m)
static void store_spd_inverse(Mat Lm, int m, std::vector<double>& pool, int64_t at) {
  if (!cholesky(Lm, m)) fail(IGAMG_ENOTSPD, "internal: edge or vertex operator not SPD");
  Mat W = lower_inverse(Lm, m);
  if (pool.size() < (size_t)at + (size_t)m * m) pool.resize((size_t)at + (size_t)m * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      double s = 0.0;
      for (int a = std::max(i, j); a < m; ++a) s += W[(size_t)a * m + i] * W[(size_t)a * m + j];
      pool[(size_t)at + (size_t)i * m + j] = s;
    }
}

// Gather list of one edge or vertex piece for its exact restriction
// A_l[g, g]: entry (i, j) sums, over the patches holding copies x of g_i and
// y of g_j, the coupling of x with y, read from the symmetric half-band at
// (row x, plane of the offset y - x) or, for an offset of the lower half, at
// (row y, plane of x - y).
static void add_direct_gather(const ProblemH& P, LevelH& L, const std::vector<int64_t>& g) {
  const int d = P.d, p = P.p, nb = 2 * p + 1, lc = (band_lines(d, p) - 1) / 2;
  if (L.dg_ptr.empty()) L.dg_ptr.push_back(0);
  auto tensor = [&](int64_t x, int k, int t[3]) {
    const auto& n = L.n[k];
    const int64_t r = x - L.off[k];
    t[0] = (int)(r % n[0]);
    t[1] = (int)((r / n[0]) % n[1]);
    t[2] = (int)(r / ((int64_t)n[0] * n[1]));
  };
  for (int64_t gi : g)
    for (int64_t gj : g) {
      for (int64_t ci = L.gptr[gi]; ci < L.gptr[gi + 1]; ++ci)
        for (int64_t cj = L.gptr[gj]; cj < L.gptr[gj + 1]; ++cj) {
          const int64_t x = L.gidx[ci], y = L.gidx[cj];
          const int k = patch_of(L, x);
          if (patch_of(L, y) != k) continue;
          int a[3], b[3], o[3] = {0, 0, 0};
          tensor(x, k, a);
          tensor(y, k, b);
          bool near = true;
          for (int c = 0; c < d; ++c) {
            o[c] = b[c] - a[c] + p;
            near = near && o[c] >= 0 && o[c] < nb;
          }
          if (!near) continue;
          const int line = o[1] + (d == 3 ? nb * o[2] : 0);
          const int pl = band_half_plane(d, p, o[0], line);
          if (pl >= 0) {
            L.dg_row.push_back(x);
            L.dg_plane.push_back(pl);
          } else {
            L.dg_row.push_back(y);
            L.dg_plane.push_back(band_half_plane(d, p, 2 * p - o[0], 2 * lc - line));
          }
        }
      L.dg_ptr.push_back((int64_t)L.dg_row.size());
    }
}

void finish_direct_pieces(LevelH& L, const std::vector<double>& vals) {
  size_t e = 0;
  for (size_t q = 0; q < L.dense.size(); ++q) {
    if (!L.direct[q]) continue;
    const int m = L.dense[q].m;
    Mat Lm(vals.begin() + e, vals.begin() + e + (size_t)m * m);
    e += (size_t)m * m;
    store_spd_inverse(Lm, m, L.densemat, L.dense[q].Linv);
  }
}

static void make_smoother(const ProblemH& P, const Options& O, LevelH& L) {
  const int d = P.d, p = P.p;
  std::vector<PieceH> pcs = make_pieces(P, L);
  // 1D factors by (element count, sigma): sigma depends on the patch only
  // through h, which is 1/nel unless the physical-h reading is chosen
  using Key = std::pair<std::vector<double>, double>;
  std::map<Key, OneD> cache;
  std::map<Key, int64_t> Uoff, muoff;
  L.fdmat.clear();
  // every U_c is stored followed by its transpose; dummy direction: U = U^T = [1], mu = [0]
  const int64_t dummyU = 0, dummyMu = 2;
  L.fdmat.push_back(1.0);
  L.fdmat.push_back(1.0);
  L.fdmat.push_back(0.0);
  // h of patch k in direction c
  auto hdir = [&](int k, int c) -> double {
    const auto& b = L.brk[(size_t)k * 3 + c];
    double h = b[1] - b[0];
    for (size_t i = 1; i + 1 < b.size(); ++i) h = std::min(h, b[i + 1] - b[i]);
    if (O.physical_h) h *= L.length[k][c];
    return h;
  };
  auto key1d = [&](int k, int c) -> Key {
    const double h = hdir(k, c);
    return Key(L.brk[(size_t)k * 3 + c], O.sigma_scale / (h * h));
  };
  auto get1d = [&](int k, int c) -> const OneD& {
    const Key key = key1d(k, c);
    auto it = cache.find(key);
    if (it == cache.end()) {
      // interior functions: n - 2 = nel + p - 2 (checked before the eigenproblem)
      if ((int64_t)key.first.size() - 1 + p - 2 > MAX_FD)
        fail(IGAMG_EINVAL, "patch too fine for the FD smoother (n-2 > " + std::to_string(MAX_FD) + ")");
      OneD o = one_d(p, key.first, key.second, O.s1_sigma != 0);
      Uoff[key] = (int64_t)L.fdmat.size();
      L.fdmat.insert(L.fdmat.end(), o.U.begin(), o.U.end());
      for (int i = 0; i < o.m; ++i)
        for (int j = 0; j < o.m; ++j) L.fdmat.push_back(o.U[(size_t)j * o.m + i]);
      muoff[key] = (int64_t)L.fdmat.size();
      L.fdmat.insert(L.fdmat.end(), o.mu.begin(), o.mu.end());
      it = cache.emplace(key, std::move(o)).first;
    }
    return it->second;
  };
  L.fd.clear();
  L.dense.clear();
  L.densemat.clear();
  L.direct.clear();
  L.dg_ptr.clear();
  L.dg_row.clear();
  L.dg_plane.clear();
  L.fdscr = 0;
  L.fd_maxm = 1;
  // interiors first
  for (const auto& pc : pcs) {
    if (pc.kind != 0) continue;
    const int k = pc.owner;
    const auto& n = L.n[k];
    FDItem it{};
    it.src_if = 0;
    it.base = L.off[k] + 1 + n[0] + (d == 3 ? (int64_t)n[0] * n[1] : 0);
    it.stride[0] = 1;
    it.stride[1] = n[0];
    it.stride[2] = (int64_t)n[0] * n[1];
    for (int c = 0; c < 3; ++c) {
      if (c < d) {
        const OneD& o = get1d(k, c);
        it.m[c] = o.m;
        it.U[c] = Uoff[key1d(k, c)];
        it.mu[c] = muoff[key1d(k, c)];
        L.fd_maxm = std::max(L.fd_maxm, o.m);
      } else {
        it.m[c] = 1;
        it.U[c] = dummyU;
        it.mu[c] = dummyMu;
        it.stride[c] = 0;
      }
    }
    it.pref = O.geometry_scaling ? L.omega[k] : 1.0;
    it.extra = 0.0;
    it.scr = L.fdscr;
    L.fdscr += (int64_t)it.m[0] * it.m[1] * it.m[2];
    L.fd.push_back(it);
  }
  L.nfd_interior = (int)L.fd.size();
  // interface vector: faces, edges, vertices in piece order
  L.nif = 0;
  L.if_ptr.assign(1, 0);
  L.if_idx.clear();
  for (const auto& pc : pcs) {
    if (pc.kind == 0) continue;
    const int64_t seg = L.nif;
    for (int64_t g : pc.g) {
      for (int64_t c = L.gptr[g]; c < L.gptr[g + 1]; ++c) L.if_idx.push_back(L.gidx[c]);
      L.if_ptr.push_back((int64_t)L.if_idx.size());
    }
    L.nif += (int64_t)pc.g.size();
    double om = 0.0, lh = 0.0;
    int nh = 0;
    for (const auto& a : pc.adj) {
      om += O.geometry_scaling ? L.omega[a.first] : 1.0;
      for (int c : a.second) {
        lh += std::log(hdir(a.first, c));
        ++nh;
      }
    }
    om /= (double)pc.adj.size();
    if (O.iface_multiplicity) om *= (double)pc.adj.size();
    const double h = std::exp(lh / nh);
    const double hp = h / p;
    if (pc.kind == 1) {  // face: FD in the two free directions of the owner
      const int k = pc.owner;
      FDItem it{};
      it.src_if = 1;
      it.base = seg;
      for (int j = 0; j < 2; ++j) {
        const OneD& o = get1d(k, pc.ft[j]);
        it.m[j] = o.m;
        it.U[j] = Uoff[key1d(k, pc.ft[j])];
        it.mu[j] = muoff[key1d(k, pc.ft[j])];
      }
      it.m[2] = 1;
      it.U[2] = dummyU;
      it.mu[2] = dummyMu;
      it.stride[0] = 1;
      it.stride[1] = it.m[0];
      it.stride[2] = 0;
      it.pref = om * hp;
      it.extra = 1.0 / (hp * hp);
      it.scr = L.fdscr;
      L.fdscr += (int64_t)it.m[0] * it.m[1];
      L.fd.push_back(it);
    } else {
      DensePiece dp{};
      dp.seg = seg;
      dp.m = (int)pc.g.size();
      dp.Linv = (int64_t)L.densemat.size();
      const int m = dp.m;
      if (O.iface_direct) {
        // the exact restriction of A_l to the piece: its entries are gathered
        // from the assembled band once it exists (finish_direct_pieces)
        add_direct_gather(P, L, pc.g);
        L.direct.push_back(1);
        L.densemat.resize(L.densemat.size() + (size_t)m * m, 0.0);
        L.dense.push_back(dp);
        continue;
      }
      L.direct.push_back(0);
      Mat Lm((size_t)m * m, 0.0);
      if (pc.kind == 3) {
        Lm[0] = om * std::pow(hp, d - 2);
      } else {
        const OneD& o = get1d(pc.owner, pc.ft[0]);
        if (o.m != m) fail(IGAMG_ETOPO, "internal: edge size mismatch");
        for (size_t i = 0; i < Lm.size(); ++i)
          Lm[i] = om * (std::pow(hp, d - 1) * o.Ki[i] + std::pow(hp, d - 3) * o.Mi[i]);
      }
      store_spd_inverse(Lm, m, L.densemat, dp.Linv);
      L.dense.push_back(dp);
    }
  }
}

// ---------------------------------------------------------------------------
// transfers between level l-1 and l
// ---------------------------------------------------------------------------
static void make_transfers(const ProblemH& P, const LevelH& C, LevelH& F) {
  const int d = P.d, p = P.p;
  using Brk = std::vector<double>;
  std::map<Brk, std::vector<double>> Pm;   // coarse breakpoints -> P (n_f x n_c)
  for (int k = 0; k < P.K; ++k)
    for (int c = 0; c < d; ++c) {
      const Brk& e = C.brk[(size_t)k * 3 + c];
      if (!Pm.count(e)) Pm[e] = refinement_matrix(open_knots(p, e));
    }
  // widths
  int WP = 1, WR = 1;
  for (auto& kv : Pm) {
    const int ne = (int)kv.first.size() - 1;
    const int nc = ne + p, nf = 2 * ne + p;
    const auto& M = kv.second;
    for (int i = 0; i < nf; ++i) {
      int lo = nc, hi = -1;
      for (int j = 0; j < nc; ++j)
        if (M[(size_t)i * nc + j] != 0.0) {
          lo = std::min(lo, j);
          hi = std::max(hi, j);
        }
      WP = std::max(WP, hi - lo + 1);
    }
    for (int j = 0; j < nc; ++j) {
      int lo = nf, hi = -1;
      for (int i = 0; i < nf; ++i)
        if (M[(size_t)i * nc + j] != 0.0) {
          lo = std::min(lo, i);
          hi = std::max(hi, i);
        }
      WR = std::max(WR, hi - lo + 1);
    }
  }
  F.WP = WP;
  F.WR = WR;
  F.tr_idx.clear();
  F.tr_val.clear();
  std::map<Brk, std::array<int64_t, 4>> tabs;  // coarse breakpoints -> (Pst, Pval, Rst, Rval)
  auto build = [&](const Brk& e) {
    if (tabs.count(e)) return tabs[e];
    std::array<int64_t, 4> t;
    const int ne = (int)e.size() - 1;
    const int nc = ne + p, nf = 2 * ne + p;
    const auto& M = Pm[e];
    t[0] = (int64_t)F.tr_idx.size();
    t[1] = (int64_t)F.tr_val.size();
    for (int i = 0; i < nf; ++i) {
      int lo = 0;
      while (lo < nc - 1 && M[(size_t)i * nc + lo] == 0.0) ++lo;
      lo = std::min(lo, std::max(0, nc - WP));
      F.tr_idx.push_back(lo);
      for (int w = 0; w < WP; ++w) F.tr_val.push_back(lo + w < nc ? M[(size_t)i * nc + lo + w] : 0.0);
    }
    t[2] = (int64_t)F.tr_idx.size();
    t[3] = (int64_t)F.tr_val.size();
    for (int j = 0; j < nc; ++j) {
      int lo = 0;
      while (lo < nf - 1 && M[(size_t)lo * nc + j] == 0.0) ++lo;
      lo = std::min(lo, std::max(0, nf - WR));
      F.tr_idx.push_back(lo);
      for (int w = 0; w < WR; ++w) F.tr_val.push_back(lo + w < nf ? M[(size_t)(lo + w) * nc + j] : 0.0);
    }
    tabs[e] = t;
    return t;
  };
  // dummy direction: identity of size 1
  const int64_t dPst = (int64_t)F.tr_idx.size(), dPval = (int64_t)F.tr_val.size();
  F.tr_idx.push_back(0);
  F.tr_val.push_back(1.0);
  for (int w = 1; w < std::max(WP, WR); ++w) F.tr_val.push_back(0.0);
  F.pd.resize(P.K);
  for (int k = 0; k < P.K; ++k) {
    PatchDev& pd = F.pd[k];
    for (int c = 0; c < 3; ++c) {
      pd.n[c] = F.n[k][c];
      pd.nc[c] = C.n[k][c];
      if (c < d) {
        auto t = build(C.brk[(size_t)k * 3 + c]);
        pd.Pst[c] = t[0];
        pd.Pval[c] = t[1];
        pd.Rst[c] = t[2];
        pd.Rval[c] = t[3];
      } else {
        pd.Pst[c] = pd.Rst[c] = dPst;
        pd.Pval[c] = pd.Rval[c] = dPval;
      }
    }
    pd.off = F.off[k];
    pd.offc = C.off[k];
    pd.rows = F.rows[k];
    pd.rowsc = C.rows[k];
  }
}

static void plain_patch_table(const ProblemH& P, LevelH& L) {
  L.pd.resize(P.K);
  for (int k = 0; k < P.K; ++k) {
    PatchDev& pd = L.pd[k];
    pd = PatchDev{};
    for (int c = 0; c < 3; ++c) {
      pd.n[c] = L.n[k][c];
      pd.nc[c] = 1;
    }
    pd.off = L.off[k];
    pd.rows = L.rows[k];
  }
}

// ---------------------------------------------------------------------------
// drivers
// ---------------------------------------------------------------------------
void setup_progress(const char* what, double value) {
  static const bool on = std::getenv("IGAMG_VERBOSE") != nullptr;
  if (!on) return;
  using clk = std::chrono::steady_clock;
  static const clk::time_point t0 = clk::now();
  std::fprintf(stderr, "[igamg setup %7.1f s] %s %.6g\n", std::chrono::duration<double>(clk::now() - t0).count(),
               what, value);
  std::fflush(stderr);
}

void build_topology(Hierarchy& H, bool with_numerics) {
  const ProblemH& P = H.prob;
  H.lv.assign(P.levels, LevelH{});
  for (int l = 0; l < P.levels; ++l) {
    H.lv[l].l = l;
    make_level_dofs(P, H.lv[l]);
  }
  if (H.lv[0].N == 0) fail(IGAMG_EINVAL, "no free degrees of freedom");
  std::vector<double> om(P.K, 1.0);
  std::vector<std::array<double, 3>> len(P.K, std::array<double, 3>{1.0, 1.0, 1.0});
  // the physical-h reading keys the 1D factors by h, so the sizing pass
  // needs the patch lengths too
  for (int k = 0; k < P.K; ++k) {
    if (with_numerics) om[k] = patch_omega(P, k);
    if (with_numerics || H.opt.physical_h) len[k] = patch_lengths(P, k);
  }
  for (auto& L : H.lv) {
    L.omega = om;
    L.length = len;
  }
  for (int l = 1; l < P.levels; ++l) {
    make_smoother(P, H.opt, H.lv[l]);
    make_transfers(P, H.lv[l - 1], H.lv[l]);
  }
  plain_patch_table(P, H.lv[0]);
  if (with_numerics) setup_progress("topology, smoothers and transfers done; finest local rows", (double)H.lv.back().NL);
}

void build_all(Hierarchy& H, bool device) {
  build_topology(H, true);
  const ProblemH& P = H.prob;
  const int nasm = assemble_on_device(H.opt, device) ? 1 : P.levels;
  for (int l = 0; l < nasm; ++l) {
    assemble_level(P, H.lv[l]);
    setup_progress("assembled level", l);
    LevelH& L = H.lv[l];
    if (l > 0 && !L.dg_row.empty()) {
      // exact edge and vertex pieces from the host band (full storage: the
      // half-band plane of offset (o0, line) is the full offset o0 + nb*line)
      const int p = P.p, nb = 2 * p + 1, lc = (band_lines(P.d, p) - 1) / 2;
      std::vector<double> vals(L.dg_ptr.size() - 1, 0.0);
      for (size_t e = 0; e + 1 < L.dg_ptr.size(); ++e)
        for (int64_t c = L.dg_ptr[e]; c < L.dg_ptr[e + 1]; ++c) {
          const int pl = L.dg_plane[c];
          const int full = pl <= p ? (pl + p) + nb * lc : (pl - p - 1) % nb + nb * (lc + 1 + (pl - p - 1) / nb);
          vals[e] += L.band[(size_t)full * L.NL + L.dg_row[c]];
        }
      finish_direct_pieces(L, vals);
    }
  }
  // coarse matrix (dense, free dofs of level 0) and its inverse Cholesky factor
  LevelH& L0 = H.lv[0];
  const int64_t N0 = L0.N;
  if (N0 > 100000) fail(IGAMG_EINVAL, "coarse problem too large for the dense coarse solver");
  // a host-only handle of a large coarse problem needs no coarse solver
  if (!coarse_on_device(H.opt, N0, device) && N0 > COARSE_HOST_MAX && H.opt.coarse_factor != 1) return;
  DenseBuf A((size_t)N0 * N0);   // zeroed below, row block by row block
  const int d = P.d, p = P.p;
  const int nb0 = 2 * p + 1, nb1 = 2 * p + 1, p2 = (d == 3) ? p : 0, nb2 = 2 * p2 + 1;
  // Each block of global rows is zeroed and filled by one thread.  A row gi
  // takes its copies in ascending local order and each copy's couplings in
  // offset order: every entry receives the same sums in the same order as a
  // serial pass over patches, rows and offsets.
  const int nblk = (int)std::min<int64_t>(N0, 256);
  parallel_for(nblk, [&](int b) {
    const int64_t r0 = N0 * b / nblk, r1 = N0 * (b + 1) / nblk;
    std::fill(A.begin() + r0 * N0, A.begin() + r1 * N0, 0.0);
    for (int64_t gi = r0; gi < r1; ++gi)
      for (int64_t c = L0.gptr[gi]; c < L0.gptr[gi + 1]; ++c) {
        const int64_t x = L0.gidx[c];
        const int k = patch_of(L0, x);
        const auto& n = L0.n[k];
        const int64_t r = x - L0.off[k];
        const int i0 = (int)(r % n[0]), i1 = (int)((r / n[0]) % n[1]), i2 = (int)(r / ((int64_t)n[0] * n[1]));
        for (int o2 = 0; o2 < nb2; ++o2)
          for (int o1 = 0; o1 < nb1; ++o1)
            for (int o0 = 0; o0 < nb0; ++o0) {
              const int j0 = i0 + o0 - p, j1 = i1 + o1 - p, j2 = i2 + o2 - p2;
              if (j0 < 0 || j0 >= n[0] || j1 < 0 || j1 >= n[1] || j2 < 0 || j2 >= n[2]) continue;
              const int64_t y = L0.off[k] + j0 + (int64_t)n[0] * (j1 + (int64_t)n[1] * j2);
              const int64_t gj = L0.gid[y];
              if (gj < 0) continue;
              const int64_t o = o0 + (int64_t)nb0 * (o1 + (int64_t)nb1 * o2);
              A[(size_t)gi * N0 + gj] += L0.band[o * L0.NL + x];
            }
      }
  });
  setup_progress("dense coarse matrix built; coarse unknowns", (double)N0);
  if (coarse_on_device(H.opt, N0, device)) {
    H.A0 = std::move(A);   // factored after upload
    return;
  }
  Mat Ah(A.begin(), A.end());
  DenseBuf().swap(A);
  if (!cholesky(Ah, (int)N0)) fail(IGAMG_ENOTSPD, "coarse matrix is not positive definite (is any side Dirichlet?)");
  // A_0^{-1} = L^{-T} L^{-1} from the Cholesky factor: the two triangular
  // solves of the exact coarse solver become one dense mat-vec on the device
  Mat W = lower_inverse(Ah, (int)N0);
  H.Ainv.assign((size_t)N0 * N0, 0.0);
  parallel_for((int)N0, [&](int i) {
    for (int64_t j = i; j < N0; ++j) {
      double s = 0.0;
      for (int64_t k = j; k < N0; ++k) s += W[(size_t)k * N0 + i] * W[(size_t)k * N0 + j];
      H.Ainv[(size_t)i * N0 + j] = s;
      H.Ainv[(size_t)j * N0 + i] = s;
    }
  });
}

std::vector<double> load_vector(const Hierarchy& H, double amp, double freq) {
  const ProblemH& P = H.prob;
  const LevelH& L = H.lv.back();
  const int d = P.d, p = P.p;
  std::vector<std::vector<double>> loc(P.K);
  parallel_for(P.K, [&](int k) {
    const auto& n = L.n[k];
    Quad1D Q[3];
    for (int c = 0; c < 3; ++c) Q[c] = quad_1d(p, L.brk[(size_t)k * 3 + c], c >= d);
    GeoEval ge = make_geo(P, k);
    for (int c = 0; c < d; ++c) ge.tables(c, Q[c].x);
    std::vector<double>& f = loc[k];
    f.assign(L.rows[k], 0.0);
    const double pi = 3.14159265358979323846;
    for (int e2 = 0; e2 < Q[2].nel; ++e2)
      for (int e1 = 0; e1 < Q[1].nel; ++e1)
        for (int e0 = 0; e0 < Q[0].nel; ++e0)
          for (int a2 = 0; a2 < Q[2].nq; ++a2)
            for (int a1 = 0; a1 < Q[1].nq; ++a1)
              for (int a0 = 0; a0 < Q[0].nq; ++a0) {
                const int q0 = e0 * Q[0].nq + a0, q1 = e1 * Q[1].nq + a1, q2 = e2 * Q[2].nq + a2;
                double X[3], J[9], G[9];
                ge.eval(q0, q1, q2, X, J);
                double det = metric(d, J, G);
                double src = amp;
                for (int c = 0; c < d; ++c) src *= std::sin(freq * pi * X[c]);
                const double wv = src * std::fabs(det) * Q[0].w[q0] * Q[1].w[q1] * Q[2].w[q2];
                const double* v0 = &Q[0].val[(size_t)q0 * (Q[0].pc + 1)];
                const double* v1 = &Q[1].val[(size_t)q1 * (Q[1].pc + 1)];
                const double* v2 = &Q[2].val[(size_t)q2 * (Q[2].pc + 1)];
                for (int l2 = 0; l2 <= Q[2].pc; ++l2)
                  for (int l1 = 0; l1 <= Q[1].pc; ++l1) {
                    const double w12 = wv * v2[l2] * v1[l1];
                    const int64_t rb = (int64_t)n[0] * ((e1 + l1) + (int64_t)n[1] * (e2 + l2)) + e0;
                    for (int l0 = 0; l0 <= Q[0].pc; ++l0) f[rb + l0] += w12 * v0[l0];
                  }
              }
  });
  std::vector<double> out(L.N, 0.0);
  for (int k = 0; k < P.K; ++k)
    for (int64_t r = 0; r < L.rows[k]; ++r) {
      int64_t g = L.gid[L.off[k] + r];
      if (g >= 0) out[g] += loc[k][r];
    }
  return out;
}

}  // namespace igamg
