// Per-entry arithmetic of the device assembly stages (assemble.hip): each
// function computes the output entry with linear index t of one stage, so a
// kernel runs it once per thread.  The index layouts, all with i0 fastest:
//   Gs[ab][q2][q1][q0]           ab = a*D + b, q2 local to the element slab
//   T1[ab][q2][q1][o0][i0]
//   T2[g][q2][i1][o1][o0][i0]     g = 2*(a == 2) + (b == 2)  (one group in 2D)
//   band[(row/256)*nbt*256 + plane*256 + row%256]: the symmetric half-band of
//   layout.hpp, plane = band_half_plane(o0, L), L = o1 + nb*o2
// 1D tables: val/der[(e*nq + q)*(pc+1) + l] is basis function e + l (value or
// derivative) at Gauss point q of element e.
#pragma once

#include <cmath>
#include <cstddef>
#include <cstdint>

#include "layout.hpp"
#include "assemble_layout.hpp"

#ifndef IGAMG_HD
#define IGAMG_HD __host__ __device__
#endif

namespace igamg {

IGAMG_HD inline int asm_imax(int a, int b) { return a > b ? a : b; }
IGAMG_HD inline int asm_imin(int a, int b) { return a < b ? a : b; }

// doubles of one slab's Gs, T1 and T2
inline void asm_sizes(int d, const AsmPatch& P, size_t out[3]) {
  const int64_t dd = (int64_t)d * d, g4 = (d == 3) ? 4 : 1;
  const int64_t Q0 = (int64_t)P.nel[0] * P.nq[0], Q1 = (int64_t)P.nel[1] * P.nq[1], NQ2 = P.nq[2];
  const int64_t nb = 2 * P.pc[0] + 1;
  out[0] = (size_t)(dd * NQ2 * Q1 * Q0);
  out[1] = (size_t)(dd * NQ2 * Q1 * nb * P.n[0]);
  out[2] = (size_t)(g4 * NQ2 * P.n[1] * nb * nb * P.n[0]);
}

// threads of the direction-0 and direction-1 stages (one per row entry and
// all its offsets)
inline int64_t asm_dir0_threads(int d, const AsmPatch& P) {
  return (int64_t)d * d * P.nq[2] * P.nel[1] * P.nq[1] * P.n[0];
}
inline int64_t asm_dir1_threads(int d, const AsmPatch& P) {
  const int64_t nb = 2 * P.pc[0] + 1;
  return (int64_t)((d == 3) ? 4 : 1) * P.nq[2] * P.n[1] * nb * P.n[0];
}

// threads of the direction-2 stage: one per (i0, o0, o1, i1)
IGAMG_HD inline int64_t asm_dir2_threads(const AsmPatch& P) {
  const int64_t nb = 2 * P.pc[0] + 1;
  return (int64_t)P.n[1] * nb * nb * P.n[0];
}

// Gauss point t = (q2*Q1 + q1)*Q0 + q0 of slab e2: the Jacobian of the Bezier
// map, then w |det J| J^{-1} J^{-T} into Gs; returns det J
template <int D>
IGAMG_HD inline double asm_metric_point(const AsmPatch& P, const double* tab, int e2, int64_t t, double* Gs) {
  const int Q0 = P.nel[0] * P.nq[0], Q1 = P.nel[1] * P.nq[1], NQ2 = P.nq[2];
  const int64_t tot = (int64_t)NQ2 * Q1 * Q0;
  const int q0 = (int)(t % Q0), q1 = (int)((t / Q0) % Q1), q2l = (int)(t / ((int64_t)Q0 * Q1));
  const int q2 = e2 * NQ2 + q2l;
  const int g0 = P.g[0] + 1, g1 = P.g[1] + 1, g2 = P.g[2] + 1;
  const double* v0 = tab + P.gv[0] + (int64_t)q0 * g0;
  const double* d0 = tab + P.gd[0] + (int64_t)q0 * g0;
  const double* v1 = tab + P.gv[1] + (int64_t)q1 * g1;
  const double* d1 = tab + P.gd[1] + (int64_t)q1 * g1;
  const double* v2 = tab + P.gv[2] + (int64_t)q2 * g2;
  const double* d2 = tab + P.gd[2] + (int64_t)q2 * g2;
  const double* cp = tab + P.ctrl;
  double J[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  for (int a2 = 0; a2 < g2; ++a2)
    for (int a1 = 0; a1 < g1; ++a1)
      for (int a0 = 0; a0 < g0; ++a0) {
        const double* c = cp + ((int64_t)(a2 * g1 + a1) * g0 + a0) * D;
        const double b0 = d0[a0] * v1[a1] * v2[a2];
        const double b1 = v0[a0] * d1[a1] * v2[a2];
        const double b2 = v0[a0] * v1[a1] * d2[a2];
        for (int i = 0; i < D; ++i) {
          J[i][0] += c[i] * b0;
          J[i][1] += c[i] * b1;
          if (D == 3) J[i][2] += c[i] * b2;
        }
      }
  double inv[3][3];
  double det;
  if (D == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    inv[0][0] = J[1][1] / det;
    inv[0][1] = -J[0][1] / det;
    inv[1][0] = -J[1][0] / det;
    inv[1][1] = J[0][0] / det;
  } else {
    inv[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    inv[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    inv[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    inv[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    inv[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    inv[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    inv[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    inv[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    inv[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    det = J[0][0] * inv[0][0] + J[0][1] * inv[1][0] + J[0][2] * inv[2][0];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) inv[i][j] /= det;
  }
  const double wt = fabs(det) * tab[P.w[0] + q0] * tab[P.w[1] + q1] * tab[P.w[2] + q2];
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) {
      double s = 0.0;
      for (int c = 0; c < D; ++c) s += inv[a][c] * inv[b][c];
      Gs[(int64_t)(a * D + b) * tot + t] = wt * s;
    }
  return det;
}

// direction 0 for thread t = (i0, q2*Q1 + q1, ab): the T1 entries of every
// offset o0 of row i0 at once, so that each Gauss value and basis value is
// loaded once rather than once per offset.  Each entry sums over the elements
// e shared by i0 and j0 = i0 + o0 - P (element by element, point by point).
template <int D, int P>
IGAMG_HD inline void asm_dir0_row(const AsmPatch& Pt, const double* tab, const double* Gs, double* T1, int64_t t) {
  constexpr int NB = 2 * P + 1, W = P + 1;
  const int n0 = Pt.n[0], nq = Pt.nq[0], nel0 = Pt.nel[0];
  const int Q0 = nel0 * nq;
  const int64_t plane = (int64_t)Pt.nq[2] * Pt.nel[1] * Pt.nq[1];
  const int i0 = (int)(t % n0);
  const int64_t r = t / n0;
  const int64_t qq = r % plane;
  const int ab = (int)(r / plane);
  const int a = ab / D, b = ab % D;
  const double* Fs = tab + (a == 0 ? Pt.der[0] : Pt.val[0]);
  const double* Ft = tab + (b == 0 ? Pt.der[0] : Pt.val[0]);
  const double* g = Gs + ((int64_t)ab * plane + qq) * Q0;
  double acc[NB];
#pragma unroll
  for (int o = 0; o < NB; ++o) acc[o] = 0.0;
#pragma unroll
  for (int el = 0; el < W; ++el) {
    const int e = i0 - P + el;   // i0 is local function P - el of element e
    if (e < 0 || e >= nel0) continue;
    for (int q = 0; q < nq; ++q) {
      const int x = e * nq + q;
      const double gs = g[x] * Fs[x * W + P - el];
#pragma unroll
      for (int lp = 0; lp < W; ++lp) acc[el + lp] += gs * Ft[x * W + lp];   // j0 = e + lp
    }
  }
  double* out = T1 + ((int64_t)ab * plane + qq) * NB * n0 + i0;
#pragma unroll
  for (int o = 0; o < NB; ++o) out[(int64_t)o * n0] = acc[o];
}

// direction 1 for thread t = (i0, o0, i1, q2, g): the T2 entries of every
// offset o1 at once, the (a, b) pairs of group g summed in turn
template <int D, int P>
IGAMG_HD inline void asm_dir1_row(const AsmPatch& Pt, const double* tab, const double* T1, double* T2, int64_t t) {
  constexpr int NB = 2 * P + 1, W = P + 1;
  const int n0 = Pt.n[0], n1 = Pt.n[1], nq = Pt.nq[1], nel1 = Pt.nel[1];
  const int NQ2 = Pt.nq[2], Q1 = nel1 * nq;
  const int i0 = (int)(t % n0);
  int64_t r = t / n0;
  const int o0 = (int)(r % NB);
  r /= NB;
  const int i1 = (int)(r % n1);
  r /= n1;
  const int q2l = (int)(r % NQ2);
  const int grp = (int)(r / NQ2);
  const int s2 = grp >> 1, t2 = grp & 1;
  const int64_t qstride = (int64_t)NB * n0;
  double acc[NB];
#pragma unroll
  for (int o = 0; o < NB; ++o) acc[o] = 0.0;
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) {
      if ((a == 2 ? 1 : 0) != s2 || (b == 2 ? 1 : 0) != t2) continue;
      const double* Fs = tab + (a == 1 ? Pt.der[1] : Pt.val[1]);
      const double* Ft = tab + (b == 1 ? Pt.der[1] : Pt.val[1]);
      const double* src = T1 + ((int64_t)(a * D + b) * NQ2 + q2l) * Q1 * qstride + (int64_t)o0 * n0 + i0;
#pragma unroll
      for (int el = 0; el < W; ++el) {
        const int e = i1 - P + el;
        if (e < 0 || e >= nel1) continue;
        for (int q = 0; q < nq; ++q) {
          const int x = e * nq + q;
          const double sv = src[(int64_t)x * qstride];
          const double fs = Fs[x * W + P - el];
#pragma unroll
          for (int lp = 0; lp < W; ++lp) acc[el + lp] += fs * Ft[x * W + lp] * sv;
        }
      }
    }
  double* out = T2 + (((int64_t)grp * NQ2 + q2l) * n1 + i1) * NB * NB * n0 + (int64_t)o0 * n0 + i0;
#pragma unroll
  for (int o = 0; o < NB; ++o) out[(int64_t)o * NB * n0] = acc[o];
}

// direction 2 for thread t = (i0, o0, o1, i1): adds slab e2's (P2+1)^2
// couplings (i2 = e2 + l, j2 = e2 + lp) to the band
template <int D, int P2>
IGAMG_HD inline void asm_dir2_entry(const AsmPatch& P, const double* tab, int e2, const double* T2, double* band,
                                    int nbt, int64_t t) {
  constexpr int G4 = (D == 3) ? 4 : 1, NQ2 = P2 + 1, W = P2 + 1;
  const int n0 = P.n[0], n1 = P.n[1], p = P.pc[0], nb = 2 * p + 1;
  const int64_t inner = asm_dir2_threads(P);
  const int i0 = (int)(t % n0);
  int64_t r = t / n0;
  const int o0 = (int)(r % nb);
  r /= nb;
  const int o1 = (int)(r % nb);
  const int i1 = (int)(r / nb);
  double v[G4][NQ2];
#pragma unroll
  for (int g = 0; g < G4; ++g)
#pragma unroll
    for (int q = 0; q < NQ2; ++q) v[g][q] = T2[((int64_t)g * NQ2 + q) * inner + t];
  const double* fv = tab + P.val[2] + (int64_t)e2 * NQ2 * W;
  const double* fd = tab + P.der[2] + (int64_t)e2 * NQ2 * W;
#pragma unroll
  for (int l = 0; l < W; ++l)
#pragma unroll
    for (int lp = 0; lp < W; ++lp) {
      double acc = 0.0;
#pragma unroll
      for (int g = 0; g < G4; ++g) {
        const double* Fs = (g >> 1) ? fd : fv;
        const double* Ft = (g & 1) ? fd : fv;
#pragma unroll
        for (int q = 0; q < NQ2; ++q) acc += Fs[q * W + l] * Ft[q * W + lp] * v[g][q];
      }
      // only the upper half is stored (the lower half is its transpose)
      const int plane = band_half_plane(D, p, o0, o1 + nb * (lp - l + P2));
      if (plane >= 0) {
        const int64_t row = P.off + i0 + (int64_t)n0 * (i1 + (int64_t)n1 * (e2 + l));
        band[((row >> 8) * nbt + plane) * 256 + (row & 255)] += acc;
      }
    }
}

// band entry t: zero when the coupling touches a Dirichlet function or leaves
// the patch (padding rows and blocks stay as they are: zero)
template <int D>
IGAMG_HD inline void asm_mask_entry(const PatchDev* pd, const int* bpatch, const uint8_t* isfree, double* band,
                                    int nbt, int p, int64_t t) {
  const int rr = (int)(t & 255);
  const int64_t bo = t >> 8;
  const int plane = (int)(bo % nbt);
  const int64_t blk = bo / nbt;
  const int k = bpatch[blk];
  if (k < 0) return;
  const PatchDev& P = pd[k];
  const int64_t row = blk * 256 + rr;
  const int64_t r = row - P.off;
  if (r < 0 || r >= P.rows) return;
  const int n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
  const int i0 = (int)(r % n0), i1 = (int)((r / n0) % n1), i2 = (int)(r / ((int64_t)n0 * n1));
  const int nb = 2 * p + 1, p2 = (D == 3) ? p : 0, lc = (band_lines(D, p) - 1) / 2;
  // the index-form offset of the stored plane (layout.hpp)
  int o0, L;
  if (plane <= p) {
    o0 = plane + p;
    L = lc;
  } else {
    o0 = (plane - p - 1) % nb;
    L = lc + 1 + (plane - p - 1) / nb;
  }
  const int j0 = i0 + o0 - p, j1 = i1 + L % nb - p, j2 = i2 + ((D == 3) ? L / nb : 0) - p2;
  bool zero = j0 < 0 || j0 >= n0 || j1 < 0 || j1 >= n1 || j2 < 0 || j2 >= n2 || !isfree[row];
  if (!zero) zero = !isfree[P.off + j0 + (int64_t)n0 * (j1 + (int64_t)n1 * j2)];
  if (zero) band[t] = 0.0;
}

}  // namespace igamg
