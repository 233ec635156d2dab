// Test helper, built with g++ by test_assembly_stages_host.py (not part of
// the library): runs the device-assembly stages (the arithmetic of
// assemble.hip) on the host over exactly sized buffers and compares the tiled
// band with the host assembly of every level >= 1; and compares the parallel
// dense coarse build with a serial one.
#define IGAMG_HD
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "assemble_stages.hpp"
#include "host_setup.hpp"

using namespace igamg;

namespace {

template <int D, int P>
void slab(const AsmPatch& Pt, const std::vector<double>& tab, int e2, std::vector<double>& band, int nbt, int& flag) {
  constexpr int P2 = (D == 3) ? P : 0;
  size_t sz[3];
  asm_sizes(D, Pt, sz);
  std::vector<double> Gs(sz[0]), T1(sz[1]), T2(sz[2]);
  for (int64_t t = 0; t < (int64_t)sz[0] / (D * D); ++t) {
    const double det = asm_metric_point<D>(Pt, tab.data(), e2, t, Gs.data());
    flag |= det > 0 ? 1 : det < 0 ? 2 : 4;
  }
  for (int64_t t = 0; t < asm_dir0_threads(D, Pt); ++t) asm_dir0_row<D, P>(Pt, tab.data(), Gs.data(), T1.data(), t);
  for (int64_t t = 0; t < asm_dir1_threads(D, Pt); ++t) asm_dir1_row<D, P>(Pt, tab.data(), T1.data(), T2.data(), t);
  for (int64_t t = 0; t < asm_dir2_threads(Pt); ++t)
    asm_dir2_entry<D, P2>(Pt, tab.data(), e2, T2.data(), band.data(), nbt, t);
}

template <int D>
void slab_p(const AsmPatch& Pt, const std::vector<double>& tab, int e2, std::vector<double>& band, int nbt,
            int& flag) {
  switch (Pt.pc[0]) {
    case 1: slab<D, 1>(Pt, tab, e2, band, nbt, flag); break;
    case 2: slab<D, 2>(Pt, tab, e2, band, nbt, flag); break;
    case 3: slab<D, 3>(Pt, tab, e2, band, nbt, flag); break;
    case 4: slab<D, 4>(Pt, tab, e2, band, nbt, flag); break;
    case 5: slab<D, 5>(Pt, tab, e2, band, nbt, flag); break;
    case 6: slab<D, 6>(Pt, tab, e2, band, nbt, flag); break;
    case 7: slab<D, 7>(Pt, tab, e2, band, nbt, flag); break;
    default: slab<D, 8>(Pt, tab, e2, band, nbt, flag); break;
  }
}

}  // namespace

// Largest |band_stages - band_host| / max |band_host| over levels >= 1 in
// *rel, and the det J flags ORed over all patches in *flags; returns 0, or 1
// when the host setup fails.
extern "C" int asm_stages_vs_host(const void* cprob, double* rel, int* flags) {
  try {
    Hierarchy H;
    H.prob = read_problem(cprob);
    build_all(H, false);
    const ProblemH& P = H.prob;
    double worst = 0.0;
    int fl = 0;
    for (size_t l = 1; l < H.lv.size(); ++l) {
      const LevelH& L = H.lv[l];
      std::vector<AsmPatch> pt;
      std::vector<double> tab;
      make_assembly_tables(P, L, pt, tab);
      const int nbt = band_half_planes(P.d, P.p);   // the stored (upper) planes
      const int nb1 = 2 * P.p + 1, lc = (band_lines(P.d, P.p) - 1) / 2;
      std::vector<double> band((size_t)nbt * L.NL, 0.0);
      for (int k = 0; k < P.K; ++k)
        for (int e2 = 0; e2 < pt[k].nel[2]; ++e2) {
          if (P.d == 2)
            slab_p<2>(pt[k], tab, e2, band, nbt, fl);
          else
            slab_p<3>(pt[k], tab, e2, band, nbt, fl);
        }
      std::vector<int> bp(L.bpatch);
      for (int64_t t = 0; t < (int64_t)band.size(); ++t) {
        if (P.d == 2)
          asm_mask_entry<2>(L.pd.data(), bp.data(), L.isfree.data(), band.data(), nbt, P.p, t);
        else
          asm_mask_entry<3>(L.pd.data(), bp.data(), L.isfree.data(), band.data(), nbt, P.p, t);
      }
      double mx = 0.0, df = 0.0;
      for (int64_t row = 0; row < L.NL; ++row)
        for (int pl = 0; pl < nbt; ++pl) {
          // the host band keeps every offset o0 + nb*L (L = o1 + nb*o2)
          const int o0 = pl <= P.p ? pl + P.p : (pl - P.p - 1) % nb1;
          const int L1 = pl <= P.p ? lc : lc + 1 + (pl - P.p - 1) / nb1;
          const double h = L.band[(size_t)(o0 + nb1 * L1) * L.NL + row];
          const double g = band[((row >> 8) * nbt + pl) * 256 + (row & 255)];
          mx = std::max(mx, std::fabs(h));
          df = std::max(df, std::fabs(h - g));
        }
      worst = std::max(worst, df / mx);
    }
    *rel = worst;
    *flags = fl;
    return 0;
  } catch (const SetupError&) {
    return 1;
  }
}

// The dense coarse matrix of a device setup (built by blocks of global rows
// in parallel, kept for upload) against a serial pass over patches, rows and
// offsets: returns the number of entries that differ in any bit (-1 when the
// coarse problem is small enough for the host factorization, -2 on a setup
// error).
extern "C" long coarse_dense_vs_serial(const void* cprob) {
  try {
    Hierarchy H;
    H.prob = read_problem(cprob);
    build_all(H, true);
    if (H.A0.empty()) return -1;
    const ProblemH& P = H.prob;
    const LevelH& L0 = H.lv[0];
    const int64_t N0 = L0.N;
    std::vector<double> A((size_t)N0 * N0, 0.0);
    const int d = P.d, p = P.p, nb0 = 2 * p + 1, nb1 = 2 * p + 1, p2 = (d == 3) ? p : 0, nb2 = 2 * p2 + 1;
    for (int k = 0; k < P.K; ++k) {
      const auto& n = L0.n[k];
      for (int64_t r = 0; r < L0.rows[k]; ++r) {
        const int64_t x = L0.off[k] + r, gi = L0.gid[x];
        if (gi < 0) continue;
        const int i0 = (int)(r % n[0]), i1 = (int)((r / n[0]) % n[1]), i2 = (int)(r / ((int64_t)n[0] * n[1]));
        for (int o2 = 0; o2 < nb2; ++o2)
          for (int o1 = 0; o1 < nb1; ++o1)
            for (int o0 = 0; o0 < nb0; ++o0) {
              const int j0 = i0 + o0 - p, j1 = i1 + o1 - p, j2 = i2 + o2 - p2;
              if (j0 < 0 || j0 >= n[0] || j1 < 0 || j1 >= n[1] || j2 < 0 || j2 >= n[2]) continue;
              const int64_t y = L0.off[k] + j0 + (int64_t)n[0] * (j1 + (int64_t)n[1] * j2);
              const int64_t gj = L0.gid[y];
              if (gj < 0) continue;
              A[(size_t)gi * N0 + gj] += L0.band[(o0 + (int64_t)nb0 * (o1 + (int64_t)nb1 * o2)) * L0.NL + x];
            }
      }
    }
    long diff = 0;
    for (size_t i = 0; i < A.size(); ++i) diff += std::memcmp(&A[i], &H.A0[i], sizeof(double)) != 0;
    return diff;
  } catch (const SetupError&) {
    return -2;
  }
}

// Work-items of the largest single dispatch the device assembly of this
// problem makes (per element slab: metric, direction 0, 1 and 2 stages), over
// every level >= 1; the mask stage is a grid-stride loop with a capped grid.
// Returns -1 on a setup error.
extern "C" long long asm_max_dispatch_items(const void* cprob) {
  try {
    Hierarchy H;
    H.prob = read_problem(cprob);
    build_topology(H, false);
    const ProblemH& P = H.prob;
    long long worst = 0;
    for (size_t l = 1; l < H.lv.size(); ++l) {
      std::vector<AsmPatch> pt;
      std::vector<double> tab;
      make_assembly_tables(P, H.lv[l], pt, tab);
      for (int k = 0; k < P.K; ++k) {
        size_t sz[3];
        asm_sizes(P.d, pt[k], sz);
        worst = std::max<long long>(worst, (long long)(sz[0] / (size_t)(P.d * P.d)));
        worst = std::max<long long>(worst, asm_dir0_threads(P.d, pt[k]));
        worst = std::max<long long>(worst, asm_dir1_threads(P.d, pt[k]));
        worst = std::max<long long>(worst, asm_dir2_threads(pt[k]));
      }
    }
    return worst;
  } catch (const SetupError& e) {
    std::fprintf(stderr, "asm_max_dispatch_items: %s\n", e.msg.c_str());
    return -1;
  }
}
