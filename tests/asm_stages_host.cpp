// Test helper: runs the device-assembly stages (the per-entry arithmetic of
// assemble.hip) on the host over exactly sized buffers and compares the tiled
// band with the host assembly of every level >= 1.  Built by
// test_assembly_stages_host.py with g++; not part of the library.
#define IGAMG_HD
#include <algorithm>
#include <cmath>
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
      int nbt = 1;
      for (int c = 0; c < P.d; ++c) nbt *= 2 * P.p + 1;
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
        for (int o = 0; o < nbt; ++o) {
          const double h = L.band[(size_t)o * L.NL + row];
          const double g = band[((row >> 8) * nbt + o) * 256 + (row & 255)];
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
