// C-ABI of the library: workspace planning, upload, the multigrid cycle of
// Algorithm 1 on the device, the PCG driver of Sec. 4 (FP64, or FP32 inner
// solves inside FP64 iterative refinement), and per-operator entry points.
// Every step of the cycle runs in the kernels of kernels.hip; the host only
// sequences launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "host_setup.hpp"
#include "igamg.h"
#include "kernels.hpp"

using namespace igamg;

static thread_local std::string g_err;

static int set_err(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_OK(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) throw SetupError{IGAMG_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)}; \
  } while (0)

namespace {

// storage of one level in one precision
template <typename T>
struct LevelData {
  T *band = nullptr, *u = nullptr, *f = nullptr, *w = nullptr;
  T *fdmat = nullptr, *densemat = nullptr, *tr_val = nullptr, *scr = nullptr;
};

struct DevLevel {
  int64_t NL = 0, N = 0, rows = 0;
  int nb = 0, nbh = 0, nfd = 0, nfd_int = 0, ndense = 0, WP = 0, WR = 0, fd_maxm = 1, max_dense = 1;
  int mfma_grid = 1;
  int64_t sym_ws = 0;   // > 0: the banded apply in scatter form, sym_ws window values per tile
  int* bpatch = nullptr;
  PatchDev* pd = nullptr;
  uint8_t* isfree = nullptr;
  int64_t *gptr = nullptr, *gidx = nullptr, *if_ptr = nullptr, *if_idx = nullptr;
  FDItem* fd = nullptr;
  DensePiece* dense = nullptr;
  int64_t* tr_idx = nullptr;
  int slab_grid = 1, mid_grid = 1, max_m2 = 1;
  int slab_grid4 = 1;
  int fdv[2] = {IGAMG_FD_VEC8, IGAMG_FD_VEC8};   // smoother variant per precision: [0] FP64, [1] FP32
  LevelData<double> d64;
  LevelData<float> d32;
};

template <typename T>
LevelData<T>& dat(DevLevel& D);
template <>
LevelData<double>& dat<double>(DevLevel& D) {
  return D.d64;
}
template <>
LevelData<float>& dat<float>(DevLevel& D) {
  return D.d32;
}

template <typename T>
struct PcgVecs {
  T *x = nullptr, *p = nullptr, *q = nullptr;
};

struct Bump {
  char* base;
  size_t pos = 0;
  template <typename T>
  T* take(size_t n) {
    pos = (pos + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + pos) : nullptr;
    pos += std::max<size_t>(n, 1) * sizeof(T);
    return p;
  }
};

}  // namespace

// scratch of the device coarse factorization: the factor and the inverse
// factor, each in packed lower tiles
static size_t coarse_ws_bytes(int64_t n) { return 2 * (size_t)coarse_packed_entries(n) * sizeof(double); }

struct igamg_ctx {
  Hierarchy H;
  int d = 2, p = 2, L = 1;
  bool mixed = false;
  std::vector<DevLevel> dl;
  double* Ainv = nullptr;          // A_0^{-1}, packed lower tiles
  float* Ainv32 = nullptr;         // the same rounded to FP32, for the FP32 cycle (mixed precision)
  double* cpart = nullptr;         // partial products of the coarse solve (coarse_tiles(N0)^2 * 64)
  void* coarse_ws = nullptr;       // device coarse factorization scratch (overlaps level data)
  size_t coarse_ws_bytes = 0;
  int* coarse_info = nullptr;
  size_t scratch_at = 0;          // workspace offset where the level data (and that scratch) begins
  // device assembly scratch (setup only; after the level data): per-patch
  // det J sign flags, a level's tables, one element slab's intermediates
  int* asm_flag = nullptr;
  double *asm_tab = nullptr, *asm_gs = nullptr, *asm_t1 = nullptr, *asm_t2 = nullptr;
  // setup-only gather lists of the exact edge and vertex pieces
  int64_t *dg_ptr = nullptr, *dg_row = nullptr;
  int* dg_plane = nullptr;
  double* dg_out = nullptr;
  double* cb = nullptr;
  void* symwin = nullptr;          // windows of the scatter-form banded apply (one level at a time)
  // the coarse levels of a cycle as one persistent launch (options.persistent)
  struct Tail {
    int level = 0, nph = 0, grid = 0;
    int64_t total = 0;
    size_t lds = 0;
    Phase* prog = nullptr;
    unsigned long long* ctr = nullptr;
    std::vector<Phase> host;
  } tail[2];   // [0] FP64, [1] FP32
  int64_t N0 = 0;
  PcgVecs<double> v64;
  PcgVecs<float> v32;
  double* fsave = nullptr;       // mixed: the right-hand side (patch-local, distributed)
  double *part = nullptr, *scal = nullptr;
  double* host_scal = nullptr;   // pinned (a plain host array for no-allocation handles)
  bool on_device = false;
  // igamg_setup_noalloc: the setup scratch lives in the static device array
  bool noalloc = false;
  char* setup_base = nullptr;
  size_t setup_bytes = 0;
  double host_scal_own[16] = {};
  // optional event timing of the banded apply
  bool prof = false;
  struct Rec {
    int level;
    double bytes;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;               // launches recorded outside graphs
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
  hipStream_t prof_stream = nullptr;

  void* ws = nullptr;
  size_t bytes = 0;
  struct igamg_batch_ctx* solo = nullptr;   // driver of igamg_solve
  // PCG bodies A and B of this hierarchy as graphs: [0], [1] in the handle's
  // precision; [2], [3] the FP64 bodies a mixed solve falls back to
  hipGraphExec_t gx[4] = {nullptr, nullptr, nullptr, nullptr};
};

template <typename T>
static void plan_level_data(Bump& b, const LevelH& L, DevLevel& D, LevelData<T>& X, bool solver_level) {
  X.u = b.take<T>(L.NL);
  X.f = b.take<T>(L.NL);
  X.w = b.take<T>(L.NL);
  if (!solver_level) return;
  // FP64: the symmetric half band; FP32: the full band, or the half band
  // where the level applies it in scatter form
  X.band = b.take<T>((size_t)(sizeof(T) == 8 || D.sym_ws > 0 ? D.nbh : D.nb) * L.NL);
  X.fdmat = b.take<T>(L.fdmat.size());
  X.densemat = b.take<T>(L.densemat.size());
  X.tr_val = b.take<T>(L.tr_val.size());
  X.scr = b.take<T>(L.fdscr);
}

template <typename T>
static const T* coarse_inverse_of(const igamg_ctx& C) {
  if constexpr (std::is_same<T, float>::value) return C.Ainv32;
  else return C.Ainv;
}

// Rows up to which a level belongs to the persistent coarse cycle: below
// this size a level's kernels are launch-bound.
constexpr int64_t TAIL_MAX_ROWS = 1 << 16;
// workgroups of the persistent launch
constexpr int TAIL_GRID = 128;

// The work list of cycle(Lp) from a zero guess (Algorithm 1 with mu = 1) over
// the levels 1..Lp, Lp the largest level below the finest whose levels are
// all at most TAIL_MAX_ROWS rows: smoothing products, residuals, transfers
// and the coarse solve, in the order the separate launches run them.  Needs
// the level data planned (pointers are null in the sizing pass).
template <typename T>
static void tail_program(igamg_ctx& C, igamg_ctx::Tail& tl) {
  const Options& O = C.H.opt;
  if (!O.persistent || O.mu != 1 || C.dl.size() < 3) return;
  int Lp = 0;
  for (int l = 1; l + 1 < (int)C.dl.size() && C.dl[l].NL <= TAIL_MAX_ROWS; ++l) Lp = l;
  if (Lp < 1) return;
  std::vector<Phase>& prog = tl.host;
  int64_t total = 0;
  // a phase has at most TAIL_GRID tickets, as many as the launch has workgroups
  auto push = [&](Phase ph) {
    if (ph.n <= 0) return;
    ph.chunk = (ph.n + TAIL_GRID - 1) / TAIL_GRID;
    ph.ntk = (ph.n + ph.chunk - 1) / ph.chunk;
    ph.first = total;
    total += ph.ntk;
    prog.push_back(ph);
  };
  auto band = [&](int l) {
    DevLevel& D = C.dl[l];
    LevelData<T>& X = dat<T>(D);
    Phase ph{};
    ph.kind = PH_BAND;
    ph.gx = 1;
    ph.n = D.NL / 64;
    ph.resid = 1;
    const void* a[] = {X.band, X.u, X.f, X.w, D.bpatch, D.pd};
    for (int i = 0; i < 6; ++i) ph.a[i] = a[i];
    push(ph);
  };
  auto smooth = [&](int l, const T* src, bool add) {
    DevLevel& D = C.dl[l];
    LevelData<T>& X = dat<T>(D);
    Phase ph{};
    ph.kind = PH_FD_FWD;
    ph.gx = D.slab_grid;
    ph.n = (int64_t)D.slab_grid * (D.nfd + D.ndense);
    ph.nitems = D.nfd;
    ph.tau = O.tau;
    ph.add = add;
    ph.rb = 8;
    const void* a[] = {D.fd, D.dense, X.densemat, X.fdmat, src, X.u, D.if_ptr, D.if_idx, X.scr};
    for (int i = 0; i < 9; ++i) ph.a[i] = a[i];
    push(ph);
    if (C.d == 3 && D.nfd_int > 0 && D.max_m2 > 1) {
      Phase m{};
      m.kind = PH_FD_MID;
      m.gx = D.mid_grid;
      m.n = (int64_t)D.mid_grid * D.nfd_int;
      m.a[0] = D.fd;
      m.a[1] = X.fdmat;
      m.a[2] = X.scr;
      push(m);
    }
    Phase v{};
    v.kind = PH_FD_INV;
    v.gx = D.slab_grid;
    v.n = (int64_t)D.slab_grid * D.nfd;
    v.tau = O.tau;
    v.add = add;
    v.rb = 8;
    const void* b2[] = {D.fd, X.fdmat, X.u, D.if_ptr, D.if_idx, X.scr};
    for (int i = 0; i < 6; ++i) v.a[i] = b2[i];
    push(v);
  };
  for (int l = Lp; l >= 1; --l) {
    DevLevel& F = C.dl[l];
    DevLevel& Cc = C.dl[l - 1];
    LevelData<T>& X = dat<T>(F);
    LevelData<T>& Xc = dat<T>(Cc);
    for (int i = 0; i < O.nu; ++i) {
      if (i == 0) {
        smooth(l, X.f, false);
      } else {
        band(l);
        smooth(l, X.w, true);
      }
    }
    band(l);
    Phase r{};
    r.kind = PH_RESTRICT;
    r.gx = 1;
    r.n = Cc.NL / ROW_ALIGN;
    r.w = F.WR;
    const void* a[] = {X.w, Xc.f, F.pd, Cc.bpatch, F.tr_idx, X.tr_val, Cc.isfree};
    for (int i = 0; i < 7; ++i) r.a[i] = a[i];
    push(r);
  }
  {
    DevLevel& D0 = C.dl[0];
    LevelData<T>& X0 = dat<T>(D0);
    Phase g{};
    g.kind = PH_GATHER;
    g.gx = 1;
    g.len = C.N0;
    g.n = (C.N0 + 255) / 256;
    const void* a[] = {X0.f, C.cb, D0.gptr, D0.gidx};
    for (int i = 0; i < 4; ++i) g.a[i] = a[i];
    push(g);
    const int64_t Tc = coarse_tiles(C.N0);
    Phase m{};
    m.kind = PH_CTILES;
    m.gx = 1;
    m.len = C.N0;
    m.n = Tc * (Tc + 1) / 2;
    const void* b2[] = {coarse_inverse_of<T>(C), C.cb, C.cpart};
    for (int i = 0; i < 3; ++i) m.a[i] = b2[i];
    push(m);
    Phase r{};
    r.kind = PH_CREDUCE;
    r.gx = 1;
    r.len = C.N0;
    r.n = Tc;
    const void* b3[] = {C.cpart, X0.u, D0.gptr, D0.gidx};
    for (int i = 0; i < 4; ++i) r.a[i] = b3[i];
    push(r);
  }
  for (int l = 1; l <= Lp; ++l) {
    DevLevel& F = C.dl[l];
    DevLevel& Cc = C.dl[l - 1];
    LevelData<T>& X = dat<T>(F);
    LevelData<T>& Xc = dat<T>(Cc);
    Phase pr{};
    pr.kind = PH_PROLONG;
    pr.gx = 1;
    pr.n = F.NL / ROW_ALIGN;
    pr.w = F.WP;
    const void* a[] = {Xc.u, X.u, F.pd, F.bpatch, F.tr_idx, X.tr_val, F.isfree};
    for (int i = 0; i < 7; ++i) pr.a[i] = a[i];
    push(pr);
    for (int i = 0; i < O.nu; ++i) {
      band(l);
      smooth(l, X.w, true);
    }
  }
  tl.level = Lp;
  tl.nph = (int)prog.size();
  tl.total = total;
  tl.grid = TAIL_GRID;
  tl.lds = 0;
  for (int l = 1; l <= Lp; ++l)
    tl.lds = std::max(tl.lds, cycle_tail_lds(C.dl[l].fd_maxm, C.dl[l].max_dense, sizeof(T)));
  if (tl.lds > 64 * 1024) tl = igamg_ctx::Tail{};   // pieces too large for one workgroup's default LDS
}

// Rows above which options.band_form = 0 applies a 2D level in scatter
// form.  Measured at p = 4: at 78K rows both precisions are faster in the
// gather form; at 282K rows the FP64 apply is 15% faster in scatter form but
// the FP32 one 8% slower (the windows cost more in 2D, one line per layer);
// from 1.1M rows both are faster (13-24% up to 10M rows).  A mixed handle's
// levels take one form for both precisions.
constexpr int64_t SYM_MIN_ROWS_2D_FP64 = int64_t(1) << 17;
constexpr int64_t SYM_MIN_ROWS_2D_MIXED = int64_t(1) << 19;

// Window values per tile of level L's banded apply in scatter form, or 0 for
// the gather form: levels whose windows and u fit BAND_SYM_MAX_LDS in FP64
// and, with options.band_form = 0, that have more than TAIL_MAX_ROWS rows in
// 3D (smaller ones are launch-bound) or SYM_MIN_ROWS_2D_* in 2D; never the
// levels of the persistent cycle, which reads the gather form.
static int64_t band_sym_ws(const Hierarchy& H, const LevelH& L) {
  if (H.opt.band_form == 1) return 0;
  const int64_t min_rows = H.prob.d == 3                        ? TAIL_MAX_ROWS
                           : H.opt.precision == IGAMG_MIXED ? SYM_MIN_ROWS_2D_MIXED
                                                            : SYM_MIN_ROWS_2D_FP64;
  if (L.NL <= min_rows && H.opt.band_form == 0) return 0;
  if (L.NL <= TAIL_MAX_ROWS && H.opt.persistent) return 0;
  int64_t n0 = 1;
  for (const auto& n : L.n) n0 = std::max<int64_t>(n0, n[0]);
  const int64_t ws = band_sym_window(H.prob.d, H.prob.p, n0);
  return (size_t)ws * 2 * sizeof(double) <= BAND_SYM_MAX_LDS ? ws : 0;
}

static size_t plan(igamg_ctx& C, char* base) {
  Bump b{base};
  const Hierarchy& H = C.H;
  // the coarse inverse first: a device factorization uses the space after it,
  // which the level data occupies later, as its scratch
  C.N0 = H.lv[0].N;
  C.Ainv = b.take<double>((size_t)coarse_packed_entries(C.N0));
  C.Ainv32 = C.mixed ? b.take<float>((size_t)coarse_packed_entries(C.N0)) : nullptr;
  C.cpart = b.take<double>((size_t)(coarse_tiles(C.N0) * coarse_tiles(C.N0) * COARSE_TILE));
  C.cb = b.take<double>(C.N0);
  const size_t scratch_at = (b.pos + 255) & ~size_t(255);
  size_t scratch_end = 0;
  if (coarse_on_device(H.opt, C.N0, true)) {
    C.coarse_info = reinterpret_cast<int*>(base ? base + scratch_at : nullptr);
    C.coarse_ws = base ? base + scratch_at + 256 : nullptr;
    C.coarse_ws_bytes = coarse_ws_bytes(C.N0);
    scratch_end = scratch_at + 256 + C.coarse_ws_bytes;
  }
  C.dl.assign(H.lv.size(), DevLevel{});
  int64_t sym_values = 0;
  for (size_t l = 0; l < H.lv.size(); ++l) {
    const LevelH& L = H.lv[l];
    DevLevel& D = C.dl[l];
    D.NL = L.NL;
    D.N = L.N;
    D.rows = 0;
    for (int64_t r : L.rows) D.rows += r;
    int nb = 1;
    for (int c = 0; c < H.prob.d; ++c) nb *= 2 * H.prob.p + 1;
    D.nb = nb;
    D.nbh = band_half_planes(H.prob.d, H.prob.p);
    D.bpatch = b.take<int>(L.bpatch.size());
    D.pd = b.take<PatchDev>(L.pd.size());
    D.isfree = b.take<uint8_t>(L.NL);
    D.gptr = b.take<int64_t>(L.gptr.size());
    D.gidx = b.take<int64_t>(L.gidx.size());
    const bool sl = l > 0;
    D.sym_ws = sl ? band_sym_ws(H, L) : 0;
    sym_values = std::max(sym_values, D.sym_ws * (L.NL / ROW_ALIGN));
    plan_level_data(b, L, D, D.d64, sl);
    if (C.mixed) plan_level_data(b, L, D, D.d32, sl);
    if (!sl) continue;
    D.if_ptr = b.take<int64_t>(L.if_ptr.size());
    D.if_idx = b.take<int64_t>(L.if_idx.size());
    D.nfd = (int)L.fd.size();
    D.nfd_int = L.nfd_interior;
    D.fd = b.take<FDItem>(L.fd.size());
    D.ndense = (int)L.dense.size();
    D.dense = b.take<DensePiece>(L.dense.size());
    D.tr_idx = b.take<int64_t>(L.tr_idx.size());
    D.WP = L.WP;
    D.WR = L.WR;
    D.fd_maxm = L.fd_maxm;
    D.max_dense = 1;
    for (const auto& dp : L.dense) D.max_dense = std::max(D.max_dense, dp.m);
    D.max_m2 = 1;
    for (const auto& it : L.fd) D.max_m2 = std::max(D.max_m2, it.m[2]);
    D.slab_grid = fd_slab_grid(L.fd.data(), (int)L.fd.size(), 8);
    D.slab_grid4 = fd_slab_grid(L.fd.data(), (int)L.fd.size(), 4);
    D.mfma_grid = fd_mfma_grid(L.fd.data(), (int)L.fd.size());
    D.mid_grid = fd_mid_grid(L.fd.data(), L.nfd_interior);
  }
  const int64_t NLf = H.lv.back().NL;
  C.v64.x = b.take<double>(NLf);
  C.v64.p = b.take<double>(NLf);
  C.v64.q = b.take<double>(NLf);
  if (C.mixed) {
    C.v32.x = b.take<float>(NLf);
    C.v32.p = b.take<float>(NLf);
    C.v32.q = b.take<float>(NLf);
    C.fsave = b.take<double>(NLf);
  }
  for (int prec = 0; prec < (C.mixed ? 2 : 1); ++prec) {
    igamg_ctx::Tail& tl = C.tail[prec];
    tl = igamg_ctx::Tail{};
    if (prec == 0) tail_program<double>(C, tl);
    else tail_program<float>(C, tl);
    // reserved by a bound that does not depend on the level data, which the
    // sizing pass has not filled in: per level nu pre- and post-smoothing
    // steps of at most 4 phases, a residual, a restriction and a
    // prolongation; the coarse gather, tile products and sums
    const int max_phases = (H.opt.persistent && H.opt.mu == 1) ? (int)C.dl.size() * (3 + 8 * H.opt.nu) + 3 : 0;
    if (max_phases > 0) {
      tl.prog = b.take<Phase>((size_t)max_phases);
      tl.ctr = b.take<unsigned long long>((size_t)max_phases + 2);
    }
    if (tl.nph > max_phases) tl = igamg_ctx::Tail{};
  }
  C.part = b.take<double>(2 * RED_BLOCKS);
  C.scal = b.take<double>(16);
  C.symwin = sym_values > 0 ? static_cast<void*>(b.take<double>((size_t)sym_values)) : nullptr;
  C.scratch_at = scratch_at;
  if (assemble_on_device(H.opt, true) && H.lv.size() > 1) {
    // the setup-only scratch: at the end of the workspace, or in the static
    // device array of a no-allocation setup
    Bump sb{C.setup_base};
    Bump& a = C.noalloc ? sb : b;
    size_t pool = 0, sz_max[3] = {0, 0, 0};
    for (size_t l = 1; l < H.lv.size(); ++l) {
      std::vector<AsmPatch> pt;
      std::vector<double> tab;
      make_assembly_tables(H.prob, H.lv[l], pt, tab);
      pool = std::max(pool, tab.size());
      for (const AsmPatch& a : pt) {
        size_t sz[3];
        asm_slab_sizes(H.prob.d, a, sz);
        for (int i = 0; i < 3; ++i) sz_max[i] = std::max(sz_max[i], sz[i]);
      }
    }
    C.asm_flag = a.take<int>(H.prob.K);
    C.asm_tab = a.take<double>(pool);
    // Gs is dead once direction 0 has read it, and T2 is written only after
    // that (the next slab's metric stage follows this slab's last stage on
    // the stream), so the two share one region
    C.asm_gs = a.take<double>(std::max(sz_max[0], sz_max[2]));
    C.asm_t2 = C.asm_gs;
    C.asm_t1 = a.take<double>(sz_max[1]);
    size_t ne = 0, nc = 0;
    for (size_t l = 1; l < H.lv.size(); ++l)
      if (!H.lv[l].dg_ptr.empty()) {
        ne = std::max(ne, H.lv[l].dg_ptr.size());
        nc = std::max(nc, H.lv[l].dg_row.size());
      }
    if (ne > 0) {
      C.dg_ptr = a.take<int64_t>(ne);
      C.dg_row = a.take<int64_t>(nc);
      C.dg_plane = a.take<int>(nc);
      C.dg_out = a.take<double>(ne);
    }
    if (C.noalloc) C.setup_bytes = sb.pos;
  }
  return std::max(b.pos, scratch_end) + 256;
}

template <typename T, typename Alloc>
static void up(T* dst, const std::vector<T, Alloc>& src, hipStream_t st) {
  if (!src.empty()) {
    HIP_OK(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st));
    HIP_OK(hipStreamSynchronize(st));
  }
}

static std::vector<float> to_float(const std::vector<double>& v) { return std::vector<float>(v.begin(), v.end()); }

// A symmetric n x n matrix (full, row-major) in packed lower tiles
// (layout.hpp), padding rows and columns zero with `pad` on the diagonal.
static DenseBuf pack_coarse_tiles(const double* A, int64_t n, double pad) {
  const int64_t T = coarse_tiles(n);
  DenseBuf out((size_t)coarse_packed_entries(n));
  for (int64_t I = 0; I < T; ++I)
    for (int64_t J = 0; J <= I; ++J) {
      double* t = out.data() + coarse_tile_at(I, J);
      for (int r = 0; r < COARSE_TILE; ++r) {
        const int64_t i = I * COARSE_TILE + r;
        for (int c = 0; c < COARSE_TILE; ++c) {
          const int64_t j = J * COARSE_TILE + c;
          t[r * COARSE_TILE + c] = (i < n && j < n) ? A[i * n + j] : (i == j ? pad : 0.0);
        }
      }
    }
  return out;
}

// The exact coarse solver of large coarse problems (Sec. 4): A_0^{-1} formed
// on the device by the library's own tiled Cholesky factorization and
// inversion (coarse.hip) in the scratch region, which the level data
// occupies later.  No library handle, allocation or lock is involved.
static void factor_coarse_on_device(igamg_ctx& C, hipStream_t st) {
  const int64_t n = C.N0;
  double* Lt = static_cast<double*>(C.coarse_ws);
  double* Yt = Lt + coarse_packed_entries(n);
  {
    const DenseBuf packed = pack_coarse_tiles(C.H.A0.data(), n, 1.0);
    up(Lt, packed, st);
  }
  coarse_inverse(Lt, Yt, C.Ainv, n, C.coarse_info, st);
  HIP_OK(hipGetLastError());
  int info = 0;
  HIP_OK(hipMemcpyAsync(&info, C.coarse_info, sizeof(info), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  if (info != 0)
    throw SetupError{IGAMG_ENOTSPD, "coarse matrix is not positive definite (pivot " + std::to_string(info) +
                                        "; is any side Dirichlet?)"};
  setup_progress("coarse inverse on the device; unknowns", (double)n);
}

// The FP32 copy of a level's band from its FP64 half band on the device: the
// half band rounded (scatter form) or the full band expanded from it.
static void fp32_band(igamg_ctx& C, DevLevel& D, hipStream_t st) {
  if (D.sym_ws > 0)
    launch_to_float(D.d64.band, D.d32.band, (int64_t)D.nbh * D.NL, st);
  else
    launch_band_half_to_full(C.d, C.p, D.d32.band, D.d64.band, D.bpatch, D.pd, D.NL, st);
  HIP_OK(hipGetLastError());
}

// Assembles level l's banded patch matrices on the device, straight into its
// tiled FP64 band (and the FP32 copy); the level's patch table, free flags and
// row-block map must be on the device already.
static void device_assemble(igamg_ctx& C, size_t l, hipStream_t st) {
  const Hierarchy& H = C.H;
  const LevelH& L = H.lv[l];
  DevLevel& D = C.dl[l];
  const int d = H.prob.d, K = H.prob.K;
  std::vector<AsmPatch> pt;
  std::vector<double> tab;
  make_assembly_tables(H.prob, L, pt, tab);
  up(C.asm_tab, tab, st);
  HIP_OK(hipMemsetAsync(C.asm_flag, 0, (size_t)K * sizeof(int), st));
  for (int k = 0; k < K; ++k)
    for (int e2 = 0; e2 < pt[k].nel[2]; ++e2)
      HIP_OK(launch_asm_slab(d, pt[k], C.asm_tab, e2, C.asm_gs, C.asm_t1, C.asm_t2, D.d64.band, D.nbh, C.asm_flag + k,
                             st));
  launch_asm_mask(d, H.prob.p, D.pd, D.bpatch, D.isfree, D.d64.band, D.nbh, D.NL, st);
  HIP_OK(hipGetLastError());
  std::vector<int> flags(K, 0);
  HIP_OK(hipMemcpyAsync(flags.data(), C.asm_flag, (size_t)K * sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  for (int k = 0; k < K; ++k)
    if ((flags[k] & 4) || ((flags[k] & 1) && (flags[k] & 2)))
      throw SetupError{IGAMG_EGEOM, "patch " + std::to_string(k) + ": det J vanishes or changes sign"};
  if (C.mixed) fp32_band(C, D, st);
  HIP_OK(hipStreamSynchronize(st));
  setup_progress("assembled on the device: level", (double)l);
}

static void upload(igamg_ctx& C, hipStream_t st) {
  Hierarchy& H = C.H;
  HIP_OK(hipMemsetAsync(C.ws, 0, C.bytes, st));
  if (!H.A0.empty()) {
    factor_coarse_on_device(C, st);
    DenseBuf().swap(H.A0);
    // the scratch was lent from the level data: zero it again
    HIP_OK(hipMemsetAsync(static_cast<char*>(C.ws) + C.scratch_at, 0, C.bytes - C.scratch_at, st));
    HIP_OK(hipStreamSynchronize(st));
  } else {
    up(C.Ainv, pack_coarse_tiles(H.Ainv.data(), C.N0, 0.0), st);
  }
  if (C.mixed) launch_to_float(C.Ainv, C.Ainv32, coarse_packed_entries(C.N0), st);
  for (size_t l = 0; l < H.lv.size(); ++l) {
    LevelH& L = H.lv[l];
    DevLevel& D = C.dl[l];
    up(D.bpatch, L.bpatch, st);
    up(D.pd, L.pd, st);
    up(D.isfree, L.isfree, st);
    up(D.gptr, L.gptr, st);
    up(D.gidx, L.gidx, st);
    if (l == 0) continue;
    if (assemble_on_device(H.opt, true)) {
      device_assemble(C, l, st);
      if (!L.dg_row.empty()) {
        // exact edge and vertex pieces: gather their entries from the band
        const int64_t ne = (int64_t)L.dg_ptr.size() - 1;
        up(C.dg_ptr, L.dg_ptr, st);
        up(C.dg_row, L.dg_row, st);
        up(C.dg_plane, L.dg_plane, st);
        launch_band_gather(D.d64.band, D.nbh, C.dg_ptr, C.dg_row, C.dg_plane, ne, C.dg_out, st);
        HIP_OK(hipGetLastError());
        std::vector<double> vals(ne);
        HIP_OK(hipMemcpyAsync(vals.data(), C.dg_out, ne * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        finish_direct_pieces(L, vals);
      }
    } else {
      // tiled symmetric half-band (layout.hpp): the stored planes of each
      // 256-row block are contiguous, band[(row/256)*nbh*256 + plane*256 + row%256];
      // plane P+1+(L-LC-1)*NB+o0 (or o0-P on the centre line) is the full
      // band's offset o0 + NB*L
      const int p = H.prob.p, nb1 = 2 * p + 1, lc = (band_lines(H.prob.d, p) - 1) / 2;
      std::vector<int> full_of(D.nbh);
      for (int pl = 0; pl < D.nbh; ++pl)
        full_of[pl] = pl <= p ? (pl + p) + nb1 * lc : (pl - p - 1) % nb1 + nb1 * (lc + 1 + (pl - p - 1) / nb1);
      std::vector<double> tiled((size_t)D.nbh * L.NL);
      const int64_t nblk = L.NL / ROW_ALIGN;
      for (int64_t bk = 0; bk < nblk; ++bk)
        for (int pl = 0; pl < D.nbh; ++pl)
          std::memcpy(&tiled[((size_t)bk * D.nbh + pl) * ROW_ALIGN],
                      &L.band[(size_t)full_of[pl] * L.NL + bk * ROW_ALIGN], ROW_ALIGN * sizeof(double));
      up(D.d64.band, tiled, st);
      if (C.mixed && D.sym_ws > 0) {
        fp32_band(C, D, st);
      } else if (C.mixed) {
        // the FP32 copy keeps every plane, band[(row/256)*nb*256 + o*256 + row%256]
        std::vector<float> full32((size_t)D.nb * L.NL);
        for (int64_t bk = 0; bk < nblk; ++bk)
          for (int o = 0; o < D.nb; ++o)
            for (int r = 0; r < ROW_ALIGN; ++r)
              full32[((size_t)bk * D.nb + o) * ROW_ALIGN + r] = (float)L.band[(size_t)o * L.NL + bk * ROW_ALIGN + r];
        up(D.d32.band, full32, st);
      }
      std::vector<double>().swap(L.band);
      setup_progress("uploaded band of level", (double)l);
    }
    up(D.if_ptr, L.if_ptr, st);
    up(D.if_idx, L.if_idx, st);
    up(D.fd, L.fd, st);
    up(D.dense, L.dense, st);
    up(D.tr_idx, L.tr_idx, st);
    up(D.d64.fdmat, L.fdmat, st);
    up(D.d64.densemat, L.densemat, st);
    up(D.d64.tr_val, L.tr_val, st);
    if (C.mixed) {
      up(D.d32.fdmat, to_float(L.fdmat), st);
      up(D.d32.densemat, to_float(L.densemat), st);
      up(D.d32.tr_val, to_float(L.tr_val), st);
    }
  }
  for (auto& tl : C.tail)
    if (tl.nph > 0) up(tl.prog, tl.host, st);
  // the bands are large and no longer needed on the host
  for (auto& L : H.lv) std::vector<double>().swap(L.band);
  std::vector<double>().swap(H.Ainv);
}

// ---------------------------------------------------------------------------
// the cycle, templated on the storage precision
// ---------------------------------------------------------------------------
static hipEvent_t next_event(igamg_ctx& C) {
  if (C.pool_used == C.pool.size()) {
    hipEvent_t e;
    HIP_OK(hipEventCreate(&e));
    C.pool.push_back(e);
  }
  return C.pool[C.pool_used++];
}

template <typename T>
static void band_op(igamg_ctx& C, int l, const T* u, const T* f, T* r, bool resid, hipStream_t st) {
  DevLevel& D = C.dl[l];
  const T* band = dat<T>(D).band;
  T* win = static_cast<T*>(C.symwin);
  if (!C.prof) {
    if (D.sym_ws > 0)
      HIP_OK(launch_band_sym<T>(C.d, C.p, band, u, f, r, D.bpatch, D.pd, D.NL, D.sym_ws, win, resid, st));
    else
      HIP_OK(launch_band<T>(C.d, C.p, band, u, f, r, D.bpatch, D.pd, D.NL, resid, st));
    return;
  }
  igamg_ctx::Rec rc;
  rc.level = l + (sizeof(T) == 4 ? (int)C.dl.size() : 0);
  rc.bytes = (double)D.rows * sizeof(T) * ((double)(sizeof(T) == 8 || D.sym_ws > 0 ? D.nbh : D.nb) + (resid ? 3 : 2));
  rc.a = next_event(C);
  rc.b = next_event(C);
  if (D.sym_ws > 0)
    HIP_OK(launch_band_sym<T>(C.d, C.p, band, u, f, r, D.bpatch, D.pd, D.NL, D.sym_ws, win, resid, st, rc.a, rc.b));
  else
    HIP_OK(launch_band<T>(C.d, C.p, band, u, f, r, D.bpatch, D.pd, D.NL, resid, st, rc.a, rc.b));
  C.recs.push_back(rc);
  C.prof_stream = st;
}

// u <- u + tau L^{-1} src (or u = tau L^{-1} src when !add); src distributed.
// Forward products (+ D^{-1} for 2D tensors, + the dense pieces), for 3D
// interiors the scaled middle direction over pencils, inverse products.
template <typename T>
static void smoother_apply(igamg_ctx& C, int l, const T* src, T* u, bool add, double tau, hipStream_t st) {
  DevLevel& D = C.dl[l];
  LevelData<T>& X = dat<T>(D);
  const int variant = D.fdv[std::is_same<T, float>::value ? 1 : 0];
  if constexpr (std::is_same<T, float>::value) {
    const bool bf16 = variant == IGAMG_FD_MFMA_BF16;
    if ((variant == IGAMG_FD_FUSED || bf16) && D.max_m2 == 1) {
      // every item is a 2D tensor: one launch, each item held in LDS
      launch_fd2_fused(D.fd, D.nfd, D.ndense, fd2_fused_lds(D.fd_maxm, D.max_dense), D.dense, X.densemat, X.fdmat,
                       src, u, D.if_ptr, D.if_idx, tau, add, bf16, st);
      return;
    }
    if (variant == IGAMG_FD_MFMA || variant == IGAMG_FD_FUSED || bf16) {
      // FP32: forward and inverse mode products on the matrix cores
      const size_t lds = std::max(fd_mfma_lds(D.fd_maxm), fd_dense_lds(D.max_dense, sizeof(T)));
      launch_fd_fwd_mfma(D.fd, D.nfd, D.ndense, D.mfma_grid, lds, D.dense, X.densemat, X.fdmat, src, u, D.if_ptr,
                         D.if_idx, X.scr, tau, add, bf16, st);
      if (C.d == 3 && D.nfd_int > 0 && D.max_m2 > 1)
        launch_fd_mid<T>(D.fd, D.nfd_int, D.mid_grid, fd_mid_lds(D.fd_maxm, sizeof(T)), X.fdmat, X.scr, st);
      launch_fd_inv_mfma(D.fd, D.nfd, D.mfma_grid, fd_mfma_lds(D.fd_maxm), X.fdmat, u, D.if_ptr, D.if_idx, X.scr,
                         tau, add, bf16, st);
      return;
    }
  }
  {
    const int rb = variant == IGAMG_FD_VEC4 ? 4 : 8;
    const int grid = variant == IGAMG_FD_VEC4 ? D.slab_grid4 : D.slab_grid;
    const size_t lds = std::max(fd_slab_lds(D.fd_maxm, sizeof(T)), fd_dense_lds(D.max_dense, sizeof(T)));
    launch_fd_fwd<T>(D.fd, D.nfd, D.ndense, grid, lds, D.dense, X.densemat, X.fdmat, src, u, D.if_ptr, D.if_idx,
                     X.scr, tau, add, rb, st);
    if (C.d == 3 && D.nfd_int > 0 && D.max_m2 > 1)
      launch_fd_mid<T>(D.fd, D.nfd_int, D.mid_grid, fd_mid_lds(D.fd_maxm, sizeof(T)), X.fdmat, X.scr, st);
    launch_fd_inv<T>(D.fd, D.nfd, grid, fd_slab_lds(D.fd_maxm, sizeof(T)), X.fdmat, u, D.if_ptr, D.if_idx, X.scr,
                     tau, add, rb, st);
  }
}

template <typename T>
static void coarse_solve(igamg_ctx& C, const T* f0, T* u0, hipStream_t st) {
  DevLevel& D = C.dl[0];
  launch_coarse<T>(coarse_inverse_of<T>(C), f0, C.cb, C.cpart, u0, D.gptr, D.gidx, C.N0, st);
}

template <typename T>
static void restrict_to(igamg_ctx& C, int l, const T* rf, T* rc, hipStream_t st) {
  DevLevel& F = C.dl[l];
  DevLevel& Cc = C.dl[l - 1];
  launch_restrict<T>(C.d, rf, rc, F.pd, Cc.bpatch, Cc.NL, F.tr_idx, dat<T>(F).tr_val, F.WR, Cc.isfree, st);
}

template <typename T>
static void prolong_add(igamg_ctx& C, int l, const T* uc, T* uf, hipStream_t st) {
  DevLevel& F = C.dl[l];
  launch_prolong_add<T>(C.d, uc, uf, F.pd, F.bpatch, F.NL, F.tr_idx, dat<T>(F).tr_val, F.WP, F.isfree, st);
}

// Algorithm 1 on level l >= 1 with u_l, f_l in dat<T>(dl[l]).u / .f
template <typename T>
static void cycle(igamg_ctx& C, int l, bool zero_init, hipStream_t st) {
  const igamg_ctx::Tail& tl = C.tail[std::is_same<T, float>::value ? 1 : 0];
  if (tl.nph > 0 && l == tl.level && zero_init) {
    // the whole cycle from here down, in one persistent launch
    HIP_OK(launch_cycle_tail<T>(C.d, C.p, tl.prog, tl.nph, tl.total, tl.ctr, tl.grid, tl.lds,
                                dat<T>(C.dl[tl.level]).u, st));
    return;
  }
  LevelData<T>& X = dat<T>(C.dl[l]);
  LevelData<T>& Xc = dat<T>(C.dl[l - 1]);
  const Options& O = C.H.opt;
  for (int i = 0; i < O.nu; ++i) {
    if (zero_init && i == 0) {
      smoother_apply<T>(C, l, X.f, X.u, false, O.tau, st);
    } else {
      band_op<T>(C, l, X.u, X.f, X.w, true, st);
      smoother_apply<T>(C, l, X.w, X.u, true, O.tau, st);
    }
  }
  band_op<T>(C, l, X.u, X.f, X.w, true, st);
  restrict_to<T>(C, l, X.w, Xc.f, st);
  if (l == 1) {
    coarse_solve<T>(C, Xc.f, Xc.u, st);
  } else {
    for (int j = 0; j < O.mu; ++j) cycle<T>(C, l - 1, j == 0, st);
  }
  prolong_add<T>(C, l, Xc.u, X.u, st);
  for (int i = 0; i < O.nu; ++i) {
    band_op<T>(C, l, X.u, X.f, X.w, true, st);
    smoother_apply<T>(C, l, X.w, X.u, true, O.tau, st);
  }
}

static bool trace_enabled() {
  static const bool on = std::getenv("IGAMG_TRACE") != nullptr;
  return on;
}

static double fetch(igamg_ctx& C, int slot, hipStream_t st) {
  HIP_OK(hipMemcpyAsync(C.host_scal + slot, C.scal + slot, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  return C.host_scal[slot];
}

template <typename T>
static PcgVecs<T>& vecs(igamg_ctx& C);
template <>
PcgVecs<double>& vecs<double>(igamg_ctx& C) {
  return C.v64;
}
template <>
PcgVecs<float>& vecs<float>(igamg_ctx& C) {
  return C.v32;
}

// ---------------------------------------------------------------------------
// PCG with one cycle as preconditioner (Sec. 4) on the finest level in
// precision T, split into the pieces the solve driver sequences.  The
// right-hand side is in dat<T>(finest).f and becomes the (canonical,
// distributed) recurrence residual; the iterate is vecs<T>.x.
// Direction update: classical beta = rho_new / rho for the FP64 solve; the
// flexible form beta = -alpha (z_new . q) / rho for the FP32 inner solves,
// whose cycle is symmetric only up to rounding.
// ---------------------------------------------------------------------------
template <typename T>
static void pcg_start(igamg_ctx& C, hipStream_t st) {
  DevLevel& D = C.dl[C.L];
  launch_fill<T>(vecs<T>(C).x, D.NL, 0.0, st);
  launch_norm2_dist<T>(dat<T>(D).f, D.gptr, D.gidx, D.N, C.part, C.scal, 6, true, st);
  HIP_OK(hipMemcpyAsync(C.host_scal + 6, C.scal + 6, sizeof(double), hipMemcpyDeviceToHost, st));
}

template <typename T>
static void pcg_first(igamg_ctx& C, hipStream_t st) {
  DevLevel& D = C.dl[C.L];
  LevelData<T>& X = dat<T>(D);
  cycle<T>(C, C.L, true, st);
  launch_dot<T>(X.f, X.u, D.NL, C.part, C.scal, 0, 0, st);
  launch_copy<T>(vecs<T>(C).p, X.u, D.NL, st);
}

// q = A p, alpha = rho / (p.q), x += alpha p, r -= alpha q, ||r||^2 to the host
template <typename T>
static void pcg_body_a(igamg_ctx& C, hipStream_t st) {
  DevLevel& D = C.dl[C.L];
  LevelData<T>& X = dat<T>(D);
  PcgVecs<T>& V = vecs<T>(C);
  band_op<T>(C, C.L, V.p, nullptr, V.q, false, st);
  launch_dot<T>(V.p, V.q, D.NL, C.part, C.scal, 1, 1, st);
  launch_axpy2<T>(V.x, V.p, X.f, V.q, D.NL, C.scal, st);
  launch_norm2_dist<T>(X.f, D.gptr, D.gidx, D.N, C.part, C.scal, 5, true, st);
  HIP_OK(hipMemcpyAsync(C.host_scal + 5, C.scal + 5, sizeof(double), hipMemcpyDeviceToHost, st));
}

// z = B r, beta, p = z + beta p
template <typename T>
static void pcg_body_b(igamg_ctx& C, hipStream_t st, bool flexible) {
  DevLevel& D = C.dl[C.L];
  LevelData<T>& X = dat<T>(D);
  PcgVecs<T>& V = vecs<T>(C);
  cycle<T>(C, C.L, true, st);
  if (flexible)
    launch_dot2_flex<T>(X.f, V.q, X.u, D.NL, C.part, C.scal, st);
  else
    launch_dot<T>(X.f, X.u, D.NL, C.part, C.scal, 3, 2, st);
  launch_xpby<T>(V.p, X.u, D.NL, C.scal, st);
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
#define API_BEGIN try {
#define API_END                                        \
  }                                                    \
  catch (const SetupError& e) {                        \
    return set_err(e.code, e.msg);                     \
  }                                                    \
  catch (const std::bad_alloc&) {                      \
    return set_err(IGAMG_EINVAL, "host out of memory"); \
  }                                                    \
  catch (const std::exception& e) {                    \
    return set_err(IGAMG_EINVAL, e.what());            \
  }

static void read_opts(const igamg_options* o, Options& O) {
  igamg_options def;
  igamg_default_options(&def);
  if (!o) o = &def;
  O.tau = o->tau;
  O.sigma_scale = o->sigma_scale;
  O.nu = o->nu;
  O.mu = o->mu;
  O.precision = o->precision;
  O.maxit = o->maxit;
  O.geometry_scaling = o->geometry_scaling;
  O.inner_maxit = o->inner_maxit;
  O.inner_tol = o->inner_tol;
  O.graphs = o->graphs;
  O.fd_mfma = o->fd_mfma;
  O.coarse_factor = o->coarse_factor;
  O.autotune = o->autotune;
  O.assembly = o->assembly;
  O.s1_sigma = o->s1_sigma;
  O.iface_multiplicity = o->iface_multiplicity;
  O.physical_h = o->physical_h;
  O.iface_direct = o->iface_direct;
  O.persistent = o->persistent;
  O.band_form = o->band_form;
  if (O.precision == IGAMG_MIXED_BF16) {
    if (O.fd_mfma != 0 && O.fd_mfma != 3) throw SetupError{IGAMG_EINVAL, "IGAMG_MIXED_BF16 sets fd_mfma = 3"};
    O.precision = IGAMG_MIXED;
    O.fd_mfma = 3;
  }
  if (O.s1_sigma < 0 || O.s1_sigma > 1 || O.iface_multiplicity < 0 || O.iface_multiplicity > 1 || O.physical_h < 0 ||
      O.physical_h > 1 || O.geometry_scaling < 0 || O.geometry_scaling > 1 || O.iface_direct < 0 ||
      O.iface_direct > 1 || O.persistent < 0 || O.persistent > 1 || O.band_form < 0 || O.band_form > 2)
    throw SetupError{IGAMG_EINVAL, "invalid options"};
  if (!(O.tau > 0) || !(O.sigma_scale > 0) || O.nu < 1 || O.nu > 8 || (O.mu != 1 && O.mu != 2) ||
      (O.precision != IGAMG_FP64 && O.precision != IGAMG_MIXED) || O.maxit < 1 || O.inner_maxit < 1 ||
      !(O.inner_tol > 0 && O.inner_tol < 1) || O.fd_mfma < 0 || O.fd_mfma > 3 || O.autotune < 0 || O.autotune > 1 ||
      O.coarse_factor < 0 || O.coarse_factor > 2 || O.assembly < 0 || O.assembly > 1)
    throw SetupError{IGAMG_EINVAL, "invalid options"};
}

static int check_level(igamg_ctx* h, int level) {
  if (level < 0) level = h->L;
  if (level > h->L) throw SetupError{IGAMG_EINVAL, "level out of range"};
  return level;
}

static void need_device(igamg_ctx* h) {
  if (!h) throw SetupError{IGAMG_EINVAL, "null handle"};
  if (!h->on_device) throw SetupError{IGAMG_EINVAL, "handle was set up without a workspace"};
}


// ---------------------------------------------------------------------------
// autotuner of the smoother variants (tile shapes), run once per handle at
// setup: per level and precision, every candidate is timed over a few
// smoother applications on the device and the fastest is kept.  Choices are
// cached per process (and in the JSON file named by IGAMG_TUNE_CACHE) under
// a key of the level's piece shapes, degree and precision.
// ---------------------------------------------------------------------------
namespace {
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;

const char* tune_file() { return std::getenv("IGAMG_TUNE_CACHE"); }

// the cache file is a flat JSON object of "key": variant pairs (keys are made
// of digits, letters and the characters x , : / only)
void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = tune_file();
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
  std::fclose(f);
  size_t pos = 0;
  while ((pos = text.find('"', pos)) != std::string::npos) {
    const size_t end = text.find('"', pos + 1);
    if (end == std::string::npos) break;
    const std::string key = text.substr(pos + 1, end - pos - 1);
    const size_t colon = text.find(':', end);
    if (colon == std::string::npos) break;
    const int v = std::atoi(text.c_str() + colon + 1);
    if (v >= IGAMG_FD_VEC8 && v <= IGAMG_FD_FUSED) g_tune[key] = v;
    pos = text.find_first_of(",}", colon);
    if (pos == std::string::npos) break;
  }
}

void tune_save_locked() {
  const char* path = tune_file();
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  std::fprintf(f, "{\n");
  size_t i = 0;
  for (const auto& kv : g_tune)
    std::fprintf(f, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++i < g_tune.size() ? "," : "");
  std::fprintf(f, "}\n");
  std::fclose(f);
  std::rename(tmp.c_str(), path);
}
}  // namespace

static std::string tune_key(const igamg_ctx& C, int l, bool fp32) {
  const LevelH& L = C.H.lv[l];
  std::string k = "gfx950/d" + std::to_string(C.d) + "p" + std::to_string(C.p) + (fp32 ? "/f32/" : "/f64/");
  for (const auto& it : L.fd)
    k += std::to_string(it.m[0]) + "x" + std::to_string(it.m[1]) + "x" + std::to_string(it.m[2]) +
         (it.src_if ? "f," : ",");
  k += ":" + std::to_string(L.dense.size()) + "x" + std::to_string(C.dl[l].max_dense);
  return k;
}

template <typename T>
static double time_smoother(igamg_ctx& C, int l, hipStream_t st) {
  LevelData<T>& X = dat<T>(C.dl[l]);
  hipEvent_t a, b;
  HIP_OK(hipEventCreate(&a));
  HIP_OK(hipEventCreate(&b));
  for (int i = 0; i < 2; ++i) smoother_apply<T>(C, l, X.f, X.u, false, C.H.opt.tau, st);
  HIP_OK(hipEventRecord(a, st));
  constexpr int reps = 5;
  for (int i = 0; i < reps; ++i) smoother_apply<T>(C, l, X.f, X.u, false, C.H.opt.tau, st);
  HIP_OK(hipEventRecord(b, st));
  HIP_OK(hipEventSynchronize(b));
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms / reps;
}

template <typename T>
static void tune_level(igamg_ctx& C, int l, hipStream_t st) {
  constexpr bool fp32 = std::is_same<T, float>::value;
  DevLevel& D = C.dl[l];
  int& v = D.fdv[fp32 ? 1 : 0];
  const Options& O = C.H.opt;
  // the matrix-core variants stage whole tensors in LDS: sides up to FD_LDS_M
  const bool mfma_ok = D.fd_maxm <= FD_LDS_M && D.max_dense <= FD_LDS_M;
  if (fp32 && O.fd_mfma == 1 && mfma_ok) { v = D.max_m2 == 1 ? IGAMG_FD_FUSED : IGAMG_FD_MFMA; return; }
  if (fp32 && O.fd_mfma == 2) { v = IGAMG_FD_VEC8; return; }
  if (fp32 && O.fd_mfma == 3 && mfma_ok) { v = IGAMG_FD_MFMA_BF16; return; }
  if (fp32 && O.fd_mfma != 0 && !mfma_ok) { v = IGAMG_FD_VEC8; return; }
  if (!O.autotune || D.nfd + D.ndense == 0) { v = IGAMG_FD_VEC8; return; }
  const std::string key = tune_key(C, l, fp32);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(key);
    if (it != g_tune.end()) { v = it->second; return; }
  }
  std::vector<int> cand{IGAMG_FD_VEC8, IGAMG_FD_VEC4};
  if (fp32 && mfma_ok) cand.push_back(IGAMG_FD_MFMA);
  if (fp32 && mfma_ok && D.max_m2 == 1) cand.push_back(IGAMG_FD_FUSED);
  int best = IGAMG_FD_VEC8;
  double best_ms = 1e300;
  for (int c : cand) {
    v = c;
    const double ms = time_smoother<T>(C, l, st);
    if (ms < best_ms) { best_ms = ms; best = c; }
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto ins = g_tune.emplace(key, best);   // a concurrent setup may have tuned the same shapes first
  v = ins.first->second;
  if (ins.second) tune_save_locked();
}

static void autotune(igamg_ctx& C, hipStream_t st) {
  for (int l = 1; l <= C.L; ++l) {
    tune_level<double>(C, l, st);
    if (C.mixed) tune_level<float>(C, l, st);
  }
  HIP_OK(hipStreamSynchronize(st));
  setup_progress("smoother variants chosen", 0);
}

// ---------------------------------------------------------------------------
// solve driver: per-request state machines stepped in lockstep.  One step is
// one PCG iteration of every iterating request, as two HIP graphs (body A:
// apply, alpha, update, residual norm; body B: cycle, beta, direction) in
// which every request is an independent branch on its own stream.  Between
// the graphs the host reads every request's residual norm; starts of a PCG
// and the FP64 refinement steps of mixed requests run outside the graphs.
// ---------------------------------------------------------------------------
enum { RQ_FREE = 0, RQ_START_READ, RQ_ITER, RQ_OUTER_READ, RQ_DONE };

struct Req {
  igamg_ctx* C = nullptr;
  const double* rhs = nullptr;
  double* u = nullptr;
  double tol = 1e-8;
  int state = RQ_FREE;
  bool mixed = false, first_outer = true, fresh_done = false;
  // mixed: the FP32 inner solves stalled, and the solve was restarted as the
  // FP64 PCG from u = 0
  bool fp64_tail = false;
  int it = 0, iters = 0, outer = 0, code = IGAMG_OK;
  double n02 = 0.0, nf2 = 0.0, rel = 1.0, prev_rel = 1.0;
  double inner_target = 1e-4;   // relative residual reduction the current inner solve stops at
  std::chrono::steady_clock::time_point t0;
  double solve_ms = 0.0;
};

struct igamg_batch_ctx {
  hipStream_t ds = nullptr;
  std::vector<hipStream_t> br;
  std::vector<hipEvent_t> ev_join;
  hipEvent_t ev_fork = nullptr, ev_in = nullptr;
  std::vector<Req> reqs;
  ~igamg_batch_ctx() {
    for (auto e : ev_join) (void)hipEventDestroy(e);
    for (auto s : br) (void)hipStreamDestroy(s);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ds) (void)hipStreamDestroy(ds);
  }
};

static void batch_init(igamg_batch_ctx& B) {
  if (B.ds) return;
  HIP_OK(hipStreamCreateWithFlags(&B.ds, hipStreamNonBlocking));
  HIP_OK(hipEventCreateWithFlags(&B.ev_fork, hipEventDisableTiming));
  HIP_OK(hipEventCreateWithFlags(&B.ev_in, hipEventDisableTiming));
}

static void batch_branches(igamg_batch_ctx& B, size_t n) {
  while (B.br.size() < n) {
    hipStream_t s;
    hipEvent_t e;
    HIP_OK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    B.br.push_back(s);
    B.ev_join.push_back(e);
  }
}

// per-launch event timing (igamg_profile) runs with direct launches: HIP does
// not time events that were recorded into a graph
static bool graphs_enabled(const igamg_batch_ctx& B, const std::vector<int>& set) {
  for (int i : set)
    if (!B.reqs[i].C->H.opt.graphs || B.reqs[i].C->prof) return false;
  return true;
}

static void sync_driver(igamg_batch_ctx& B) { HIP_OK(hipStreamSynchronize(B.ds)); }

static void body(Req& q, int which, hipStream_t st) {
  igamg_ctx& C = *q.C;
  const bool f32 = q.mixed && !q.fp64_tail;
  if (which == 0) {
    if (f32) pcg_body_a<float>(C, st); else pcg_body_a<double>(C, st);
  } else {
    if (f32) pcg_body_b<float>(C, st, true); else pcg_body_b<double>(C, st, false);
  }
}

// The PCG bodies of one hierarchy, captured once as graphs.  A body touches
// only its own hierarchy's memory, so the same graph serves every batch the
// hierarchy ever joins, whatever the other members are.
// The hierarchy's graph of body `which`, captured on first use.
static hipGraphExec_t request_graph(igamg_batch_ctx& B, Req& q, int which) {
  igamg_ctx& C = *q.C;
  const int slot = which + (q.mixed && q.fp64_tail ? 2 : 0);
  if (!C.gx[slot]) {
    hipGraph_t g = nullptr;
    HIP_OK(hipStreamBeginCapture(B.ds, hipStreamCaptureModeThreadLocal));
    body(q, which, B.ds);
    HIP_OK(hipStreamEndCapture(B.ds, &g));
    HIP_OK(hipGraphInstantiate(&C.gx[slot], g, nullptr, nullptr, 0));
    HIP_OK(hipGraphDestroy(g));
  }
  return C.gx[slot];
}

// run body `which` for the requests in `set` on the driver stream
static void run_bodies(igamg_batch_ctx& B, const std::vector<int>& set, int which) {
  if (set.empty()) return;
  if (!graphs_enabled(B, set)) {
    for (int i : set) body(B.reqs[i], which, B.ds);
    return;
  }
  // one graph per hierarchy, each on a branch stream of its own: requests
  // joining or leaving the batch cost no capture
  std::vector<hipGraphExec_t> gs;
  for (int i : set) gs.push_back(request_graph(B, B.reqs[i], which));
  if (gs.size() == 1) {
    HIP_OK(hipGraphLaunch(gs[0], B.ds));
    return;
  }
  batch_branches(B, gs.size());
  HIP_OK(hipEventRecord(B.ev_fork, B.ds));
  for (size_t k = 0; k < gs.size(); ++k) {
    HIP_OK(hipStreamWaitEvent(B.br[k], B.ev_fork, 0));
    HIP_OK(hipGraphLaunch(gs[k], B.br[k]));
    HIP_OK(hipEventRecord(B.ev_join[k], B.br[k]));
    HIP_OK(hipStreamWaitEvent(B.ds, B.ev_join[k], 0));
  }
}

static void rq_finish(Req& q, int code, hipStream_t st) {
  igamg_ctx& C = *q.C;
  DevLevel& D = C.dl[C.L];
  launch_gather(C.v64.x, q.u, D.gptr, D.gidx, D.N, false, st);
  q.code = code;
  q.state = RQ_DONE;
  q.fresh_done = true;
}

// mixed: start an inner FP32 solve for the current FP64 residual
static void rq_start_inner(Req& q, hipStream_t st) {
  igamg_ctx& C = *q.C;
  DevLevel& D = C.dl[C.L];
  // reduce the outer residual (relative value q.rel) just past the target,
  // with a margin of 2, but never ask an FP32 solve for more than inner_tol
  q.inner_target = std::max(C.H.opt.inner_tol, 0.5 * q.tol / std::max(q.rel, 1e-300));
  launch_to_f32(D.d32.f, D.d64.f, D.NL, st);
  pcg_start<float>(C, st);
  q.it = 0;
  q.state = RQ_START_READ;
}

// mixed: x += d, r = f - A x in FP64, ||r||^2 to the host
static void rq_outer_update(Req& q, hipStream_t st) {
  igamg_ctx& C = *q.C;
  DevLevel& D = C.dl[C.L];
  launch_add_f32(C.v64.x, C.v32.x, D.NL, st);
  band_op<double>(C, C.L, C.v64.x, C.fsave, D.d64.f, true, st);
  launch_norm2_dist<double>(D.d64.f, D.gptr, D.gidx, D.N, C.part, C.scal, 7, true, st);
  HIP_OK(hipMemcpyAsync(C.host_scal + 7, C.scal + 7, sizeof(double), hipMemcpyDeviceToHost, st));
  q.state = RQ_OUTER_READ;
}

// mixed: the inner FP32 solves stopped reducing the FP64 residual, or broke
// down (a non-finite inner residual).  The solve restarts as the FP64 PCG
// from u = 0, the FP64 handle's own algorithm: an iterate that FP32 could not
// improve may lie far from the solution, and a correction solved from it
// would need more than FP64's attainable accuracy on such ill-conditioned
// operators.
static void rq_fallback_fp64(Req& q, hipStream_t st) {
  igamg_ctx& C = *q.C;
  DevLevel& D = C.dl[C.L];
  if (trace_enabled()) std::fprintf(stderr, "[igamg] %p FP64 PCG from u = 0 (rel %.3e)\n", (void*)q.C, q.rel);
  launch_copy<double>(D.d64.f, C.fsave, D.NL, st);
  q.fp64_tail = true;
  q.rel = 1.0;
  q.it = 0;
  pcg_start<double>(C, st);
  q.state = RQ_START_READ;
}

static void rq_begin(Req& q, hipStream_t st) {
  igamg_ctx& C = *q.C;
  DevLevel& D = C.dl[C.L];
  q.t0 = std::chrono::steady_clock::now();
  q.it = q.iters = q.outer = 0;
  q.code = IGAMG_OK;
  q.rel = q.prev_rel = 1.0;
  q.first_outer = true;
  q.fp64_tail = false;
  if (!q.mixed) {
    launch_scatter(q.rhs, D.d64.f, D.gptr, D.gidx, D.N, true, st);
    pcg_start<double>(C, st);
    q.state = RQ_START_READ;
  } else {
    launch_scatter(q.rhs, C.fsave, D.gptr, D.gidx, D.N, true, st);
    launch_fill<double>(C.v64.x, D.NL, 0.0, st);
    launch_copy<double>(D.d64.f, C.fsave, D.NL, st);
    launch_norm2_dist<double>(D.d64.f, D.gptr, D.gidx, D.N, C.part, C.scal, 7, true, st);
    HIP_OK(hipMemcpyAsync(C.host_scal + 7, C.scal + 7, sizeof(double), hipMemcpyDeviceToHost, st));
    q.state = RQ_OUTER_READ;
  }
}

static void trace_iter(const Req& q, double rel) {
  if (trace_enabled())
    std::fprintf(stderr, "[igamg] %p pcg<%s> it %d rel %.3e\n", (void*)q.C, q.mixed && !q.fp64_tail ? "f32" : "f64",
                 q.it, rel);
}

// process a request whose host readback (start or outer norm) is available
static void rq_process_read(Req& q, hipStream_t st) {
  igamg_ctx& C = *q.C;
  const Options& O = C.H.opt;
  if (q.state == RQ_START_READ) {
    const double n02 = C.host_scal[6];
    if (!std::isfinite(n02)) return rq_finish(q, IGAMG_ENAN, st);
    if (n02 == 0.0) {
      if (!q.mixed || q.fp64_tail) {
        q.rel = 0.0;
        return rq_finish(q, IGAMG_OK, st);
      }
      return rq_outer_update(q, st);
    }
    q.n02 = n02;
    if (q.mixed && !q.fp64_tail) pcg_first<float>(C, st); else pcg_first<double>(C, st);
    q.state = RQ_ITER;
    return;
  }
  if (q.state == RQ_OUTER_READ) {
    const double rr = C.host_scal[7];
    if (!std::isfinite(rr)) return rq_finish(q, IGAMG_ENAN, st);
    if (q.first_outer) {
      q.first_outer = false;
      q.nf2 = rr;
      if (rr == 0.0) {
        q.rel = 0.0;
        return rq_finish(q, IGAMG_OK, st);
      }
    } else {
      q.outer++;
      q.rel = std::sqrt(rr / q.nf2);
      if (trace_enabled()) std::fprintf(stderr, "[igamg] %p refinement %d rel %.3e\n", (void*)q.C, q.outer, q.rel);
      if (q.rel <= q.tol) return rq_finish(q, IGAMG_OK, st);
      if (q.iters >= O.maxit || q.outer >= 60) return rq_finish(q, IGAMG_ENOCONV, st);
      // a refinement asked for at least a 10x reduction that cut the
      // residual by less than 4x: FP32 cannot resolve this operator (high
      // degree in 3D), so finish in FP64
      if (q.inner_target <= 0.1 && !(q.rel <= 0.25 * q.prev_rel)) return rq_fallback_fp64(q, st);
      q.prev_rel = q.rel;
    }
    return rq_start_inner(q, st);
  }
}

// after body A: one PCG iteration done for q
static bool rq_after_iter(Req& q, hipStream_t st) {
  igamg_ctx& C = *q.C;
  const Options& O = C.H.opt;
  const double rr = C.host_scal[5];
  q.it++;
  q.iters++;
  if (!std::isfinite(rr)) {
    if (q.mixed && !q.fp64_tail) rq_fallback_fp64(q, st);   // an FP32 breakdown
    else rq_finish(q, IGAMG_ENAN, st);
    return false;
  }
  const double rel = std::sqrt(rr / q.n02);
  trace_iter(q, rel);
  if (!q.mixed || q.fp64_tail) {
    q.rel = rel;
    if (q.rel <= q.tol) {
      rq_finish(q, IGAMG_OK, st);
      return false;
    }
    if (q.iters >= O.maxit) {
      rq_finish(q, IGAMG_ENOCONV, st);
      return false;
    }
    return true;
  }
  // an inner solve that has not halved its residual in 20 iterations is
  // stalled: end it, and the outer test decides on the FP64 restart
  if (rel <= q.inner_target || q.it >= O.inner_maxit || q.iters >= O.maxit || (q.it >= 20 && rel > 0.5)) {
    rq_outer_update(q, st);
    return false;
  }
  return true;
}

static int batch_step(igamg_batch_ctx& B, hipStream_t caller) {
  batch_init(B);
  HIP_OK(hipEventRecord(B.ev_in, caller));
  HIP_OK(hipStreamWaitEvent(B.ds, B.ev_in, 0));
  // settle every pending readback (a start may lead to another start)
  for (int pass = 0; pass < 8; ++pass) {
    bool pending = false;
    for (auto& q : B.reqs) pending |= (q.state == RQ_START_READ || q.state == RQ_OUTER_READ);
    if (!pending) break;
    sync_driver(B);
    std::vector<int> idx;
    for (size_t i = 0; i < B.reqs.size(); ++i)
      if (B.reqs[i].state == RQ_START_READ || B.reqs[i].state == RQ_OUTER_READ) idx.push_back((int)i);
    for (int i : idx) rq_process_read(B.reqs[i], B.ds);
  }
  std::vector<int> set;
  for (size_t i = 0; i < B.reqs.size(); ++i)
    if (B.reqs[i].state == RQ_ITER) set.push_back((int)i);
  bool finished = false;
  if (!set.empty()) {
    run_bodies(B, set, 0);
    sync_driver(B);
    std::vector<int> cont;
    for (int i : set) {
      if (rq_after_iter(B.reqs[i], B.ds))
        cont.push_back(i);
      else
        finished |= (B.reqs[i].state == RQ_DONE);
    }
    run_bodies(B, cont, 1);
  }
  for (auto& q : B.reqs) finished |= q.fresh_done;
  // a request reported done must have its result in place; otherwise the
  // next step's work queues behind this one without a host round trip
  if (finished) {
    sync_driver(B);
    const auto now = std::chrono::steady_clock::now();
    for (auto& q : B.reqs)
      if (q.fresh_done) {
        q.fresh_done = false;
        q.solve_ms = std::chrono::duration<double, std::milli>(now - q.t0).count();
      }
  }
  int active = 0;
  for (auto& q : B.reqs) active += (q.state != RQ_FREE && q.state != RQ_DONE);
  return active;
}

static int batch_add(igamg_batch_ctx& B, igamg_ctx* h, const double* rhs, double* u, double tol, hipStream_t caller) {
  need_device(h);
  if (!rhs || !u || rhs == u) throw SetupError{IGAMG_EINVAL, "bad vector arguments"};
  if (!(tol > 0)) throw SetupError{IGAMG_EINVAL, "tol must be positive"};
  for (auto& q : B.reqs)
    if (q.C == h && q.state != RQ_FREE && q.state != RQ_DONE)
      throw SetupError{IGAMG_EINVAL, "handle already has a running solve in this batch"};
  batch_init(B);
  HIP_OK(hipEventRecord(B.ev_in, caller));
  HIP_OK(hipStreamWaitEvent(B.ds, B.ev_in, 0));
  int slot = -1;
  for (size_t i = 0; i < B.reqs.size(); ++i)
    if (B.reqs[i].state == RQ_FREE) {
      slot = (int)i;
      break;
    }
  if (slot < 0) {
    slot = (int)B.reqs.size();
    B.reqs.emplace_back();
  }
  Req& q = B.reqs[slot];
  q = Req{};
  q.C = h;
  q.rhs = rhs;
  q.u = u;
  q.tol = tol;
  q.mixed = h->mixed;
  rq_begin(q, B.ds);
  return slot;
}

static void fill_info(const Req& q, igamg_solve_info* info) {
  if (!info) return;
  info->iterations = q.iters;
  info->outer_iterations = q.outer;
  info->converged = (q.state == RQ_DONE && q.code == IGAMG_OK);
  info->rel_residual = q.rel;
  info->solve_ms = q.solve_ms;
  info->fp64_fallback = q.fp64_tail ? 1 : 0;
}

// ---------------------------------------------------------------------------
// exported entry points
// ---------------------------------------------------------------------------
// the no-allocation setup's scratch (igamg_setup_noalloc)
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
static std::mutex g_noalloc_mu;             // one no-allocation setup at a time
static std::map<int, char*> g_scratch_at;   // device -> address of its `scratch`, under g_noalloc_mu

// The address of `scratch` on the current device, looked up once per device.
static char* noalloc_scratch() {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  auto it = g_scratch_at.find(dev);
  if (it != g_scratch_at.end()) return it->second;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    throw SetupError{IGAMG_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
  g_scratch_at[dev] = static_cast<char*>(ptr);
  return static_cast<char*>(ptr);
}

extern "C" {

void igamg_default_options(igamg_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tau = 0.25;
  o->sigma_scale = 5.0;
  o->nu = 1;
  o->mu = 1;
  o->precision = IGAMG_FP64;
  o->maxit = 500;
  o->geometry_scaling = 0;
  o->s1_sigma = 1;
  o->inner_maxit = 100;
  o->inner_tol = 1e-4;
  o->graphs = 1;
  o->autotune = 1;
}

const char* igamg_last_error(void) { return g_err.c_str(); }

int igamg_workspace_size(const igamg_problem* prob, const igamg_options* opts, size_t* bytes) {
  API_BEGIN
  if (!bytes) return set_err(IGAMG_EINVAL, "bytes is NULL");
  igamg_ctx C;
  C.H.prob = read_problem(prob);
  read_opts(opts, C.H.opt);
  C.mixed = C.H.opt.precision == IGAMG_MIXED;
  build_topology(C.H, false);
  *bytes = plan(C, nullptr);
  return IGAMG_OK;
  API_END
}

int igamg_setup(const igamg_problem* prob, const igamg_options* opts, void* workspace, size_t bytes, void* stream,
                igamg_handle* out) {
  API_BEGIN
  if (!out) return set_err(IGAMG_EINVAL, "out is NULL");
  *out = nullptr;
  igamg_ctx* C = new igamg_ctx();
  try {
    C->H.prob = read_problem(prob);
    read_opts(opts, C->H.opt);
    C->mixed = C->H.opt.precision == IGAMG_MIXED;
    C->d = C->H.prob.d;
    C->p = C->H.prob.p;
    C->L = C->H.prob.levels - 1;
    build_all(C->H, workspace != nullptr);
    size_t need = plan(*C, nullptr);
    if (workspace) {
      if (bytes < need) throw SetupError{IGAMG_ENOMEM, "workspace too small: need " + std::to_string(need)};
      if (reinterpret_cast<uintptr_t>(workspace) & 255) throw SetupError{IGAMG_EINVAL, "workspace not 256-byte aligned"};
      C->ws = workspace;
      C->bytes = need;
      plan(*C, static_cast<char*>(workspace));
      HIP_OK(hipHostMalloc(reinterpret_cast<void**>(&C->host_scal), 16 * sizeof(double), hipHostMallocDefault));
      upload(*C, static_cast<hipStream_t>(stream));
      C->on_device = true;
      autotune(*C, static_cast<hipStream_t>(stream));
    }
  } catch (...) {
    igamg_destroy(C);   // also frees what a partial setup acquired (pinned scalars, graphs, events)
    throw;
  }
  *out = C;
  return IGAMG_OK;
  API_END
}

// Setup without any allocation: the setup-only scratch of the device
// assembly (quadrature and geometry tables, det J flags, one element slab's
// intermediates, the gather lists of exact edge and vertex pieces) is taken
// from this static device array instead of the workspace.  Every GPU keeps
// its own copy for the life of the process; its address on the current
// device comes from hipGetSymbolAddress (the array's name is a host stand-in
// in host code, not a device address).  Calls are serialised by a mutex, and
// each call clears what it needs zeroed (the flags) and writes every other
// region before reading it, so nothing depends on what the last call left.
int igamg_setup_noalloc(const igamg_problem* prob, const igamg_options* opts, void* workspace, size_t bytes,
                        void* stream, igamg_handle* out, size_t* needed) {
  API_BEGIN
  if (!workspace && !needed) return set_err(IGAMG_EINVAL, "workspace and needed are both NULL");
  if (workspace && !out) return set_err(IGAMG_EINVAL, "out is NULL");
  if (out) *out = nullptr;
  igamg_ctx* C = new igamg_ctx();
  try {
    C->noalloc = true;
    C->H.prob = read_problem(prob);
    read_opts(opts, C->H.opt);
    // scalar readbacks go to a plain host array, which graph capture cannot
    // target: these handles launch their kernels directly
    C->H.opt.graphs = 0;
    C->mixed = C->H.opt.precision == IGAMG_MIXED;
    C->d = C->H.prob.d;
    C->p = C->H.prob.p;
    C->L = C->H.prob.levels - 1;
    build_all(C->H, true);
    const size_t need = plan(*C, nullptr);
    if (C->setup_bytes > NOALLOC_SCRATCH_BYTES)
      throw SetupError{IGAMG_EINVAL, "setup scratch of " + std::to_string(C->setup_bytes) +
                                         " bytes exceeds the static " + std::to_string(NOALLOC_SCRATCH_BYTES) +
                                         " bytes of the no-allocation setup"};
    if (needed) *needed = need;
    if (workspace) {
      if (bytes < need) throw SetupError{IGAMG_ENOMEM, "workspace too small: need " + std::to_string(need)};
      if (reinterpret_cast<uintptr_t>(workspace) & 255) throw SetupError{IGAMG_EINVAL, "workspace not 256-byte aligned"};
      std::lock_guard<std::mutex> lock(g_noalloc_mu);
      C->setup_base = noalloc_scratch();
      C->ws = workspace;
      C->bytes = need;
      plan(*C, static_cast<char*>(workspace));
      C->host_scal = C->host_scal_own;
      upload(*C, static_cast<hipStream_t>(stream));
      C->on_device = true;
      autotune(*C, static_cast<hipStream_t>(stream));
    }
  } catch (...) {
    igamg_destroy(C);
    throw;
  }
  if (!workspace) {
    igamg_destroy(C);
    return IGAMG_OK;
  }
  *out = C;
  return IGAMG_OK;
  API_END
}

int igamg_profile(igamg_handle h, int enable) {
  API_BEGIN
  need_device(h);
  h->prof = enable != 0;
  return IGAMG_OK;
  API_END
}

int igamg_profile_read(igamg_handle h, int64_t* launches, double* ms, double* bytes) {
  API_BEGIN
  need_device(h);
  const int nl = 2 * (int)h->dl.size();
  for (int l = 0; l < nl; ++l) {
    if (launches) launches[l] = 0;
    if (ms) ms[l] = 0.0;
    if (bytes) bytes[l] = 0.0;
  }
  if (!h->recs.empty()) HIP_OK(hipStreamSynchronize(h->prof_stream));
  if (h->solo && h->solo->ds) HIP_OK(hipStreamSynchronize(h->solo->ds));
  for (const auto& rc : h->recs) {
    float t = 0.0f;
    HIP_OK(hipEventElapsedTime(&t, rc.a, rc.b));
    if (launches) launches[rc.level] += 1;
    if (ms) ms[rc.level] += t;
    if (bytes) bytes[rc.level] += rc.bytes;
  }
  h->recs.clear();
  h->pool_used = 0;
  return IGAMG_OK;
  API_END
}

int igamg_destroy(igamg_handle h) {
  if (!h) return IGAMG_OK;
  // the handle's own streams drain before its graphs and events go away; work
  // that a caller's batch queued must have finished (igamg_batch_remove)
  if (h->solo && h->solo->ds) (void)hipStreamSynchronize(h->solo->ds);
  delete h->solo;
  for (hipGraphExec_t g : h->gx)
    if (g) (void)hipGraphExecDestroy(g);
  for (hipEvent_t e : h->pool) (void)hipEventDestroy(e);
  if (h->host_scal && !h->noalloc) (void)hipHostFree(h->host_scal);
  delete h;
  return IGAMG_OK;
}

int igamg_tuning(igamg_handle h, int level, int fp32, int* variant) {
  API_BEGIN
  if (!h || !variant) return set_err(IGAMG_EINVAL, "null argument");
  if (!h->on_device) return set_err(IGAMG_EINVAL, "handle has no device data");
  level = check_level(h, level);
  if (level < 1) return set_err(IGAMG_EINVAL, "level 0 has no smoother");
  if (fp32 && !h->mixed) return set_err(IGAMG_EINVAL, "not a mixed-precision handle");
  *variant = h->dl[level].fdv[fp32 ? 1 : 0];
  return IGAMG_OK;
  API_END
}

int igamg_band_form(igamg_handle h, int level, int* form) {
  API_BEGIN
  if (!h || !form) return set_err(IGAMG_EINVAL, "null argument");
  if (!h->on_device) return set_err(IGAMG_EINVAL, "handle has no device data");
  level = check_level(h, level);
  if (level < 1) return set_err(IGAMG_EINVAL, "no banded matrix on level 0");
  *form = h->dl[level].sym_ws > 0 ? IGAMG_BAND_SCATTER : IGAMG_BAND_GATHER;
  return IGAMG_OK;
  API_END
}

int igamg_num_dofs(igamg_handle h, int level, int64_t* n_free, int64_t* n_local) {
  API_BEGIN
  if (!h) return set_err(IGAMG_EINVAL, "null handle");
  level = check_level(h, level);
  const LevelH& L = h->H.lv[level];
  if (n_free) *n_free = L.N;
  if (n_local) {
    int64_t s = 0;
    for (int64_t r : L.rows) s += r;
    *n_local = s;
  }
  return IGAMG_OK;
  API_END
}

int igamg_dof_map(igamg_handle h, int level, int64_t* copy_ptr, int64_t* copy_idx, int64_t* n_free,
                  int64_t* n_copies) {
  API_BEGIN
  if (!h) return set_err(IGAMG_EINVAL, "null handle");
  level = check_level(h, level);
  const LevelH& L = h->H.lv[level];
  if (n_free) *n_free = L.N;
  if (n_copies) *n_copies = (int64_t)L.gidx.size();
  if (copy_ptr) std::memcpy(copy_ptr, L.gptr.data(), L.gptr.size() * sizeof(int64_t));
  if (copy_idx) std::memcpy(copy_idx, L.gidx.data(), L.gidx.size() * sizeof(int64_t));
  return IGAMG_OK;
  API_END
}

int igamg_load_vector(igamg_handle h, double amp, double freq, double* f_host) {
  API_BEGIN
  if (!h || !f_host) return set_err(IGAMG_EINVAL, "null argument");
  std::vector<double> f = load_vector(h->H, amp, freq);
  std::memcpy(f_host, f.data(), f.size() * sizeof(double));
  return IGAMG_OK;
  API_END
}

int igamg_vcycle(igamg_handle h, const double* r, double* z, void* stream) {
  API_BEGIN
  need_device(h);
  if (!r || !z || r == z) return set_err(IGAMG_EINVAL, "bad vector arguments");
  hipStream_t st = static_cast<hipStream_t>(stream);
  DevLevel& D = h->dl[h->L];
  launch_scatter(r, D.d64.f, D.gptr, D.gidx, D.N, true, st);
  cycle<double>(*h, h->L, true, st);
  launch_gather(D.d64.u, z, D.gptr, D.gidx, D.N, false, st);
  HIP_OK(hipGetLastError());
  return IGAMG_OK;
  API_END
}

int igamg_operator(igamg_handle h, int op, int level, const double* x, double* y, void* stream) {
  API_BEGIN
  need_device(h);
  if (!x || !y || x == y) return set_err(IGAMG_EINVAL, "bad vector arguments");
  hipStream_t st = static_cast<hipStream_t>(stream);
  level = check_level(h, level);
  DevLevel& D = h->dl[level];
  LevelData<double>& X = D.d64;
  switch (op) {
    case IGAMG_OP_APPLY: {
      if (level < 1) return set_err(IGAMG_EINVAL, "no banded matrix on level 0 (use IGAMG_OP_COARSE)");
      launch_scatter(x, X.u, D.gptr, D.gidx, D.N, false, st);
      band_op<double>(*h, level, X.u, nullptr, X.w, false, st);
      launch_gather(X.w, y, D.gptr, D.gidx, D.N, true, st);
      break;
    }
    case IGAMG_OP_SMOOTHER: {
      if (level < 1) return set_err(IGAMG_EINVAL, "smoother needs level >= 1");
      launch_scatter(x, X.f, D.gptr, D.gidx, D.N, true, st);
      smoother_apply<double>(*h, level, X.f, X.u, false, 1.0, st);
      launch_gather(X.u, y, D.gptr, D.gidx, D.N, false, st);
      break;
    }
    case IGAMG_OP_PROLONG: {
      if (level < 1) return set_err(IGAMG_EINVAL, "prolongation needs level >= 1");
      DevLevel& Dc = h->dl[level - 1];
      launch_scatter(x, Dc.d64.u, Dc.gptr, Dc.gidx, Dc.N, false, st);
      launch_fill<double>(X.w, D.NL, 0.0, st);
      prolong_add<double>(*h, level, Dc.d64.u, X.w, st);
      launch_gather(X.w, y, D.gptr, D.gidx, D.N, false, st);
      break;
    }
    case IGAMG_OP_RESTRICT: {
      if (level < 1) return set_err(IGAMG_EINVAL, "restriction needs level >= 1");
      DevLevel& Dc = h->dl[level - 1];
      launch_scatter(x, X.w, D.gptr, D.gidx, D.N, true, st);
      restrict_to<double>(*h, level, X.w, Dc.d64.f, st);
      launch_gather(Dc.d64.f, y, Dc.gptr, Dc.gidx, Dc.N, true, st);
      break;
    }
    case IGAMG_OP_COARSE: {
      if (level != 0) return set_err(IGAMG_EINVAL, "coarse solve lives on level 0");
      launch_scatter(x, X.f, D.gptr, D.gidx, D.N, true, st);
      coarse_solve<double>(*h, X.f, X.u, st);
      launch_gather(X.u, y, D.gptr, D.gidx, D.N, false, st);
      break;
    }
    case IGAMG_OP_APPLY_FP32: {
      if (!h->mixed) return set_err(IGAMG_EINVAL, "the FP32 apply needs precision IGAMG_MIXED");
      if (level < 1) return set_err(IGAMG_EINVAL, "no banded matrix on level 0 (use IGAMG_OP_COARSE)");
      launch_scatter(x, X.u, D.gptr, D.gidx, D.N, false, st);
      launch_to_f32(D.d32.u, X.u, D.NL, st);
      band_op<float>(*h, level, D.d32.u, nullptr, D.d32.w, false, st);
      launch_to_f64(X.w, D.d32.w, D.NL, st);
      launch_gather(X.w, y, D.gptr, D.gidx, D.N, true, st);
      break;
    }
    case IGAMG_OP_CYCLE_FP32: {
      if (!h->mixed) return set_err(IGAMG_EINVAL, "the FP32 cycle needs precision IGAMG_MIXED");
      if (level != h->L) return set_err(IGAMG_EINVAL, "the FP32 cycle runs on the finest level");
      launch_scatter(x, X.f, D.gptr, D.gidx, D.N, true, st);
      launch_to_f32(D.d32.f, X.f, D.NL, st);
      cycle<float>(*h, level, true, st);
      launch_to_f64(X.u, D.d32.u, D.NL, st);
      launch_gather(X.u, y, D.gptr, D.gidx, D.N, false, st);
      break;
    }
    default:
      return set_err(IGAMG_EINVAL, "unknown operator");
  }
  HIP_OK(hipGetLastError());
  return IGAMG_OK;
  API_END
}

int igamg_export(igamg_handle h, int what, int level, double* out, int64_t* rows, int64_t* cols) {
  API_BEGIN
  if (!h) return set_err(IGAMG_EINVAL, "null handle");
  level = check_level(h, level);
  const Hierarchy& H = h->H;
  const LevelH& L = H.lv[level];
  const int d = H.prob.d, p = H.prob.p;
  if (what == IGAMG_EXPORT_MATRIX) {
    if (L.band.empty()) return set_err(IGAMG_EINVAL, "matrix not kept on the host (set up without a workspace)");
    if (rows) *rows = L.N;
    if (cols) *cols = L.N;
    if (!out) return IGAMG_OK;
    std::memset(out, 0, sizeof(double) * (size_t)L.N * L.N);
    const int nb0 = 2 * p + 1, p2 = (d == 3) ? p : 0, nb2 = 2 * p2 + 1;
    for (int k = 0; k < H.prob.K; ++k) {
      const auto& n = L.n[k];
      for (int64_t r = 0; r < L.rows[k]; ++r) {
        const int64_t x = L.off[k] + r, gi = L.gid[x];
        if (gi < 0) continue;
        const int i0 = (int)(r % n[0]), i1 = (int)((r / n[0]) % n[1]), i2 = (int)(r / ((int64_t)n[0] * n[1]));
        for (int o2 = 0; o2 < nb2; ++o2)
          for (int o1 = 0; o1 < nb0; ++o1)
            for (int o0 = 0; o0 < nb0; ++o0) {
              const int j0 = i0 + o0 - p, j1 = i1 + o1 - p, j2 = i2 + o2 - p2;
              if (j0 < 0 || j0 >= n[0] || j1 < 0 || j1 >= n[1] || j2 < 0 || j2 >= n[2]) continue;
              const int64_t gj = L.gid[L.off[k] + j0 + (int64_t)n[0] * (j1 + (int64_t)n[1] * j2)];
              if (gj < 0) continue;
              const int64_t o = o0 + (int64_t)nb0 * (o1 + (int64_t)nb0 * o2);
              out[gi * L.N + gj] += L.band[o * L.NL + x];
            }
      }
    }
    return IGAMG_OK;
  }
  if (what == IGAMG_EXPORT_PROLONG) {
    if (level < 1) return set_err(IGAMG_EINVAL, "prolongation needs level >= 1");
    const LevelH& Cl = H.lv[level - 1];
    if (rows) *rows = L.N;
    if (cols) *cols = Cl.N;
    if (!out) return IGAMG_OK;
    std::memset(out, 0, sizeof(double) * (size_t)L.N * Cl.N);
    std::vector<char> done(L.N, 0);
    for (int k = 0; k < H.prob.K; ++k) {
      const PatchDev& P = L.pd[k];
      for (int64_t r = 0; r < P.rows; ++r) {
        const int64_t gi = L.gid[P.off + r];
        if (gi < 0 || done[gi]) continue;
        done[gi] = 1;
        const int i[3] = {(int)(r % P.n[0]), (int)((r / P.n[0]) % P.n[1]), (int)(r / ((int64_t)P.n[0] * P.n[1]))};
        int s[3];
        const double* w[3];
        for (int c = 0; c < 3; ++c) {
          s[c] = (int)L.tr_idx[P.Pst[c] + i[c]];
          w[c] = &L.tr_val[P.Pval[c] + (int64_t)i[c] * L.WP];
        }
        const int W2 = (d == 3) ? L.WP : 1;
        for (int a2 = 0; a2 < W2; ++a2)
          for (int a1 = 0; a1 < L.WP; ++a1)
            for (int a0 = 0; a0 < L.WP; ++a0) {
              const double v = w[0][a0] * w[1][a1] * w[2][a2];
              if (v == 0.0) continue;
              const int j0 = s[0] + a0, j1 = s[1] + a1, j2 = s[2] + a2;
              const int64_t gj = Cl.gid[P.offc + j0 + (int64_t)P.nc[0] * (j1 + (int64_t)P.nc[1] * j2)];
              if (gj >= 0) out[gi * Cl.N + gj] += v;
            }
      }
    }
    return IGAMG_OK;
  }
  return set_err(IGAMG_EINVAL, "unknown export");
  API_END
}

int igamg_solve(igamg_handle h, const double* rhs, double* u, double tol, igamg_solve_info* info, void* stream) {
  API_BEGIN
  need_device(h);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!h->solo) h->solo = new igamg_batch_ctx();
  igamg_batch_ctx& B = *h->solo;
  B.reqs.clear();
  const int slot = batch_add(B, h, rhs, u, tol, st);
  while (batch_step(B, st) > 0) {
  }
  Req& q = B.reqs[slot];
  fill_info(q, info);
  const int code = q.code;
  q.state = RQ_FREE;
  if (code == IGAMG_ENOCONV) return set_err(code, "iteration cap reached above the tolerance");
  if (code == IGAMG_ENAN) return set_err(code, "non-finite residual");
  return code;
  API_END
}

int igamg_batch_create(igamg_batch* out) {
  API_BEGIN
  if (!out) return set_err(IGAMG_EINVAL, "out is NULL");
  *out = new igamg_batch_ctx();
  return IGAMG_OK;
  API_END
}

int igamg_batch_destroy(igamg_batch b) {
  delete b;
  return IGAMG_OK;
}

int igamg_batch_add(igamg_batch b, igamg_handle h, const double* rhs, double* u, double tol, void* stream,
                    int* slot) {
  API_BEGIN
  if (!b || !slot) return set_err(IGAMG_EINVAL, "null argument");
  *slot = batch_add(*b, h, rhs, u, tol, static_cast<hipStream_t>(stream));
  return IGAMG_OK;
  API_END
}

int igamg_batch_step(igamg_batch b, void* stream, int* n_active) {
  API_BEGIN
  if (!b) return set_err(IGAMG_EINVAL, "null batch");
  const int a = batch_step(*b, static_cast<hipStream_t>(stream));
  if (n_active) *n_active = a;
  return IGAMG_OK;
  API_END
}

int igamg_batch_poll(igamg_batch b, int slot, int* done, igamg_solve_info* info, int* code) {
  API_BEGIN
  if (!b || slot < 0 || slot >= (int)b->reqs.size() || b->reqs[slot].state == RQ_FREE)
    return set_err(IGAMG_EINVAL, "bad batch slot");
  const Req& q = b->reqs[slot];
  if (done) *done = (q.state == RQ_DONE);
  fill_info(q, info);
  if (code) *code = (q.state == RQ_DONE) ? q.code : IGAMG_OK;
  return IGAMG_OK;
  API_END
}

int igamg_batch_remove(igamg_batch b, int slot) {
  API_BEGIN
  if (!b || slot < 0 || slot >= (int)b->reqs.size()) return set_err(IGAMG_EINVAL, "bad batch slot");
  if (b->reqs[slot].state != RQ_DONE && b->reqs[slot].state != RQ_FREE) HIP_OK(hipStreamSynchronize(b->ds));
  b->reqs[slot] = Req{};
  return IGAMG_OK;
  API_END
}

int igamg_solve_batch(igamg_handle const* hs, const double* const* rhs, double* const* u, int n, double tol,
                      igamg_solve_info* infos, int* codes, void* stream) {
  API_BEGIN
  if (n < 0 || (n > 0 && (!hs || !rhs || !u))) return set_err(IGAMG_EINVAL, "bad batch arguments");
  hipStream_t st = static_cast<hipStream_t>(stream);
  igamg_batch_ctx B;
  std::vector<int> slots;
  for (int i = 0; i < n; ++i) slots.push_back(batch_add(B, hs[i], rhs[i], u[i], tol, st));
  while (batch_step(B, st) > 0) {
  }
  int worst = IGAMG_OK;
  for (int i = 0; i < n; ++i) {
    const Req& q = B.reqs[slots[i]];
    if (infos) fill_info(q, &infos[i]);
    if (codes) codes[i] = q.code;
    if (q.code != IGAMG_OK) worst = q.code;
  }
  if (worst != IGAMG_OK) return set_err(worst, "at least one request did not converge");
  return IGAMG_OK;
  API_END
}

}  // extern "C"
