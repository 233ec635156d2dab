// Host setup of the multigrid hierarchy (the four setup phases of Sec. 5 plus
// the patch-wise assembly of Sec. 4).  Produces flat arrays ready to upload.
#pragma once

#include <array>
#include <memory>
#include <utility>
#include <cstdint>
#include <string>
#include <vector>

#include "layout.hpp"
#include "assemble_layout.hpp"

namespace igamg {

struct ProblemH {
  int d = 2, p = 2, K = 1, levels = 2;
  std::vector<int> nel0;                  // K*d
  std::vector<std::vector<double>> brk0;  // K*d coarsest breakpoints; empty = uniform
  std::vector<int> gdeg;                  // K*d
  std::vector<std::vector<double>> ctrl;  // per patch, prod(g+1)*d
  std::vector<std::array<int, 5>> iface;
  std::vector<int> bc;                    // K*2d
};

// Coarse problems above this size are factored on the device when one is
// available (O(N0^3) on the host takes minutes beyond a few thousand).
constexpr int64_t COARSE_HOST_MAX = 3000;

struct Options {
  double tau = 0.25, sigma_scale = 5.0;
  int nu = 1, mu = 1, precision = 0, maxit = 500, geometry_scaling = 0;
  int inner_maxit = 100;
  double inner_tol = 1e-4;
  int graphs = 1;
  int fd_mfma = 0;
  int coarse_factor = 0;   // 0 auto, 1 host, 2 device
  int autotune = 1;
  int assembly = 0;        // levels >= 1: 0 on the device when there is one, 1 on the host
  int s1_sigma = 1;        // 1: K + sigma M on the complement S1 of the interior smoother, 0: K
  int iface_multiplicity = 0;  // 1: interface piece operators times their number of adjacent patches
  int physical_h = 0;      // 1: h_c = (mean length of the c-th Jacobian column) / nel_c
  int iface_direct = 0;    // 1: edges and vertices solved with the exact restriction of A_l
  int persistent = 0;      // 1: the coarse levels of each cycle as one persistent launch
  int band_form = 0;       // 0: scatter form of the symmetric band on large 3D levels, 1: gather form
                           // everywhere, 2: scatter form on every 3D level that fits
};

// Error with an igamg return code.
struct SetupError {
  int code;
  std::string msg;
};

// One grid level.
struct LevelH {
  int l = 0;
  std::vector<std::array<int, 3>> n, nel;   // per patch (unused dims: n = 1, nel = 1)
  std::vector<std::vector<double>> brk;     // K*3 breakpoints per patch and direction (unused: {0, 1})
  std::vector<int64_t> off, rows;
  int64_t NL = 0;                            // padded local length
  std::vector<int64_t> gid;                  // NL entries: free id or -1
  int64_t N = 0;
  std::vector<int64_t> gptr, gidx;           // copies of each free dof (local positions)
  std::vector<int> bpatch;                   // patch of each 256-row block (-1: none)
  std::vector<uint8_t> isfree;               // NL
  // banded patch matrices, coefficient-major: band[o * NL + row]
  int nb = 0;                                // (2p+1)^d
  std::vector<double> band;
  // interface vector (faces, edges, vertices): copies CSR
  int64_t nif = 0;
  std::vector<int64_t> if_ptr, if_idx;
  // smoother
  std::vector<FDItem> fd;                    // interiors first, then faces
  int nfd_interior = 0;
  std::vector<double> fdmat;                 // U matrices and mu vectors
  int64_t fdscr = 0;                         // scratch entries per buffer
  int fd_maxm = 1;
  std::vector<DensePiece> dense;
  std::vector<double> densemat;
  // exact edge and vertex pieces (options.iface_direct): direct[q] = 1 for
  // dense piece q whose m*m entries (piece by piece, row-major) gather the
  // half-band entries (dg_row, dg_plane)[dg_ptr[e] .. dg_ptr[e+1])
  std::vector<char> direct;
  std::vector<int64_t> dg_ptr, dg_row;
  std::vector<int> dg_plane;
  // transfers from level l-1 (empty for l = 0)
  int WP = 0, WR = 0;
  std::vector<int64_t> tr_idx;
  std::vector<double> tr_val;
  std::vector<PatchDev> pd;
  std::vector<double> omega;                 // per patch
  std::vector<std::array<double, 3>> length; // per patch: mean |dG/dxi_c| over (0,1)^d
};

// A vector of doubles whose elements start uninitialised: the dense coarse
// matrix (N0^2 doubles, up to 75 GB) is zeroed and filled by row blocks in
// parallel instead of by a serial value-initialisation.
template <class T>
struct UninitAlloc : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = UninitAlloc<U>;
  };
  UninitAlloc() = default;
  template <class U>
  UninitAlloc(const UninitAlloc<U>&) noexcept {}
  template <class U>
  void construct(U* p) noexcept {
    ::new (static_cast<void*>(p)) U;
  }
  template <class U, class... A>
  void construct(U* p, A&&... a) {
    ::new (static_cast<void*>(p)) U(std::forward<A>(a)...);
  }
};
using DenseBuf = std::vector<double, UninitAlloc<double>>;

struct Hierarchy {
  ProblemH prob;
  Options opt;
  std::vector<LevelH> lv;
  // coarse solver: A_0^{-1} = L^{-T} L^{-1} with A_0 = L L^T (dense, row-major, N0 x N0),
  // factored on the host; or the dense A_0 itself, to be factored on the device
  std::vector<double> Ainv;
  DenseBuf A0;
};



// Validate and copy the C problem description.  Throws SetupError.
ProblemH read_problem(const void* cprob);
// Topology only (dof maps, pieces sizes): enough to size the workspace.
void build_topology(Hierarchy& H, bool with_numerics);
// Everything (assembly, smoothers, transfers, coarse factor).  Levels >= 1
// are left unassembled when they will be assembled on the device.
void build_all(Hierarchy& H, bool device);
// Inverts the exact edge and vertex pieces of a level from their gathered
// entries (vals[e] for the entries listed by dg_ptr) into densemat.
void finish_direct_pieces(LevelH& L, const std::vector<double>& vals);
// Whether levels >= 1 are assembled on the device.
inline bool assemble_on_device(const Options& o, bool device) { return device && o.assembly == 0; }
// Quadrature, basis and geometry tables of every patch of level L for device
// assembly: one descriptor per patch, offsets into `pool`.
void make_assembly_tables(const ProblemH& P, const LevelH& L, std::vector<AsmPatch>& pt, std::vector<double>& pool);
// One line on stderr per setup phase when IGAMG_VERBOSE is set.
void setup_progress(const char* what, double value);
// Whether the coarse problem is factored on the device (a device is
// available and the options or the size ask for it).
inline bool coarse_on_device(const Options& o, int64_t N0, bool device) {
  return device && (o.coarse_factor == 2 || (o.coarse_factor == 0 && N0 > COARSE_HOST_MAX));
}
// Load vector of the finest level for src = amp * prod sin(freq*pi*x_c).
std::vector<double> load_vector(const Hierarchy& H, double amp, double freq);

}  // namespace igamg
