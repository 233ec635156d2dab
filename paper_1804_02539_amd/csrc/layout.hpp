// Device-side descriptors shared by the host setup and the HIP kernels.
//
// Vectors of a level live in the patch-local layout of Sec. 4: every patch
// stores all of its local functions (interface layers duplicated, Dirichlet
// functions kept as zeros), x fastest, patch blocks aligned to ROW_ALIGN
// entries so that every 256-row block of a level belongs to one patch.
#pragma once

#include <cstddef>
#include <cstdint>

namespace igamg {

constexpr int ROW_ALIGN = 256;   // patch block alignment (entries) and apply block size
constexpr int MAX_P = 8;         // highest spline degree with a compiled apply kernel
constexpr int MAX_FD = 256;      // largest 1D interior size handled by the FD kernels (one thread per row)
constexpr int FD_LDS_M = 84;     // largest 1D interior size whose tensors the FD kernels stage in LDS
                                 // (L^2 + 1024 doubles); larger ones read their operands from memory

// Symmetric half-band storage of the banded patch matrices.  An offset of the
// (2P+1)^D stencil is written in index form (o0, o1, o2), o_c in [0, 2P]
// (actual offset o_c - P); its stencil line is L = o1 + NB*o2 (2D: L = o1),
// NB = 2P+1, and the centre line LC = (NLINE-1)/2 holds the diagonal.  Only
// the offsets whose linear displacement in the patch is >= 0 are stored:
//   centre line, o0 = P..2P:    plane o0 - P      (plane 0: the diagonal)
//   lines L > LC (all o0):      plane P + 1 + (L - LC - 1)*NB + o0
// The other half follows from symmetry, A[i][i+d] = A[i+d][i]: row i reads
// it from row i+d at the plane of the negated offset.  Per 256-row tile the
// band_half_planes(D, P) planes are contiguous:
//   band[(row/256)*nbh*256 + plane*256 + row%256].
constexpr int band_lines(int d, int p) { return d == 2 ? 2 * p + 1 : (2 * p + 1) * (2 * p + 1); }
constexpr int band_half_planes(int d, int p) { return p + 1 + (band_lines(d, p) - 1) / 2 * (2 * p + 1); }
// plane of index-form offset (o0, line L), or -1 for an offset of the lower half
constexpr int band_half_plane(int d, int p, int o0, int L) {
  return L == (band_lines(d, p) - 1) / 2 ? (o0 >= p ? o0 - p : -1)
         : L > (band_lines(d, p) - 1) / 2 ? p + 1 + (L - (band_lines(d, p) - 1) / 2 - 1) * (2 * p + 1) + o0
                                          : -1;
}

// Scatter form of the symmetric half-band apply: the stored offsets of a
// 256-row tile reach the rows of the tile shifted by a layer's stride (3D:
// layer a2 = 0..p of the stencil, stride n0 n1; 2D: line a1 = 0..p, stride
// n0) plus at most band_sym_reach either way (3D: p + p n0; 2D: p); the
// tile's windows (layer 0: 256 + reach rows, layers 1..p: 256 + 2 reach)
// hold band_sym_window values in all; a workgroup keeps them in LDS in FP64,
// beside the u values of the same rows.
constexpr int64_t band_sym_reach(int d, int p, int64_t n0) { return d == 3 ? p + p * n0 : p; }
constexpr int64_t band_sym_window(int d, int p, int64_t n0) {
  return (int64_t)(p + 1) * ROW_ALIGN + (2 * p + 1) * band_sym_reach(d, p, n0);
}
constexpr size_t BAND_SYM_MAX_LDS = 96 * 1024;   // windows and u of one tile in LDS, at most

// One patch on one level l (coarse data refers to level l-1).
struct PatchDev {
  int n[3];          // local functions per direction at level l (1 for unused directions)
  int nc[3];         // the same at level l-1
  int64_t off;       // start of the patch block in level-l vectors
  int64_t offc;      // start of the patch block in level-(l-1) vectors
  int64_t rows;      // n0*n1*n2
  int64_t rowsc;     // nc0*nc1*nc2
  int64_t Pst[3];    // prolongation table (per fine row: first coarse index) in `tr_idx`
  int64_t Pval[3];   // prolongation weights (per fine row: WP values) in `tr_val`
  int64_t Rst[3];    // restriction table (per coarse row: first fine index)
  int64_t Rval[3];   // restriction weights (per coarse row: WR values)
};

// One tensor item of the fast-diagonalisation smoother: a patch interior
// (src = patch-local vectors) or a face piece (src = interface vector).
struct FDItem {
  int m[3];          // interior sizes per direction (1 for unused)
  int src_if;        // 0: patch-local vectors, 1: interface vector
  int64_t base;      // position of tensor element (0,0,0) in the source/destination
  int64_t stride[3]; // strides of the source/destination view
  int64_t scr;       // offset of this item's compact scratch tensor
  int64_t U[3];      // offsets of U_c (m_c x m_c, row-major), followed by U_c^T, in the FD pool
  int64_t mu[3];     // offsets of mu_c (m_c values) in the FD matrix pool
  double pref;       // D = pref * (mu0 + mu1 + mu2 + extra)
  double extra;
};

// One phase of the persistent coarse cycle (k_cycle_tail): `n` work items,
// item t is block (t % gx, t / gx) of the launch the phase replaces; ticket
// first + j covers items j*chunk .. min(n, (j+1)*chunk) - 1, ntk tickets in
// all.  Pointers and scalars by kind:
//   BAND      a: band, u, f, r, bpatch, pd;                        resid
//   FD_FWD    a: items, dense, densemat, mat, src, u, if_ptr, if_idx, scr;  nitems, tau, add, rb
//   FD_MID    a: items, mat, scr
//   FD_INV    a: items, mat, u, if_ptr, if_idx, scr;               tau, add, rb
//   RESTRICT  a: rf, rc, pd, bpatch_c, tidx, tval, isfree_c;       w
//   PROLONG   a: uc, uf, pd, bpatch_f, tidx, tval, isfree_f;       w
//   GATHER    a: loc, glob (double), ptr, idx;                     len
//   CTILES    a: Ainv (packed tiles), b, part;                     len
//   CREDUCE   a: part, u0, ptr, idx;                               len
enum PhaseKind : int {
  PH_BAND = 0, PH_FD_FWD, PH_FD_MID, PH_FD_INV, PH_RESTRICT, PH_PROLONG, PH_GATHER, PH_CTILES, PH_CREDUCE
};
struct Phase {
  int kind;
  int gx;
  int64_t n;
  int64_t first;
  int64_t ntk;
  int64_t chunk;
  int resid, add, w, nitems, rb, pad;
  int64_t len;
  double tau;
  const void* a[10];
};

// The dense coarse inverse A_0^{-1} (and the Cholesky factor it is formed
// from) in packed lower tiles: n is padded to T = ceil(n / COARSE_TILE) tiles
// per side, tile (I, J), J <= I, holds rows COARSE_TILE*I .. and columns
// COARSE_TILE*J .. row-major at entry coarse_tile_at(I, J).  Diagonal tiles
// hold both triangles; padding rows and columns hold the identity.
constexpr int COARSE_TILE = 64;
constexpr int64_t coarse_tiles(int64_t n) { return (n + COARSE_TILE - 1) / COARSE_TILE; }
constexpr int64_t coarse_tile_at(int64_t I, int64_t J) {
  return (I * (I + 1) / 2 + J) * (int64_t)COARSE_TILE * COARSE_TILE;
}
constexpr int64_t coarse_packed_entries(int64_t n) { return coarse_tile_at(coarse_tiles(n), 0); }

// A piece applied by a dense inverse (edges, vertices).
struct DensePiece {
  int64_t seg;       // first entry in the interface vector
  int m;             // size
  int pad;
  int64_t Linv;      // offset of the m x m inverse (row-major) in the dense pool
};

}  // namespace igamg
