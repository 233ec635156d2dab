// HIP kernels of the multigrid cycle for gfx950 (64-wide wavefronts).
//
// All level vectors are in the patch-local layout (see layout.hpp).  The
// kernels are written for one level of one problem; the cycle (Algorithm 1)
// and the PCG loop (Sec. 4) are sequenced on one stream by igamg.hip.
// Every kernel is a template over its storage type: double for the FP64
// solver and the outer refinement residual, float for the inner solve of the
// mixed-precision solver (reductions always accumulate in double).
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>

#include "kernels.hpp"
#include "layout.hpp"

namespace igamg {

#define DYN_LDS(T, name)                                      \
  extern __shared__ __align__(16) unsigned char lds_raw_[];   \
  T* name = reinterpret_cast<T*>(lds_raw_)

// ---------------------------------------------------------------------------
// banded stiffness apply: r = f - A u  (RESID) or r = A u   (Sec. 4: A_{l,k}
// applied patch by patch to accumulated u gives a distributed result).
// FP64 (k_band_half): the band holds the upper half of each symmetric patch
// matrix (layout.hpp):
// a row reads its own stored planes, and each coupling of the lower half from
// the row it couples to (A[i][i+d] = A[i+d][i], d < 0), at the plane of the
// negated offset.  Each coefficient is fetched from HBM once and read twice;
// the second read finds it in the caches (the mirrored rows lie at most
// P (n0 n1 + n0 + 1) rows back).
// A workgroup takes a strip of 64 rows (one row per lane); its 4 waves split
// the stencil lines (o1, o2) between them (the single stencil entries, in
// 2D) and add their partial sums in LDS, so a launch has 4 x (rows / 256) x 4
// waves to hide HBM latency with.  Every band read of a wave, own or
// mirrored, is a run of 64 consecutive rows of one plane: one coalesced
// segment, two where it crosses a 256-row tile.
// ---------------------------------------------------------------------------
constexpr int BAND_STRIP = 64;

// Band entry `plane` of row gg (global) in the tiled half-band.
template <int NBH, typename TB>
__device__ __forceinline__ TB band_at(const TB* __restrict__ band, int64_t gg, int plane) {
  return band[((gg >> 8) * NBH + plane) * ROW_ALIGN + (gg & (ROW_ALIGN - 1))];
}

// The lower-half couplings of one stencil line L <= LC (index form) for row
// rl: the rows rl + d of the patch (a row outside the patch couples nothing),
// read at the planes of the negated offsets.
template <int D, int P, typename TB, typename TV>
__device__ __forceinline__ TV band_mirror_line(const TB* __restrict__ band, const TV* __restrict__ ub, int64_t off,
                                               int64_t rows, int64_t rl, int64_t dl, int L, int o0_end) {
  constexpr int NB = 2 * P + 1, NLINE = band_lines(D, P), LC = (NLINE - 1) / 2;
  constexpr int NBH = band_half_planes(D, P);
  // plane of the negated offset (2P - o0, line 2 LC - L): pbase - o0
  const int pbase = (L < LC) ? P + 1 + (LC - L - 1) * NB + 2 * P : P;
  const int64_t r0 = rl + dl - P;
  TV s = 0;
#pragma unroll
  for (int o0 = 0; o0 < NB; ++o0) {
    if (o0 < o0_end) {
      const int64_t rr = r0 + o0;
      const bool in = rr >= 0 && rr < rows;
      const int64_t rc = in ? rr : rl;
      const TV v = (TV)band_at<NBH>(band, off + rc, pbase - o0) * ub[rc];
      s += in ? v : (TV)0;
    }
  }
  return s;
}

// 2D: the NB^2 stencil entries are dealt to the 4 waves one by one (entry t
// to wave t mod 4); the wave index is a template argument so every entry's
// offsets are compile-time constants.
template <int P, int W, typename TB, typename TV>
__device__ __forceinline__ TV band_entries_2d(const TB* __restrict__ band, const TV* __restrict__ ub, int64_t off,
                                              int64_t rows, int64_t g, int64_t rl, const int* c0, const int* c1,
                                              int n0) {
  constexpr int NB = 2 * P + 1, LC = P, NBH = band_half_planes(2, P);
  TV s = 0;
#pragma unroll
  for (int t = W; t < NB * NB; t += 4) {
    const int o0 = t % NB, L = t / NB;
    const int pl = band_half_plane(2, P, o0, L);
    if (pl >= 0) {
      s += (TV)band_at<NBH>(band, g, pl) * ub[c1[L] + c0[o0]];
    } else {
      // lower half: row rl + d, plane of the negated offset
      const int pn = band_half_plane(2, P, 2 * P - o0, 2 * LC - L);
      const int64_t rr = rl + (int64_t)(L - P) * n0 + (o0 - P);
      const bool in = rr >= 0 && rr < rows;
      const int64_t rc = in ? rr : rl;
      const TV v = (TV)band_at<NBH>(band, off + rc, pn) * ub[rc];
      s += in ? v : (TV)0;
    }
  }
  return s;
}

// strip bx of 64 rows (the body of one workgroup of k_band_half)
template <int D, int P, bool RESID, typename TB, typename TV>
__device__ __forceinline__ void band_half_strip(int64_t bx, const TB* __restrict__ band, const TV* __restrict__ u,
                                                const TV* __restrict__ f, TV* __restrict__ r,
                                                const int* __restrict__ bpatch, const PatchDev* __restrict__ pd) {
  constexpr int NB = 2 * P + 1;
  constexpr int NLINE = band_lines(D, P);                 // stencil lines (o1, o2)
  constexpr int LC = (NLINE - 1) / 2;
  constexpr int NBH = band_half_planes(D, P);
  __shared__ TV part[3][BAND_STRIP];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t g = bx * BAND_STRIP + lane;
  const int64_t tile = g / ROW_ALIGN;                    // the same for the whole workgroup
  const int k = bpatch[tile];
  if (k < 0) return;                                     // uniform: a padding tile
  const int64_t off = pd[k].off;
  const int64_t rows = pd[k].rows;
  const int64_t rl0 = g - off;
  const bool valid = rl0 < rows;
  const int64_t rl = valid ? rl0 : rows - 1;             // padding lanes compute a real row, never store
  const int64_t gr = off + rl;
  const int n0 = pd[k].n[0], n1 = pd[k].n[1], n2 = pd[k].n[2];
  const int i0 = (int)(rl % n0);
  const int64_t t = rl / n0;
  const int i1 = (int)(t % n1);
  const int i2 = (int)(t / n1);
  int c0[NB];
#pragma unroll
  for (int o = 0; o < NB; ++o) c0[o] = min(max(i0 + o - P, 0), n0 - 1);
  const TV* ub = u + off;
  const int64_t pl = (int64_t)n0 * n1;
  TV s = 0;
  if constexpr (D == 2) {
    int c1[NB];
#pragma unroll
    for (int o = 0; o < NB; ++o) c1[o] = min(max(i1 + o - P, 0), n1 - 1) * n0;
    switch (w) {
      case 0: s = band_entries_2d<P, 0, TB, TV>(band, ub, off, rows, gr, rl, c0, c1, n0); break;
      case 1: s = band_entries_2d<P, 1, TB, TV>(band, ub, off, rows, gr, rl, c0, c1, n0); break;
      case 2: s = band_entries_2d<P, 2, TB, TV>(band, ub, off, rows, gr, rl, c0, c1, n0); break;
      default: s = band_entries_2d<P, 3, TB, TV>(band, ub, off, rows, gr, rl, c0, c1, n0); break;
    }
  } else {
    const TB* bt = band + (gr >> 8) * NBH * ROW_ALIGN + (gr & (ROW_ALIGN - 1));
    for (int L = w; L < NLINE; L += 4) {
      const int o1 = L % NB, o2 = L / NB;
      if (L >= LC) {
        // upper half (and the centre line's o0 >= P): this row's own planes;
        // out-of-patch columns hold zeros, so their u index is only clamped
        const int64_t base = (int64_t)min(max(i1 + o1 - P, 0), n1 - 1) * n0 +
                             (int64_t)min(max(i2 + o2 - P, 0), n2 - 1) * pl;
        const TV* ur = ub + base;
        if (L > LC) {
          const TB* bq = bt + (int64_t)(P + 1 + (L - LC - 1) * NB) * ROW_ALIGN;
#pragma unroll
          for (int o0 = 0; o0 < NB; ++o0) s += (TV)bq[o0 * ROW_ALIGN] * ur[c0[o0]];
        } else {
#pragma unroll
          for (int o0 = P; o0 < NB; ++o0) s += (TV)bt[(o0 - P) * ROW_ALIGN] * ur[c0[o0]];
        }
      }
      if (L <= LC) {
        const int64_t dl = (int64_t)(o1 - P) * n0 + (int64_t)(o2 - P) * pl;
        s += band_mirror_line<D, P, TB, TV>(band, ub, off, rows, rl, dl, L, L == LC ? P : NB);
      }
    }
  }
  if (w > 0) part[w - 1][lane] = s;
  __syncthreads();
  if (w == 0 && valid) {
    s += part[0][lane] + part[1][lane] + part[2][lane];
    if constexpr (RESID) r[g] = f[g] - s; else r[g] = s;
  }
}

template <int D, int P, bool RESID, typename TB, typename TV>
__global__ __launch_bounds__(256) void k_band_half(const TB* __restrict__ band, const TV* __restrict__ u,
                                                   const TV* __restrict__ f, TV* __restrict__ r,
                                                   const int* __restrict__ bpatch, const PatchDev* __restrict__ pd) {
  band_half_strip<D, P, RESID, TB, TV>(blockIdx.x, band, u, f, r, bpatch, pd);
}

// The full band (all (2P+1)^D planes per row, the layout of the FP32 copy):
// each row reads its own planes only.  2D FP64 deals single planes to the
// waves (plane o to wave o mod 4), everything else whole stencil lines.
template <int P, int W, typename TB, typename TV>
__device__ __forceinline__ TV band_planes_2d(const TB* __restrict__ bp, const TV* __restrict__ ub, const int* c0,
                                             const int* c1) {
  constexpr int NB = 2 * P + 1;
  TV s = 0;
#pragma unroll
  for (int o = W; o < NB * NB; o += 4) s += (TV)bp[o * ROW_ALIGN] * ub[c1[o / NB] + c0[o % NB]];
  return s;
}

template <int D, int P, bool RESID, typename TB, typename TV>
__device__ __forceinline__ void band_full_strip(int64_t bx, const TB* __restrict__ band, const TV* __restrict__ u,
                                                const TV* __restrict__ f, TV* __restrict__ r,
                                                const int* __restrict__ bpatch, const PatchDev* __restrict__ pd) {
  constexpr int NB = 2 * P + 1;
  constexpr int NLINE = (D == 2) ? NB : NB * NB;        // stencil lines (o1, o2)
  constexpr int NBT = NLINE * NB;
  __shared__ TV part[3][BAND_STRIP];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t g = bx * BAND_STRIP + lane;
  const int64_t tile = g / ROW_ALIGN;                    // the same for the whole workgroup
  const int k = bpatch[tile];
  if (k < 0) return;                                     // uniform: a padding tile
  const int64_t off = pd[k].off;
  const int64_t rows = pd[k].rows;
  const int64_t rl0 = g - off;
  const bool valid = rl0 < rows;
  const int64_t rl = valid ? rl0 : rows - 1;             // padding lanes compute a real row, never store
  const int n0 = pd[k].n[0], n1 = pd[k].n[1], n2 = pd[k].n[2];
  const int i0 = (int)(rl % n0);
  const int64_t t = rl / n0;
  const int i1 = (int)(t % n1);
  const int i2 = (int)(t / n1);
  int c0[NB];
#pragma unroll
  for (int o = 0; o < NB; ++o) c0[o] = min(max(i0 + o - P, 0), n0 - 1);
  const TV* ub = u + off;
  const TB* bp = band + tile * NBT * ROW_ALIGN + (g - tile * ROW_ALIGN);
  const int64_t pl = (int64_t)n0 * n1;
  TV s = 0;
  if constexpr (D == 2 && sizeof(TB) == 8) {
    int c1[NB];
#pragma unroll
    for (int o = 0; o < NB; ++o) c1[o] = min(max(i1 + o - P, 0), n1 - 1) * n0;
    switch (w) {
      case 0: s = band_planes_2d<P, 0, TB, TV>(bp, ub, c0, c1); break;
      case 1: s = band_planes_2d<P, 1, TB, TV>(bp, ub, c0, c1); break;
      case 2: s = band_planes_2d<P, 2, TB, TV>(bp, ub, c0, c1); break;
      default: s = band_planes_2d<P, 3, TB, TV>(bp, ub, c0, c1); break;
    }
  } else {
    for (int L = w; L < NLINE; L += 4) {
      const int o1 = L % NB, o2 = L / NB;
      int64_t base = (int64_t)min(max(i1 + o1 - P, 0), n1 - 1) * n0;
      if constexpr (D == 3) base += (int64_t)min(max(i2 + o2 - P, 0), n2 - 1) * pl;
      const TV* ur = ub + base;
      const TB* bq = bp + (int64_t)L * NB * ROW_ALIGN;
#pragma unroll
      for (int o0 = 0; o0 < NB; ++o0) s += (TV)bq[o0 * ROW_ALIGN] * ur[c0[o0]];
    }
  }
  if (w > 0) part[w - 1][lane] = s;
  __syncthreads();
  if (w == 0 && valid) {
    s += part[0][lane] + part[1][lane] + part[2][lane];
    if constexpr (RESID) r[g] = f[g] - s; else r[g] = s;
  }
}

template <int D, int P, bool RESID, typename TB, typename TV>
__global__ __launch_bounds__(256) void k_band_full(const TB* __restrict__ band, const TV* __restrict__ u,
                                                   const TV* __restrict__ f, TV* __restrict__ r,
                                                   const int* __restrict__ bpatch, const PatchDev* __restrict__ pd) {
  band_full_strip<D, P, RESID, TB, TV>(blockIdx.x, band, u, f, r, bpatch, pd);
}

// ---------------------------------------------------------------------------
// The symmetric half band in scatter form.  Every stored coefficient
// a = A[j][j+d] (d >= 0) is fetched once and used twice: y_j += a u_{j+d}
// (forward) and, d > 0, y_{j+d} += a u_j (its mirror, A[j+d][j] = a).
//
// A workgroup takes one 256-row tile (local rows s .. s+255) with one wave
// per layer of the stored offsets: in 3D the layer a2 = 0..P of
// (a0, a1, a2), LS = n0 n1 rows apart; in 2D the line a1 = 0..P of
// (a0, a1), LS = n0 rows apart.  A wave adds the mirrored terms of its layer
// into a window of LDS over the rows they reach: layer 0 the rows
// s .. s+255+W, layer kk >= 1 the rows s + kk LS - W .. s + 255 + kk LS + W,
// with W = P + P n0 in 3D and P in 2D (band_sym_reach).  Beside the window
// it stages the u of the same rows, so a forward term reads u at the
// position where its mirrored term lands.
//
// Each window has one owner wave, which adds into it with LDS atomics; a
// wave's LDS operations execute in program order, so every position
// receives its terms in a fixed order.  The windows are FP64 for both
// storage types: FP32 products are exact in FP64, and LDS FP32 atomic adds
// measured about 20x slower per instruction than FP64 ones on this pattern
// (consecutive addresses, one instruction after another).
//
// The windows go to global memory (per tile band_sym_window values: layer 0,
// then layers 1..P), the first 256 positions of layer 0 with the tile's
// forward sums added, and k_band_sym_reduce sums, for each row, the
// positions of the tiles whose windows cover it, in a fixed order (layer,
// then tile), into r = f - y (or y).  The windows cost (P+1)*256 + (2P+1)*W
// values per tile, written once and read once, against nbh*256 coefficients.

// element idx of a uniform base, with a 32-bit byte offset (one VGPR per
// address instead of two)
template <typename T>
__device__ __forceinline__ T ld_off32(const T* __restrict__ base, uint32_t idx) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (uint32_t)sizeof(T));
}

// Lines of coefficients in flight per wave of k_band_sym_scatter: per degree
// and type the deepest buffering (of 2..5 lines) that the compiler fits
// without spilling at the occupancy the LDS allows, read off its register
// counts.
template <int D, int P, typename T>
constexpr int band_sym_nbuf() {
  if (D == 2) return 1;   // a 2D layer is a single line
  if (sizeof(T) == 4) return P == 7 ? 2 : (P == 4 || P == 8) ? 4 : 5;
  return (P == 1 || P == 2) ? 5 : P == 3 ? 3 : P == 4 ? 4 : 2;
}

template <int D, int P, typename T>
__global__ __launch_bounds__(64 * (P + 1)) void k_band_sym_scatter(const T* __restrict__ band,
                                                                   const T* __restrict__ u, T* __restrict__ win,
                                                                   int64_t wstride, const int* __restrict__ bpatch,
                                                                   const PatchDev* __restrict__ pd) {
  constexpr int NB = 2 * P + 1, NBH = band_half_planes(D, P);
  constexpr int NBUF = band_sym_nbuf<D, P, T>();
  extern __shared__ __align__(16) unsigned char sym_lds[];
  const int lane = threadIdx.x & 63;
  // the layer is the wave index: uniform across the wave (a scalar)
  const int kk = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t b = blockIdx.x;
  const int k = bpatch[b];
  if (k < 0) return;                                     // uniform: a padding tile
  const int64_t off = pd[k].off, rows = pd[k].rows;
  const int n0 = pd[k].n[0];
  const int64_t LS = D == 3 ? (int64_t)n0 * pd[k].n[1] : n0;   // rows between layers
  const int W = (int)band_sym_reach(D, P, n0);
  const int len = kk ? ROW_ALIGN + 2 * W : ROW_ALIGN + W;
  const int wo = kk ? ROW_ALIGN + W + (kk - 1) * (ROW_ALIGN + 2 * W) : 0;
  // LDS: the windows (FP64), then u at the same positions (storage type):
  // position q of layer kk's window and segment is local row
  // s + kk LS - (kk ? W : 0) + q, so the forward term of an offset reads u
  // where its mirrored term goes.  Rows outside the patch read 0 (their
  // coefficients are 0 too).
  double* lw = reinterpret_cast<double*>(sym_lds) + wo;
  T* lu = reinterpret_cast<T*>(reinterpret_cast<double*>(sym_lds) + wstride) + wo;
  const int64_t s = b * ROW_ALIGN - off;
  const T* ub = u + off;
  const int64_t base = s + kk * LS - (kk ? W : 0);
  for (int i = lane; i < len; i += 64) {
    lw[i] = 0.0;
    const int64_t row = base + i;
    lu[i] = (row >= 0 && row < rows) ? ub[row] : T(0);
  }
  __syncthreads();
  // the tile's planes; loads index them with 32-bit offsets from this base
  const T* bt = band + (b * NBH) * ROW_ALIGN;
  // 3D: the lines (a1) of this wave's layer, a1 = 0..P in layer 0 (the
  // centre line a1 = 0 stores a0 = 0..P only), a1 = -P..P in the others.
  // 2D: the layer is the line a1 = kk (kk = 0: the centre line).
  const int a1_first = (D == 3 && kk) ? -P : 0, nline = D == 2 ? 1 : kk ? NB : P + 1;
  const int plane0 = D == 2 ? P + 1 + (kk - 1) * NB : kk ? P + 1 + P * NB + (kk - 1) * NB * NB : 0;
  T y[4];
#pragma unroll 1
  for (int g = 0; g < 4; ++g) {
    const int64_t j = s + 64 * g + lane;
    const bool valid = j < rows;                         // padding rows add nothing
    const double uj = valid ? (double)ub[j] : 0.0;
    const uint32_t rt = 64 * g + lane;
    const int pos = 64 * g + lane + (kk ? W : 0);        // window position of row j itself
    // the coefficients of line li (a1 = a1_first + li), o0 = a0 + P; the
    // centre line's lower half (o0 < P) is not stored and reads as 0
    auto load_line = [&](int li, T* vb) {
      const int a1 = a1_first + li;
      const bool centre = kk == 0 && a1 == 0;
      const uint32_t bq =
          (uint32_t)(centre ? -P : D == 2 ? plane0 : plane0 + (kk ? li * NB : P + 1 + (a1 - 1) * NB)) * ROW_ALIGN + rt;
#pragma unroll
      for (int o0 = 0; o0 < NB; ++o0) vb[o0] = (centre && o0 < P) ? T(0) : ld_off32(bt, bq + (uint32_t)(o0 * ROW_ALIGN));
    };
    T acc = T(0);
    // forward terms of line li from the staged u, its mirrored terms into
    // the window (offsets d > 0: the centre line's a0 <= 0 has none)
    auto add_line = [&](int li, const T* vb) {
      const int a1 = a1_first + li;
      const bool centre = kk == 0 && a1 == 0;
      const int q0 = pos + (D == 3 ? a1 * n0 : 0) - P;
      T uq[NB];
#pragma unroll
      for (int o0 = 0; o0 < NB; ++o0) uq[o0] = lu[(centre && o0 < P) ? q0 + P : q0 + o0];
#pragma unroll
      for (int o0 = 0; o0 < NB; ++o0) {
        acc += vb[o0] * uq[o0];
        if (!(centre && o0 <= P))
          __hip_atomic_fetch_add(lw + q0 + o0, valid ? (double)vb[o0] * uj : 0.0, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    };
    // Loads are not issued ahead of an earlier (ordered) LDS atomic, so the
    // lines rotate through NBUF register buffers: the loads of line li + NBUF
    // are issued right after the atomics of line li, and NBUF lines are in
    // flight.  The main loop's loads are unconditional; the last lines are
    // peeled.
    T vb[NBUF][NB];
#pragma unroll
    for (int q = 0; q < NBUF; ++q)
      if (q < nline) load_line(q, vb[q]);
    int li = 0;
#pragma unroll 1
    for (; li + 2 * NBUF - 1 < nline; li += NBUF) {
#pragma unroll
      for (int q = 0; q < NBUF; ++q) {
        add_line(li + q, vb[q]);
        load_line(li + q + NBUF, vb[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < 2 * NBUF - 1; ++q) {
      if (li + q < nline) {
        add_line(li + q, vb[q % NBUF]);
        if (li + q + NBUF < nline) load_line(li + q + NBUF, vb[q % NBUF]);
      }
    }
    y[g] = acc;
  }
  __syncthreads();
  // the windows out; layer 0's first 256 positions wait for the forward sums
  T* wg = win + b * wstride + wo;
  for (int i = lane + (kk ? 0 : ROW_ALIGN); i < len; i += 64) wg[i] = (T)lw[i];
  __syncthreads();
  if (kk > 0) {
#pragma unroll
    for (int g = 0; g < 4; ++g) lw[64 * g + lane] = (double)y[g];
  }
  __syncthreads();
  if (kk == 0) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      double fw = (double)y[g];
      for (int q = 1; q <= P; ++q) fw += reinterpret_cast<double*>(sym_lds)[ROW_ALIGN + W + (q - 1) * (ROW_ALIGN + 2 * W) + 64 * g + lane];
      wg[64 * g + lane] = (T)(lw[64 * g + lane] + fw);
    }
  }
}

// One row per thread: the sum of the window positions that cover it (layer
// 0..P, then tile, ascending, in FP64), and r = f - y (RESID) or r = y.
template <int D, int P, bool RESID, typename T>
__global__ __launch_bounds__(256) void k_band_sym_reduce(const T* __restrict__ win, int64_t wstride,
                                                         const T* __restrict__ f, T* __restrict__ r,
                                                         const int* __restrict__ bpatch,
                                                         const PatchDev* __restrict__ pd) {
  const int64_t b = blockIdx.x;
  const int k = bpatch[b];
  if (k < 0) return;
  const int64_t off = pd[k].off, rows = pd[k].rows;
  const int64_t t = b * ROW_ALIGN - off + threadIdx.x;
  if (t >= rows) return;
  const int n0 = pd[k].n[0];
  const int64_t LS = D == 3 ? (int64_t)n0 * pd[k].n[1] : n0;
  const int W = (int)band_sym_reach(D, P, n0);
  const int64_t ntile = (rows + ROW_ALIGN - 1) / ROW_ALIGN;
  const T* wb = win + (off / ROW_ALIGN) * wstride;     // the patch's first tile
  double acc = 0.0;
#pragma unroll
  for (int kk = 0; kk <= P; ++kk) {
    const int len = kk ? ROW_ALIGN + 2 * W : ROW_ALIGN + W;
    const int wo = kk ? ROW_ALIGN + W + (kk - 1) * (ROW_ALIGN + 2 * W) : 0;
    // row t sits at position q - 256 sg of tile sg's layer-kk window
    const int64_t q = kk ? t - kk * LS + W : t;
    if (q < 0) continue;
    const int64_t lo = q - len + 1 <= 0 ? 0 : (q - len + ROW_ALIGN) / ROW_ALIGN;
    const int64_t hi = min(ntile - 1, q / ROW_ALIGN);
    for (int64_t sg = lo; sg <= hi; ++sg) acc += wb[sg * wstride + wo + (q - sg * ROW_ALIGN)];
  }
  const int64_t g = off + t;
  if constexpr (RESID) r[g] = (T)((double)f[g] - acc);
  else r[g] = (T)acc;
}

// The FP32 full band from the FP64 half band: entry (row, o) of the full
// band is the stored plane of o at the row, or, for an offset of the lower
// half, the stored plane of -o at row + d(o) (zero outside the patch).
template <int D>
__global__ __launch_bounds__(256) void k_band_half_to_full(float* __restrict__ full, const double* __restrict__ half,
                                                           const int* __restrict__ bpatch,
                                                           const PatchDev* __restrict__ pd, int p, int64_t tot) {
  const int nb = 2 * p + 1, nline = (D == 2) ? nb : nb * nb, nbt = nline * nb, lc = (nline - 1) / 2;
  const int nbh = band_half_planes(D, p);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += stride) {
    const int64_t blk = e / ((int64_t)nbt * ROW_ALIGN);
    const int o = (int)((e / ROW_ALIGN) % nbt);
    const int64_t row = blk * ROW_ALIGN + (e % ROW_ALIGN);
    const int k = bpatch[blk];
    float v = 0.f;
    if (k >= 0) {
      const int o0 = o % nb, L = o / nb;
      const int pl = band_half_plane(D, p, o0, L);
      if (pl >= 0) {
        v = (float)half[((row >> 8) * nbh + pl) * ROW_ALIGN + (row & (ROW_ALIGN - 1))];
      } else {
        const PatchDev& P = pd[k];
        const int o1 = L % nb, o2 = (D == 3) ? L / nb : p;
        const int64_t d = (int64_t)(o0 - p) + (int64_t)(o1 - p) * P.n[0] + (int64_t)(o2 - p) * P.n[0] * P.n[1];
        const int64_t rr = row - P.off + d;
        if (row - P.off < P.rows && rr >= 0 && rr < P.rows) {
          const int64_t g2 = P.off + rr;
          const int pn = band_half_plane(D, p, 2 * p - o0, 2 * lc - L);
          v = (float)half[((g2 >> 8) * nbh + pn) * ROW_ALIGN + (g2 & (ROW_ALIGN - 1))];
        }
      }
    }
    full[e] = v;
  }
}

void launch_band_half_to_full(int d, int p, float* full, const double* half, const int* bpatch, const PatchDev* pd,
                              int64_t NL, hipStream_t st) {
  int nbt = 1;
  for (int c = 0; c < d; ++c) nbt *= 2 * p + 1;
  const int64_t tot = (int64_t)nbt * NL;
  if (tot <= 0) return;
  const dim3 grid((unsigned)std::min<int64_t>((tot + 255) / 256, (int64_t)1 << 20));
  if (d == 2)
    hipLaunchKernelGGL(k_band_half_to_full<2>, grid, dim3(256), 0, st, full, half, bpatch, pd, p, tot);
  else
    hipLaunchKernelGGL(k_band_half_to_full<3>, grid, dim3(256), 0, st, full, half, bpatch, pd, p, tot);
}

template <int D, int P, typename T>
static hipError_t launch_band_dp(const T* band, const T* u, const T* f, T* r, const int* bpatch, const PatchDev* pd,
                                 int64_t NL, bool resid, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  dim3 grid((unsigned)(NL / BAND_STRIP)), block(256);
  // FP64: the symmetric half band; FP32: the full band (faster at FP32,
  // where the mirrored reads of the half band cost more than they save)
  constexpr bool HALF = sizeof(T) == 8;
  const void* fn = HALF ? (resid ? reinterpret_cast<const void*>(&k_band_half<D, P, true, T, T>)
                                 : reinterpret_cast<const void*>(&k_band_half<D, P, false, T, T>))
                        : (resid ? reinterpret_cast<const void*>(&k_band_full<D, P, true, T, T>)
                                 : reinterpret_cast<const void*>(&k_band_full<D, P, false, T, T>));
  if (ev0) {
    // timed launch: the events take the dispatch's own start and end stamps
    void* args[] = {(void*)&band, (void*)&u, (void*)&f, (void*)&r, (void*)&bpatch, (void*)&pd};
    return hipExtLaunchKernel(fn, grid, block, args, 0, st, ev0, ev1, 0);
  }
  if (resid) {
    if constexpr (HALF)
      hipLaunchKernelGGL((k_band_half<D, P, true, T, T>), grid, block, 0, st, band, u, f, r, bpatch, pd);
    else
      hipLaunchKernelGGL((k_band_full<D, P, true, T, T>), grid, block, 0, st, band, u, f, r, bpatch, pd);
  } else {
    if constexpr (HALF)
      hipLaunchKernelGGL((k_band_half<D, P, false, T, T>), grid, block, 0, st, band, u, f, r, bpatch, pd);
    else
      hipLaunchKernelGGL((k_band_full<D, P, false, T, T>), grid, block, 0, st, band, u, f, r, bpatch, pd);
  }
  return hipSuccess;
}

template <typename T>
hipError_t launch_band(int d, int p, const T* band, const T* u, const T* f, T* r, const int* bpatch,
                       const PatchDev* pd, int64_t NL, bool resid, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
#define IGAMG_BAND_CASE(DD, PP) \
  if (d == DD && p == PP) return launch_band_dp<DD, PP, T>(band, u, f, r, bpatch, pd, NL, resid, st, ev0, ev1);
  IGAMG_BAND_CASE(2, 1) IGAMG_BAND_CASE(2, 2) IGAMG_BAND_CASE(2, 3) IGAMG_BAND_CASE(2, 4)
  IGAMG_BAND_CASE(2, 5) IGAMG_BAND_CASE(2, 6) IGAMG_BAND_CASE(2, 7) IGAMG_BAND_CASE(2, 8)
  IGAMG_BAND_CASE(3, 1) IGAMG_BAND_CASE(3, 2) IGAMG_BAND_CASE(3, 3) IGAMG_BAND_CASE(3, 4)
  IGAMG_BAND_CASE(3, 5) IGAMG_BAND_CASE(3, 6) IGAMG_BAND_CASE(3, 7) IGAMG_BAND_CASE(3, 8)
#undef IGAMG_BAND_CASE
  return hipErrorInvalidValue;
}

template <int D, int P, typename T>
static hipError_t launch_band_sym_p(const T* band, const T* u, const T* f, T* r, const int* bpatch,
                                    const PatchDev* pd, int64_t NL, int64_t ws, T* win, bool resid, hipStream_t st,
                                    hipEvent_t ev0, hipEvent_t ev1) {
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_band_sym_scatter<D, P, T>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)BAND_SYM_MAX_LDS);
  if (attr != hipSuccess) return attr;
  const dim3 grid((unsigned)(NL / ROW_ALIGN)), b1(64 * (P + 1)), b2(256);
  const size_t lds = (size_t)ws * (sizeof(double) + sizeof(T));   // FP64 windows, u segments
  if (ev0) {
    // timed: the start of the scatter pass to the end of the reduction
    const void* f1 = reinterpret_cast<const void*>(&k_band_sym_scatter<D, P, T>);
    const void* f2 = resid ? reinterpret_cast<const void*>(&k_band_sym_reduce<D, P, true, T>)
                           : reinterpret_cast<const void*>(&k_band_sym_reduce<D, P, false, T>);
    void* a1[] = {(void*)&band, (void*)&u, (void*)&win, (void*)&ws, (void*)&bpatch, (void*)&pd};
    void* a2[] = {(void*)&win, (void*)&ws, (void*)&f, (void*)&r, (void*)&bpatch, (void*)&pd};
    const hipError_t e = hipExtLaunchKernel(f1, grid, b1, a1, lds, st, ev0, nullptr, 0);
    if (e != hipSuccess) return e;
    return hipExtLaunchKernel(f2, grid, b2, a2, 0, st, nullptr, ev1, 0);
  }
  hipLaunchKernelGGL((k_band_sym_scatter<D, P, T>), grid, b1, lds, st, band, u, win, ws, bpatch, pd);
  if (resid)
    hipLaunchKernelGGL((k_band_sym_reduce<D, P, true, T>), grid, b2, 0, st, win, ws, f, r, bpatch, pd);
  else
    hipLaunchKernelGGL((k_band_sym_reduce<D, P, false, T>), grid, b2, 0, st, win, ws, f, r, bpatch, pd);
  return hipSuccess;
}

template <typename T>
hipError_t launch_band_sym(int d, int p, const T* band, const T* u, const T* f, T* r, const int* bpatch,
                           const PatchDev* pd, int64_t NL, int64_t ws, T* win, bool resid, hipStream_t st,
                           hipEvent_t ev0, hipEvent_t ev1) {
  if (ws <= 0 || (size_t)ws * (sizeof(double) + sizeof(T)) > BAND_SYM_MAX_LDS) return hipErrorInvalidValue;
#define IGAMG_SYM_CASE(DD, PP) \
  if (d == DD && p == PP) return launch_band_sym_p<DD, PP, T>(band, u, f, r, bpatch, pd, NL, ws, win, resid, st, ev0, ev1);
  IGAMG_SYM_CASE(2, 1) IGAMG_SYM_CASE(2, 2) IGAMG_SYM_CASE(2, 3) IGAMG_SYM_CASE(2, 4)
  IGAMG_SYM_CASE(2, 5) IGAMG_SYM_CASE(2, 6) IGAMG_SYM_CASE(2, 7) IGAMG_SYM_CASE(2, 8)
  IGAMG_SYM_CASE(3, 1) IGAMG_SYM_CASE(3, 2) IGAMG_SYM_CASE(3, 3) IGAMG_SYM_CASE(3, 4)
  IGAMG_SYM_CASE(3, 5) IGAMG_SYM_CASE(3, 6) IGAMG_SYM_CASE(3, 7) IGAMG_SYM_CASE(3, 8)
#undef IGAMG_SYM_CASE
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// smoother kernels over 2D tensors (a 2D patch interior, a 3D face, or one
// z-slab of a 3D patch interior), split into chunks of rb output columns K
// (rb = 8 or 4, chosen per level by the autotuner):
//   forward:  Y[:, K] = U0^T (X U1[:, K])     (columns K of U0^T X U1)
//   inverse:  Z[:, K] = U0 (Y U1^T[:, K])     (columns K of U0 Y U1^T)
// For 2D tensors the forward kernel applies D^{-1}; for 3D interiors the
// middle direction (with D^{-1}) runs in between as a pencil pass.  The
// forward launch also runs the dense pieces (edges, vertices).  Interface
// items gather their residual from all copies (the accumulation Sigma) and
// add tau z to every copy; interiors use the patch-local vectors directly.
// ---------------------------------------------------------------------------
constexpr int FD_RB = 8;   // widest chunk; also the column stride of the LDS tile C
// columns of a chunk per thread: a 256-thread block has 256 / m0 >= 3 row
// groups for m0 <= FD_LDS_M, so 8 columns need at most 3 per thread; larger
// tensors (m0 <= MAX_FD: at least one group) take up to all 8
constexpr int FD_RPT = 3;
static_assert(256 / FD_LDS_M >= 3 && (FD_RB + 2) / 3 <= FD_RPT, "chunk columns per thread");
static_assert(256 / MAX_FD >= 1, "one row per thread");

// A chunk is rb <= FD_RB columns (second tensor index) of one z-slab, so that the
// results of a chunk are whole columns, contiguous in memory.
__device__ __forceinline__ void fd_chunk(const FDItem& it, int rb, int bx, int& z, int& c0, int& nc) {
  const int nch = (it.m[1] + rb - 1) / rb;
  z = bx / nch;
  c0 = (bx - z * nch) * rb;
  nc = min(rb, it.m[1] - c0);
}

// Thread (j, g) of a block: row j of the tensor, columns g*cpg .. of the chunk.
struct FdLanes {
  int j, a0, na;
  bool act;
  __device__ FdLanes(int m0, int nc) {
    const int G = blockDim.x / m0;
    const int cpg = (nc + G - 1) / G;
    const int g = threadIdx.x / m0;
    j = threadIdx.x - g * m0;
    a0 = g * cpg;
    act = g < G && a0 < nc;
    na = act ? min(cpg, nc - a0) : 0;
  }
};

// acc[i] = sum_b A(j, b) C[b * FD_RB + c_i]  (C: k x FD_RB in LDS), with
// A(j, b) = A[j + m0 b] (column-major, LDS or memory) or given by `at`
template <int RPT, typename T, typename F>
__device__ __forceinline__ void fd_rows_times_chunk_f(F at, const T* C, int k, const FdLanes& L, int nc, T* acc) {
  int cc[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    cc[i] = min(L.a0 + i, nc - 1);
    acc[i] = 0;
  }
  if (!L.act) return;
#pragma unroll 8
  for (int b = 0; b < k; ++b) {
    const T x = at(L.j, b);
#pragma unroll
    for (int i = 0; i < RPT; ++i) acc[i] += x * C[b * FD_RB + cc[i]];
  }
}

template <typename T>
__device__ __forceinline__ void fd_rows_times_chunk(const T* A, const T* C, int m0, int k, const FdLanes& L, int nc,
                                                    T* acc) {
  fd_rows_times_chunk_f<FD_RPT>([=](int j, int b) { return A[j + m0 * b]; }, C, k, L, nc, acc);
}

// Dense piece (edge or vertex): gather the residual over all copies (Sigma),
// z = L^{-1} r with L^{-1} staged in LDS by coalesced loads (row k is thread
// k's), and add (or set) tau z on every copy.
template <typename T>
__device__ void fd_dense_piece(const DensePiece pc, const T* __restrict__ densemat, const T* __restrict__ src,
                               T* __restrict__ u, const int64_t* __restrict__ if_ptr,
                               const int64_t* __restrict__ if_idx, T tau, int add, T* lds) {
  const int m = pc.m;
  const bool big = m > FD_LDS_M;   // L^{-1} read from memory
  T* sA = lds;                     // L^{-1}, row-major m x m
  T* sr = lds + (big ? 0 : m * m); // gathered residual
  const T* A = densemat + pc.Linv;
  if (!big)
    for (int t = threadIdx.x; t < m * m; t += blockDim.x) sA[t] = A[t];
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    T v = 0;
    for (int64_t c = if_ptr[pc.seg + j]; c < if_ptr[pc.seg + j + 1]; ++c) v += src[if_idx[c]];
    sr[j] = v;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < m; k += blockDim.x) {
    T zz = 0;
    const T* ar = (big ? A : sA) + k * m;
#pragma unroll 8
    for (int j = 0; j < m; ++j) zz += ar[j] * sr[j];
    zz *= tau;
    for (int64_t c = if_ptr[pc.seg + k]; c < if_ptr[pc.seg + k + 1]; ++c) {
      const int64_t x = if_idx[c];
      u[x] = add ? u[x] + zz : zz;
    }
  }
}

// block (bx, by) of the forward launch (by >= nitems: dense piece by - nitems)
template <typename T>
__device__ __forceinline__ void fd_fwd_block(int bx, int by, const FDItem* __restrict__ items, int nitems,
                                             const DensePiece* __restrict__ dense, const T* __restrict__ densemat,
                                             const T* __restrict__ mat, const T* __restrict__ src,
                                             T* __restrict__ u, const int64_t* __restrict__ if_ptr,
                                             const int64_t* __restrict__ if_idx, T* __restrict__ scr, T tau, int add,
                                             int rb) {
  DYN_LDS(T, lds);
  const int y = by;
  if (y >= nitems) {
    if (bx == 0) fd_dense_piece(dense[y - nitems], densemat, src, u, if_ptr, if_idx, tau, add, lds);
    return;
  }
  // Y[:, c0 + c] = U0^T (X U1[:, c0 + c]) for the chunk's columns
  const FDItem it = items[y];
  const int m0 = it.m[0], m1 = it.m[1];
  int z, c0, nc;
  fd_chunk(it, rb, bx, z, c0, nc);
  if (z >= it.m[2]) return;
  const int n = m0 * m1;
  const int64_t zoff = (int64_t)z * it.stride[2];
  const T* U0 = mat + it.U[0];
  const T* U1 = mat + it.U[1];
  const FdLanes L(m0, nc);
  T acc[FD_RB];
  if (max(m0, m1) > FD_LDS_M) {
    // large tensor: X and U0 read from memory (coalesced along j), only the
    // chunk of U1 and the intermediate V staged in LDS
    T* C = lds;                      // U1[b, c0 + c] as C[b FD_RB + c]
    T* V = lds + m1 * FD_RB;         // V[j FD_RB + c]
    for (int t = threadIdx.x; t < m1 * FD_RB; t += blockDim.x) {
      const int c = t % FD_RB, b = t / FD_RB;
      C[t] = c < nc ? U1[(int64_t)b * m1 + c0 + c] : (T)0;
    }
    __syncthreads();
    if (it.src_if)
      fd_rows_times_chunk_f<FD_RB>(
          [=](int j, int b) {
            const int64_t e = it.base + j + (int64_t)m0 * b;
            T v = 0;
            for (int64_t c = if_ptr[e]; c < if_ptr[e + 1]; ++c) v += src[if_idx[c]];
            return v;
          },
          C, m1, L, nc, acc);
    else
      fd_rows_times_chunk_f<FD_RB>(
          [=](int j, int b) { return src[it.base + j * it.stride[0] + b * it.stride[1] + zoff]; }, C, m1, L, nc,
          acc);
    for (int i = 0; i < L.na; ++i) V[L.j * FD_RB + L.a0 + i] = acc[i];
    __syncthreads();
    fd_rows_times_chunk_f<FD_RB>([=](int j, int b) { return U0[j + (int64_t)m0 * b]; }, V, m0, L, nc, acc);
  } else {
    T* X = lds;                        // X[j + m0 b]; later U0[j m0 + a]
    T* C = lds + max(n, m0 * m0);      // U1[b, c0 + c] as C[b FD_RB + c]; later V[j FD_RB + c]
    if (it.src_if) {
      for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const int64_t e = it.base + t;  // face tensors are stored j fastest
        T v = 0;
        for (int64_t c = if_ptr[e]; c < if_ptr[e + 1]; ++c) v += src[if_idx[c]];
        X[t] = v;
      }
    } else {
      for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const int j = t % m0, b = t / m0;
        X[t] = src[it.base + j * it.stride[0] + b * it.stride[1] + zoff];
      }
    }
    for (int t = threadIdx.x; t < m1 * FD_RB; t += blockDim.x) {
      const int c = t % FD_RB, b = t / FD_RB;
      C[t] = c < nc ? U1[(int64_t)b * m1 + c0 + c] : (T)0;
    }
    __syncthreads();
    fd_rows_times_chunk(X, C, m0, m1, L, nc, acc);     // V[j, c] = sum_b X[j, b] U1[b, c0 + c]
    __syncthreads();
    for (int i = 0; i < L.na; ++i) C[L.j * FD_RB + L.a0 + i] = acc[i];
    for (int t = threadIdx.x; t < m0 * m0; t += blockDim.x) X[t] = U0[t];
    __syncthreads();
    // Y[a, c] = sum_j U0[j, a] V[j, c]: row a is this thread's j; U0 is read as
    // U0[j m0 + a] = column-major access of U0^T, hence the same helper
    fd_rows_times_chunk(X, C, m0, m0, L, nc, acc);
  }
  if (!L.act) return;
  const T* mu0 = mat + it.mu[0];
  const T* mu1 = mat + it.mu[1];
  const T mu2 = mat[it.mu[2]];
  const bool full = (it.m[2] == 1);
  T* S = scr + it.scr + (int64_t)z * n;
  const int a = L.j;
  for (int i = 0; i < L.na; ++i) {
    const int k = c0 + L.a0 + i;
    T v = acc[i];
    if (full) v /= (T)it.pref * (mu0[a] + mu1[k] + mu2 + (T)it.extra);
    S[a + m0 * k] = v;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fd_fwd(const FDItem* __restrict__ items, int nitems,
                                                const DensePiece* __restrict__ dense,
                                                const T* __restrict__ densemat, const T* __restrict__ mat,
                                                const T* __restrict__ src, T* __restrict__ u,
                                                const int64_t* __restrict__ if_ptr, const int64_t* __restrict__ if_idx,
                                                T* __restrict__ scr, T tau, int add, int rb) {
  fd_fwd_block<T>(blockIdx.x, blockIdx.y, items, nitems, dense, densemat, mat, src, u, if_ptr, if_idx, scr, tau, add,
                  rb);
}

// block (bx, by) of the inverse launch
template <typename T>
__device__ __forceinline__ void fd_inv_block(int bx, int by, const FDItem* __restrict__ items,
                                             const T* __restrict__ mat, T* __restrict__ u,
                                             const int64_t* __restrict__ if_ptr, const int64_t* __restrict__ if_idx,
                                             const T* __restrict__ scr, T tau, int add, int rb) {
  // Z[:, c0 + c] = U0 (Y U1^T[:, c0 + c]) for the chunk's columns
  DYN_LDS(T, lds);
  const FDItem it = items[by];
  const int m0 = it.m[0], m1 = it.m[1];
  int z, c0, nc;
  fd_chunk(it, rb, bx, z, c0, nc);
  if (z >= it.m[2]) return;
  const int n = m0 * m1;
  const T* S = scr + it.scr + (int64_t)z * n;
  const T* U0T = mat + it.U[0] + (int64_t)m0 * m0;
  const T* U1T = mat + it.U[1] + (int64_t)m1 * m1;
  const FdLanes L(m0, nc);
  T acc[FD_RB];
  if (max(m0, m1) > FD_LDS_M) {
    // large tensor: Y and U0^T read from memory, the chunk and V in LDS
    T* C = lds;                      // U1[c0 + c, b] as C[b FD_RB + c]
    T* V = lds + m1 * FD_RB;         // V[j FD_RB + c]
    for (int t = threadIdx.x; t < m1 * FD_RB; t += blockDim.x) {
      const int c = t % FD_RB, b = t / FD_RB;
      C[t] = c < nc ? U1T[(int64_t)b * m1 + c0 + c] : (T)0;
    }
    __syncthreads();
    fd_rows_times_chunk_f<FD_RB>([=](int j, int b) { return S[j + (int64_t)m0 * b]; }, C, m1, L, nc, acc);
    for (int i = 0; i < L.na; ++i) V[L.j * FD_RB + L.a0 + i] = acc[i];
    __syncthreads();
    fd_rows_times_chunk_f<FD_RB>([=](int j, int b) { return U0T[j + (int64_t)m0 * b]; }, V, m0, L, nc, acc);
  } else {
    T* Y = lds;                        // Y[j + m0 b]; later U0^T[j m0 + a]
    T* C = lds + max(n, m0 * m0);      // U1[c0 + c, b] as C[b FD_RB + c]; later V[j FD_RB + c]
    for (int t = threadIdx.x; t < n; t += blockDim.x) Y[t] = S[t];
    for (int t = threadIdx.x; t < m1 * FD_RB; t += blockDim.x) {
      const int c = t % FD_RB, b = t / FD_RB;
      C[t] = c < nc ? U1T[(int64_t)b * m1 + c0 + c] : (T)0;
    }
    __syncthreads();
    fd_rows_times_chunk(Y, C, m0, m1, L, nc, acc);     // V[j, c] = sum_b Y[j, b] U1[c0 + c, b]
    __syncthreads();
    for (int i = 0; i < L.na; ++i) C[L.j * FD_RB + L.a0 + i] = acc[i];
    for (int t = threadIdx.x; t < m0 * m0; t += blockDim.x) Y[t] = U0T[t];
    __syncthreads();
    fd_rows_times_chunk(Y, C, m0, m0, L, nc, acc);     // Z[a, c] = sum_j U0[a, j] V[j, c]
  }
  if (!L.act) return;
  const int64_t zoff = (int64_t)z * it.stride[2];
  const int a = L.j;
  for (int i = 0; i < L.na; ++i) {
    const int k = c0 + L.a0 + i;
    const T v = tau * acc[i];
    if (it.src_if) {
      const int64_t e = it.base + a + (int64_t)m0 * k;
      for (int64_t c = if_ptr[e]; c < if_ptr[e + 1]; ++c) {
        const int64_t x = if_idx[c];
        u[x] = add ? u[x] + v : v;
      }
    } else {
      const int64_t x = it.base + a * it.stride[0] + k * it.stride[1] + zoff;
      u[x] = add ? u[x] + v : v;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fd_inv(const FDItem* __restrict__ items, const T* __restrict__ mat,
                                                T* __restrict__ u, const int64_t* __restrict__ if_ptr,
                                                const int64_t* __restrict__ if_idx, const T* __restrict__ scr, T tau,
                                                int add, int rb) {
  fd_inv_block<T>(blockIdx.x, blockIdx.y, items, mat, u, if_ptr, if_idx, scr, tau, add, rb);
}

// ---------------------------------------------------------------------------
// The same forward and inverse products for FP32 on the matrix cores: every
// mode product of a chunk is a (rows x K) x (K x 16) product done as 16x16
// output tiles of v_mfma_f32_16x16x4f32 (16x4 by 4x16 per instruction, fp32
// accumulation).  Operands are staged in LDS, zero-padded to whole tiles:
// rows to 16, K to 4.  A chunk is 16 columns of one z-slab.
//   lane l of a wave holds A[l % 16][l / 16] and B[l / 16][l % 16] of each
//   4-wide K step, and D[4 (l / 16) + r][l % 16], r = 0..3, of the output tile.
// ---------------------------------------------------------------------------
typedef float fd_f4 __attribute__((ext_vector_type(4)));
constexpr int FDM_N = 16;          // MFMA tile width
constexpr int FDM_CW = 8;          // columns per chunk (<= FDM_N; the rest of the tile is zero)
constexpr int FDM_TILES = 2;       // output row tiles per wave (4 waves x 2 x 16 >= 96 >= FD_LDS_M rows)
static_assert(4 * FDM_TILES * 16 >= FD_LDS_M, "row tiles per wave");

__device__ __forceinline__ int fdm_up(int x, int q) { return (x + q - 1) / q * q; }

typedef short fd_s4 __attribute__((ext_vector_type(4)));

// float to bfloat16, rounded to nearest even (the operands are finite)
__device__ __forceinline__ short fd_bf16(float x) {
  unsigned int v = __float_as_uint(x);
  v += 0x7fffu + ((v >> 16) & 1u);
  return (short)(v >> 16);
}

__device__ __forceinline__ void fdm_chunk(const FDItem& it, int& z, int& c0, int& nc) {
  const int nch = (it.m[1] + FDM_CW - 1) / FDM_CW;
  z = blockIdx.x / nch;
  c0 = (blockIdx.x - z * nch) * FDM_CW;
  nc = min(FDM_CW, it.m[1] - c0);
}

// acc[t] = (A B) rows 16 (w + 4 t) .. of the (mp x kp) A (column-major, leading
// dimension mp) times the (kp x 16) B (row-major), for the tiles of wave w
// With BF16 the operands are rounded to bfloat16 and kp must be a multiple
// of 16 (v_mfma_f32_16x16x16bf16_1k: lane l holds k = 4 (l / 16) .. + 3).
template <bool BF16>
__device__ __forceinline__ void fdm_product(const float* A, int mp, const float* B, int kp, fd_f4* acc) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = l & 15, lk = l >> 4;
#pragma unroll
  for (int t = 0; t < FDM_TILES; ++t) acc[t] = fd_f4{0.f, 0.f, 0.f, 0.f};
  if constexpr (BF16) {
    for (int ks = 0; ks < kp; ks += 16) {
      const int k = ks + 4 * lk;
      fd_s4 b;
#pragma unroll
      for (int q = 0; q < 4; ++q) b[q] = fd_bf16(B[(k + q) * FDM_N + li]);
#pragma unroll
      for (int t = 0; t < FDM_TILES; ++t) {
        const int mt = w + 4 * t;
        if (mt * 16 < mp) {
          fd_s4 a;
#pragma unroll
          for (int q = 0; q < 4; ++q) a[q] = fd_bf16(A[(mt * 16 + li) + mp * (k + q)]);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
        }
      }
    }
  } else {
    for (int ks = 0; ks < kp; ks += 4) {
      const float b = B[(ks + lk) * FDM_N + li];
#pragma unroll
      for (int t = 0; t < FDM_TILES; ++t) {
        const int mt = w + 4 * t;
        if (mt * 16 < mp) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[(mt * 16 + li) + mp * (ks + lk)], b, acc[t], 0, 0, 0);
      }
    }
  }
}

template <bool BF16>
__global__ __launch_bounds__(256) void k_fd_fwd_mfma(const FDItem* __restrict__ items, int nitems,
                                                     const DensePiece* __restrict__ dense,
                                                     const float* __restrict__ densemat, const float* __restrict__ mat,
                                                     const float* __restrict__ src, float* __restrict__ u,
                                                     const int64_t* __restrict__ if_ptr,
                                                     const int64_t* __restrict__ if_idx, float* __restrict__ scr,
                                                     float tau, int add) {
  DYN_LDS(float, lds);
  const int y = blockIdx.y;
  if (y >= nitems) {
    if (blockIdx.x == 0) fd_dense_piece(dense[y - nitems], densemat, src, u, if_ptr, if_idx, tau, add, lds);
    return;
  }
  // Y[:, c0 + c] = U0^T (X U1[:, c0 + c])
  const FDItem it = items[y];
  const int m0 = it.m[0], m1 = it.m[1];
  int z, c0, nc;
  fdm_chunk(it, z, c0, nc);
  if (z >= it.m[2]) return;
  const int kq = BF16 ? 16 : 4;
  const int m0p = fdm_up(m0, 16), m1k = fdm_up(m1, kq), m0k = fdm_up(m0, kq);
  float* X = lds;                                   // X[j + m0p b]; later U0 as A[a + m0p k] = U0[k, a]
  float* C = lds + max(m0p * m1k, m0p * m0k);       // U1[k, c0 + c] as C[k 16 + c]; later V[i 16 + c]
  const int64_t zoff = (int64_t)z * it.stride[2];
  const float* U0 = mat + it.U[0];
  const float* U1 = mat + it.U[1];
  for (int t = threadIdx.x; t < m0p * m1k; t += blockDim.x) {
    const int j = t % m0p, b = t / m0p;
    float v = 0.f;
    if (j < m0 && b < m1) {
      if (it.src_if) {
        const int64_t e = it.base + j + (int64_t)m0 * b;   // face tensors are stored j fastest
        for (int64_t c = if_ptr[e]; c < if_ptr[e + 1]; ++c) v += src[if_idx[c]];
      } else {
        v = src[it.base + j * it.stride[0] + b * it.stride[1] + zoff];
      }
    }
    X[t] = v;
  }
  for (int t = threadIdx.x; t < m1k * FDM_N; t += blockDim.x) {
    const int c = t % FDM_N, k = t / FDM_N;
    C[t] = (k < m1 && c < nc) ? U1[(int64_t)k * m1 + c0 + c] : 0.f;
  }
  __syncthreads();
  fd_f4 acc[FDM_TILES];
  fdm_product<BF16>(X, m0p, C, m1k, acc);            // V = X U1[:, chunk]
  __syncthreads();
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = l & 15, lr = 4 * (l >> 4);
#pragma unroll
  for (int t = 0; t < FDM_TILES; ++t) {
    const int mt = w + 4 * t;
    if (mt * 16 < m0p)
      for (int r = 0; r < 4; ++r) C[(mt * 16 + lr + r) * FDM_N + li] = acc[t][r];   // rows >= m0 hold 0
  }
  for (int t = threadIdx.x; t < m0k * m0p; t += blockDim.x) {
    const int a = t % m0p, k = t / m0p;
    X[t] = (a < m0 && k < m0) ? U0[(int64_t)k * m0 + a] : 0.f;
  }
  __syncthreads();
  fdm_product<BF16>(X, m0p, C, m0k, acc);            // Y = U0^T V
  const float* mu0 = mat + it.mu[0];
  const float* mu1 = mat + it.mu[1];
  const float mu2 = mat[it.mu[2]];
  const bool full = (it.m[2] == 1);
  float* S = scr + it.scr + (int64_t)z * m0 * m1;
#pragma unroll
  for (int t = 0; t < FDM_TILES; ++t) {
    const int mt = w + 4 * t;
    if (mt * 16 >= m0p) continue;
    const int k = c0 + li;
    for (int r = 0; r < 4; ++r) {
      const int a = mt * 16 + lr + r;
      if (a < m0 && li < nc) {
        float v = acc[t][r];
        if (full) v /= (float)it.pref * (mu0[a] + mu1[k] + mu2 + (float)it.extra);
        S[a + m0 * k] = v;
      }
    }
  }
}

template <bool BF16>
__global__ __launch_bounds__(256) void k_fd_inv_mfma(const FDItem* __restrict__ items, const float* __restrict__ mat,
                                                     float* __restrict__ u, const int64_t* __restrict__ if_ptr,
                                                     const int64_t* __restrict__ if_idx, const float* __restrict__ scr,
                                                     float tau, int add) {
  // Z[:, c0 + c] = U0 (Y U1^T[:, c0 + c])
  DYN_LDS(float, lds);
  const FDItem it = items[blockIdx.y];
  const int m0 = it.m[0], m1 = it.m[1];
  int z, c0, nc;
  fdm_chunk(it, z, c0, nc);
  if (z >= it.m[2]) return;
  const int kq = BF16 ? 16 : 4;
  const int m0p = fdm_up(m0, 16), m1k = fdm_up(m1, kq), m0k = fdm_up(m0, kq);
  float* X = lds;                                   // Y[j + m0p b]; later U0 as A[a + m0p k] = U0[a, k]
  float* C = lds + max(m0p * m1k, m0p * m0k);       // U1[c0 + c, k] as C[k 16 + c]; later V[i 16 + c]
  const float* S = scr + it.scr + (int64_t)z * m0 * m1;
  const float* U0T = mat + it.U[0] + (int64_t)m0 * m0;
  const float* U1T = mat + it.U[1] + (int64_t)m1 * m1;
  for (int t = threadIdx.x; t < m0p * m1k; t += blockDim.x) {
    const int j = t % m0p, b = t / m0p;
    X[t] = (j < m0 && b < m1) ? S[j + m0 * b] : 0.f;
  }
  for (int t = threadIdx.x; t < m1k * FDM_N; t += blockDim.x) {
    const int c = t % FDM_N, k = t / FDM_N;
    C[t] = (k < m1 && c < nc) ? U1T[(int64_t)k * m1 + c0 + c] : 0.f;
  }
  __syncthreads();
  fd_f4 acc[FDM_TILES];
  fdm_product<BF16>(X, m0p, C, m1k, acc);            // V = Y U1^T[:, chunk]
  __syncthreads();
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = l & 15, lr = 4 * (l >> 4);
#pragma unroll
  for (int t = 0; t < FDM_TILES; ++t) {
    const int mt = w + 4 * t;
    if (mt * 16 < m0p)
      for (int r = 0; r < 4; ++r) C[(mt * 16 + lr + r) * FDM_N + li] = acc[t][r];
  }
  for (int t = threadIdx.x; t < m0k * m0p; t += blockDim.x) {
    const int a = t % m0p, k = t / m0p;
    X[t] = (a < m0 && k < m0) ? U0T[(int64_t)k * m0 + a] : 0.f;
  }
  __syncthreads();
  fdm_product<BF16>(X, m0p, C, m0k, acc);            // Z = U0 V
  const int64_t zoff = (int64_t)z * it.stride[2];
#pragma unroll
  for (int t = 0; t < FDM_TILES; ++t) {
    const int mt = w + 4 * t;
    if (mt * 16 >= m0p) continue;
    const int k = c0 + li;
    for (int r = 0; r < 4; ++r) {
      const int a = mt * 16 + lr + r;
      if (a >= m0 || li >= nc) continue;
      const float v = tau * acc[t][r];
      if (it.src_if) {
        const int64_t e = it.base + a + (int64_t)m0 * k;
        for (int64_t c = if_ptr[e]; c < if_ptr[e + 1]; ++c) {
          const int64_t x = if_idx[c];
          u[x] = add ? u[x] + v : v;
        }
      } else {
        const int64_t x = it.base + a * it.stride[0] + k * it.stride[1] + zoff;
        u[x] = add ? u[x] + v : v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// One launch per smoothing for 2D tensors (2D patch interiors, 3D faces): a
// workgroup owns one item and keeps it in LDS through all four mode products,
// D^{-1} and the damped update (Sec. 3, the subspace corrected mass smoother
// in fast-diagonalization form):
//   T = X U1,  Y = U0^T T,  Y /= D,  T = Y U1^T,  Z = U0 T,  u += tau Z
// Every product runs on the matrix cores over 16x16 output tiles: FP32
// operands with v_mfma_f32_16x16x4f32, or operands rounded to bfloat16 (FP32
// accumulation) with v_mfma_f32_16x16x16bf16_1k.  Matrices sit in LDS
// row-major, zero-padded to multiples of 16, with an odd leading dimension
// p + 1 so that the 16 rows a wave reads at once fall into distinct banks.
// The dense pieces (edges, vertices) take the workgroups after the items.
// ---------------------------------------------------------------------------
// C (Mp x Np) = A (Mp x Kp) B (Kp x Np), all in LDS; A(i, k) = A[i lda + k]
// or, with TA, A[k lda + i]; B(k, j) = B[k ldb + j] or, with TB, B[j ldb + k].
// Tile t of the (Mp/16) x (Np/16) output goes to wave t mod 4; each wave
// runs two tiles side by side so their accumulation chains interleave.
template <bool TA, bool TB, bool BF16>
__device__ __forceinline__ void fd2_mm(const float* A, int lda, const float* B, int ldb, float* C, int ldc, int Mp,
                                       int Np, int Kp) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = l & 15, lk = l >> 4;
  const int tn = Np / 16, nt = (Mp / 16) * tn;
  auto a_at = [&](int i, int k) { return TA ? A[k * lda + i] : A[i * lda + k]; };
  auto b_at = [&](int k, int j) { return TB ? B[j * ldb + k] : B[k * ldb + j]; };
  for (int t0 = w; t0 < nt; t0 += 8) {
    const int t1 = t0 + 4;
    const bool two = t1 < nt;
    const int r0 = (t0 / tn) * 16 + li, c0 = (t0 % tn) * 16 + li;
    const int r1 = two ? (t1 / tn) * 16 + li : r0, c1 = two ? (t1 % tn) * 16 + li : c0;
    fd_f4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    if constexpr (BF16) {
      for (int ks = 0; ks < Kp; ks += 16) {
        const int k = ks + 4 * lk;
        fd_s4 a0, b0, a1, b1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          a0[q] = fd_bf16(a_at(r0, k + q));
          b0[q] = fd_bf16(b_at(k + q, c0));
          a1[q] = fd_bf16(a_at(r1, k + q));
          b1[q] = fd_bf16(b_at(k + q, c1));
        }
        acc0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b0, acc0, 0, 0, 0);
        if (two) acc1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b1, acc1, 0, 0, 0);
      }
    } else {
      for (int ks = 0; ks < Kp; ks += 4) {
        const int k = ks + lk;
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a_at(r0, k), b_at(k, c0), acc0, 0, 0, 0);
        if (two) acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a_at(r1, k), b_at(k, c1), acc1, 0, 0, 0);
      }
    }
    // lane l holds rows 4 (l / 16) + q of the tile, column l % 16
    const int rr0 = (t0 / tn) * 16 + 4 * lk, rr1 = (t1 / tn) * 16 + 4 * lk;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      C[(rr0 + q) * ldc + c0] = acc0[q];
      if (two) C[(rr1 + q) * ldc + c1] = acc1[q];
    }
  }
}

template <bool BF16>
__global__ __launch_bounds__(256) void k_fd2_fused(const FDItem* __restrict__ items, int nitems,
                                                   const DensePiece* __restrict__ dense,
                                                   const float* __restrict__ densemat, const float* __restrict__ mat,
                                                   const float* __restrict__ src, float* __restrict__ u,
                                                   const int64_t* __restrict__ if_ptr,
                                                   const int64_t* __restrict__ if_idx, float tau, int add) {
  DYN_LDS(float, lds);
  const int y = blockIdx.x;
  if (y >= nitems) {
    fd_dense_piece(dense[y - nitems], densemat, src, u, if_ptr, if_idx, tau, add, lds);
    return;
  }
  const FDItem it = items[y];
  const int m0 = it.m[0], m1 = it.m[1];
  const int p0 = (m0 + 15) / 16 * 16, p1 = (m1 + 15) / 16 * 16;
  const int l0 = p0 + 1, l1 = p1 + 1;          // leading dimensions
  float* X = lds;                              // p0 x p1, ld l1: X, then Y, then Z
  float* T = X + p0 * l1;                      // p0 x p1, ld l1
  float* U0 = T + p0 * l1;                     // p0 x p0, ld l0: U0(i, a)
  float* U1 = U0 + p0 * l0;                    // p1 x p1, ld l1: U1(j, b)
  const float* g0 = mat + it.U[0];
  const float* g1 = mat + it.U[1];
  for (int t = threadIdx.x; t < p0 * p1; t += blockDim.x) {
    const int i = t / p1, j = t % p1;
    float v = 0.f;
    if (i < m0 && j < m1) {
      if (it.src_if) {
        const int64_t e = it.base + i + (int64_t)m0 * j;   // face tensors are stored i fastest
        for (int64_t c = if_ptr[e]; c < if_ptr[e + 1]; ++c) v += src[if_idx[c]];
      } else {
        v = src[it.base + i * it.stride[0] + j * it.stride[1]];
      }
    }
    X[i * l1 + j] = v;
  }
  for (int t = threadIdx.x; t < p0 * p0; t += blockDim.x) {
    const int i = t / p0, a = t % p0;
    U0[i * l0 + a] = (i < m0 && a < m0) ? g0[(int64_t)i * m0 + a] : 0.f;
  }
  for (int t = threadIdx.x; t < p1 * p1; t += blockDim.x) {
    const int j = t / p1, b = t % p1;
    U1[j * l1 + b] = (j < m1 && b < m1) ? g1[(int64_t)j * m1 + b] : 0.f;
  }
  __syncthreads();
  fd2_mm<false, false, BF16>(X, l1, U1, l1, T, l1, p0, p1, p1);    // T = X U1
  __syncthreads();
  fd2_mm<true, false, BF16>(U0, l0, T, l1, X, l1, p0, p1, p0);     // Y = U0^T T
  __syncthreads();
  const float* mu0 = mat + it.mu[0];
  const float* mu1 = mat + it.mu[1];
  const float mu2 = mat[it.mu[2]];
  for (int t = threadIdx.x; t < p0 * p1; t += blockDim.x) {
    const int a = t / p1, b = t % p1;
    X[a * l1 + b] = (a < m0 && b < m1) ? X[a * l1 + b] / ((float)it.pref * (mu0[a] + mu1[b] + mu2 + (float)it.extra))
                                       : 0.f;
  }
  __syncthreads();
  fd2_mm<false, true, BF16>(X, l1, U1, l1, T, l1, p0, p1, p1);     // T = Y U1^T
  __syncthreads();
  fd2_mm<false, false, BF16>(U0, l0, T, l1, X, l1, p0, p1, p0);    // Z = U0 T
  __syncthreads();
  for (int t = threadIdx.x; t < m0 * m1; t += blockDim.x) {
    const int i = t % m0, j = t / m0;
    const float v = tau * X[i * l1 + j];
    if (it.src_if) {
      const int64_t e = it.base + i + (int64_t)m0 * j;
      for (int64_t c = if_ptr[e]; c < if_ptr[e + 1]; ++c) {
        const int64_t x = if_idx[c];
        u[x] = add ? u[x] + v : v;
      }
    } else {
      const int64_t x = it.base + i * it.stride[0] + j * it.stride[1];
      u[x] = add ? u[x] + v : v;
    }
  }
}

size_t fd2_fused_lds(int maxm, int max_dense) {
  const size_t p = (size_t)(maxm + 15) / 16 * 16;
  const size_t items = (3 * p * (p + 1) + p * (p + 1)) * sizeof(float);
  const size_t pieces = ((size_t)max_dense * max_dense + max_dense) * sizeof(float) + 64;
  return std::max(items, pieces);
}

void launch_fd2_fused(const FDItem* items, int nitems, int ndense, size_t lds, const DensePiece* dense,
                      const float* densemat, const float* mat, const float* src, float* u, const int64_t* if_ptr,
                      const int64_t* if_idx, double tau, bool add, bool bf16, hipStream_t st) {
  const int n = nitems + ndense;
  if (n <= 0) return;
  // up to 146 KB of LDS per workgroup (of the 160 KB a CU has)
  static const bool attr = [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fd2_fused<false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fd2_fused<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    return true;
  }();
  (void)attr;
  if (bf16)
    hipLaunchKernelGGL(k_fd2_fused<true>, dim3(n), dim3(256), lds, st, items, nitems, dense, densemat, mat, src, u,
                       if_ptr, if_idx, (float)tau, (int)add);
  else
    hipLaunchKernelGGL(k_fd2_fused<false>, dim3(n), dim3(256), lds, st, items, nitems, dense, densemat, mat, src, u,
                       if_ptr, if_idx, (float)tau, (int)add);
}

// Middle direction of 3D patch interiors, in place on the compact scratch
// tensor: along direction 2, y = U2 diag(1/D) U2^T x for every (i0, i1).
__device__ __forceinline__ int fd_mid_lines(int L) { return max(1, min(64, 512 / L)); }

template <typename T>
__device__ __forceinline__ void fd_mid_block(int bx, int by, const FDItem* __restrict__ items,
                                             const T* __restrict__ mat, T* __restrict__ scr) {
  DYN_LDS(T, lds);
  const FDItem it = items[by];
  const int L = it.m[2];
  if (L <= 1) return;
  const int m0 = it.m[0];
  const int64_t lines = (int64_t)m0 * it.m[1];
  const int LB = fd_mid_lines(L);
  const int64_t line0 = (int64_t)bx * LB;
  if (line0 >= lines) return;
  const int nl = (int)min((int64_t)LB, lines - line0);
  const T* U = mat + it.U[2];
  const bool big = L > FD_LDS_M;     // U read from memory
  T* sx = lds + (big ? 0 : L * L);
  T* sy = sx + LB * L;
  const T* sU = big ? U : lds;
  if (!big)
    for (int i = threadIdx.x; i < L * L; i += blockDim.x) lds[i] = U[i];
  T* S = scr + it.scr;
  const int64_t plane = lines;
  const int total = nl * L;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int j = t / nl, line = t - j * nl;  // lines are consecutive in memory
    sx[line * L + j] = S[line0 + line + j * plane];
  }
  __syncthreads();
  const T* mu0 = mat + it.mu[0];
  const T* mu1 = mat + it.mu[1];
  const T* mu2 = mat + it.mu[2];
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int line = t / L, kk = t - line * L;
    const T* x = sx + line * L;
    T s = 0;
    for (int j = 0; j < L; ++j) s += sU[j * L + kk] * x[j];
    const int64_t gl = line0 + line;
    const int i0 = (int)(gl % m0), i1 = (int)(gl / m0);
    sy[t] = s / ((T)it.pref * (mu0[i0] + mu1[i1] + mu2[kk] + (T)it.extra));
  }
  __syncthreads();
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int line = t / L, kk = t - line * L;
    const T* x = sy + line * L;
    const T* ur = sU + kk * L;
    T s = 0;
    for (int j = 0; j < L; ++j) s += ur[j] * x[j];
    sx[t] = s;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int j = t / nl, line = t - j * nl;
    S[line0 + line + j * plane] = sx[line * L + j];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fd_mid(const FDItem* __restrict__ items, const T* __restrict__ mat,
                                                T* __restrict__ scr) {
  fd_mid_block<T>(blockIdx.x, blockIdx.y, items, mat, scr);
}

size_t fd_mfma_lds(int maxm) {
  // K padded to 16 (enough for both precisions)
  const size_t mp = (size_t)(maxm + 15) / 16 * 16;
  return (mp * mp + (size_t)FDM_N * mp) * sizeof(float) + 64;
}

int fd_mfma_grid(const FDItem* items, int nitems) {
  int g = 1;
  for (int i = 0; i < nitems; ++i) g = std::max(g, items[i].m[2] * ((items[i].m[1] + FDM_CW - 1) / FDM_CW));
  return g;
}

void launch_fd_fwd_mfma(const FDItem* items, int nitems, int ndense, int gridx, size_t lds, const DensePiece* dense,
                        const float* densemat, const float* mat, const float* src, float* u, const int64_t* if_ptr,
                        const int64_t* if_idx, float* scr, double tau, bool add, bool bf16, hipStream_t st) {
  const int ny = nitems + ndense;
  if (ny <= 0) return;
  if (bf16)
    hipLaunchKernelGGL(k_fd_fwd_mfma<true>, dim3(gridx, ny), dim3(256), lds, st, items, nitems, dense, densemat, mat,
                       src, u, if_ptr, if_idx, scr, (float)tau, (int)add);
  else
    hipLaunchKernelGGL(k_fd_fwd_mfma<false>, dim3(gridx, ny), dim3(256), lds, st, items, nitems, dense, densemat, mat,
                       src, u, if_ptr, if_idx, scr, (float)tau, (int)add);
}

void launch_fd_inv_mfma(const FDItem* items, int nitems, int gridx, size_t lds, const float* mat, float* u,
                        const int64_t* if_ptr, const int64_t* if_idx, const float* scr, double tau, bool add,
                        bool bf16, hipStream_t st) {
  if (nitems <= 0) return;
  if (bf16)
    hipLaunchKernelGGL(k_fd_inv_mfma<true>, dim3(gridx, nitems), dim3(256), lds, st, items, mat, u, if_ptr, if_idx,
                       scr, (float)tau, (int)add);
  else
    hipLaunchKernelGGL(k_fd_inv_mfma<false>, dim3(gridx, nitems), dim3(256), lds, st, items, mat, u, if_ptr, if_idx,
                       scr, (float)tau, (int)add);
}

// the exact edge and vertex pieces' entries: sums of listed half-band
// entries (setup only; one thread per entry, the list order fixes the sum)
__global__ __launch_bounds__(256) void k_band_gather(const double* __restrict__ band, int nbh,
                                                     const int64_t* __restrict__ ptr, const int64_t* __restrict__ row,
                                                     const int* __restrict__ plane, int64_t ne,
                                                     double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  double s = 0.0;
  for (int64_t c = ptr[e]; c < ptr[e + 1]; ++c) {
    const int64_t g = row[c];
    s += band[((g >> 8) * nbh + plane[c]) * ROW_ALIGN + (g & (ROW_ALIGN - 1))];
  }
  out[e] = s;
}

void launch_band_gather(const double* band, int nbh, const int64_t* ptr, const int64_t* row, const int* plane,
                        int64_t ne, double* out, hipStream_t st) {
  if (ne <= 0) return;
  hipLaunchKernelGGL(k_band_gather, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, band, nbh, ptr, row, plane,
                     ne, out);
}

// LDS of the vector FD kernels for tensors of sides up to maxm: those up to
// FD_LDS_M staged whole, larger ones only their chunk and intermediate
size_t fd_dense_lds(int maxm, size_t elem) {
  const size_t s = (size_t)std::min(maxm, FD_LDS_M);
  return std::max(s * s + s, (size_t)maxm) * elem + 64;
}
size_t fd_slab_lds(int maxm, size_t elem) {
  const size_t s = (size_t)std::min(maxm, FD_LDS_M);
  return std::max(s * s + (size_t)FD_RB * s, (size_t)(2 * FD_RB) * maxm) * elem + 64;
}

int fd_slab_grid(const FDItem* items, int nitems, int rb) {
  int g = 1;
  for (int i = 0; i < nitems; ++i) g = std::max(g, items[i].m[2] * ((items[i].m[1] + rb - 1) / rb));
  return g;
}

int fd_mid_grid(const FDItem* items, int nitems) {
  int64_t g = 1;
  for (int i = 0; i < nitems; ++i) {
    const int L = std::max(1, items[i].m[2]);
    const int LB = std::max(1, std::min(64, 512 / L));
    g = std::max(g, ((int64_t)items[i].m[0] * items[i].m[1] + LB - 1) / LB);
  }
  return (int)g;
}

size_t fd_mid_lds(int maxm, size_t elem) {
  const size_t s = (size_t)std::min(maxm, FD_LDS_M);
  return (s * s + 2 * std::max<size_t>(512, (size_t)maxm)) * elem + 64;
}

template <typename T>
void launch_fd_fwd(const FDItem* items, int nitems, int ndense, int gridx, size_t lds, const DensePiece* dense,
                   const T* densemat, const T* mat, const T* src, T* u, const int64_t* if_ptr, const int64_t* if_idx,
                   T* scr, double tau, bool add, int rb, hipStream_t st) {
  const int ny = nitems + ndense;
  if (ny <= 0) return;
  hipLaunchKernelGGL(k_fd_fwd<T>, dim3(gridx, ny), dim3(256), lds, st, items, nitems, dense, densemat, mat, src, u,
                     if_ptr, if_idx, scr, (T)tau, (int)add, rb);
}

template <typename T>
void launch_fd_mid(const FDItem* items, int nitems, int gridx, size_t lds, const T* mat, T* scr, hipStream_t st) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(k_fd_mid<T>, dim3(gridx, nitems), dim3(256), lds, st, items, mat, scr);
}

template <typename T>
void launch_fd_inv(const FDItem* items, int nitems, int gridx, size_t lds, const T* mat, T* u, const int64_t* if_ptr,
                   const int64_t* if_idx, const T* scr, double tau, bool add, int rb, hipStream_t st) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(k_fd_inv<T>, dim3(gridx, nitems), dim3(256), lds, st, items, mat, u, if_ptr, if_idx, scr, (T)tau,
                     (int)add, rb);
}

// ---------------------------------------------------------------------------
// transfers (Sec. 3: P_l and P_l^T, per patch as a Kronecker product of the
// univariate knot-insertion matrices; Sec. 4: P maps accumulated to
// accumulated, P^T distributed to distributed vectors)
// ---------------------------------------------------------------------------
template <int D, int WR, typename T>
__device__ __forceinline__ void restrict_block(int64_t b, const T* __restrict__ rf, T* __restrict__ rc,
                                               const PatchDev* __restrict__ pd, const int* __restrict__ bpatch_c,
                                               const int64_t* __restrict__ tidx, const T* __restrict__ tval,
                                               const uint8_t* __restrict__ isfree_c) {
  const int k = bpatch_c[b];
  if (k < 0) return;
  const PatchDev& P = pd[k];
  const int64_t g = (int64_t)b * ROW_ALIGN + threadIdx.x;
  const int64_t rl = g - P.offc;
  if (rl >= P.rowsc) return;
  if (!isfree_c[g]) {
    rc[g] = 0;
    return;
  }
  const int j0 = (int)(rl % P.nc[0]);
  const int64_t t = rl / P.nc[0];
  const int j1 = (int)(t % P.nc[1]);
  const int j2 = (int)(t / P.nc[1]);
  const int s0 = (int)tidx[P.Rst[0] + j0], s1 = (int)tidx[P.Rst[1] + j1], s2 = (int)tidx[P.Rst[2] + j2];
  const T* w0 = tval + P.Rval[0] + (int64_t)j0 * WR;
  const T* w1 = tval + P.Rval[1] + (int64_t)j1 * WR;
  const T* w2 = tval + P.Rval[2] + (int64_t)j2 * WR;
  const int n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
  const T* src = rf + P.off;
  // WR is the table width: rows with fewer weights are padded with zeros, and
  // clamped indices keep every read inside the patch
  T v0[WR], v1[WR];
  int ix0[WR];
#pragma unroll
  for (int a = 0; a < WR; ++a) {
    v0[a] = w0[a];
    v1[a] = w1[a];
    ix0[a] = min(s0 + a, n0 - 1);
  }
  T s = 0;
  constexpr int W2 = (D == 3) ? WR : 1;
#pragma unroll
  for (int a2 = 0; a2 < W2; ++a2) {
    const T c2 = (D == 3) ? w2[a2] : T(1);
    const int64_t z = (int64_t)min(s2 + a2, n2 - 1) * n0 * n1;
#pragma unroll
    for (int a1 = 0; a1 < WR; ++a1) {
      const T* row = src + z + (int64_t)min(s1 + a1, n1 - 1) * n0;
      T acc = 0;
#pragma unroll
      for (int a0 = 0; a0 < WR; ++a0) acc += v0[a0] * row[ix0[a0]];
      s += c2 * v1[a1] * acc;
    }
  }
  rc[g] = s;
}

template <int D, int WR, typename T>
__global__ __launch_bounds__(256) void k_restrict(const T* __restrict__ rf, T* __restrict__ rc,
                                                  const PatchDev* __restrict__ pd, const int* __restrict__ bpatch_c,
                                                  const int64_t* __restrict__ tidx, const T* __restrict__ tval,
                                                  const uint8_t* __restrict__ isfree_c) {
  restrict_block<D, WR, T>(blockIdx.x, rf, rc, pd, bpatch_c, tidx, tval, isfree_c);
}

template <int D, int WP, typename T>
__device__ __forceinline__ void prolong_block(int64_t b, const T* __restrict__ uc, T* __restrict__ uf,
                                              const PatchDev* __restrict__ pd, const int* __restrict__ bpatch_f,
                                              const int64_t* __restrict__ tidx, const T* __restrict__ tval,
                                              const uint8_t* __restrict__ isfree_f) {
  const int k = bpatch_f[b];
  if (k < 0) return;
  const PatchDev& P = pd[k];
  const int64_t g = (int64_t)b * ROW_ALIGN + threadIdx.x;
  const int64_t rl = g - P.off;
  if (rl >= P.rows) return;
  if (!isfree_f[g]) return;
  const int i0 = (int)(rl % P.n[0]);
  const int64_t t = rl / P.n[0];
  const int i1 = (int)(t % P.n[1]);
  const int i2 = (int)(t / P.n[1]);
  const int s0 = (int)tidx[P.Pst[0] + i0], s1 = (int)tidx[P.Pst[1] + i1], s2 = (int)tidx[P.Pst[2] + i2];
  const T* w0 = tval + P.Pval[0] + (int64_t)i0 * WP;
  const T* w1 = tval + P.Pval[1] + (int64_t)i1 * WP;
  const T* w2 = tval + P.Pval[2] + (int64_t)i2 * WP;
  const int n0 = P.nc[0], n1 = P.nc[1], n2 = P.nc[2];
  const T* src = uc + P.offc;
  T v0[WP], v1[WP];
  int ix0[WP];
#pragma unroll
  for (int a = 0; a < WP; ++a) {
    v0[a] = w0[a];
    v1[a] = w1[a];
    ix0[a] = min(s0 + a, n0 - 1);
  }
  T s = 0;
  constexpr int W2 = (D == 3) ? WP : 1;
#pragma unroll
  for (int a2 = 0; a2 < W2; ++a2) {
    const T c2 = (D == 3) ? w2[a2] : T(1);
    const int64_t z = (int64_t)min(s2 + a2, n2 - 1) * n0 * n1;
#pragma unroll
    for (int a1 = 0; a1 < WP; ++a1) {
      const T* row = src + z + (int64_t)min(s1 + a1, n1 - 1) * n0;
      T acc = 0;
#pragma unroll
      for (int a0 = 0; a0 < WP; ++a0) acc += v0[a0] * row[ix0[a0]];
      s += c2 * v1[a1] * acc;
    }
  }
  uf[g] += s;
}

template <int D, int WP, typename T>
__global__ __launch_bounds__(256) void k_prolong_add(const T* __restrict__ uc, T* __restrict__ uf,
                                                     const PatchDev* __restrict__ pd,
                                                     const int* __restrict__ bpatch_f,
                                                     const int64_t* __restrict__ tidx, const T* __restrict__ tval,
                                                     const uint8_t* __restrict__ isfree_f) {
  prolong_block<D, WP, T>(blockIdx.x, uc, uf, pd, bpatch_f, tidx, tval, isfree_f);
}

template <int D, typename T>
static void restrict_w(const T* rf, T* rc, const PatchDev* pd, const int* bpatch_c, int64_t NLc, const int64_t* tidx,
                       const T* tval, int WR, const uint8_t* isfree_c, hipStream_t st) {
  dim3 grid((unsigned)(NLc / ROW_ALIGN)), block(ROW_ALIGN);
  switch (WR) {
#define IGAMG_W(W) \
  case W: hipLaunchKernelGGL((k_restrict<D, W, T>), grid, block, 0, st, rf, rc, pd, bpatch_c, tidx, tval, isfree_c); return;
    IGAMG_W(1) IGAMG_W(2) IGAMG_W(3) IGAMG_W(4) IGAMG_W(5) IGAMG_W(6) IGAMG_W(7) IGAMG_W(8) IGAMG_W(9) IGAMG_W(10)
#undef IGAMG_W
    default: break;
  }
}

template <int D, typename T>
static void prolong_w(const T* uc, T* uf, const PatchDev* pd, const int* bpatch_f, int64_t NLf, const int64_t* tidx,
                      const T* tval, int WP, const uint8_t* isfree_f, hipStream_t st) {
  dim3 grid((unsigned)(NLf / ROW_ALIGN)), block(ROW_ALIGN);
  switch (WP) {
#define IGAMG_W(W) \
  case W: hipLaunchKernelGGL((k_prolong_add<D, W, T>), grid, block, 0, st, uc, uf, pd, bpatch_f, tidx, tval, isfree_f); return;
    IGAMG_W(1) IGAMG_W(2) IGAMG_W(3) IGAMG_W(4) IGAMG_W(5) IGAMG_W(6) IGAMG_W(7) IGAMG_W(8) IGAMG_W(9) IGAMG_W(10)
#undef IGAMG_W
    default: break;
  }
}

// table widths are at most p + 2 <= 10 (p <= 8)
template <typename T>
void launch_restrict(int d, const T* rf, T* rc, const PatchDev* pd, const int* bpatch_c, int64_t NLc,
                     const int64_t* tidx, const T* tval, int WR, const uint8_t* isfree_c, hipStream_t st) {
  if (d == 2)
    restrict_w<2, T>(rf, rc, pd, bpatch_c, NLc, tidx, tval, WR, isfree_c, st);
  else
    restrict_w<3, T>(rf, rc, pd, bpatch_c, NLc, tidx, tval, WR, isfree_c, st);
}

template <typename T>
void launch_prolong_add(int d, const T* uc, T* uf, const PatchDev* pd, const int* bpatch_f, int64_t NLf,
                        const int64_t* tidx, const T* tval, int WP, const uint8_t* isfree_f, hipStream_t st) {
  if (d == 2)
    prolong_w<2, T>(uc, uf, pd, bpatch_f, NLf, tidx, tval, WP, isfree_f, st);
  else
    prolong_w<3, T>(uc, uf, pd, bpatch_f, NLf, tidx, tval, WP, isfree_f, st);
}

// ---------------------------------------------------------------------------
// global <-> patch-local conversions and the coarse solve (Sec. 4,
// chi A_0^{-1} Sigma_glob): b = sum of copies, x = A_0^{-1} b in FP64, x to
// every copy
// ---------------------------------------------------------------------------
template <typename TL, typename TG>
__device__ __forceinline__ void gather_dist_block(int64_t bx, const TL* __restrict__ loc, TG* __restrict__ glob,
                                                  const int64_t* __restrict__ ptr, const int64_t* __restrict__ idx,
                                                  int64_t n) {
  const int64_t g = bx * blockDim.x + threadIdx.x;
  if (g >= n) return;
  double s = 0.0;
  for (int64_t c = ptr[g]; c < ptr[g + 1]; ++c) s += (double)loc[idx[c]];
  glob[g] = (TG)s;
}

template <typename TL, typename TG>
__global__ __launch_bounds__(256) void k_gather_dist(const TL* __restrict__ loc, TG* __restrict__ glob,
                                                     const int64_t* __restrict__ ptr,
                                                     const int64_t* __restrict__ idx, int64_t n) {
  gather_dist_block<TL, TG>(blockIdx.x, loc, glob, ptr, idx, n);
}

__global__ __launch_bounds__(256) void k_gather_acc(const double* __restrict__ loc, double* __restrict__ glob,
                                                    const int64_t* __restrict__ ptr, const int64_t* __restrict__ idx,
                                                    int64_t n) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  glob[g] = loc[idx[ptr[g]]];
}

__global__ __launch_bounds__(256) void k_scatter_acc(const double* __restrict__ glob, double* __restrict__ loc,
                                                     const int64_t* __restrict__ ptr,
                                                     const int64_t* __restrict__ idx, int64_t n) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const double v = glob[g];
  for (int64_t c = ptr[g]; c < ptr[g + 1]; ++c) loc[idx[c]] = v;
}

__global__ __launch_bounds__(256) void k_scatter_dist(const double* __restrict__ glob, double* __restrict__ loc,
                                                      const int64_t* __restrict__ ptr,
                                                      const int64_t* __restrict__ idx, int64_t n) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const int64_t c0 = ptr[g];
  loc[idx[c0]] = glob[g];
  for (int64_t c = c0 + 1; c < ptr[g + 1]; ++c) loc[idx[c]] = 0.0;
}

void launch_gather(const double* loc, double* glob, const int64_t* ptr, const int64_t* idx, int64_t n, bool dist,
                   hipStream_t st) {
  if (n <= 0) return;
  dim3 grid((unsigned)((n + 255) / 256));
  if (dist)
    hipLaunchKernelGGL((k_gather_dist<double, double>), grid, dim3(256), 0, st, loc, glob, ptr, idx, n);
  else
    hipLaunchKernelGGL(k_gather_acc, grid, dim3(256), 0, st, loc, glob, ptr, idx, n);
}

void launch_scatter(const double* glob, double* loc, const int64_t* ptr, const int64_t* idx, int64_t n, bool dist,
                    hipStream_t st) {
  if (n <= 0) return;
  dim3 grid((unsigned)((n + 255) / 256));
  if (dist)
    hipLaunchKernelGGL(k_scatter_dist, grid, dim3(256), 0, st, glob, loc, ptr, idx, n);
  else
    hipLaunchKernelGGL(k_scatter_acc, grid, dim3(256), 0, st, glob, loc, ptr, idx, n);
}

// x = A_0^{-1} b with the symmetric inverse in packed lower tiles (each
// stored tile read once).  Tile (I, J), J < I, gives its product with b_J to
// block row I and its transpose's product with b_I to block row J; a
// diagonal tile (both triangles stored) gives only the first.  The partial
// results go to part[(R * T + X) * 64 + r] for block row R and the other
// block index X (each slot written by exactly one tile), and the second pass
// sums the T slots of each row in a fixed order: the result does not depend
// on the order in which tiles run.  Row i of x then goes to every local copy
// of coarse dof i (the restriction chi of the coarse solve).
__device__ __forceinline__ void tri_index(int64_t t, int64_t& a, int64_t& b) {
  int64_t x = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (x * (x + 1) / 2 > t) --x;
  while ((x + 1) * (x + 2) / 2 <= t) ++x;
  a = x;
  b = t - x * (x + 1) / 2;
}

// Sums v[0..2H) over the 64 lanes of a wavefront by halving: at each step a
// lane keeps one half of its values (the upper if `lane & off`), adds the
// partner's copy of that half and passes the other half on.  Returns the
// full sum of value index `row` (written), equal on the four lanes that
// differ only in bits 0 and 1.
template <int H>
__device__ __forceinline__ double lane_transpose_sum(const double (&v)[2 * H], int lane, int& row) {
  double k[H];
  const bool up = lane & (2 * H * 2);   // offsets 32, 16, 8, 4 for H = 8, 4, 2, 1
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const double give = up ? v[i] : v[H + i];
    k[i] = (up ? v[H + i] : v[i]) + __shfl_xor(give, 2 * H * 2, 64);
  }
  row += up ? H : 0;
  if constexpr (H == 1) {
    double s = k[0];
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    return s;
  } else {
    return lane_transpose_sum<H / 2>(k, lane, row);
  }
}

template <typename M>
__device__ __forceinline__ void coarse_tiles_block(int64_t bx, const M* __restrict__ Ainv,
                                                   const double* __restrict__ b, double* __restrict__ part,
                                                   int64_t n) {
  constexpr int CT = COARSE_TILE;
  __shared__ double s_bj[CT], s_bi[CT], s_red[4][CT];
  int64_t I, J;
  tri_index(bx, I, J);
  const int64_t T = coarse_tiles(n);
  const int c = threadIdx.x & (CT - 1), g = threadIdx.x >> 6;
  if (threadIdx.x < CT) {
    const int64_t j = J * CT + threadIdx.x;
    s_bj[threadIdx.x] = j < n ? b[j] : 0.0;
  } else if (threadIdx.x < 2 * CT) {
    const int64_t i = I * CT + threadIdx.x - CT;
    s_bi[threadIdx.x - CT] = i < n ? b[i] : 0.0;
  }
  __syncthreads();
  // wavefront g holds rows 16 g .. 16 g + 15 of the tile, lane c column c
  const M* tile = Ainv + coarse_tile_at(I, J);
  double v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = (double)tile[(g * 16 + i) * CT + c];
  const double bj = s_bj[c];
  double colsum = 0.0, pr[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    pr[i] = v[i] * bj;
    colsum += v[i] * s_bi[g * 16 + i];
  }
  s_red[g][c] = colsum;
  int row = 0;
  const double rs = lane_transpose_sum<8>(pr, c, row);
  if ((c & 3) == 0) part[(I * T + J) * CT + g * 16 + row] = rs;
  __syncthreads();
  if (I != J && threadIdx.x < CT)
    part[(J * T + I) * CT + threadIdx.x] = (s_red[0][threadIdx.x] + s_red[1][threadIdx.x]) +
                                           (s_red[2][threadIdx.x] + s_red[3][threadIdx.x]);
}

template <typename T>
__device__ __forceinline__ void coarse_reduce_block(int64_t bx, const double* __restrict__ part, T* __restrict__ u0,
                                                    const int64_t* __restrict__ ptr, const int64_t* __restrict__ idx,
                                                    int64_t n) {
  // block bx = tile row R: wave w sums the partial products of tile
  // columns [w T / 4, (w + 1) T / 4) for the tile's 64 rows, and wave 0 adds
  // the four quarters in a fixed order
  constexpr int CT = COARSE_TILE;
  __shared__ double s_q[4][CT];
  const int r = threadIdx.x & (CT - 1), w = threadIdx.x >> 6;
  const int64_t Tn = coarse_tiles(n);
  const double* pr = part + bx * Tn * CT + r;
  const int64_t x0 = Tn * w / 4, x1 = Tn * (w + 1) / 4;
  double s = 0.0;
#pragma unroll 4
  for (int64_t x = x0; x < x1; ++x) s += pr[x * CT];
  s_q[w][r] = s;
  __syncthreads();
  const int64_t row = bx * CT + r;
  if (w == 0 && row < n) {
    const double t = (s_q[0][r] + s_q[1][r]) + (s_q[2][r] + s_q[3][r]);
    for (int64_t c = ptr[row]; c < ptr[row + 1]; ++c) u0[idx[c]] = (T)t;
  }
}

template <typename M>
__global__ __launch_bounds__(256) void k_coarse_tiles(const M* __restrict__ Ainv, const double* __restrict__ b,
                                                      double* __restrict__ part, int64_t n) {
  coarse_tiles_block<M>(blockIdx.x, Ainv, b, part, n);
}

__global__ __launch_bounds__(256) void k_to_float(const double* __restrict__ x, float* __restrict__ y, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = (float)x[i];
}

void launch_to_float(const double* x, float* y, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, (int64_t)1 << 16);
  hipLaunchKernelGGL(k_to_float, dim3((unsigned)blocks), dim3(256), 0, st, x, y, n);
}

template <typename T>
__global__ __launch_bounds__(256) void k_coarse_reduce(const double* __restrict__ part, T* __restrict__ u0,
                                                       const int64_t* __restrict__ ptr,
                                                       const int64_t* __restrict__ idx, int64_t n) {
  coarse_reduce_block<T>(blockIdx.x, part, u0, ptr, idx, n);
}

template <typename T>
void launch_coarse(const T* Ainv, const T* f0, double* b, double* part, T* u0, const int64_t* ptr,
                   const int64_t* idx, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  const int64_t Tn = coarse_tiles(n);
  hipLaunchKernelGGL((k_gather_dist<T, double>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, f0, b, ptr, idx,
                     n);
  hipLaunchKernelGGL(k_coarse_tiles<T>, dim3((unsigned)(Tn * (Tn + 1) / 2)), dim3(256), 0, st, Ainv, b, part, n);
  hipLaunchKernelGGL(k_coarse_reduce<T>, dim3((unsigned)Tn), dim3(256), 0, st, part, u0, ptr, idx, n);
}

// ---------------------------------------------------------------------------
// The coarse levels of a cycle in one persistent launch.  The phases of the
// cycle below a level (smoothing products, residuals, transfers, the coarse
// solve) form one work list; a workgroup takes the next ticket (a run of
// consecutive items of one phase), waits until every ticket of the previous
// phase has finished (a completion counter per phase), runs its items with
// the same bodies as the separate launches would, and counts the ticket
// done.  Tickets are taken in order, so every ticket a workgroup waits for
// was taken before by a running workgroup that is not itself waiting on a
// later ticket: the list always drains, whatever number of workgroups is
// resident (no co-residency assumption, no grid barrier).  The counters are
// at agent scope with release/acquire fences, so results written on one XCD
// are seen on another; the wait polls with relaxed loads and acquires once,
// since an acquire invalidates the L2 of the waiting XCD.  ctr[0] is the
// ticket counter, ctr[1 + k] the finished tickets of phase k, ctr[1 + nph]
// an overflow flag set if a wait ever exceeded its (very large) spin bound.
// ---------------------------------------------------------------------------
template <int D, int P, typename T>
__device__ __forceinline__ void tail_item(const Phase& ph, int64_t t) {
  const int bx = (int)(t % ph.gx), by = (int)(t / ph.gx);
  const void* const* a = ph.a;
  switch (ph.kind) {
    case PH_BAND: {
      const T* band = static_cast<const T*>(a[0]);
      const T* u = static_cast<const T*>(a[1]);
      const T* f = static_cast<const T*>(a[2]);
      T* r = const_cast<T*>(static_cast<const T*>(a[3]));
      const int* bp = static_cast<const int*>(a[4]);
      const PatchDev* pd = static_cast<const PatchDev*>(a[5]);
      if constexpr (sizeof(T) == 8) {
        if (ph.resid) band_half_strip<D, P, true, T, T>(t, band, u, f, r, bp, pd);
        else band_half_strip<D, P, false, T, T>(t, band, u, f, r, bp, pd);
      } else {
        if (ph.resid) band_full_strip<D, P, true, T, T>(t, band, u, f, r, bp, pd);
        else band_full_strip<D, P, false, T, T>(t, band, u, f, r, bp, pd);
      }
      break;
    }
    case PH_FD_FWD:
      fd_fwd_block<T>(bx, by, static_cast<const FDItem*>(a[0]), ph.nitems, static_cast<const DensePiece*>(a[1]),
                      static_cast<const T*>(a[2]), static_cast<const T*>(a[3]), static_cast<const T*>(a[4]),
                      const_cast<T*>(static_cast<const T*>(a[5])), static_cast<const int64_t*>(a[6]),
                      static_cast<const int64_t*>(a[7]), const_cast<T*>(static_cast<const T*>(a[8])), (T)ph.tau,
                      ph.add, ph.rb);
      break;
    case PH_FD_MID:
      fd_mid_block<T>(bx, by, static_cast<const FDItem*>(a[0]), static_cast<const T*>(a[1]),
                      const_cast<T*>(static_cast<const T*>(a[2])));
      break;
    case PH_FD_INV:
      fd_inv_block<T>(bx, by, static_cast<const FDItem*>(a[0]), static_cast<const T*>(a[1]),
                      const_cast<T*>(static_cast<const T*>(a[2])), static_cast<const int64_t*>(a[3]),
                      static_cast<const int64_t*>(a[4]), static_cast<const T*>(a[5]), (T)ph.tau, ph.add, ph.rb);
      break;
    case PH_RESTRICT:
    case PH_PROLONG: {
      const T* x = static_cast<const T*>(a[0]);
      T* y = const_cast<T*>(static_cast<const T*>(a[1]));
      const PatchDev* pd = static_cast<const PatchDev*>(a[2]);
      const int* bp = static_cast<const int*>(a[3]);
      const int64_t* ti = static_cast<const int64_t*>(a[4]);
      const T* tv = static_cast<const T*>(a[5]);
      const uint8_t* fr = static_cast<const uint8_t*>(a[6]);
      // table widths run up to P + 2
#define IGAMG_TAIL_W(W)                                                              \
  case W:                                                                            \
    if (ph.kind == PH_RESTRICT) restrict_block<D, W, T>(t, x, y, pd, bp, ti, tv, fr); \
    else prolong_block<D, W, T>(t, x, y, pd, bp, ti, tv, fr);                        \
    break;
      switch (ph.w) {
        IGAMG_TAIL_W(1) IGAMG_TAIL_W(2) IGAMG_TAIL_W(3) IGAMG_TAIL_W(4) IGAMG_TAIL_W(5)
        IGAMG_TAIL_W(6) IGAMG_TAIL_W(7) IGAMG_TAIL_W(8) IGAMG_TAIL_W(9) IGAMG_TAIL_W(10)
        default: break;
      }
#undef IGAMG_TAIL_W
      break;
    }
    case PH_GATHER:
      gather_dist_block<T, double>(t, static_cast<const T*>(a[0]), const_cast<double*>(static_cast<const double*>(a[1])),
                                   static_cast<const int64_t*>(a[2]), static_cast<const int64_t*>(a[3]), ph.len);
      break;
    case PH_CTILES:
      coarse_tiles_block<T>(t, static_cast<const T*>(a[0]), static_cast<const double*>(a[1]),
                         const_cast<double*>(static_cast<const double*>(a[2])), ph.len);
      break;
    case PH_CREDUCE:
      coarse_reduce_block<T>(t, static_cast<const double*>(a[0]), const_cast<T*>(static_cast<const T*>(a[1])),
                             static_cast<const int64_t*>(a[2]), static_cast<const int64_t*>(a[3]), ph.len);
      break;
    default:
      break;
  }
}

constexpr unsigned TAIL_SPIN_LIMIT = 1u << 22;   // seconds of polling; a phase takes microseconds

template <int D, int P, typename T>
__global__ __launch_bounds__(256) void k_cycle_tail(const Phase* __restrict__ prog, int nph, int64_t total,
                                                    unsigned long long* __restrict__ ctr) {
  __shared__ int64_t s_ticket;
  int ph = 0, ready = 0;   // phases < ready are known complete
  for (;;) {
    if (threadIdx.x == 0) s_ticket = (int64_t)atomicAdd(&ctr[0], 1ull);
    __syncthreads();
    const int64_t t = s_ticket;
    __syncthreads();                      // s_ticket is read by every thread before it changes
    if (t >= total) break;
    while (ph + 1 < nph && t >= prog[ph + 1].first) ++ph;
    if (ph > 0 && ready < ph) {
      if (threadIdx.x == 0) {
        const unsigned long long need = (unsigned long long)prog[ph - 1].ntk;
        unsigned spins = 0;
        while (__hip_atomic_load(&ctr[ph], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins > TAIL_SPIN_LIMIT) {
            __hip_atomic_store(&ctr[1 + nph], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      __syncthreads();
      ready = ph;
    }
    const Phase& P_ = prog[ph];
    const int64_t i0 = (t - P_.first) * P_.chunk;
    const int64_t i1 = i0 + P_.chunk < P_.n ? i0 + P_.chunk : P_.n;
    for (int64_t i = i0; i < i1; ++i) {
      if (i > i0) __syncthreads();         // the item bodies reuse the LDS
      tail_item<D, P, T>(P_, i);
    }
    // every wave makes its own stores visible at agent scope before the
    // workgroup counts the ticket done
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(&ctr[1 + ph], 1ull);
  }
}

// zero the counters of one launch (a kernel, so that graphs may hold it)
__global__ __launch_bounds__(64) void k_tail_reset(unsigned long long* __restrict__ ctr, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) ctr[i] = 0ull;
}

// after the persistent launch, in stream order: a wait that exceeded its
// bound left the work list's results unordered, so the cycle's output is
// made a NaN, which the solve reports (ENAN) instead of a wrong result
template <typename T>
__global__ __launch_bounds__(64) void k_tail_check(const unsigned long long* __restrict__ ctr, int nph,
                                                   T* __restrict__ out) {
  if (threadIdx.x == 0 && ctr[1 + nph] != 0ull) out[0] = (T)NAN;
}

size_t cycle_tail_lds(int maxm, int max_dense, size_t elem) {
  return std::max({fd_slab_lds(maxm, elem), fd_dense_lds(max_dense, elem), fd_mid_lds(maxm, elem)});
}

template <typename T>
hipError_t launch_cycle_tail(int d, int p, const Phase* prog, int nph, int64_t total, unsigned long long* ctr,
                             int grid, size_t lds, T* out, hipStream_t st) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tail_reset, dim3(1), dim3(64), 0, st, ctr, nph + 2);
#define IGAMG_TAIL_CASE(DD, PP)                                                                          \
  if (d == DD && p == PP) {                                                                              \
    hipLaunchKernelGGL((k_cycle_tail<DD, PP, T>), dim3(grid), dim3(256), lds, st, prog, nph, total, ctr); \
    hipLaunchKernelGGL(k_tail_check<T>, dim3(1), dim3(64), 0, st, ctr, nph, out);                      \
    return hipGetLastError();                                                                            \
  }
  IGAMG_TAIL_CASE(2, 1) IGAMG_TAIL_CASE(2, 2) IGAMG_TAIL_CASE(2, 3) IGAMG_TAIL_CASE(2, 4)
  IGAMG_TAIL_CASE(2, 5) IGAMG_TAIL_CASE(2, 6) IGAMG_TAIL_CASE(2, 7) IGAMG_TAIL_CASE(2, 8)
  IGAMG_TAIL_CASE(3, 1) IGAMG_TAIL_CASE(3, 2) IGAMG_TAIL_CASE(3, 3) IGAMG_TAIL_CASE(3, 4)
  IGAMG_TAIL_CASE(3, 5) IGAMG_TAIL_CASE(3, 6) IGAMG_TAIL_CASE(3, 7) IGAMG_TAIL_CASE(3, 8)
#undef IGAMG_TAIL_CASE
  return hipErrorInvalidValue;
}

template hipError_t launch_cycle_tail<double>(int, int, const Phase*, int, int64_t, unsigned long long*, int, size_t,
                                              double*, hipStream_t);
template hipError_t launch_cycle_tail<float>(int, int, const Phase*, int, int64_t, unsigned long long*, int, size_t,
                                             float*, hipStream_t);

// ---------------------------------------------------------------------------
// vector kernels of the PCG loop (deterministic two-stage reductions in FP64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
  return s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_dot_partial(const T* __restrict__ a, const T* __restrict__ b, int64_t n,
                                                     double* __restrict__ part) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += (double)a[i] * (double)b[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// two dots in one pass: r.z into part[0..g) and q.z into part[g..2g)
template <typename T>
__global__ __launch_bounds__(256) void k_dot2_partial(const T* __restrict__ r, const T* __restrict__ q,
                                                      const T* __restrict__ z, int64_t n, double* __restrict__ part) {
  __shared__ double sh[4];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double zi = (double)z[i];
    s1 += (double)r[i] * zi;
    s2 += (double)q[i] * zi;
  }
  s1 = block_sum(s1, sh);
  __syncthreads();
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s1;
    part[gridDim.x + blockIdx.x] = s2;
  }
}

// flexible CG direction update: scal[3] = r.z (new rho), scal[8] = q.z,
// beta = scal[4] = -alpha (q.z) / rho_old, rho <- rho_new
__global__ __launch_bounds__(256) void k_finalize2(const double* __restrict__ part, int np, double* __restrict__ scal) {
  __shared__ double sh[4];
  double s1 = 0.0, s2 = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    s1 += part[i];
    s2 += part[np + i];
  }
  s1 = block_sum(s1, sh);
  __syncthreads();
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    scal[3] = s1;
    scal[8] = s2;
    scal[4] = -scal[2] * s2 / scal[0];
    scal[0] = s1;
  }
}

// squared norm of the accumulated version of a distributed vector.  With
// `canon`, the vector is also rewritten in canonical distributed form: the
// sum of the copies (taken in FP64) on the first copy, zero on the others.
// The copies of an interface dof carry the one-sided contributions of their
// patches, which grow large and opposite while their sum (the residual)
// shrinks; canonical form keeps the stored values at the size of the residual.
template <typename T>
__global__ __launch_bounds__(256) void k_norm2_dist_partial(T* __restrict__ r, const int64_t* __restrict__ ptr,
                                                            const int64_t* __restrict__ idx, int64_t n,
                                                            double* __restrict__ part, int canon) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c0 = ptr[g], c1 = ptr[g + 1];
    double v = 0.0;
    for (int64_t c = c0; c < c1; ++c) v += (double)r[idx[c]];
    if (canon && c1 - c0 > 1) {
      r[idx[c0]] = (T)v;
      for (int64_t c = c0 + 1; c < c1; ++c) r[idx[c]] = T(0);
    }
    s += v * v;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// scal[slot] = sum(part); then the scalar recurrence `op`:
//   0: none; 1: scal[2] = scal[0] / scal[1] (alpha = rho / pq);
//   2: scal[4] = scal[3] / scal[0], scal[0] = scal[3] (beta, rho <- rho_new)
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ part, int np, double* __restrict__ scal,
                                                  int slot, int op) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    scal[slot] = s;
    if (op == 1) scal[2] = scal[0] / scal[1];
    if (op == 2) {
      scal[4] = scal[3] / scal[0];
      scal[0] = scal[3];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_axpy2(T* __restrict__ x, const T* __restrict__ p, T* __restrict__ r,
                                               const T* __restrict__ q, int64_t n, const double* __restrict__ scal) {
  const T a = (T)scal[2];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    x[i] += a * p[i];
    r[i] -= a * q[i];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_xpby(T* __restrict__ p, const T* __restrict__ z, int64_t n,
                                              const double* __restrict__ scal) {
  const T b = (T)scal[4];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = z[i] + b * p[i];
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T* __restrict__ x, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

template <typename TS, typename TD>
__global__ __launch_bounds__(256) void k_convert(TD* __restrict__ y, const TS* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (TD)x[i];
}

__global__ __launch_bounds__(256) void k_add_f32(double* __restrict__ x, const float* __restrict__ d, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] += (double)d[i];
}

static unsigned red_grid(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(RED_BLOCKS, (n + 255) / 256));
}

template <typename T>
void launch_dot(const T* a, const T* b, int64_t n, double* part, double* scal, int slot, int op, hipStream_t st) {
  const unsigned g = red_grid(n);
  hipLaunchKernelGGL(k_dot_partial<T>, dim3(g), dim3(256), 0, st, a, b, n, part);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, part, (int)g, scal, slot, op);
}

template <typename T>
void launch_dot2_flex(const T* r, const T* q, const T* z, int64_t n, double* part, double* scal, hipStream_t st) {
  const unsigned g = red_grid(n);
  hipLaunchKernelGGL(k_dot2_partial<T>, dim3(g), dim3(256), 0, st, r, q, z, n, part);
  hipLaunchKernelGGL(k_finalize2, dim3(1), dim3(256), 0, st, part, (int)g, scal);
}

template <typename T>
void launch_norm2_dist(T* r, const int64_t* ptr, const int64_t* idx, int64_t n, double* part, double* scal, int slot,
                       bool canon, hipStream_t st) {
  const unsigned g = red_grid(n);
  hipLaunchKernelGGL(k_norm2_dist_partial<T>, dim3(g), dim3(256), 0, st, r, ptr, idx, n, part, (int)canon);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, part, (int)g, scal, slot, 0);
}

template <typename T>
void launch_axpy2(T* x, const T* p, T* r, const T* q, int64_t n, const double* scal, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy2<T>, dim3(red_grid(n)), dim3(256), 0, st, x, p, r, q, n, scal);
}

template <typename T>
void launch_xpby(T* p, const T* z, int64_t n, const double* scal, hipStream_t st) {
  hipLaunchKernelGGL(k_xpby<T>, dim3(red_grid(n)), dim3(256), 0, st, p, z, n, scal);
}

template <typename T>
void launch_fill(T* x, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill<T>, dim3(red_grid(n)), dim3(256), 0, st, x, n, (T)v);
}

template <typename T>
void launch_copy(T* y, const T* x, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_convert<T, T>), dim3(red_grid(n)), dim3(256), 0, st, y, x, n);
}

void launch_to_f32(float* y, const double* x, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_convert<double, float>), dim3(red_grid(n)), dim3(256), 0, st, y, x, n);
}

void launch_to_f64(double* y, const float* x, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_convert<float, double>), dim3(red_grid(n)), dim3(256), 0, st, y, x, n);
}

void launch_add_f32(double* x, const float* d, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_add_f32, dim3(red_grid(n)), dim3(256), 0, st, x, d, n);
}

// explicit instantiations for the two storage types
#define IGAMG_INST(T)                                                                                                  \
  template hipError_t launch_band<T>(int, int, const T*, const T*, const T*, T*, const int*, const PatchDev*, int64_t,   \
                                     bool, hipStream_t, hipEvent_t, hipEvent_t);                                       \
  template hipError_t launch_band_sym<T>(int, int, const T*, const T*, const T*, T*, const int*, const PatchDev*,        \
                                         int64_t, int64_t, T*, bool, hipStream_t, hipEvent_t, hipEvent_t);            \
  template void launch_fd_fwd<T>(const FDItem*, int, int, int, size_t, const DensePiece*, const T*, const T*,          \
                                 const T*, T*, const int64_t*, const int64_t*, T*, double, bool, int, hipStream_t);    \
  template void launch_fd_mid<T>(const FDItem*, int, int, size_t, const T*, T*, hipStream_t);                          \
  template void launch_fd_inv<T>(const FDItem*, int, int, size_t, const T*, T*, const int64_t*, const int64_t*,        \
                                 const T*, double, bool, int, hipStream_t);                                            \
  template void launch_restrict<T>(int, const T*, T*, const PatchDev*, const int*, int64_t, const int64_t*, const T*,  \
                                   int, const uint8_t*, hipStream_t);                                                  \
  template void launch_prolong_add<T>(int, const T*, T*, const PatchDev*, const int*, int64_t, const int64_t*,         \
                                      const T*, int, const uint8_t*, hipStream_t);                                     \
  template void launch_coarse<T>(const T*, const T*, double*, double*, T*, const int64_t*, const int64_t*,            \
                                 int64_t, hipStream_t);                                                                \
  template void launch_dot<T>(const T*, const T*, int64_t, double*, double*, int, int, hipStream_t);                   \
  template void launch_dot2_flex<T>(const T*, const T*, const T*, int64_t, double*, double*, hipStream_t);             \
  template void launch_norm2_dist<T>(T*, const int64_t*, const int64_t*, int64_t, double*, double*, int, bool,        \
                                     hipStream_t);                                                                     \
  template void launch_axpy2<T>(T*, const T*, T*, const T*, int64_t, const double*, hipStream_t);                      \
  template void launch_xpby<T>(T*, const T*, int64_t, const double*, hipStream_t);                                     \
  template void launch_fill<T>(T*, int64_t, double, hipStream_t);                                                      \
  template void launch_copy<T>(T*, const T*, int64_t, hipStream_t);
IGAMG_INST(double)
IGAMG_INST(float)
#undef IGAMG_INST

}  // namespace igamg
