// HIP kernels of the multigrid cycle for gfx950 (64-wide wavefronts).
//
// All level vectors are in the patch-local layout (see layout.hpp).  The
// kernels are written for one level of one problem; the cycle (Algorithm 1)
// and the PCG loop (Sec. 4) are sequenced on one stream by igamg.hip.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"
#include "layout.hpp"

namespace igamg {

// ---------------------------------------------------------------------------
// banded stiffness apply: r = f - A u  (RESID) or r = A u   (Sec. 4: A_{l,k}
// applied patch by patch to accumulated u gives a distributed result)
// ---------------------------------------------------------------------------
template <int D, int P, bool RESID, typename TB>
__global__ __launch_bounds__(256) void k_band(const TB* __restrict__ band, const double* __restrict__ u,
                                              const double* __restrict__ f, double* __restrict__ r,
                                              const int* __restrict__ bpatch, const PatchDev* __restrict__ pd,
                                              int64_t NL) {
  constexpr int NB = 2 * P + 1;
  const int b = blockIdx.x;
  const int k = bpatch[b];
  if (k < 0) return;
  const int64_t off = pd[k].off;
  const int64_t rows = pd[k].rows;
  const int64_t g = (int64_t)b * ROW_ALIGN + threadIdx.x;
  const int64_t rl = g - off;
  if (rl >= rows) return;
  const int n0 = pd[k].n[0], n1 = pd[k].n[1], n2 = pd[k].n[2];
  const int i0 = (int)(rl % n0);
  const int64_t t = rl / n0;
  const int i1 = (int)(t % n1);
  const int i2 = (int)(t / n1);
  int c0[NB], c1[NB];
#pragma unroll
  for (int o = 0; o < NB; ++o) {
    c0[o] = min(max(i0 + o - P, 0), n0 - 1);
    c1[o] = min(max(i1 + o - P, 0), n1 - 1) * n0;
  }
  const double* ub = u + off;
  // tiled coefficient-major band: this block's (2P+1)^D planes are contiguous
  constexpr int NBT = (D == 2) ? NB * NB : NB * NB * NB;
  const TB* bp = band + (int64_t)b * NBT * ROW_ALIGN + threadIdx.x;
  double s = 0.0;
  if constexpr (D == 2) {
#pragma unroll
    for (int o1 = 0; o1 < NB; ++o1) {
      const double* ur = ub + c1[o1];
#pragma unroll
      for (int o0 = 0; o0 < NB; ++o0) s += (double)bp[(o0 + NB * o1) * ROW_ALIGN] * ur[c0[o0]];
    }
  } else {
    const int64_t pl = (int64_t)n0 * n1;
    for (int o2 = 0; o2 < NB; ++o2) {
      const int64_t z = (int64_t)min(max(i2 + o2 - P, 0), n2 - 1) * pl;
#pragma unroll
      for (int o1 = 0; o1 < NB; ++o1) {
        const double* ur = ub + z + c1[o1];
        const TB* bq = bp + (NB * (o1 + NB * o2)) * ROW_ALIGN;
#pragma unroll
        for (int o0 = 0; o0 < NB; ++o0) s += (double)bq[o0 * ROW_ALIGN] * ur[c0[o0]];
      }
    }
  }
  if constexpr (RESID) r[g] = f[g] - s; else r[g] = s;
}

template <int D, int P>
static void launch_band_dp(const double* band, const double* u, const double* f, double* r, const int* bpatch,
                           const PatchDev* pd, int64_t NL, bool resid, hipStream_t st) {
  dim3 grid((unsigned)(NL / ROW_ALIGN)), block(ROW_ALIGN);
  if (resid)
    hipLaunchKernelGGL((k_band<D, P, true, double>), grid, block, 0, st, band, u, f, r, bpatch, pd, NL);
  else
    hipLaunchKernelGGL((k_band<D, P, false, double>), grid, block, 0, st, band, u, f, r, bpatch, pd, NL);
}

void launch_band(int d, int p, const double* band, const double* u, const double* f, double* r, const int* bpatch,
                 const PatchDev* pd, int64_t NL, bool resid, hipStream_t st) {
#define IGAMG_BAND_CASE(DD, PP) \
  if (d == DD && p == PP) return launch_band_dp<DD, PP>(band, u, f, r, bpatch, pd, NL, resid, st);
  IGAMG_BAND_CASE(2, 1) IGAMG_BAND_CASE(2, 2) IGAMG_BAND_CASE(2, 3) IGAMG_BAND_CASE(2, 4)
  IGAMG_BAND_CASE(2, 5) IGAMG_BAND_CASE(2, 6) IGAMG_BAND_CASE(2, 7) IGAMG_BAND_CASE(2, 8)
  IGAMG_BAND_CASE(3, 1) IGAMG_BAND_CASE(3, 2) IGAMG_BAND_CASE(3, 3) IGAMG_BAND_CASE(3, 4)
  IGAMG_BAND_CASE(3, 5) IGAMG_BAND_CASE(3, 6) IGAMG_BAND_CASE(3, 7) IGAMG_BAND_CASE(3, 8)
#undef IGAMG_BAND_CASE
}

// ---------------------------------------------------------------------------
// fast-diagonalisation pencil pass: one direction of (x)U^T, the scaled middle
// direction U diag(1/D) U^T, or one direction of (x)U, over the FD items of a
// level (used for the middle direction of 3D patch interiors)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int fd_lines_per_block(int L) { return max(1, min(64, 512 / L)); }

__global__ __launch_bounds__(256) void k_fd_pass(const FDItem* __restrict__ items, int dir, int mode, int in_sel,
                                                 int out_sel, const double* __restrict__ mat,
                                                 const double* __restrict__ src_loc,
                                                 const double* __restrict__ src_if, double* __restrict__ dst_loc,
                                                 double* __restrict__ dst_if, double* __restrict__ scrA,
                                                 double* __restrict__ scrB, double tau, int add) {
  extern __shared__ double lds[];
  const FDItem it = items[blockIdx.y];
  const int L = it.m[dir];
  const int oa = (dir == 0) ? 1 : 0;
  const int ob = (dir == 2) ? 1 : 2;
  const int ma = it.m[oa];
  const int64_t lines = (int64_t)ma * it.m[ob];
  const int LB = fd_lines_per_block(L);
  const int64_t line0 = (int64_t)blockIdx.x * LB;
  if (line0 >= lines) return;
  const int nl = (int)min((int64_t)LB, lines - line0);
  double* sU = lds;
  double* sx = lds + L * L;
  double* sy = sx + LB * L;
  const double* U = mat + it.U[dir];
  for (int i = threadIdx.x; i < L * L; i += blockDim.x) sU[i] = U[i];

  // source view
  const double* in;
  int64_t ibase, is[3];
  if (in_sel == 0) {
    in = it.src_if ? src_if : src_loc;
    ibase = it.base;
    is[0] = it.stride[0];
    is[1] = it.stride[1];
    is[2] = it.stride[2];
  } else {
    in = (in_sel == 1) ? scrA : scrB;
    ibase = it.scr;
    is[0] = 1;
    is[1] = it.m[0];
    is[2] = (int64_t)it.m[0] * it.m[1];
  }
  const int total = nl * L;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    int line, j;
    if (dir == 0) {
      line = t / L;
      j = t - line * L;
    } else {
      j = t / nl;
      line = t - j * nl;
    }
    const int64_t gl = line0 + line;
    const int64_t a = gl % ma, bq = gl / ma;
    sx[line * L + j] = in[ibase + j * is[dir] + a * is[oa] + bq * is[ob]];
  }
  __syncthreads();
  double* res;
  if (mode == 0) {  // forward: y_k = sum_j U[j,k] x_j
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
      const int line = t / L, kk = t - line * L;
      const double* x = sx + line * L;
      double s = 0.0;
      for (int j = 0; j < L; ++j) s += sU[j * L + kk] * x[j];
      sy[t] = s;
    }
    res = sy;
  } else if (mode == 1) {  // inverse: y_k = sum_j U[k,j] x_j
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
      const int line = t / L, kk = t - line * L;
      const double* x = sx + line * L;
      const double* ur = sU + kk * L;
      double s = 0.0;
      for (int j = 0; j < L; ++j) s += ur[j] * x[j];
      sy[t] = s;
    }
    res = sy;
  } else {  // middle: y = U diag(1/D) U^T x along dir
    const double* mu0 = mat + it.mu[0];
    const double* mu1 = mat + it.mu[1];
    const double* mu2 = mat + it.mu[2];
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
      const int line = t / L, kk = t - line * L;
      const double* x = sx + line * L;
      double s = 0.0;
      for (int j = 0; j < L; ++j) s += sU[j * L + kk] * x[j];
      const int64_t gl = line0 + line;
      int idx[3];
      idx[dir] = kk;
      idx[oa] = (int)(gl % ma);
      idx[ob] = (int)(gl / ma);
      const double Dv = it.pref * (mu0[idx[0]] + mu1[idx[1]] + mu2[idx[2]] + it.extra);
      sy[t] = s / Dv;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < total; t += blockDim.x) {
      const int line = t / L, kk = t - line * L;
      const double* x = sy + line * L;
      const double* ur = sU + kk * L;
      double s = 0.0;
      for (int j = 0; j < L; ++j) s += ur[j] * x[j];
      sx[t] = s;
    }
    res = sx;
  }
  __syncthreads();
  // destination view
  double* out;
  int64_t obase, os[3];
  const bool final_out = (out_sel == 0);
  if (final_out) {
    out = it.src_if ? dst_if : dst_loc;
    obase = it.base;
    os[0] = it.stride[0];
    os[1] = it.stride[1];
    os[2] = it.stride[2];
  } else {
    out = (out_sel == 1) ? scrA : scrB;
    obase = it.scr;
    os[0] = 1;
    os[1] = it.m[0];
    os[2] = (int64_t)it.m[0] * it.m[1];
  }
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    int line, j;
    if (dir == 0) {
      line = t / L;
      j = t - line * L;
    } else {
      j = t / nl;
      line = t - j * nl;
    }
    const int64_t gl = line0 + line;
    const int64_t a = gl % ma, bq = gl / ma;
    const int64_t pos = obase + j * os[dir] + a * os[oa] + bq * os[ob];
    const double v = res[line * L + j];
    if (final_out && !it.src_if) {
      out[pos] = add ? out[pos] + tau * v : tau * v;
    } else {
      out[pos] = v;
    }
  }
}

int fd_grid_x(const FDItem* items, int nitems, int dir) {
  int64_t g = 1;
  for (int i = 0; i < nitems; ++i) {
    const int L = items[i].m[dir];
    const int oa = (dir == 0) ? 1 : 0, ob = (dir == 2) ? 1 : 2;
    const int64_t lines = (int64_t)items[i].m[oa] * items[i].m[ob];
    const int LB = std::max(1, std::min(64, 512 / L));
    g = std::max(g, (lines + LB - 1) / LB);
  }
  return (int)g;
}

size_t fd_lds_bytes(int maxm) {
  // U (L x L) plus two line blocks of at most max(512, L) values each
  const size_t L = (size_t)maxm;
  return (L * L + 2 * std::max<size_t>(512, L)) * sizeof(double);
}

void launch_fd_pass(const FDItem* items, int nitems, int gridx, size_t lds, int dir, int mode, int in_sel, int out_sel,
                    const double* mat, const double* src_loc, const double* src_if, double* dst_loc, double* dst_if,
                    double* scrA, double* scrB, double tau, bool add, hipStream_t st) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(k_fd_pass, dim3(gridx, nitems), dim3(256), lds, st, items, dir, mode, in_sel, out_sel, mat,
                     src_loc, src_if, dst_loc, dst_if, scrA, scrB, tau, (int)add);
}

// ---------------------------------------------------------------------------
// smoother kernels over 2D tensors (a 2D patch interior, a 3D face, or one
// z-slab of a 3D patch interior), split into chunks of RB output rows:
//   forward:  Y[I, :] = (U0[:, I]^T X) U1     (rows I of U0^T X U1)
//   inverse:  Z[J, :] = (U0[J, :] Y) U1^T     (rows J of U0 Y U1^T)
// For 2D tensors the forward kernel applies D^{-1}; for 3D interiors the
// middle direction (with D^{-1}) runs in between as a pencil pass.  The
// forward launch also runs the dense pieces (edges, vertices).  Interface
// items gather their residual from all copies (the accumulation Sigma) and
// add tau z to every copy; interiors use the patch-local vectors directly.
// ---------------------------------------------------------------------------
constexpr int FD_RB = 8;

__device__ __forceinline__ void fd_chunk(const FDItem& it, int& z, int& r0, int& nr) {
  const int nch = (it.m[0] + FD_RB - 1) / FD_RB;
  z = blockIdx.x / nch;
  r0 = (blockIdx.x - z * nch) * FD_RB;
  nr = min(FD_RB, it.m[0] - r0);
}

__global__ __launch_bounds__(256) void k_fd_fwd(const FDItem* __restrict__ items, int nitems,
                                                const DensePiece* __restrict__ dense,
                                                const double* __restrict__ densemat, const double* __restrict__ mat,
                                                const double* __restrict__ src, double* __restrict__ u,
                                                const int64_t* __restrict__ if_ptr, const int64_t* __restrict__ if_idx,
                                                double* __restrict__ scr, double tau, int add) {
  extern __shared__ double lds[];
  const int y = blockIdx.y;
  if (y >= nitems) {
    // dense piece: gather (Sigma), z = L^{-1} r, scatter tau z to all copies
    if (blockIdx.x != 0) return;
    const DensePiece pc = dense[y - nitems];
    double* sr = lds;
    for (int j = threadIdx.x; j < pc.m; j += blockDim.x) {
      double v = 0.0;
      for (int64_t c = if_ptr[pc.seg + j]; c < if_ptr[pc.seg + j + 1]; ++c) v += src[if_idx[c]];
      sr[j] = v;
    }
    __syncthreads();
    const double* A = densemat + pc.Linv;
    for (int k = threadIdx.x; k < pc.m; k += blockDim.x) {
      double zz = 0.0;
      for (int j = 0; j < pc.m; ++j) zz += A[(int64_t)k * pc.m + j] * sr[j];
      zz *= tau;
      for (int64_t c = if_ptr[pc.seg + k]; c < if_ptr[pc.seg + k + 1]; ++c) {
        const int64_t x = if_idx[c];
        u[x] = add ? u[x] + zz : zz;
      }
    }
    return;
  }
  const FDItem it = items[y];
  const int m0 = it.m[0], m1 = it.m[1];
  int z, r0, nr;
  fd_chunk(it, z, r0, nr);
  if (z >= it.m[2]) return;
  const int n = m0 * m1;
  double* XT = lds;            // XT[j * m1 + b] = X[j, b]
  double* W = lds + n;         // W[a * m1 + b], a < RB
  const int64_t zoff = (int64_t)z * it.stride[2];
  // X[j, b] is read with j fastest (coalesced) and stored transposed
  if (it.src_if) {
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
      const int j = t % m0, b = t / m0;
      const int64_t e = it.base + t;  // face tensors are stored j fastest
      double v = 0.0;
      for (int64_t c = if_ptr[e]; c < if_ptr[e + 1]; ++c) v += src[if_idx[c]];
      XT[j * m1 + b] = v;
    }
  } else {
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
      const int j = t % m0, b = t / m0;
      XT[j * m1 + b] = src[it.base + j * it.stride[0] + b * it.stride[1] + zoff];
    }
  }
  __syncthreads();
  const double* U0 = mat + it.U[0];
  const double* U1 = mat + it.U[1];
  // W[a, b] = sum_j U0[j, r0 + a] X[j, b]
  for (int t = threadIdx.x; t < nr * m1; t += blockDim.x) {
    const int b = t % m1, a = t / m1;
    double s = 0.0;
    for (int j = 0; j < m0; ++j) s += U0[j * m0 + r0 + a] * XT[j * m1 + b];
    W[a * m1 + b] = s;
  }
  __syncthreads();
  // Y[a, k] = sum_b W[a, b] U1[b, k]
  const double* mu0 = mat + it.mu[0];
  const double* mu1 = mat + it.mu[1];
  const double mu2 = mat[it.mu[2]];
  const bool full = (it.m[2] == 1);
  double* S = scr + it.scr + (int64_t)z * n;
  for (int t = threadIdx.x; t < nr * m1; t += blockDim.x) {
    const int k = t % m1, a = t / m1;
    const double* w = W + a * m1;
    double s = 0.0;
    for (int b = 0; b < m1; ++b) s += w[b] * U1[b * m1 + k];
    if (full) s /= it.pref * (mu0[r0 + a] + mu1[k] + mu2 + it.extra);
    S[(r0 + a) + m0 * k] = s;
  }
}

__global__ __launch_bounds__(256) void k_fd_inv(const FDItem* __restrict__ items, const double* __restrict__ mat,
                                                double* __restrict__ u, const int64_t* __restrict__ if_ptr,
                                                const int64_t* __restrict__ if_idx, const double* __restrict__ scr,
                                                double tau, int add) {
  extern __shared__ double lds[];
  const FDItem it = items[blockIdx.y];
  const int m0 = it.m[0], m1 = it.m[1];
  int z, r0, nr;
  fd_chunk(it, z, r0, nr);
  if (z >= it.m[2]) return;
  const int n = m0 * m1;
  double* YT = lds;      // YT[j * m1 + b] = Y[j, b]
  double* W = lds + n;   // W[a * m1 + b]
  const double* S = scr + it.scr + (int64_t)z * n;
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    const int j = t % m0, b = t / m0;
    YT[j * m1 + b] = S[t];
  }
  __syncthreads();
  const double* U0 = mat + it.U[0];
  const double* U1T = mat + it.U[1] + (int64_t)m1 * m1;
  // W[a, b] = sum_j U0[r0 + a, j] Y[j, b]
  for (int t = threadIdx.x; t < nr * m1; t += blockDim.x) {
    const int b = t % m1, a = t / m1;
    const double* ur = U0 + (int64_t)(r0 + a) * m0;
    double s = 0.0;
    for (int j = 0; j < m0; ++j) s += ur[j] * YT[j * m1 + b];
    W[a * m1 + b] = s;
  }
  __syncthreads();
  // Z[a, k] = sum_b W[a, b] U1[k, b] = sum_b W[a, b] U1T[b, k]
  const int64_t zoff = (int64_t)z * it.stride[2];
  for (int t = threadIdx.x; t < nr * m1; t += blockDim.x) {
    const int k = t % m1, a = t / m1;
    const double* w = W + a * m1;
    double s = 0.0;
    for (int b = 0; b < m1; ++b) s += w[b] * U1T[b * m1 + k];
    const double v = tau * s;
    if (it.src_if) {
      const int64_t e = it.base + (r0 + a) + (int64_t)m0 * k;
      for (int64_t c = if_ptr[e]; c < if_ptr[e + 1]; ++c) {
        const int64_t x = if_idx[c];
        u[x] = add ? u[x] + v : v;
      }
    } else {
      const int64_t x = it.base + (r0 + a) * it.stride[0] + k * it.stride[1] + zoff;
      u[x] = add ? u[x] + v : v;
    }
  }
}

size_t fd_slab_lds(int maxm) { return ((size_t)maxm * maxm + (size_t)FD_RB * maxm) * sizeof(double) + 64; }

int fd_slab_grid(const FDItem* items, int nitems) {
  int g = 1;
  for (int i = 0; i < nitems; ++i) g = std::max(g, items[i].m[2] * ((items[i].m[0] + FD_RB - 1) / FD_RB));
  return g;
}

void launch_fd_fwd(const FDItem* items, int nitems, int ndense, int gridx, size_t lds, const DensePiece* dense,
                   const double* densemat, const double* mat, const double* src, double* u, const int64_t* if_ptr,
                   const int64_t* if_idx, double* scr, double tau, bool add, hipStream_t st) {
  const int ny = nitems + ndense;
  if (ny <= 0) return;
  hipLaunchKernelGGL(k_fd_fwd, dim3(gridx, ny), dim3(256), lds, st, items, nitems, dense, densemat, mat, src, u,
                     if_ptr, if_idx, scr, tau, (int)add);
}

void launch_fd_inv(const FDItem* items, int nitems, int gridx, size_t lds, const double* mat, double* u,
                   const int64_t* if_ptr, const int64_t* if_idx, const double* scr, double tau, bool add,
                   hipStream_t st) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(k_fd_inv, dim3(gridx, nitems), dim3(256), lds, st, items, mat, u, if_ptr, if_idx, scr, tau,
                     (int)add);
}

// ---------------------------------------------------------------------------
// transfers (Sec. 3: P_l and P_l^T, per patch as a Kronecker product of the
// univariate knot-insertion matrices; Sec. 4: P maps accumulated to
// accumulated, P^T distributed to distributed vectors)
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_restrict(const double* __restrict__ rf, double* __restrict__ rc,
                                                  const PatchDev* __restrict__ pd, const int* __restrict__ bpatch_c,
                                                  const int64_t* __restrict__ tidx, const double* __restrict__ tval,
                                                  int WR, const uint8_t* __restrict__ isfree_c) {
  const int b = blockIdx.x;
  const int k = bpatch_c[b];
  if (k < 0) return;
  const PatchDev& P = pd[k];
  const int64_t g = (int64_t)b * ROW_ALIGN + threadIdx.x;
  const int64_t rl = g - P.offc;
  if (rl >= P.rowsc) return;
  if (!isfree_c[g]) {
    rc[g] = 0.0;
    return;
  }
  const int j0 = (int)(rl % P.nc[0]);
  const int64_t t = rl / P.nc[0];
  const int j1 = (int)(t % P.nc[1]);
  const int j2 = (int)(t / P.nc[1]);
  const int s0 = (int)tidx[P.Rst[0] + j0], s1 = (int)tidx[P.Rst[1] + j1], s2 = (int)tidx[P.Rst[2] + j2];
  const double* w0 = tval + P.Rval[0] + (int64_t)j0 * WR;
  const double* w1 = tval + P.Rval[1] + (int64_t)j1 * WR;
  const double* w2 = tval + P.Rval[2] + (int64_t)j2 * WR;
  const int n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
  const double* src = rf + P.off;
  double s = 0.0;
  const int W2 = (D == 3) ? WR : 1;
  for (int a2 = 0; a2 < W2; ++a2) {
    const double c2 = w2[a2];
    if (c2 == 0.0) continue;
    const int64_t z = (int64_t)min(s2 + a2, n2 - 1) * n0 * n1;
    for (int a1 = 0; a1 < WR; ++a1) {
      const double c1 = w1[a1] * c2;
      if (c1 == 0.0) continue;
      const double* row = src + z + (int64_t)min(s1 + a1, n1 - 1) * n0;
      double acc = 0.0;
      for (int a0 = 0; a0 < WR; ++a0) acc += w0[a0] * row[min(s0 + a0, n0 - 1)];
      s += c1 * acc;
    }
  }
  rc[g] = s;
}

template <int D>
__global__ __launch_bounds__(256) void k_prolong_add(const double* __restrict__ uc, double* __restrict__ uf,
                                                     const PatchDev* __restrict__ pd,
                                                     const int* __restrict__ bpatch_f,
                                                     const int64_t* __restrict__ tidx,
                                                     const double* __restrict__ tval, int WP,
                                                     const uint8_t* __restrict__ isfree_f) {
  const int b = blockIdx.x;
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
  const double* w0 = tval + P.Pval[0] + (int64_t)i0 * WP;
  const double* w1 = tval + P.Pval[1] + (int64_t)i1 * WP;
  const double* w2 = tval + P.Pval[2] + (int64_t)i2 * WP;
  const int n0 = P.nc[0], n1 = P.nc[1], n2 = P.nc[2];
  const double* src = uc + P.offc;
  double s = 0.0;
  const int W2 = (D == 3) ? WP : 1;
  for (int a2 = 0; a2 < W2; ++a2) {
    const double c2 = w2[a2];
    if (c2 == 0.0) continue;
    const int64_t z = (int64_t)min(s2 + a2, n2 - 1) * n0 * n1;
    for (int a1 = 0; a1 < WP; ++a1) {
      const double c1 = w1[a1] * c2;
      if (c1 == 0.0) continue;
      const double* row = src + z + (int64_t)min(s1 + a1, n1 - 1) * n0;
      double acc = 0.0;
      for (int a0 = 0; a0 < WP; ++a0) acc += w0[a0] * row[min(s0 + a0, n0 - 1)];
      s += c1 * acc;
    }
  }
  uf[g] += s;
}

void launch_restrict(int d, const double* rf, double* rc, const PatchDev* pd, const int* bpatch_c, int64_t NLc,
                     const int64_t* tidx, const double* tval, int WR, const uint8_t* isfree_c, hipStream_t st) {
  dim3 grid((unsigned)(NLc / ROW_ALIGN)), block(ROW_ALIGN);
  if (d == 2)
    hipLaunchKernelGGL(k_restrict<2>, grid, block, 0, st, rf, rc, pd, bpatch_c, tidx, tval, WR, isfree_c);
  else
    hipLaunchKernelGGL(k_restrict<3>, grid, block, 0, st, rf, rc, pd, bpatch_c, tidx, tval, WR, isfree_c);
}

void launch_prolong_add(int d, const double* uc, double* uf, const PatchDev* pd, const int* bpatch_f, int64_t NLf,
                        const int64_t* tidx, const double* tval, int WP, const uint8_t* isfree_f, hipStream_t st) {
  dim3 grid((unsigned)(NLf / ROW_ALIGN)), block(ROW_ALIGN);
  if (d == 2)
    hipLaunchKernelGGL(k_prolong_add<2>, grid, block, 0, st, uc, uf, pd, bpatch_f, tidx, tval, WP, isfree_f);
  else
    hipLaunchKernelGGL(k_prolong_add<3>, grid, block, 0, st, uc, uf, pd, bpatch_f, tidx, tval, WP, isfree_f);
}

// ---------------------------------------------------------------------------
// coarse solve (Sec. 4, chi A_0^{-1} Sigma_glob): b = sum of copies,
// y = W b, x = W^T y with W = L^{-1}, A_0 = L L^T; x to every copy
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gather_dist(const double* __restrict__ loc, double* __restrict__ glob,
                                                     const int64_t* __restrict__ ptr,
                                                     const int64_t* __restrict__ idx, int64_t n) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  double s = 0.0;
  for (int64_t c = ptr[g]; c < ptr[g + 1]; ++c) s += loc[idx[c]];
  glob[g] = s;
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
    hipLaunchKernelGGL(k_gather_dist, grid, dim3(256), 0, st, loc, glob, ptr, idx, n);
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

// x = A_0^{-1} b (dense, n x n row-major), one wavefront per row; x_i goes to
// every local copy of coarse dof i (the restriction chi of the coarse solve)
__global__ __launch_bounds__(256) void k_coarse_gemv(const double* __restrict__ Ainv, const double* __restrict__ b,
                                                     double* __restrict__ u0, const int64_t* __restrict__ ptr,
                                                     const int64_t* __restrict__ idx, int n) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const double* ar = Ainv + (int64_t)row * n;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += ar[j] * b[j];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  const int64_t c0 = ptr[row], c1 = ptr[row + 1];
  s = __shfl(s, 0, 64);
  for (int64_t c = c0 + lane; c < c1; c += 64) u0[idx[c]] = s;
}

void launch_coarse(const double* Ainv, const double* b, double* u0, const int64_t* ptr, const int64_t* idx, int n,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_coarse_gemv, dim3((n + 3) / 4), dim3(256), 0, st, Ainv, b, u0, ptr, idx, n);
}

// ---------------------------------------------------------------------------
// vector kernels of the PCG loop (deterministic two-stage reductions)
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

__global__ __launch_bounds__(256) void k_dot_partial(const double* __restrict__ a, const double* __restrict__ b,
                                                     int64_t n, double* __restrict__ part) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += a[i] * b[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// squared norm of the accumulated version of a distributed vector
__global__ __launch_bounds__(256) void k_norm2_dist_partial(const double* __restrict__ r,
                                                            const int64_t* __restrict__ ptr,
                                                            const int64_t* __restrict__ idx, int64_t n,
                                                            double* __restrict__ part) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int64_t c = ptr[g]; c < ptr[g + 1]; ++c) v += r[idx[c]];
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

__global__ __launch_bounds__(256) void k_axpy2(double* __restrict__ x, const double* __restrict__ p,
                                               double* __restrict__ r, const double* __restrict__ q, int64_t n,
                                               const double* __restrict__ scal) {
  const double a = scal[2];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    x[i] += a * p[i];
    r[i] -= a * q[i];
  }
}

__global__ __launch_bounds__(256) void k_xpby(double* __restrict__ p, const double* __restrict__ z, int64_t n,
                                              const double* __restrict__ scal) {
  const double b = scal[4];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = z[i] + b * p[i];
}

__global__ __launch_bounds__(256) void k_fill(double* __restrict__ x, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

__global__ __launch_bounds__(256) void k_copy(double* __restrict__ y, const double* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i];
}

static unsigned red_grid(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(RED_BLOCKS, (n + 255) / 256)); }

void launch_dot(const double* a, const double* b, int64_t n, double* part, double* scal, int slot, int op,
                hipStream_t st) {
  const unsigned g = red_grid(n);
  hipLaunchKernelGGL(k_dot_partial, dim3(g), dim3(256), 0, st, a, b, n, part);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, part, (int)g, scal, slot, op);
}

void launch_norm2_dist(const double* r, const int64_t* ptr, const int64_t* idx, int64_t n, double* part, double* scal,
                       int slot, hipStream_t st) {
  const unsigned g = red_grid(n);
  hipLaunchKernelGGL(k_norm2_dist_partial, dim3(g), dim3(256), 0, st, r, ptr, idx, n, part);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, part, (int)g, scal, slot, 0);
}

void launch_axpy2(double* x, const double* p, double* r, const double* q, int64_t n, const double* scal,
                  hipStream_t st) {
  hipLaunchKernelGGL(k_axpy2, dim3(red_grid(n)), dim3(256), 0, st, x, p, r, q, n, scal);
}

void launch_xpby(double* p, const double* z, int64_t n, const double* scal, hipStream_t st) {
  hipLaunchKernelGGL(k_xpby, dim3(red_grid(n)), dim3(256), 0, st, p, z, n, scal);
}

void launch_fill(double* x, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(red_grid(n)), dim3(256), 0, st, x, n, v);
}

void launch_copy(double* y, const double* x, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_copy, dim3(red_grid(n)), dim3(256), 0, st, y, x, n);
}

}  // namespace igamg
