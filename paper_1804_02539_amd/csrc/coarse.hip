// The exact coarse solver's setup on the device (Sec. 4: the coarsest level
// is solved exactly, with a direct factorization of the dense A_0): the
// Cholesky factorization A_0 = L L^T, the inverse factor Y = L^{-1}, and the
// inverse A_0^{-1} = Y^T Y, all on packed lower 64 x 64 tiles (layout.hpp).
//
// Every step is a tiled right-looking sweep with one tile product per
// workgroup and launch, so that a launch has as many independent tiles as
// the step allows and no workgroup carries a long chain of products:
//   factor   for k:  L_kk = chol(A_kk) and W_kk = L_kk^{-1} (one workgroup),
//                    L_ik = A_ik W_kk^T                      (i > k),
//                    A_ij -= L_ik L_jk^T                     (k < j <= i);
//   inverse  Y_kk = W_kk; for k: Y_kj = -W_kk S_kj (j < k), then
//                    S_ij += L_ik Y_kj  (i > k, j <= k)  and
//                    X_ij += Y_ki^T Y_kj (j <= i <= k), X = A_0^{-1}.
// S_ij accumulates in Y's tile (i, j) until row i is final.  The sums run in
// a fixed order, so the result is deterministic.  2/3 n^3 + O(n^2 64) FLOP in
// FP64; no allocation and no library call.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"
#include "layout.hpp"

namespace igamg {

namespace {

constexpr int CT = COARSE_TILE;
constexpr int KH = 32;        // depth of one LDS stage of a tile product
constexpr int LDK = CT + 4;   // LDS row length (doubles) of a staged operand

__device__ __forceinline__ void tri_pair(int64_t t, int64_t& a, int64_t& b) {
  int64_t x = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (x * (x + 1) / 2 > t) --x;
  while ((x + 1) * (x + 2) / 2 <= t) ++x;
  a = x;
  b = t - x * (x + 1) / 2;
}

// acc += op(A) op(B) for 64 x 64 row-major tiles in global memory, op the
// transpose when TA / TB.  256 threads; thread (ty, tx) = (tid / 16, tid % 16)
// owns rows 4 ty .. 4 ty + 3 and columns 4 tx .. 4 tx + 3 of the product.
// The operands pass through LDS in two stages of 32 along the inner index,
// stored inner-index-major (As[k][row], Bs[k][col]) so that a thread reads
// its four rows and four columns as contiguous pairs.
template <bool TA, bool TB>
__device__ __forceinline__ void tile_mac(const double* __restrict__ A, const double* __restrict__ B,
                                         double (&acc)[4][4], double* __restrict__ As, double* __restrict__ Bs) {
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  for (int k0 = 0; k0 < CT; k0 += KH) {
    __syncthreads();   // the previous stage (or caller's use of LDS) is done
#pragma unroll
    for (int it = 0; it < CT * KH / 256; ++it) {
      const int e = it * 256 + tid;
      if (TA) {   // op(A)[row][k] = A[k][row]: read along row
        const int kk = e / CT, row = e % CT;
        As[kk * LDK + row] = A[(k0 + kk) * CT + row];
      } else {    // op(A)[row][k] = A[row][k]: read along k
        const int row = e / KH, kk = e % KH;
        As[kk * LDK + row] = A[row * CT + k0 + kk];
      }
      if (TB) {   // op(B)[k][col] = B[col][k]: read along k
        const int col = e / KH, kk = e % KH;
        Bs[kk * LDK + col] = B[col * CT + k0 + kk];
      } else {    // op(B)[k][col] = B[k][col]: read along col
        const int kk = e / CT, col = e % CT;
        Bs[kk * LDK + col] = B[(k0 + kk) * CT + col];
      }
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < KH; ++kk) {
      const double2 a01 = *reinterpret_cast<const double2*>(&As[kk * LDK + 4 * ty]);
      const double2 a23 = *reinterpret_cast<const double2*>(&As[kk * LDK + 4 * ty + 2]);
      const double2 b01 = *reinterpret_cast<const double2*>(&Bs[kk * LDK + 4 * tx]);
      const double2 b23 = *reinterpret_cast<const double2*>(&Bs[kk * LDK + 4 * tx + 2]);
      const double a[4] = {a01.x, a01.y, a23.x, a23.y};
      const double b[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
  }
  __syncthreads();   // every operand read is done: the caller may overwrite A or B
}

__device__ __forceinline__ void acc_zero(double (&acc)[4][4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
}

// C = s * acc (ADD: C += s * acc) for a tile C in global memory
template <bool ADD>
__device__ __forceinline__ void acc_store(double* __restrict__ C, const double (&acc)[4][4], double s) {
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double* c = C + (4 * ty + i) * CT + 4 * tx;
    double2 lo = {s * acc[i][0], s * acc[i][1]}, hi = {s * acc[i][2], s * acc[i][3]};
    if (ADD) {
      const double2 o0 = *reinterpret_cast<const double2*>(c), o1 = *reinterpret_cast<const double2*>(c + 2);
      lo.x += o0.x;
      lo.y += o0.y;
      hi.x += o1.x;
      hi.y += o1.y;
    }
    *reinterpret_cast<double2*>(c) = lo;
    *reinterpret_cast<double2*>(c + 2) = hi;
  }
}

#define IGAMG_TILE_LDS                         \
  __shared__ __align__(16) double As[KH * LDK]; \
  __shared__ __align__(16) double Bs[KH * LDK];

// Cholesky factor of diagonal tile k and its inverse, in LDS: the factor by
// columns (scale the column below the pivot, update the trailing lower part),
// then the inverse W by forward substitution against I, one column c per
// thread.  W's strict lower part is kept transposed in the strict upper part
// of the same array (thread c writes row c there, which no other thread
// reads) and its diagonal 1 / L_cc apart.
__global__ __launch_bounds__(256) void k_chol_diag(double* __restrict__ Lt, double* __restrict__ Yt, int64_t k,
                                                   int* __restrict__ info) {
  __shared__ double a[CT][CT + 1];
  __shared__ double wd[CT];
  __shared__ int fail;
  const int tid = threadIdx.x;
  double* src = Lt + coarse_tile_at(k, k);
  for (int e = tid; e < CT * CT; e += 256) a[e / CT][e % CT] = src[e];
  if (tid == 0) fail = 0;
  for (int j = 0; j < CT; ++j) {
    __syncthreads();
    double d = a[j][j];
    if (!(d > 0.0) || !(d < HUGE_VAL)) {
      if (tid == 0 && fail == 0) fail = j + 1;
      d = 1.0;
    }
    const double l = sqrt(d);
    __syncthreads();   // every thread has read the pivot
    if (tid == 0) a[j][j] = l;
    if (tid > j && tid < CT) a[tid][j] = a[tid][j] / l;
    __syncthreads();
    for (int e = tid; e < CT * CT; e += 256) {
      const int i = e / CT, c = e % CT;
      if (c > j && c <= i) a[i][c] = fma(-a[i][j], a[c][j], a[i][c]);
    }
  }
  __syncthreads();
  if (tid < CT) {
    const int c = tid;
    const double dc = 1.0 / a[c][c];
    wd[c] = dc;
    // w[r][c] = -(sum_{m = c}^{r - 1} L[r][m] w[m][c]) / L[r][r] for r > c,
    // with w[c][c] = dc and w[m][c] (m > c) at a[c][m]
    for (int r = 1; r < CT; ++r) {
      if (r <= c) continue;
      double s = -a[r][c] * dc;
      for (int m = c + 1; m < r; ++m) s = fma(-a[r][m], a[c][m], s);
      a[c][r] = s / a[r][r];
    }
  }
  __syncthreads();
  double* y = Yt + coarse_tile_at(k, k);
  for (int e = tid; e < CT * CT; e += 256) {
    const int i = e / CT, c = e % CT;
    src[e] = c < i ? a[i][c] : (c == i ? a[i][i] : 0.0);
    y[e] = c < i ? a[c][i] : (c == i ? wd[i] : 0.0);
  }
  if (tid == 0 && fail != 0 && *info == 0) *info = (int)(k * CT + fail);
}

// L_ik = A_ik W_kk^T for i = k + 1 + blockIdx.x
__global__ __launch_bounds__(256) void k_chol_panel(double* __restrict__ Lt, const double* __restrict__ Yt,
                                                    int64_t k) {
  IGAMG_TILE_LDS
  const int64_t i = k + 1 + blockIdx.x;
  double acc[4][4];
  acc_zero(acc);
  double* Aik = Lt + coarse_tile_at(i, k);
  tile_mac<false, true>(Aik, Yt + coarse_tile_at(k, k), acc, As, Bs);
  acc_store<false>(Aik, acc, 1.0);
}

// A_ij -= L_ik L_jk^T for the pair (i, j) = k + 1 + (a, b) of blockIdx.x
__global__ __launch_bounds__(256) void k_chol_update(double* __restrict__ Lt, int64_t k) {
  IGAMG_TILE_LDS
  int64_t a, b;
  tri_pair(blockIdx.x, a, b);
  const int64_t i = k + 1 + a, j = k + 1 + b;
  double acc[4][4];
  acc_zero(acc);
  tile_mac<false, true>(Lt + coarse_tile_at(i, k), Lt + coarse_tile_at(j, k), acc, As, Bs);
  acc_store<true>(Lt + coarse_tile_at(i, j), acc, -1.0);
}

// row k of Y: Y_kj = -W_kk S_kj for j = blockIdx.x < k (in place)
__global__ __launch_bounds__(256) void k_inv_row(double* __restrict__ Yt, int64_t k) {
  IGAMG_TILE_LDS
  double* S = Yt + coarse_tile_at(k, blockIdx.x);
  double acc[4][4];
  acc_zero(acc);
  tile_mac<false, false>(Yt + coarse_tile_at(k, k), S, acc, As, Bs);
  acc_store<false>(S, acc, -1.0);
}

// with row k of Y final: the first nU workgroups add L_ik Y_kj to S_ij
// (i > k, j <= k), the others Y_ki^T Y_kj to X_ij (j <= i <= k)
__global__ __launch_bounds__(256) void k_inv_update(const double* __restrict__ Lt, double* __restrict__ Yt,
                                                    double* __restrict__ X, int64_t k, int64_t nU) {
  IGAMG_TILE_LDS
  double acc[4][4];
  acc_zero(acc);
  const int64_t t = blockIdx.x;
  if (t < nU) {
    const int64_t i = k + 1 + t / (k + 1), j = t % (k + 1);
    tile_mac<false, false>(Lt + coarse_tile_at(i, k), Yt + coarse_tile_at(k, j), acc, As, Bs);
    acc_store<true>(Yt + coarse_tile_at(i, j), acc, 1.0);
  } else {
    int64_t i, j;
    tri_pair(t - nU, i, j);
    tile_mac<true, false>(Yt + coarse_tile_at(k, i), Yt + coarse_tile_at(k, j), acc, As, Bs);
    acc_store<true>(X + coarse_tile_at(i, j), acc, 1.0);
  }
}

}  // namespace

void coarse_inverse(double* Lt, double* Yt, double* Ainv, int64_t n, int* info, hipStream_t st) {
  const int64_t T = coarse_tiles(n);
  for (int64_t k = 0; k < T; ++k) {
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, st, Lt, Yt, k, info);
    const int64_t m = T - k - 1;
    if (m > 0) {
      hipLaunchKernelGGL(k_chol_panel, dim3((unsigned)m), dim3(256), 0, st, Lt, Yt, k);
      hipLaunchKernelGGL(k_chol_update, dim3((unsigned)(m * (m + 1) / 2)), dim3(256), 0, st, Lt, k);
    }
  }
  for (int64_t k = 0; k < T; ++k) {
    if (k > 0) hipLaunchKernelGGL(k_inv_row, dim3((unsigned)k), dim3(256), 0, st, Yt, k);
    const int64_t nU = (T - k - 1) * (k + 1), nX = (k + 1) * (k + 2) / 2;
    hipLaunchKernelGGL(k_inv_update, dim3((unsigned)(nU + nX)), dim3(256), 0, st, Lt, Yt, Ainv, k, nU);
  }
}

}  // namespace igamg
