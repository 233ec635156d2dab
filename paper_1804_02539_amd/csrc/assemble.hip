// Device assembly of the banded patch matrices A_{l,k} (Sec. 4):
//
//   A_k[i][j] = sum over Gauss points x of w(x) grad B_i(x)^T C(x) grad B_j(x),
//   C = |det J| J^{-1} J^{-T}, J the Jacobian of the patch's Bezier map,
//
// with p+1 Gauss points per element and direction.  The tensor-product rule
// is contracted one direction at a time (sum factorisation), one element slab
// of direction 2 at a time:
//   metric  Gs[ab][q2][q1][q0]        = w C_ab at the slab's points
//   dir 0   T1[ab][q2][q1][o0][i0]     = sum_q0 Gs[ab] F0^{a==0}_{i0} F0^{b==0}_{j0}
//   dir 1   T2[g][q2][i1][o1][o0][i0]  = sum_{(a,b) in g} sum_q1 F1^{a==1}_{i1} F1^{b==1}_{j1} T1[ab]
//   dir 2   band[(i0,i1,i2)][(o0,o1,o2)] += sum_g sum_q2 F2^{s}_{i2} F2^{t}_{j2} T2[g]
// where F^1 is the derivative and F^0 the value of a 1D basis function, j =
// i + o - p, and g groups the (a, b) pairs by their direction-2 flags
// (s, t) = (a == 2, b == 2).  Every output entry is owned by one thread, the
// slabs of a patch are ordered on the stream, and i0 is the fastest index of
// every intermediate, so all stages read and write coalesced and the last one
// writes whole rows of the tiled band
// band[(row/256)*nb*256 + o*256 + row%256].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "assemble_stages.hpp"
#include "kernels.hpp"

namespace igamg {

namespace {

// one thread per item; the per-slab stages stay far below the 2^32 work-items
// of a dispatch (the largest slab of a 48^3-element p=8 patch has about 2.6e8
// direction-2 threads), and launch_slab checks it
inline dim3 grid_for(int64_t tot) { return dim3((unsigned)((tot + 255) / 256)); }
constexpr int64_t MAX_DISPATCH_ITEMS = ((int64_t)1 << 32) - 256;

// grid-stride launches cap their grid at this many workgroups
constexpr int64_t STRIDE_BLOCKS = (int64_t)1 << 20;

template <int D>
__global__ __launch_bounds__(256) void k_asm_metric(AsmPatch P, const double* __restrict__ tab, int e2,
                                                    double* __restrict__ Gs, int* __restrict__ flag) {
  const int64_t tot = (int64_t)P.nq[2] * P.nel[1] * P.nq[1] * P.nel[0] * P.nq[0];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = t < tot;
  const double det = valid ? asm_metric_point<D>(P, tab, e2, t, Gs) : 1.0;
  // the sign of det J over the patch, one atomic per wave: bit 0 positive,
  // bit 1 negative, bit 2 zero or not a number
  const unsigned long long pos = __ballot(valid && det > 0.0);
  const unsigned long long neg = __ballot(valid && det < 0.0);
  const unsigned long long bad = __ballot(valid && !(det > 0.0 || det < 0.0));
  if ((threadIdx.x & 63) == 0) {
    const int f = (pos ? 1 : 0) | (neg ? 2 : 0) | (bad ? 4 : 0);
    if (f) atomicOr(flag, f);
  }
}

template <int D, int P>
__global__ __launch_bounds__(256) void k_asm_dir0(AsmPatch Pt, const double* __restrict__ tab,
                                                  const double* __restrict__ Gs, double* __restrict__ T1,
                                                  int64_t tot) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < tot) asm_dir0_row<D, P>(Pt, tab, Gs, T1, t);
}

template <int D, int P>
__global__ __launch_bounds__(256) void k_asm_dir1(AsmPatch Pt, const double* __restrict__ tab,
                                                  const double* __restrict__ T1, double* __restrict__ T2,
                                                  int64_t tot) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < tot) asm_dir1_row<D, P>(Pt, tab, T1, T2, t);
}

template <int D, int P2>
__global__ __launch_bounds__(256) void k_asm_dir2(AsmPatch P, const double* __restrict__ tab, int e2,
                                                  const double* __restrict__ T2, double* __restrict__ band, int nbt,
                                                  int64_t tot) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < tot) asm_dir2_entry<D, P2>(P, tab, e2, T2, band, nbt, t);
}

template <int D>
__global__ __launch_bounds__(256) void k_asm_mask(const PatchDev* __restrict__ pd, const int* __restrict__ bpatch,
                                                  const uint8_t* __restrict__ isfree, double* __restrict__ band,
                                                  int nbt, int p, int64_t tot) {
  // grid-stride: a whole level's band can hold more than 2^32 entries
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += stride)
    asm_mask_entry<D>(pd, bpatch, isfree, band, nbt, p, t);
}

// the four launches of one slab; the direction-2 stage has degree P in 3D
// and none in 2D
template <int D, int P>
hipError_t launch_slab(const AsmPatch& Pt, const double* tab, int e2, double* Gs, double* T1, double* T2,
                       double* band, int nbt, int* flag, hipStream_t st) {
  constexpr int P2 = (D == 3) ? P : 0;
  size_t sz[3];
  asm_sizes(D, Pt, sz);
  const int64_t t0 = asm_dir0_threads(D, Pt), t1 = asm_dir1_threads(D, Pt), t2 = asm_dir2_threads(Pt);
  if ((int64_t)sz[0] / (D * D) > MAX_DISPATCH_ITEMS || t0 > MAX_DISPATCH_ITEMS || t1 > MAX_DISPATCH_ITEMS ||
      t2 > MAX_DISPATCH_ITEMS)
    return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(k_asm_metric<D>, grid_for((int64_t)sz[0] / (D * D)), dim3(256), 0, st, Pt, tab, e2, Gs, flag);
  hipLaunchKernelGGL((k_asm_dir0<D, P>), grid_for(t0), dim3(256), 0, st, Pt, tab, Gs, T1, t0);
  hipLaunchKernelGGL((k_asm_dir1<D, P>), grid_for(t1), dim3(256), 0, st, Pt, tab, T1, T2, t1);
  hipLaunchKernelGGL((k_asm_dir2<D, P2>), grid_for(t2), dim3(256), 0, st, Pt, tab, e2, T2, band, nbt, t2);
  return hipSuccess;
}

template <int D>
hipError_t launch_slab_d(const AsmPatch& Pt, const double* tab, int e2, double* Gs, double* T1, double* T2,
                         double* band, int nbt, int* flag, hipStream_t st) {
  hipError_t e = hipSuccess;
  switch (Pt.pc[0]) {
    case 1: e = launch_slab<D, 1>(Pt, tab, e2, Gs, T1, T2, band, nbt, flag, st); break;
    case 2: e = launch_slab<D, 2>(Pt, tab, e2, Gs, T1, T2, band, nbt, flag, st); break;
    case 3: e = launch_slab<D, 3>(Pt, tab, e2, Gs, T1, T2, band, nbt, flag, st); break;
    case 4: e = launch_slab<D, 4>(Pt, tab, e2, Gs, T1, T2, band, nbt, flag, st); break;
    case 5: e = launch_slab<D, 5>(Pt, tab, e2, Gs, T1, T2, band, nbt, flag, st); break;
    case 6: e = launch_slab<D, 6>(Pt, tab, e2, Gs, T1, T2, band, nbt, flag, st); break;
    case 7: e = launch_slab<D, 7>(Pt, tab, e2, Gs, T1, T2, band, nbt, flag, st); break;
    case 8: e = launch_slab<D, 8>(Pt, tab, e2, Gs, T1, T2, band, nbt, flag, st); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace

void asm_slab_sizes(int d, const AsmPatch& P, size_t out[3]) { asm_sizes(d, P, out); }

hipError_t launch_asm_slab(int d, const AsmPatch& P, const double* tab, int e2, double* Gs, double* T1, double* T2,
                           double* band, int nbt, int* flag, hipStream_t st) {
  if (d == 2) return launch_slab_d<2>(P, tab, e2, Gs, T1, T2, band, nbt, flag, st);
  if (d == 3) return launch_slab_d<3>(P, tab, e2, Gs, T1, T2, band, nbt, flag, st);
  return hipErrorInvalidValue;
}

void launch_asm_mask(int d, int p, const PatchDev* pd, const int* bpatch, const uint8_t* isfree, double* band,
                     int nbt, int64_t NL, hipStream_t st) {
  const int64_t tot = NL * nbt;
  if (tot <= 0) return;
  const dim3 grid((unsigned)std::min<int64_t>((tot + 255) / 256, STRIDE_BLOCKS));
  if (d == 2)
    hipLaunchKernelGGL(k_asm_mask<2>, grid, dim3(256), 0, st, pd, bpatch, isfree, band, nbt, p, tot);
  else
    hipLaunchKernelGGL(k_asm_mask<3>, grid, dim3(256), 0, st, pd, bpatch, isfree, band, nbt, p, tot);
}

}  // namespace igamg
