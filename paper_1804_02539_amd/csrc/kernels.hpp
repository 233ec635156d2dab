// Launchers of the HIP kernels (kernels.hip).  All take the stream last.
// Templates are instantiated for double and float storage.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "layout.hpp"
#include "assemble_layout.hpp"

namespace igamg {

constexpr int RED_BLOCKS = 512;   // partial sums per reduction (the flexible dot uses 2x)

// ev0/ev1 (optional): timing events that record the dispatch's own start
// and end; an unsupported (d, p) returns hipErrorInvalidValue
template <typename T>
hipError_t launch_band(int d, int p, const T* band, const T* u, const T* f, T* r, const int* bpatch,
                       const PatchDev* pd, int64_t NL, bool resid, hipStream_t st, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr);
// The same in the scatter form of the symmetric half band (two kernels,
// each coefficient fetched once): `ws` = band_sym_window(d, p, largest n0 of
// the level's patches) values of window per 256-row tile, `win` holds
// NL / 256 * ws of them; ws * (8 + sizeof(T)) <= BAND_SYM_MAX_LDS (FP64
// windows and the u of their rows in LDS).  The events time both kernels
// together.
template <typename T>
hipError_t launch_band_sym(int d, int p, const T* band, const T* u, const T* f, T* r, const int* bpatch,
                           const PatchDev* pd, int64_t NL, int64_t ws, T* win, bool resid, hipStream_t st,
                           hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

size_t fd_slab_lds(int maxm, size_t elem);
size_t fd_dense_lds(int maxm, size_t elem);
// vector FD kernels: chunks of rb in {2, 4, 8} columns (FD_RB_MAX = 8)
constexpr int FD_RB_MAX = 8;
int fd_slab_grid(const FDItem* items, int nitems, int rb);
int fd_mid_grid(const FDItem* items, int nitems);
size_t fd_mid_lds(int maxm, size_t elem);
template <typename T>
void launch_fd_fwd(const FDItem* items, int nitems, int ndense, int gridx, size_t lds, const DensePiece* dense,
                   const T* densemat, const T* mat, const T* src, T* u, const int64_t* if_ptr, const int64_t* if_idx,
                   T* scr, double tau, bool add, int rb, hipStream_t st);
// FP32 forward/inverse products on the matrix cores (16-column chunks), with
// FP32 operands or operands rounded to bfloat16 (FP32 accumulation)
size_t fd_mfma_lds(int maxm);
// One launch per smoothing for 2D tensors (2D interiors, 3D faces) and the
// dense pieces: items[0 .. nitems) must all have m[2] == 1, every m <= MAX_FD.
size_t fd2_fused_lds(int maxm, int max_dense);
void launch_fd2_fused(const FDItem* items, int nitems, int ndense, size_t lds, const DensePiece* dense,
                      const float* densemat, const float* mat, const float* src, float* u, const int64_t* if_ptr,
                      const int64_t* if_idx, double tau, bool add, bool bf16, hipStream_t st);
int fd_mfma_grid(const FDItem* items, int nitems);
void launch_fd_fwd_mfma(const FDItem* items, int nitems, int ndense, int gridx, size_t lds, const DensePiece* dense,
                        const float* densemat, const float* mat, const float* src, float* u, const int64_t* if_ptr,
                        const int64_t* if_idx, float* scr, double tau, bool add, bool bf16, hipStream_t st);
void launch_fd_inv_mfma(const FDItem* items, int nitems, int gridx, size_t lds, const float* mat, float* u,
                        const int64_t* if_ptr, const int64_t* if_idx, const float* scr, double tau, bool add,
                        bool bf16, hipStream_t st);
template <typename T>
void launch_fd_mid(const FDItem* items, int nitems, int gridx, size_t lds, const T* mat, T* scr, hipStream_t st);
template <typename T>
void launch_fd_inv(const FDItem* items, int nitems, int gridx, size_t lds, const T* mat, T* u, const int64_t* if_ptr,
                   const int64_t* if_idx, const T* scr, double tau, bool add, int rb, hipStream_t st);

template <typename T>
void launch_restrict(int d, const T* rf, T* rc, const PatchDev* pd, const int* bpatch_c, int64_t NLc,
                     const int64_t* tidx, const T* tval, int WR, const uint8_t* isfree_c, hipStream_t st);
template <typename T>
void launch_prolong_add(int d, const T* uc, T* uf, const PatchDev* pd, const int* bpatch_f, int64_t NLf,
                        const int64_t* tidx, const T* tval, int WP, const uint8_t* isfree_f, hipStream_t st);

void launch_gather(const double* loc, double* glob, const int64_t* ptr, const int64_t* idx, int64_t n, bool dist,
                   hipStream_t st);
void launch_scatter(const double* glob, double* loc, const int64_t* ptr, const int64_t* idx, int64_t n, bool dist,
                    hipStream_t st);
template <typename T>
void launch_coarse(const T* Ainv, const T* f0, double* b, double* part, T* u0, const int64_t* ptr,
                   const int64_t* idx, int64_t n, hipStream_t st);
void launch_to_float(const double* x, float* y, int64_t n, hipStream_t st);
// A_0^{-1} of the dense SPD coarse matrix in packed lower tiles (layout.hpp):
// Lt holds A_0 on entry (identity padding) and its Cholesky factor on exit,
// Yt (zero on entry) the inverse factor L^{-1}, Ainv (zero on entry) the
// inverse.  *info (zero on entry) gets 1 + the first column whose pivot is
// not positive and finite.  Stream-ordered, no allocation, no library.
void coarse_inverse(double* Lt, double* Yt, double* Ainv, int64_t n, int* info, hipStream_t st);

template <typename T>
void launch_dot(const T* a, const T* b, int64_t n, double* part, double* scal, int slot, int op, hipStream_t st);
template <typename T>
void launch_dot2_flex(const T* r, const T* q, const T* z, int64_t n, double* part, double* scal, hipStream_t st);
template <typename T>
void launch_norm2_dist(T* r, const int64_t* ptr, const int64_t* idx, int64_t n, double* part, double* scal, int slot,
                       bool canon, hipStream_t st);
template <typename T>
void launch_axpy2(T* x, const T* p, T* r, const T* q, int64_t n, const double* scal, hipStream_t st);
template <typename T>
void launch_xpby(T* p, const T* z, int64_t n, const double* scal, hipStream_t st);
template <typename T>
void launch_fill(T* x, int64_t n, double v, hipStream_t st);
template <typename T>
void launch_copy(T* y, const T* x, int64_t n, hipStream_t st);
void launch_to_f32(float* y, const double* x, int64_t n, hipStream_t st);

// device assembly (assemble.hip): doubles of one element slab's metric (Gs),
// direction-0 (T1) and direction-1 (T2) intermediates of a patch
void asm_slab_sizes(int d, const AsmPatch& P, size_t out[3]);
// The coarse levels of a cycle as one persistent launch over a work list of
// phases (prog, nph entries, total items), preceded by a one-workgroup reset
// of the nph + 2 counters at ctr (ticket, one completion count per phase,
// overflow flag).
size_t cycle_tail_lds(int maxm, int max_dense, size_t elem);
template <typename T>
hipError_t launch_cycle_tail(int d, int p, const Phase* prog, int nph, int64_t total, unsigned long long* ctr,
                             int grid, size_t lds, T* out, hipStream_t st);
// FP32 full band (all (2p+1)^d planes per tile) from the FP64 symmetric half band
void launch_band_half_to_full(int d, int p, float* full, const double* half, const int* bpatch, const PatchDev* pd,
                              int64_t NL, hipStream_t st);
// out[e] = sum of the half-band entries (row[c], plane[c]), c in [ptr[e], ptr[e+1])
void launch_band_gather(const double* band, int nbh, const int64_t* ptr, const int64_t* row, const int* plane,
                        int64_t ne, double* out, hipStream_t st);
// adds slab e2's contribution of patch P to the tiled FP64 band (nbt =
// (2p+1)^d coefficients per row); ORs the sign bits of det J into *flag
hipError_t launch_asm_slab(int d, const AsmPatch& P, const double* tab, int e2, double* Gs, double* T1, double* T2,
                           double* band, int nbt, int* flag, hipStream_t st);
// zeroes the couplings of Dirichlet functions and those leaving the patch
void launch_asm_mask(int d, int p, const PatchDev* pd, const int* bpatch, const uint8_t* isfree, double* band,
                     int nbt, int64_t NL, hipStream_t st);
void launch_to_f64(double* y, const float* x, int64_t n, hipStream_t st);
void launch_add_f32(double* x, const float* d, int64_t n, hipStream_t st);

}  // namespace igamg
