// Launchers of the HIP kernels (kernels.hip).  All take the stream last.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "layout.hpp"

namespace igamg {

constexpr int RED_BLOCKS = 512;   // partial sums per reduction

void launch_band(int d, int p, const double* band, const double* u, const double* f, double* r, const int* bpatch,
                 const PatchDev* pd, int64_t NL, bool resid, hipStream_t st);
int fd_grid_x(const FDItem* items, int nitems, int dir);
size_t fd_lds_bytes(int maxm);
void launch_fd_pass(const FDItem* items, int nitems, int gridx, size_t lds, int dir, int mode, int in_sel, int out_sel,
                    const double* mat, const double* src_loc, const double* src_if, double* dst_loc, double* dst_if,
                    double* scrA, double* scrB, double tau, bool add, hipStream_t st);
size_t fd_slab_lds(int maxm);
int fd_slab_grid(const FDItem* items, int nitems);
void launch_fd_fwd(const FDItem* items, int nitems, int ndense, int gridx, size_t lds, const DensePiece* dense,
                   const double* densemat, const double* mat, const double* src, double* u, const int64_t* if_ptr,
                   const int64_t* if_idx, double* scr, double tau, bool add, hipStream_t st);
void launch_fd_inv(const FDItem* items, int nitems, int gridx, size_t lds, const double* mat, double* u,
                   const int64_t* if_ptr, const int64_t* if_idx, const double* scr, double tau, bool add,
                   hipStream_t st);
void launch_restrict(int d, const double* rf, double* rc, const PatchDev* pd, const int* bpatch_c, int64_t NLc,
                     const int64_t* tidx, const double* tval, int WR, const uint8_t* isfree_c, hipStream_t st);
void launch_prolong_add(int d, const double* uc, double* uf, const PatchDev* pd, const int* bpatch_f, int64_t NLf,
                        const int64_t* tidx, const double* tval, int WP, const uint8_t* isfree_f, hipStream_t st);
void launch_gather(const double* loc, double* glob, const int64_t* ptr, const int64_t* idx, int64_t n, bool dist,
                   hipStream_t st);
void launch_scatter(const double* glob, double* loc, const int64_t* ptr, const int64_t* idx, int64_t n, bool dist,
                    hipStream_t st);
void launch_coarse(const double* Ainv, const double* b, double* u0, const int64_t* ptr, const int64_t* idx, int n,
                   hipStream_t st);
void launch_dot(const double* a, const double* b, int64_t n, double* part, double* scal, int slot, int op,
                hipStream_t st);
void launch_norm2_dist(const double* r, const int64_t* ptr, const int64_t* idx, int64_t n, double* part, double* scal,
                       int slot, hipStream_t st);
void launch_axpy2(double* x, const double* p, double* r, const double* q, int64_t n, const double* scal,
                  hipStream_t st);
void launch_xpby(double* p, const double* z, int64_t n, const double* scal, hipStream_t st);
void launch_fill(double* x, int64_t n, double v, hipStream_t st);
void launch_copy(double* y, const double* x, int64_t n, hipStream_t st);

}  // namespace igamg
