/*
 * igamg -- multigrid for C0 multi-patch isogeometric Poisson problems on MI355X.
 *
 * Method: Hofer & Takacs, "A parallel multigrid solver for multi-patch
 * Isogeometric Analysis".  The Poisson model problem -Laplace u = f with
 * homogeneous Dirichlet data on Gamma_D and homogeneous Neumann data elsewhere
 * (Sec. 2) is discretised by C0-coupled tensor-product B-splines of degree p on
 * K fully matching patches (Sec. 2, the space V_l).  The solver is PCG
 * preconditioned by one multigrid V-cycle (Sec. 4) whose smoother is the
 * additive combination of patch-interior, face, edge and vertex smoothers
 * (Sec. 3, eq. of L_l^{-1}) and whose coarsest level is solved exactly by a
 * Cholesky factorisation (Sec. 4, the global coarse solver; Algorithm 1).
 *
 * Conventions used by every entry point:
 *  - Device vectors are double arrays in the global free-dof numbering of a
 *    level: patches in order, local functions x-fastest inside a patch, a dof
 *    numbered when its class (the copies of an interface function) is first
 *    met; Dirichlet functions are eliminated.  Length = igamg_num_dofs().
 *  - All device memory is the caller's: one workspace buffer of
 *    igamg_workspace_size() bytes (256-byte aligned) plus the vectors passed
 *    to each call.  The library never allocates device memory.
 *  - `stream` is a hipStream_t (NULL = the default stream).  A handle must not
 *    be used from two streams at once; work is enqueued asynchronously except
 *    where a call says it synchronises.
 *  - Every entry point returns IGAMG_OK (0) or a negative error code and never
 *    throws; igamg_last_error() gives a message for the calling thread.
 */
#ifndef IGAMG_H
#define IGAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IGAMG_OK 0
#define IGAMG_EINVAL (-1)  /* bad argument: sizes, degree, levels, null pointers   */
#define IGAMG_ETOPO (-2)   /* interface sides do not match, bad side/patch index    */
#define IGAMG_EGEOM (-3)   /* det J vanishes or changes sign inside a patch          */
#define IGAMG_ENOMEM (-4)  /* workspace smaller than igamg_workspace_size()          */
#define IGAMG_ENOTSPD (-5) /* coarse matrix not positive definite (no Dirichlet side)*/
#define IGAMG_ENOCONV (-6) /* solve stopped at maxit above the tolerance            */
#define IGAMG_ENAN (-7)    /* non-finite value met in the right-hand side or solve  */
#define IGAMG_EDEVICE (-8) /* a HIP call failed                                     */

/* Problem description (Sec. 2).
 * Patch k maps (0,1)^dim onto Omega_k by one tensor-product Bezier element of
 * degree geo_degree[k*dim + c] in direction c; its control points are stored
 * x-fastest, each with `dim` coordinates, patch after patch in geo_ctrl.
 * Level l has nel0[k*dim + c] * 2^l elements per patch and direction and
 * open knot vectors (p+1 copies of each end, simple interior knots: maximal
 * smoothness C^{p-1}, Sec. 2), l = 0 .. levels-1.  The coarsest breakpoints
 * are uniform, or given in knots0: for patch k and direction c in that order
 * (direction fastest), nel0[k*dim + c] + 1 values 0 = x_0 < ... < x_nel = 1;
 * each refinement halves every span (Sec. 3).  Interfaces must match: the
 * breakpoints of paired tangential directions agree (reversed where the
 * orientation reverses the axis), else ETOPO.
 * Side s = 2*dir + end of a patch is where parameter `dir` equals `end`.
 * iface[5*i .. 5*i+4] = (patch a, side a, patch b, side b, orient): the
 * tangential axes (t0 < t1) of side a meet the axes (u0 < u1) of side b; bit 0
 * of orient pairs t0 with u1 and t1 with u0, bit 1 reverses the axis paired
 * with t0, bit 2 the one paired with t1 (2D uses bit 1 only).
 * bc[k*2*dim + s] = 1 puts side s of patch k on Gamma_D (u = 0), 0 on Gamma_N;
 * entries of interface sides are ignored.  The arrays are read during
 * igamg_setup / igamg_workspace_size only.                                     */
typedef struct {
  int dim;                /* 2 or 3                                         */
  int degree;             /* spline degree p, 1 <= p <= 8                  */
  int npatch;             /* K >= 1                                         */
  int levels;             /* number of grid levels, >= 2                    */
  const int* nel0;        /* [npatch*dim] coarsest element counts, >= 1     */
  const double* knots0;   /* NULL: uniform; else the coarsest breakpoints   */
  const int* geo_degree;  /* [npatch*dim] Bezier degree of each map, >= 1   */
  const double* geo_ctrl; /* control points, see above                      */
  int nif;                /* number of interfaces                           */
  const int* iface;       /* [nif*5]                                        */
  const int* bc;          /* [npatch*2*dim]                                 */
} igamg_problem;

/* Solver parameters; igamg_default_options() gives the paper's choice
 * (Sec. 5): tau = 0.25, sigma = 5 h^-2, 1+1 smoothing, V-cycle; the readings
 * of the smoother's constants that reproduce the paper's Fichera iteration
 * table (geometry_scaling = 0, s1_sigma = 1).                               */
typedef struct {
  double tau;            /* smoothing damping                                */
  double sigma_scale;    /* sigma = sigma_scale * h^-2 in the interior smoother */
  int nu;                /* pre- and post-smoothing steps                    */
  int mu;                /* 1 = V-cycle, 2 = W-cycle                         */
  int precision;         /* IGAMG_FP64; IGAMG_MIXED (FP32 inner solve inside FP64 iterative
                            refinement); IGAMG_MIXED_BF16 (the same with the smoother's mode
                            products on the matrix cores from bfloat16 operands, FP32
                            accumulation: IGAMG_MIXED with fd_mfma = 3).  FP32 cannot
                            resolve 3D patch operators of high degree (their condition
                            grows fast with p): 3D p = 7 needs ~4x the FP64 iterations,
                            and coarse-dominated 3D problems at p >= 7 end in ENOCONV or
                            ENAN; use IGAMG_FP64 there                                     */
  int maxit;             /* iteration cap of igamg_solve                    */
  int geometry_scaling;  /* 0 (default): piece operators in parameter-domain units, as the
                            paper's Fichera iteration table indicates; 1: each scaled by
                            the patch's mean |det J| tr(J^{-1} J^{-T}) / d                  */
  int inner_maxit;       /* mixed: inner PCG iteration cap per refinement step (100) */
  double inner_tol;      /* mixed: the largest reduction an inner FP32 solve is asked for (1e-4) */
  int graphs;            /* 1: replay each PCG iteration as HIP graphs (default); 0: direct launches */
  int fd_mfma;           /* FP32 fast-diagonalization mode products (mixed precision): 0 (default) as the
                            autotuner chooses among vector FMAs and FP32 matrix cores, 1 always on the
                            matrix cores (v_mfma_f32_16x16x4f32: FUSED on levels of 2D tensors, MFMA
                            otherwise), 2 always vector FMAs, 3 always on the matrix cores with the
                            operands rounded to bfloat16 (v_mfma_f32_16x16x16bf16_1k, FP32
                            accumulation) */
  int coarse_factor;     /* factorization of the dense coarse matrix: 0 (default) on the host up to
                            3000 coarse unknowns and on the device (the library's tiled Cholesky
                            factorization and inversion, in the workspace) above; 1 always on the
                            host; 2 always on the device; at most 100000 coarse unknowns */
  int autotune;          /* 1 (default): at setup, time the smoother variants of every level and
                            precision on the device and keep the fastest (igamg_tuning); 0: vector
                            FMAs with 8-column chunks */
  int assembly;          /* banded matrices of levels >= 1: 0 (default) assembled on the device by
                            sum-factorised Gauss quadrature, straight into the workspace; 1 on the host
                            and uploaded (level 0, which forms the coarse matrix, is always assembled
                            on the host) */
  /* Readings of the smoother's constants, which the paper leaves to its
   * references (Sec. 3) and to an equivalence of the physical and the
   * parameter-domain operators up to geometry-dependent factors (Sec. 2);
   * the defaults are the library's reading:                                */
  int s1_sigma;           /* 1 (default): K + sigma M on the complement S1 of the interior
                             subspace corrected mass smoother; 0: K                        */
  int iface_multiplicity; /* 0 (default): face, edge and vertex operators as printed; 1: each
                             times the number of patches adjacent to the piece             */
  int physical_h;         /* 0 (default): h_c = 1/nel_c of the parameter domain; 1: the
                             patch's mean physical length in direction c over nel_c        */
  int iface_direct;       /* 0 (default): the edge and vertex smoothers of Sec. 3, (h/p)^{d-1} K
                             + (h/p)^{d-3} M and (h/p)^{d-2}; 1: the exact restriction of A_l
                             to each edge and vertex, solved directly (the variant Sec. 3
                             cites from its reference)                                    */
  int persistent;         /* 1: the levels of at most 65536 local rows below the finest run as one
                             persistent launch per cycle (a work list of the cycle's phases,
                             V-cycle only); 0 (default): one launch per kernel               */
  int band_form;          /* banded apply of the symmetric half band (Sec. 4's patch matrices):
                             0 (default): levels above 65536 local rows in 3D, or in 2D
                             2^17 (FP64 handles) or 2^19 (mixed handles),
                             read each stored coefficient once and add its mirrored term
                             through per-tile windows (two kernels; the FP32 copy of those
                             levels is the half band too), where a tile's windows and the u
                             of their rows fit 96 KiB of LDS in FP64: 16 ((p+1) 256 +
                             (2p+1) W) bytes, W = p + p n0 in 3D (n0 the level's largest
                             patch size along x) and p in 2D; 1: every level reads the
                             mirrored half from the rows it couples to (one kernel);
                             2: the scatter form on every level whose windows fit, the
                             persistent cycle's levels (options.persistent) excepted          */
} igamg_options;

#define IGAMG_FP64 0
#define IGAMG_MIXED 1
#define IGAMG_MIXED_BF16 2

typedef struct {
  int iterations;        /* PCG iterations (mixed: inner iterations summed) */
  int outer_iterations;  /* mixed: refinement steps; FP64: 0                */
  int converged;         /* 1 if ||f - A u|| <= tol ||f||                    */
  double rel_residual;   /* final ||f - A u||_2 / ||f||_2 (FP64 residual)   */
  double solve_ms;       /* wall time of the call on the stream             */
  int fp64_fallback;     /* mixed: 1 if a refinement asked for 10x cut the FP64 residual by
                            less than 4x, or an inner FP32 solve broke down, and the solve
                            was restarted as the FP64 PCG from u = 0 (iterations counts
                            both phases)                                                    */
} igamg_solve_info;

typedef struct igamg_ctx* igamg_handle;

void igamg_default_options(igamg_options* opts);

/* Bytes of device workspace that igamg_setup needs for this problem.  Runs
 * the topology part of the setup on the host (no assembly, no device use). */
int igamg_workspace_size(const igamg_problem* prob, const igamg_options* opts, size_t* bytes);

/* Host setup (Sec. 5's setup phases: dof maps, refinement and transfer
 * matrices, piece smoothers, coarse factorisation) and patch-wise Gauss
 * assembly of the banded matrices A_{l,k} (Sec. 4), uploaded into `workspace`
 * on `stream`.  By default (options.assembly) the levels above the coarsest
 * are assembled on the device, directly into the workspace, with a part of
 * the workspace as scratch.  Coarse problems factored on the device (see
 * options.coarse_factor) are factored and inverted there by the library's own
 * kernels, with a part of the workspace as scratch; then the smoother
 * variants are autotuned (see igamg_tuning).  Synchronises the stream before returning.  The handle
 * keeps host copies of nothing large; the workspace must outlive it.
 * IGAMG_VERBOSE set in the environment prints one line per setup phase.
 * With workspace == NULL the handle stays on the host (for igamg_export and
 * the size queries; the solver entry points then return EINVAL).
 * Errors: EINVAL, ETOPO, EGEOM, ENOTSPD, ENOMEM (bytes too small), EDEVICE.  */
int igamg_setup(const igamg_problem* prob, const igamg_options* opts, void* workspace,
                size_t bytes, void* stream, igamg_handle* out);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): igamg_setup without any
 * allocation by the library.  The hierarchy goes into the caller's
 * `workspace` as with igamg_setup, but the setup-only scratch of the device
 * assembly lives in a static device array of 64 MiB per GPU (held until the
 * process ends), so the workspace is smaller than igamg_workspace_size():
 * with workspace == NULL the call only writes the bytes it needs to *needed
 * (out may then be NULL).  No hipMalloc, hipFree, pinned host memory or
 * library allocation is made (the coarse matrix is factored as
 * options.coarse_factor says, on the device in the workspace), the
 * handle reads its scalars back into ordinary host memory and so launches
 * its solves directly (options.graphs is ignored), and a problem whose
 * setup scratch exceeds the static array is rejected with EINVAL.  Calls are
 * serialised inside the process; the array keeps the last call's contents,
 * and each call clears what it needs zeroed.  Other errors as igamg_setup.   */
int igamg_setup_noalloc(const igamg_problem* prob, const igamg_options* opts, void* workspace, size_t bytes,
                        void* stream, igamg_handle* out, size_t* needed);

/* Free and local sizes of level `level` (-1 = finest): n_free = unique free
 * dofs, n_local = sum over patches of their local function counts.          */
int igamg_num_dofs(igamg_handle h, int level, int64_t* n_free, int64_t* n_local);

/* Load vector f_i = int_Omega src(x) phi_i(x) dx of the finest level for
 * src(x) = amp * prod_c sin(freq * pi * x_c), by Gauss quadrature on the host,
 * written to the host array f_host[n_free].                                   */
int igamg_load_vector(igamg_handle h, double amp, double freq, double* f_host);

/* One multigrid cycle with zero initial guess on the finest level, i.e. the
 * preconditioner z = B r of Sec. 4 (Algorithm 1 called on level L).  r and z
 * are device vectors of length n_free (finest); they may not alias.         */
int igamg_vcycle(igamg_handle h, const double* r, double* z, void* stream);

/* PCG with one cycle as preconditioner from u = 0 (Sec. 4), stopping when
 * ||f - A u||_2 <= tol ||f||_2 (Sec. 5).  With precision IGAMG_MIXED, FP64
 * iterative refinement around FP32 PCG solves: the residual f - A u and the
 * update u += d are FP64 (FP64 band), each correction d is an FP32 PCG solve
 * (FP32 bands, smoothers, transfers; the coarse solve reads A_0^{-1} rounded
 * to FP32 and sums in FP64) that
 * reduces its residual by max(inner_tol, tol / (2 r)), r the outer relative
 * residual before it (the last correction aims just past tol instead of a
 * whole further inner_tol), and `maxit` caps the inner iterations summed.  rhs and u: device vectors of
 * length n_free (finest).  Synchronises the stream (reads the residual norm
 * back once per iteration).  Returns ENOCONV when maxit is reached and ENAN
 * on a non-finite residual; `info` (may be NULL) is filled in either case.  */
int igamg_solve(igamg_handle h, const double* rhs, double* u, double tol, igamg_solve_info* info,
                void* stream);

/* Batched solves (continuous batching).  A batch steps any number of resident
 * solves in lockstep: each step is one PCG iteration of every active request.
 * Each handle captures the two halves of its PCG iteration as HIP graphs once
 * (they stay with the handle until igamg_destroy) and the batch replays them,
 * one branch stream per request, so the requests' kernels overlap on the
 * device and requests joining or leaving cost no new capture.  Requests may
 * be added and removed between steps; mixed-precision requests run their FP64
 * refinement steps between inner solves.  A batch owns HIP streams and events
 * (no device memory); one host thread drives it.
 *   igamg_batch_add     starts the solve of A u = rhs on handle h (device vectors
 *                       of length n_free; no other solve may use h meanwhile);
 *                       returns the request's slot id in *slot
 *   igamg_batch_step    runs one lockstep step on `stream` and synchronises it;
 *                       *n_active = requests still running afterwards
 *   igamg_batch_poll    *done = 1 once the request finished; *info and its code
 *                       are then final (OK, ENOCONV or ENAN), u holds the result
 *   igamg_batch_remove  frees a slot (a running request is abandoned)
 * igamg_solve_batch solves n requests to completion with one batch.          */
typedef struct igamg_batch_ctx* igamg_batch;
int igamg_batch_create(igamg_batch* out);
int igamg_batch_destroy(igamg_batch b);
int igamg_batch_add(igamg_batch b, igamg_handle h, const double* rhs, double* u, double tol, void* stream,
                    int* slot);
int igamg_batch_step(igamg_batch b, void* stream, int* n_active);
int igamg_batch_poll(igamg_batch b, int slot, int* done, igamg_solve_info* info, int* code);
int igamg_batch_remove(igamg_batch b, int slot);
int igamg_solve_batch(igamg_handle const* hs, const double* const* rhs, double* const* u, int n, double tol,
                      igamg_solve_info* infos, int* codes, void* stream);

/* The operators of one level on global free vectors, for checking the parts of
 * the cycle one at a time:
 *   IGAMG_OP_APPLY     y = A_l x                          (x, y on level l)
 *   IGAMG_OP_SMOOTHER  y = L_l^{-1} x                     (level l >= 1)
 *   IGAMG_OP_PROLONG   y = P_l x  (x on level l-1, y on level l, l >= 1)
 *   IGAMG_OP_RESTRICT  y = P_l^T x (x on level l, y on level l-1, l >= 1)
 *   IGAMG_OP_COARSE    y = A_0^{-1} x                     (level 0)
 *   IGAMG_OP_CYCLE_FP32 y = B r with the FP32 data of a IGAMG_MIXED handle
 *                      (finest level; x rounded to FP32, y returned in FP64)
 *   IGAMG_OP_APPLY_FP32 y = A_l x with the FP32 band of a IGAMG_MIXED handle
 *                      (level >= 1; x rounded to FP32, the patch products in
 *                      the level's band form, the copies summed in FP64)
 * Device vectors; x and y may not alias.                                      */
#define IGAMG_OP_APPLY 0
#define IGAMG_OP_SMOOTHER 1
#define IGAMG_OP_PROLONG 2
#define IGAMG_OP_RESTRICT 3
#define IGAMG_OP_COARSE 4
#define IGAMG_OP_CYCLE_FP32 5
#define IGAMG_OP_APPLY_FP32 6
int igamg_operator(igamg_handle h, int op, int level, const double* x, double* y, void* stream);

/* Copies of the global free dofs of a level in the library's patch-local
 * layout: for dof g, local positions copy_idx[copy_ptr[g] .. copy_ptr[g+1]).
 * Host arrays; pass NULL pointers to query the sizes (n_free, n_copies).    */
int igamg_dof_map(igamg_handle h, int level, int64_t* copy_ptr, int64_t* copy_idx,
                  int64_t* n_free, int64_t* n_copies);

/* Setup products as dense host matrices, for inspection of small problems:
 *   IGAMG_EXPORT_MATRIX   the assembled A_l on free dofs (n_free x n_free); only
 *                         on handles set up without a workspace (the bands are
 *                         dropped from host memory after an upload)
 *   IGAMG_EXPORT_PROLONG  P_l (n_free(l) x n_free(l-1)), level >= 1
 * Pass out = NULL to query rows/cols.  Row-major doubles.                      */
#define IGAMG_EXPORT_MATRIX 0
#define IGAMG_EXPORT_PROLONG 1
int igamg_export(igamg_handle h, int what, int level, double* out, int64_t* rows, int64_t* cols);

/* Kernel timing of the banded stiffness apply (the bandwidth-bound kernel of
 * the cycle).  enable = 1 starts recording a HIP event pair around every
 * banded-apply launch on every level (events are created by the library on
 * first use; recording adds no synchronisation), enable = 0 stops.  While
 * recording, solves launch their kernels directly instead of replaying HIP
 * graphs (HIP does not time events recorded into graphs).
 * igamg_profile_read synchronises the stream of the last recorded launch and
 * returns, per level l, the launch count, the summed kernel time in ms (timing
 * events attached to each dispatch, so the time is the kernel's own) and the
 * algorithmic bytes moved (rows * s (planes + vectors): FP64, s = 8 and the
 * ((2p+1)^d + 1)/2 stored planes of the symmetric half band; FP32, s = 4 and
 * all (2p+1)^d planes);
 * arrays have 2*levels entries: [l] for FP64 launches, [levels + l] for FP32
 * launches of a mixed-precision handle.  Then it clears the record.          */
int igamg_profile(igamg_handle h, int enable);
int igamg_profile_read(igamg_handle h, int64_t* launches, double* ms, double* bytes);

/* Smoother variants (tile shapes of the fast-diagonalization kernels).      */
#define IGAMG_FD_VEC8 0   /* vector FMAs, chunks of 8 columns per workgroup     */
#define IGAMG_FD_VEC4 1   /* vector FMAs, chunks of 4 columns per workgroup     */
#define IGAMG_FD_MFMA 2   /* FP32 only: 16x16x4 matrix-core tiles, 8 columns    */
#define IGAMG_FD_FUSED 3  /* FP32 only, levels whose items are all 2D tensors: one
                             launch per smoothing, each item in LDS through the four
                             mode products on the matrix cores                     */
#define IGAMG_FD_MFMA_BF16 4 /* FP32 solves: the matrix-core products (FUSED on 2D
                             levels, MFMA otherwise) with operands rounded to
                             bfloat16, FP32 accumulation; only by options.fd_mfma = 3 */

/* The smoother variant level `level` (>= 1) uses in FP64 (fp32 = 0) or in
 * the FP32 inner solves (fp32 = 1).  With options.autotune = 1 setup times
 * each candidate (VEC8, VEC4; for FP32 also MFMA, and FUSED on levels of 2D
 * tensors, on levels whose tensors fit in LDS: sides up to 84; unless fd_mfma
 * fixes the choice) on the device over a few smoother applications and keeps
 * the fastest.  The
 * choice is cached per process under a key of the level's piece shapes, the
 * degree and the precision, so handles of the same problem agree (and their
 * results are identical); the environment variable IGAMG_TUNE_CACHE names a
 * JSON file that persists the cache between processes.                      */
int igamg_tuning(igamg_handle h, int level, int fp32, int* variant);

/* The form of level `level`'s (>= 1) banded apply, the same in both
 * precisions (options.band_form): IGAMG_BAND_GATHER (each row reads the
 * mirrored half of the symmetric band from the rows it couples to; the FP32
 * copy is the full band) or IGAMG_BAND_SCATTER (each stored coefficient read
 * once, its mirrored term added through per-tile windows; the FP32 copy is
 * the half band).                                                           */
#define IGAMG_BAND_GATHER 0
#define IGAMG_BAND_SCATTER 1
int igamg_band_form(igamg_handle h, int level, int* form);

/* Release the handle (not the workspace).                                    */
int igamg_destroy(igamg_handle h);

/* Message of the last error on the calling thread ("" if none).            */
const char* igamg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* IGAMG_H */
