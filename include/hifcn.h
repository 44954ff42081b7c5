/* hifcn.h -- HIF-preconditioned Crank-Nicolson solves on AMD Instinct MI355X (gfx950).
 *
 * Method: Feliu-Faba & Ying, "Hierarchical Interpolative Factorization Preconditioner for
 * Parabolic Equations".  The equation u_t = div(a grad u) + r(u) (Sec. 1, eq1) on the unit
 * square/cube with zero Dirichlet data is discretised by the five/seven-point stencil (Sec. 2)
 * and stepped by Crank-Nicolson with explicit reaction (Sec. 2.1, eq_CN):
 *     (I - dt/2 M) u^{k+1} = (I + dt/2 M) u^k + dt r(u^k).
 * Each step is solved by CG preconditioned with the inverse of the recursively preconditioned
 * hierarchical interpolative factorization F of A = I - dt/2 M (Sec. 2.2, eqAinv; Algorithm 1).
 *
 * Conventions shared by every entry point:
 *   - Grids: n interior nodes per axis (equal on every axis), h = 1/(n+1); node arrays are
 *     FP64, C-contiguous, shape n^dim with the x index fastest.  The coefficient a lives on the
 *     (n+1)^dim cells between nodes (same ordering); a link's coefficient is the mean of the
 *     cells sharing it.
 *   - Pointers named *_dev are DEVICE pointers owned by the caller; the library never frees
 *     them.  Host pointers are named explicitly.  A handle owns all device memory it allocates.
 *   - Every call is ordered on the HIP stream passed as `hip_stream` (a hipStream_t; NULL =
 *     the null stream) and may return before the GPU work ends, except where stated.
 *   - Errors are reported only through the status code; no exception crosses this boundary.
 *     hif_last_error() returns a thread-local message for the last non-OK status.  On error
 *     an output handle is set to NULL and caller buffers are untouched, except as stated for
 *     HIF_ERR_NO_CONV.
 *   - One handle may be used by one host thread / stream at a time.
 */
#ifndef HIFCN_H
#define HIFCN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t dim;    /* 2 or 3 */
  int32_t n[3];   /* interior nodes per axis; n[0] == n[1] (== n[2] in 3D) is required */
  int32_t leaf;   /* leaf cell size m: L = max{l : m 2^l <= n+1} levels, separators at k m 2^l */
} hif_grid_t;

/* Storage precision of the factor blocks used by hif_apply (the build is always FP64;
 * FP32/BF16 forms accumulate in FP32, the FP64 form in FP64). */
typedef enum { HIF_STORE_F64 = 0, HIF_STORE_F32 = 1, HIF_STORE_BF16 = 2 } hif_store_t;

typedef enum {
  HIF_OK = 0,
  HIF_ERR_ARG = 1,      /* invalid argument (grid, sizes, NULL pointer, bad blob) */
  HIF_ERR_OOM = 2,      /* device allocation failed */
  HIF_ERR_NOT_SPD = 3,  /* a Cholesky pivot was not positive (A not SPD, e.g. a <= 0) */
  HIF_ERR_NO_CONV = 4,  /* PCG hit maxit or produced a non-finite residual */
  HIF_ERR_HIP = 5       /* a HIP runtime call failed */
} hif_status_t;

typedef struct hif_handle_s* hif_handle_t;

/* Reaction term r(u) (eq1, eq_nr): kind 0 -> none; kind 1 -> k1 u (1 - u/k2). */
typedef struct { int32_t kind; double k1; double k2; } hif_reaction_t;

/* PCG options (Algorithm 1): stop when ||r_i||_2 <= rtol ||g||_2 (recurrence residual), at
 * most maxit iterations (1 .. 2^24 - 1).  warm_start 0: x0 = 0 (the default reading of
 * Algorithm 1's pcg); 1: x0 = u^k, the state before the step (r0 = g - A u^k, the same test;
 * a step whose r0 already meets it takes no iteration and keeps u; g = 0 still gives u = 0).
 * cn_step and cn_solve take either; cn_batch_step requires 0 (HIF_ERR_ARG otherwise). */
typedef struct { double rtol; int32_t maxit; int32_t warm_start; } hif_cg_opts_t;

/* Build the PHIF factor of A = I - dt/2 M (Sec. 2.2: per level cell elimination, block Jacobi,
 * edge/face skeletonization by ID at relative precision eps; root Cholesky) on the GPU in FP64
 * and store its blocks in `store` precision.  a_cells_dev: (n+1)^dim FP64 values > 0.
 * Synchronises `hip_stream` (the level structure depends on the ranks found).
 * Errors: HIF_ERR_ARG (grid, dt <= 0, eps < 0), HIF_ERR_NOT_SPD, HIF_ERR_OOM, HIF_ERR_HIP. */
hif_status_t hif_factor(const double* a_cells_dev, double dt, const hif_grid_t* grid,
                        double eps, hif_store_t store, void* hip_stream, hif_handle_t* out);

/* Build options.  dense_top: the largest number of entries the dense top of the apply may hold
 * (the stages from some level's group step up to the root and back, formed at build time as
 * one symmetric matrix; see hif_get_info's top_level): < 0 the library's default (or the
 * HIFCN_DENSE_TOP environment variable), 0 none.  Forming it costs build time that a solve of
 * few steps may not win back.  flags: 0 or HIF_FACTOR_SKEL_EDGES.  reserved: must be 0. */
typedef struct { int64_t dense_top; int64_t flags; int64_t reserved[2]; } hif_factor_opts_t;

/* 3D: skeletonize the edges of every level as well as its faces in step (3) (Sec. 2.2, 3D
 * paragraph: the paper's variant that lowers the build's complexity).  Edges are ID'd from the
 * same matrix as the faces (level-synchronous).  No effect in 2D, where the edges are the
 * skeletonized groups anyway. */
#define HIF_FACTOR_SKEL_EDGES 1

/* hif_factor with options (opts may be NULL: the defaults).  Errors as hif_factor, and
 * HIF_ERR_ARG for unknown flags or nonzero reserved fields. */
hif_status_t hif_factor_ex(const double* a_cells_dev, double dt, const hif_grid_t* grid,
                           double eps, hif_store_t store, const hif_factor_opts_t* opts,
                           void* hip_stream, hif_handle_t* out);

/* Test fixture: like hif_factor, but the factor blocks are read from `blob_host` (nbytes, host
 * memory) written in the HIFB format below instead of being built, so that hif_apply can be
 * checked independently of the build.  Synchronises `hip_stream`.
 *
 * HIFB format (little endian; i32 = int32, f64 = IEEE double; matrices row-major, full):
 *   i32 magic 0x42464948 ("HIFB"), i32 version 1, i32 dim, i32 n, i32 leaf, i32 nlevels
 *   per level: i32 ncell,  per cell : i32 nI, i32 nB, i32 I[nI], i32 B[nB],
 *                                     f64 L[nI*nI] (chol(A_II), lower), f64 G[nI*nB] (L^-1 A_IB)
 *              i32 ngroup, per group: i32 n, i32 idx[n], f64 Lg[n*n] (chol(A_gg), lower)
 *              i32 nskel,  per edge : i32 nr, i32 k, i32 red[nr], i32 skel[k],
 *                                     f64 T[k*nr], f64 Ls[nr*nr] (chol(I + T^T T), lower)
 *   i32 nroot, i32 root[nroot], f64 Lr[nroot*nroot]
 * DOF ids are global node indices (C order, x fastest).  Every skeletonized edge must also
 * appear, with the same DOF set, among the groups of its level. */
hif_status_t hif_import(const double* a_cells_dev, double dt, const hif_grid_t* grid,
                        const void* blob_host, size_t nbytes, hif_store_t store,
                        void* hip_stream, hif_handle_t* out);

/* Time-dependent coefficients (Sec. 4: with a(x, t) the factor is rebuilt, or, when a changes
 * slowly, rebuilt once every few steps and reused in between).
 *
 * hif_set_coefficient: the operator of every later call (hif_spmv, the A and the
 * I + dt/2 M of cn_step, cn_solve, cn_solve_direct, cn_batch_step) becomes the one of
 * a_cells_dev ((n+1)^dim FP64 values > 0, same grid and dt); the factor is kept, so PCG is
 * preconditioned by the factor of the coefficient it was built from.  Ordered on hip_stream.
 *
 * hif_refactor: rebuilds the factor from a_cells_dev with the handle's grid, dt, eps, storage
 * and dense-top budget, and sets the operator as hif_set_coefficient does.  The handle keeps
 * its address; the old factor is freed once the new one is built, so both are resident for a
 * moment.  Synchronises hip_stream (as hif_factor does); no work on the handle may be in
 * flight on another stream.  On error the handle keeps its old factor and operator.
 * Errors: HIF_ERR_ARG (NULL argument; a handle made by hif_import, which has no eps),
 * HIF_ERR_NOT_SPD, HIF_ERR_OOM, HIF_ERR_HIP. */
hif_status_t hif_set_coefficient(hif_handle_t h, const double* a_cells_dev, void* hip_stream);
hif_status_t hif_refactor(hif_handle_t h, const double* a_cells_dev, void* hip_stream);

/* y = F^-1 x (eqAinv: forward sweep E^T C^T K^T over levels 0..L-1, root solve, backward sweep
 * K C E over levels L-1..0).  x_dev, y_dev: N FP64 values; may alias. */
hif_status_t hif_apply(hif_handle_t h, const double* x_dev, double* y_dev, void* hip_stream);

/* y = A x with A = I - dt/2 M (five/seven-point stencil, Sec. 2).  x_dev, y_dev must not alias. */
hif_status_t hif_spmv(hif_handle_t h, const double* x_dev, double* y_dev, void* hip_stream);

/* One Crank-Nicolson step (eq_CN, Algorithm 1): g = (I + dt/2 M)u + dt r(u), then PCG with
 * preconditioner F^-1 from x0 = 0; u_dev (N FP64) is replaced by u^{k+1}.  *iters_host and
 * *relres_host (may be NULL) receive the iteration count and ||r||/||g||.  Synchronises the
 * stream.  HIF_ERR_NO_CONV: u_dev holds the last iterate and *iters_host = maxit; or, when
 * ||g||^2 is not finite (a NaN or Inf in u, or an overflowing reaction), the step stops before
 * its first iteration with u_dev unchanged and *iters_host = 0.  g = 0 gives u = 0, 0 iterations,
 * HIF_OK. */
hif_status_t cn_step(hif_handle_t h, const hif_reaction_t* r, const hif_cg_opts_t* opts,
                     double* u_dev, int32_t* iters_host, double* relres_host, void* hip_stream);

/* nsteps Crank-Nicolson steps; iters_host[nsteps], relres_host[nsteps] (host arrays, may be
 * NULL) receive per-step statistics, copied once at the end.  Synchronises the stream at
 * most a few times per step (PCG convergence checks) and at the end. */
hif_status_t cn_solve(hif_handle_t h, const hif_reaction_t* r, const hif_cg_opts_t* opts,
                      double* u_dev, int32_t nsteps, int32_t* iters_host, double* relres_host,
                      void* hip_stream);

/* nsteps Crank-Nicolson steps with the factor as the solver, without CG (Sec. 3: at
 * eps = 1e-6 the factor approximates A^-1 well enough to bypass CG): u^{k+1} = F^-1 g^k with
 * g^k = (I + dt/2 M) u^k + dt r(u^k) as in cn_step.  Since every eigenvalue of A is >= 1, one
 * step differs from the exact CN step by at most ||I - A F^-1||_2 ||g^k||_2.  u_dev (N FP64) is
 * replaced by u^{nsteps}.  Queues the steps without synchronising; the values are not checked
 * (a non-finite u propagates).  Uses the handle's PCG workspace: not concurrently with another
 * call on the same handle.  Errors: HIF_ERR_ARG (NULL handle or u_dev, nsteps < 0, reaction). */
hif_status_t cn_solve_direct(hif_handle_t h, const hif_reaction_t* r, double* u_dev,
                             int32_t nsteps, void* hip_stream);

/* Continuous batching: one Crank-Nicolson step (as cn_step) for each of `count` independent
 * solves, handle h[i] with state u_dev[i] (device, N_i FP64), reaction r[i] (array, may be
 * NULL: none) and options opts[i], each queued on its own stream hip_streams[i] (array, may be
 * NULL: the null stream).  The PCG iterations of all solves are queued in lockstep with one
 * convergence read-back per round for the whole batch, so the kernels of different solves
 * overlap on the device, and each solve's result is exactly what cn_step gives for it alone.
 * iters_host[i], relres_host[i], status_host[i] (host arrays, each may be NULL) receive the
 * statistics and each solve's own status (HIF_OK or HIF_ERR_NO_CONV).  A handle may appear at
 * most once.  Synchronises every stream.  Returns HIF_ERR_NO_CONV if any solve failed to
 * converge; every other solve still completes its step. */
hif_status_t cn_batch_step(hif_handle_t* h, const hif_reaction_t* r, const hif_cg_opts_t* opts,
                           double** u_dev, int32_t count, int32_t* iters_host,
                           double* relres_host, int32_t* status_host, void** hip_streams);

/* Estimate of ||I - A F^-1||_2, how far the factor is from A^-1 (Sec. 3, Example 1, where the
 * paper estimates this norm by a randomized power iteration: 7.9e-6 at eps = 1e-6 on 4095^2).
 * With E = I - A F^-1 (E^T = I - F^-1 A, A and F^-1 being symmetric): x = x0 / ||x0||, then
 * `iters` times y = E^T E x, lambda = ||y||, x = y / lambda; *est_host = sqrt(lambda), a lower
 * bound of ||E||_2 that rises towards it (0 for iters = 0).  x0_dev: the caller's start vector
 * (device, N FP64, not modified; a random one makes the bound hold with high probability).
 * Scratch: 4 N + 520 FP64 values, allocated for the call and freed before it returns.  The
 * estimate is deterministic (fixed-order reductions).  Synchronises `hip_stream`.  Uses the
 * handle's apply buffers: not concurrently with another call on the same handle.
 * Errors: HIF_ERR_ARG (NULL argument, iters < 0), HIF_ERR_OOM, HIF_ERR_HIP. */
hif_status_t hif_inverse_error(hif_handle_t h, const double* x0_dev, int32_t iters,
                               double* est_host, void* hip_stream);

/* hif_inverse_error without any allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same iteration and kernels, with its scratch in a fixed device array that the library holds
 * on each GPU it runs on until the process ends (8.4 MB: N <= 262144, e.g. 512^2 or 64^3
 * grids).  Results equal hif_inverse_error's bit for bit.  Every call on one GPU shares that
 * array: calls that overlap on one GPU (other streams or host threads) race and must be
 * serialised by the caller.  Calls no hipMalloc, hipFree or allocating library routine.
 * Synchronises `hip_stream`.  Errors: HIF_ERR_ARG (NULL argument, iters < 0, N above the
 * limit: nothing is launched), HIF_ERR_HIP. */
hif_status_t hif_inverse_error_noalloc(hif_handle_t h, const double* x0_dev, int32_t iters,
                                       double* est_host, void* hip_stream);

/* Stored factor bytes (unpadded, in the storage precision; without the dense forms that
 * hif_get_info's device_bytes includes). */
size_t hif_factor_bytes(hif_handle_t h);

/* Structure summary: number of levels, root size, stored factor entries, every byte of device
 * memory the handle holds (factor, descriptors and PCG workspace; what a server admitting solves
 * by HBM footprint accounts for), the part of the build that ran on the FP64 matrix cores
 * (large cells, the root and the dense forms of blocks too large for one workgroup, Sec. 2.2):
 * its algorithmic flops and the summed duration of those kernels (0 for imported factors), and
 * the algorithmic bytes of one hif_apply (the sum over its stages, as hif_profile_read reports
 * them: factor blocks in the form the apply reads them, index lists and FP64 vectors), and the
 * level from which the apply runs as one dense matrix (the group steps of that level and every
 * stage above it, the root included; reported as the root stage), or -1.  top_fold: 1 when
 * the backward cell stage of that level takes the dense top's results straight from its
 * partial sums (no separate write-back launch), else 0. */
typedef struct {
  int32_t levels;
  int32_t root;
  int64_t entries;
  int64_t N;
  int32_t store;
  int32_t dim;
  int64_t device_bytes;
  int64_t build_mfma_flops;
  double build_mfma_ms;
  int64_t apply_bytes;
  int32_t top_level;
  int32_t top_fold;
} hif_info_t;
hif_status_t hif_get_info(hif_handle_t h, hif_info_t* info);

/* Timing of one stage of hif_apply with HIP events recorded around its launches on the stream
 * they run on (for bandwidth accounting).  Stages of level l (0 <= l < levels): 0 cell forward
 * (E_l^T), 1 group forward (C_l^T K_l^T), 3 group backward (K_l C_l), 4 cell backward (E_l);
 * stage 2 is the root solve (level = levels).  Launches that returned at once because PCG had
 * already converged are not counted. */
typedef struct {
  int32_t level;
  int32_t stage;
  int64_t launches;  /* launches timed since hif_profile_stage(..., enable = 1) */
  double ms;         /* their total elapsed time */
  int64_t bytes;     /* algorithmic bytes one launch moves: factor blocks in the storage
                        precision + FP64 vector and contribution traffic + int32 indices */
  char kernel[32];   /* the kernel the last timed launch used, NUL-terminated ("" if not named) */
} hif_stage_prof_t;

/* Start (enable != 0: counters reset) or stop timing the launches of (level, stage). */
hif_status_t hif_profile_stage(hif_handle_t h, int32_t level, int32_t stage, int32_t enable);

/* Totals of the timed stage so far; synchronises the device. */
hif_status_t hif_profile_read(hif_handle_t h, hif_stage_prof_t* out);

/* Releases every device allocation of the handle (synchronises the device first). */
void hif_destroy(hif_handle_t h);

/* Thread-local message describing the last non-OK status returned on this thread. */
const char* hif_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HIFCN_H */
