/*
 * ibmi.h -- C ABI of the MI355X (gfx950) IBMI library, libibmi.so.
 *
 * IBMI (Iterative Block Matrix Inversion; Paterson, Pestana and Dolean) refines an
 * approximation H of A^{-1} for a dense symmetric positive definite A.  The problem as the
 * paper states it (Algorithm 1): given A, a tolerance, index sets I_1..I_K and an initial
 * approximation of the inverse Schur complement on I_1^c, return the final H and the
 * number of iterations r.  Every iteration ("sweep") applies the approximate block
 * inverse of eq. (IBMI) for k = 1..K in order, always using the latest H:
 *
 *     W = A_I^{-1} A_{I,I^c}
 *     H[I,I^c] = -W H[I^c,I^c]        H[I^c,I] = H[I,I^c]^T
 *     H[I,I]   = A_I^{-1} + W H[I^c,I^c] W^T
 *
 * and H[I^c,I^c] is left unchanged.  This library checks ||I - A H||_F after each sweep.
 *
 * Conventions for every entry point:
 *  - Matrices are dense, row-major, FP64, with a leading dimension (elements between rows).
 *    A is symmetric, so for A the layout is immaterial.  H is written in full (both
 *    triangles) and is bitwise symmetric after every sweep.
 *  - Pointers named d* are device pointers (HIP device memory of the current device);
 *    all others are host pointers.
 *  - The caller owns A, H and the workspace.  The library never allocates device memory:
 *    all scratch lives in the caller's workspace, sized by ibmi_workspace_bytes().
 *  - All device work is enqueued on the plan's HIP stream.  A plan is not thread-safe;
 *    distinct plans on distinct streams may run concurrently.
 *  - Every function returns an ibmi_status; nothing else crosses the ABI.
 */
#ifndef IBMI_H_
#define IBMI_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  IBMI_OK = 0,
  IBMI_ERR_INVALID_ARG = 1,   /* bad size, pointer, partition, option                     */
  IBMI_ERR_NOT_SPD = 2,       /* a diagonal block A_{I_k} has a non-positive/NaN pivot   */
  IBMI_ERR_OUT_OF_MEMORY = 3, /* the workspace given is smaller than required            */
  IBMI_ERR_HIP = 4,           /* a HIP runtime call failed                               */
  IBMI_ERR_NONFINITE = 5      /* the residual became NaN or Inf                          */
} ibmi_status;

/* Arithmetic of the H-update products.  FP64 everywhere is the paper's method.  The other
 * forms run the large update product of each set in low precision on the matrix cores, in
 * the correction form of the same block update driven by an FP64 residual (the change made
 * to H since the residual was taken is what enters the low-precision product, so its error
 * shrinks with the iteration); block factors, the small products and the residual stay FP64.
 *   FP32_UPDATE  : FP32 operands, FP32 products and accumulation.
 *   BF16X3_UPDATE: each FP32 operand split into two bfloat16 terms, three bf16 products
 *                  (dropping lo*lo), FP32 accumulation: about 16 significant bits.
 *   BF16X6_UPDATE: three bfloat16 terms, six products: about FP32's 24 bits. */
typedef enum {
  IBMI_PREC_FP64 = 0,
  IBMI_PREC_FP32_UPDATE = 1,
  IBMI_PREC_BF16X3_UPDATE = 2,
  IBMI_PREC_BF16X6_UPDATE = 3
} ibmi_precision;

/* Initial approximation (Algorithm 1 input; only H0[I_1^c, I_1^c] is read).
 * IDENTITY is the paper's default choice.  BLOCKDIAG_INV sets H0 = blockdiag(A_{I_k}^{-1})
 * and needs disjoint sets.  GIVEN uses the caller's H as passed to ibmi_solve (resume). */
typedef enum { IBMI_INIT_IDENTITY = 0, IBMI_INIT_BLOCKDIAG_INV = 1, IBMI_INIT_GIVEN = 2 } ibmi_init;

/* Stop test after each sweep, on R = I - A H.
 * FRO:       ||R||_F < tol.
 * REL_BOUND: ||R||_F / (lambda_min * ||H||_F) < tol, a bound on the relative Frobenius error
 *            of H when lambda_min is a lower bound on the smallest eigenvalue of A (e.g. the
 *            nugget of a covariance matrix).  Loose by up to cond(A) for rounding errors.
 * REL_HR:    x / (1 - x) < tol with x = ||H R||_F / ((1 - ||R||_F) ||H||_F), also a bound on
 *            the relative Frobenius error of H (from E (R - I) = H R for E = H - A^{-1}, valid
 *            when ||R||_F < 1) and tight to first order in ||R||.  It costs a second p^3
 *            product, so it is evaluated only at some sweeps: the first with ||R||_F < 1, each
 *            one at which ||R||_F has fallen tenfold since the last evaluation, and each one at
 *            which (last bound / last ||R||_F) * ||R||_F is below tol; the stop value of the
 *            other sweeps is that prediction (inf before the first evaluation), and only an
 *            evaluated bound can stop the solve.  With fixed_sweeps the last sweep is
 *            evaluated.  Needs p * p * 8 more workspace bytes in the FP64 form. */
/* PAPER:     ||(H A)[I_K, I_K^c]||_F < tol for the last set I_K: the paper's eq. (error)
 *            estimate (the (1,2) block of H A, which vanishes at A^{-1}) in the Frobenius norm,
 *            an upper bound of the spectral norm the paper uses.  Costs a 2 b p (p - b)
 *            product per sweep on top of the residual, which is still reported. */
typedef enum {
  IBMI_STOP_FRO = 0,
  IBMI_STOP_REL_BOUND = 1,
  IBMI_STOP_REL_HR = 2,
  IBMI_STOP_PAPER = 3
} ibmi_stop;

typedef struct {
  int64_t p;               /* order of A                                                  */
  int32_t block_rows;      /* partitioner: rows per interior set (max 1024)                */
  int32_t overlap;         /* partitioner: rows shared by consecutive sets (< block_rows)  */
  const int64_t* bounds;   /* optional host array of n_blocks [start, end) pairs; NULL =   */
  int32_t n_blocks;        /*   use the partitioner.  Sets must cover [0,p), sorted by start */
  int32_t precision;       /* ibmi_precision                                               */
  int32_t init;            /* ibmi_init                                                    */
  int32_t stop;            /* ibmi_stop                                                    */
  double tol;              /* > 0                                                          */
  double lambda_min;       /* > 0 when stop = REL_BOUND                                    */
  int32_t max_sweeps;      /* >= 1; hitting it is not an error (converged = 0)             */
  int32_t stagnation_guard;/* 1: stop (floor_limited = 1) once the best stop value (the     */
                           /*    quantity compared with tol) is below 100 tol and 16      */
                           /*    sweeps in a row failed to improve it by 1%                */
  int32_t fixed_sweeps;    /* > 0: run exactly this many sweeps, ignore tol and the guard  */
  int32_t reserved;
} ibmi_options;

typedef struct {
  int32_t sweeps;          /* sweeps completed (r in Algorithm 1)                          */
  int32_t converged;       /* 1 if the stop test passed                                    */
  int32_t failed_block;    /* set index k with a bad pivot (NOT_SPD), else -1              */
  int32_t floor_limited;   /* 1 if the stagnation guard stopped the loop                   */
  double residual;         /* ||I - A H||_F after the last sweep                           */
  double stop_value;       /* the quantity compared with tol                               */
  int32_t cancelled;       /* 1 if the progress callback ended the solve early             */
  int32_t evaluations;     /* sweeps at which the REL_HR bound was evaluated               */
} ibmi_info;

typedef struct ibmi_plan_s* ibmi_plan_t;

/* Human-readable name of a status code (static string). */
const char* ibmi_status_str(ibmi_status s);

/* The default partition (host only, no device work): the multi-block overlapping sets of
 * the paper's multi-block section with end sets of m+h rows and interior sets of m+2h rows
 * (cost section).  Core stride m = block_rows - overlap, K = ceil(p/m) (K = 1 if
 * p <= block_rows), each core extended by floor(overlap/2) rows left and ceil(overlap/2)
 * rows right, clipped to [0,p); a last core shorter than overlap merges into the previous.
 * Writes up to `capacity` pairs to bounds_out (may be NULL to query) and the count to
 * *n_out.  INVALID_ARG if p < 1, block_rows < 1, overlap < 0 or overlap >= block_rows. */
ibmi_status ibmi_partition(int64_t p, int32_t block_rows, int32_t overlap,
                           int64_t* bounds_out, int32_t capacity, int32_t* n_out);

/* Device workspace (bytes) a plan with these options needs; 0 if the options are invalid.
 * Used for admission by HBM footprint. */
size_t ibmi_workspace_bytes(const ibmi_options* opts);

/* Build a plan: partition, then for every set (all sets in one launch each) the Cholesky
 * factor of A_{I_k}, A_{I_k}^{-1} (symmetrised) and W_k = A_{I_k}^{-1} A_{I_k,I_k^c}.  These
 * depend on A only, so they are computed once and reused by every sweep.
 *  dA       p x p SPD matrix, leading dimension lda >= p.  Borrowed: must stay alive and
 *           unmodified until ibmi_plan_destroy.  Must not overlap H or the workspace.
 *  dWork    device workspace of at least ibmi_workspace_bytes(opts) bytes, 256-byte
 *           aligned.  Borrowed like dA.
 *  stream   hipStream_t to enqueue on (NULL = default stream).
 * Synchronises the stream once to read the pivot status.  On NOT_SPD no plan is returned
 * and ibmi_plan_failed_block() reports the set.  *out is set only on IBMI_OK.
 * A is not scanned for NaN/Inf: one inside a diagonal block fails that set's pivot test
 * (NOT_SPD); one elsewhere reaches W and is reported by the first sweep (NONFINITE).
 * Every argument check (INVALID_ARG, OUT_OF_MEMORY) runs on the host before device work. */
ibmi_status ibmi_plan(ibmi_plan_t* out, const ibmi_options* opts, const double* dA, int64_t lda,
                      void* dWork, size_t work_bytes, void* stream);

/* Set index of the last NOT_SPD failure of ibmi_plan on this thread (-1 if none). */
int32_t ibmi_plan_failed_block(void);

/* Number of sets and their [start, end) bounds (host array of 2*n, may be NULL). */
ibmi_status ibmi_plan_blocks(ibmi_plan_t plan, int32_t* n_blocks, int64_t* bounds);

/* Run Algorithm 1: initialise H per opts->init, then sweeps until the stop test passes,
 * max_sweeps is reached or the guard fires.  dH is p x p with leading dimension ldh >= p,
 * written in place (read as well for INIT_GIVEN).  Synchronises once per sweep to read the
 * residual.  info (host, required) receives the outcome; history (host, nullable, length
 * max_sweeps or fixed_sweeps) receives ||I - A H||_F after each sweep.
 * NONFINITE if the residual is NaN/Inf (H then holds the offending iterate). */
ibmi_status ibmi_solve(ibmi_plan_t plan, double* dH, int64_t ldh, ibmi_info* info, double* history);

/* Progress callback of ibmi_solve: called on the calling thread after every sweep with the
 * number of sweeps done, ||I - A H||_F and the stop value.  A nonzero return ends the solve
 * after that sweep (status OK, converged = 0, cancelled = 1).  fn = NULL removes it. */
typedef int32_t (*ibmi_progress_fn)(int32_t sweep, double residual, double stop_value,
                                    void* user);
ibmi_status ibmi_set_progress(ibmi_plan_t plan, ibmi_progress_fn fn, void* user);

/* One sweep (sets k = 1..K in order) in the plan's precision form, then ||I - A H||_F written
 * to *residual (host, nullable); synchronises once.  The low-precision update forms carry
 * the residual matrix of the previous sweep in the workspace: pass restart = 1 on the first
 * call for an H, or whenever H was changed by anything but ibmi_sweep on this plan.
 * NONFINITE if the residual is NaN/Inf. */
ibmi_status ibmi_sweep(ibmi_plan_t plan, double* dH, int64_t ldh, int32_t restart,
                       double* residual);

/* Enqueue one application of eq. (IBMI) for set k (0-based) on dH in FP64, with no
 * synchronisation, whatever the plan's precision.  Reads H[I_k^c, I_k^c], writes rows and
 * columns I_k. */
ibmi_status ibmi_block_step(ibmi_plan_t plan, double* dH, int64_t ldh, int32_t k);

/* Enqueue the initial H of opts->init (IDENTITY or BLOCKDIAG_INV; GIVEN leaves dH as is). */
ibmi_status ibmi_init_h(ibmi_plan_t plan, double* dH, int64_t ldh);

/* ||I - A H||_F for the plan's A (FP64, deterministic fixed-order reduction).  Synchronises
 * the plan's stream and writes the value to *out (host). */
ibmi_status ibmi_residual(ibmi_plan_t plan, const double* dH, int64_t ldh, double* out);

/* Kernel timing, for measurement.  While enabled, launches are bracketed by HIP events on the
 * plan's stream in three categories.  FP64 form: 0 = panel GEMM V = W H[I^c,I^c] with its
 * scatter into H (2 b c^2 flops), 1 = diagonal update (split-K W H[I^c,I] and H[I,I];
 * 2 b^2 c), 2 = residual (2 p^3).  Low-precision forms: 0 = the update product
 * R[I,:] - A[I,:] D in FP32 or split bfloat16 (2 b (u p + (p-u) u) FP32-level flops, u = rows
 * already updated in the sweep; the split forms' partial-sum pass included), 1 = the FP64
 * corrections of the set (4 b^2 c + 2 b^3), 2 = residual with its store (2 p^3).  The
 * REL_HR and PAPER stop evaluations are not timed.
 * ibmi_kernel_times synchronises the stream, then returns and resets, per category:
 * accumulated milliseconds, launch counts and flops.  Host arrays of length 3; any may be NULL. */
ibmi_status ibmi_set_profiling(ibmi_plan_t plan, int32_t on);
ibmi_status ibmi_kernel_times(ibmi_plan_t plan, double* ms, int64_t* launches, double* flops);

/* Release the host-side plan object.  Does not free A or the workspace (caller-owned). */
ibmi_status ibmi_plan_destroy(ibmi_plan_t plan);

/* ---------------------------------------------------------------------------------------
 * Batched form: many independent SPD matrices of uneven order solved together.  All
 * matrices share block_rows, overlap, tol, max_sweeps and the stagnation guard of opts
 * (init = IDENTITY, stop = FRO, precision = FP64).  Every sweep of every matrix is one
 * replay of a captured HIP graph: per set index j, one grouped launch of the panel products
 * of set j of all matrices, one grouped split-K diagonal launch and one grouped
 * finalisation; then a grouped residual, a per-matrix reduction and an on-device stop test
 * that marks converged or capped matrices inactive.  Inactive matrices are skipped by every
 * later kernel, so their H stays at the sweep where they stopped.
 * --------------------------------------------------------------------------------------- */
typedef struct ibmi_batch_s* ibmi_batch_t;

/* Workspace bytes for n matrices of orders p[0..n) (host array). 0 if invalid. */
size_t ibmi_batch_workspace_bytes(int32_t n, const int64_t* p, const ibmi_options* opts);

/* Plan the batch: block factors of every set of every matrix (one launch per stage).
 *  dA     host array of n device pointers; matrix i is p[i] x p[i] with leading dimension
 *         lda[i] >= p[i].  Borrowed until ibmi_batch_destroy.
 *  dWork  device workspace, 256-byte aligned, >= ibmi_batch_workspace_bytes bytes.
 * NOT_SPD if any diagonal block of any matrix has a bad pivot. */
ibmi_status ibmi_batch_plan(ibmi_batch_t* out, int32_t n, const int64_t* p,
                            const double* const* dA, const int64_t* lda, const ibmi_options* opts,
                            void* dWork, size_t work_bytes, void* stream);

/* Solve all matrices: H_i = I, then graph replays until every matrix has converged, hit
 * max_sweeps or stopped on the guard.  dH: host array of n device pointers (p[i] x p[i],
 * leading dimension ldh[i]).  infos: host array of n.  The task tables and the graph are
 * built on the first call and rebuilt only when the H pointers or the tuning change.
 * NONFINITE if some residual became NaN/Inf (its info shows which). */
ibmi_status ibmi_batch_solve(ibmi_batch_t batch, double* const* dH, const int64_t* ldh,
                             ibmi_info* infos);

/* Tile configurations (0 <= cfg < 11; see the GEMM configuration table in the sources) of
 * the grouped panel, diagonal and residual launches; INVALID_ARG outside that range.  A new
 * choice takes effect at the next ibmi_batch_solve (the graph is captured again). */
ibmi_status ibmi_batch_set_tuning(ibmi_batch_t batch, int32_t panel, int32_t diag,
                                  int32_t resid);
ibmi_status ibmi_batch_get_tuning(ibmi_batch_t batch, int32_t* cfg3);

/* Autotuner: times `reps` graph replays (sweeps from H = I) for each candidate set of tile
 * configurations on these H buffers, keeps the fastest, and returns it (cfg3, host array of
 * 3) with its time per sweep in ms.  H contents are overwritten. */
ibmi_status ibmi_batch_autotune(ibmi_batch_t batch, double* const* dH, const int64_t* ldh,
                                int32_t reps, int32_t* cfg3, double* ms_per_sweep);

/* Release the batch object with its task tables and captured graph (ibmi_batch_solve and
 * ibmi_batch_autotune synchronise before they return, so no replay is in flight between
 * calls).  A, H and the workspace are the caller's and stay untouched.  INVALID_ARG for a
 * NULL batch. */
ibmi_status ibmi_batch_destroy(ibmi_batch_t batch);

#ifdef __cplusplus
}
#endif
#endif /* IBMI_H_ */
