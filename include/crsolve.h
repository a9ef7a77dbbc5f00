/*
 * crsolve.h -- block cyclic reduction for Hermitian positive definite
 * block-tridiagonal linear systems on AMD Instinct MI355X (gfx950).
 *
 * The method follows "Review of Cyclic Reduction for Parallel Solution of
 * Hermitian Positive Definite Block-Tridiagonal Linear Systems"
 * (M. Neuenhofen, arXiv 1807.00370).
 *
 * Problem (Section 1, Eq. (Axb) and Eq. (Data)): for each system s of a batch,
 * complex blocks A_1..A_N (m x m, Hermitian), B_1..B_{N-1} (m x m; B_j is the
 * block at block row j+1, column j, and B_j^H the block at row j, column j+1)
 * and right-hand sides y_1..y_N (m x k) are given; x_1..x_N (m x k) solve
 * A x = y.  The matrix must be positive definite; when it is not, a block
 * Cholesky factorization inside the reduction breaks down (Section 2,
 * "Determination of Positive Definiteness"; Section 4) and the library
 * reports it as data in crsolve_info, not as an error code.
 *
 * MEMORY LAYOUT (all device memory, interleaved complex (re, im), row-major
 * blocks; systems of a batch are packed back to back in batch order):
 *   A : sum_s N_s m_s^2 elements;  A_j of system s is the (j-1)-th m x m block.
 *       Only the lower triangle and the real part of the diagonal are read
 *       (the Hermitian reading; the strict upper triangle and Im(diag) are
 *       ignored).
 *   B : sum_s (N_s - 1) m_s^2 elements; B_j is the (j-1)-th block.
 *   y, x, grad_x, grad_y : sum_s N_s m_s k_s elements; block j is m x k.
 *   grad_A : like A (full blocks, not Hermitian-projected); grad_B : like B.
 * Element type: CRSOLVE_C128 -> double[2], CRSOLVE_C64 -> float[2],
 * CRSOLVE_R64 -> double, CRSOLVE_R32 -> float.  With
 * CRSOLVE_PREC_FP32_REFINE the inputs and outputs are C128.
 * Every pointer must be aligned to its element size.
 *
 * OWNERSHIP: the caller owns every device buffer, including the workspace
 * (size from crsolve_workspace_size) and the crsolve_info array (one entry per
 * system).  The library never allocates device memory.  Inputs are read only.
 * The factorization lives in the workspace and stays valid until the caller
 * overwrites or frees it; a plan holds host metadata only.
 *
 * Every call that takes the workspace also takes its size in bytes, checked
 * against crsolve_workspace_size.
 *
 * STREAMS: every call enqueues its work on the given stream (a hipStream_t
 * passed as void*, NULL for the null stream) and returns without waiting,
 * except where a call's comment says it synchronizes.
 *
 * ERRORS: every call returns CRSOLVE_OK (0) when its work was enqueued, or a
 * negative code for synchronous errors, in which case nothing was enqueued:
 *   CRSOLVE_EINVAL        invalid argument (sizes < 1, NULL or misaligned
 *                         pointer, unknown enum value)
 *   CRSOLVE_EHIP          a HIP runtime call failed
 *   CRSOLVE_EWORKSPACE    workspace smaller than crsolve_workspace_size
 *   CRSOLVE_EUNSUPPORTED  combination not provided (PCR with C64 or with
 *                         FP32_REFINE; m > 256; N > 2^24 with m > 64;
 *                         N >= 2^30)
 *   CRSOLVE_ESTATE        call out of order: crsolve_solve or
 *                         crsolve_backward on a workspace that this plan
 *                         has not factored (the plan keeps a host record of
 *                         the workspace pointers passed to a successful
 *                         crsolve_factor, crsolve_check_hpd, one-sided
 *                         crsolve_factor_solve or crsolve_autotune; it
 *                         cannot see a workspace overwritten or reallocated
 *                         at the same address in between)
 * Numerical status (not positive definite) is data in crsolve_info; the
 * solution of a failed system is NaN.
 */
#ifndef CRSOLVE_H
#define CRSOLVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* C128 / C64: complex double / float.  R64 / R32: real symmetric systems
 * (the real case of Section 1: A_j symmetric, B_j real, conjugate
 * transposes become transposes) in real double / float arrays; NATIVE and
 * CR only, no crsolve_backward, no crsolve_residual.  The levels keep the
 * complex workspace layout with zero imaginary parts; the products of the
 * tiled kernels (blocks above 32) take one real MFMA per step. */
typedef enum { CRSOLVE_C128 = 0, CRSOLVE_C64 = 1, CRSOLVE_R64 = 2, CRSOLVE_R32 = 3 } crsolve_dtype;

/* NATIVE: every level in the dtype.  FP32_REFINE (C128 inputs only): the
 * reduction runs in complex FP32 except for levels with at most
 * fp64_tail_blocks blocks, which run in FP64; the solution is then refined
 * with FP64 residuals r = y - A x until ||r||_F / ||y||_F <= rtol.  A
 * system falls back to an FP64 factorization and solve of its own
 * (crsolve_info.fp64_fallback = 1) when its FP32 factorization breaks down,
 * when its residual fails to decrease from one correction to the next, or
 * when it still misses rtol after max_refine corrections.  The fallback runs
 * one system at a time in a workspace region sized for the largest system. */
typedef enum { CRSOLVE_PREC_NATIVE = 0, CRSOLVE_PREC_FP32_REFINE = 1 } crsolve_precision;

/* CR: one-sided reduction.  At each level the odd-position blocks are
 * eliminated and the even system of Eq. (even) (formulas of Eq. (Formulas))
 * is kept; the odd unknowns are recovered afterwards from the first block
 * row of the reordered system of Section 2.
 * PCR: Algorithm 1 as printed -- at each level both the odd system Eq. (odd)
 * and the even system Eq. (even) are formed (every block is eliminated for
 * its neighbours), until every block is uncoupled.  C128 and NATIVE only; it
 * keeps no factorization (use crsolve_factor_solve). */
typedef enum { CRSOLVE_SCHED_CR = 0, CRSOLVE_SCHED_PCR = 1 } crsolve_schedule;

enum {
    CRSOLVE_OK = 0,
    CRSOLVE_EINVAL = -1,
    CRSOLVE_EHIP = -2,
    CRSOLVE_EWORKSPACE = -3,
    CRSOLVE_EUNSUPPORTED = -4,
    CRSOLVE_ESTATE = -5
};

typedef struct {
    int32_t batch;            /* number of independent systems, >= 1        */
    const int32_t *N, *m, *k; /* host arrays [batch]: 1 <= N < 2^30
                                 (N <= 2^24 when m > 64), 1 <= m <= 256,
                                 k >= 1                                     */
    crsolve_dtype dtype;
    crsolve_precision precision;
    crsolve_schedule schedule;
    double rtol;              /* FP32_REFINE target, e.g. 1e-12             */
    int32_t max_refine;       /* FP32_REFINE correction cap, e.g. 30        */
    int32_t fp64_tail_blocks; /* FP32_REFINE: levels with <= this many
                                 blocks run in FP64, e.g. 8                 */
    int32_t pcr_tail_blocks;  /* CR, NATIVE: once a level holds at most this
                                 many blocks, the rest of the system is
                                 solved by Algorithm 1 in place (both half
                                 systems at every level, no back
                                 substitution for those levels; Section 3,
                                 "Time-Complexity"); the breakdown record
                                 numbers its levels on from the switch.
                                 0: one-sided throughout.  Must be 0 with
                                 FP32_REFINE; ignored by PCR.  The Python
                                 binding's default by the plan's largest
                                 block: 64 up to 32, 16 up to 64, 8 above. */
} crsolve_desc;

/* One per system, in device memory, written by factor / solve. */
typedef struct {
    int32_t status;       /* 0: positive definite, solved; 1: not positive
                             definite (a Cholesky pivot was not > 0)        */
    int32_t level;        /* level of the first breakdown (lexicographic
                             minimum over (level, block)), -1 if none       */
    int64_t block;        /* 1-based index, in the original numbering, of
                             the block row whose pivot broke down, -1       */
    int32_t refine_iters; /* FP32_REFINE: corrections applied to the
                             returned x (0 for a system that fell back)     */
    int32_t fp64_fallback;/* FP32_REFINE: 1 if the system was factored and
                             solved in FP64 (FP32 breakdown, stalled or
                             unconverged refinement)                        */
    double rel_residual;  /* FP32_REFINE: final ||y - A x||_F / ||y||_F     */
} crsolve_info;

typedef struct crsolve_plan crsolve_plan;

/* Validate a description and build a plan (host only, no device work).
 * Errors: EINVAL, EUNSUPPORTED. */
int crsolve_plan_create(const crsolve_desc *desc, crsolve_plan **out);

/* Bytes of device workspace the plan needs (factors of every level, the
 * reduced systems, right-hand-side temporaries and the level tables; for
 * FP32_REFINE also the FP64 residual and correction buffers and the FP64
 * fallback region of the largest system).  Host only. */
int crsolve_workspace_size(const crsolve_plan *plan, size_t *bytes);

/* Factor: run the matrix part of every reduction level (Section 2, phase 1
 * and 2 of the method; Eq. (Formulas) through the Section 4 recipe
 * L = chol(M), Gt = L \ G, Z = Gt^H Gt) and store the factors in ws.
 * info[s].status/level/block are written on the stream.  CR only.
 * With FP32_REFINE the call synchronizes the stream once to detect an FP32
 * breakdown and, if needed, refactors in FP64. */
int crsolve_factor(crsolve_plan *plan, const void *A, const void *B, void *ws, size_t ws_bytes,
                   crsolve_info *info, void *stream);

/* Positive-definiteness test (Section 2, "Determination of Positive
 * Definiteness", and Section 4): the block matrix is HPD if and only if
 * every Cholesky factorization of the reduction succeeds.  Runs the matrix
 * part of the levels only (no right-hand side; the levels after a
 * breakdown skip their work) and writes info[s].status = 0 (HPD) or 1 with
 * the first failing (level, block).  Same arguments, errors and stream
 * behaviour as crsolve_factor, whose factors it leaves in ws (a solve may
 * follow).  With FP32_REFINE the verdict of every system is the FP64 one:
 * after the FP32 factorization each system is factored again by its FP64
 * plan (one system at a time; the call synchronizes once per system), its
 * record is the FP64 record, and a system that fails in either precision is
 * marked in ws for the FP64 path of later solves.  CR only. */
int crsolve_check_hpd(crsolve_plan *plan, const void *A, const void *B, void *ws,
                      size_t ws_bytes, crsolve_info *info, void *stream);

/* Solve with the factors in ws: forward reduction of y through the levels,
 * then recovery of the eliminated unknowns level by level (Section 2, phase
 * 3).  A and B are read only by FP32_REFINE (FP64 residuals); they may be
 * NULL otherwise.  info (may be NULL) receives the factorization's record
 * of every system: a system whose factorization failed gets status 1 and
 * NaN in x.  CRSOLVE_ESTATE if this plan has not factored ws.
 * The solve uses a scratch region of ws that the factors do not occupy, so
 * two solves on the same ws must not overlap in time.  With
 * FP32_REFINE the call synchronizes the stream once per correction to test
 * convergence, runs the FP64 fallback of the systems that need it, and
 * writes refine_iters, fp64_fallback and rel_residual.  CR only. */
int crsolve_solve(const crsolve_plan *plan, void *ws, size_t ws_bytes, const void *A,
                  const void *B, const void *y, void *x, crsolve_info *info, void *stream);

/* Factor and solve in one pass over the levels (the right-hand side is
 * reduced together with the matrix).  Equivalent to crsolve_factor followed
 * by crsolve_solve; the only entry point of the PCR schedule. */
int crsolve_factor_solve(crsolve_plan *plan, const void *A, const void *B, const void *y,
                         void *ws, size_t ws_bytes, void *x, crsolve_info *info, void *stream);

/* crsolve_factor_solve without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  The workspace is a
 * library-owned device array of 256 MiB per GPU (present from library load
 * until the process ends; its address is looked up once per device on the
 * first call there).  The call allocates nothing: no hipMalloc, hipFree or
 * allocating library routine.  NATIVE plans whose crsolve_workspace_size
 * is at most 256 MiB (e.g. N = 4096, m = 16, k = 4); larger plans return
 * CRSOLVE_EWORKSPACE, other precisions CRSOLVE_EUNSUPPORTED, before any
 * device work.  Runs on the current device, whose stream `stream` must be;
 * launches are eager (no graph, no per-kernel timing).  Every call on a GPU
 * shares that GPU's array and leaves the last call's contents in it:
 * calls that overlap in time on one GPU (other streams, other threads)
 * race.  The factors do not stay usable for crsolve_solve. */
int crsolve_factor_solve_noalloc(crsolve_plan *plan, const void *A, const void *B, const void *y,
                                 void *x, crsolve_info *info, void *stream);

/* Adjoint of x = A^{-1} y for a real loss L with gradient grad_x = dL/dx
 * (conjugate-Wirtinger convention, as PyTorch): solves A lam = grad_x with
 * the stored factors (A is Hermitian, so A^{-H} = A^{-1}) and forms
 *   grad_y = lam,  grad_A_j = -lam_j x_j^H,
 *   grad_B_j = -(lam_{j+1} x_j^H + x_{j+1} lam_j^H).
 * x must be the solution computed with these factors.  grad_y may alias
 * nothing else.  A failed factorization gives NaN gradients.
 * CRSOLVE_ESTATE if this plan has not factored ws.  CR and NATIVE only. */
int crsolve_backward(const crsolve_plan *plan, void *ws, size_t ws_bytes, const void *x,
                     const void *grad_x, void *grad_y, void *grad_A, void *grad_B, void *stream);

/* Relative residuals ||y - A x||_F / ||y||_F of Eq. (Axb), one per system,
 * computed in FP64 on the device (Hermitian reading of A_j, Frobenius norms
 * over all N m k entries).  C128 inputs (NATIVE C128 or FP32_REFINE plans);
 * the workspace must be the plan's.  Synchronizes the stream and writes
 * rel[batch] to host memory.  EUNSUPPORTED for C64 plans. */
int crsolve_residual(const crsolve_plan *plan, void *ws, size_t ws_bytes, const void *A,
                     const void *B, const void *x, const void *y, double *rel, void *stream);

/* HIP graphs.  With graphs enabled, crsolve_factor_solve (NATIVE plans) and
 * the factor part and each solve/correction pass of FP32_REFINE plans are
 * recorded once per distinct set of pointers (A, B, y, x, ws, info) into a
 * HIP graph on a plan-owned capture stream and afterwards replayed on the
 * caller's stream (one graph launch instead of one launch per level and
 * kernel).  A recorded graph binds the workspace: it must not be used by
 * another plan or for other data while the plan lives.  The graphs contain
 * kernel nodes only.  enable = 0 releases the recorded graphs. */
int crsolve_set_graphs(crsolve_plan *plan, int enable);

/* Autotuner.  For every (block-size class, precision) present in the plan it
 * times, on the given data, the two kernel variants of each level role --
 * one-wave/MFMA kernels and work-group kernels -- for the elimination, the
 * reduced-system formation and the back substitution, and keeps the faster
 * one (synchronizes; overwrites x and the workspace).  Blocks of 33..64 have
 * one elimination and one back-substitution kernel (tiled) and two variants
 * of the reduced-system formation (16 x 16 tiles, or one wave per block), so
 * only that role is tuned for them; blocks above 64 have one kernel per role
 * and are not tuned.  When blocks of 9..32 are present it also times whole
 * steps for the launch shapes of their few-block levels -- the waves a level
 * splits its eliminations over (1024, 2048, 4096) and the block count below
 * which a reduced system is formed one wave per 16 x 16 tile (512, 1024,
 * 2048) -- and keeps the fastest pair.  The choice is returned as a short
 * text (cap bytes, NUL-terminated), one token
 * "r<role>c<class>f<fp64>=<variant>;" per tuned role plus "tw=<waves>;" and
 * "tb=<blocks>;", that crsolve_set_tuning applies to another plan, e.g. from
 * a cache file.  NATIVE plans only. */
int crsolve_autotune(crsolve_plan *plan, const void *A, const void *B, const void *y, void *ws,
                     size_t ws_bytes, void *x, void *stream, char *choice, size_t cap);
int crsolve_set_tuning(crsolve_plan *plan, const char *choice);

/* Per-kernel timing, for measurement.  While enabled, every launch the plan
 * makes is bracketed by two HIP events recorded on the launch's stream (the
 * events come from a pool owned by the plan; no device memory is allocated).
 * crsolve_timing_enable(plan, 1) enables and clears the records, 0 disables.
 * crsolve_timing_read waits for the last recorded event and fills up to cap
 * entries, one per kernel name, with the number of launches and the summed
 * event-measured durations since the last enable; *n receives the number of
 * kernel names. */
typedef struct {
    char name[32];
    int32_t launches;
    double total_ms;
} crsolve_kernel_time;

int crsolve_timing_enable(crsolve_plan *plan, int enable);
int crsolve_timing_read(crsolve_plan *plan, crsolve_kernel_time *out, int cap, int *n);

/* Release a plan (host memory only). */
int crsolve_plan_destroy(crsolve_plan *plan);

/* Static description of an error code. */
const char *crsolve_error_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* CRSOLVE_H */
