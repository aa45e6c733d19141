/*
 * hqr.h -- C ABI of the MI355X (gfx950) tiled hierarchical Householder QR.
 *
 * The library factors a dense double-precision M x N matrix (M >= N) with the
 * tiled QR algorithms of Dongarra, Faverge, Herault, Langou and Robert,
 * "Hierarchical QR factorization algorithms for multi-core cluster systems":
 * the matrix is cut into b x b tiles, every tile below the diagonal is zeroed
 * by an elimination elim(i, killer(i,k), k) (Section II, Algorithm 1), each
 * elimination runs as tile kernels GEQRT/UNMQR + TSQRT/TSMQR or TTQRT/TTMQR
 * (Algorithm 2), and the order of eliminations -- the elimination list -- is
 * produced by the reduction trees of Section III and their hierarchical
 * composition of Section IV.  All kernels of one factorization run inside a
 * single persistent GPU launch that fires each task when its input tiles are
 * ready (Section IV-B, "Execution scheme").
 *
 * Conventions shared by every entry point
 *   - Matrices are column-major with a leading dimension (LAPACK layout):
 *     element (r, c) of A is dA[r + c * lda].
 *   - Device pointers are HIP device memory of the current device; the caller
 *     owns them.  Host pointers are ordinary host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls that take a stream only enqueue work on it and return before the
 *     GPU has finished; results are valid once the stream is synchronized.
 *   - Return value 0 is success.  A negative value -i means argument i
 *     (1-based) is invalid and nothing was enqueued.  Positive values are
 *     runtime failures (see hqr_strerror).  No C++ exception crosses the ABI.
 */
#ifndef HQR_H_
#define HQR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Reduction-tree kinds (Section III: flat tree / Sameh-Kuck, binary tree,
 * Greedy; Fibonacci is named in Sections III-C and V; CHAIN is the "domino"
 * coupling tree of Section IV-B). */
enum {
  HQR_FLAT = 0,
  HQR_BINARY = 1,
  HQR_GREEDY = 2,
  HQR_FIBONACCI = 3,
  HQR_CHAIN = 4
};

/* Elimination kinds (Section II: TS = triangle on top of square, TT =
 * triangle on top of triangle). */
enum { HQR_KIND_TS = 0, HQR_KIND_TT = 1 };

/* Runtime error codes (positive). */
enum {
  HQR_ERR_HIP = 1,        /* a HIP runtime call failed */
  HQR_ERR_WATCHDOG = 2,   /* a task waited longer than the spin limit; results are invalid */
  HQR_ERR_WORKSPACE = 3,  /* workspace too small */
  HQR_ERR_NOMEM = 4,      /* host or device allocation for the task plan failed */
  HQR_ERR_INTERNAL = 5,   /* internal inconsistency (bug) */
  HQR_ERR_INVALID_LIST = 6, /* an elimination list breaks the rules of Section II */
  HQR_ERR_TIMEOUT = 7,      /* hqr_status_ex: the stream did not finish in time */
  HQR_ERR_SINGULAR = 8,     /* hqr_lstsq: R has a zero diagonal entry (reported by hqr_status) */
  HQR_ERR_FACTORS = 9       /* apply/solve: the workspace does not hold the factorization its arguments
                               describe (other shape, tile size, tree or precision, or none); nothing was
                               applied (reported by hqr_status on the apply workspace) */
};

/* Arithmetic of the tile kernels (hqr_params.precision). */
enum {
  HQR_PREC_FP64 = 0, /* FP64 tiles, FP64 MFMA (hqr_factor, hqr_lstsq, batches) */
  HQR_PREC_FP32 = 1, /* FP32 tiles, FP32 MFMA (hqr_factor_f32, hqr_lstsq_ir) */
  HQR_PREC_BF16 = 2  /* FP32 tiles; the block-reflector products take their operands rounded to BF16
                        and accumulate in FP32 on the BF16 MFMA (hqr_factor_f32, hqr_lstsq_ir) */
};

/* Parameters of the hierarchical algorithm (Section IV-A and V-A).
 *   nb        tile size b: 64, 128 or 256.
 *   ib        inner blocking of the tile kernels; must be 16.
 *   p         virtual clusters of the cyclic row mapping (>= 1): row i goes to
 *             cluster i mod p with local index i / p.
 *   a         TS domain size in tiles (>= 1); a = 1 means TT kernels only,
 *             a >= number of tile rows with p = 1 is the flat tree with TS
 *             kernels.
 *   low       level-1 tree inside a cluster (FLAT, BINARY, GREEDY, FIBONACCI).
 *   high      level-3 tree over the p top tiles of a panel (same choices).
 *   coupling  level-2 tree (CHAIN is the domino scheme; any tree is allowed).
 *   domino    1 = coupling level on, 0 = off.
 *   precision HQR_PREC_*: FP64 for the double entry points; for the float
 *             ones (hqr_factor_f32, hqr_lstsq_ir) FP32 (0 is read as FP32
 *             there) or BF16 operands with FP32 accumulation.  It does not
 *             change the elimination list or the task graph. */
typedef struct hqr_params {
  int32_t nb;
  int32_t ib;
  int32_t p;
  int32_t a;
  int32_t low;
  int32_t high;
  int32_t coupling;
  int32_t domino;
  int32_t precision;
} hqr_params;

/* A finished factorization as seen from the host: the shape, parameters and
 * precision given to hqr_factor / hqr_factor_f32 / hqr_lstsq, and the
 * workspace that holds its T factors and factored tiles.  It points into that
 * workspace (and the tiles copied back into dA) without owning them: keep the
 * workspace unchanged while the handle is used.  Created by those entry
 * points when their `out` argument is not NULL; freed by
 * hqr_factors_destroy.  The handle is host memory only. */
typedef struct hqr_factors hqr_factors;

/* Execution controls of the persistent scheduler (not part of the algorithm).
 *   workers     persistent workgroups; 0 = one per free slot on the device
 *               (2 per compute unit); 1 = one workgroup that runs the tasks
 *               strictly in list order.  Any value gives bitwise identical
 *               results.
 *   order       0 = tasks are handed out by a critical-path priority order
 *               (a topological order of the task graph); 1 = in the canonical
 *               program order of Algorithm 2.
 *   spin_limit  polls of the dependency counters of one task before the
 *               launch is aborted (every workgroup stops taking tasks) and
 *               HQR_ERR_WATCHDOG is reported; 0 = a built-in limit of a few
 *               seconds of polling.
 *   ev_begin, ev_end  NULL, or hipEvent_t handles (created by the caller)
 *               recorded on the call's stream right before and right after
 *               the persistent launch of a factorization (hqr_factor,
 *               hqr_factor_f32, hqr_lstsq, hqr_batch_run): the time between
 *               them is the tile kernels' alone, without the copies into and
 *               out of the workspace. */
typedef struct hqr_exec {
  int32_t workers;
  int32_t order;
  int64_t spin_limit;
  void* ev_begin;
  void* ev_end;
} hqr_exec;

/* One elimination elim(victim, killer, k) (Section II).  `level` is the
 * hierarchical level 0..3 of Section IV-B (0 = TS domain, 1 = low tree,
 * 2 = coupling, 3 = high tree); `round` is the round of the tree that
 * produced it (the unit-time step for Greedy). */
typedef struct hqr_elim {
  int32_t k, victim, killer, kind, level, round;
} hqr_elim;

/* Summary of the kernel task graph of an elimination list (Algorithm 2). */
typedef struct hqr_dag_info {
  int64_t eliminations;   /* records in the list */
  int64_t tasks;          /* GEQRT+UNMQR+TSQRT+TSMQR+TTQRT+TTMQR tasks (unsplit) */
  int64_t count[6];       /* per kernel, in that order */
  int64_t weight;         /* sum of kernel weights in units of b^3/3 flops */
  int64_t critical_path;  /* longest weighted path through the task graph */
  int64_t device_tasks;   /* tasks after column-chunk splitting of the updates */
} hqr_dag_info;

/* Elimination list of the hierarchical algorithm (Sections III and IV) for a
 * matrix of mt x nt tiles, in canonical order: panel by panel; inside a
 * panel level 0 by (cluster, killer, victim), levels 1 and 2 by (cluster,
 * round, victim), level 3 by (round, victim).
 *   out    host array of `cap` records, or NULL to only count.
 *   count  receives the number of records (sum over k < min(mt,nt) of
 *          mt - k - 1).
 * Errors: -1/-2 if mt or nt < 1, -3 for bad params, -5 if out != NULL and
 * cap is too small (count is still set). */
int hqr_elimlist(int32_t mt, int32_t nt, const hqr_params* params, hqr_elim* out, int64_t cap,
                 int64_t* count);

/* Check a host elimination list against the rules of Section II: every tile
 * (i,k) below the diagonal killed exactly once; when elim(i, piv, k) runs,
 * rows i and piv are zero in every panel k' < k and piv is not yet killed in
 * panel k; a TS victim is never a killer in its panel.  Returns 0 if valid,
 * HQR_ERR_INVALID_LIST otherwise, -1..-4 for bad arguments. */
int hqr_elimlist_validate(int32_t mt, int32_t nt, const hqr_elim* list, int64_t count);

/* Task-graph summary for (mt, nt, params) (Algorithm 2 expansion; weights of
 * Section II: GEQRT 4, UNMQR 6, TSQRT 6, TSMQR 12, TTQRT 2, TTMQR 6). */
int hqr_dag_stats(int32_t mt, int32_t nt, const hqr_params* params, hqr_dag_info* out);

/* One task of the persistent launch, as the device reads it.  op: 0 GEQRT,
 * 1 UNMQR, 2 TSQRT, 3 TSMQR, 4 TTQRT, 5 TTMQR (Algorithm 2).  `chunk` is the
 * 64-column chunk of an update task (tile columns are split into nb/64
 * chunks).  `row` is the tile row of GEQRT/UNMQR or the victim of a kill,
 * `killer` the killer row (= row for GEQRT/UNMQR), `k` the panel, `j` the
 * updated tile column (= k for panel tasks); for a panel task `chunk` is the
 * number of column chunks of tile column k that hold matrix columns (chunks
 * of zero padding are never touched).  Before running, the task waits
 * until the dependency counters of the tiles it touches reach v[0..2]:
 *   GEQRT  chunks 0..chunk-1 of (row,k) >= v0
 *   UNMQR  (row,k) chunk 0 >= v0, (row,j) chunk `chunk` >= v1
 *   TSQRT/TTQRT  chunks 0..chunk-1 of (killer,k) >= v0 and of (row,k) >= v1
 *   TSMQR/TTMQR  (row,k) chunk 0 >= v0, (killer,j) and (row,j) chunk
 *                `chunk` >= v1 and v2
 * and afterwards bumps by one the counters of the tiles (chunks) it wrote. */
typedef struct hqr_task {
  uint8_t op, chunk;
  uint16_t row, killer, k, j, pad;
  uint32_t v[3];
} hqr_task;

/* Task table of the persistent launch for (mt, nt, params) in dispatch order
 * (order 0: critical-path priority; 1: program order).  out may be NULL to
 * count.  Errors: -1..-4 bad arguments, -6 cap too small. */
int hqr_plan_tasks(int32_t mt, int32_t nt, const hqr_params* params, int32_t order, hqr_task* out, int64_t cap,
                   int64_t* count);

/* Bytes of device workspace hqr_factor needs for an M x N matrix: the T
 * factors of every tile kernel, the per-tile dependency counters, a status
 * word and a tile-contiguous copy of A (each nb x nb tile stored
 * contiguously, zero-padded beyond M and N) that the kernels work on. */
int hqr_workspace_size(int64_t M, int64_t N, const hqr_params* params, size_t* bytes);

/* QR factorization A = Q R (Section II; the result is the Householder QR of
 * the whole matrix, reached through the elimination list of `params`).
 *   dA      device, M x N, lda >= M; overwritten: R in the upper triangle of
 *           the leading N x N block, Householder vectors of every tile kernel
 *           elsewhere.  Q is never formed.
 *   M >= N >= 1.
 *   dwork   device workspace of at least hqr_workspace_size bytes; it holds
 *           the T factors and the factored tiles, so keep it unchanged while
 *           the factorization is used (hqr_apply_qt).  Any alignment of dA
 *           and any lda >= M are accepted: the kernels work on the workspace's
 *           tile-contiguous copy, filled from dA before the launch and copied
 *           back after it, on `stream`.
 *   exec    NULL for defaults.
 *   out     NULL, or receives a new hqr_factors handle of this
 *           factorization (for hqr_factors_apply_qt / _apply_q / _solve);
 *           free it with hqr_factors_destroy.  Set only on success.
 * Errors: -1 if dA is NULL, -2 if M < N or M < 1 (or more than 65535 tile
 * rows), -3 if N < 1, -4 if lda < M, -5 bad params (or precision not FP64),
 * -6 bad exec.order, -7 if dwork is NULL, -8 workspace too small;
 * HQR_ERR_NOMEM if the handle cannot be allocated.  Runtime failures inside
 * the launch (watchdog) are reported by hqr_status.
 * Ownership: the caller owns dA and dwork.  The first call for a given (tile
 * grid, params, exec.order) builds the task plan on the host and uploads it
 * to device memory that the library allocates itself (hipMalloc, about 24
 * bytes per task) and keeps until hqr_release_plans; this is the only device
 * memory the library allocates on this path. */
int hqr_factor(double* dA, int64_t M, int64_t N, int64_t lda, const hqr_params* params,
               const hqr_exec* exec, void* dwork, size_t work_bytes, void* stream, hqr_factors** out);

/* ---- Single precision ----
 *
 * The same tiled algorithm, elimination lists and persistent launch with
 * FP32 tiles and FP32 arithmetic (tile kernels on v_mfma_f32_16x16x4f32).
 * Workspace bytes of hqr_factor_f32 (tiles and T factors in float).  Errors
 * as hqr_workspace_size. */
int hqr_workspace_size_f32(int64_t M, int64_t N, const hqr_params* params, size_t* bytes);

/* QR of the column-major float matrix dA (M x N, lda >= M) in place, as
 * hqr_factor: R in the upper triangle, the Householder vectors below it,
 * the T factors (float) in dwork.  params->precision selects FP32 (0 or 1)
 * or BF16 operands with FP32 accumulation (2) for the block-reflector
 * products.  out as for hqr_factor.  Errors as hqr_factor. */
int hqr_factor_f32(float* dA, int64_t M, int64_t N, int64_t lda, const hqr_params* params, const hqr_exec* exec,
                   void* dwork, size_t work_bytes, void* stream, hqr_factors** out);

/* Bytes of the second workspace that hqr_apply_qt and hqr_apply_q need for a
 * right-hand side B of M rows and nrhs columns: a
 * status word, one dependency counter per block and B in blocks of nb rows x
 * 64 columns (zero-padded).  Errors: -1 M < 1, -2 nrhs < 1, -3 bad params. */
int hqr_apply_workspace_size(int64_t M, int32_t nrhs, const hqr_params* params, size_t* bytes);

/* B <- Q^T B with the Q of a finished hqr_factor (Section I: the update
 * kernels UNMQR/TSMQR/TTMQR of Algorithm 2 replayed on B in the order of the
 * elimination list).
 *   M, N, params  exactly those given to hqr_factor.
 *   dwork         the factorization's workspace (read only: V tiles, T).
 *   dB            device, M x nrhs, column-major, ldb >= M; overwritten.
 *   bwork         device workspace of hqr_apply_workspace_size(M, nrhs)
 *                 bytes (scratch; its status word is read by hqr_status).
 * Asynchronous on `stream`, which must be the factorization's stream or
 * ordered after it.  dwork may be the workspace of hqr_factor or of
 * hqr_lstsq (any nrhs) with the same (M, N, params): the T factors and
 * tiles sit at the same offsets in both.  The launch first compares the
 * signature that the factorization wrote into dwork's control words with
 * (M, N, params); on a mismatch nothing is applied, B is left as it was, and
 * hqr_status(bwork) reports HQR_ERR_FACTORS.  Errors: -2 M < N or M < 1, -3
 * N < 1, -4 bad params, -6 dwork NULL, -7 work_bytes too small for (M, N),
 * -8 dB NULL, -9 ldb < M, -10 nrhs < 1, -11 bwork NULL, -12 bwork too
 * small. */
int hqr_apply_qt(int64_t M, int64_t N, const hqr_params* params, const hqr_exec* exec, const void* dwork,
                 size_t work_bytes, double* dB, int64_t ldb, int32_t nrhs, void* bwork, size_t bwork_bytes,
                 void* stream);

/* B <- Q B (the transformations in reverse order, each one untransposed).
 * Arguments and errors as hqr_apply_qt. */
int hqr_apply_q(int64_t M, int64_t N, const hqr_params* params, const hqr_exec* exec, const void* dwork,
                size_t work_bytes, double* dB, int64_t ldb, int32_t nrhs, void* bwork, size_t bwork_bytes,
                void* stream);

/* Bytes of device workspace hqr_lstsq needs: that of hqr_factor plus the
 * right-hand sides as further (zero-padded) tile columns.  Errors: -1 M < N
 * or M < 1, -2 N < 1, -3 nrhs < 1, -4 bad params. */
int hqr_lstsq_workspace_size(int64_t M, int64_t N, int32_t nrhs, const hqr_params* params, size_t* bytes);

/* Least squares min ||A x - b|| for each column of B (M >= N, A of full
 * rank).  B is carried through the factorization as further tile columns,
 * so the update kernels transform it by Q^T inside the same persistent
 * launch (no second pass over the Householder vectors); then
 * x = R^{-1} (Q^T B)(0:N) by back substitution with the leading N x N block
 * of R (one launch, a workgroup per right-hand-side column).  On return (after the stream) A holds the
 * factorization as after hqr_factor, B(0:N, :) the solutions and B(N:M, :)
 * the components of Q^T B whose norm is the residual norm.  dwork:
 * hqr_lstsq_workspace_size bytes; it also holds Q's factors for
 * hqr_apply_qt with the same (M, N, params).  A zero diagonal entry of R is
 * reported by hqr_status(dwork) as HQR_ERR_SINGULAR with detail[0] = its
 * index (the solution is then not finite).  Errors: -1 dA NULL, -2 M < N or
 * M < 1, -3 N < 1, -4 lda < M, -5 dB NULL, -6 ldb < M, -7 nrhs < 1, -8 bad
 * params, -9 bad exec.order, -10 dwork NULL, -11 dwork too small.  out
 * (may be NULL) receives a handle of the factorization, as for
 * hqr_factor. */
int hqr_lstsq(double* dA, int64_t M, int64_t N, int64_t lda, double* dB, int64_t ldb, int32_t nrhs,
              const hqr_params* params, const hqr_exec* exec, void* dwork, size_t work_bytes, void* stream,
              hqr_factors** out);

/* ---- Factorization handles ----
 *
 * The same operations as hqr_apply_qt / hqr_apply_q / hqr_solve, with the
 * shape, parameters, precision and workspace taken from a handle instead of
 * repeated by the caller.  bwork: hqr_factors_apply_workspace_size bytes.
 * Errors: -1 f NULL, -3 dB NULL, -4 ldb < M, -5 nrhs < 1, -6 bwork NULL,
 * -7 bwork too small; hqr_factors_solve returns -1 for FP32/BF16 factors
 * (it solves with a double R).  A workspace overwritten by another
 * factorization since the handle was made is reported as for hqr_apply_qt. */
int hqr_factors_apply_workspace_size(const hqr_factors* f, int32_t nrhs, size_t* bytes);
int hqr_factors_apply_qt(const hqr_factors* f, const hqr_exec* exec, double* dB, int64_t ldb, int32_t nrhs,
                         void* bwork, size_t bwork_bytes, void* stream);
int hqr_factors_apply_q(const hqr_factors* f, const hqr_exec* exec, double* dB, int64_t ldb, int32_t nrhs,
                        void* bwork, size_t bwork_bytes, void* stream);
int hqr_factors_solve(const hqr_factors* f, const hqr_exec* exec, double* dB, int64_t ldb, int32_t nrhs,
                      void* bwork, size_t bwork_bytes, void* stream);
/* Shape, parameters (precision included) and workspace of a handle; any
 * output may be NULL.  Errors: -1 f NULL. */
int hqr_factors_query(const hqr_factors* f, int64_t* M, int64_t* N, hqr_params* params, const void** dwork,
                      size_t* work_bytes);
/* Frees the handle (NULL is ignored); the workspace and dA are untouched. */
void hqr_factors_destroy(hqr_factors* f);

/* ---- Least squares without device allocation ----
 *
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): hqr_lstsq
 * with its workspace and task plan held in a static device array of
 * HQR_NOALLOC_SCRATCH_BYTES that the library's code object carries (each
 * device the library runs on holds its own copy until the process ends).
 * The call makes no hipMalloc, hipFree or other device allocation; on the
 * first call for a shape and tree it builds the task plan in host memory,
 * and it uploads the plan into the array whenever the previous call on the
 * device used another one.  All calls on one device share the array and it
 * keeps the last call's contents: calls that overlap in time on one device
 * (two streams, or two host threads) race and give wrong results; calls
 * ordered on one stream are safe.
 *   dA, M, N, lda, dB, ldb, nrhs, params, exec  as for hqr_lstsq: on return
 *           (after the stream) A holds R and V, B(0:N, :) the solutions.
 *   dinfo   NULL, or 8 int32 of device memory that receive, after the
 *           call's work, the status word (0, HQR_ERR_WATCHDOG or
 *           HQR_ERR_SINGULAR) in dinfo[0] and the detail of hqr_status_ex
 *           in dinfo[1..4].
 * The factorization stays in the array only until the next call, so no
 * handle is returned.  Errors: as hqr_lstsq for arguments -1 .. -9;
 * HQR_ERR_WORKSPACE (nothing enqueued, message in hqr_last_error) when the
 * workspace of hqr_lstsq_workspace_size plus the task plan (24 bytes per
 * task) exceeds HQR_NOALLOC_SCRATCH_BYTES (64 MiB: 8192 x 512 or 4096 x
 * 1024 at nb = 256 with one right-hand side fit, 16384 x 512 does not). */
#define HQR_NOALLOC_SCRATCH_BYTES (64u << 20)
int hqr_lstsq_noalloc(double* dA, int64_t M, int64_t N, int64_t lda, double* dB, int64_t ldb, int32_t nrhs,
                      const hqr_params* params, const hqr_exec* exec, int32_t* dinfo, void* stream);

/* ---- Mixed-precision least squares ----
 *
 * min ||A x - b|| for a double A (M x N, M >= N, full rank) and one
 * right-hand side: A is rounded to float and factored by the FP32 tiled QR
 * (as hqr_factor_f32, with b carried along as a further tile column so that
 * the factorization also forms Q^T b); the first iterate is the FP32
 * solution x = R^{-1} (Q^T b)(0:N) with r = b - A x in FP64; then the
 * augmented system [I A; A^T 0][r; x] = [b; 0]
 * is refined (Bjorck's iterative refinement for least squares): each
 * iteration forms f = b - r - A x and g = -A^T r in FP64 from the original
 * double A, solves the correction with the FP32 factors (Q applied in FP32,
 * triangular solves with the float R in FP64 arithmetic) and updates x and r
 * in FP64.  It converges when the condition number of A times the float
 * unit roundoff (6e-8) is well below 1. */
typedef struct hqr_ir_info {
  int32_t iterations;  /* corrections applied, the FP32 solution counted as the first */
  int32_t converged;   /* 1 when eta <= tol */
  double eta;          /* backward error of the returned (x, r), see hqr_lstsq_ir */
  double history[32];  /* eta before each of the first 32 corrections (history[0] = 1: x = r = 0;
                          history[1] = eta of the FP32 solution) */
  int32_t history_len; /* entries of history written (a last one larger than the one before it is the
                          eta of a rejected correction) */
} hqr_ir_info;

/* Workspace bytes of hqr_lstsq_ir (FP32 factorization, one FP32 block
 * column for Q, and FP64 vectors).  Errors: -1 M < 1 or M < N, -2 N < 1, -3
 * bad params, -4 bytes NULL. */
int hqr_lstsq_ir_workspace_size(int64_t M, int64_t N, const hqr_params* params, size_t* bytes);

/* Solves min ||A x - b||: dA (lda >= M) and db (M) are read only; dx (N)
 * receives x, dr (M, may be NULL) the residual r of the augmented system
 * (b - A x at convergence).  The iterate is judged by the normwise backward
 * error of the augmented system, eta = sqrt(||f||^2 + ||g||^2) /
 * (||A||_F (||x|| + ||r||) + ||b||); the loop stops when eta <= tol, when
 * a correction did not lower eta (the iterate before that correction is
 * returned, with its eta), or after max_iter corrections; info (may be
 * NULL) reports the count of corrections kept and the eta history.  The forward error of x
 * is about kappa(A) times the final eta: tol near the FP64 unit roundoff
 * (1e-15) gives FP64 accuracy.  Synchronizes `stream` once per correction (eta is read on the
 * host).  Errors: -1 dA NULL, -2 M < N or
 * M < 1, -3 N < 1, -4 lda < M, -5 db NULL, -6 dx NULL, -8 bad params, -9 bad
 * exec.order, -10 max_iter < 1, -11 tol < 0 or NaN, -12 dwork NULL, -13
 * dwork too small; HQR_ERR_WATCHDOG if a launch was aborted. */
int hqr_lstsq_ir(const double* dA, int64_t M, int64_t N, int64_t lda, const double* db, double* dx, double* dr,
                 const hqr_params* params, const hqr_exec* exec, int32_t max_iter, double tol, void* dwork,
                 size_t work_bytes, void* stream, hqr_ir_info* info);

/* ---- Batched problems (one persistent launch for many small QRs) ----
 *
 * Many independent factorizations or least-squares solves, each with its own
 * shape (M_q x N_q, M_q >= N_q) and right-hand sides, run as one batch: one
 * copy-in launch, one persistent launch whose task list is the union of the
 * problems' task graphs (Algorithm 2 per problem, merged by the same
 * critical-path priority that orders one problem's tasks, each problem's own
 * order kept), one back-substitution launch and one copy-out launch.  All
 * problems of a batch share one hqr_params (one tile size nb).  The batch
 * object holds the host plan; the caller owns every device buffer.  Results
 * per problem are those of hqr_lstsq (nrhs_q > 0) or hqr_factor (nrhs_q = 0)
 * on that problem alone. */
typedef struct hqr_batch hqr_batch;

/* Plans a batch of `count` (1..65535) problems: M[q] x N[q] matrices with
 * nrhs[q] right-hand sides each (nrhs may be NULL: no right-hand sides,
 * factorization only).  Host memory only; nothing is enqueued.  Errors: -1
 * count out of range, -2 M NULL or some M[q] < 1 (or too many tile rows), -3
 * N NULL or some N[q] < 1 or > M[q], -4 some nrhs[q] < 0, -5 bad params, -6
 * bad exec.order, -7 out NULL. */
int hqr_batch_create(int32_t count, const int64_t* M, const int64_t* N, const int32_t* nrhs,
                     const hqr_params* params, const hqr_exec* exec, hqr_batch** out);

/* Device workspace bytes of the batch (control words, per-problem status,
 * dependency counters, task list, and per problem the T factors and the
 * tiles of A and B).  Errors: -1 b NULL, -2 bytes NULL. */
int hqr_batch_workspace_size(const hqr_batch* b, size_t* bytes);

/* The merged task list of the batch in dispatch order (records as
 * hqr_plan_tasks) and the problem index of each task; either output may be
 * NULL, both NULL only counts.  Errors: -1 b NULL, -4 cap too small, -5
 * count NULL. */
int hqr_batch_num_tasks(const hqr_batch* b, hqr_task* tasks, int32_t* prob, int64_t cap, int64_t* count);

/* Binds the caller's matrices to the batch: host arrays of `count` device
 * pointers dA[q] (column-major, leading dimension lda[q] >= M[q]) and dB[q]
 * (ldb[q] >= M[q]; dB and ldb may be NULL when no problem has right-hand
 * sides, and dB[q] is ignored when nrhs[q] = 0), and the workspace dwork.
 * Enqueues on `stream` the upload of the problem descriptors and the task
 * list into dwork (from library-owned pinned host memory).  Not
 * graph-capturable; the batch may be run any number of times after one
 * bind.  Errors: -1 b NULL, -2 dA NULL or an entry NULL, -3 lda NULL or an
 * entry < M[q], -4 dB missing where needed, -5 ldb missing or an entry <
 * M[q], -6 dwork NULL, -7 work_bytes too small. */
int hqr_batch_bind(hqr_batch* b, double* const* dA, const int64_t* lda, double* const* dB, const int64_t* ldb,
                   void* dwork, size_t work_bytes, void* stream);

/* Runs the bound batch on `stream`: copies every A_q (and B_q) into the
 * workspace, factors all problems in one persistent launch, solves
 * R_q x = (Q_q^T B_q)(0:N_q) for problems with right-hand sides, and copies
 * A_q (R and V as after hqr_factor) and B_q (x in rows 0..N_q-1, the
 * residual components below) back.  Only kernel launches are enqueued (no
 * host work, copies or memsets), so the call can be captured into a HIP
 * graph and replayed; each replay starts again from the caller's A_q and
 * B_q.  Errors: -1 b NULL, -2 dwork NULL or not the workspace of the last
 * bind, -3 work_bytes too small. */
int hqr_batch_run(const hqr_batch* b, void* dwork, size_t work_bytes, void* stream);

/* Waits for the stream (timeout_s as hqr_status_ex) and reports the batch
 * status in *status (0, HQR_ERR_WATCHDOG, or HQR_ERR_SINGULAR when some
 * problem's R has a zero diagonal entry) and, if first_zero is not NULL,
 * per problem the index of its first zero diagonal entry of R, or -1.
 * Errors: -1 b NULL, -2 dwork NULL, -5 status NULL; HQR_ERR_TIMEOUT. */
int hqr_batch_status(const hqr_batch* b, const void* dwork, void* stream, double timeout_s, int32_t* status,
                     int32_t* first_zero);

/* The same report without a host wait or a device-to-host copy, for a
 * serving loop that polls many batches: enqueues on `stream`, after the
 * batch's work, one single-workgroup kernel that writes host[0] = status
 * and host[1 + q] = first zero diagonal index of problem q (or -1) for the
 * b->count problems.  host: count + 1 int32 of pinned host memory
 * (hipHostMalloc), which the kernel addresses directly; the values are
 * valid once that work has completed (an event recorded after it), and stay
 * until the next call with the same buffer.  Errors: -1 b NULL, -2 dwork
 * NULL, -3 host NULL. */
int hqr_batch_publish_status(const hqr_batch* b, const void* dwork, int32_t* host, void* stream);

/* Copies the factorization of problem q (its T factors and the tiles of its
 * matrix) out of the batch workspace into dst, a workspace of
 * hqr_workspace_size(M[q], N[q]) bytes laid out as hqr_factor leaves it,
 * so that the factors stay on the device after the batch workspace is
 * reused (hqr_apply_qt / hqr_apply_q / hqr_solve take dst).  Enqueued on
 * `stream` after the batch.  Errors: -1 b NULL, -2 q out of range, -3 dwork
 * NULL, -4 dst NULL, -5 dst_bytes too small. */
int hqr_batch_export_factors(const hqr_batch* b, int32_t q, const void* dwork, void* dst, size_t dst_bytes,
                             void* stream);

/* hqr_batch_export_factors for every problem q with dst[q] not NULL, in one
 * launch on `stream` (plus the upload of count small descriptors into the
 * batch workspace, which must be the one bound last): each dst[q] (device
 * memory of dst_bytes[q] >= hqr_workspace_size(M_q, N_q) bytes, owned by the
 * caller) receives problem q's factors in the hqr_factor workspace layout,
 * with zero control words.  The batch's run must have been enqueued before.
 * Errors: -1 b NULL, -2 dwork NULL or not the bound workspace, -3 dst NULL,
 * -4 dst_bytes NULL, -5 some dst_bytes[q] too small (nothing enqueued). */
int hqr_batch_export_all(const hqr_batch* b, void* dwork, void* const* dst, const size_t* dst_bytes, void* stream);

/* Frees the host batch object (the caller's device buffers are untouched). */
void hqr_batch_destroy(hqr_batch* b);

/* One-call batched least squares: create, bind and run a batch, then free
 * it (the work stays enqueued).  Arguments as hqr_batch_create/_bind; nrhs
 * may be NULL (factorizations only).  Errors: -1 count out of range, -2 dA,
 * -3 M, -4 N, -5 lda, -6 dB, -7 ldb, -8 nrhs, -9 params, -10 exec.order, -11
 * dwork NULL, -12 work_bytes too small (hqr_lstsq_batched_workspace_size). */
int hqr_lstsq_batched(int32_t count, double* const* dA, const int64_t* M, const int64_t* N, const int64_t* lda,
                      double* const* dB, const int64_t* ldb, const int32_t* nrhs, const hqr_params* params,
                      const hqr_exec* exec, void* dwork, size_t work_bytes, void* stream);

/* Workspace bytes of hqr_lstsq_batched.  Errors as hqr_batch_create (-1 .. -5),
 * -6 bytes NULL. */
int hqr_lstsq_batched_workspace_size(int32_t count, const int64_t* M, const int64_t* N, const int32_t* nrhs,
                                     const hqr_params* params, size_t* bytes);

/* Least squares with a finished factorization: B (M x nrhs) <- Q^T B, then
 * x = R^{-1} (Q^T B)(0:N) in rows 0..N-1 of B (rows N..M-1 keep the
 * residual components), with the factorization of hqr_factor (or one
 * exported by hqr_batch_export_factors) in dwork and bwork as for
 * hqr_apply_qt.  A zero diagonal entry of R is reported by hqr_status(bwork)
 * as HQR_ERR_SINGULAR.  Errors as hqr_apply_qt. */
int hqr_solve(int64_t M, int64_t N, const hqr_params* params, const hqr_exec* exec, const void* dwork,
              size_t work_bytes, double* dB, int64_t ldb, int32_t nrhs, void* bwork, size_t bwork_bytes,
              void* stream);

/* Status word of the last launch that used the workspace `dwork` (a
 * factorization or least-squares workspace, or the bwork of hqr_apply_qt/_q):
 * waits for the stream (at most 300 s), then reports 0, HQR_ERR_WATCHDOG or
 * (hqr_lstsq) HQR_ERR_SINGULAR in *status.  Returns HQR_ERR_TIMEOUT if the
 * stream is still busy after the wait. */
int hqr_status(const void* dwork, void* stream, int32_t* status);

/* As hqr_status with an explicit time limit (<= 0: 300 s).  When the launch
 * was aborted by the watchdog, detail[0..3] (if not NULL) receive the task
 * index that gave up, the dependency counter it waited on (index into the
 * counter array: (row * nt + col) * chunks + chunk), the count it waited for
 * and the count it last saw. */
int hqr_status_ex(const void* dwork, void* stream, double timeout_s, int32_t* status, int32_t* detail);

/* Free every cached task plan (host and device).  Not thread-safe with
 * respect to concurrent hqr_factor calls. */
void hqr_release_plans(void);

/* Message for an error code. */
const char* hqr_strerror(int code);

/* "where: message" of the last failed HIP call made by this thread inside the
 * library (empty if none). */
const char* hqr_last_error(void);

/* Per-task timeline of the last launch in this process, recorded only when
 * the environment variable HQR_TIMELINE=1 is set (profiling aid).  For task
 * t of the dispatch order (see hqr_plan_tasks): out[4t] = clock when a
 * workgroup picked it, out[4t+1] = when its inputs were ready, out[4t+2] =
 * when it finished (100 MHz real-time clock ticks), out[4t+3] = workgroup
 * index | XCD index << 16.  Synchronizes `stream`.  out may be NULL to count.
 * Errors: -3 cap too small, -4 count is NULL. */
int hqr_timeline(void* stream, uint64_t* out, int64_t cap, int64_t* count);

/* Library version string. */
const char* hqr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HQR_H_ */
