/*
 * Reference QR oracle (test infrastructure only).
 *
 * This file is the plain, slow, obviously correct CPU definition of what the
 * tiled factorization computes: an unblocked Householder QR in double
 * precision, one reflector per column, applied column by column (the standard
 * Householder algorithm whose flop count, 2MN^2 - 2N^3/3, the paper equates
 * with the total weight of any tiled elimination list; Section II, the
 * paragraph after Algorithm 2).  It shares no code with the GPU library and
 * is only ever loaded by the tests, the smoke check and the CPU-baseline leg
 * of the benchmark.
 *
 * Conventions (LAPACK geqr2 semantics, written from the definition):
 *   column-major storage, element (r, c) at A[r + c * lda];
 *   reflector j is H_j = I - tau_j v_j v_j^T with v_j(j) = 1, v_j(r) = 0 for
 *   r < j, and v_j(r) for r > j stored in A below the diagonal;
 *   R is left in the upper triangle of A;
 *   alpha = A(j,j), sigma = ||A(j+1:m, j)||_2;
 *   sigma == 0  -> tau = 0 (H_j = I), R(j,j) = alpha;
 *   otherwise   beta = -sign(alpha) * sqrt(alpha^2 + sigma^2),
 *               tau = (beta - alpha) / beta, v = x / (alpha - beta),
 *               R(j,j) = beta.
 *   No overflow-avoiding rescaling is done: inputs are assumed to have
 *   entries far from the overflow threshold (|a| < 1e150).
 *
 * Threads: the update of the trailing columns by one reflector is split over
 * worker threads by column; each column is updated by exactly one thread in
 * the same order as the sequential loop, so the result does not depend on the
 * thread count.
 */
#define _POSIX_C_SOURCE 200809L
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* One Householder reflector from x = A(j:m, j).  Returns tau; overwrites
 * A(j,j) with R(j,j) and A(j+1:m, j) with v(j+1:m). */
static double make_reflector(int64_t m, double* col, int64_t j) {
  double alpha = col[j];
  double ss = 0.0;
  for (int64_t r = j + 1; r < m; ++r) ss += col[r] * col[r];
  if (ss == 0.0) return 0.0;
  double beta = sqrt(alpha * alpha + ss);
  if (alpha >= 0.0) beta = -beta;
  double tau = (beta - alpha) / beta;
  double scale = 1.0 / (alpha - beta);
  for (int64_t r = j + 1; r < m; ++r) col[r] *= scale;
  col[j] = beta;
  return tau;
}

/* c <- (I - tau v v^T) c for one column c, v taken from column vcol of the
 * factored matrix (implicit unit at row j). */
static void apply_reflector(int64_t m, const double* vcol, int64_t j, double tau, double* c) {
  if (tau == 0.0) return;
  double w = c[j];
  for (int64_t r = j + 1; r < m; ++r) w += vcol[r] * c[r];
  w *= tau;
  c[j] -= w;
  for (int64_t r = j + 1; r < m; ++r) c[r] -= vcol[r] * w;
}

typedef struct {
  int64_t m, n, lda, k;
  double* A;
  double* tau;
  int tid, nthreads;
  pthread_barrier_t* bar;
} geqr2_job;

/* Column-cyclic worker: thread t owns columns c with c % nthreads == t.
 * Step j: the owner of column j builds reflector j (all of its earlier
 * updates are done), a barrier publishes it, then every thread applies it to
 * the columns c > j it owns, and a second barrier ends the step. */
static void* geqr2_worker(void* p) {
  geqr2_job* jb = (geqr2_job*)p;
  for (int64_t j = 0; j < jb->k; ++j) {
    if (j % jb->nthreads == jb->tid) jb->tau[j] = make_reflector(jb->m, jb->A + j * jb->lda, j);
    pthread_barrier_wait(jb->bar);
    const double* v = jb->A + j * jb->lda;
    for (int64_t c = j + 1; c < jb->n; ++c)
      if (c % jb->nthreads == jb->tid) apply_reflector(jb->m, v, j, jb->tau[j], jb->A + c * jb->lda);
    pthread_barrier_wait(jb->bar);
  }
  return NULL;
}

/* Unblocked Householder QR of the m x n column-major matrix A (in place).
 * tau must hold min(m, n) doubles.  Returns 0, or -1 on bad arguments. */
int oracle_geqr2(int64_t m, int64_t n, double* A, int64_t lda, double* tau, int nthreads) {
  if (m < 0 || n < 0 || lda < (m > 1 ? m : 1) || !A || !tau) return -1;
  int64_t k = m < n ? m : n;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 64) nthreads = 64;
  if (nthreads == 1 || n < 2 * nthreads) {
    for (int64_t j = 0; j < k; ++j) {
      tau[j] = make_reflector(m, A + j * lda, j);
      for (int64_t c = j + 1; c < n; ++c) apply_reflector(m, A + j * lda, j, tau[j], A + c * lda);
    }
    return 0;
  }
  pthread_barrier_t bar;
  pthread_barrier_init(&bar, NULL, (unsigned)nthreads);
  pthread_t th[64];
  geqr2_job jobs[64];
  for (int t = 0; t < nthreads; ++t) {
    jobs[t] = (geqr2_job){m, n, lda, k, A, tau, t, nthreads, &bar};
    if (t > 0) pthread_create(&th[t], NULL, geqr2_worker, &jobs[t]);
  }
  geqr2_worker(&jobs[0]);
  for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
  pthread_barrier_destroy(&bar);
  return 0;
}

/* B <- Q^T B with Q = H_0 H_1 ... H_{k-1} from oracle_geqr2 (B is m x nrhs). */
int oracle_apply_qt(int64_t m, int64_t n, const double* A, int64_t lda, const double* tau,
                    double* B, int64_t ldb, int64_t nrhs) {
  if (m < 0 || n < 0 || nrhs < 0 || lda < (m > 1 ? m : 1) || ldb < (m > 1 ? m : 1)) return -1;
  int64_t k = m < n ? m : n;
  for (int64_t c = 0; c < nrhs; ++c)
    for (int64_t j = 0; j < k; ++j) apply_reflector(m, A + j * lda, j, tau[j], B + c * ldb);
  return 0;
}

/* B <- Q B (reflectors applied in reverse order). */
int oracle_apply_q(int64_t m, int64_t n, const double* A, int64_t lda, const double* tau,
                   double* B, int64_t ldb, int64_t nrhs) {
  if (m < 0 || n < 0 || nrhs < 0 || lda < (m > 1 ? m : 1) || ldb < (m > 1 ? m : 1)) return -1;
  int64_t k = m < n ? m : n;
  for (int64_t c = 0; c < nrhs; ++c)
    for (int64_t j = k - 1; j >= 0; --j) apply_reflector(m, A + j * lda, j, tau[j], B + c * ldb);
  return 0;
}
