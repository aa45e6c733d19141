// Launch interface between the host planner/ABI and the persistent GPU
// scheduler.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "elim.hpp"
#include "layout.hpp"

namespace hqr {

// One problem of a batched launch (hqr_batch_*).  Offsets are bytes from the
// start of the batch workspace; the problem's tiles, T factors and
// dependency counters are laid out there exactly as for a single
// factorization of the same shape.
struct ProbDesc {
  double* A;         // caller's M x N matrix (column-major, lda): copied in, R and V copied back
  double* B;         // caller's M x nrhs right-hand sides (ldb), null when nrhs = 0
  int64_t lda, ldb;
  int64_t M, N;
  int64_t tiles;     // tile-contiguous copy of A followed by the right-hand-side tile columns
  int64_t tg, tk;    // T factors (GEQRT, TSQRT/TTQRT)
  int64_t cnt;       // dependency counters, mt * (nt + nrt) * chunks
  int32_t nrhs, mt, nt, nrt;
};
static_assert(sizeof(ProbDesc) == 96, "problem descriptor layout");

struct LaunchArgs {
  double* A;          // tile-contiguous matrix: tile (r, c) at (c * mt + r) * nb * nb
  int64_t lda;        // leading dimension inside a tile (= nb)
  double* Tg;         // T factors of GEQRT, one block column of nb x 16 per tile
  double* Tk;         // T factors of TSQRT/TTQRT, same layout
  int32_t* cnt;       // dependency counters, mt * nt * chunks
  int32_t* ctrl;      // [0] task cursor, [1] status
  const DevTask* tasks;
  int64_t ntasks;
  int64_t spin_limit;
  int32_t* trace;     // optional host-visible progress words, 2 per workgroup (null: off)
  uint64_t* timeline; // optional per-task timestamps, 4 words per task (null: off)
  double* B;          // hqr_apply_qt/_q: B in blocks of nb x 64 (block (r, j) at (j * mt + r) * nb * 64); null
                      // for a factorization
  int32_t mt, nt, chunks;
  int32_t cnt_cols;   // columns of the counter grid (nt, or the number of B blocks)
  int32_t trans;      // apply: 1 = Q^T, 0 = Q
  // batched launch: problem descriptors and the problem of every task (null
  // for a single problem); offsets in the descriptors are relative to ctrl,
  // the start of the workspace
  const ProbDesc* probs;
  const int32_t* task_prob;
};

// Progress phases published per workgroup when tracing is on.
enum TracePhase { TR_POPPED = 1, TR_READY = 2, TR_DONE = 3, TR_EXIT = 4, TR_ABORT = 5 };
constexpr int kTraceSlots = 4096;  // workgroups traced

// Zero `n` int32 words on `stream` with a fill kernel.
int launch_zero_i32(int32_t* p, int64_t n, void* stream);

// Start of a factorization launch: the kCtrlWords control words are zeroed
// except the signature words (kSigWord..), which receive `sig`, and the
// `ncnt` dependency counters at `cnt` are zeroed (cnt may be null when
// ncnt = 0).  One fill kernel.
int launch_init_ctrl(int32_t* ctrl, const FactorSig& sig, int32_t* cnt, int64_t ncnt, void* stream);

// Apply launches: if the signature words of the factorization workspace
// `fctrl` differ from `sig`, sets the status word bctrl[1] of the apply
// workspace to HQR_ERR_FACTORS, which stops the persistent launch that
// follows before its first task.
int launch_check_sig(const int32_t* fctrl, const FactorSig& sig, int32_t* bctrl, void* stream);

// Run every task of the plan in one persistent launch of `workers`
// workgroups.  nb is 64, 128 or 256.
// f32: the tiles, T factors and B blocks hold float and the tile kernels
// run in FP32 (single-problem launches only); bf16 (with f32, factorization
// launches only): the block-reflector products take BF16 operands and
// accumulate in FP32.
int launch_persistent(int nb, const LaunchArgs& a, int workers, void* stream, bool f32 = false, bool bf16 = false);

// Copies the column-major M x N matrix A (leading dimension lda) into the
// blocked buffer At (mt x nt blocks of nb rows x tw columns, zero padding
// beyond M and N) when `in`, or the M x N part of At back into A otherwise.
int launch_tile_copy(double* A, int64_t lda, double* At, int64_t M, int64_t N, int nb, int tw, int mt, int nt,
                     bool in, void* stream);
// The same with the element type of each side chosen: a_f32 / at_f32 = 1
// for float (double -> float copies round to nearest; float -> double is
// not offered for the matrix side).
int launch_tile_copy(void* A, int a_f32, int64_t lda, void* At, int at_f32, int64_t M, int64_t N, int nb, int tw,
                     int mt, int nt, bool in, void* stream);

// Back substitution with the leading N x N triangle of the factored tiles R
// on the first N rows of the nrhs columns of Y (blocks of nb rows x cw
// columns: cw = nb for the tile columns of B in a factorization workspace,
// 64 for the blocks of the apply path), one workgroup per column.
int launch_trsv(int nb, const double* R, double* Y, int cw, int32_t* ctrl, int64_t N, int mt, int nrhs,
                void* stream);

// Stores "where: message" of a failed HIP call for hqr_last_error(); returns
// HQR_ERR_HIP on failure, 0 on success.
int record_hip(hipError_t e, const char* where);
const char* last_error();
// Sets the message hqr_last_error() returns (this thread).
void set_last_error(const char* msg);

// Batched launches (one launch for `count` problems described by the
// device array `d`, offsets relative to the workspace base `w`): copy the
// matrices and right-hand sides into their tiles (in) or A and B back out;
// back substitution of every problem's right-hand sides (first zero
// diagonal entry j of problem q recorded as info[q] = max(N - j)).
// max_elems: padded elements (matrix and right-hand sides) of the largest
// problem, which sizes the copy grid.
int launch_copy_batched(const ProbDesc* d, char* w, int count, int nb, bool in, int64_t max_elems, void* stream);
int launch_trsv_batched(int nb, const ProbDesc* d, char* w, int32_t* ctrl, int32_t* info, int count, int max_nrhs,
                        void* stream);

// Least-squares refinement steps (FP64 vectors; R as float tiles of nb,
// mt tile rows): f = b - r - A x (r may be null); g = -A^T r (r null: g_j =
// squared norm of column j); y <- R^{-1} y or R^{-T} y; y = d(0:N) - h
// then d(0:N) = h; x += dx, r += dr; out[k] = ||v[k]||^2 (n[k] entries,
// k < 4).
int launch_ir_residual(const double* A, int64_t lda, int64_t M, int64_t N, const double* x, const double* b,
                       const double* r, double* f, void* stream);
int launch_ir_atr(const double* A, int64_t lda, int64_t M, int64_t N, const double* r, double* g, void* stream);
int launch_ir_trsv(const float* R, int nb, int mt, int64_t N, double* y, bool trans, void* stream);
int launch_ir_split(double* d, const double* h, double* y, int64_t N, void* stream);
int launch_ir_update(double* x, const double* dx, int64_t N, double* r, const double* dr, int64_t M, void* stream);
int launch_ir_norms(const double* const* v, const int64_t* n, double* out, void* stream);

// Workgroups that fit on the device at once (per CU occupancy x CUs).
int default_workers(int nb, bool f32 = false);

}  // namespace hqr
