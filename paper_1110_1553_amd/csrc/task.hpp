// Launch interface between the host planner/ABI and the persistent GPU
// scheduler.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "elim.hpp"

namespace hqr {

struct LaunchArgs {
  double* A;          // tiled matrix, column-major, lda even, 16-byte aligned
  int64_t lda;
  double* Tg;         // T factors of GEQRT, one block column of nb x 16 per tile
  double* Tk;         // T factors of TSQRT/TTQRT, same layout
  int32_t* cnt;       // dependency counters, mt * nt * chunks
  int32_t* ctrl;      // [0] task cursor, [1] status
  const DevTask* tasks;
  int64_t ntasks;
  int64_t spin_limit;
  int32_t* trace;     // optional host-visible progress words, 2 per workgroup (null: off)
  uint64_t* timeline; // optional per-task timestamps, 4 words per task (null: off)
  int32_t mt, nt, chunks;
};

// Progress phases published per workgroup when tracing is on.
enum TracePhase { TR_POPPED = 1, TR_READY = 2, TR_DONE = 3, TR_EXIT = 4, TR_ABORT = 5 };
constexpr int kTraceSlots = 4096;  // workgroups traced

// Zero `n` int32 words on `stream` with a fill kernel.
int launch_zero_i32(int32_t* p, int64_t n, void* stream);

// Run every task of the plan in one persistent launch of `workers`
// workgroups.  nb is 64, 128 or 256.
int launch_persistent(int nb, const LaunchArgs& a, int workers, void* stream);

// Copy an m x n column-major block (device to device).
int launch_copy2d(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t m, int64_t n,
                  void* stream);
// Zero an m x n column-major block.
int launch_zero2d(double* dst, int64_t ldd, int64_t m, int64_t n, void* stream);

// Stores "where: message" of a failed HIP call for hqr_last_error(); returns
// HQR_ERR_HIP on failure, 0 on success.
int record_hip(hipError_t e, const char* where);
const char* last_error();

// Workgroups that fit on the device at once (per CU occupancy x CUs).
int default_workers(int nb);

}  // namespace hqr
