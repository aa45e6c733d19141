// Host-side elimination lists and kernel task graphs.
//
// Elimination lists follow Sections III and IV of the paper (reduction trees
// and their hierarchical composition); the task graph is the kernel expansion
// of Algorithm 2 with one triangularisation per tile (the tile-state model of
// Section II: square -> triangle -> zero).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hqr.h"

namespace hqr {

struct Elim {
  int32_t k, victim, killer, kind, level, round;
};

// Reduction tree on an ascending participant list `rows` (rows[0] survives).
// Appends (victim, killer, round) triples.
struct Kill {
  int32_t victim, killer, round;
};

void tree_static(int kind, const std::vector<int32_t>& rows, std::vector<Kill>& out);

// Checks params; returns 0 or a negative code for the offending field.
int check_params(const hqr_params& p);

std::vector<Elim> make_elimlist(int32_t mt, int32_t nt, const hqr_params& p);

// Empty string when the list obeys the rules of Section II; else a reason.
std::string validate_elimlist(int32_t mt, int32_t nt, const Elim* list, int64_t count);

enum Op : uint8_t { GEQRT = 0, UNMQR = 1, TSQRT = 2, TSMQR = 3, TTQRT = 4, TTMQR = 5 };

inline int op_weight(int op) {
  static const int w[6] = {4, 6, 6, 12, 2, 6};
  return w[op];
}

// One kernel task of Algorithm 2.  Unused fields are -1.
struct Task {
  uint8_t op;
  int32_t row;     // GEQRT/UNMQR: the tile row; TS/TT: the victim i
  int32_t killer;  // TS/TT only
  int32_t k;       // panel
  int32_t j;       // updated tile column (UNMQR, TSMQR, TTMQR)
};

// Kernel tasks of a list in program order: per panel, first GEQRT(r,k) and
// UNMQR(r,k,j>k) for every row r >= k that is not a TS victim, then each
// elimination as TSQRT+TSMQR or TTQRT+TTMQR over j > k.  The updates run
// over ncols >= nt tile columns (columns nt.. hold right-hand sides that are
// transformed but not factored); ncols < 0 means nt.
std::vector<Task> expand_tasks(int32_t mt, int32_t nt, const std::vector<Elim>& list, int32_t ncols = -1);

// Device task record (24 bytes).  The persistent kernel waits until the
// dependency counters of the tiles it touches reach v[0..2] and bumps the
// counters of the tiles it writes when done.
struct DevTask {
  uint8_t op;
  uint8_t chunk;   // column chunk of an update task (0 for panel tasks)
  uint16_t row;    // GEQRT/UNMQR row, or victim
  uint16_t killer;
  uint16_t k;
  uint16_t j;
  uint16_t pad;
  uint32_t v[3];
};
static_assert(sizeof(DevTask) == 24, "device task record must stay 24 bytes");

struct Plan {
  int32_t mt = 0, nt = 0, nb = 0, chunks = 1;
  std::vector<Elim> list;
  std::vector<DevTask> dev;  // in dispatch order
  std::vector<int64_t> prio; // dispatch priority of each task of dev (factorization plans)
  hqr_dag_info info{};
};

// Active column chunks of the tile columns of a launch: the factored
// columns 0..nt-1 (the last one `last_a` chunks wide: chunks that hold only
// zero padding are never touched) and `nrhs_cols` right-hand-side columns
// appended as further tile columns (B is transformed with the matrix and
// never factored).
struct ColumnChunks {
  int32_t last_a = 0;     // 0: every chunk
  int32_t nrhs_cols = 0;  // right-hand-side columns (0: none)
};

// Builds the device plan.  `order` 0 = critical-path priority order, 1 =
// program order.  `chunks` = dependency counters per tile (64-column
// sub-chunks).  A panel task's `chunk` field holds the number of active
// sub-chunks of its tile column (the blocks it waits for and publishes one
// by one).  An update task covers 128 columns (two sub-chunks; one at
// nb = 64 or at the ragged end of a tile): `chunk` is its first sub-chunk,
// `pad` = (sub-chunks covered << 8) | the factored tile's last active
// sub-chunk, which it waits for.
int build_plan(int32_t mt, int32_t nt, const hqr_params& p, int order, int chunks, Plan& plan,
               const ColumnChunks& cc = ColumnChunks());

// Host plan of a factorization (build_plan with `order` and `cc`), built
// once per (tile grid, params, order, active columns) and kept for the life
// of the process in host memory only; thread-safe.
int host_plan(int32_t mt, int32_t nt, const hqr_params& p, int order, const ColumnChunks& cc, const Plan** out);

// Device plan of B <- Q^T B (trans = 1) or B <- Q B (trans = 0) for the
// factorization of an mt x nt tile grid, on a B of mt tile rows and `nbc`
// blocks of 64 columns.  The update tasks of the factorization (UNMQR,
// TSMQR, TTMQR) are replayed on B's blocks, in program order for Q^T and in
// reverse program order for Q.  A task's `j` is the B block; its counters are
// indexed (row * nbc + j), one per block; v[0] (the factored tile) is 0
// because the factorization has finished.
int build_apply_plan(int32_t mt, int32_t nt, int32_t nbc, const hqr_params& p, int trans, Plan& plan);

}  // namespace hqr
