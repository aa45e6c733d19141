// C ABI of the tiled hierarchical QR library (declared in include/hqr.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>

#include "../../include/hqr.h"
#include "elim.hpp"
#include "layout.hpp"
#include "task.hpp"

namespace hqr {
namespace {


// order: 0/1 for factorization plans, 2 + trans for apply plans (nbc = B
// blocks); last_a / nrhs: the active chunks of the factorization (ColumnChunks).
struct PlanKey {
  int32_t mt, nt, nb, p, a, low, high, coupling, domino, order, device, nbc, last_a, nrhs;
  bool operator<(const PlanKey& o) const {
    return std::tie(mt, nt, nb, p, a, low, high, coupling, domino, order, device, nbc, last_a, nrhs) <
           std::tie(o.mt, o.nt, o.nb, o.p, o.a, o.low, o.high, o.coupling, o.domino, o.order, o.device, o.nbc,
                    o.last_a, o.nrhs);
  }
};

struct DevicePlan {
  Plan plan;
  DevTask* d_tasks = nullptr;
};

std::mutex g_mu;
int32_t* g_trace = nullptr;  // pinned host words written by the GPU when HQR_TRACE is set

// Per-task timestamps of the last launch when HQR_TIMELINE is set.
uint64_t* g_timeline = nullptr;
int64_t g_timeline_cap = 0, g_timeline_n = 0;

uint64_t* timeline_buffer(int64_t ntasks) {
  static bool want = [] {
    const char* e = getenv("HQR_TIMELINE");
    return e && atoi(e) != 0;
  }();
  if (!want) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_timeline_cap < ntasks) {
    if (g_timeline) (void)hipFree(g_timeline);
    g_timeline = nullptr;
    g_timeline_cap = 0;
    if (hipMalloc(&g_timeline, (size_t)ntasks * 4 * sizeof(uint64_t)) != hipSuccess) return nullptr;
    g_timeline_cap = ntasks;
  }
  g_timeline_n = ntasks;
  return g_timeline;
}

int32_t* trace_buffer() {
  static bool want = [] {
    const char* e = getenv("HQR_TRACE");
    return e && atoi(e) != 0;
  }();
  if (!want) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_trace) {
    void* p = nullptr;
    if (hipHostMalloc(&p, 2 * kTraceSlots * sizeof(int32_t), hipHostMallocDefault) != hipSuccess) return nullptr;
    g_trace = (int32_t*)p;
  }
  return g_trace;
}
std::map<PlanKey, std::unique_ptr<DevicePlan>> g_plans;

// Cached device plan: order 0/1 = factorization, 2 + trans = apply on nbc
// blocks of B.
int get_plan(int32_t mt, int32_t nt, const hqr_params& p, int order, DevicePlan** out, int32_t nbc = 0,
             const ColumnChunks& cc = ColumnChunks()) {
  int dev = 0;
  if (int rc = record_hip(hipGetDevice(&dev), "hipGetDevice")) return rc;
  PlanKey key{mt, nt, p.nb, p.p, p.a, p.low, p.high, p.coupling, p.domino, order, dev, nbc, cc.last_a, cc.nrhs_cols};
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) {
    *out = it->second.get();
    return 0;
  }
  std::unique_ptr<DevicePlan> dp(new DevicePlan());
  int rc = order >= 2 ? build_apply_plan(mt, nt, nbc, p, order - 2, dp->plan)
                      : build_plan(mt, nt, p, order, chunks_for(p.nb), dp->plan, cc);
  if (rc) return rc;
  const size_t bytes = dp->plan.dev.size() * sizeof(DevTask);
  if (bytes) {
    if (record_hip(hipMalloc(&dp->d_tasks, bytes), "hipMalloc(task plan)")) return HQR_ERR_NOMEM;
    if (int rc = record_hip(hipMemcpy(dp->d_tasks, dp->plan.dev.data(), bytes, hipMemcpyHostToDevice),
                            "hipMemcpy(task plan)")) {
      (void)hipFree(dp->d_tasks);
      return rc;
    }
  }
  *out = dp.get();
  g_plans[key] = std::move(dp);
  return 0;
}

}  // namespace

// B (M x nrhs) <- Q^T B (trans = 1) or Q B with the factorization held in
// dwork; B is copied into the blocks of bwork, transformed, and copied back
// when copy_out.
int run_apply(int trans, int64_t M, int64_t N, const hqr_params& p, const hqr_exec* exec, const void* dwork,
              size_t work_bytes, double* dB, int64_t ldb, int32_t nrhs, void* bwork, size_t bwork_bytes,
              void* stream, bool copy_out, bool f32) {
  const size_t es = f32 ? sizeof(float) : sizeof(double);
  const Layout L = layout_for(M, N, p, 0, es);
  const ApplyLayout AL = apply_layout_for(M, nrhs, p, es);
  if (L.mt > 65535 || L.nt > 65535 || AL.nbc > 65535) return -2;
  if (work_bytes < L.total) return -7;
  if (bwork_bytes < AL.total) return -12;
  hqr_exec ex{0, 0, 0, nullptr, nullptr};
  if (exec) ex = *exec;
  DevicePlan* dp = nullptr;
  int rc = get_plan(L.mt, L.nt, p, 2 + trans, &dp, AL.nbc);
  if (rc) return rc;
  const char* w = (const char*)dwork;
  char* bw = (char*)bwork;
  LaunchArgs a{};
  a.A = (double*)(w + L.tiles);
  a.lda = p.nb;
  a.Tg = (double*)(w + L.tg);
  a.Tk = (double*)(w + L.tk);
  a.ctrl = (int32_t*)(bw + AL.ctrl);
  a.cnt = (int32_t*)(bw + AL.cnt);
  a.B = (double*)(bw + AL.blocks);
  a.tasks = dp->d_tasks;
  a.ntasks = (int64_t)dp->plan.dev.size();
  a.spin_limit = ex.spin_limit > 0 ? ex.spin_limit : kDefaultSpinLimit;
  a.mt = L.mt;
  a.nt = L.nt;
  a.chunks = 1;
  a.cnt_cols = AL.nbc;
  a.trans = trans;
  if ((rc = launch_tile_copy(dB, 0, ldb, a.B, f32, M, nrhs, p.nb, 64, AL.mt, AL.nbc, true, stream))) return rc;
  const int64_t nwords = (int64_t)((AL.blocks - AL.ctrl) / sizeof(int32_t));  // ctrl + counters
  if ((rc = launch_zero_i32(a.ctrl, nwords, stream))) return rc;
  // a workspace that holds another factorization (or none) stops the launch
  // before its first task
  if ((rc = launch_check_sig((const int32_t*)(w + L.ctrl), factor_sig(L, p, es), a.ctrl, stream))) return rc;
  if (a.ntasks > 0) {
    int workers = ex.workers > 0 ? ex.workers : default_workers(p.nb, f32);
    if ((rc = launch_persistent(p.nb, a, workers, stream, f32))) return rc;
  }
  if (copy_out && (rc = launch_tile_copy(dB, 0, ldb, a.B, f32, M, nrhs, p.nb, 64, AL.mt, AL.nbc, false, stream)))
    return rc;
  return 0;
}

int check_apply_args(int64_t M, int64_t N, const hqr_params* params, const void* dwork, const double* dB,
                     int64_t ldb, int32_t nrhs, const void* bwork) {
  if (M < 1 || M < N) return -2;
  if (N < 1) return -3;
  if (!params || check_params(*params) || params->precision != HQR_PREC_FP64) return -4;
  if (!dwork) return -6;
  if (!dB) return -8;
  if (ldb < M) return -9;
  if (nrhs < 1) return -10;
  if (!bwork) return -11;
  return 0;
}

// One factorization launch: copy A (and the nrhs right-hand sides B, which
// are transformed by Q^T as further tile columns) into the workspace's
// tiles, run every task of the plan, copy A back when copy_a_out.  The
// caller has checked the arguments.
// f32: the factorization runs in FP32 on float tiles; a_f32: dA holds
// float (else double, rounded to float on the way in when f32).
int run_factor(void* dA, int64_t M, int64_t N, int64_t lda, const hqr_params& p, const hqr_exec& ex, void* dwork,
               double* dB, int64_t ldb, int32_t nrhs, void* stream, bool copy_a_out, bool f32, bool a_f32,
               const void* tasks, int64_t ntasks) {
  const size_t es = f32 ? sizeof(float) : sizeof(double);
  const Layout L = layout_for(M, N, p, nrhs, es);
  int rc = 0;
  LaunchArgs a{};
  if (tasks) {
    a.tasks = (const DevTask*)tasks;
    a.ntasks = ntasks;
  } else {
    ColumnChunks cc;
    cc.last_a = L.last_a;
    cc.nrhs_cols = nrhs;
    DevicePlan* dp = nullptr;
    if ((rc = get_plan(L.mt, L.nt, p, ex.order, &dp, 0, cc))) return rc;
    a.tasks = dp->d_tasks;
    a.ntasks = (int64_t)dp->plan.dev.size();
    a.trace = trace_buffer();
    a.timeline = timeline_buffer(a.ntasks);
    if (a.trace) std::memset(a.trace, 0, 2 * kTraceSlots * sizeof(int32_t));
  }
  char* w = (char*)dwork;
  a.ctrl = (int32_t*)(w + L.ctrl);
  a.cnt = (int32_t*)(w + L.cnt);
  a.Tg = (double*)(w + L.tg);
  a.Tk = (double*)(w + L.tk);
  a.spin_limit = ex.spin_limit > 0 ? ex.spin_limit : kDefaultSpinLimit;
  a.mt = L.mt;
  a.nt = L.nt;
  a.chunks = L.chunks;
  a.cnt_cols = L.nt + L.nrt;
  a.B = nullptr;
  a.A = (double*)(w + L.tiles);
  a.lda = p.nb;
  if ((rc = launch_tile_copy(dA, a_f32, lda, a.A, f32, M, N, p.nb, p.nb, L.mt, L.nt, true, stream))) return rc;
  void* Bt = (char*)a.A + (size_t)L.mt * L.nt * p.nb * p.nb * es;
  if (nrhs > 0 && (rc = launch_tile_copy(dB, 0, ldb, Bt, f32, M, nrhs, p.nb, p.nb, L.mt, L.nrt, true, stream)))
    return rc;
  const int64_t ncnt = (int64_t)L.mt * (L.nt + L.nrt) * L.chunks;
  if ((rc = launch_init_ctrl(a.ctrl, factor_sig(L, p, es), a.cnt, ncnt, stream))) return rc;
  int workers = ex.workers > 0 ? ex.workers : default_workers(p.nb, f32);
  if (ex.ev_begin && (rc = record_hip(hipEventRecord((hipEvent_t)ex.ev_begin, (hipStream_t)stream),
                                      "hipEventRecord(ev_begin)")))
    return rc;
  if ((rc = launch_persistent(p.nb, a, workers, stream, f32, f32 && p.precision == HQR_PREC_BF16))) return rc;
  if (ex.ev_end && (rc = record_hip(hipEventRecord((hipEvent_t)ex.ev_end, (hipStream_t)stream),
                                    "hipEventRecord(ev_end)")))
    return rc;
  if (copy_a_out &&
      (rc = launch_tile_copy(dA, a_f32, lda, a.A, f32, M, N, p.nb, p.nb, L.mt, L.nt, false, stream)))
    return rc;
  return 0;
}

}  // namespace hqr

// Host record of a finished factorization (include/hqr.h).
struct hqr_factors {
  int64_t M = 0, N = 0;
  hqr_params p{};
  bool f32 = false;
  const void* dwork = nullptr;
  size_t work_bytes = 0;
};

namespace hqr {
namespace {

int make_handle(int64_t M, int64_t N, const hqr_params& p, bool f32, const void* dwork, size_t work_bytes,
                hqr_factors** out) {
  if (!out) return 0;
  hqr_factors* f = new (std::nothrow) hqr_factors();
  if (!f) return HQR_ERR_NOMEM;
  f->M = M;
  f->N = N;
  f->p = p;
  f->f32 = f32;
  f->dwork = dwork;
  f->work_bytes = work_bytes;
  *out = f;
  return 0;
}

int check_handle_args(const hqr_factors* f, const double* dB, int64_t ldb, int32_t nrhs, const void* bwork) {
  if (!f) return -1;
  if (!dB) return -3;
  if (ldb < f->M) return -4;
  if (nrhs < 1) return -5;
  if (!bwork) return -6;
  return 0;
}

// run_apply's argument codes (-7: dwork too small, -12: bwork too small) in
// the numbering of the handle entry points.
int map_apply_rc(int rc) {
  if (rc == -12) return -7;
  if (rc == -7 || rc == -2) return HQR_ERR_INTERNAL;  // the handle's own workspace and shape were accepted before
  return rc;
}

}  // namespace
}  // namespace hqr

using namespace hqr;

extern "C" {

int hqr_elimlist(int32_t mt, int32_t nt, const hqr_params* params, hqr_elim* out, int64_t cap, int64_t* count) {
  if (mt < 1) return -1;
  if (nt < 1) return -2;
  if (!params) return -3;
  hqr_params p = *params;
  p.nb = 64;  // tile size and inner blocking do not change the list
  p.ib = 16;
  if (check_params(p)) return -3;
  if (!count) return -6;
  std::vector<Elim> list = make_elimlist(mt, nt, p);
  *count = (int64_t)list.size();
  if (!out) return 0;
  if (cap < (int64_t)list.size()) return -5;
  for (size_t n = 0; n < list.size(); ++n)
    out[n] = hqr_elim{list[n].k, list[n].victim, list[n].killer, list[n].kind, list[n].level, list[n].round};
  return 0;
}

int hqr_elimlist_validate(int32_t mt, int32_t nt, const hqr_elim* list, int64_t count) {
  if (mt < 1) return -1;
  if (nt < 1) return -2;
  if (count < 0) return -4;
  if (!list && count > 0) return -3;
  std::vector<Elim> v(count);
  for (int64_t n = 0; n < count; ++n)
    v[n] = Elim{list[n].k, list[n].victim, list[n].killer, list[n].kind, list[n].level, list[n].round};
  return validate_elimlist(mt, nt, v.data(), count).empty() ? 0 : HQR_ERR_INVALID_LIST;
}

int hqr_dag_stats(int32_t mt, int32_t nt, const hqr_params* params, hqr_dag_info* out) {
  if (mt < 1) return -1;
  if (nt < 1 || nt > mt) return -2;
  if (!params || check_params(*params)) return -3;
  if (!out) return -4;
  if (mt > 65535) return -1;
  Plan plan;
  int rc = build_plan(mt, nt, *params, 1, chunks_for(params->nb), plan);
  if (rc) return rc;
  *out = plan.info;
  return 0;
}

int hqr_plan_tasks(int32_t mt, int32_t nt, const hqr_params* params, int32_t order, hqr_task* out, int64_t cap,
                   int64_t* count) {
  if (mt < 1 || mt > 65535) return -1;
  if (nt < 1 || nt > mt) return -2;
  if (!params || check_params(*params)) return -3;
  if (order != 0 && order != 1) return -4;
  if (!count) return -7;
  Plan plan;
  int rc = build_plan(mt, nt, *params, order, chunks_for(params->nb), plan);
  if (rc) return rc;
  *count = (int64_t)plan.dev.size();
  if (!out) return 0;
  if (cap < *count) return -6;
  static_assert(sizeof(hqr_task) == sizeof(DevTask), "task record layouts differ");
  std::memcpy(out, plan.dev.data(), plan.dev.size() * sizeof(DevTask));
  return 0;
}

int hqr_workspace_size(int64_t M, int64_t N, const hqr_params* params, size_t* bytes) {
  if (M < 1) return -1;
  if (N < 1 || N > M) return -2;
  if (!params || check_params(*params)) return -3;
  if (!bytes) return -4;
  *bytes = layout_for(M, N, *params).total;
  return 0;
}

int hqr_factor(double* dA, int64_t M, int64_t N, int64_t lda, const hqr_params* params, const hqr_exec* exec,
               void* dwork, size_t work_bytes, void* stream, hqr_factors** out) {
  if (!dA) return -1;
  if (M < 1 || M < N) return -2;
  if (N < 1) return -3;
  if (lda < M) return -4;
  if (!params || check_params(*params) || params->precision != HQR_PREC_FP64) return -5;
  if (!dwork) return -7;
  const Layout L = layout_for(M, N, *params);
  if (L.mt > 65535 || L.nt > 65535) return -2;
  if (work_bytes < L.total) return -8;
  hqr_exec ex{0, 0, 0, nullptr, nullptr};
  if (exec) ex = *exec;
  if (ex.order != 0 && ex.order != 1) return -6;
  int rc = run_factor(dA, M, N, lda, *params, ex, dwork, nullptr, 0, 0, stream, true, false, false);
  if (rc) return rc;
  return make_handle(M, N, *params, false, dwork, work_bytes, out);
}

int hqr_workspace_size_f32(int64_t M, int64_t N, const hqr_params* params, size_t* bytes) {
  if (M < 1) return -1;
  if (N < 1 || N > M) return -2;
  if (!params || check_params(*params)) return -3;
  if (!bytes) return -4;
  *bytes = layout_for(M, N, *params, 0, sizeof(float)).total;
  return 0;
}

int hqr_factor_f32(float* dA, int64_t M, int64_t N, int64_t lda, const hqr_params* params, const hqr_exec* exec,
                   void* dwork, size_t work_bytes, void* stream, hqr_factors** out) {
  if (!dA) return -1;
  if (M < 1 || M < N) return -2;
  if (N < 1) return -3;
  if (lda < M) return -4;
  if (!params || check_params(*params)) return -5;
  hqr_params p = *params;
  if (p.precision == HQR_PREC_FP64) p.precision = HQR_PREC_FP32;
  if (!dwork) return -7;
  const Layout L = layout_for(M, N, p, 0, sizeof(float));
  if (L.mt > 65535 || L.nt > 65535) return -2;
  if (work_bytes < L.total) return -8;
  hqr_exec ex{0, 0, 0, nullptr, nullptr};
  if (exec) ex = *exec;
  if (ex.order != 0 && ex.order != 1) return -6;
  int rc = run_factor(dA, M, N, lda, p, ex, dwork, nullptr, 0, 0, stream, true, true, true);
  if (rc) return rc;
  return make_handle(M, N, p, true, dwork, work_bytes, out);
}

int hqr_apply_workspace_size(int64_t M, int32_t nrhs, const hqr_params* params, size_t* bytes) {
  if (M < 1) return -1;
  if (nrhs < 1) return -2;
  if (!params || check_params(*params)) return -3;
  if (!bytes) return -4;
  *bytes = apply_layout_for(M, nrhs, *params).total;
  return 0;
}

int hqr_apply_qt(int64_t M, int64_t N, const hqr_params* params, const hqr_exec* exec, const void* dwork,
                 size_t work_bytes, double* dB, int64_t ldb, int32_t nrhs, void* bwork, size_t bwork_bytes,
                 void* stream) {
  if (int rc = check_apply_args(M, N, params, dwork, dB, ldb, nrhs, bwork)) return rc;
  return run_apply(1, M, N, *params, exec, dwork, work_bytes, dB, ldb, nrhs, bwork, bwork_bytes, stream, true, false);
}

int hqr_apply_q(int64_t M, int64_t N, const hqr_params* params, const hqr_exec* exec, const void* dwork,
                size_t work_bytes, double* dB, int64_t ldb, int32_t nrhs, void* bwork, size_t bwork_bytes,
                void* stream) {
  if (int rc = check_apply_args(M, N, params, dwork, dB, ldb, nrhs, bwork)) return rc;
  return run_apply(0, M, N, *params, exec, dwork, work_bytes, dB, ldb, nrhs, bwork, bwork_bytes, stream, true, false);
}

int hqr_lstsq_workspace_size(int64_t M, int64_t N, int32_t nrhs, const hqr_params* params, size_t* bytes) {
  if (M < 1 || M < N) return -1;
  if (N < 1) return -2;
  if (nrhs < 1) return -3;
  if (!params || check_params(*params)) return -4;
  if (!bytes) return -5;
  *bytes = layout_for(M, N, *params, nrhs).total;
  return 0;
}

int hqr_lstsq(double* dA, int64_t M, int64_t N, int64_t lda, double* dB, int64_t ldb, int32_t nrhs,
              const hqr_params* params, const hqr_exec* exec, void* dwork, size_t work_bytes, void* stream,
              hqr_factors** out) {
  if (!dA) return -1;
  if (M < 1 || M < N) return -2;
  if (N < 1) return -3;
  if (lda < M) return -4;
  if (!dB) return -5;
  if (ldb < M) return -6;
  if (nrhs < 1) return -7;
  if (!params || check_params(*params) || params->precision != HQR_PREC_FP64) return -8;
  if (!dwork) return -10;
  const hqr_params& p = *params;
  const Layout L = layout_for(M, N, p, nrhs);
  if (L.mt > 65535 || L.nt + L.nrt > 65535) return -2;
  if (work_bytes < L.total) return -11;
  hqr_exec ex{0, 0, 0, nullptr, nullptr};
  if (exec) ex = *exec;
  if (ex.order != 0 && ex.order != 1) return -9;
  int rc = run_factor(dA, M, N, lda, p, ex, dwork, dB, ldb, nrhs, stream, true, false, false);
  if (rc) return rc;
  char* w = (char*)dwork;
  const double* tiles = (const double*)(w + L.tiles);
  double* Bt = (double*)(w + L.tiles) + (size_t)L.mt * L.nt * p.nb * p.nb;
  // the right-hand sides are tile columns of nb after the matrix tiles
  if ((rc = launch_trsv(p.nb, tiles, Bt, p.nb, (int32_t*)(w + L.ctrl), N, L.mt, nrhs, stream))) return rc;
  if ((rc = launch_tile_copy(dB, ldb, Bt, M, nrhs, p.nb, p.nb, L.mt, L.nrt, false, stream))) return rc;
  return make_handle(M, N, p, false, dwork, work_bytes, out);
}

int hqr_solve(int64_t M, int64_t N, const hqr_params* params, const hqr_exec* exec, const void* dwork,
              size_t work_bytes, double* dB, int64_t ldb, int32_t nrhs, void* bwork, size_t bwork_bytes,
              void* stream) {
  if (int rc = check_apply_args(M, N, params, dwork, dB, ldb, nrhs, bwork)) return rc;
  const hqr_params& p = *params;
  // B <- Q^T B, left in bwork's blocks of nb x 64
  int rc = run_apply(1, M, N, p, exec, dwork, work_bytes, dB, ldb, nrhs, bwork, bwork_bytes, stream, false, false);
  if (rc) return rc;
  const Layout L = layout_for(M, N, p);
  const ApplyLayout AL = apply_layout_for(M, nrhs, p);
  char* bw = (char*)bwork;
  double* Bb = (double*)(bw + AL.blocks);
  const double* tiles = (const double*)((const char*)dwork + L.tiles);
  if ((rc = launch_trsv(p.nb, tiles, Bb, 64, (int32_t*)(bw + AL.ctrl), N, L.mt, nrhs, stream))) return rc;
  return launch_tile_copy(dB, ldb, Bb, M, nrhs, p.nb, 64, AL.mt, AL.nbc, false, stream);
}

int hqr_factors_apply_workspace_size(const hqr_factors* f, int32_t nrhs, size_t* bytes) {
  if (!f) return -1;
  if (nrhs < 1) return -2;
  if (!bytes) return -3;
  *bytes = apply_layout_for(f->M, nrhs, f->p, f->f32 ? sizeof(float) : sizeof(double)).total;
  return 0;
}

int hqr_factors_apply_qt(const hqr_factors* f, const hqr_exec* exec, double* dB, int64_t ldb, int32_t nrhs,
                         void* bwork, size_t bwork_bytes, void* stream) {
  if (int rc = check_handle_args(f, dB, ldb, nrhs, bwork)) return rc;
  return map_apply_rc(run_apply(1, f->M, f->N, f->p, exec, f->dwork, f->work_bytes, dB, ldb, nrhs, bwork,
                                bwork_bytes, stream, true, f->f32));
}

int hqr_factors_apply_q(const hqr_factors* f, const hqr_exec* exec, double* dB, int64_t ldb, int32_t nrhs,
                        void* bwork, size_t bwork_bytes, void* stream) {
  if (int rc = check_handle_args(f, dB, ldb, nrhs, bwork)) return rc;
  return map_apply_rc(run_apply(0, f->M, f->N, f->p, exec, f->dwork, f->work_bytes, dB, ldb, nrhs, bwork,
                                bwork_bytes, stream, true, f->f32));
}

int hqr_factors_solve(const hqr_factors* f, const hqr_exec* exec, double* dB, int64_t ldb, int32_t nrhs,
                      void* bwork, size_t bwork_bytes, void* stream) {
  if (int rc = check_handle_args(f, dB, ldb, nrhs, bwork)) return rc;
  if (f->f32) return -1;
  return map_apply_rc(hqr_solve(f->M, f->N, &f->p, exec, f->dwork, f->work_bytes, dB, ldb, nrhs, bwork,
                                bwork_bytes, stream));
}

int hqr_factors_query(const hqr_factors* f, int64_t* M, int64_t* N, hqr_params* params, const void** dwork,
                      size_t* work_bytes) {
  if (!f) return -1;
  if (M) *M = f->M;
  if (N) *N = f->N;
  if (params) *params = f->p;
  if (dwork) *dwork = f->dwork;
  if (work_bytes) *work_bytes = f->work_bytes;
  return 0;
}

void hqr_factors_destroy(hqr_factors* f) { delete f; }

int hqr_status(const void* dwork, void* stream, int32_t* status) {
  return hqr_status_ex(dwork, stream, 0.0, status, nullptr);
}

int hqr_status_ex(const void* dwork, void* stream, double timeout_s, int32_t* status, int32_t* detail) {
  if (!dwork) return -1;
  if (!status) return -4;
  if (timeout_s <= 0.0) timeout_s = 300.0;
  // bounded wait: poll the stream instead of blocking in the runtime
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    hipError_t e = hipStreamQuery((hipStream_t)stream);
    if (e == hipSuccess) break;
    if (e != hipErrorNotReady) return record_hip(e, "hipStreamQuery");
    const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (dt > timeout_s) {
      if (g_trace) {
        // what every traced workgroup was doing when the time ran out
        int counts[6] = {0, 0, 0, 0, 0, 0};
        for (int b = 0; b < kTraceSlots; ++b) {
          const int ph = g_trace[2 * b + 1];
          counts[(ph >= 0 && ph <= 5) ? ph : 0]++;
        }
        fprintf(stderr, "hqr: stream still busy after %.1f s; workgroups by phase: none %d popped %d ready %d "
                "done %d exit %d abort %d\n", dt, counts[0], counts[1], counts[2], counts[3], counts[4], counts[5]);
        int shown = 0;
        for (int b = 0; b < kTraceSlots && shown < 64; ++b) {
          const int ph = g_trace[2 * b + 1];
          if (ph == TR_POPPED || ph == TR_READY || ph == TR_DONE) {
            fprintf(stderr, "hqr:   wg %d task %d phase %d\n", b, g_trace[2 * b], ph);
            ++shown;
          }
        }
        fflush(stderr);
      }
      return HQR_ERR_TIMEOUT;
    }
    std::this_thread::sleep_for(std::chrono::microseconds(dt < 0.01 ? 20 : 1000));
  }
  int32_t ctrl[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (int rc = record_hip(hipMemcpy(ctrl, dwork, sizeof(ctrl), hipMemcpyDeviceToHost), "hipMemcpy(status)")) return rc;
  *status = ctrl[1];
  if (detail) {
    for (int q = 0; q < 4; ++q) detail[q] = ctrl[2 + q];
    if (ctrl[1] == HQR_ERR_SINGULAR) {
      detail[0] = ctrl[7] - ctrl[6];  // first zero diagonal entry of R
      detail[1] = detail[2] = detail[3] = 0;
    }
  }
  return 0;
}

void hqr_release_plans(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  for (auto& kv : g_plans)
    if (kv.second->d_tasks) (void)hipFree(kv.second->d_tasks);
  g_plans.clear();
}

const char* hqr_strerror(int code) {
  if (code == 0) return "success";
  if (code < 0) return "invalid argument";
  switch (code) {
    case HQR_ERR_HIP: return "HIP runtime error";
    case HQR_ERR_WATCHDOG: return "a task waited past the spin limit; results are invalid";
    case HQR_ERR_WORKSPACE: return "workspace too small";
    case HQR_ERR_NOMEM: return "allocation failed";
    case HQR_ERR_INTERNAL: return "internal error";
    case HQR_ERR_INVALID_LIST: return "elimination list breaks the validity rules";
    case HQR_ERR_TIMEOUT: return "the GPU work did not finish within the time limit";
    case HQR_ERR_SINGULAR: return "R has a zero diagonal entry (A is rank deficient)";
    case HQR_ERR_FACTORS: return "the workspace does not hold the factorization the arguments describe";
    default: return "unknown error";
  }
}

const char* hqr_last_error(void) { return last_error(); }

int hqr_timeline(void* stream, uint64_t* out, int64_t cap, int64_t* count) {
  if (!count) return -4;
  *count = g_timeline ? g_timeline_n : 0;
  if (!out || !g_timeline) return 0;
  if (cap < g_timeline_n) return -3;
  if (int rc = record_hip(hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize")) return rc;
  return record_hip(hipMemcpy(out, g_timeline, (size_t)g_timeline_n * 4 * sizeof(uint64_t), hipMemcpyDeviceToHost),
                    "hipMemcpy(timeline)");
}

const char* hqr_version(void) { return "hqr-mi355x 0.1"; }

}  // extern "C"
