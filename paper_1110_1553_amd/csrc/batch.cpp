// Batched factorizations and least-squares solves: many independent
// problems (each its own tile grid, elimination list and task graph) run in
// one persistent launch, plus one batched copy-in, one batched back
// substitution and one batched copy-out (entry points hqr_batch_* and
// hqr_lstsq_batched of include/hqr.h).
//
// Batch workspace (offsets from its start, which is also the control block
// read by hqr_status):
//   ctrl      kCtrlWords int32: task cursor, status, watchdog detail
//   info      count int32: per problem, max(N - j) over zero diagonal entries R_jj
//   counters  every problem's dependency counters, back to back
//   desc      count problem descriptors (ProbDesc)
//   tasks     the merged task list (DevTask) and the problem of each task
//   data      per problem: T factors of GEQRT and TSQRT/TTQRT, then the tiles
//             of A followed by the right-hand-side tile columns
// Everything from `desc` to `data` is uploaded by hqr_batch_bind; hqr_batch_run
// only launches kernels, so it can be captured into a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <queue>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/hqr.h"
#include "elim.hpp"
#include "layout.hpp"
#include "task.hpp"

namespace hqr {
// One problem's factors copied out of a batch workspace into a workspace of
// the single-problem layout (hqr_batch_export_all).  Byte offsets; every
// region is 256-byte aligned and a multiple of 16 bytes long.
struct ExportDesc {
  char* dst;          // destination workspace, null: the problem is skipped
  int64_t zero_bytes; // control words at its start, cleared (the signature words set to `sig`)
  int64_t tg_dst, tk_dst, tiles_dst;
  int64_t tg_src, tk_src, tiles_src;  // in the batch workspace
  int64_t tsz, asz;   // bytes of each T array, of the matrix tiles
  FactorSig sig;      // signature of the factorization (control words kSigWord..)
};
}  // namespace hqr

struct hqr_batch {
  int32_t count = 0;
  hqr_params p{};
  hqr_exec ex{};
  std::vector<int64_t> M, N;
  std::vector<int32_t> nrhs;
  std::vector<hqr::ProbDesc> desc;  // offsets set at creation, caller pointers at bind
  std::vector<hqr::DevTask> tasks;  // merged dispatch order
  std::vector<int32_t> prob;        // problem of each task
  size_t off_info = 0, off_cnt = 0, off_desc = 0, off_tasks = 0, off_prob = 0, off_export = 0, off_data = 0, total = 0;
  int32_t max_nrhs = 0;             // widest back substitution (workgroups per problem)
  int64_t max_elems = 0;            // padded elements of the largest problem (copy grid)
  void* bound_work = nullptr;       // workspace the descriptors were uploaded to
};

namespace hqr {
namespace {

// Host plans per shape (the tile grid, the algorithm parameters and the
// active column chunks); kept for the life of the process.
struct HostKey {
  int32_t mt, nt, nb, p, a, low, high, coupling, domino, order, last_a, nrhs;
  bool operator<(const HostKey& o) const {
    return std::tie(mt, nt, nb, p, a, low, high, coupling, domino, order, last_a, nrhs) <
           std::tie(o.mt, o.nt, o.nb, o.p, o.a, o.low, o.high, o.coupling, o.domino, o.order, o.last_a, o.nrhs);
  }
};

std::mutex g_host_mu;
std::map<HostKey, std::unique_ptr<Plan>> g_host_plans;

}  // namespace

int host_plan(int32_t mt, int32_t nt, const hqr_params& p, int order, const ColumnChunks& cc, const Plan** out) {
  HostKey key{mt, nt, p.nb, p.p, p.a, p.low, p.high, p.coupling, p.domino, order, cc.last_a, cc.nrhs_cols};
  std::lock_guard<std::mutex> lock(g_host_mu);
  auto it = g_host_plans.find(key);
  if (it == g_host_plans.end()) {
    std::unique_ptr<Plan> plan(new Plan());
    if (int rc = build_plan(mt, nt, p, order, chunks_for(p.nb), *plan, cc)) return rc;
    it = g_host_plans.emplace(key, std::move(plan)).first;
  }
  *out = it->second.get();
  return 0;
}

namespace {

// Pinned staging buffers for the uploads of hqr_batch_bind, a few per
// device, reused round robin; a buffer is rewritten only after the copy that
// last read it has completed.
struct StageSlot {
  void* host = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;
};
constexpr int kStageSlots = 4;
struct StageRing {
  StageSlot slot[kStageSlots];
  int next = 0;
};
std::mutex g_stage_mu;
std::map<int, StageRing> g_rings;

int stage_upload(void* dst, const void* src, size_t bytes, hipStream_t stream) {
  if (bytes == 0) return 0;
  int dev = 0;
  if (int rc = record_hip(hipGetDevice(&dev), "hipGetDevice")) return rc;
  std::lock_guard<std::mutex> lock(g_stage_mu);
  StageRing& ring = g_rings[dev];
  StageSlot& s = ring.slot[ring.next];
  ring.next = (ring.next + 1) % kStageSlots;
  if (s.pending) {
    if (int rc = record_hip(hipEventSynchronize(s.ev), "hipEventSynchronize(staging)")) return rc;
    s.pending = false;
  }
  if (s.cap < bytes) {
    if (s.host) (void)hipHostFree(s.host);
    s.host = nullptr;
    s.cap = 0;
    if (record_hip(hipHostMalloc(&s.host, bytes, hipHostMallocDefault), "hipHostMalloc(staging)")) return HQR_ERR_NOMEM;
    s.cap = bytes;
  }
  if (!s.ev && record_hip(hipEventCreateWithFlags(&s.ev, hipEventDisableTiming), "hipEventCreate(staging)"))
    return HQR_ERR_HIP;
  std::memcpy(s.host, src, bytes);
  if (int rc = record_hip(hipMemcpyAsync(dst, s.host, bytes, hipMemcpyHostToDevice, stream), "hipMemcpyAsync(batch)"))
    return rc;
  if (int rc = record_hip(hipEventRecord(s.ev, stream), "hipEventRecord(staging)")) return rc;
  s.pending = true;
  return 0;
}

}  // namespace
}  // namespace hqr

using namespace hqr;

// The status of a finished batch written by the device into host memory,
// in the form hqr_batch_status reports it: host[0] = status word,
// host[1 + q] = first zero diagonal index of problem q, or -1.
static __global__ void publish_status_kernel(const hqr::ProbDesc* d, const int32_t* ctrl, const int32_t* info,
                                             int count, int32_t* host) {
  if (threadIdx.x == 0) host[0] = ctrl[1];
  for (int q = threadIdx.x; q < count; q += blockDim.x) {
    const int32_t v = info[q];
    host[1 + q] = v > 0 ? (int32_t)(d[q].N - v) : -1;
  }
}

// Every kept problem of a batch in one launch: workgroup row blockIdx.y
// copies problem blockIdx.y, 16 bytes per thread and step.
static __global__ void export_batched_kernel(const hqr::ExportDesc* e, const char* w) {
  const hqr::ExportDesc d = e[blockIdx.y];
  if (!d.dst) return;
  const int64_t z = d.zero_bytes / 16, t = d.tsz / 16, a = d.asz / 16;
  const int64_t total = z + 2 * t + a;
  typedef unsigned int u4v __attribute__((ext_vector_type(4)));
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    u4v v = {0u, 0u, 0u, 0u};
    char* o;
    if (x < z) {
      o = d.dst + 16 * x;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int64_t word = 4 * x + k;
        if (word >= hqr::kSigWord && word < hqr::kSigWord + hqr::kSigWords) v[k] = (unsigned)d.sig.w[word - hqr::kSigWord];
      }
    } else if (x < z + t) {
      v = ((const u4v*)(w + d.tg_src))[x - z];
      o = d.dst + d.tg_dst + 16 * (x - z);
    } else if (x < z + 2 * t) {
      v = ((const u4v*)(w + d.tk_src))[x - z - t];
      o = d.dst + d.tk_dst + 16 * (x - z - t);
    } else {
      v = ((const u4v*)(w + d.tiles_src))[x - z - 2 * t];
      o = d.dst + d.tiles_dst + 16 * (x - z - 2 * t);
    }
    *(u4v*)o = v;
  }
}

extern "C" {

int hqr_batch_create(int32_t count, const int64_t* M, const int64_t* N, const int32_t* nrhs,
                     const hqr_params* params, const hqr_exec* exec, hqr_batch** out) {
  if (count < 1 || count > 65535) return -1;
  if (!M) return -2;
  if (!N) return -3;
  if (!params || check_params(*params) || params->precision != HQR_PREC_FP64) return -5;
  hqr_exec ex{0, 0, 0, nullptr, nullptr};
  if (exec) ex = *exec;
  if (ex.order != 0 && ex.order != 1) return -6;
  if (!out) return -7;
  *out = nullptr;
  const hqr_params& p = *params;
  for (int32_t q = 0; q < count; ++q) {
    if (M[q] < 1) return -2;
    if (N[q] < 1 || N[q] > M[q]) return -3;
    if (nrhs && nrhs[q] < 0) return -4;
  }
  std::unique_ptr<hqr_batch> b(new hqr_batch());
  b->count = count;
  b->p = p;
  b->ex = ex;
  b->M.assign(M, M + count);
  b->N.assign(N, N + count);
  b->nrhs.assign(count, 0);
  if (nrhs) b->nrhs.assign(nrhs, nrhs + count);
  b->desc.resize(count);

  // per-problem host plans and sizes
  std::vector<const Plan*> plans(count);
  std::vector<Layout> lay(count);
  size_t ncnt = 0;
  for (int32_t q = 0; q < count; ++q) {
    const Layout L = layout_for(M[q], N[q], p, b->nrhs[q]);
    if (L.mt > 65535 || L.nt + L.nrt > 65535) return -2;
    ColumnChunks cc;
    cc.last_a = L.last_a;
    cc.nrhs_cols = b->nrhs[q];
    if (int rc = host_plan(L.mt, L.nt, p, ex.order, cc, &plans[q])) return rc;
    lay[q] = L;
    ncnt += (size_t)L.mt * (L.nt + L.nrt) * L.chunks;
  }

  // merge the task lists: repeatedly take the head task of highest priority
  // (each problem's own dispatch order is kept, so the merged order is a
  // topological order of the union of the task graphs)
  size_t ntasks = 0;
  for (const Plan* pl : plans) ntasks += pl->dev.size();
  if (ntasks > (size_t)INT32_MAX) return -1;
  b->tasks.reserve(ntasks);
  b->prob.reserve(ntasks);
  typedef std::pair<int64_t, int32_t> Head;  // (priority, -problem)
  std::priority_queue<Head> heads;
  std::vector<size_t> pos(count, 0);
  for (int32_t q = 0; q < count; ++q)
    if (!plans[q]->dev.empty()) heads.push({plans[q]->prio[0], -q});
  while (!heads.empty()) {
    const int32_t q = -heads.top().second;
    heads.pop();
    const Plan* pl = plans[q];
    b->tasks.push_back(pl->dev[pos[q]]);
    b->prob.push_back(q);
    if (++pos[q] < pl->dev.size()) heads.push({pl->prio[pos[q]], -q});
  }

  // workspace layout
  size_t off = align256(kCtrlWords * sizeof(int32_t));
  b->off_info = off;
  off += (size_t)count * sizeof(int32_t);
  b->off_cnt = off;
  size_t cnt_at = off;
  off = align256(off + ncnt * sizeof(int32_t));
  b->off_desc = off;
  off = align256(off + (size_t)count * sizeof(ProbDesc));
  b->off_tasks = off;
  off = align256(off + ntasks * sizeof(DevTask));
  b->off_prob = off;
  off = align256(off + ntasks * sizeof(int32_t));
  b->off_export = off;
  off = align256(off + (size_t)count * sizeof(ExportDesc));
  b->off_data = off;
  for (int32_t q = 0; q < count; ++q) {
    const Layout& L = lay[q];
    ProbDesc& d = b->desc[q];
    std::memset(&d, 0, sizeof(d));
    d.M = M[q];
    d.N = N[q];
    d.nrhs = b->nrhs[q];
    d.mt = L.mt;
    d.nt = L.nt;
    d.nrt = L.nrt;
    d.cnt = (int64_t)cnt_at;
    cnt_at += (size_t)L.mt * (L.nt + L.nrt) * L.chunks * sizeof(int32_t);
    const size_t tiles = (size_t)L.mt * L.nt, all = (size_t)L.mt * (L.nt + L.nrt);
    d.tg = (int64_t)off;
    off = align256(off + tiles * (size_t)p.nb * 16 * sizeof(double));
    d.tk = (int64_t)off;
    off = align256(off + tiles * (size_t)p.nb * 16 * sizeof(double));
    d.tiles = (int64_t)off;
    off = align256(off + all * (size_t)p.nb * p.nb * sizeof(double));
    b->max_elems = std::max<int64_t>(b->max_elems, (int64_t)all * p.nb * p.nb);
    b->max_nrhs = std::max<int32_t>(b->max_nrhs, b->nrhs[q]);
  }
  b->total = off;
  *out = b.release();
  return 0;
}

int hqr_batch_workspace_size(const hqr_batch* b, size_t* bytes) {
  if (!b) return -1;
  if (!bytes) return -2;
  *bytes = b->total;
  return 0;
}

int hqr_batch_num_tasks(const hqr_batch* b, hqr_task* tasks, int32_t* prob, int64_t cap, int64_t* count) {
  if (!b) return -1;
  if (!count) return -5;
  *count = (int64_t)b->tasks.size();
  if (!tasks && !prob) return 0;
  if (cap < *count) return -4;
  static_assert(sizeof(hqr_task) == sizeof(DevTask), "task record layouts differ");
  if (tasks) std::memcpy(tasks, b->tasks.data(), b->tasks.size() * sizeof(DevTask));
  if (prob) std::memcpy(prob, b->prob.data(), b->prob.size() * sizeof(int32_t));
  return 0;
}

int hqr_batch_bind(hqr_batch* b, double* const* dA, const int64_t* lda, double* const* dB, const int64_t* ldb,
                   void* dwork, size_t work_bytes, void* stream) {
  if (!b) return -1;
  if (!dA) return -2;
  if (!lda) return -3;
  bool rhs = false;
  for (int32_t q = 0; q < b->count; ++q) rhs = rhs || b->nrhs[q] > 0;
  if (rhs && !dB) return -4;
  if (rhs && !ldb) return -5;
  if (!dwork) return -6;
  if (work_bytes < b->total) return -7;
  for (int32_t q = 0; q < b->count; ++q) {
    if (!dA[q]) return -2;
    if (lda[q] < b->M[q]) return -3;
    if (b->nrhs[q] > 0) {
      if (!dB[q]) return -4;
      if (ldb[q] < b->M[q]) return -5;
    }
  }
  for (int32_t q = 0; q < b->count; ++q) {
    ProbDesc& d = b->desc[q];
    d.A = dA[q];
    d.lda = lda[q];
    d.B = b->nrhs[q] > 0 ? dB[q] : nullptr;
    d.ldb = b->nrhs[q] > 0 ? ldb[q] : 0;
  }
  std::vector<char> blob(b->off_data - b->off_desc, 0);
  std::memcpy(blob.data(), b->desc.data(), b->desc.size() * sizeof(ProbDesc));
  if (!b->tasks.empty()) {
    std::memcpy(blob.data() + (b->off_tasks - b->off_desc), b->tasks.data(), b->tasks.size() * sizeof(DevTask));
    std::memcpy(blob.data() + (b->off_prob - b->off_desc), b->prob.data(), b->prob.size() * sizeof(int32_t));
  }
  if (int rc = stage_upload((char*)dwork + b->off_desc, blob.data(), blob.size(), (hipStream_t)stream)) return rc;
  b->bound_work = dwork;
  return 0;
}

int hqr_batch_run(const hqr_batch* b, void* dwork, size_t work_bytes, void* stream) {
  if (!b) return -1;
  if (!dwork || dwork != b->bound_work) return -2;
  if (work_bytes < b->total) return -3;
  char* w = (char*)dwork;
  const ProbDesc* d = (const ProbDesc*)(w + b->off_desc);
  const int nb = b->p.nb;
  // control words, per-problem info and every dependency counter
  if (int rc = launch_zero_i32((int32_t*)w, (int64_t)(b->off_desc / sizeof(int32_t)), stream)) return rc;
  if (int rc = launch_copy_batched(d, w, b->count, nb, true, b->max_elems, stream)) return rc;
  if (!b->tasks.empty()) {
    LaunchArgs a{};
    a.ctrl = (int32_t*)w;
    a.tasks = (const DevTask*)(w + b->off_tasks);
    a.task_prob = (const int32_t*)(w + b->off_prob);
    a.probs = d;
    a.ntasks = (int64_t)b->tasks.size();
    a.spin_limit = b->ex.spin_limit > 0 ? b->ex.spin_limit : kDefaultSpinLimit;
    a.chunks = chunks_for(nb);
    a.lda = nb;
    // per-problem fields (A, Tg, Tk, cnt, mt, nt, cnt_cols) are set per task
    const int workers = b->ex.workers > 0 ? b->ex.workers : default_workers(nb);
    if (b->ex.ev_begin && record_hip(hipEventRecord((hipEvent_t)b->ex.ev_begin, (hipStream_t)stream),
                                     "hipEventRecord(ev_begin)"))
      return HQR_ERR_HIP;
    if (int rc = launch_persistent(nb, a, workers, stream)) return rc;
    if (b->ex.ev_end && record_hip(hipEventRecord((hipEvent_t)b->ex.ev_end, (hipStream_t)stream),
                                   "hipEventRecord(ev_end)"))
      return HQR_ERR_HIP;
  }
  if (b->max_nrhs > 0) {
    if (int rc = launch_trsv_batched(nb, d, w, (int32_t*)w, (int32_t*)(w + b->off_info), b->count, b->max_nrhs,
                                     stream))
      return rc;
  }
  return launch_copy_batched(d, w, b->count, nb, false, b->max_elems, stream);
}

int hqr_batch_status(const hqr_batch* b, const void* dwork, void* stream, double timeout_s, int32_t* status,
                     int32_t* first_zero) {
  if (!b) return -1;
  if (!dwork) return -2;
  if (!status) return -5;
  hipStream_t s = (hipStream_t)stream;
  if (timeout_s <= 0.0) timeout_s = 300.0;
  // bounded wait for `stream`, then reads through that stream only (the
  // batch may have finished while later work still runs on another stream)
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    hipError_t e = hipStreamQuery(s);
    if (e == hipSuccess) break;
    if (e != hipErrorNotReady) return record_hip(e, "hipStreamQuery");
    if (std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > timeout_s)
      return HQR_ERR_TIMEOUT;
    std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  std::vector<int32_t> words(b->off_info / sizeof(int32_t) + b->count, 0);
  if (int rc = record_hip(hipMemcpyAsync(words.data(), dwork, words.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s),
                          "hipMemcpyAsync(batch status)"))
    return rc;
  if (int rc = record_hip(hipStreamSynchronize(s), "hipStreamSynchronize(batch status)")) return rc;
  *status = words[1];
  if (first_zero) {
    const int32_t* info = words.data() + b->off_info / sizeof(int32_t);
    for (int32_t q = 0; q < b->count; ++q) first_zero[q] = info[q] > 0 ? (int32_t)(b->N[q] - info[q]) : -1;
  }
  return 0;
}

int hqr_batch_publish_status(const hqr_batch* b, const void* dwork, int32_t* host, void* stream) {
  if (!b) return -1;
  if (!dwork) return -2;
  if (!host) return -3;
  const char* w = (const char*)dwork;
  hipLaunchKernelGGL(publish_status_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream,
                     (const ProbDesc*)(w + b->off_desc), (const int32_t*)w, (const int32_t*)(w + b->off_info),
                     b->count, host);
  return record_hip(hipGetLastError(), "publish_status_kernel launch");
}

int hqr_batch_export_factors(const hqr_batch* b, int32_t q, const void* dwork, void* dst, size_t dst_bytes,
                             void* stream) {
  if (!b) return -1;
  if (q < 0 || q >= b->count) return -2;
  if (!dwork) return -3;
  if (!dst) return -4;
  const Layout L = layout_for(b->M[q], b->N[q], b->p);
  if (dst_bytes < L.total) return -5;
  const ProbDesc& d = b->desc[q];
  const char* w = (const char*)dwork;
  char* o = (char*)dst;
  hipStream_t s = (hipStream_t)stream;
  const size_t tsz = (size_t)L.mt * L.nt * b->p.nb * 16 * sizeof(double);
  const size_t asz = (size_t)L.mt * L.nt * b->p.nb * b->p.nb * sizeof(double);
  // control words of the copy start at zero (a status read finds no error), with the signature of the
  // factorization for the apply entry points
  if (int rc = launch_init_ctrl((int32_t*)o, factor_sig(L, b->p, sizeof(double)), nullptr, 0, stream)) return rc;
  if (int rc = record_hip(hipMemcpyAsync(o + L.tg, w + d.tg, tsz, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync(Tg)"))
    return rc;
  if (int rc = record_hip(hipMemcpyAsync(o + L.tk, w + d.tk, tsz, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync(Tk)"))
    return rc;
  return record_hip(hipMemcpyAsync(o + L.tiles, w + d.tiles, asz, hipMemcpyDeviceToDevice, s),
                    "hipMemcpyAsync(tiles)");
}

int hqr_batch_export_all(const hqr_batch* b, void* dwork, void* const* dst, const size_t* dst_bytes, void* stream) {
  if (!b) return -1;
  if (!dwork || dwork != b->bound_work) return -2;
  if (!dst) return -3;
  if (!dst_bytes) return -4;
  std::vector<ExportDesc> e((size_t)b->count);
  int64_t units = 0;
  for (int32_t q = 0; q < b->count; ++q) {
    ExportDesc& x = e[q];
    std::memset(&x, 0, sizeof(x));
    if (!dst[q]) continue;
    const Layout L = layout_for(b->M[q], b->N[q], b->p);
    if (dst_bytes[q] < L.total) return -5;
    const ProbDesc& d = b->desc[q];
    x.dst = (char*)dst[q];
    x.zero_bytes = (int64_t)L.tg;
    x.sig = factor_sig(L, b->p, sizeof(double));
    x.tg_dst = (int64_t)L.tg;
    x.tk_dst = (int64_t)L.tk;
    x.tiles_dst = (int64_t)L.tiles;
    x.tg_src = d.tg;
    x.tk_src = d.tk;
    x.tiles_src = d.tiles;
    x.tsz = (int64_t)L.mt * L.nt * b->p.nb * 16 * (int64_t)sizeof(double);
    x.asz = (int64_t)L.mt * L.nt * b->p.nb * b->p.nb * (int64_t)sizeof(double);
    units = std::max<int64_t>(units, (x.zero_bytes + 2 * x.tsz + x.asz) / 16);
  }
  if (units == 0) return 0;
  char* w = (char*)dwork;
  if (int rc = stage_upload(w + b->off_export, e.data(), e.size() * sizeof(ExportDesc), (hipStream_t)stream))
    return rc;
  // workgroups per problem: about eight 16-byte steps per thread of the largest problem
  const int64_t gx = std::min<int64_t>(1024, std::max<int64_t>(1, (units + 2047) / 2048));
  hipLaunchKernelGGL(export_batched_kernel, dim3((unsigned)gx, (unsigned)b->count), dim3(256), 0,
                     (hipStream_t)stream, (const ExportDesc*)(w + b->off_export), (const char*)w);
  return record_hip(hipGetLastError(), "export_batched_kernel launch");
}

void hqr_batch_destroy(hqr_batch* b) { delete b; }

int hqr_lstsq_batched_workspace_size(int32_t count, const int64_t* M, const int64_t* N, const int32_t* nrhs,
                                     const hqr_params* params, size_t* bytes) {
  if (!bytes) return -6;
  hqr_batch* b = nullptr;
  if (int rc = hqr_batch_create(count, M, N, nrhs, params, nullptr, &b)) return rc == -7 ? -6 : rc;
  *bytes = b->total;
  hqr_batch_destroy(b);
  return 0;
}

int hqr_lstsq_batched(int32_t count, double* const* dA, const int64_t* M, const int64_t* N, const int64_t* lda,
                      double* const* dB, const int64_t* ldb, const int32_t* nrhs, const hqr_params* params,
                      const hqr_exec* exec, void* dwork, size_t work_bytes, void* stream) {
  if (count < 1 || count > 65535) return -1;
  if (!dA) return -2;
  if (!M) return -3;
  if (!N) return -4;
  if (!lda) return -5;
  hqr_batch* b = nullptr;
  int rc = hqr_batch_create(count, M, N, nrhs, params, exec, &b);
  if (rc) {
    static const int map_create[8] = {0, -1, -3, -4, -8, -9, -10, -1};  // create's argument -> this call's
    return rc < 0 ? map_create[-rc] : rc;
  }
  rc = hqr_batch_bind(b, dA, lda, dB, ldb, dwork, work_bytes, stream);
  if (rc < 0) {
    static const int map_bind[8] = {0, -1, -2, -5, -6, -7, -11, -12};
    rc = map_bind[-rc];
  }
  if (!rc) rc = hqr_batch_run(b, dwork, work_bytes, stream);
  hqr_batch_destroy(b);
  return rc;
}

}  // extern "C"
