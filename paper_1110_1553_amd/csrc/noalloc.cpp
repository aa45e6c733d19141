// Least squares without device allocation (hqr_lstsq_noalloc of
// include/hqr.h): the same launches as hqr_lstsq, with the workspace and the
// task plan in a static device array instead of caller or library
// allocations.
//
// Layout of the array for one call: the workspace of hqr_lstsq (control
// words, T factors, tiles of A and B, dependency counters) from offset 0,
// then the task plan at the next 256-byte boundary.  Everything the kernels
// read before writing is cleared or uploaded by the call itself: the control
// words and counters by the init kernel, the tiles by the copy-in kernel
// (zero padding included), the T factors by the panel tasks, the plan by an
// upload that is skipped when the array still holds the same plan at the
// same offset from the previous call on this device.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "../../include/hqr.h"
#include "elim.hpp"
#include "layout.hpp"
#include "task.hpp"

namespace hqr {
namespace {

constexpr size_t kScratchBytes = (size_t)HQR_NOALLOC_SCRATCH_BYTES;

// One copy per device, part of this library's code object and held until the
// process ends.  In host code the name stands for a host-side shadow, not a
// device address: host code uses the address hipGetSymbolAddress returns.
__device__ __attribute__((aligned(256))) unsigned char scratch[kScratchBytes];

struct DeviceScratch {
  unsigned char* ptr = nullptr;  // device address of `scratch` on this device
  const Plan* plan = nullptr;    // plan uploaded by the last call on this device
  size_t plan_off = 0;
};
constexpr int kMaxDevices = 64;
std::mutex g_mu;
DeviceScratch g_scratch[kMaxDevices];

// Status word and detail of the call, in the form of hqr_status_ex:
// out[0] = status, out[1..4] = detail.
__global__ void report_kernel(const int32_t* ctrl, int32_t* out) {
  if (threadIdx.x != 0) return;
  const int32_t st = ctrl[1];
  out[0] = st;
  if (st == HQR_ERR_SINGULAR) {
    out[1] = ctrl[7] - ctrl[6];
    out[2] = out[3] = out[4] = 0;
  } else {
    for (int q = 0; q < 4; ++q) out[1 + q] = ctrl[2 + q];
  }
}

}  // namespace
}  // namespace hqr

using namespace hqr;

extern "C" {

int hqr_lstsq_noalloc(double* dA, int64_t M, int64_t N, int64_t lda, double* dB, int64_t ldb, int32_t nrhs,
                      const hqr_params* params, const hqr_exec* exec, int32_t* dinfo, void* stream) {
  if (!dA) return -1;
  if (M < 1 || M < N) return -2;
  if (N < 1) return -3;
  if (lda < M) return -4;
  if (!dB) return -5;
  if (ldb < M) return -6;
  if (nrhs < 1) return -7;
  if (!params || check_params(*params) || params->precision != HQR_PREC_FP64) return -8;
  hqr_exec ex{0, 0, 0, nullptr, nullptr};
  if (exec) ex = *exec;
  if (ex.order != 0 && ex.order != 1) return -9;
  const hqr_params& p = *params;
  const Layout L = layout_for(M, N, p, nrhs);
  if (L.mt > 65535 || L.nt + L.nrt > 65535) return -2;
  // the host plan (host memory; built on the first call for this shape and tree)
  ColumnChunks cc;
  cc.last_a = L.last_a;
  cc.nrhs_cols = nrhs;
  const Plan* plan = nullptr;
  if (int rc = host_plan(L.mt, L.nt, p, ex.order, cc, &plan)) return rc;
  const size_t plan_off = align256(L.total);
  const size_t plan_bytes = plan->dev.size() * sizeof(DevTask);
  if (plan_off + plan_bytes > kScratchBytes) {
    char msg[256];
    snprintf(msg, sizeof(msg),
             "hqr_lstsq_noalloc: %lld x %lld with %d right-hand sides needs %zu bytes of scratch, the static array "
             "holds %zu",
             (long long)M, (long long)N, (int)nrhs, plan_off + plan_bytes, kScratchBytes);
    set_last_error(msg);
    return HQR_ERR_WORKSPACE;
  }
  int dev = 0;
  if (int rc = record_hip(hipGetDevice(&dev), "hipGetDevice")) return rc;
  if (dev < 0 || dev >= kMaxDevices) return HQR_ERR_INTERNAL;
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceScratch& ds = g_scratch[dev];
    if (!ds.ptr) {
      // once per device, with that device current: the device address of this device's copy
      void* ptr = nullptr;
      if (int rc = record_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"))
        return rc;
      ds.ptr = (unsigned char*)ptr;
    }
    base = ds.ptr;
    if (ds.plan != plan || ds.plan_off != plan_off) {
      if (plan_bytes > 0) {
        if (int rc = record_hip(hipMemcpyAsync(base + plan_off, plan->dev.data(), plan_bytes, hipMemcpyHostToDevice,
                                               (hipStream_t)stream),
                                "hipMemcpyAsync(plan into scratch)"))
          return rc;
      }
      ds.plan = plan;
      ds.plan_off = plan_off;
    }
  }
  int rc = run_factor(dA, M, N, lda, p, ex, base, dB, ldb, nrhs, stream, true, false, false, base + plan_off,
                      (int64_t)plan->dev.size());
  if (rc) return rc;
  const double* tiles = (const double*)(base + L.tiles);
  double* Bt = (double*)(base + L.tiles) + (size_t)L.mt * L.nt * p.nb * p.nb;
  if ((rc = launch_trsv(p.nb, tiles, Bt, p.nb, (int32_t*)(base + L.ctrl), N, L.mt, nrhs, stream))) return rc;
  if ((rc = launch_tile_copy(dB, ldb, Bt, M, nrhs, p.nb, p.nb, L.mt, L.nrt, false, stream))) return rc;
  if (dinfo) {
    hipLaunchKernelGGL(report_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, (const int32_t*)(base + L.ctrl),
                       dinfo);
    if ((rc = record_hip(hipGetLastError(), "report_kernel launch"))) return rc;
  }
  return 0;
}

}  // extern "C"
