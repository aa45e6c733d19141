// Mixed-precision least squares: FP32 tiled QR of A, then iterative
// refinement of the augmented system
//     [ I   A ] [ r ]   [ b ]
//     [ A^T 0 ] [ x ] = [ 0 ]
// (Bjorck's refinement for least squares) with the residuals of both block
// rows in FP64 and each correction solved with the FP32 factors
// (entry point hqr_lstsq_ir of include/hqr.h).
//
// With A = Q [R; 0], the correction of the residuals f = b - r - A x and
// g = -A^T r is
//     h = R^{-T} g,   d = Q^T f,   dx = R^{-1} (d(0:N) - h),   dr = Q [h; d(N:M)]
// and x += dx, r += dr.  The first iterate is the FP32 least-squares
// solution x = R^{-1} (Q^T b)(0:N), with Q^T b left in a tile column that
// the factorization carries along, and r = b - A x in FP64: the first
// correction from x = r = 0 gives the same x at the cost of two Q
// applications (and an FP32 r).  The iterate is judged by the
// normwise backward error of the augmented system,
//     eta = sqrt(||f||^2 + ||g||^2) / (||A||_F (||x|| + ||r||) + ||b||),
// evaluated before each correction; the loop stops once eta <= tol, when a
// correction did not lower eta (the attainable accuracy is reached; the
// iterate before that correction is returned), or after max_iter
// corrections.
//
// Workspace: the FP32 factorization (tiles and T factors, b as a further
// tile column), the FP32 block of
// the Q applications, then the FP64 vectors x (N), r (M), f (M), g (N),
// y (N) and four words for the norms.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "../../include/hqr.h"
#include "elim.hpp"
#include "layout.hpp"
#include "task.hpp"

namespace hqr {
namespace {

struct IrLayout {
  Layout fac;
  ApplyLayout app;
  size_t app_off, x, r, f, g, y, xp, rp, norms, total;
};

IrLayout ir_layout(int64_t M, int64_t N, const hqr_params& p) {
  IrLayout L{};
  L.fac = layout_for(M, N, p, 1, sizeof(float));  // b carried as a tile column
  L.app = apply_layout_for(M, 1, p, sizeof(float));
  size_t off = L.fac.total;
  L.app_off = off; off = align256(off + L.app.total);
  L.x = off; off = align256(off + (size_t)N * sizeof(double));
  L.r = off; off = align256(off + (size_t)M * sizeof(double));
  L.f = off; off = align256(off + (size_t)M * sizeof(double));
  L.g = off; off = align256(off + (size_t)N * sizeof(double));
  L.y = off; off = align256(off + (size_t)N * sizeof(double));
  L.xp = off; off = align256(off + (size_t)N * sizeof(double));
  L.rp = off; off = align256(off + (size_t)M * sizeof(double));
  L.norms = off; off = align256(off + 4 * sizeof(double));
  L.total = off;
  return L;
}

}  // namespace
}  // namespace hqr

using namespace hqr;

extern "C" {

int hqr_lstsq_ir_workspace_size(int64_t M, int64_t N, const hqr_params* params, size_t* bytes) {
  if (M < 1 || M < N) return -1;
  if (N < 1) return -2;
  if (!params || check_params(*params)) return -3;
  if (!bytes) return -4;
  *bytes = ir_layout(M, N, *params).total;
  return 0;
}

int hqr_lstsq_ir(const double* dA, int64_t M, int64_t N, int64_t lda, const double* db, double* dx, double* dr,
                 const hqr_params* params, const hqr_exec* exec, int32_t max_iter, double tol, void* dwork,
                 size_t work_bytes, void* stream, hqr_ir_info* info) {
  if (!dA) return -1;
  if (M < 1 || M < N) return -2;
  if (N < 1) return -3;
  if (lda < M) return -4;
  if (!db) return -5;
  if (!dx) return -6;
  if (!params || check_params(*params)) return -8;
  hqr_exec ex{0, 0, 0, nullptr, nullptr};
  if (exec) ex = *exec;
  if (ex.order != 0 && ex.order != 1) return -9;
  if (max_iter < 1) return -10;
  if (!(tol >= 0.0)) return -11;
  if (!dwork) return -12;
  const hqr_params& p = *params;
  const IrLayout L = ir_layout(M, N, p);
  if (L.fac.mt > 65535 || L.fac.nt > 65535) return -2;
  if (work_bytes < L.total) return -13;
  if (info) std::memset(info, 0, sizeof(*info));
  char* w = (char*)dwork;
  double* x = (double*)(w + L.x);
  double* r = (double*)(w + L.r);
  double* f = (double*)(w + L.f);
  double* g = (double*)(w + L.g);
  double* y = (double*)(w + L.y);
  double* xp = (double*)(w + L.xp);  // the iterate before the last correction
  double* rp = (double*)(w + L.rp);
  double* norms = (double*)(w + L.norms);
  double* colsq = y;  // squared column norms of A, before y is needed
  const float* Rt = (const float*)(w + L.fac.tiles);
  void* bwork = w + L.app_off;
  hipStream_t s = (hipStream_t)stream;
  int rc;
  // FP32 factorization of A with b carried along as a tile column, so that
  // the update kernels leave Q^T b in it (A and b themselves are left
  // untouched: copied and rounded into the tiles)
  if ((rc = run_factor(const_cast<double*>(dA), M, N, lda, p, ex, dwork, const_cast<double*>(db), M, 1, stream, false,
                       true, false)))
    return rc;
  // the FP32 least-squares solution x = R^{-1} (Q^T b)(0:N), and its
  // residual r = b - A x in FP64: the first correction of the iteration from
  // x = r = 0, without its two Q applications
  {
    const float* Bt = Rt + (size_t)L.fac.mt * L.fac.nt * p.nb * p.nb;
    if ((rc = launch_tile_copy(f, 0, M, const_cast<float*>(Bt), 1, M, 1, p.nb, p.nb, L.fac.mt, 1, false, stream)))
      return rc;
    if ((rc = record_hip(hipMemcpyAsync(x, f, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, s),
                         "hipMemcpyAsync(x0)")))
      return rc;
    if ((rc = launch_ir_trsv(Rt, p.nb, L.fac.mt, N, x, false, stream))) return rc;
    if ((rc = launch_ir_residual(dA, lda, M, N, x, db, nullptr, r, stream))) return rc;
  }
  // ||A||_F and ||b||, once
  auto read_norms = [&](double* host) -> int {
    if (int e = record_hip(hipMemcpyAsync(host, norms, 4 * sizeof(double), hipMemcpyDeviceToHost, s),
                           "hipMemcpyAsync(ir norms)"))
      return e;
    return record_hip(hipStreamSynchronize(s), "hipStreamSynchronize(ir)");
  };
  if ((rc = launch_ir_atr(dA, lda, M, N, nullptr, colsq, stream))) return rc;
  {
    const double* v[4] = {colsq, db, nullptr, nullptr};
    const int64_t n[4] = {N, M, 0, 0};
    if ((rc = launch_ir_norms(v, n, norms, stream))) return rc;
  }
  double nrm[4];
  if ((rc = read_norms(nrm))) return rc;
  const double normA = std::sqrt(nrm[0]), normb = std::sqrt(nrm[1]);
  int it = 1;  // the FP32 solution counts as the first correction
  if (info) {
    info->history[0] = 1.0;  // x = r = 0
    info->history_len = 1;
  }
  double eta = INFINITY, prev = INFINITY;
  bool converged = false;
  for (;;) {
    if ((rc = launch_ir_residual(dA, lda, M, N, x, db, r, f, stream))) return rc;       // f = b - r - A x
    if ((rc = launch_ir_atr(dA, lda, M, N, r, g, stream))) return rc;                   // g = -A^T r
    {
      const double* v[4] = {f, g, x, r};
      const int64_t n[4] = {M, N, N, M};
      if ((rc = launch_ir_norms(v, n, norms, stream))) return rc;
    }
    if ((rc = read_norms(nrm))) return rc;
    const double den = normA * (std::sqrt(nrm[2]) + std::sqrt(nrm[3])) + normb;
    eta = den > 0.0 ? std::sqrt(nrm[0] + nrm[1]) / den : 0.0;
    if (info && it < 32) {
      info->history[it] = eta;
      info->history_len = it + 1;
    }
    if (eta <= tol) {
      converged = true;
      break;
    }
    if (it > 0 && (!std::isfinite(eta) || eta >= prev)) {
      // the last correction did not lower eta: return the iterate before it
      if ((rc = record_hip(hipMemcpyAsync(x, xp, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, s),
                           "hipMemcpyAsync(x restore)")) ||
          (rc = record_hip(hipMemcpyAsync(r, rp, (size_t)M * sizeof(double), hipMemcpyDeviceToDevice, s),
                           "hipMemcpyAsync(r restore)")))
        return rc;
      eta = prev;
      --it;
      break;
    }
    if (it >= max_iter || !std::isfinite(eta)) break;
    prev = eta;
    if ((rc = record_hip(hipMemcpyAsync(xp, x, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, s),
                         "hipMemcpyAsync(x save)")) ||
        (rc = record_hip(hipMemcpyAsync(rp, r, (size_t)M * sizeof(double), hipMemcpyDeviceToDevice, s),
                         "hipMemcpyAsync(r save)")))
      return rc;
    if ((rc = launch_ir_trsv(Rt, p.nb, L.fac.mt, N, g, true, stream))) return rc;       // h = R^{-T} g
    if ((rc = run_apply(1, M, N, p, &ex, dwork, work_bytes, f, M, 1, bwork, L.app.total, stream, true, true)))
      return rc;                                                                         // f = Q^T f
    if ((rc = launch_ir_split(f, g, y, N, stream))) return rc;                          // y = d1 - h, d1 = h
    if ((rc = launch_ir_trsv(Rt, p.nb, L.fac.mt, N, y, false, stream))) return rc;      // dx = R^{-1} y
    if ((rc = run_apply(0, M, N, p, &ex, dwork, work_bytes, f, M, 1, bwork, L.app.total, stream, true, true)))
      return rc;                                                                         // dr = Q [h; d2]
    if ((rc = launch_ir_update(x, y, N, r, f, M, stream))) return rc;                    // x += dx, r += dr
    ++it;
  }
  // the launches record a watchdog abort in their control words
  int32_t st[2] = {0, 0};
  if ((rc = record_hip(hipMemcpyAsync(&st[0], w + L.fac.ctrl + sizeof(int32_t), sizeof(int32_t),
                                      hipMemcpyDeviceToHost, s), "hipMemcpyAsync(ir status)")))
    return rc;
  if ((rc = record_hip(hipMemcpyAsync(&st[1], w + L.app_off + L.app.ctrl + sizeof(int32_t), sizeof(int32_t),
                                      hipMemcpyDeviceToHost, s), "hipMemcpyAsync(ir status)")))
    return rc;
  if ((rc = record_hip(hipMemcpyAsync(dx, x, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, s),
                       "hipMemcpyAsync(x)")))
    return rc;
  if (dr && (rc = record_hip(hipMemcpyAsync(dr, r, (size_t)M * sizeof(double), hipMemcpyDeviceToDevice, s),
                             "hipMemcpyAsync(r)")))
    return rc;
  if ((rc = record_hip(hipStreamSynchronize(s), "hipStreamSynchronize(ir)"))) return rc;
  if (info) {
    info->iterations = it;
    info->converged = converged ? 1 : 0;
    info->eta = eta;
  }
  if (st[0] || st[1]) return st[0] ? st[0] : st[1];
  return 0;
}

}  // extern "C"
