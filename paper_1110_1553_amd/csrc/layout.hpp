// Workspace layout of a factorization, shared by the single-problem and
// batched entry points.
#pragma once

#include <cstddef>
#include <cstdint>

#include "../../include/hqr.h"

namespace hqr {

constexpr int64_t kDefaultSpinLimit = 20000000;  // polls of one counter (tens of seconds)
constexpr int kCtrlWords = 64;                    // cursor, status, spare

// Dependency counters per tile: one per 64-column sub-chunk (an update task
// covers two of them, a panel task publishes them one block at a time).
inline int chunk_cols(int nb) { (void)nb; return 64; }
inline int chunks_for(int nb) { return nb / chunk_cols(nb); }

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  int32_t mt, nt, nrt, chunks, last_a;  // nrt: tile columns of right-hand sides (hqr_lstsq)
  size_t ctrl, tg, tk, tiles, cnt, total;
};

// Workspace: control words, the T factors of the panel kernels (one nb x 16
// block column per tile and kind), the tile-contiguous copy of the matrix
// the factorization works on, followed (hqr_lstsq) by nrhs right-hand-side
// columns as further tile columns, and last the dependency counters (their
// number grows with the right-hand-side columns).  The T factors and the
// matrix tiles sit at offsets that depend on (M, N, params, esize) only, so
// a least-squares workspace holds its factorization exactly where
// hqr_apply_qt / hqr_apply_q / hqr_solve look for it.
// esize: bytes per element of the tiles and T factors (8: FP64, 4: FP32).
inline Layout layout_for(int64_t M, int64_t N, const hqr_params& p, int64_t nrhs = 0, size_t esize = sizeof(double)) {
  Layout L{};
  L.mt = (int32_t)((M + p.nb - 1) / p.nb);
  L.nt = (int32_t)((N + p.nb - 1) / p.nb);
  L.nrt = (int32_t)((nrhs + p.nb - 1) / p.nb);
  L.chunks = chunks_for(p.nb);
  const int cw = chunk_cols(p.nb);
  L.last_a = (int32_t)((N - (int64_t)(L.nt - 1) * p.nb + cw - 1) / cw);
  const size_t tiles = (size_t)L.mt * L.nt, all = (size_t)L.mt * (L.nt + L.nrt);
  size_t off = 0;
  L.ctrl = off; off = align256(off + kCtrlWords * sizeof(int32_t));
  L.tg = off; off = align256(off + tiles * (size_t)p.nb * 16 * esize);
  L.tk = off; off = align256(off + tiles * (size_t)p.nb * 16 * esize);
  L.tiles = off; off = align256(off + all * (size_t)p.nb * p.nb * esize);
  L.cnt = off; off = align256(off + all * L.chunks * sizeof(int32_t));
  L.total = off;
  return L;
}

// Signature of a factorization, written into control words kSigWord.. of its
// workspace when it is launched (and when a batch exports it): the apply
// entry points compare it with the one their arguments imply, so that a
// workspace holding another factorization (or none) is refused instead of
// read as T factors.
constexpr int kSigWord = 8;
constexpr int kSigWords = 8;
constexpr int32_t kSigMagic = 0x46525148;  // "HQRF"
struct FactorSig {
  int32_t w[kSigWords];
};
inline FactorSig factor_sig(const Layout& L, const hqr_params& p, size_t esize) {
  // FNV-1a over the tree parameters
  uint32_t h = 2166136261u;
  const int32_t f[6] = {p.p, p.a, p.low, p.high, p.coupling, p.domino};
  for (int32_t v : f)
    for (int b = 0; b < 4; ++b) {
      h ^= (uint32_t)(v >> (8 * b)) & 0xffu;
      h *= 16777619u;
    }
  FactorSig s{};
  s.w[0] = kSigMagic;
  s.w[1] = L.mt;
  s.w[2] = L.nt;
  s.w[3] = p.nb;
  s.w[4] = (int32_t)esize;
  s.w[5] = (int32_t)h;
  s.w[6] = L.last_a;
  s.w[7] = 0;
  return s;
}

// Workspace of hqr_apply_qt/_q/hqr_lstsq: control words, one dependency
// counter per block of B, and B in blocks of nb x 64.
struct ApplyLayout {
  int32_t mt, nbc;
  size_t ctrl, cnt, blocks, total;
};

inline ApplyLayout apply_layout_for(int64_t M, int64_t nrhs, const hqr_params& p, size_t esize = sizeof(double)) {
  ApplyLayout L{};
  L.mt = (int32_t)((M + p.nb - 1) / p.nb);
  L.nbc = (int32_t)((nrhs + 63) / 64);
  size_t off = 0;
  L.ctrl = off; off = align256(off + kCtrlWords * sizeof(int32_t));
  L.cnt = off; off = align256(off + (size_t)L.mt * L.nbc * sizeof(int32_t));
  L.blocks = off; off = align256(off + (size_t)L.mt * L.nbc * p.nb * 64 * esize);
  L.total = off;
  return L;
}

// Library-internal launch sequences (api.cpp).  run_factor: copies A (and
// nrhs right-hand sides) into the workspace tiles, runs the factorization
// (f32: FP32 tiles and kernels; a_f32: A holds float), copies A back when
// copy_a_out.  run_apply: B <- Q^T B (trans) or Q B with the factorization
// in dwork (f32: FP32 factors and B blocks; B itself stays double).
// `tasks` / `ntasks`: a task plan already in device memory to run instead of
// the library's cached one (then no tracing or timeline buffers either, so
// that the call allocates nothing); null: the cached plan.
int run_factor(void* dA, int64_t M, int64_t N, int64_t lda, const hqr_params& p, const hqr_exec& ex, void* dwork,
               double* dB, int64_t ldb, int32_t nrhs, void* stream, bool copy_a_out, bool f32, bool a_f32,
               const void* tasks = nullptr, int64_t ntasks = 0);
int run_apply(int trans, int64_t M, int64_t N, const hqr_params& p, const hqr_exec* exec, const void* dwork,
              size_t work_bytes, double* dB, int64_t ldb, int32_t nrhs, void* bwork, size_t bwork_bytes,
              void* stream, bool copy_out, bool f32);

}  // namespace hqr
