// Tile kernels of the tiled Householder QR and the persistent scheduler that
// runs them, for gfx950 (CDNA4).
//
// The six kernels of Algorithm 2 (GEQRT, UNMQR, TSQRT, TSMQR, TTQRT, TTMQR)
// work on b x b tiles in double precision with an inner blocking of 16:
// a panel of 16 columns is factored column by column in LDS (Householder
// reflectors, norms reduced across 16-lane groups), its compact-WY factor T
// (16 x 16, upper triangular) is formed, and the block reflector
// I - V T V^T is applied to the rest of the tile(s) with FP64 MFMA
// (v_mfma_f64_16x16x4f64).  The update kernels apply the 16-column panels of
// a finished factorization one after another with the V panels staged
// through LDS.
//
// Work split inside a workgroup (512 threads, 8 waves, one workgroup per CU
// so two waves share each SIMD): every wave owns a strip of 16 matrix
// columns and keeps the strip (b x 16 doubles) in registers as b/16 MFMA
// accumulators, so the reduction V^T C over the rows and the update
// C -= V W stay inside the wave; the waves only share the V panel and T in
// LDS.  An update task covers 128 columns (8 strips).  The column loop of
// the panel kernels runs on waves 0-3 (16 columns x 16 lanes).
//
// Register layout of an FP64 accumulator block (16 rows x 16 columns): lane
// l, element r holds MFMA row (l / 16) + 4 r, column l % 16.  Matrix rows
// are assigned to MFMA rows so that element r of lane l is matrix row
// 2 g + (r & 1) + 8 (r >> 1), g = l / 16: the four lane groups of a column
// cover its 16 rows as two contiguous 64-byte halves, each lane moving its
// rows with two 16-byte accesses (arow, roff).  The same permutation is
// applied to the reflector index of W = V^T C.  Update tasks stage their V
// panels two at a time (one barrier per pair).
#include <hip/hip_runtime.h>

#include <cstdio>

#include "task.hpp"

namespace hqr {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

// Element type E of a factorization: double (FP64 MFMA) or float (FP32
// MFMA).  V4<E> is one MFMA accumulator block per lane, V2<E> a pair.
template <typename E> struct VecOf;
template <> struct VecOf<double> { typedef d4 v4; typedef d2 v2; };
template <> struct VecOf<float> { typedef f4 v4; typedef f2 v2; };
template <typename E> using V4 = typename VecOf<E>::v4;
template <typename E> using V2 = typename VecOf<E>::v2;

constexpr int IB = 16;      // inner blocking (columns per panel)
constexpr int LDV = IB + 1; // LDS row stride of a staged panel (odd: no bank conflicts)
constexpr int NT = 512;     // threads per workgroup (8 waves, 2 per SIMD)

enum Kind { K_UNM = 0, K_TS = 1, K_TT = 2 };

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// BF16 operands with FP32 accumulation (precision HQR_PREC_BF16): each
// operand is the float rounded to the nearest bfloat16 (ties to even); the
// product of two bfloat16 values is exact in FP32, where the matrix core
// accumulates.  One v_mfma_f32_16x16x16_bf16 takes four consecutive values
// of the reduction index per lane (lane l: index 4 (l / 16) + j, j < 4), the
// same four a lane feeds into four 16x16x4 FP32 products, so it replaces a
// group of four of them with the operands packed.
typedef short s4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ short bf16_bits(float x) {
  const uint32_t u = __builtin_bit_cast(uint32_t, x);
  return (short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ s4 bf16x4(float a, float b, float c, float d) {
  s4 r;
  r.x = bf16_bits(a);
  r.y = bf16_bits(b);
  r.z = bf16_bits(c);
  r.w = bf16_bits(d);
  return r;
}
__device__ __forceinline__ s4 bf16x4(const f4& v) { return bf16x4(v.x, v.y, v.z, v.w); }
__device__ __forceinline__ f4 mfma_bf(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Reciprocal square root and reciprocal from the hardware estimates
// (v_rsq, v_rcp) refined by Newton steps to the working precision.  The
// arguments are positive normal numbers (a squared column norm and the sum
// |alpha| + norm of a Householder step), so no range scaling is needed.
//   rsq: g ~ sqrt(q) and h ~ 1 / (2 sqrt(q)) refined together (Goldschmidt),
//        then one correction of g from its residual q - g^2.
//   rcp: r <- r + r (1 - x r).
struct SqrtPair {
  double s, hs;  // sqrt(q) and 1 / (2 sqrt(q))
};
__device__ __forceinline__ SqrtPair esqrt2(double q) {
  const double y = __builtin_amdgcn_rsq(q);
  double g = q * y, h = 0.5 * y;
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, q);
  g = fma(d, h, g);
  return {g, h};
}
__device__ __forceinline__ double ercp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
struct SqrtPairF {
  float s, hs;
};
__device__ __forceinline__ SqrtPairF esqrt2(float q) {
  const float y = __builtin_amdgcn_rsqf(q);
  float g = q * y, h = 0.5f * y;
  const float r = fmaf(-g, h, 0.5f);
  g = fmaf(g, r, g);
  h = fmaf(h, r, h);
  const float d = fmaf(-g, g, q);
  g = fmaf(d, h, g);
  return {g, h};
}
__device__ __forceinline__ float ercp(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  const float e = fmaf(-x, r, 1.0f);
  return fmaf(r, e, r);
}

// Global-memory accessors for tile data inside the persistent launch.
//
// Tiles written by one workgroup are read by workgroups on other XCDs,
// whose L2 caches are not coherent with each other.  Agent-scope
// acquire/release fences would write back and invalidate a whole L2 at every
// task boundary; instead every tile access is a relaxed agent-scope access
// (coherent at device level on its own), and a task publishes its writes by
// waiting for its stores to complete before it bumps a dependency counter.
// The pointers are cast to the global address space: they reach the tile
// kernels through the task records, where the compiler would otherwise emit
// flat instructions (which also count against the LDS counter).
#ifndef HQR_GLOBAL_AS
#define HQR_GLOBAL_AS __attribute__((address_space(1)))
#endif
typedef HQR_GLOBAL_AS double gdouble;
typedef HQR_GLOBAL_AS float gfloat;

__device__ __forceinline__ double gload(const double* p) {
  return __hip_atomic_load((gdouble*)const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gstore(double* p, double v) {
  __hip_atomic_store((gdouble*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float gload(const float* p) {
  return __hip_atomic_load((gfloat*)const_cast<float*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gstore(float* p, float v) {
  __hip_atomic_store((gfloat*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ d2 gload2(const double* p) {
  d2 r;
  r.x = gload(p);
  r.y = gload(p + 1);
  return r;
}
__device__ __forceinline__ void gstore2(double* p, d2 v) {
  gstore(p, v.x);
  gstore(p + 1, v.y);
}

// Waits until this thread's global stores have completed.
__device__ __forceinline__ void stores_done() { __builtin_amdgcn_s_waitcnt(0); }

// 16-byte device-coherent accesses through a buffer resource: `base` is
// wave-uniform, `off` the element offset of this lane (< 2^28).
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
constexpr int kCoherent = 16;  // cache policy bit: coherent at device scope
// FP64 tile loads and stores: device-coherent and non-temporal (a hint;
// with it the FP64 factorizations took 0.3-1% less time, the FP32 one 1.7%
// more, so float accesses keep the plain coherent policy).
constexpr int kTileAccess = kCoherent | 2;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base) {
  // the base is wave-uniform by construction; say so, so that it lives in
  // scalar registers
  const uint64_t u = (uint64_t)base;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  void* b = (void*)(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(b, 0, 0x7fffffff, 0x00020000);
}
typedef unsigned int u2 __attribute__((ext_vector_type(2)));

// Two consecutive elements at element offset `off` (16 bytes of double, 8
// of float) and four consecutive elements (two or one 16-byte accesses).
template <typename E>
__device__ __forceinline__ V2<E> bload2(__amdgpu_buffer_rsrc_t r, int off);
template <>
__device__ __forceinline__ d2 bload2<double>(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, off * 8, 0, kTileAccess));
}
template <>
__device__ __forceinline__ f2 bload2<float>(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(r, off * 4, 0, kCoherent));
}
__device__ __forceinline__ void bstore2(__amdgpu_buffer_rsrc_t r, int off, d2 v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), r, off * 8, 0, kTileAccess);
}
// One element at byte offset voff + soff (soff a wave-uniform constant),
// plain (non-coherent) load: for kernels that read what an earlier launch
// wrote.
template <typename E>
__device__ __forceinline__ E bload1(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ double bload1<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ float bload1<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ f4 ld4(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, off * 4, 0, kCoherent));
}
__device__ __forceinline__ void st4(__amdgpu_buffer_rsrc_t r, int off, f4 v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), r, off * 4, 0, kCoherent);
}

// One DPP step on a double: each lane receives the value of the lane picked
// by `ctrl` inside its row of 16 lanes.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, true);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over the 16 lanes of a DPP row, returned in every lane of the row.
// Each step adds two partial sums in an order that does not depend on the
// lane (addition is commutative), so all 16 lanes hold bitwise the same sum.
template <typename E>
__device__ __forceinline__ E sum16(E v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x124>(v);  // row_ror:4
  v += dpp<0x128>(v);  // row_ror:8
  return v;
}

// Workgroup barrier that orders LDS accesses only: global stores still in
// flight are not waited for (the data they carry is not read by another
// wave before a full barrier).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename E, int NB>
struct Smem {
  // staged V panels (row-major, stride LDV) and T blocks: the update tasks
  // stage two panels at a time into slots {0, 1} and {2, 3} alternately;
  // the panel tasks use slots 0 and 1 only
  E V[4][NB * LDV];
  E T[4][IB * LDV];
  E R[IB * LDV];     // diagonal block of the killer's R (TS/TT panel kernels)
  E tau[IB];
  int task;  // index of the task taken by the workgroup (-1: launch aborted)
  int next;  // the following task index, taken ahead by finish_task (-2: none)
  int ok;    // 1 if the task's dependencies were met, 0 if the launch was aborted
  // partial W = V^T C of each wave (row-split updates of the panel tasks),
  // kept in V slots 2 and 3, which only the update tasks use
  static_assert(2 * NB * LDV * sizeof(E) >= 8 * 64 * sizeof(V4<E>), "xw does not fit in V slots 2-3");
  __device__ V4<E>* xw() { return reinterpret_cast<V4<E>*>(V[2]); }
};

// The scheduler's shared state and the tile kernels' staging buffers live in
// the launch's dynamic LDS.
extern __shared__ __attribute__((aligned(16))) double hqr_lds[];

template <typename E, int NB>
__device__ __forceinline__ Smem<E, NB>& smem() {
  return *reinterpret_cast<Smem<E, NB>*>(hqr_lds);
}

// Lane coordinates.
struct Lane {
  int wave, g, q, pq;
  __device__ Lane() {
    const int t = threadIdx.x;
    wave = __builtin_amdgcn_readfirstlane(t >> 6);
    g = (t >> 4) & 3;
    q = t & 15;
    pq = 2 * (q & 3) + ((q >> 2) & 1) + 8 * (q >> 3);
  }
};

// Rows of a 16 x 16 block held in an MFMA accumulator.  Element r of lane
// (g, q) (g = lane / 16, q = lane % 16) holds column q and the matrix row
//     FP64: 2g + (r & 1) + 8 (r >> 1)   (rows 2g, 2g+1, 2g+8, 2g+9)
//     FP32: 4g + r
// FP32 accumulators hold MFMA row 4g + r, so its map is the identity.  The
// FP64 accumulator holds MFMA row g + 4r (measured on gfx950); matrix row x
// then sits at MFMA row pi^-1(x) with pi(g + 4r) = 2g + (r & 1) + 8 (r >> 1).
// Either way the four lanes of a column cover its 16 rows as two contiguous
// 64-byte halves (FP64: two 16-byte accesses per lane) or one 64-byte run
// (FP32), so each access instruction writes whole segments: with four
// consecutive FP64 rows per lane the lanes of a column interleave at a
// 32-byte stride, which took twice as long to store.
template <typename E>
__device__ __forceinline__ int arow(const Lane& L) {  // row of element 0
  return sizeof(E) == 8 ? 2 * L.g : 4 * L.g;
}
template <typename E>
__device__ __forceinline__ int roff(int r) {  // row of element r minus that of element 0
  return sizeof(E) == 8 ? (r & 1) + 8 * (r >> 1) : r;
}

// MFMA row whose reduction index this lane supplies in the products with
// V^T and T^T: pi(q) for FP64, q itself for FP32.
template <typename E>
__device__ __forceinline__ int mrow(const Lane& L) {
  return sizeof(E) == 8 ? L.pq : L.q;
}

// One column's four rows of a 16-row block in accumulator order: `off` is
// the element offset of the block's row 0 in that column.
template <typename E>
__device__ __forceinline__ V4<E> ldblk(__amdgpu_buffer_rsrc_t r, int off, const Lane& L);
template <>
__device__ __forceinline__ d4 ldblk<double>(__amdgpu_buffer_rsrc_t r, int off, const Lane& L) {
  const d2 x = bload2<double>(r, off + 2 * L.g);
  const d2 y = bload2<double>(r, off + 2 * L.g + 8);
  d4 v;
  v.x = x.x; v.y = x.y; v.z = y.x; v.w = y.y;
  return v;
}
template <>
__device__ __forceinline__ f4 ldblk<float>(__amdgpu_buffer_rsrc_t r, int off, const Lane& L) {
  return ld4(r, off + 4 * L.g);
}
__device__ __forceinline__ void stblk(__amdgpu_buffer_rsrc_t r, int off, const Lane& L, d4 v) {
  d2 x, y;
  x.x = v.x; x.y = v.y; y.x = v.z; y.y = v.w;
  bstore2(r, off + 2 * L.g, x);
  bstore2(r, off + 2 * L.g + 8, y);
}
__device__ __forceinline__ void stblk(__amdgpu_buffer_rsrc_t r, int off, const Lane& L, f4 v) {
  st4(r, off + 4 * L.g, v);
}

// ---------------------------------------------------------------------------
// Block-reflector application of one panel to one 16-column strip held by a
// wave.  `acc` holds rows 0..NB-1 of the strip of the matrix the reflectors
// act on below the identity part (C2 for TS/TT, C itself for UNM).  `c1` is
// the strip of the killer tile (rows 16p..16p+15) for TS/TT, or null.
//
//   W  = V_p^T acc (+ C1_p)      reduction over the active rows
//   W  = T_p^T W                  (T_p W when applying Q instead of Q^T)
//   C1_p -= W,   acc -= V_p W
//
// Active rows: UNM rows >= 16p (V unit lower triangular), TS all rows
// (V dense), TT rows < 16p + 16 (V upper triangular).
template <typename E, int NB, int KIND>
__device__ __forceinline__ bool row_block_active(int rb, int p) {
  return (KIND == K_UNM) ? (rb >= p) : (KIND == K_TT ? rb <= p : true);
}

// The products are issued in groups (one row block in the reduction, two in
// the update) with the LDS operands of the next group loaded before the
// MFMAs of the current one; scheduling barriers keep the compiler from
// hoisting all operand loads at once, which would not fit next to the
// accumulators.  Consecutive MFMAs never write the same accumulator.
//
// A wave may hold SPW strips (columns 16 w + 64 s, s < SPW, of the chunk):
// every V operand read from LDS then feeds SPW products.
template <typename E, int NB, int KIND, bool TRANS, int SPW, bool BF = false>
__device__ __forceinline__ void apply_panel_n(V4<E> (&acc)[SPW][NB / 16], const E* __restrict__ Vs,
                                              const E* __restrict__ Ts, int p, E* c1, int64_t ldc,
                                              const Lane& L) {
  static_assert(!BF || sizeof(E) == 4, "BF16 products take float tiles");
  constexpr int NRB = NB / 16;
  V4<E> c1v[SPW];
  V4<E> w0[SPW], w1[SPW];
  const __amdgpu_buffer_rsrc_t rc1 = rsrc(c1);
#pragma unroll
  for (int s = 0; s < SPW; ++s) {
    c1v[s] = V4<E>{E(0), E(0), E(0), E(0)};
    if (KIND != K_UNM) c1v[s] = ldblk<E>(rc1, (L.q + 64 * s) * (int)ldc, L);
    w0[s] = V4<E>{E(0), E(0), E(0), E(0)};
    w1[s] = w0[s];
  }
  // ---- W = V^T acc: group rb = 4 products per strip, alternating two partial sums
  {
    const E* va = Vs + arow<E>(L) * LDV + mrow<E>(L);  // + (16 rb + roff(r)) * LDV
    E a[4], an[4];
    const int lo = (KIND == K_UNM) ? p : 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = E(0);
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
      if (rb == lo) {
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] = va[(16 * rb + roff<E>(r)) * LDV];
      }
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {
      if (row_block_active<E, NB, KIND>(rb, p)) {
        __builtin_amdgcn_sched_barrier(0);
        if (rb + 1 < NRB && row_block_active<E, NB, KIND>(rb + 1, p)) {
#pragma unroll
          for (int r = 0; r < 4; ++r) an[r] = va[(16 * (rb + 1) + roff<E>(r)) * LDV];
        }
        if constexpr (BF) {
          const s4 ab = bf16x4(a[0], a[1], a[2], a[3]);
#pragma unroll
          for (int s = 0; s < SPW; ++s) {
            if (rb & 1)
              w1[s] = mfma_bf(ab, bf16x4(acc[s][rb]), w1[s]);
            else
              w0[s] = mfma_bf(ab, bf16x4(acc[s][rb]), w0[s]);
          }
        } else {
#pragma unroll
          for (int s = 0; s < SPW; ++s) {
            w0[s] = mfma(a[0], acc[s][rb][0], w0[s]);
            w1[s] = mfma(a[1], acc[s][rb][1], w1[s]);
          }
#pragma unroll
          for (int s = 0; s < SPW; ++s) {
            w0[s] = mfma(a[2], acc[s][rb][2], w0[s]);
            w1[s] = mfma(a[3], acc[s][rb][3], w1[s]);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] = an[r];
      }
    }
  }
  V4<E> wn[SPW];
  {
    E t[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
      t[r] = TRANS ? Ts[(arow<E>(L) + roff<E>(r)) * LDV + mrow<E>(L)] : Ts[mrow<E>(L) * LDV + arow<E>(L) + roff<E>(r)];
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
      V4<E> w = w0[s] + w1[s];
      if (KIND != K_UNM) w += c1v[s];
      V4<E> w2t = {E(0), E(0), E(0), E(0)};
      if constexpr (BF) {
        w2t = mfma_bf(bf16x4(t[0], t[1], t[2], t[3]), bf16x4(w), w2t);
      } else {
        // two chains of two products: the T product sits between the two
        // halves of the panel's work, where the two waves of a SIMD arrive
        // together
        V4<E> x1 = {E(0), E(0), E(0), E(0)};
        w2t = mfma(t[0], w[0], w2t);
        x1 = mfma(t[1], w[1], x1);
        w2t = mfma(t[2], w[2], w2t);
        x1 = mfma(t[3], w[3], x1);
        w2t += x1;
      }
      if (KIND != K_UNM) stblk(rc1, (L.q + 64 * s) * (int)ldc, L, c1v[s] - w2t);
      wn[s] = -w2t;
    }
  }
  // ---- acc -= V W: groups of two row blocks, products interleaved
  {
    const E* vc = Vs + mrow<E>(L) * LDV + arow<E>(L);  // + 16 rb LDV + roff(r)
#pragma unroll
    for (int rb = 0; rb < NRB; rb += 2) {
      const bool act0 = row_block_active<E, NB, KIND>(rb, p);
      const bool act1 = row_block_active<E, NB, KIND>(rb + 1, p);
      if (act0 || act1) {
        __builtin_amdgcn_sched_barrier(0);
        E b0[4], b1[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          b0[r] = act0 ? vc[16 * rb * LDV + roff<E>(r)] : E(0);
          b1[r] = act1 ? vc[16 * (rb + 1) * LDV + roff<E>(r)] : E(0);
        }
        if constexpr (BF) {
          const s4 bb0 = bf16x4(b0[0], b0[1], b0[2], b0[3]);
          const s4 bb1 = bf16x4(b1[0], b1[1], b1[2], b1[3]);
#pragma unroll
          for (int s = 0; s < SPW; ++s) {
            const s4 wb = bf16x4(wn[s]);
            if (act0) acc[s][rb] = mfma_bf(bb0, wb, acc[s][rb]);
            if (act1) acc[s][rb + 1] = mfma_bf(bb1, wb, acc[s][rb + 1]);
          }
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int s = 0; s < SPW; ++s) {
              if (act0) acc[s][rb] = mfma(b0[r], wn[s][r], acc[s][rb]);
              if (act1) acc[s][rb + 1] = mfma(b1[r], wn[s][r], acc[s][rb + 1]);
            }
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
}

// One strip per wave.
template <typename E, int NB, int KIND, bool TRANS = true, bool BF = false>
__device__ __forceinline__ void apply_panel(V4<E> (&acc)[NB / 16], const E* __restrict__ Vs,
                                            const E* __restrict__ Ts, int p, E* c1, int64_t ldc,
                                            const Lane& L) {
  apply_panel_n<E, NB, KIND, TRANS, 1, BF>(reinterpret_cast<V4<E> (&)[1][NB / 16]>(acc), Vs, Ts, p, c1, ldc, L);
}

template <typename E, int NB, int KIND>
__device__ __forceinline__ void load_strip(V4<E> (&acc)[NB / 16], const E* base, int64_t ld, int p,
                                           const Lane& L) {
#pragma unroll
  for (int rb = 0; rb < NB / 16; ++rb) {
    const bool active = (KIND == K_UNM) ? (rb >= p) : (KIND == K_TT ? rb <= p : true);
    if (active) acc[rb] = ldblk<E>(rsrc(base), 16 * rb + L.q * (int)ld, L);
  }
}

template <typename E, int NB, int KIND>
__device__ __forceinline__ void store_strip(const V4<E> (&acc)[NB / 16], E* base, int64_t ld, int p,
                                            const Lane& L) {
#pragma unroll
  for (int rb = 0; rb < NB / 16; ++rb) {
    const bool active = (KIND == K_UNM) ? (rb >= p) : (KIND == K_TT ? rb <= p : true);
    if (active) stblk(rsrc(base), 16 * rb + L.q * (int)ld, L, acc[rb]);
  }
}

// Staging of V panel p (rows 0..NB-1, columns 16p..16p+15 of tile `V`) into
// LDS with the structure of the kind: UNM unit diagonal and zeros above it
// in the diagonal block; TT zeros below the diagonal; rows that no product
// reads are skipped.
template <typename E, int NB>
struct PanelPrefetch {
  static constexpr int PER = NB * 8 / NT;  // double2 loads per thread
  V2<E> v[PER];
  E t;
};

template <typename E, int NB, int KIND>
__device__ __forceinline__ void prefetch_panel(PanelPrefetch<E, NB>& pf, const E* V, int64_t ld,
                                               const E* Tblk, int p) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int it = 0; it < PanelPrefetch<E, NB>::PER; ++it) {
    const int e = it * NT + tid;
    const int col = e / (NB / 2), row = 2 * (e % (NB / 2));
    const bool needed = (KIND == K_UNM) ? (row >= 16 * p) : (KIND == K_TT ? row < 16 * p + 16 : true);
    if (needed) pf.v[it] = bload2<E>(rsrc(V), row + (16 * p + col) * (int)ld);
  }
  if (tid < 256) pf.t = gload(Tblk + tid);
}

template <typename E, int NB, int KIND>
__device__ __forceinline__ void stage_panel(const PanelPrefetch<E, NB>& pf, E* Vs, E* Ts, int p) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int it = 0; it < PanelPrefetch<E, NB>::PER; ++it) {
    const int e = it * NT + tid;
    const int col = e / (NB / 2), row = 2 * (e % (NB / 2));
    const bool needed = (KIND == K_UNM) ? (row >= 16 * p) : (KIND == K_TT ? row < 16 * p + 16 : true);
    if (needed) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = row + h;
        E x = pf.v[it][h];
        const int a = r - 16 * p;  // row inside the diagonal block
        if (a >= 0 && a < 16) {
          if (KIND == K_UNM) x = (a == col) ? E(1) : (a < col ? E(0) : x);
          if (KIND == K_TT) x = (a > col) ? E(0) : x;
        }
        Vs[r * LDV + col] = x;
      }
    }
  }
  if (tid < 256) Ts[(tid & 15) * LDV + (tid >> 4)] = pf.t;
}

// ---------------------------------------------------------------------------
// Update task: one 64-column chunk of UNMQR / TSMQR / TTMQR.
//   V, T: the factored tile and its T (block column nb x 16).
//   C2: tile updated below the identity part (UNM: the tile itself).
//   C1: killer tile (TS/TT).
// TRANS applies Q^T (the panels in factorization order, T^T); otherwise Q
// (the panels in reverse order, T).  Only the first np panels are applied:
// the panels after them are identities (T = 0, the zero padding beyond the
// last matrix column of a ragged tile column).
template <typename E, int NB, int KIND, bool TRANS, int CW, bool BF = false>
__device__ __forceinline__ void run_update(Smem<E, NB>& sm, const E* V, const E* T, E* C1, E* C2,
                                           int64_t ld, int np = NB / IB) {
  const int NP = __builtin_amdgcn_readfirstlane(np);
  const Lane L;
  const bool on = 16 * L.wave < CW;  // waves holding a strip of the chunk (uniform per wave)
  V4<E> acc[NB / 16];
  const int64_t coloff = (int64_t)(16 * L.wave) * ld;
  // Panels are staged two at a time, with one barrier per pair: panel it + 2
  // is prefetched into registers before panel it is applied and written to
  // the other pair of slots right after (those slots were last read by the
  // pair before, which every wave finished before the last barrier).
  PanelPrefetch<E, NB> pf;
  auto pan = [&](int it) { return TRANS ? it : NP - 1 - it; };
  auto prefetch = [&](int it) { prefetch_panel<E, NB, KIND>(pf, V, ld, T + pan(it) * 256, pan(it)); };
  auto apply = [&](int it, int slot) {
    const int p = pan(it);
    if (on)
      apply_panel<E, NB, KIND, TRANS, BF>(acc, sm.V[slot], sm.T[slot], p, KIND == K_UNM ? nullptr : C1 + coloff + 16 * p,
                                          ld, L);
  };
  prefetch(0);
  stage_panel<E, NB, KIND>(pf, sm.V[0], sm.T[0], pan(0));
  if (NP > 1) {
    prefetch(1);
    stage_panel<E, NB, KIND>(pf, sm.V[1], sm.T[1], pan(1));
  }
  // the chunk is loaded last: the first panel's products take its row
  // blocks in order as they arrive
  if (on) load_strip<E, NB, K_TS>(acc, C2 + coloff, ld, 0, L);
  lds_barrier();
#pragma unroll 1
  for (int it = 0; it < NP; it += 2) {
    const int sl = it & 2, sn = sl ^ 2;  // slots of this pair and of the next
    if (it + 2 < NP) prefetch(it + 2);
    apply(it, sl);
    if (it + 2 < NP) stage_panel<E, NB, KIND>(pf, sm.V[sn], sm.T[sn], pan(it + 2));
    if (it + 1 < NP) {
      if (it + 3 < NP) prefetch(it + 3);
      apply(it + 1, sl + 1);
      if (it + 3 < NP) stage_panel<E, NB, KIND>(pf, sm.V[sn + 1], sm.T[sn + 1], pan(it + 3));
    }
    lds_barrier();
  }
  if (on) store_strip<E, NB, K_TS>(acc, C2 + coloff, ld, 0, L);
}

// ---------------------------------------------------------------------------
// Panel task: GEQRT (KIND = UNM: the tile factors itself), TSQRT (TS: the
// triangle R on top of the square tile A), TTQRT (TT: the triangle R on top
// of the triangle A).  `A` is the tile zeroed (or triangularised for GEQRT),
// `R` the killer tile (TS/TT).  T blocks go to `T`.
//
// Column j of panel p: head = the diagonal entry of the triangle on top
// (GEQRT: A(j,j); TS/TT: R(j,j)), tail = the entries of the column that the
// reflector zeroes (GEQRT: A(j+1:nb, j); TS: A(0:nb, j); TT: A(0:j+1, j)).
// With alpha = head and s = ||tail||: s = 0 gives tau = 0 (H = I);
// otherwise beta = -sign(alpha) sqrt(alpha^2 + s^2), tau = (beta - alpha)/beta,
// tail /= (alpha - beta), head = beta.
//
// The tile is processed in blocks of 64 columns (four 16-column panels),
// left-looking: a block first receives the task's earlier panels, then each
// of its panels is factored (panel_columns) and applied to the block's
// remaining strips (panel_block; panel_left_update_4w and panel_strips_4w
// for FP32).

// Reads lane `lane` (wave-uniform) of a double held in VGPRs.
__device__ __forceinline__ float readlane(float v, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}
__device__ __forceinline__ double readlane(double v, int lane) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Factors panel p (columns c0 = 16p .. c0+15).  The 16 columns stay in
// registers during the column loop: thread (cc, q) = (tid / 16, tid % 16)
// holds column c0 + cc at the rows base + q + 16 m (base = c0 for GEQRT,
// 0 otherwise), so the reductions over rows are 16-lane DPP sums inside one
// wavefront.  The only data crossing groups is the reflector being applied,
// published through LDS (double buffered), which costs one workgroup
// barrier per column.  Leaves V_p in sm.V[0] (with the structure of the
// kind), T_p in sm.T[0] and in `T`, and the factored columns in A (and R).
// XL: the panel's columns are taken from sm.V[0] (row-major, stride LDV,
// left there by panel_block) instead of from memory.
template <typename E, int NB, int KIND, bool XL, int NS>
__device__ __forceinline__ void panel_columns_ns(E* A, E* R, E* T, int p) {
  // NS row slots per thread are held (NB / 16 for TS; for GEQRT and TT the
  // slots that can hold rows of this panel, rounded up to a multiple of 4)
  constexpr int NM = NS;
  p = __builtin_amdgcn_readfirstlane(p);  // uniform: row-slot guards become scalar branches
  Smem<E, NB>& sm = smem<E, NB>();
  const int tid = threadIdx.x;
  // waves 0-3 hold the panel; waves 4-7 only take part in the barriers
  const bool ct = tid < 256;
  const int cc = ct ? tid >> 4 : 16;  // panel column of this thread (16: none)
  const int q = tid & 15;             // its rows are base + q + 16 m
  const int c0 = 16 * p;
  const int base = (KIND == K_UNM) ? c0 : 0;
  // row slots that can hold rows of the panel (uniform): GEQRT rows < NB,
  // TT rows <= c0 + 15.  The other slots hold zeros; the column loop runs
  // over all slots (branch-free), only loads and stores skip them.
  const int nm = (KIND == K_UNM) ? NB / 16 - p : (KIND == K_TT ? p + 1 : NB / 16);
  E* Vs = sm.V[0];
  E* Ts = sm.T[0];
  E* Zs = sm.R;     // Gram entries v_i^T v_j of the panel
  E* Vb = sm.V[1];  // published reflector, two buffers of NB
  E* col = A + (int64_t)(c0 + cc) * NB;
  E x[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    const int r = base + q + 16 * m;
    // TT: rows below the diagonal hold the tile's own GEQRT reflectors
    const bool act = ct && m < nm && (KIND != K_TT || r <= c0 + cc);
    x[m] = act ? (XL ? sm.V[0][r * LDV + cc] : gload(col + r)) : E(0);
  }
  E rv = E(0);  // TS/TT: R(c0 + q, c0 + cc) of the killer's diagonal block
  if (KIND != K_UNM && ct && q <= cc) rv = gload(R + (c0 + q) + (int64_t)(c0 + cc) * NB);
  if (ct) Zs[cc * LDV + q] = E(0);  // entries (i, j) with i >= j stay zero
  // T is formed column by column on lanes 0-15 of wave 4 (idle in the column
  // loop), one row of T per lane: column k = jj - 1 once z(0:k, k) and
  // tau_k are visible (after the barrier of iteration jj).
  //   T(k,k) = tau_k,  T(i,k) = -tau_k sum_{i <= l < k} T(i,l) z(l,k)
  const bool tl = tid >= 256 && tid < 272;
  const int ti = tid - 256;
  E trow[16];
#pragma unroll
  for (int l = 0; l < 16; ++l) trow[l] = E(0);
  // Branch-free for a run-time k: every product of the sum is formed, those
  // with l >= k are exact zeros (z(l,k) = 0 for l >= k, and trow[l] = 0
  // until column l of T is formed); all 16 LDS reads are issued together.
  auto t_column = [&](int k) {
    const E tk = sm.tau[k];
    E z[16];
#pragma unroll
    for (int l = 0; l < 16; ++l) z[l] = Zs[l * LDV + k];
    E a0 = E(0), a1 = E(0), a2 = E(0), a3 = E(0);
#pragma unroll
    for (int l = 0; l < 16; l += 4) {
      a0 += trow[l] * z[l];
      a1 += trow[l + 1] * z[l + 1];
      a2 += trow[l + 2] * z[l + 2];
      a3 += trow[l + 3] * z[l + 3];
    }
    const E acc = (a0 + a1) + (a2 + a3);
    const E val = (ti < k) ? -tk * acc : (ti == k ? tk : E(0));
#pragma unroll
    for (int l = 0; l < 16; ++l) trow[l] = (l == k) ? val : trow[l];
  };
  // kept as a loop: unrolled, the sixteen column steps of each panel kind
  // take tens of KB of code and the panel tasks miss in the instruction
  // cache that a compute unit pair shares
#pragma unroll 1
  for (int jj = 0; jj < 16; ++jj) {
    E* vb = Vb + (jj & 1) * NB;
    if (cc == jj) {
      // the group owning column jj: wave jj / 4, lanes 16 (jj % 4) .. + 15;
      // the head is in its lane q = jj (GEQRT: slot 0; TS/TT: rv)
      const E alpha = readlane(KIND == K_UNM ? x[0] : rv, (jj & 3) * 16 + jj);
      E s0 = E(0), s1 = E(0), s2 = E(0), s3 = E(0);
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        E t = x[m];
        if (KIND == K_UNM && m == 0 && q <= jj) t = E(0);  // rows <= j are not in the tail
        if ((m & 3) == 0) s0 += t * t;
        if ((m & 3) == 1) s1 += t * t;
        if ((m & 3) == 2) s2 += t * t;
        if ((m & 3) == 3) s3 += t * t;
      }
      const E ss = sum16((s0 + s1) + (s2 + s3));
      E tau = E(0), beta = alpha, scale = E(1);
      if (ss != E(0)) {
        // beta = -sign(alpha) n with n = sqrt(alpha^2 + ss); then
        // tau = (beta - alpha) / beta = 1 + |alpha| / n and
        // 1 / (alpha - beta) = sign(alpha) / (|alpha| + n)
        const auto sq = esqrt2(fma(alpha, alpha, ss));
        const E aa = alpha >= E(0) ? alpha : -alpha;
        beta = alpha >= E(0) ? -sq.s : sq.s;
        tau = fma(aa, sq.hs + sq.hs, E(1));
        const E ri = ercp(aa + sq.s);
        scale = alpha >= E(0) ? ri : -ri;
      }
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        if (KIND == K_UNM && m == 0) {
          if (q > jj) x[0] *= scale;
          if (q == jj) x[0] = beta;
          vb[q] = (q > jj) ? x[0] : (q == jj ? E(1) : E(0));
        } else {
          x[m] *= scale;
          vb[q + 16 * m] = x[m];
        }
      }
      if (KIND != K_UNM && q == jj) rv = beta;
      if (q == 0) sm.tau[jj] = tau;
    }
    lds_barrier();
    if (tl && jj > 0) t_column(jj - 1);
    if (ct && cc != jj) {
      // tau is read together with v (kept above the products), not after the
      // reduction where only the update needs it
      const E tau = sm.tau[jj];
      E v[NM];
#pragma unroll
      for (int m = 0; m < NM; ++m) v[m] = vb[q + 16 * m];
      __builtin_amdgcn_sched_barrier(0);
      E d0 = E(0), d1 = E(0), d2 = E(0), d3 = E(0);
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        if ((m & 3) == 0) d0 += v[m] * x[m];
        if ((m & 3) == 1) d1 += v[m] * x[m];
        if ((m & 3) == 2) d2 += v[m] * x[m];
        if ((m & 3) == 3) d3 += v[m] * x[m];
      }
      // TS/TT: the unit entry of v sits in row j of the triangle on top,
      // where lane q = jj of column c0 + cc holds R(j, c0 + cc)
      if (KIND != K_UNM && cc > jj && q == jj) d0 += rv;
      const E d = sum16((d0 + d1) + (d2 + d3));
      if (cc > jj) {
        if (tau != E(0)) {
          const E f = tau * d;
#pragma unroll
          for (int m = 0; m < NM; ++m) x[m] -= f * v[m];
          if (KIND != K_UNM && q == jj) rv -= f;
        }
      } else if (q == 0) {
        Zs[cc * LDV + jj] = d;  // v_cc^T v_jj, consumed when T is formed
      }
    }
  }
  lds_barrier();
  // ---- the last column of T, then T to LDS (for the strips) and to memory
  if (tl) {
    t_column(15);
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      Ts[ti * LDV + jj] = trow[jj];
      gstore(T + p * 256 + ti + 16 * jj, trow[jj]);
    }
  }
  // ---- the factored panel back to the tiles, and V_p into LDS
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    if (ct && m < nm) {
      const int r = base + q + 16 * m;
      const bool act = KIND != K_TT || r <= c0 + cc;
      if (act) {
        gstore(col + r, x[m]);
        E vv = x[m];
        if (KIND == K_UNM && m == 0 && q <= cc) vv = (q == cc) ? E(1) : E(0);  // unit diagonal, R above
        Vs[r * LDV + cc] = vv;
      } else {
        Vs[r * LDV + cc] = E(0);  // TT: zero below the diagonal of V
      }
    }
  }
  if (KIND != K_UNM && ct && q <= cc) gstore(R + (c0 + q) + (int64_t)(c0 + cc) * NB, rv);
  // V_p and T_p in LDS are what the strips of the block need next; the
  // columns just stored are read back (block update) only after a full barrier
  lds_barrier();
}

// The column loop's cost follows the rows a panel can hold: GEQRT panel p
// has rows 16p .. NB-1 (NB/16 - p slots), TTQRT panel p rows 0 .. 16p+15
// (p + 1 slots); TSQRT always all NB/16.  The slot count is rounded up to a
// multiple of 4 so that each kind has at most four instantiations.
template <typename E, int NB, int KIND, bool XL = false>
__device__ __forceinline__ void panel_columns(E* A, E* R, E* T, int p) {
  constexpr int NM = NB / 16;
  p = __builtin_amdgcn_readfirstlane(p);
  if constexpr (KIND == K_TS || NM <= 4) {
    panel_columns_ns<E, NB, KIND, XL, NM>(A, R, T, p);
  } else {
    const int nm = (KIND == K_UNM) ? NM - p : p + 1;
    const int g = (nm + 3) >> 2;  // uniform
    if (g == 1) {
      panel_columns_ns<E, NB, KIND, XL, 4>(A, R, T, p);
    } else if (g == 2) {
      panel_columns_ns<E, NB, KIND, XL, 8>(A, R, T, p);
    } else if constexpr (NM > 8) {
      if (g == 3)
        panel_columns_ns<E, NB, KIND, XL, 12>(A, R, T, p);
      else
        panel_columns_ns<E, NB, KIND, XL, NM>(A, R, T, p);
    }
  }
}

// Row-split application of panel p inside a panel task: the strip of 16
// columns at `strip` is shared by waves w and w + 4, wave half h = wave / 4
// holding row blocks h NB/32 .. (h + 1) NB/32 - 1 of it in `acc`.  Each wave
// reduces its rows' part of W = V_p^T C, the two parts are exchanged through
// LDS and added in a fixed order (lower half + upper half, so both waves
// hold bitwise the same W), then each wave updates its own rows; the wave of
// the upper half (h = 0) also updates C1_p (TS/TT).  Every thread of the
// workgroup calls this (it contains a barrier); `on` says whether the wave
// holds a strip.
template <typename E, int NB, int KIND>
__device__ __forceinline__ void apply_panel_half(V4<E> (&acc)[NB / 32], const E* __restrict__ Vs,
                                                 const E* __restrict__ Ts, int p, E* c1, int64_t ldc, const Lane& L,
                                                 int h, bool on, V4<E>* xw) {
  constexpr int HRB = NB / 32;
  const int lane = threadIdx.x & 63;
  V4<E> w0 = {E(0), E(0), E(0), E(0)}, w1 = w0, c1v = w0;
  if (on) {
    if (KIND != K_UNM) c1v = ldblk<E>(rsrc(c1), L.q * (int)ldc, L);
    const E* va = Vs + arow<E>(L) * LDV + mrow<E>(L);
#pragma unroll
    for (int i = 0; i < HRB; ++i) {
      const int rb = h * HRB + i;
      if (row_block_active<E, NB, KIND>(rb, p)) {
        E a[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] = va[(16 * rb + roff<E>(r)) * LDV];
        w0 = mfma(a[0], acc[i][0], w0);
        w1 = mfma(a[1], acc[i][1], w1);
        w0 = mfma(a[2], acc[i][2], w0);
        w1 = mfma(a[3], acc[i][3], w1);
      }
    }
    xw[L.wave * 64 + lane] = w0 + w1;
  }
  lds_barrier();
  if (on) {
    const V4<E> lo = xw[(L.wave & 3) * 64 + lane], hi = xw[((L.wave & 3) + 4) * 64 + lane];
    V4<E> w = lo + hi;
    if (KIND != K_UNM) w += c1v;
    E t[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) t[r] = Ts[(arow<E>(L) + roff<E>(r)) * LDV + mrow<E>(L)];
    V4<E> w2t = {E(0), E(0), E(0), E(0)};
#pragma unroll
    for (int r = 0; r < 4; ++r) w2t = mfma(t[r], w[r], w2t);
    if (KIND != K_UNM && h == 0) stblk(rsrc(c1), L.q * (int)ldc, L, c1v - w2t);
    const V4<E> wn = -w2t;
    const E* vc = Vs + mrow<E>(L) * LDV + arow<E>(L);
#pragma unroll
    for (int i = 0; i < HRB; ++i) {
      const int rb = h * HRB + i;
      if (row_block_active<E, NB, KIND>(rb, p)) {
        E b0[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) b0[r] = vc[16 * rb * LDV + roff<E>(r)];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i] = mfma(b0[r], wn[r], acc[i]);
      }
    }
  }
}

// Block b of a panel task (columns 64b .. 64b+63) with its four strips
// kept in registers from start to end: strip 4b + w lives in waves w and
// w + 4 (row halves).  The strips are loaded once, receive this task's
// earlier panels (left-looking), and then for each panel p of the block the
// strip of p is handed to the column loop through LDS (sm.V[0]) and the
// panel is applied to the block's later strips in registers; the factored
// columns reach memory through the column loop (GEQRT: the rows of a strip
// above its diagonal block, which the column loop does not cover, are
// stored at the hand-over).  No strip goes through memory between the
// panels of a block.
template <typename E, int NB, int KIND>
__device__ __forceinline__ void panel_block(E* A, E* R, E* T, int b) {
  constexpr int HRB = NB / 32;
  b = __builtin_amdgcn_readfirstlane(b);
  Smem<E, NB>& sm = smem<E, NB>();
  const Lane L;
  const int w = L.wave & 3, h = L.wave >> 2;
  const int s = 4 * b + w;   // this wave's strip
  const int np = 4 * b;      // earlier panels of this task
  // row blocks held: TT rows up to the block's last diagonal block (below
  // them a TT victim holds its own GEQRT reflectors), otherwise all
  const int hi = (KIND == K_TT) ? 4 * b + 3 : NB / 16 - 1;
  E* strip = A + (int64_t)(16 * s) * NB;
  E* c1s = KIND == K_UNM ? nullptr : R + (int64_t)(16 * s) * NB;  // killer's strip s
  V4<E> acc[HRB];
#pragma unroll
  for (int i = 0; i < HRB; ++i)
    if (h * HRB + i <= hi) acc[i] = ldblk<E>(rsrc(strip), 16 * (h * HRB + i) + L.q * NB, L);
  if (np > 0) {
    PanelPrefetch<E, NB> pf;
    prefetch_panel<E, NB, KIND>(pf, A, NB, T, 0);
    for (int p = 0; p < np; ++p) {
      E* Vs = sm.V[p & 1];
      E* Ts = sm.T[p & 1];
      stage_panel<E, NB, KIND>(pf, Vs, Ts, p);
      lds_barrier();
      if (p + 1 < np) prefetch_panel<E, NB, KIND>(pf, A, NB, T + (p + 1) * 256, p + 1);
      apply_panel_half<E, NB, KIND>(acc, Vs, Ts, p, KIND == K_UNM ? nullptr : c1s + 16 * p, NB, L, h, true, sm.xw());
    }
  }
  for (int p = 4 * b; p < 4 * b + 4; ++p) {
    lds_barrier();  // every wave is done with the V panel and T in sm.V[0], sm.T[0]
    if (s == p) {
      E* H = sm.V[0];
#pragma unroll
      for (int i = 0; i < HRB; ++i) {
        const int rb = h * HRB + i;
        if (rb <= hi) {
#pragma unroll
          for (int r = 0; r < 4; ++r) H[(16 * rb + arow<E>(L) + roff<E>(r)) * LDV + L.q] = acc[i][r];
          // GEQRT: rows above the diagonal block are final R entries
          if (KIND == K_UNM && rb < p) stblk(rsrc(strip), 16 * rb + L.q * NB, L, acc[i]);
        }
      }
    }
    lds_barrier();
    panel_columns<E, NB, KIND, true>(A, R, T, p);
    if (p < 4 * b + 3)
      apply_panel_half<E, NB, KIND>(acc, sm.V[0], sm.T[0], p, KIND == K_UNM ? nullptr : c1s + 16 * p, NB, L, h, s > p,
                                    sm.xw());
  }
}

// FP32 panel tasks take the block in the form below instead (strips
// through memory between panels, one wave per strip): the register-resident
// form above makes the float register allocation spill.
//
// Applies panel p (V_p, T_p staged in sm.V[0], sm.T[0]) to the strips
// p+1 .. s_last of the tile(s) (at most 3): wave w takes strip p + 1 + w.
template <typename E, int NB, int KIND, bool BF = false>
__device__ __forceinline__ void panel_strips_4w(E* A, E* R, int p, int s_last) {
  p = __builtin_amdgcn_readfirstlane(p);
  s_last = __builtin_amdgcn_readfirstlane(s_last);
  Smem<E, NB>& sm = smem<E, NB>();
  const Lane L;
  const int s = p + 1 + L.wave;
  if (s <= s_last) {
    V4<E> acc[NB / 16];
    E* strip = A + (int64_t)(16 * s) * NB;
    load_strip<E, NB, KIND>(acc, strip, NB, p, L);
    apply_panel<E, NB, KIND, true, BF>(acc, sm.V[0], sm.T[0], p, KIND == K_UNM ? nullptr : R + (int64_t)(16 * s) * NB + 16 * p,
                          NB, L);
    store_strip<E, NB, KIND>(acc, strip, NB, p, L);
  }
  stores_done();
  __syncthreads();  // the next panel's column loop reads these strips from memory
}

// Left-looking update of block b (strips 4b .. 4b+3, one per wave 0-3):
// the panels 0 .. 4b-1 of this task are applied to it, V from the tile(s)
// already factored and T from `T`, the strips held in registers across the
// panels.  Done right before block b is factored, so that block b depends on
// nothing that a predecessor task writes later than its own block b.
template <typename E, int NB, int KIND, bool BF = false>
__device__ __forceinline__ void panel_left_update_4w(E* A, E* R, const E* T, int b) {
  constexpr int NRB = NB / 16;
  b = __builtin_amdgcn_readfirstlane(b);
  Smem<E, NB>& sm = smem<E, NB>();
  const Lane L;
  const int np = 4 * b;  // panels applied
  const bool on = L.wave < 4;
  const int s = 4 * b + L.wave;
  // row blocks the panels touch: UNM and TS all, TT rows < 16 np (below them,
  // a TT victim holds its own GEQRT reflectors)
  const int hi = (KIND == K_TT) ? np - 1 : NRB - 1;
  E* strip = A + (int64_t)(16 * s) * NB;
  V4<E> acc[NRB];
#pragma unroll
  for (int rb = 0; rb < NRB; ++rb)
    if (on && rb <= hi) acc[rb] = ldblk<E>(rsrc(strip), 16 * rb + L.q * NB, L);
  PanelPrefetch<E, NB> pf;
  prefetch_panel<E, NB, KIND>(pf, A, NB, T, 0);
  for (int p = 0; p < np; ++p) {
    E* Vs = sm.V[p & 1];
    E* Ts = sm.T[p & 1];
    stage_panel<E, NB, KIND>(pf, Vs, Ts, p);
    lds_barrier();
    if (p + 1 < np) prefetch_panel<E, NB, KIND>(pf, A, NB, T + (p + 1) * 256, p + 1);
    if (on)
      apply_panel<E, NB, KIND, true, BF>(acc, Vs, Ts, p, KIND == K_UNM ? nullptr : R + (int64_t)(16 * s) * NB + 16 * p, NB, L);
  }
#pragma unroll
  for (int rb = 0; rb < NRB; ++rb)
    if (on && rb <= hi) stblk(rsrc(strip), 16 * rb + L.q * NB, L, acc[rb]);
  stores_done();
  __syncthreads();  // the column loop of block b reads these strips from memory
}

// ---------------------------------------------------------------------------
// Scheduler steps.

// Waits until every lane's counter *c >= v (one counter per lane of the
// calling wave).  Returns false when the launch has been aborted: by this
// wait running past the spin limit (it then records the abort and what it
// was waiting for in ctrl[1..5]) or by another workgroup's abort.
// Every lane of the wave calls it; a lane with c == null or v == 0 has
// nothing to wait for.  The counters are polled in parallel instead of one
// after another.  Returns the same (uniform) result in every lane; on a
// time-out the lowest lane still waiting records its counter.
__device__ __forceinline__ bool wait_lanes(int32_t* c, uint32_t v, const LaunchArgs& a, int t) {
  bool done = (c == nullptr) || (v == 0);
  int64_t spins = 0;
  const int lane = threadIdx.x & 63;
  for (;;) {
    uint32_t seen = 0;
    if (!done) {
      seen = (uint32_t)__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      done = seen >= v;
    }
    const uint64_t pending = __ballot(!done);
    if (pending == 0) return true;
    ++spins;
    if (spins > a.spin_limit) {
      if (lane == __ffsll((unsigned long long)pending) - 1) {
        int32_t none = 0;
        if (__hip_atomic_compare_exchange_strong(&a.ctrl[1], &none, (int32_t)HQR_ERR_WATCHDOG, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          __hip_atomic_store(&a.ctrl[2], t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&a.ctrl[3], (int32_t)(c - a.cnt), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&a.ctrl[4], (int32_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&a.ctrl[5], (int32_t)seen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      return false;
    }
    if ((spins & 63) == 0) {
      const int st = __builtin_amdgcn_readfirstlane(
          __hip_atomic_load(&a.ctrl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      if (st != 0) return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

__device__ __forceinline__ void trace(const LaunchArgs& a, int t, int phase) {
  if (a.trace && blockIdx.x < kTraceSlots) {
    __hip_atomic_store(&a.trace[2 * blockIdx.x], t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&a.trace[2 * blockIdx.x + 1], phase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// Index of the XCD (accelerator complex die) running the wave.
__device__ __forceinline__ int xcc_id() {
  int x = 0;
  __asm__ __volatile__("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
  return x & 0xf;
}

// Timeline record of task t: [0] picked, [1] inputs ready, [2] done (100 MHz
// real-time clock), [3] workgroup | XCD << 16.
__device__ __forceinline__ void stamp(const LaunchArgs& a, int t, int slot) {
  if (a.timeline && t >= 0) {
    a.timeline[4 * (int64_t)t + slot] = __builtin_amdgcn_s_memrealtime();
    if (slot == 0) a.timeline[4 * (int64_t)t + 3] = (uint64_t)blockIdx.x | ((uint64_t)xcc_id() << 16);
  }
}

__device__ __forceinline__ int32_t* counter(const LaunchArgs& a, int r, int c, int chunk) {
  return a.cnt + ((int64_t)r * a.cnt_cols + c) * a.chunks + chunk;
}

// The steps of one scheduler iteration are separate, non-inlined functions
// on purpose: each one holds the lane-divergent part of its step (the work
// of thread 0) together with the workgroup barrier that ends it, so the loop
// in the kernel contains only uniform control flow.  When these steps were
// inlined, the compiler moved thread 0's tail of an iteration out of the
// loop behind a divergent exit, and the other lanes re-ran the same task.

// Takes the next task index (uniform), or -1 when every task has been
// handed out or the launch was aborted.
template <typename E, int NB>
__device__ __noinline__ int take_task(const LaunchArgs& a) {
  Smem<E, NB>& sm = smem<E, NB>();
  if (threadIdx.x == 0) {
    int t = sm.next;
    sm.next = -2;
    // an aborted launch hands out no more tasks: every workgroup leaves at
    // its next pick, so the kernel ends soon after the first time-out
    if (__hip_atomic_load(&a.ctrl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
      t = -1;
    else if (t == -2)
      t = __hip_atomic_fetch_add(&a.ctrl[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (t >= a.ntasks) t = -1;
    sm.task = t;
    trace(a, t, t < 0 ? TR_EXIT : TR_POPPED);
    stamp(a, t, 0);
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(sm.task);
}

// Dependency counters count 64-column sub-chunks of a tile.  A panel task
// works through its tile(s) block by block (64 columns each): it waits for
// block b's sub-chunk before touching block b and publishes it when the
// block is final, so a chain of panel tasks on one tile (a TS domain, a
// tree) advances one block behind its predecessor.  The last active
// sub-chunk is published only when the whole task is done, which is what
// the update tasks reading the factored tile wait for (task.pad & 0xff).
// An update task covers task.pad >> 8 sub-chunks starting at sub-chunk
// task.chunk.

// Thread 0 waits for the task's input versions (panel tasks: block 0);
// returns 1 (uniform) when they were reached, 0 when the launch was aborted.
template <typename E, int NB>
__device__ __noinline__ int wait_task(const LaunchArgs& a, int t, const DevTask& task) {
  Smem<E, NB>& sm = smem<E, NB>();
  if (threadIdx.x < 64) {
    // lane l waits for the l-th (counter, version) pair of the task
    const int l = threadIdx.x;
    const int op = task.op, i = task.row, piv = task.killer, k = task.k, j = task.j;
    int32_t* c = nullptr;
    uint32_t v = 0;
    if (a.B) {
      // apply launch: one counter per block of B
      if (op == UNMQR) {
        if (l == 0) c = counter(a, i, j, 0), v = task.v[1];
      } else {
        if (l == 0) c = counter(a, piv, j, 0), v = task.v[1];
        if (l == 1) c = counter(a, i, j, 0), v = task.v[2];
      }
    } else {
      const int c0 = task.chunk, cn = task.pad >> 8, cv = task.pad & 0xff;
      switch (op) {
        case GEQRT:
          if (l == 0) c = counter(a, i, k, 0), v = task.v[0];
          break;
        case TSQRT:
        case TTQRT:
          if (l == 0) c = counter(a, piv, k, 0), v = task.v[0];
          if (l == 1) c = counter(a, i, k, 0), v = task.v[1];
          break;
        case UNMQR:
          if (l == 0) c = counter(a, i, k, cv), v = task.v[0];
          if (l >= 1 && l <= cn) c = counter(a, i, j, c0 + l - 1), v = task.v[1];
          break;
        default:
          if (l == 0) c = counter(a, i, k, cv), v = task.v[0];
          if (l >= 1 && l <= cn) c = counter(a, piv, j, c0 + l - 1), v = task.v[1];
          if (l > cn && l <= 2 * cn) c = counter(a, i, j, c0 + l - cn - 1), v = task.v[2];
          break;
      }
    }
    const bool ok = wait_lanes(c, v, a, t);
    if (l == 0) {
      sm.ok = ok ? 1 : 0;
      trace(a, t, ok ? TR_READY : TR_ABORT);
      stamp(a, t, 1);
    }
  }
  __syncthreads();
  const int ok = __builtin_amdgcn_readfirstlane(sm.ok);
  // the producers' stores had completed when they bumped the counters, and
  // tile loads are device-coherent: no cache invalidation is needed
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  return ok;
}

// Panel tasks, inside the task: wait for block b (b >= 1) of the tile(s).
template <typename E, int NB>
__device__ __noinline__ int wait_block(const LaunchArgs& a, int t, const DevTask& task, int b) {
  Smem<E, NB>& sm = smem<E, NB>();
  __syncthreads();
  if (threadIdx.x < 64) {
    const int l = threadIdx.x;
    int32_t* c = nullptr;
    uint32_t v = 0;
    if (task.op == GEQRT) {
      if (l == 0) c = counter(a, task.row, task.k, b), v = task.v[0];
    } else {
      if (l == 0) c = counter(a, task.killer, task.k, b), v = task.v[0];
      if (l == 1) c = counter(a, task.row, task.k, b), v = task.v[1];
    }
    const bool ok = wait_lanes(c, v, a, t);
    if (l == 0) sm.ok = ok ? 1 : 0;
  }
  __syncthreads();
  const int ok = __builtin_amdgcn_readfirstlane(sm.ok);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  return ok;
}

// Panel tasks, inside the task: block b of the tile(s) is final.
template <typename E, int NB>
__device__ __noinline__ void release_block(const LaunchArgs& a, const DevTask& task, int b) {
  stores_done();
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(counter(a, task.row, task.k, b), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (task.op != GEQRT)
      __hip_atomic_fetch_add(counter(a, task.killer, task.k, b), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Publishes the task's tile writes and bumps the counters of the tiles it
// wrote (panel tasks: the last active block; the others went out with
// release_block).
template <typename E, int NB>
__device__ __noinline__ void finish_task(const LaunchArgs& a, int t, const DevTask& task) {
  // the next task index is taken while this task's stores drain
  int next = -2;
  if (threadIdx.x == 0) next = __hip_atomic_fetch_add(&a.ctrl[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  stores_done();
  __syncthreads();
  if (threadIdx.x == 0) {
    smem<E, NB>().next = next;
    trace(a, t, TR_DONE);
    stamp(a, t, 2);
    const int op = task.op, i = task.row, piv = task.killer, k = task.k, j = task.j;
    auto bump = [&](int32_t* c) { __hip_atomic_fetch_add(c, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); };
    if (a.B) {
      if (op != UNMQR) bump(counter(a, piv, j, 0));
      bump(counter(a, i, j, 0));
    } else {
      const int c0 = task.chunk, cn = task.pad >> 8;
      switch (op) {
        case GEQRT:
          bump(counter(a, i, k, task.chunk - 1));
          break;
        case TSQRT:
        case TTQRT:
          bump(counter(a, piv, k, task.chunk - 1));
          bump(counter(a, i, k, task.chunk - 1));
          break;
        case UNMQR:
          for (int c = c0; c < c0 + cn; ++c) bump(counter(a, i, j, c));
          break;
        default:
          for (int c = c0; c < c0 + cn; ++c) {
            bump(counter(a, piv, j, c));
            bump(counter(a, i, j, c));
          }
          break;
      }
    }
  }
}

// Tiles are stored contiguously (tile (r, c) at index c * mt + r, each one
// column-major with leading dimension nb), so a tile spans a few pages only.
template <typename E>
__device__ __forceinline__ E* tile_ptr(const LaunchArgs& a, int nb, int r, int c) {
  return (E*)a.A + ((int64_t)c * a.mt + r) * nb * nb;
}

template <typename E>
__device__ __forceinline__ E* t_block(void* T, const LaunchArgs& a, int nb, int r, int c) {
  return (E*)T + ((int64_t)r * a.nt + c) * nb * 16;
}

// One tile kernel per function (each gets its own register allocation).
// Panel tasks are on the critical path of the factorization: their waves
// run at raised priority.  The tile(s) are processed block by block (64
// columns) up to the last block holding matrix columns, left-looking: block
// b waits for the predecessor's block b,
// takes this task's earlier panels, is factored, and is published at once
// (except the last active block, published by finish_task).  Returns 0 when
// the launch was aborted while waiting.
template <typename E, int NB, int KIND, bool BF = false>
__device__ __noinline__ int panel_task(const LaunchArgs& a, int t, const DevTask& task) {
  E* T = t_block<E>((KIND == K_UNM) ? a.Tg : a.Tk, a, NB, task.row, task.k);
  E* A = tile_ptr<E>(a, NB, task.row, task.k);
  E* R = KIND == K_UNM ? nullptr : tile_ptr<E>(a, NB, task.killer, task.k);
  const int active = task.chunk;  // blocks holding matrix columns
  __builtin_amdgcn_s_setprio(2);
  for (int b = 0; b < NB / 64; ++b) {
    if (b >= active) {
      // blocks beyond the last matrix column (zero padding) are not factored:
      // their reflectors are the identity, T = 0 (what factoring the zero
      // columns would give), and the padding stays zero
      for (int e = threadIdx.x; e < (NB / 16 - 4 * b) * 256; e += NT) gstore(T + 4 * b * 256 + e, E(0));
      break;
    }
    if (b > 0 && !wait_block<E, NB>(a, t, task, b)) {
      __builtin_amdgcn_s_setprio(0);
      return 0;
    }
    if constexpr (sizeof(E) == 4) {
      if (b > 0) panel_left_update_4w<E, NB, KIND, BF>(A, R, T, b);
      for (int p = 4 * b; p < 4 * b + 4; ++p) {
        panel_columns<E, NB, KIND>(A, R, T, p);
        if (p < 4 * b + 3) panel_strips_4w<E, NB, KIND, BF>(A, R, p, 4 * b + 3);
      }
    } else {
      panel_block<E, NB, KIND>(A, R, T, b);
    }
    if (b + 1 < active) {
      release_block<E, NB>(a, task, b);
    } else {
      stores_done();
      __syncthreads();  // the next block reads the columns and T stored by this one
    }
  }
  __builtin_amdgcn_s_setprio(0);
  return 1;
}

// An update task covers one or two 64-column sub-chunks (one 16-column
// strip per wave; one sub-chunk at nb = 64 and at the ragged end of a tile).
template <typename E, int NB, int KIND, bool BF = false>
__device__ __noinline__ void update_task(const LaunchArgs& a, const DevTask& task) {
  void* T = (KIND == K_UNM) ? a.Tg : a.Tk;
  const int64_t colchunk = (int64_t)task.chunk * 64 * NB;
  const E* V = tile_ptr<E>(a, NB, task.row, task.k);
  const E* Tb = t_block<E>(T, a, NB, task.row, task.k);
  E* C1 = KIND == K_UNM ? nullptr : tile_ptr<E>(a, NB, task.killer, task.j) + colchunk;
  E* C2 = tile_ptr<E>(a, NB, task.row, task.j) + colchunk;
  // panels of the factored tile column that hold matrix columns: four per
  // 64-column block up to its last active block (task.pad & 0xff)
  const int np = 4 * ((task.pad & 0xff) + 1) < NB / IB ? 4 * ((task.pad & 0xff) + 1) : NB / IB;
  if (NB >= 128 && (task.pad >> 8) == 2)
    run_update<E, NB, KIND, true, 128, BF>(smem<E, NB>(), V, Tb, C1, C2, NB, np);
  else
    run_update<E, NB, KIND, true, 64, BF>(smem<E, NB>(), V, Tb, C1, C2, NB, np);
}

// Block of 64 columns of B (nb x 64, column-major) of tile row r.
template <typename E>
__device__ __forceinline__ E* b_block(const LaunchArgs& a, int nb, int r, int j) {
  return (E*)a.B + ((int64_t)j * a.mt + r) * nb * 64;
}

// The same transformation applied to a block of B (hqr_apply_qt/_q).
template <typename E, int NB, int KIND, bool TRANS>
__device__ __noinline__ void apply_task(const LaunchArgs& a, const DevTask& task) {
  void* T = (KIND == K_UNM) ? a.Tg : a.Tk;
  run_update<E, NB, KIND, TRANS, 64>(smem<E, NB>(), tile_ptr<E>(a, NB, task.row, task.k),
                                     t_block<E>(T, a, NB, task.row, task.k),
                                     KIND == K_UNM ? nullptr : b_block<E>(a, NB, task.killer, task.j),
                                     b_block<E>(a, NB, task.row, task.j), NB);
}

// Points the per-problem fields of `la` (tiles, T factors, counters, tile
// grid) at the problem of task t of a batched launch.
__device__ __forceinline__ void bind_problem(LaunchArgs& la, const LaunchArgs& a, int t) {
  const ProbDesc* d = a.probs + a.task_prob[t];
  char* w = (char*)a.ctrl;
  la.A = (double*)(w + d->tiles);
  la.Tg = (double*)(w + d->tg);
  la.Tk = (double*)(w + d->tk);
  la.cnt = (int32_t*)(w + d->cnt);
  la.mt = d->mt;
  la.nt = d->nt;
  la.cnt_cols = d->nt + d->nrt;
}

// Persistent scheduler.  Workgroups take task indices from a global cursor
// in dispatch order (a topological order of the task graph), wait until the
// dependency counters of the tiles the task touches reach the versions in
// the task record, run it, and bump the counters of the tiles it wrote.
// Every task a workgroup waits for was taken earlier by a running
// workgroup, so the wait always ends.  BATCH: the tasks of many independent
// problems share the cursor (each task names its problem).
template <typename E, int NB, bool BATCH, bool BF = false>
__global__ __launch_bounds__(NT, 1) void persistent_kernel(LaunchArgs args) {
  LaunchArgs la = args;
  if (threadIdx.x == 0) smem<E, NB>().next = -2;
  for (;;) {
    const int t = take_task<E, NB>(args);
    if (t < 0) break;
    const DevTask task = args.tasks[t];
    if (BATCH) bind_problem(la, args, t);
    const LaunchArgs& a = BATCH ? la : args;
    if (!wait_task<E, NB>(a, t, task)) break;
    int ok = 1;
    if (a.B) {
      if (a.trans) {
        switch (task.op) {
          case UNMQR: apply_task<E, NB, K_UNM, true>(a, task); break;
          case TSMQR: apply_task<E, NB, K_TS, true>(a, task); break;
          default: apply_task<E, NB, K_TT, true>(a, task); break;
        }
      } else {
        switch (task.op) {
          case UNMQR: apply_task<E, NB, K_UNM, false>(a, task); break;
          case TSMQR: apply_task<E, NB, K_TS, false>(a, task); break;
          default: apply_task<E, NB, K_TT, false>(a, task); break;
        }
      }
    } else {
      switch (task.op) {
        case GEQRT: ok = panel_task<E, NB, K_UNM, BF>(a, t, task); break;
        case TSQRT: ok = panel_task<E, NB, K_TS, BF>(a, t, task); break;
        case TTQRT: ok = panel_task<E, NB, K_TT, BF>(a, t, task); break;
        case UNMQR: update_task<E, NB, K_UNM, BF>(a, task); break;
        case TSMQR: update_task<E, NB, K_TS, BF>(a, task); break;
        default: update_task<E, NB, K_TT, BF>(a, task); break;
      }
    }
    if (!ok) break;  // aborted inside a panel task
    finish_task<E, NB>(a, t, task);
  }
}

// ---------------------------------------------------------------------------
// Small helpers.

__global__ void zero_i32_kernel(int32_t* p, int64_t n) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
    p[x] = 0;
}

__global__ void init_ctrl_kernel(int32_t* ctrl, FactorSig sig, int32_t* cnt, int64_t ncnt) {
  const int64_t x0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x0 < kCtrlWords) {
    const int w = (int)x0;
    ctrl[w] = (w >= kSigWord && w < kSigWord + kSigWords) ? sig.w[w - kSigWord] : 0;
  }
  for (int64_t x = x0; x < ncnt; x += (int64_t)gridDim.x * blockDim.x) cnt[x] = 0;
}

__global__ void check_sig_kernel(const int32_t* fctrl, FactorSig sig, int32_t* bctrl) {
  const int w = threadIdx.x;
  const bool bad = w < kSigWords && fctrl[kSigWord + w] != sig.w[w];
  if (__any(bad) && w == 0) bctrl[1] = HQR_ERR_FACTORS;
}

// Column-major M x N matrix (leading dimension lda) <-> blocks of nb rows
// x tw columns (block (i, j) at index j * mt + i, column-major inside with
// leading dimension nb; tw = nb for the tiles of A, 64 for the blocks of
// B).  `in` fills the blocks and zeroes the padding beyond M and N; `out`
// copies the M x N part back.  One thread per element of the padded matrix,
// rows fastest.
// The matrix holds S elements, the blocks E elements (a float copy of a
// double matrix rounds each element to nearest).
template <typename S, typename E>
__device__ __forceinline__ void tile_copy_elem(S* A, int64_t lda, E* At, int64_t M, int64_t N, int nb, int tw,
                                               int mt, int64_t x, int in) {
  const int64_t Mp = (int64_t)mt * nb;
  const int64_t r = x % Mp, c = x / Mp;
  const int64_t i = r / nb, j = c / tw;
  E* t = At + ((j * mt + i) * tw + (c - j * tw)) * nb + (r - i * nb);
  const bool inside = r < M && c < N;
  if (in)
    *t = inside ? (E)A[r + c * lda] : E(0);
  else if (inside)
    A[r + c * lda] = (S)*t;
}

template <typename S, typename E>
__global__ void tile_copy_kernel(S* A, int64_t lda, E* At, int64_t M, int64_t N, int nb, int tw, int mt, int nt,
                                 int in) {
  const int64_t total = (int64_t)mt * nb * (int64_t)nt * tw;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x)
    tile_copy_elem(A, lda, At, M, N, nb, tw, mt, x, in);
}

// Batched copy: workgroup row blockIdx.y serves problem blockIdx.y, first
// its matrix (nt tile columns), then its right-hand sides (nrt tile columns
// appended to the same tile array).
__global__ void copy_batched_kernel(const ProbDesc* descs, char* w, int nb, int in) {
  const ProbDesc* d = descs + blockIdx.y;
  double* At = (double*)(w + d->tiles);
  double* Bt = At + (int64_t)d->mt * d->nt * nb * nb;
  const int64_t Mp = (int64_t)d->mt * nb;
  const int64_t ta = Mp * d->nt * nb, tb = d->nrhs > 0 ? Mp * d->nrt * nb : 0;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < ta + tb;
       x += (int64_t)gridDim.x * blockDim.x) {
    if (x < ta)
      tile_copy_elem<double, double>(d->A, d->lda, At, d->M, d->N, nb, nb, d->mt, x, in);
    else
      tile_copy_elem<double, double>(d->B, d->ldb, Bt, d->M, d->nrhs, nb, nb, d->mt, x - ta, in);
  }
}

// ---------------------------------------------------------------------------
// Triangular solves with the leading N x N upper triangle R of factored tiles
// (tile (i, j) at (j mt + i) NB^2, column-major inside, leading dimension
// NB; element type E, arithmetic in FP64), one right-hand side per
// workgroup of 256 threads, y overwritten by the solution:
//   TRANS = 0: R x = y (back substitution),  TRANS = 1: R^T x = y (forward).
// Row a of y is at y[(a / NB) rs + a % NB]: rs = NB for a contiguous vector,
// NB cw for a column of a matrix kept in tile-row blocks of cw columns.
// Unknowns are taken 64 at a time (from the bottom for TRANS = 0): wave 0
// holds the block's 64 x 64 triangle in registers, one equation per lane,
// and solves it lane by lane (reciprocals of the diagonal taken in
// parallel, each new unknown broadcast with a lane read); then every thread
// removes the block from one of the rows still to be solved at a time,
// with all 64 products' loads issued together.  With ctrl not null a zero
// diagonal entry R_jj is recorded there (status HQR_ERR_SINGULAR, *info =
// max over such j of N - j; nword, when not null, receives N).
template <typename E, int NB, int TRANS>
__device__ void trsv_solve(const E* R, int mt, int64_t N, double* y, int64_t rs, int32_t* ctrl, int32_t* info,
                           int32_t* nword) {
  __shared__ double xb[64];
  __shared__ double Rd[64 * 65];  // Rd[i * 65 + j] = R(k0 + i, k0 + j), zero outside the triangle
  const int t = threadIdx.x, lane = t & 63;
  const int64_t tsz = (int64_t)NB * NB;
  const int64_t nblk = (N + 63) / 64;
  for (int64_t bi = 0; bi < nblk; ++bi) {
    const int64_t blk = TRANS ? bi : nblk - 1 - bi;
    const int64_t k0 = blk * 64;
    const int nv = (int)((N - k0) < 64 ? (N - k0) : 64);
    const int64_t kt = k0 / NB, ko = k0 - kt * NB;  // the 64 rows / columns lie in tile row / column kt
    const E* Rkk = R + (kt * mt + kt) * tsz + ko + ko * NB;
    {
      // the whole 64 x 64 square lies inside tile (kt, kt): every load is
      // issued before the first is used
      E rv[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int e = t + 256 * k, i = e & 63, j = e >> 6;
        rv[k] = Rkk[i + (int64_t)j * NB];
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int e = t + 256 * k, i = e & 63, j = e >> 6;
        Rd[i * 65 + j] = (i < nv && j < nv && i <= j) ? (double)rv[k] : 0.0;
      }
    }
    double* yk = y + kt * rs + ko;  // y(k0)
    __syncthreads();
    if (t < 64) {
      // cf[s]: coefficient of unknown k0 + s in this lane's equation; a lane
      // beyond the nv unknowns solves 1 x = 0 and touches no other lane
      double cf[64];
#pragma unroll
      for (int s = 0; s < 64; ++s) cf[s] = TRANS ? Rd[s * 65 + lane] : Rd[lane * 65 + s];
      const bool in = lane < nv;
      const double dg = in ? Rd[lane * 66] : 1.0;
      if (ctrl && in && dg == 0.0) {
        int32_t none = 0;
        __hip_atomic_compare_exchange_strong(&ctrl[1], &none, (int32_t)HQR_ERR_SINGULAR, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_max(info, (int32_t)(N - (k0 + lane)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (nword) __hip_atomic_store(nword, (int32_t)N, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      const double rinv = 1.0 / dg;
      double v = in ? yk[lane] : 0.0;
#pragma unroll
      for (int st = 0; st < 64; ++st) {
        const int s = TRANS ? st : 63 - st;
        const double xs = readlane(v * rinv, s);
        // lanes whose unknown is still open take the product; solved lanes keep theirs
        const double u = v - cf[s] * xs;
        v = (lane == s) ? xs : ((TRANS ? lane > s : lane < s) ? u : v);
      }
      xb[lane] = lane < nv ? v : 0.0;
      if (lane < nv) yk[lane] = v;
    }
    __syncthreads();
    // rows still open: TRANS those after the block (R(k0 + c, a), contiguous
    // in c: 16-byte loads), else those before it (R(a, k0 + c), stride NB in
    // c).  The 64 rows of a wave lie in one tile row (lo and the wave's first
    // row are multiples of 64), so the tile is addressed through a buffer
    // resource with one lane offset and a constant offset per column.  Only
    // the bottom block of TRANS = 0 can hold fewer than 64 unknowns.
    const int64_t lo = TRANS ? k0 + 64 : 0, hi = TRANS ? N : k0;
    for (int64_t a = lo + t; a < hi; a += 256) {
      const int64_t at = a / NB, ao = a - at * NB;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      if (TRANS) {
        const __amdgpu_buffer_rsrc_t rr = rsrc(R + (at * mt + kt) * tsz);  // tile (kt, at)
        const int vo = (int)((ko + ao * NB) * (int64_t)sizeof(E));
        constexpr int PER = 16 / (int)sizeof(E);  // elements per 16-byte load
        u4 raw[64 / PER];
#pragma unroll
        for (int q = 0; q < 64 / PER; ++q) raw[q] = __builtin_amdgcn_raw_buffer_load_b128(rr, vo + 16 * q, 0, 0);
#pragma unroll
        for (int q = 0; q < 64 / PER; ++q) {
          if constexpr (sizeof(E) == 8) {
            const d2 x = __builtin_bit_cast(d2, raw[q]);
            acc[(2 * q) & 3] += x.x * xb[2 * q];
            acc[(2 * q + 1) & 3] += x.y * xb[2 * q + 1];
          } else {
            const f4 x = __builtin_bit_cast(f4, raw[q]);
            acc[0] += (double)x.x * xb[4 * q];
            acc[1] += (double)x.y * xb[4 * q + 1];
            acc[2] += (double)x.z * xb[4 * q + 2];
            acc[3] += (double)x.w * xb[4 * q + 3];
          }
        }
      } else {
        const __amdgpu_buffer_rsrc_t rr = rsrc(R + (kt * mt + at) * tsz);  // tile (at, kt)
        const int vo = (int)((ao + ko * NB) * (int64_t)sizeof(E));
        constexpr int CS = NB * (int)sizeof(E);  // bytes from one column to the next
        if (nv == 64) {
          E r0[64];
#pragma unroll
          for (int c = 0; c < 64; ++c) r0[c] = bload1<E>(rr, vo, c * CS);
#pragma unroll
          for (int c = 0; c < 64; ++c) acc[c & 3] += (double)r0[c] * xb[c];
        } else {
          for (int c = 0; c < nv; ++c) acc[c & 3] += (double)bload1<E>(rr, vo, c * CS) * xb[c];
        }
      }
      y[at * rs + ao] -= (acc[0] + acc[1]) + (acc[2] + acc[3]);
    }
    __syncthreads();
  }
}

// R x = y for column c of a matrix Y kept in tile-row blocks of cw columns
// (block (i, jb) at Y + (jb mt + i) NB cw, column-major with leading
// dimension NB): the tile columns of B appended to the factorization
// (cw = NB) or the blocks of B of the apply path (cw = 64).
template <int NB>
__device__ __forceinline__ void trsv_column(const double* R, double* Y, int cw, int mt, int64_t N, int c,
                                            int32_t* ctrl, int32_t* info, int32_t* nword) {
  double* y = Y + (int64_t)(c / cw) * mt * NB * cw + (int64_t)(c % cw) * NB;
  trsv_solve<double, NB, 0>(R, mt, N, y, (int64_t)NB * cw, ctrl, info, nword);
}

// One problem: workgroup x = right-hand-side column.  A zero diagonal entry
// sets ctrl[6] = max(N - j) and ctrl[7] = N.
template <int NB>
__global__ __launch_bounds__(256) void trsv_kernel(const double* R, double* Y, int cw, int mt, int64_t N,
                                                   int32_t* ctrl) {
  trsv_column<NB>(R, Y, cw, mt, N, blockIdx.x, ctrl, &ctrl[6], &ctrl[7]);
}

// Every problem of a batch in one launch: workgroup (x, q) solves
// right-hand-side column x of problem q (its B tile columns follow the
// matrix tiles).
template <int NB>
__global__ __launch_bounds__(256) void trsv_batched_kernel(const ProbDesc* descs, char* w, int32_t* ctrl,
                                                           int32_t* info) {
  const ProbDesc* d = descs + blockIdx.y;
  if ((int)blockIdx.x >= d->nrhs) return;
  const double* R = (const double*)(w + d->tiles);
  double* Y = (double*)(w + d->tiles) + (int64_t)d->mt * d->nt * NB * NB;
  trsv_column<NB>(R, Y, NB, d->mt, d->N, blockIdx.x, ctrl, info + blockIdx.y, nullptr);
}

// ---------------------------------------------------------------------------
// Iterative refinement of least squares (FP64 residuals, FP32 factors).

// f = b - r - A x (r may be null).  A: M x N column-major (lda).  Workgroup
// of 256 threads = 64 rows x 4 column groups (each group sums every fourth
// column, eight loads in flight), partial sums combined in a fixed order.
__global__ __launch_bounds__(256) void ir_residual_kernel(const double* A, int64_t lda, int64_t M, int64_t N,
                                                          const double* x, const double* b, const double* r,
                                                          double* f) {
  __shared__ double part[4][64];
  const int lr = threadIdx.x & 63, cg = threadIdx.x >> 6;
  const int64_t row = (int64_t)blockIdx.x * 64 + lr;
  double s = 0.0;
  if (row < M) {
#pragma unroll 8
    for (int64_t j = cg; j < N; j += 4) s += A[row + j * lda] * x[j];
  }
  part[cg][lr] = s;
  __syncthreads();
  if (cg == 0 && row < M)
    f[row] = b[row] - (r ? r[row] : 0.0) - ((part[0][lr] + part[1][lr]) + (part[2][lr] + part[3][lr]));
}

// g = -A^T r (SQ = 0), or g_j = sum_i A_ij^2 (SQ = 1, r unused).
// Workgroup per IR_ATR_COLS columns (so that a launch has several
// workgroups per compute unit); 256 threads stride over the rows, four rows
// in flight each; a fixed reduction tree per column.
constexpr int IR_ATR_COLS = 2;
template <int SQ>
__global__ __launch_bounds__(256) void ir_atr_kernel(const double* A, int64_t lda, int64_t M, int64_t N,
                                                     const double* r, double* g) {
  constexpr int C = IR_ATR_COLS;
  __shared__ double part[C][257];
  const int t = threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.x * C;
  const int nc = (int)((N - c0) < C ? (N - c0) : C);
  double s[C];
#pragma unroll
  for (int c = 0; c < C; ++c) s[c] = 0.0;
#pragma unroll 4
  for (int64_t i = t; i < M; i += 256) {
    const double ri = SQ ? 0.0 : r[i];
#pragma unroll
    for (int c = 0; c < C; ++c)
      if (c < nc) {
        const double aij = A[i + (c0 + c) * lda];
        s[c] += aij * (SQ ? aij : ri);
      }
  }
#pragma unroll
  for (int c = 0; c < C; ++c) part[c][t] = s[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
#pragma unroll
      for (int c = 0; c < C; ++c) part[c][t] += part[c][t + w];
    }
    __syncthreads();
  }
  if (t < nc) g[c0 + t] = SQ ? part[t][0] : -part[t][0];
}

// Triangular solves of the refinement with the float tiles R of the FP32
// factorization, in FP64 arithmetic, y (contiguous) overwritten:
//   TRANS = 0: R x = y,  TRANS = 1: R^T x = y.
template <int NB, int TRANS>
__global__ __launch_bounds__(256) void ir_trsv_kernel(const float* R, int mt, int64_t N, double* y) {
  trsv_solve<float, NB, TRANS>(R, mt, N, y, NB, nullptr, nullptr, nullptr);
}

// y = d(0:N) - h;  then d(0:N) = h  (the two uses of h in one correction).
__global__ void ir_split_kernel(double* d, const double* h, double* y, int64_t N) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    y[i] = d[i] - h[i];
    d[i] = h[i];
  }
}

// x += dx (N), r += dr (M).
__global__ void ir_update_kernel(double* x, const double* dx, int64_t N, double* r, const double* dr, int64_t M) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
    if (i < N) x[i] += dx[i];
    r[i] += dr[i];
  }
}

// out[k] = sum of squares of vector k (v[k], n[k] entries; a null vector
// gives 0), k < 4; one workgroup, fixed order.
struct Vec4Args {
  const double* v[4];
  int64_t n[4];
};
__global__ __launch_bounds__(256) void ir_norms_kernel(Vec4Args a, double* out) {
  __shared__ double part[4][256];
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double sk = 0.0;
    if (a.v[k])
      for (int64_t i = t; i < a.n[k]; i += 256) sk += a.v[k][i] * a.v[k][i];
    part[k][t] = sk;
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
#pragma unroll
      for (int k = 0; k < 4; ++k) part[k][t] += part[k][t + w];
    }
    __syncthreads();
  }
  if (t < 4) out[t] = part[t][0];
}

// Records the last HIP failure for hqr_last_error().
static thread_local char g_last_error[256];

int record_hip(hipError_t e, const char* where) {
  if (e == hipSuccess) return 0;
  snprintf(g_last_error, sizeof(g_last_error), "%s: %s", where, hipGetErrorString(e));
  return HQR_ERR_HIP;
}

const char* last_error() { return g_last_error; }

void set_last_error(const char* msg) { snprintf(g_last_error, sizeof(g_last_error), "%s", msg); }

static int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

int launch_ir_residual(const double* A, int64_t lda, int64_t M, int64_t N, const double* x, const double* b,
                       const double* r, double* f, void* stream) {
  hipLaunchKernelGGL(ir_residual_kernel, dim3((unsigned)((M + 63) / 64)), dim3(256), 0, (hipStream_t)stream, A, lda,
                     M, N, x, b, r, f);
  return record_hip(hipGetLastError(), "ir_residual_kernel launch");
}

int launch_ir_atr(const double* A, int64_t lda, int64_t M, int64_t N, const double* r, double* g, void* stream) {
  if (r)
    hipLaunchKernelGGL(ir_atr_kernel<0>, dim3((unsigned)((N + IR_ATR_COLS - 1) / IR_ATR_COLS)), dim3(256), 0,
                       (hipStream_t)stream, A, lda, M, N, r, g);
  else
    hipLaunchKernelGGL(ir_atr_kernel<1>, dim3((unsigned)((N + IR_ATR_COLS - 1) / IR_ATR_COLS)), dim3(256), 0,
                       (hipStream_t)stream, A, lda, M, N, r, g);
  return record_hip(hipGetLastError(), "ir_atr_kernel launch");
}

int launch_ir_trsv(const float* R, int nb, int mt, int64_t N, double* y, bool trans, void* stream) {
  hipStream_t s = (hipStream_t)stream;
#define HQR_IR_TRSV(NBV)                                                                        \
  if (trans)                                                                                    \
    hipLaunchKernelGGL((ir_trsv_kernel<NBV, 1>), dim3(1), dim3(256), 0, s, R, mt, N, y);        \
  else                                                                                          \
    hipLaunchKernelGGL((ir_trsv_kernel<NBV, 0>), dim3(1), dim3(256), 0, s, R, mt, N, y);
  switch (nb) {
    case 64: HQR_IR_TRSV(64) break;
    case 128: HQR_IR_TRSV(128) break;
    default: HQR_IR_TRSV(256) break;
  }
#undef HQR_IR_TRSV
  return record_hip(hipGetLastError(), "ir_trsv_kernel launch");
}

int launch_ir_split(double* d, const double* h, double* y, int64_t N, void* stream) {
  hipLaunchKernelGGL(ir_split_kernel, dim3(grid_for(N)), dim3(256), 0, (hipStream_t)stream, d, h, y, N);
  return record_hip(hipGetLastError(), "ir_split_kernel launch");
}

int launch_ir_update(double* x, const double* dx, int64_t N, double* r, const double* dr, int64_t M, void* stream) {
  hipLaunchKernelGGL(ir_update_kernel, dim3(grid_for(M)), dim3(256), 0, (hipStream_t)stream, x, dx, N, r, dr, M);
  return record_hip(hipGetLastError(), "ir_update_kernel launch");
}

int launch_ir_norms(const double* const* v, const int64_t* n, double* out, void* stream) {
  Vec4Args a;
  for (int k = 0; k < 4; ++k) {
    a.v[k] = v[k];
    a.n[k] = n[k];
  }
  hipLaunchKernelGGL(ir_norms_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, a, out);
  return record_hip(hipGetLastError(), "ir_norms_kernel launch");
}

int launch_zero_i32(int32_t* p, int64_t n, void* stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(zero_i32_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, p, n);
  return record_hip(hipGetLastError(), "zero_i32_kernel launch");
}

int launch_init_ctrl(int32_t* ctrl, const FactorSig& sig, int32_t* cnt, int64_t ncnt, void* stream) {
  const int64_t n = ncnt > kCtrlWords ? ncnt : kCtrlWords;
  hipLaunchKernelGGL(init_ctrl_kernel, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, ctrl, sig, cnt, ncnt);
  return record_hip(hipGetLastError(), "init_ctrl_kernel launch");
}

int launch_check_sig(const int32_t* fctrl, const FactorSig& sig, int32_t* bctrl, void* stream) {
  hipLaunchKernelGGL(check_sig_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, fctrl, sig, bctrl);
  return record_hip(hipGetLastError(), "check_sig_kernel launch");
}

int launch_tile_copy(void* A, int a_f32, int64_t lda, void* At, int at_f32, int64_t M, int64_t N, int nb, int tw,
                     int mt, int nt, bool in, void* stream) {
  const int64_t total = (int64_t)mt * nb * (int64_t)nt * tw;
  const dim3 g(grid_for(total)), b(256);
  hipStream_t s = (hipStream_t)stream;
  const int i = in ? 1 : 0;
  if (!a_f32 && !at_f32)
    hipLaunchKernelGGL((tile_copy_kernel<double, double>), g, b, 0, s, (double*)A, lda, (double*)At, M, N, nb, tw, mt,
                       nt, i);
  else if (!a_f32 && at_f32)
    hipLaunchKernelGGL((tile_copy_kernel<double, float>), g, b, 0, s, (double*)A, lda, (float*)At, M, N, nb, tw, mt,
                       nt, i);
  else if (a_f32 && at_f32)
    hipLaunchKernelGGL((tile_copy_kernel<float, float>), g, b, 0, s, (float*)A, lda, (float*)At, M, N, nb, tw, mt, nt,
                       i);
  else
    return HQR_ERR_INTERNAL;
  return record_hip(hipGetLastError(), "tile_copy_kernel launch");
}

int launch_tile_copy(double* A, int64_t lda, double* At, int64_t M, int64_t N, int nb, int tw, int mt, int nt,
                     bool in, void* stream) {
  return launch_tile_copy(A, 0, lda, At, 0, M, N, nb, tw, mt, nt, in, stream);
}

int launch_trsv(int nb, const double* R, double* Y, int cw, int32_t* ctrl, int64_t N, int mt, int nrhs,
                void* stream) {
  if (nrhs <= 0) return 0;
  hipStream_t s = (hipStream_t)stream;
  switch (nb) {
    case 64: hipLaunchKernelGGL(trsv_kernel<64>, dim3(nrhs), dim3(256), 0, s, R, Y, cw, mt, N, ctrl); break;
    case 128: hipLaunchKernelGGL(trsv_kernel<128>, dim3(nrhs), dim3(256), 0, s, R, Y, cw, mt, N, ctrl); break;
    default: hipLaunchKernelGGL(trsv_kernel<256>, dim3(nrhs), dim3(256), 0, s, R, Y, cw, mt, N, ctrl); break;
  }
  return record_hip(hipGetLastError(), "trsv_kernel launch");
}

int launch_copy_batched(const ProbDesc* d, char* w, int count, int nb, bool in, int64_t max_elems, void* stream) {
  if (count <= 0) return 0;
  // workgroups per problem: enough for about 8 elements per thread of the largest problem
  int64_t gx = (max_elems + 2047) / 2048;
  if (gx < 1) gx = 1;
  if (gx > 4096) gx = 4096;
  hipLaunchKernelGGL(copy_batched_kernel, dim3((unsigned)gx, count), dim3(256), 0, (hipStream_t)stream, d, w, nb,
                     in ? 1 : 0);
  return record_hip(hipGetLastError(), "copy_batched_kernel launch");
}

int launch_trsv_batched(int nb, const ProbDesc* d, char* w, int32_t* ctrl, int32_t* info, int count, int max_nrhs,
                        void* stream) {
  if (count <= 0 || max_nrhs <= 0) return 0;
  const dim3 grid(max_nrhs, count), block(256);
  hipStream_t s = (hipStream_t)stream;
  switch (nb) {
    case 64: hipLaunchKernelGGL(trsv_batched_kernel<64>, grid, block, 0, s, d, w, ctrl, info); break;
    case 128: hipLaunchKernelGGL(trsv_batched_kernel<128>, grid, block, 0, s, d, w, ctrl, info); break;
    default: hipLaunchKernelGGL(trsv_batched_kernel<256>, grid, block, 0, s, d, w, ctrl, info); break;
  }
  return record_hip(hipGetLastError(), "trsv_batched_kernel launch");
}

template <typename E, int NB>
static int occupancy_workers() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, persistent_kernel<E, NB, false>, NT, sizeof(Smem<E, NB>)) != hipSuccess ||
      per < 1)
    per = 1;
  return cus * per;
}

int default_workers(int nb, bool f32) {
  if (f32) {
    switch (nb) {
      case 64: return occupancy_workers<float, 64>();
      case 128: return occupancy_workers<float, 128>();
      default: return occupancy_workers<float, 256>();
    }
  }
  switch (nb) {
    case 64: return occupancy_workers<double, 64>();
    case 128: return occupancy_workers<double, 128>();
    default: return occupancy_workers<double, 256>();
  }
}

template <typename E, bool BF = false>
static int launch_persistent_t(int nb, const LaunchArgs& a, int workers, hipStream_t s) {
  const dim3 g(workers), b(NT);
  if (a.probs) {
    switch (nb) {
      case 64: hipLaunchKernelGGL((persistent_kernel<E, 64, true>), g, b, sizeof(Smem<E, 64>), s, a); break;
      case 128: hipLaunchKernelGGL((persistent_kernel<E, 128, true>), g, b, sizeof(Smem<E, 128>), s, a); break;
      case 256: hipLaunchKernelGGL((persistent_kernel<E, 256, true>), g, b, sizeof(Smem<E, 256>), s, a); break;
      default: return HQR_ERR_INTERNAL;
    }
  } else {
    switch (nb) {
      case 64: hipLaunchKernelGGL((persistent_kernel<E, 64, false, BF>), g, b, sizeof(Smem<E, 64>), s, a); break;
      case 128: hipLaunchKernelGGL((persistent_kernel<E, 128, false, BF>), g, b, sizeof(Smem<E, 128>), s, a); break;
      case 256: hipLaunchKernelGGL((persistent_kernel<E, 256, false, BF>), g, b, sizeof(Smem<E, 256>), s, a); break;
      default: return HQR_ERR_INTERNAL;
    }
  }
  return record_hip(hipGetLastError(), "persistent_kernel launch");
}

int launch_persistent(int nb, const LaunchArgs& a, int workers, void* stream, bool f32, bool bf16) {
  if (workers < 1) workers = 1;
  // the batched path runs in FP64 only; BF16 products take float tiles
  if (f32 && a.probs) return HQR_ERR_INTERNAL;
  if (bf16 && (!f32 || a.B)) return HQR_ERR_INTERNAL;
  if (bf16) return launch_persistent_t<float, true>(nb, a, workers, (hipStream_t)stream);
  return f32 ? launch_persistent_t<float>(nb, a, workers, (hipStream_t)stream)
             : launch_persistent_t<double>(nb, a, workers, (hipStream_t)stream);
}

}  // namespace hqr
