// cr_lib.hip -- kernels and the C ABI of libcr (gfx950).
//
// One elementwise map kernel per function (a template over the function's
// evaluator).  Each workgroup stages the function's <= 16-entry tables in LDS
// once, then each thread loads U float4 vectors (128-bit, coalesced: lane i of
// a wave touches bytes [16 i, 16 i + 16) of a contiguous 1 KiB span), evaluates
// the 4U elements and stores U float4 vectors.  Pointers that are not 16-byte
// aligned, and ragged tails, go through a scalar grid-stride kernel.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <vector>
#include <mutex>

#include "../../include/cr.h"
#include "cr_f32_exp.h"
#include "cr_f32_log.h"
#include "cr_f32_rsqrt.h"
#include "cr_f32_trig.h"
#include "cr_f32_atan.h"
#include "cr_f32_hyp.h"
#include "cr_f64.h"
#include "cr_f32_dir.h"
#include "cr_split_exp.h"
#include "cr_split_log.h"
#include "cr_split_trig.h"
#include "cr_split_rsqrt.h"
#include "cr_split_atan.h"
#include "cr_split_hyp.h"
#include "cr_split_acc.h"

using namespace cr;

namespace {

// Counters are spread over NSLOT cache lines (slot = block index mod NSLOT)
// so that concurrent workgroups do not serialise on one address; the host
// sums them when they are read.
constexpr int NSLOT = 64;
struct alignas(128) CounterSlot {
  unsigned long long fallback_lanes, fallback_waves;
  unsigned long long pad[14];
};
struct DevStats {
  CounterSlot slot[NSLOT];
  unsigned long long escapes;
  unsigned long long escape_index[16];
};

// Launch-shape knobs (compile-time; the grid size is a run-time knob).
#ifndef CR_TILE_U
#define CR_TILE_U 2
#endif
#ifndef CR_PREFETCH
#define CR_PREFETCH 1
#endif
#ifndef CR_BLOCKS_PER_CU
#define CR_BLOCKS_PER_CU 16
#endif
constexpr int BLOCK = 256;
constexpr int TILE_U = CR_TILE_U;           // float4 vectors per thread per tile (sincosf)
// Batch tiles: BATCH_U float4 vectors per thread, TILE elements per tile.
// Measured on the 4096-request batch (three alternating runs per build),
// 4096-element tiles against 2048: +0.9% binary64-internal, +1.6%
// binary32-only, within the run-to-run spread (larger tiles mean fewer
// tile-table reads and queue checks per element, smaller ones a shorter tail).
#ifndef CR_BATCH_U
#define CR_BATCH_U 4
#endif
constexpr int BATCH_U = CR_BATCH_U;
constexpr int TILE = BLOCK * 4 * BATCH_U;   // 4096 elements per tile
constexpr int QCAP = 512;                   // deferred elements held in LDS
constexpr int QCHECK = 8;                   // tiles between two looks at the queue
constexpr int QFLUSH = QCAP / 2;            // flush when the queue is fuller than this

// Streaming accesses: each input is read once and each output written once,
// so the 128-bit loads and stores carry the nontemporal hint (measured on
// MI355X: a plain 2^26-float copy moves 5.1-5.5 TB/s without it and
// 5.8-6.6 TB/s with it, depending on the grid).
#ifndef CR_NT
#define CR_NT 1
#endif
typedef float v4f_t __attribute__((ext_vector_type(4)));
typedef double v2d_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float4 ld_stream(const float4* p) {
  if (!CR_NT) return *p;
  v4f_t v = __builtin_nontemporal_load(reinterpret_cast<const v4f_t*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st_stream(float4* p, float4 a) {
  if (!CR_NT) {
    *p = a;
    return;
  }
  v4f_t v = {a.x, a.y, a.z, a.w};
  __builtin_nontemporal_store(v, reinterpret_cast<v4f_t*>(p));
}
__device__ __forceinline__ double2 ld_stream(const double2* p) {
  if (!CR_NT) return *p;
  v2d_t v = __builtin_nontemporal_load(reinterpret_cast<const v2d_t*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void st_stream(double2* p, double2 a) {
  if (!CR_NT) {
    *p = a;
    return;
  }
  v2d_t v = {a.x, a.y};
  __builtin_nontemporal_store(v, reinterpret_cast<v2d_t*>(p));
}

// ------------------------------------------------------------ evaluators
// Op::fast(x, tab, ok): binary64 fast path and rounding test (inlined).
// Op::accurate(x, tab): double-double path from x alone (out of line).
// Op::dir<RM>(x, tab): the result in a directed rounding mode (out of line).
template <int K>
struct OpExp {
  using Tab = ExpTab;
  static constexpr int qcheck = QCHECK;
  static __device__ __forceinline__ void load(Tab& t, int tid) { exp_tab_load(t, tid); }
  static __device__ __forceinline__ float fast(float x, const Tab& t, bool& ok) {
    return exp_fast<K>(x, t, ok);
  }
  static __device__ __forceinline__ AccResult accurate(float x, const Tab& t) {
    return exp_accurate<K>(x, t);
  }
  template <int RM>
  static __device__ __forceinline__ AccResult dir(float x, const Tab& t) {
    return exp_dir<K, RM>(x, t);
  }
};

// sincos: two outputs per element (planar)
struct SinCosF64 {
  using Tab = TrigTab;
  static constexpr int qcheck = QCHECK;
  static __device__ __forceinline__ void load(Tab& t, int tid) { trig_tab_load(t, tid); }
  static __device__ __forceinline__ float fast(float x, const Tab& t, float& c, bool& ok) {
    return sincos_fast(x, t, c, ok);
  }
  static __device__ __forceinline__ AccResult2 accurate(float x, const Tab& t) {
    return sincos_accurate(x, t);
  }
  template <int RM>
  static __device__ __forceinline__ AccResult2 dir(float x, const Tab& t) {
    return sincos_dir<RM>(x, t);
  }
};
struct SinCosSplit {
  using Tab = STrigTab;
  static constexpr int qcheck = 1;
  static __device__ __forceinline__ void load(Tab& t, int tid) { strig_tab_load(t, tid); }
  static __device__ __forceinline__ float fast(float x, const Tab& t, float& c, bool& ok) {
    return ssincos_fast(x, t, c, ok);
  }
  static __device__ __forceinline__ AccResult2 accurate(float x, const Tab& t) {
    return ssincos_acc(x, t.w);
  }
};

struct OpSRsqrt {
  using Tab = NoTab;
  static constexpr int qcheck = QCHECK;
  static __device__ __forceinline__ void load(Tab&, int) {}
  static __device__ __forceinline__ float fast(float x, const Tab&, bool& ok) {
    return srsqrt_fast(x, ok);
  }
  static __device__ __forceinline__ AccResult accurate(float x, const Tab&) {
    bool ok;
    return {srsqrt_fast(x, ok), 1};
  }
};

template <int KIND>
struct OpSAtan {
  using Tab = SAtanTab;
  static constexpr int qcheck = 1;  // more lanes fail: look at the queue every tile
  static __device__ __forceinline__ void load(Tab& t, int tid) { satan_tab_load(t, tid); }
  static __device__ __forceinline__ float fast(float x, const Tab& t, bool& ok) {
    return satan_fast<KIND>(x, t, ok);
  }
  static __device__ __forceinline__ AccResult accurate(float x, const Tab& t) {
    return satan_acc<KIND>(x);
  }
};

template <int KIND>
struct OpSHyp {
  using Tab = SHypTab;
  static constexpr int qcheck = 1;  // more lanes fail: look at the queue every tile
  static __device__ __forceinline__ void load(Tab& t, int tid) { shyp_tab_load(t, tid); }
  static __device__ __forceinline__ float fast(float x, const Tab& t, bool& ok) {
    return shyp_fast<KIND>(x, t, ok);
  }
  static __device__ __forceinline__ AccResult accurate(float x, const Tab& t) {
    return shyp_acc<KIND>(x);
  }
};

template <int KIND>
struct OpSTrig {
  using Tab = STrigTab;
  static constexpr int qcheck = 1;  // more lanes fail: look at the queue every tile
  static __device__ __forceinline__ void load(Tab& t, int tid) { strig_tab_load(t, tid); }
  static __device__ __forceinline__ float fast(float x, const Tab& t, bool& ok) {
    return strig_fast<KIND>(x, t, ok);
  }
  static __device__ __forceinline__ AccResult accurate(float x, const Tab& t) {
    return strig_acc<KIND>(x, t.w);
  }
};

// binary32-only (float-float) fast paths; failing lanes take the triple-float
// step (cr_split_acc.h): no binary64 operation on the whole path
template <int K>
struct OpSExp {
  using Tab = SExpTab;
  static constexpr int qcheck = 1;  // more lanes fail: look at the queue every tile
  static __device__ __forceinline__ void load(Tab& t, int tid) { sexp_tab_load<K>(t, tid); }
  static __device__ __forceinline__ float fast(float x, const Tab& t, bool& ok) {
    return sexp_fast<K>(x, t, ok);
  }
  static __device__ __forceinline__ AccResult accurate(float x, const Tab& t) {
    return sexp_acc<K>(x);
  }
};

template <int K>
struct OpSLog {
  using Tab = SLogTab;
  static constexpr int qcheck = 1;  // more lanes fail: look at the queue every tile
  static __device__ __forceinline__ void load(Tab& t, int tid) { slog_tab_load<K>(t, tid); }
  static __device__ __forceinline__ float fast(float x, const Tab& t, bool& ok) {
    return slog_fast<K>(x, t, ok);
  }
  static __device__ __forceinline__ AccResult accurate(float x, const Tab& t) {
    return slog_acc<K>(x);
  }
};

template <int K>
struct OpLog {
  using Tab = LogTab;
  static constexpr int qcheck = QCHECK;
  static __device__ __forceinline__ void load(Tab& t, int tid) { log_tab_load<K>(t, tid); }
  static __device__ __forceinline__ float fast(float x, const Tab& t, bool& ok) {
    return log_fast<K>(x, t, ok);
  }
  static __device__ __forceinline__ AccResult accurate(float x, const Tab& t) {
    return log_accurate<K>(x, t);
  }
  template <int RM>
  static __device__ __forceinline__ AccResult dir(float x, const Tab& t) {
    return log_dir<K, RM>(x, t);
  }
};

// rsqrtf decides its rounding exactly in the fast path: nothing is deferred.
struct OpRsqrt {
  using Tab = NoTab;
  static constexpr int qcheck = QCHECK;
  static __device__ __forceinline__ void load(Tab&, int) {}
  static __device__ __forceinline__ float fast(float x, const Tab&, bool& ok) {
    return rsqrt_fast(x, ok);
  }
  static __device__ __noinline__ AccResult accurate(float x, const Tab&) {
    bool ok;
    return {rsqrt_fast(x, ok), 1};
  }
  template <int RM>
  static __device__ __forceinline__ AccResult dir(float x, const Tab&) {
    return rsqrt_dir<RM>(x);
  }
};

template <int KIND>
struct OpTrig {
  using Tab = TrigTab;
  static constexpr int qcheck = QCHECK;
  static __device__ __forceinline__ void load(Tab& t, int tid) { trig_tab_load(t, tid); }
  static __device__ __forceinline__ float fast(float x, const Tab& t, bool& ok) {
    return trig_fast<KIND>(x, t, ok);
  }
  static __device__ __forceinline__ AccResult accurate(float x, const Tab& t) {
    return trig_accurate<KIND>(x, t);
  }
  template <int RM>
  static __device__ __forceinline__ AccResult dir(float x, const Tab& t) {
    return trig_dir<KIND, RM>(x, t);
  }
};

template <int KIND>
struct OpAtan {
  using Tab = AtanTab;
  static constexpr int qcheck = QCHECK;
  static __device__ __forceinline__ void load(Tab& t, int tid) { atan_tab_load(t, tid); }
  static __device__ __forceinline__ float fast(float x, const Tab& t, bool& ok) {
    return atan_fast<KIND>(x, t, ok);
  }
  static __device__ __forceinline__ AccResult accurate(float x, const Tab& t) {
    return atan_accurate<KIND>(x, t);
  }
  template <int RM>
  static __device__ __forceinline__ AccResult dir(float x, const Tab& t) {
    return atan_dir<KIND, RM>(x, t);
  }
};

template <int KIND>
struct OpHyp {
  using Tab = ExpTab;
  static constexpr int qcheck = QCHECK;
  static __device__ __forceinline__ void load(Tab& t, int tid) { exp_tab_load(t, tid); }
  static __device__ __forceinline__ float fast(float x, const Tab& t, bool& ok) {
    return hyp_fast<KIND>(x, t, ok);
  }
  static __device__ __forceinline__ AccResult accurate(float x, const Tab& t) {
    return hyp_accurate<KIND>(x, t);
  }
  template <int RM>
  static __device__ __forceinline__ AccResult dir(float x, const Tab& t) {
    return hyp_dir<KIND, RM>(x, t);
  }
};

// Block-level bookkeeping of the accurate path, kept in LDS.
struct Deferred {
  unsigned n;                 // entries in the queue
  unsigned lanes, waves;      // counters of this workgroup
  unsigned idx[QCAP];         // element index (relative to the launch)
  float x[QCAP];              // the input value (the output may alias it)
};

__device__ __forceinline__ void note_escape(DevStats* st, long long idx) {
  unsigned long long slot = atomicAdd(&st->escapes, 1ull);
  if (slot < 16) st->escape_index[slot] = (unsigned long long)idx;
}

// Runs body(k) on every queued entry k, 256 at a time (whole waves).
// FINAL = false: then empties the queue; all threads of the workgroup take
// part.  FINAL = true: the workgroup's last flush, after its final barrier; no
// barrier follows, so waves with no entry retire at once and free their slots
// for the next workgroup while the others run the accurate path, and the
// workgroup's counters go to the device statistics.
template <bool FINAL, class Q, class Body>
__device__ __forceinline__ void run_queue(Q& q, DevStats* st, Body body) {
  // q.n counts every enqueue attempt; entries past QCAP were never stored
  // (those elements took the accurate path in place), so only QCAP are valid
  const unsigned n = q.n < QCAP ? q.n : QCAP;
  for (unsigned k = threadIdx.x; k < n; k += BLOCK) body(k);
  if (FINAL) {
    if (threadIdx.x == 0) {
      const unsigned lanes = q.lanes + n, waves = q.waves + (n + 63) / 64;
      if (lanes) {
        CounterSlot& c = st->slot[blockIdx.x % NSLOT];
        atomicAdd(&c.fallback_lanes, (unsigned long long)lanes);
        atomicAdd(&c.fallback_waves, (unsigned long long)waves);
      }
    }
  } else {
    if (threadIdx.x == 0) {
      q.lanes += n;
      q.waves += (n + 63) / 64;
    }
    __syncthreads();
    if (threadIdx.x == 0) q.n = 0;
    __syncthreads();
  }
}

template <class Op, bool FINAL = false>
__device__ __forceinline__ void flush_queue(Deferred& q, const typename Op::Tab& tab, float* out,
                                            DevStats* st, long long elem_base) {
  run_queue<FINAL>(q, st, [&](unsigned k) {
    AccResult a = Op::accurate(q.x[k], tab);
    out[q.idx[k]] = a.r;
    if (!a.ok) note_escape(st, elem_base + q.idx[k]);
  });
}

// ---------------------------------------------------------------- kernels
// Persistent elementwise map over 16-byte aligned data.  Each workgroup walks
// tiles of 2048 elements (tile t, t + gridDim.x, ...).  Per tile every thread
// loads two float4 (lane i of a wave touches bytes [16 i, 16 i + 16) of a
// contiguous 1 KiB span), runs the fast path on its 8 elements and stores.
// Elements whose fast result is not certified are queued in LDS (index and
// input value) and re-evaluated by the accurate path a whole workgroup at a
// time -- when the queue passes QFLUSH and at the end -- so a rare failing
// lane does not make a 64-lane wave run the slow path for it alone.
// Launch-shape variants (chosen per function by the autotuner, cr_autotune):
//   U   float4 vectors per thread per tile (4U elements per thread),
//   PF  1: the next tile's vectors are loaded while this one is evaluated,
//   TP  table placement: 0 = staged in LDS per workgroup, 1 = read from a
//       device-global copy through the vector caches (no staging).
template <class Op>
__device__ typename Op::Tab g_tab;

template <class Op>
__global__ void k_tab_init() {
  Op::load(g_tab<Op>, threadIdx.x);
}

template <class Op, int U, int PF, int TP>
__global__ void __launch_bounds__(BLOCK)
    k_map_f32(const float4* in, float4* out, long long n4, DevStats* st,
              unsigned flags, long long elem_base) {
  __shared__ typename Op::Tab lds_tab;
  __shared__ Deferred q;
  const typename Op::Tab& tab = TP ? g_tab<Op> : lds_tab;
  if (!TP) Op::load(lds_tab, threadIdx.x);
  if (threadIdx.x == 0) {
    q.n = 0;
    q.lanes = q.waves = 0;
  }
  __syncthreads();
  const bool force = flags & CR_FLAG_FORCE_FALLBACK;
  float* outf = reinterpret_cast<float*>(out);
  const long long ntiles = (n4 + BLOCK * U - 1) / (BLOCK * U);
  // software pipelining: the next tile's vectors are loaded while this tile
  // is evaluated
  float4 nxt[U];
  if (PF) {
    long long base = (long long)blockIdx.x * (BLOCK * U) + threadIdx.x;
#pragma unroll
    for (int u = 0; u < U; u++) {
      long long i = base + (long long)u * BLOCK;
      nxt[u] = i < n4 ? ld_stream(in + i) : make_float4(1.0f, 1.0f, 1.0f, 1.0f);
    }
  }
  int iter = 0;
  for (long long t = blockIdx.x; t < ntiles; t += gridDim.x, iter++) {
    long long base = t * (BLOCK * U) + threadIdx.x;
    float4 v[U];
    if (PF) {
#pragma unroll
      for (int u = 0; u < U; u++) v[u] = nxt[u];
    } else {
#pragma unroll
      for (int u = 0; u < U; u++) {
        long long i = base + (long long)u * BLOCK;
        v[u] = i < n4 ? ld_stream(in + i) : make_float4(1.0f, 1.0f, 1.0f, 1.0f);
      }
    }
    if (PF) {
      long long nb = (t + gridDim.x) * (BLOCK * U) + threadIdx.x;
#pragma unroll
      for (int u = 0; u < U; u++) {
        long long i = nb + (long long)u * BLOCK;
        nxt[u] = i < n4 ? ld_stream(in + i) : make_float4(1.0f, 1.0f, 1.0f, 1.0f);
      }
    }
    // Evaluate every element of the tile first -- straight-line code with no
    // branch between elements, so the scheduler can interleave their
    // dependency chains -- then queue the elements that failed the test.
    // Slots past the end hold stale values: evaluated, never stored or queued.
    float xin[4 * U];
    unsigned fail = 0;
#pragma unroll
    for (int u = 0; u < U; u++) {
      const bool live = base + (long long)u * BLOCK < n4;
      float* e = reinterpret_cast<float*>(&v[u]);
#pragma unroll
      for (int c = 0; c < 4; c++) {
        bool ok;
        xin[4 * u + c] = e[c];
        e[c] = Op::fast(e[c], tab, ok);
        fail |= (unsigned)(live && (!ok || force)) << (4 * u + c);
      }
    }
    if (fail) {
#pragma unroll
      for (int u = 0; u < U; u++) {
        float* e = reinterpret_cast<float*>(&v[u]);
#pragma unroll
        for (int c = 0; c < 4; c++) {
          if (fail & (1u << (4 * u + c))) {
            const long long i = base + (long long)u * BLOCK;
            const float x = xin[4 * u + c];
            unsigned pos = atomicAdd(&q.n, 1u);
            if (pos < QCAP) {
              q.idx[pos] = (unsigned)(4 * i + c);
              q.x[pos] = x;
            } else {  // queue full (only with pathological inputs or force)
              AccResult a = Op::accurate(x, tab);
              e[c] = a.r;
              atomicAdd(&q.lanes, 1u);
              if (!a.ok) note_escape(st, elem_base + 4 * i + c);
            }
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      long long i = base + (long long)u * BLOCK;
      if (i < n4) st_stream(out + i, v[u]);
    }
    if (iter % Op::qcheck == Op::qcheck - 1) {
      // every thread must see the same fill level: read it between two
      // barriers (no thread can queue more elements before all have read it)
      __syncthreads();
      const unsigned nq = q.n;
      __syncthreads();
      if (nq > QFLUSH) flush_queue<Op>(q, tab, outf, st, elem_base);
    }
  }
  __syncthreads();
  flush_queue<Op, true>(q, tab, outf, st, elem_base);
}

// Scalar form for unaligned heads, ragged tails and pointers whose alignment
// differs; the accurate path runs in place.
template <class Op>
__global__ void __launch_bounds__(BLOCK)
    k_map_f32_scalar(const float* in, float* out, long long n, DevStats* st,
                     unsigned flags, long long elem_base) {
  __shared__ typename Op::Tab tab;
  Op::load(tab, threadIdx.x);
  __syncthreads();
  const bool force = flags & CR_FLAG_FORCE_FALLBACK;
  unsigned lanes = 0;
  for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n;
       i += (long long)gridDim.x * BLOCK) {
    bool ok;
    float x = in[i];
    float r = Op::fast(x, tab, ok);
    if (!ok || force) {
      AccResult a = Op::accurate(x, tab);
      r = a.r;
      lanes++;
      if (!a.ok) note_escape(st, elem_base + i);
    }
    out[i] = r;
  }
  if (lanes) {
    CounterSlot& c = st->slot[blockIdx.x % NSLOT];
    atomicAdd(&c.fallback_lanes, (unsigned long long)lanes);
    atomicAdd(&c.fallback_waves, 1ull);
  }
}

// sincosf: the map kernel with two planar outputs (sin block, cos block); the
// input and the sine block 16-byte aligned (the host checks; otherwise the
// scalar form below runs).
template <class SC, bool FINAL = false>
__device__ __forceinline__ void flush_queue_sincos(Deferred& q, const typename SC::Tab& tab,
                                                   float* os, float* oc, DevStats* st,
                                                   long long elem_base) {
  run_queue<FINAL>(q, st, [&](unsigned k) {
    AccResult2 a = SC::accurate(q.x[k], tab);
    os[q.idx[k]] = a.s;
    oc[q.idx[k]] = a.c;
    if (!a.ok) note_escape(st, elem_base + q.idx[k]);
  });
}

// CVEC: the cosine block is 16-byte aligned as well (n a multiple of 4);
// otherwise its four values per vector are stored one by one (still
// contiguous across the lanes of a wave).
template <class SC, bool CVEC>
__global__ void __launch_bounds__(BLOCK)
    k_map_sincos(const float4* in, float4* outs, float* outc, long long n4, DevStats* st,
                 unsigned flags, long long elem_base) {
  __shared__ typename SC::Tab tab;
  __shared__ Deferred q;
  SC::load(tab, threadIdx.x);
  if (threadIdx.x == 0) {
    q.n = 0;
    q.lanes = q.waves = 0;
  }
  __syncthreads();
  const bool force = flags & CR_FLAG_FORCE_FALLBACK;
  const long long ntiles = (n4 + BLOCK * TILE_U - 1) / (BLOCK * TILE_U);
  int iter = 0;
  for (long long t = blockIdx.x; t < ntiles; t += gridDim.x, iter++) {
    long long base = t * (BLOCK * TILE_U) + threadIdx.x;
    float4 v[TILE_U], c4[TILE_U];
#pragma unroll
    for (int u = 0; u < TILE_U; u++) {
      long long i = base + (long long)u * BLOCK;
      if (i < n4) v[u] = ld_stream(in + i);
    }
#pragma unroll
    for (int u = 0; u < TILE_U; u++) {
      long long i = base + (long long)u * BLOCK;
      if (i < n4) {
        float* e = reinterpret_cast<float*>(&v[u]);
        float* ec = reinterpret_cast<float*>(&c4[u]);
#pragma unroll
        for (int c = 0; c < 4; c++) {
          bool ok;
          float x = e[c];
          e[c] = SC::fast(x, tab, ec[c], ok);
          if (!ok || force) {
            unsigned pos = atomicAdd(&q.n, 1u);
            if (pos < QCAP) {
              q.idx[pos] = (unsigned)(4 * i + c);
              q.x[pos] = x;
            } else {
              AccResult2 a = SC::accurate(x, tab);
              e[c] = a.s;
              ec[c] = a.c;
              atomicAdd(&q.lanes, 1u);
              if (!a.ok) note_escape(st, elem_base + 4 * i + c);
            }
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < TILE_U; u++) {
      long long i = base + (long long)u * BLOCK;
      if (i < n4) {
        st_stream(outs + i, v[u]);
        if (CVEC) {
          st_stream(reinterpret_cast<float4*>(outc) + i, c4[u]);
        } else {
          float* p = outc + 4 * i;
          p[0] = c4[u].x;
          p[1] = c4[u].y;
          p[2] = c4[u].z;
          p[3] = c4[u].w;
        }
      }
    }
    if (iter % SC::qcheck == SC::qcheck - 1) {
      __syncthreads();
      const unsigned nq = q.n;
      __syncthreads();
      if (nq > QFLUSH)
        flush_queue_sincos<SC>(q, tab, reinterpret_cast<float*>(outs), outc, st, elem_base);
    }
  }
  __syncthreads();
  flush_queue_sincos<SC, true>(q, tab, reinterpret_cast<float*>(outs), outc, st, elem_base);
}

template <class SC>
__global__ void __launch_bounds__(BLOCK)
    k_map_sincos_scalar(const float* in, float* outs, float* outc, long long n, DevStats* st,
                        unsigned flags, long long elem_base) {
  __shared__ typename SC::Tab tab;
  SC::load(tab, threadIdx.x);
  __syncthreads();
  const bool force = flags & CR_FLAG_FORCE_FALLBACK;
  unsigned lanes = 0;
  for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n;
       i += (long long)gridDim.x * BLOCK) {
    bool ok;
    float x = in[i], c;
    float s = SC::fast(x, tab, c, ok);
    if (!ok || force) {
      AccResult2 a = SC::accurate(x, tab);
      s = a.s;
      c = a.c;
      lanes++;
      if (!a.ok) note_escape(st, elem_base + i);
    }
    outs[i] = s;
    outc[i] = c;
  }
  if (lanes) {
    CounterSlot& c = st->slot[blockIdx.x % NSLOT];
    atomicAdd(&c.fallback_lanes, (unsigned long long)lanes);
    atomicAdd(&c.fallback_waves, 1ull);
  }
}

// ------------------------------------------------------------ binary64 map
struct OpExp64 {
  using Tab = Exp64Tab;
  static constexpr int qcheck = QCHECK;
  static __device__ __forceinline__ void load(Tab& t, int tid) { exp64_tab_load(t, tid); }
  static __device__ __forceinline__ double fast(double x, const Tab& t, bool& ok) {
    return exp64_fast(x, t, ok);
  }
  static __device__ __forceinline__ AccResultD accurate(double x, const Tab& t) {
    return exp64_accurate(x, t);
  }
};
struct OpLog64 {
  using Tab = Log64Tab;
  static constexpr int qcheck = QCHECK;
  static __device__ __forceinline__ void load(Tab& t, int tid) { log64_tab_load(t, tid); }
  static __device__ __forceinline__ double fast(double x, const Tab& t, bool& ok) {
    return log64_fast(x, t, ok);
  }
  static __device__ __forceinline__ AccResultD accurate(double x, const Tab& t) {
    return log64_accurate(x, t);
  }
};

// binary64 log with the paper's 128-entry scaled-integer table (main path);
// lanes that fail its test take the 16-entry accurate path
struct OpLog128 {
  using Tab = Log128Tab;
  static constexpr int qcheck = QCHECK;
  static __device__ __forceinline__ void load(Tab& t, int tid) { log128_tab_load(t, tid); }
  static __device__ __forceinline__ double fast(double x, const Tab& t, bool& ok) {
    return log128_fast(x, t, ok);
  }
  static __device__ __forceinline__ AccResultD accurate(double x, const Tab& t) {
    return log64_accurate(x, t.acc);
  }
};
struct OpExp2_64 {
  using Tab = Exp2_64Tab;
  static constexpr int qcheck = QCHECK;
  static __device__ __forceinline__ void load(Tab& t, int tid) { exp2_64_tab_load(t, tid); }
  static __device__ __forceinline__ double fast(double x, const Tab& t, bool& ok) {
    return exp2_64_fast(x, t, ok);
  }
  static __device__ __forceinline__ AccResultD accurate(double x, const Tab& t) {
    return exp2_64_accurate(x, t);
  }
};

struct Deferred64 {
  unsigned n, lanes, waves;
  unsigned idx[QCAP];
  double x[QCAP];
};

template <class Op, bool FINAL = false>
__device__ __forceinline__ void flush_queue64(Deferred64& q, const typename Op::Tab& tab,
                                              double* out, DevStats* st, long long elem_base) {
  run_queue<FINAL>(q, st, [&](unsigned k) {
    AccResultD a = Op::accurate(q.x[k], tab);
    out[q.idx[k]] = a.r;
    if (!a.ok) note_escape(st, elem_base + q.idx[k]);
  });
}

// The binary64 form of k_map_f32: tiles of BLOCK U double2 vectors (U per
// thread).  Launch-shape variants (chosen per function by the autotuner):
//   SL 0: each element is evaluated and, if its test fails, queued before the
//         next one (a branch between elements),
//   SL 1: as in k_map_f32, every element of the tile is evaluated in
//         straight-line code first (the scheduler interleaves their
//         dependency chains) and the failing ones are queued afterwards.
template <class Op, int U, int SL>
__global__ void __launch_bounds__(BLOCK)
    k_map_f64(const double2* in, double2* out, long long n2, DevStats* st, unsigned flags,
              long long elem_base) {
  __shared__ typename Op::Tab tab;
  __shared__ Deferred64 q;
  Op::load(tab, threadIdx.x);
  if (threadIdx.x == 0) {
    q.n = 0;
    q.lanes = q.waves = 0;
  }
  __syncthreads();
  const bool force = flags & CR_FLAG_FORCE_FALLBACK;
  double* outd = reinterpret_cast<double*>(out);
  const long long ntiles = (n2 + BLOCK * U - 1) / (BLOCK * U);
  // queue element j (index 2 i + c of this launch) with input x, or run its
  // accurate path in place when the queue is full
  auto enqueue = [&](long long j, double x, double& res) {
    unsigned pos = atomicAdd(&q.n, 1u);
    if (pos < QCAP) {
      q.idx[pos] = (unsigned)j;
      q.x[pos] = x;
    } else {
      AccResultD a = Op::accurate(x, tab);
      res = a.r;
      atomicAdd(&q.lanes, 1u);
      if (!a.ok) note_escape(st, elem_base + j);
    }
  };
  int iter = 0;
  for (long long t = blockIdx.x; t < ntiles; t += gridDim.x, iter++) {
    long long base = t * (BLOCK * U) + threadIdx.x;
    double2 v[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      long long i = base + (long long)u * BLOCK;
      v[u] = i < n2 ? ld_stream(in + i) : make_double2(1.0, 1.0);
    }
    if (SL) {
      // slots past the end hold 1.0: evaluated, never stored or queued
      double xin[2 * U];
      unsigned fail = 0;
#pragma unroll
      for (int u = 0; u < U; u++) {
        const bool live = base + (long long)u * BLOCK < n2;
        double* e = reinterpret_cast<double*>(&v[u]);
#pragma unroll
        for (int c = 0; c < 2; c++) {
          bool ok;
          xin[2 * u + c] = e[c];
          e[c] = Op::fast(e[c], tab, ok);
          fail |= (unsigned)(live && (!ok || force)) << (2 * u + c);
        }
      }
      if (fail) {
#pragma unroll
        for (int u = 0; u < U; u++) {
          double* e = reinterpret_cast<double*>(&v[u]);
          const long long i = base + (long long)u * BLOCK;
#pragma unroll
          for (int c = 0; c < 2; c++)
            if ((fail >> (2 * u + c)) & 1u) enqueue(2 * i + c, xin[2 * u + c], e[c]);
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; u++) {
        long long i = base + (long long)u * BLOCK;
        if (i < n2) {
          double* e = reinterpret_cast<double*>(&v[u]);
#pragma unroll
          for (int c = 0; c < 2; c++) {
            bool ok;
            double x = e[c];
            e[c] = Op::fast(x, tab, ok);
            if (!ok || force) enqueue(2 * i + c, x, e[c]);
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      long long i = base + (long long)u * BLOCK;
      if (i < n2) st_stream(out + i, v[u]);
    }
    if (iter % Op::qcheck == Op::qcheck - 1) {
      __syncthreads();
      const unsigned nq = q.n;
      __syncthreads();
      if (nq > QFLUSH) flush_queue64<Op>(q, tab, outd, st, elem_base);
    }
  }
  __syncthreads();
  flush_queue64<Op, true>(q, tab, outd, st, elem_base);
}

template <class Op>
__global__ void __launch_bounds__(BLOCK)
    k_map_f64_scalar(const double* in, double* out, long long n, DevStats* st, unsigned flags,
                     long long elem_base) {
  __shared__ typename Op::Tab tab;
  Op::load(tab, threadIdx.x);
  __syncthreads();
  const bool force = flags & CR_FLAG_FORCE_FALLBACK;
  unsigned lanes = 0;
  for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n;
       i += (long long)gridDim.x * BLOCK) {
    bool ok;
    double x = in[i];
    double r = Op::fast(x, tab, ok);
    if (!ok || force) {
      AccResultD a = Op::accurate(x, tab);
      r = a.r;
      lanes++;
      if (!a.ok) note_escape(st, elem_base + i);
    }
    out[i] = r;
  }
  if (lanes) {
    CounterSlot& c = st->slot[blockIdx.x % NSLOT];
    atomicAdd(&c.fallback_lanes, (unsigned long long)lanes);
    atomicAdd(&c.fallback_waves, 1ull);
  }
}

// ------------------------------------------------- directed rounding modes
// Every element through the function's ~2^-100 double-double evaluation with
// both ends of its error interval rounded in the mode RM (cr_f32_dir.h); the
// paper's GPU runs leave these modes out (Sec. III-C).  A grid-stride map with
// the tables in LDS; each element counts as an accurate-path lane.
template <class Op, int RM>
__global__ void __launch_bounds__(BLOCK)
    k_map_f32_dir(const float* in, float* out, long long n, DevStats* st, long long elem_base) {
  __shared__ typename Op::Tab tab;
  Op::load(tab, threadIdx.x);
  __syncthreads();
  unsigned lanes = 0;
  for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n;
       i += (long long)gridDim.x * BLOCK) {
    AccResult a = Op::template dir<RM>(in[i], tab);
    out[i] = a.r;
    lanes++;
    if (!a.ok) note_escape(st, elem_base + i);
  }
  if (lanes) {
    CounterSlot& c = st->slot[blockIdx.x % NSLOT];
    atomicAdd(&c.fallback_lanes, (unsigned long long)lanes);
    atomicAdd(&c.fallback_waves, 1ull);
  }
}

template <class SC, int RM>
__global__ void __launch_bounds__(BLOCK)
    k_sincos_dir(const float* in, float* outs, float* outc, long long n, DevStats* st,
                 long long elem_base) {
  __shared__ typename SC::Tab tab;
  SC::load(tab, threadIdx.x);
  __syncthreads();
  unsigned lanes = 0;
  for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n;
       i += (long long)gridDim.x * BLOCK) {
    AccResult2 a = SC::template dir<RM>(in[i], tab);
    outs[i] = a.s;
    outc[i] = a.c;
    lanes++;
    if (!a.ok) note_escape(st, elem_base + i);
  }
  if (lanes) {
    CounterSlot& c = st->slot[blockIdx.x % NSLOT];
    atomicAdd(&c.fallback_lanes, (unsigned long long)lanes);
    atomicAdd(&c.fallback_waves, 1ull);
  }
}

// ------------------------------------------------- application workloads
// The paper's two synthetic applications built on the correctly rounded
// binary32 functions (Sec. III-A): complex expf, logf and sinf accurate to
// 2 ulps, and spectral interpolation by a brute-force DFT that spends its time
// in sincosf.  Each correctly rounded ingredient is evaluated by its fast path
// and, in a lane whose rounding test fails (rare on these workloads: no
// hard-to-round inputs are planted), by its accurate path in place; the steps
// between them are single IEEE operations in the stated formats.

// One binary32 function, correctly rounded: fast path, accurate path if needed.
struct LaneCount {
  unsigned fails;
  unsigned escapes;
};
template <class Op>
__device__ __forceinline__ float cr1(float x, const typename Op::Tab& t, bool force, LaneCount& lc) {
  bool ok;
  float r = Op::fast(x, t, ok);
  if (!ok || force) {
    AccResult a = Op::accurate(x, t);
    r = a.r;
    lc.fails++;
    lc.escapes += a.ok ? 0u : 1u;
  }
  return r;
}
__device__ __forceinline__ float cr_sincos(float x, const TrigTab& t, float& c, bool force,
                                           LaneCount& lc) {
  bool ok;
  float s = sincos_fast(x, t, c, ok);
  if (!ok || force) {
    AccResult2 a = sincos_accurate(x, t);
    s = a.s;
    c = a.c;
    lc.fails++;
    lc.escapes += a.ok ? 0u : 1u;
  }
  return s;
}

// exp(x + iy) = e^x cos y + i e^x sin y: re = RN32(expf(x) cosf(y)),
// im = RN32(expf(x) sinf(y)).  Each part is the correctly rounded product of
// two correctly rounded factors: within 2 ulps.
struct CExpF {
  struct Tab {
    ExpTab e;
    TrigTab t;
  };
  static __device__ __forceinline__ void load(Tab& T, int tid) {
    exp_tab_load(T.e, tid);
    trig_tab_load(T.t, tid);
  }
  static __device__ __forceinline__ float2 eval(float x, float y, const Tab& T, bool force,
                                                LaneCount& lc) {
    const float E = cr1<OpExp<EXPK_E>>(x, T.e, force, lc);
    float C;
    const float S = cr_sincos(y, T.t, C, force, lc);
    return make_float2(E * C, E * S);
  }
};

// sin(x + iy) = sin x cosh y + i cos x sinh y, each product of correctly
// rounded factors rounded once: within 2 ulps.
struct CSinF {
  struct Tab {
    ExpTab e;
    TrigTab t;
  };
  static __device__ __forceinline__ void load(Tab& T, int tid) {
    exp_tab_load(T.e, tid);
    trig_tab_load(T.t, tid);
  }
  static __device__ __forceinline__ float2 eval(float x, float y, const Tab& T, bool force,
                                                LaneCount& lc) {
    float C;
    const float S = cr_sincos(x, T.t, C, force, lc);
    const float Ch = cr1<OpHyp<HYPK_COSH>>(y, T.e, force, lc);
    const float Sh = cr1<OpHyp<HYPK_SINH>>(y, T.e, force, lc);
    return make_float2(S * Ch, C * Sh);
  }
};

// log(x + iy) = log|z| + i atan2(y, x), valid for finite z with
// 2^-63 <= |z| < 2^63.  With a = max(|x|, |y|), b = min(|x|, |y|):
//  * imaginary part: A = atanf(RN32(b / a)) correctly rounded, then in
//    binary64 v = A, v = RN64(pi/2) - v if |y| > |x|, v = RN64(pi) - v if
//    x < 0; the result is RN32(v) with the sign of y (below 1.5 ulps: the
//    quotient's rounding moves atan by at most 2^-24 t/(1 + t^2));
//  * real part: s = RN64(a^2 + b^2) (the squares are exact in binary64).
//    For 0.5 <= s < 2, d = RN64((a^2 - 1) + b^2) (a^2 - 1 exact), d = dh + dl
//    with dh = RN32(d) and dl exact, and log|z| = (log1pf(dh) + dl/(1 + dh))/2;
//    otherwise s = sh + sl, sh = RN32(s), and log|z| = (logf(sh) + sl/sh)/2,
//    the correction term's second-order error being below 2^-46 relative:
//    below 1.5 ulps.
struct CLogF {
  struct Tab {
    AtanTab a;
    LogTab l;
  };
  static __device__ __forceinline__ void load(Tab& T, int tid) {
    atan_tab_load(T.a, tid);
    log_tab_load<LOGK_E>(T.l, tid);  // logf and log1pf share the natural-log table
  }
  static __device__ __forceinline__ float2 eval(float x, float y, const Tab& T, bool force,
                                                LaneCount& lc) {
    const float ax = fabsf(x), ay = fabsf(y);
    const float a = fmaxf(ax, ay), b = fminf(ax, ay);
    const float A = cr1<OpAtan<ATANK_ATAN>>(b / a, T.a, force, lc);
    double v = (double)A;
    if (ay > ax) v = 0x1.921fb54442d18p+0 - v;  // RN64(pi/2) - v
    if (x < 0.0f) v = 0x1.921fb54442d18p+1 - v;  // RN64(pi) - v
    const float im = copysignf((float)v, y);
    const double a2 = (double)a * (double)a, b2 = (double)b * (double)b;
    const double s = a2 + b2;
    double re;
    if (s >= 0.5 && s < 2.0) {
      const double d = (a2 - 1.0) + b2;
      const float dh = (float)d;
      const double dl = d - (double)dh;
      const float L = cr1<OpLog<LOGK_1P>>(dh, T.l, force, lc);
      re = 0.5 * ((double)L + dl / (1.0 + (double)dh));
    } else {
      const float sh = (float)s;
      const double sl = s - (double)sh;
      const float L = cr1<OpLog<LOGK_E>>(sh, T.l, force, lc);
      re = 0.5 * ((double)L + sl / (double)sh);
    }
    return make_float2((float)re, im);
  }
};

// Complex map: interleaved (re, im) binary32 pairs, two complex numbers per
// 128-bit load and store.  Persistent grid, tables staged in LDS.
template <class CF>
__global__ void __launch_bounds__(BLOCK)
    k_complex(const float4* in, float4* out, long long n2, DevStats* st, unsigned flags,
              long long elem_base) {
  __shared__ typename CF::Tab tab;
  __shared__ unsigned fails;
  CF::load(tab, threadIdx.x);
  if (threadIdx.x == 0) fails = 0;
  __syncthreads();
  const bool force = flags & CR_FLAG_FORCE_FALLBACK;
  LaneCount tot = {0u, 0u};
  for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n2;
       i += (long long)gridDim.x * BLOCK) {
    const float4 v = ld_stream(in + i);
    LaneCount lc = {0u, 0u};
    const float2 r0 = CF::eval(v.x, v.y, tab, force, lc);
    if (lc.escapes) note_escape(st, elem_base + 2 * i);
    tot.fails += lc.fails;
    lc = {0u, 0u};
    const float2 r1 = CF::eval(v.z, v.w, tab, force, lc);
    if (lc.escapes) note_escape(st, elem_base + 2 * i + 1);
    tot.fails += lc.fails;
    st_stream(out + i, make_float4(r0.x, r0.y, r1.x, r1.y));
  }
  if (tot.fails) atomicAdd(&fails, tot.fails);
  __syncthreads();
  if (threadIdx.x == 0 && fails) {
    CounterSlot& c = st->slot[blockIdx.x % NSLOT];
    atomicAdd(&c.fallback_lanes, (unsigned long long)fails);
    atomicAdd(&c.fallback_waves, 1ull);
  }
}

// Scalar form for unaligned buffers and a ragged last element (4-byte loads).
template <class CF>
__global__ void __launch_bounds__(BLOCK)
    k_complex_scalar(const float* in, float* out, long long n, DevStats* st, unsigned flags,
                     long long elem_base) {
  __shared__ typename CF::Tab tab;
  CF::load(tab, threadIdx.x);
  __syncthreads();
  const bool force = flags & CR_FLAG_FORCE_FALLBACK;
  unsigned fails = 0;
  for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n;
       i += (long long)gridDim.x * BLOCK) {
    LaneCount lc = {0u, 0u};
    const float2 r = CF::eval(in[2 * i], in[2 * i + 1], tab, force, lc);
    if (lc.escapes) note_escape(st, elem_base + i);
    fails += lc.fails;
    out[2 * i] = r.x;
    out[2 * i + 1] = r.y;
  }
  if (fails) {
    CounterSlot& c = st->slot[blockIdx.x % NSLOT];
    atomicAdd(&c.fallback_lanes, (unsigned long long)fails);
    atomicAdd(&c.fallback_waves, 1ull);
  }
}

// Brute-force DFT of real samples at per-output angles (spectral
// interpolation): X_k = sum_n x[n] (cos t - i sin t), t = RN32(w_k n), with
// sincosf correctly rounded.  Each product x[n] cos t is exact in binary64;
// the sums are carried as double-doubles (TwoSum per term), so X_k is within
// about N 2^-104 sum |x c| of the exact sum of the exact products before its
// final rounding.  Block (s, k) covers samples [s L, (s + 1) L) of output k
// and writes its partial sums (re.hi, re.lo, im.hi, im.lo); a second kernel
// adds the S partials of each k in a fixed order, so results do not depend
// on timing.
__device__ __forceinline__ void dd_acc(double& hi, double& lo, double p) {
  const dd t = two_sum(hi, p);
  hi = t.hi;
  lo += t.lo;
}
__device__ __forceinline__ void dd_acc2(double& hi, double& lo, double h2, double l2) {
  const dd t = two_sum(hi, h2);
  const dd u = fast_two_sum(t.hi, t.lo + (lo + l2));
  hi = u.hi;
  lo = u.lo;
}

__global__ void __launch_bounds__(BLOCK)
    k_dft(const float* x, long long n, const float* w, long long slice, double4* part, int S,
          DevStats* st, unsigned flags, long long k0) {
  __shared__ TrigTab tab;
  __shared__ double4 red[BLOCK / 64];
  __shared__ unsigned fails;
  trig_tab_load(tab, threadIdx.x);
  if (threadIdx.x == 0) fails = 0;
  __syncthreads();
  const bool force = flags & CR_FLAG_FORCE_FALLBACK;
  const long long k = blockIdx.y;
  const float wk = w[k];
  const long long n0 = (long long)blockIdx.x * slice;
  const long long n1 = n0 + slice < n ? n0 + slice : n;
  double rh = 0.0, rl = 0.0, ih = 0.0, il = 0.0;
  LaneCount lc = {0u, 0u};
  for (long long i = n0 + threadIdx.x; i < n1; i += BLOCK) {
    const float th = wk * (float)i;  // RN32(w_k n), n < 2^24 exact
    float c;
    const float s = cr_sincos(th, tab, c, force, lc);
    const double xd = (double)x[i];
    dd_acc(rh, rl, xd * (double)c);
    dd_acc(ih, il, xd * (double)s);
  }
  if (lc.escapes) note_escape(st, k0 + k);
  // wave reduction in a fixed order (xor butterfly), then across the 4 waves
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double a = __shfl_xor(rh, off), b = __shfl_xor(rl, off);
    const double c = __shfl_xor(ih, off), d = __shfl_xor(il, off);
    dd_acc2(rh, rl, a, b);
    dd_acc2(ih, il, c, d);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = make_double4(rh, rl, ih, il);
  if (lc.fails) atomicAdd(&fails, lc.fails);
  __syncthreads();
  if (threadIdx.x == 0) {
    double4 acc = red[0];
    for (int q = 1; q < BLOCK / 64; q++) {
      dd_acc2(acc.x, acc.y, red[q].x, red[q].y);
      dd_acc2(acc.z, acc.w, red[q].z, red[q].w);
    }
    part[k * S + blockIdx.x] = acc;
    if (fails) {
      CounterSlot& cs = st->slot[(blockIdx.y * gridDim.x + blockIdx.x) % NSLOT];
      atomicAdd(&cs.fallback_lanes, (unsigned long long)fails);
      atomicAdd(&cs.fallback_waves, 1ull);
    }
  }
}

__global__ void __launch_bounds__(BLOCK)
    k_dft_finish(const double4* part, int S, long long m, double2* X) {
  const long long k = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (k >= m) return;
  double4 acc = part[k * S];
  for (int q = 1; q < S; q++) {
    const double4 p = part[k * S + q];
    dd_acc2(acc.x, acc.y, p.x, p.y);
    dd_acc2(acc.z, acc.w, p.z, p.w);
  }
  X[k] = make_double2(acc.x + acc.y, -(acc.z + acc.w));
}

// ------------------------------------------------------------ ragged batch
// One persistent kernel evaluates a whole plan: a request table (function,
// pointers, length) and a tile table (request, start, count; tiles of TILE
// elements).  Each workgroup walks a contiguous range of tiles; requests are
// ordered by function when the plan is built, so consecutive tiles mostly
// share a function and its LDS table, which is reloaded only when the
// function changes.  The function switch is per tile, hence wave-uniform.
struct BReq {
  const void* in;
  void* out;
  long long n;
  int func;
  int aligned;  // in and out (and the cos block for sincosf) are 16-byte aligned
  int key;      // func + BSPLIT for the binary32-only implementation
  int orig;     // index of the request in the caller's array
};
constexpr int BSPLIT = 32;
struct BTile {
  int req;
  int count;
  long long start;
};

// Static device memory of the library.  Each device the library runs on holds
// its own copy, zero-initialised when the code object loads, until the
// process ends.  Host code never passes these names to a kernel or a copy
// (in host code they are host-side stand-ins): get_state() resolves their
// per-device addresses with hipGetSymbolAddress.
//   g_dev_stats  the statistics counters and escape list of every entry point
//   scratch      the request and tile tables of cr_eval_batch_noalloc:
//                CR_NOALLOC_MAX_REQUESTS BReq, then CR_NOALLOC_MAX_TILES BTile
__device__ __align__(256) DevStats g_dev_stats;
constexpr size_t NOALLOC_REQ_BYTES =
    ((size_t)CR_NOALLOC_MAX_REQUESTS * sizeof(BReq) + 255) / 256 * 256;
constexpr size_t SCRATCH_BYTES = NOALLOC_REQ_BYTES + (size_t)CR_NOALLOC_MAX_TILES * sizeof(BTile);
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

struct BDeferred {
  unsigned n, lanes, waves;
  unsigned req[QCAP];
  unsigned idx[QCAP];
  float x[QCAP];
};

// Escapes of a batch are recorded as (request << 32) | element index within
// the request.
__device__ __forceinline__ long long batch_escape_id(unsigned req, unsigned idx) {
  return (long long)(((unsigned long long)req << 32) | idx);
}

template <class Op>
__device__ __forceinline__ void batch_enqueue(BDeferred& q, const typename Op::Tab& tab,
                                              unsigned req, unsigned orig, unsigned idx, float x,
                                              float& res, DevStats* st) {
  unsigned pos = atomicAdd(&q.n, 1u);
  if (pos < QCAP) {
    q.req[pos] = req;
    q.idx[pos] = idx;
    q.x[pos] = x;
  } else {
    AccResult a = Op::accurate(x, tab);
    res = a.r;
    atomicAdd(&q.lanes, 1u);
    if (!a.ok) note_escape(st, batch_escape_id(orig, idx));
  }
}

template <class Op>
__device__ __forceinline__ void batch_tile(BReq R, BTile T, const typename Op::Tab& tab,
                                        BDeferred& q, bool force, DevStats* st) {
  const float* in = reinterpret_cast<const float*>(R.in) + T.start;
  float* out = reinterpret_cast<float*>(R.out) + T.start;
  const int cnt = T.count;
  const unsigned base = (unsigned)T.start;
  if (R.aligned) {
    const int n4 = cnt >> 2;
#pragma unroll
    for (int u = 0; u < BATCH_U; u++) {
      int i = threadIdx.x + u * BLOCK;
      if (i < n4) {
        float4 v = ld_stream(reinterpret_cast<const float4*>(in) + i);
        float* e = reinterpret_cast<float*>(&v);
#pragma unroll
        for (int c = 0; c < 4; c++) {
          bool ok;
          float x = e[c];
          e[c] = Op::fast(x, tab, ok);
          if (!ok || force)
            batch_enqueue<Op>(q, tab, T.req, R.orig, base + 4 * i + c, x, e[c], st);
        }
        st_stream(reinterpret_cast<float4*>(out) + i, v);
      }
    }
    int i = 4 * n4 + threadIdx.x;
    if (i < cnt) {
      bool ok;
      float x = in[i];
      float r = Op::fast(x, tab, ok);
      if (!ok || force) batch_enqueue<Op>(q, tab, T.req, R.orig, base + i, x, r, st);
      out[i] = r;
    }
  } else {
    for (int i = threadIdx.x; i < cnt; i += BLOCK) {
      bool ok;
      float x = in[i];
      float r = Op::fast(x, tab, ok);
      if (!ok || force) batch_enqueue<Op>(q, tab, T.req, R.orig, base + i, x, r, st);
      out[i] = r;
    }
  }
}

template <class SC>
__device__ __forceinline__ void batch_tile_sincos(BReq R, BTile T, const typename SC::Tab& tab,
                                               BDeferred& q, bool force, DevStats* st) {
  const float* in = reinterpret_cast<const float*>(R.in) + T.start;
  float* os = reinterpret_cast<float*>(R.out) + T.start;
  float* oc = reinterpret_cast<float*>(R.out) + R.n + T.start;
  const int cnt = T.count;
  const unsigned base = (unsigned)T.start;
  // one element: fast path, queue or accurate path in place
  auto one = [&](int i, float x, float& sv, float& c) {
    bool ok;
    sv = SC::fast(x, tab, c, ok);
    if (!ok || force) {
      unsigned pos = atomicAdd(&q.n, 1u);
      if (pos < QCAP) {
        q.req[pos] = T.req;
        q.idx[pos] = base + i;
        q.x[pos] = x;
      } else {
        AccResult2 a = SC::accurate(x, tab);
        sv = a.s;
        c = a.c;
        atomicAdd(&q.lanes, 1u);
        if (!a.ok) note_escape(st, batch_escape_id(R.orig, base + i));
      }
    }
  };
  int i0 = 0;
  if (R.aligned) {  // input, sine block and cosine block 16-byte aligned
    const int n4 = cnt >> 2;
#pragma unroll
    for (int u = 0; u < BATCH_U; u++) {
      int i = threadIdx.x + u * BLOCK;
      if (i < n4) {
        float4 v = ld_stream(reinterpret_cast<const float4*>(in) + i), cv;
        float* e = reinterpret_cast<float*>(&v);
        float* ec = reinterpret_cast<float*>(&cv);
#pragma unroll
        for (int c = 0; c < 4; c++) one(4 * i + c, e[c], e[c], ec[c]);
        st_stream(reinterpret_cast<float4*>(os) + i, v);
        st_stream(reinterpret_cast<float4*>(oc) + i, cv);
      }
    }
    i0 = 4 * n4;
  }
  for (int i = i0 + threadIdx.x; i < cnt; i += BLOCK) {
    float sv, c;
    one(i, in[i], sv, c);
    os[i] = sv;
    oc[i] = c;
  }
}

// Run the accurate path on the queued elements (see run_queue).
template <class Op, bool FINAL = false>
__device__ __forceinline__ void batch_flush_one(BDeferred& q, const typename Op::Tab& tab,
                                                const BReq* reqs, DevStats* st) {
  run_queue<FINAL>(q, st, [&](unsigned k) {
    AccResult a = Op::accurate(q.x[k], tab);
    float* out = reinterpret_cast<float*>(reqs[q.req[k]].out);
    out[q.idx[k]] = a.r;
    if (!a.ok) note_escape(st, batch_escape_id(reqs[q.req[k]].orig, q.idx[k]));
  });
}

template <class SC, bool FINAL = false>
__device__ __forceinline__ void batch_flush_one_sincos(BDeferred& q, const typename SC::Tab& tab,
                                                       const BReq* reqs, DevStats* st) {
  run_queue<FINAL>(q, st, [&](unsigned k) {
    AccResult2 a = SC::accurate(q.x[k], tab);
    const BReq& R = reqs[q.req[k]];
    float* out = reinterpret_cast<float*>(R.out);
    out[q.idx[k]] = a.s;
    out[R.n + q.idx[k]] = a.c;
    if (!a.ok) note_escape(st, batch_escape_id(reqs[q.req[k]].orig, q.idx[k]));
  });
}

// The batch runs one persistent kernel per function present (implementation
// and function: the tiles are sorted by both), all captured in the plan's one
// graph and run back to back.  Each kernel is specialised on its function, so
// it keeps only that function's tables in LDS and only that function's
// registers (one kernel over all functions would run every function at the
// occupancy of the largest).  Workgroup b takes tiles t0 + b, t0 + b + grid,
// ... of its function's contiguous range [t0, t1).
template <class Op>
__global__ void __launch_bounds__(BLOCK)
    k_tiles(const BReq* reqs, const BTile* tiles, long long t0, long long t1, DevStats* st,
            unsigned flags) {
  __shared__ typename Op::Tab tab;
  __shared__ BDeferred q;
  Op::load(tab, threadIdx.x);
  if (threadIdx.x == 0) {
    q.n = 0;
    q.lanes = q.waves = 0;
  }
  __syncthreads();
  const bool force = flags & CR_FLAG_FORCE_FALLBACK;
  int iter = 0;
  for (long long t = t0 + blockIdx.x; t < t1; t += gridDim.x, iter++) {
    const BTile T = tiles[t];
    batch_tile<Op>(reqs[T.req], T, tab, q, force, st);
    if (iter % Op::qcheck == Op::qcheck - 1) {
      __syncthreads();
      const unsigned nq = q.n;
      __syncthreads();
      if (nq > QFLUSH) batch_flush_one<Op>(q, tab, reqs, st);
    }
  }
  __syncthreads();
  batch_flush_one<Op, true>(q, tab, reqs, st);
}

template <class SC>
__global__ void __launch_bounds__(BLOCK)
    k_tiles_sincos(const BReq* reqs, const BTile* tiles, long long t0, long long t1,
                   DevStats* st, unsigned flags) {
  __shared__ typename SC::Tab tab;
  __shared__ BDeferred q;
  SC::load(tab, threadIdx.x);
  if (threadIdx.x == 0) {
    q.n = 0;
    q.lanes = q.waves = 0;
  }
  __syncthreads();
  const bool force = flags & CR_FLAG_FORCE_FALLBACK;
  int iter = 0;
  for (long long t = t0 + blockIdx.x; t < t1; t += gridDim.x, iter++) {
    const BTile T = tiles[t];
    batch_tile_sincos<SC>(reqs[T.req], T, tab, q, force, st);
    if (iter % SC::qcheck == SC::qcheck - 1) {
      __syncthreads();
      const unsigned nq = q.n;
      __syncthreads();
      if (nq > QFLUSH) batch_flush_one_sincos<SC>(q, tab, reqs, st);
    }
  }
  __syncthreads();
  batch_flush_one_sincos<SC, true>(q, tab, reqs, st);
}

__global__ void k_zero_stats(DevStats* st) {
  unsigned long long* p = reinterpret_cast<unsigned long long*>(st);
  for (int i = threadIdx.x; i < (int)(sizeof(DevStats) / 8); i += blockDim.x) p[i] = 0;
}

// ------------------------------------------------------------- host side
constexpr int MAX_DEV = 64;
std::mutex g_mu;
std::atomic<unsigned long long> g_elems[MAX_DEV];
thread_local int t_last_hip = 0;

int hip_fail(hipError_t e) {
  t_last_hip = (int)e;
  return CR_E_HIP;
}

// Per-device addresses of the library's static device memory (g_dev_stats,
// scratch), resolved once per device with that device current.
struct DevState {
  DevStats* stats;
  unsigned char* scratch;
};
DevState g_state[MAX_DEV];
bool g_state_ok[MAX_DEV];

int get_state(DevState** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  if (dev < 0 || dev >= MAX_DEV) return CR_E_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_state_ok[dev]) {
    void* ps = nullptr;
    void* pb = nullptr;
    e = hipGetSymbolAddress(&ps, HIP_SYMBOL(g_dev_stats));
    if (e != hipSuccess) return hip_fail(e);
    e = hipGetSymbolAddress(&pb, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e);
    if (!ps || !pb) return CR_E_HIP;
    g_state[dev].stats = static_cast<DevStats*>(ps);
    g_state[dev].scratch = static_cast<unsigned char*>(pb);
    g_state_ok[dev] = true;
  }
  *out = &g_state[dev];
  return CR_OK;
}

int get_stats(DevStats** out) {
  DevState* ds = nullptr;
  int rc = get_state(&ds);
  if (rc) return rc;
  *out = ds->stats;
  return CR_OK;
}

int g_cus = 0;  // compute units of the current device (cached on first use)

int num_cus() {
  if (!g_cus) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    g_cus = cus > 0 ? cus : 256;
  }
  return g_cus;
}

// default workgroups per compute unit of the persistent grids
int default_bpc() {
  static int per = 0;
  if (!per) {
    int v = CR_BLOCKS_PER_CU;
    if (const char* e = getenv("CR_BLOCKS_PER_CU")) v = atoi(e);
    per = v < 1 ? 1 : (v > 64 ? 64 : v);
  }
  return per;
}

int grid_blocks() { return num_cus() * default_bpc(); }

// The table copy read by the global-placement variants, filled once per device
// (synchronously, on first use).
template <class Op>
int ensure_gtab() {
  static std::atomic<unsigned long long> done{0};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  const unsigned long long bit = 1ull << (dev & 63);
  if (done.load() & bit) return CR_OK;
  std::lock_guard<std::mutex> lk(g_mu);
  if (done.load() & bit) return CR_OK;
  hipLaunchKernelGGL(k_tab_init<Op>, dim3(1), dim3(BLOCK), 0, 0);
  e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e);
  done |= bit;
  return CR_OK;
}

template <class Op, int U, int PF, int TP>
int launch_map_f32(const float* in, float* out, size_t n, hipStream_t s, unsigned flags,
                   DevStats* st, int grid) {
  if (TP) {
    int rc = ensure_gtab<Op>();
    if (rc) return rc;
  }
  uintptr_t ai = (uintptr_t)in, ao = (uintptr_t)out;
  size_t head = 0;
  if ((ai & 15) == (ao & 15)) {
    head = ((16 - (ai & 15)) & 15) / 4;
    if (head > n) head = n;
  } else {
    head = n;  // incompatible alignment: all scalar
  }
  size_t body4 = (n - head) / 4;
  size_t tail = n - head - 4 * body4;
  if (head) {
    size_t g = (head + BLOCK - 1) / BLOCK;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_map_f32_scalar<Op>, dim3((unsigned)g), dim3(BLOCK), 0, s, in, out,
                       (long long)head, st, flags, 0LL);
  }
  // the deferred queue stores 32-bit indices: split bodies beyond 2^32 elements
  for (size_t done = 0; done < body4;) {
    size_t chunk4 = body4 - done;
    if (chunk4 > ((size_t)1 << 29)) chunk4 = (size_t)1 << 29;
    size_t tiles = (chunk4 + BLOCK * U - 1) / (BLOCK * U);
    size_t g = tiles < (size_t)grid ? tiles : (size_t)grid;
    size_t off = head + 4 * done;
    hipLaunchKernelGGL((k_map_f32<Op, U, PF, TP>), dim3((unsigned)g), dim3(BLOCK), 0, s,
                       reinterpret_cast<const float4*>(in + off),
                       reinterpret_cast<float4*>(out + off), (long long)chunk4, st, flags,
                       (long long)off);
    done += chunk4;
  }
  if (tail) {
    size_t off = head + 4 * body4;
    hipLaunchKernelGGL(k_map_f32_scalar<Op>, dim3(1), dim3(BLOCK), 0, s, in + off, out + off,
                       (long long)tail, st, flags, (long long)off);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e);
  return CR_OK;
}

// The launch variants the autotuner chooses from: {U, PF, TP} of k_map_f32.
constexpr int NVARIANT = 7;
constexpr int VARIANTS[NVARIANT][3] = {{2, 1, 0}, {1, 1, 0}, {4, 1, 0}, {2, 0, 0},
                                       {4, 0, 0}, {1, 0, 0}, {2, 1, 1}};

template <class Op>
int launch_variant(const float* in, float* out, size_t n, hipStream_t s, unsigned flags,
                   DevStats* st, int variant, int grid) {
  switch (variant) {
    case 0: return launch_map_f32<Op, 2, 1, 0>(in, out, n, s, flags, st, grid);
    case 1: return launch_map_f32<Op, 1, 1, 0>(in, out, n, s, flags, st, grid);
    case 2: return launch_map_f32<Op, 4, 1, 0>(in, out, n, s, flags, st, grid);
    case 3: return launch_map_f32<Op, 2, 0, 0>(in, out, n, s, flags, st, grid);
    case 4: return launch_map_f32<Op, 4, 0, 0>(in, out, n, s, flags, st, grid);
    case 5: return launch_map_f32<Op, 1, 0, 0>(in, out, n, s, flags, st, grid);
    case 6: return launch_map_f32<Op, 2, 1, 1>(in, out, n, s, flags, st, grid);
  }
  return CR_E_TUNE;
}

template <class SC>
int launch_sincos(const float* in, float* out, size_t n, hipStream_t s, unsigned flags,
                  DevStats* st, int grid) {
  float* outc = out + n;
  uintptr_t ai = (uintptr_t)in, ao = (uintptr_t)out, ac = (uintptr_t)outc;
  // vector body when the input and the sine block are 16-byte aligned; the
  // cosine block (at out + n) is stored by vectors too when it is aligned
  bool vec = (ai & 15) == 0 && (ao & 15) == 0;
  bool cvec = (ac & 15) == 0;
  size_t body4 = vec ? n / 4 : 0;
  size_t done4 = 0;
  while (done4 < body4) {
    size_t chunk4 = body4 - done4;
    if (chunk4 > ((size_t)1 << 29)) chunk4 = (size_t)1 << 29;
    size_t tiles = (chunk4 + BLOCK * TILE_U - 1) / (BLOCK * TILE_U);
    size_t g = tiles < (size_t)grid ? tiles : (size_t)grid;
    size_t off = 4 * done4;
    auto k = cvec ? k_map_sincos<SC, true> : k_map_sincos<SC, false>;
    hipLaunchKernelGGL(k, dim3((unsigned)g), dim3(BLOCK), 0, s,
                       reinterpret_cast<const float4*>(in + off),
                       reinterpret_cast<float4*>(out + off), outc + off, (long long)chunk4, st,
                       flags, (long long)off);
    done4 += chunk4;
  }
  size_t off = 4 * body4;
  if (off < n) {
    size_t rest = n - off;
    size_t g = (rest + BLOCK - 1) / BLOCK;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_map_sincos_scalar<SC>, dim3((unsigned)g), dim3(BLOCK), 0, s, in + off,
                       out + off, outc + off, (long long)rest, st, flags, (long long)off);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e);
  return CR_OK;
}

template <class Op, int U, int SL>
int launch_map_f64(const double* in, double* out, size_t n, hipStream_t s, unsigned flags,
                   DevStats* st, int grid) {
  uintptr_t ai = (uintptr_t)in, ao = (uintptr_t)out;
  size_t head = 0;
  if ((ai & 15) == (ao & 15)) {
    head = ((16 - (ai & 15)) & 15) / 8;
    if (head > n) head = n;
  } else {
    head = n;
  }
  size_t body2 = (n - head) / 2;
  size_t tail = n - head - 2 * body2;
  if (head) {
    hipLaunchKernelGGL(k_map_f64_scalar<Op>, dim3((unsigned)((head + BLOCK - 1) / BLOCK > 65536
                                                               ? 65536
                                                               : (head + BLOCK - 1) / BLOCK)),
                       dim3(BLOCK), 0, s, in, out, (long long)head, st, flags, 0LL);
  }
  for (size_t done = 0; done < body2;) {
    size_t chunk2 = body2 - done;
    if (chunk2 > ((size_t)1 << 30)) chunk2 = (size_t)1 << 30;
    size_t tiles = (chunk2 + BLOCK * U - 1) / (BLOCK * U);
    size_t g = tiles < (size_t)grid ? tiles : (size_t)grid;
    size_t off = head + 2 * done;
    hipLaunchKernelGGL((k_map_f64<Op, U, SL>), dim3((unsigned)g), dim3(BLOCK), 0, s,
                       reinterpret_cast<const double2*>(in + off),
                       reinterpret_cast<double2*>(out + off), (long long)chunk2, st, flags,
                       (long long)off);
    done += chunk2;
  }
  if (tail) {
    size_t off = head + 2 * body2;
    hipLaunchKernelGGL(k_map_f64_scalar<Op>, dim3(1), dim3(BLOCK), 0, s, in + off, out + off,
                       (long long)tail, st, flags, (long long)off);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e);
  return CR_OK;
}

// The binary64 launch variants: {U, SL} of k_map_f64 (variant 0: four vectors
// per thread, an element at a time).
constexpr int NVARIANT64 = 4;
template <class Op>
int launch_variant64(const double* in, double* out, size_t n, hipStream_t s, unsigned flags,
                     DevStats* st, int variant, int grid) {
  switch (variant) {
    case 0: return launch_map_f64<Op, 4, 0>(in, out, n, s, flags, st, grid);
    case 1: return launch_map_f64<Op, 1, 1>(in, out, n, s, flags, st, grid);
    case 2: return launch_map_f64<Op, 2, 1>(in, out, n, s, flags, st, grid);
    case 3: return launch_map_f64<Op, 4, 1>(in, out, n, s, flags, st, grid);
  }
  return CR_E_TUNE;
}

// Complex binary32 map (n complex numbers, interleaved): 16-byte aligned
// body of two complex numbers per vector, scalar head and tail.
template <class CF>
int launch_complex(const float* in, float* out, size_t n, hipStream_t s, unsigned flags,
                   DevStats* st, int grid) {
  uintptr_t ai = (uintptr_t)in, ao = (uintptr_t)out;
  size_t head = 0;
  if ((ai & 15) == (ao & 15) && (ai & 7) == 0) {
    head = (ai & 15) ? 1 : 0;
    if (head > n) head = n;
  } else {
    head = n;
  }
  const size_t body2 = (n - head) / 2;
  const size_t tail = n - head - 2 * body2;
  auto scalar = [&](size_t off, size_t cnt) {
    size_t g = (cnt + BLOCK - 1) / BLOCK;
    if (g > (size_t)grid) g = grid;
    hipLaunchKernelGGL(k_complex_scalar<CF>, dim3((unsigned)g), dim3(BLOCK), 0, s, in + 2 * off,
                       out + 2 * off, (long long)cnt, st, flags, (long long)off);
  };
  if (head) scalar(0, head);
  for (size_t done = 0; done < body2;) {
    size_t chunk = body2 - done;
    if (chunk > ((size_t)1 << 30)) chunk = (size_t)1 << 30;
    size_t g = (chunk + BLOCK - 1) / BLOCK;
    if (g > (size_t)grid) g = grid;
    const size_t off = head + 2 * done;
    hipLaunchKernelGGL(k_complex<CF>, dim3((unsigned)g), dim3(BLOCK), 0, s,
                       reinterpret_cast<const float4*>(in + 2 * off),
                       reinterpret_cast<float4*>(out + 2 * off), (long long)chunk, st, flags,
                       (long long)off);
    done += chunk;
  }
  if (tail) scalar(head + 2 * body2, tail);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e);
  return CR_OK;
}

bool func_complex(int f) { return f == CR_CEXPF || f == CR_CLOGF || f == CR_CSINF; }
bool impl_valid(int impl) {
  return impl == CR_IMPL_AUTO || impl == CR_IMPL_F64_INTERNAL || impl == CR_IMPL_SPLIT_F32 ||
         impl == CR_IMPL_LOG128;
}
bool func_f64(int f) { return f == CR_EXP || f == CR_LOG || f == CR_EXP2; }
bool func_valid(int f) { return (f >= 0 && f < CR_NUM_F32) || func_f64(f) || func_complex(f); }
bool func_built(int f) {
  return (f >= CR_EXPF && f <= CR_TANHF) || func_f64(f) || func_complex(f);
}
// bytes of one input element (complex: two binary32) and of the output per element
size_t elem_bytes(int f) { return func_f64(f) || func_complex(f) ? 8 : 4; }
// functions with a binary32-only (split) implementation
bool split_built(int f) { return f >= CR_EXPF && f <= CR_TANHF; }

int dispatch_f32_split(int f, const float* in, float* out, size_t n, hipStream_t s,
                       unsigned flags, DevStats* st, int v, int g) {
  switch (f) {
    case CR_EXPF: return launch_variant<OpSExp<EXPK_E>>(in, out, n, s, flags, st, v, g);
    case CR_EXP2F: return launch_variant<OpSExp<EXPK_2>>(in, out, n, s, flags, st, v, g);
    case CR_EXP10F: return launch_variant<OpSExp<EXPK_10>>(in, out, n, s, flags, st, v, g);
    case CR_EXPM1F: return launch_variant<OpSExp<EXPK_EM1>>(in, out, n, s, flags, st, v, g);
    case CR_LOGF: return launch_variant<OpSLog<LOGK_E>>(in, out, n, s, flags, st, v, g);
    case CR_LOG2F: return launch_variant<OpSLog<LOGK_2>>(in, out, n, s, flags, st, v, g);
    case CR_LOG10F: return launch_variant<OpSLog<LOGK_10>>(in, out, n, s, flags, st, v, g);
    case CR_LOG1PF: return launch_variant<OpSLog<LOGK_1P>>(in, out, n, s, flags, st, v, g);
    case CR_RSQRTF: return launch_variant<OpSRsqrt>(in, out, n, s, flags, st, v, g);
    case CR_SINF: return launch_variant<OpSTrig<TRIGK_SIN>>(in, out, n, s, flags, st, v, g);
    case CR_COSF: return launch_variant<OpSTrig<TRIGK_COS>>(in, out, n, s, flags, st, v, g);
    case CR_TANF: return launch_variant<OpSTrig<TRIGK_TAN>>(in, out, n, s, flags, st, v, g);
    case CR_SINCOSF: return launch_sincos<SinCosSplit>(in, out, n, s, flags, st, g);
    case CR_ASINF: return launch_variant<OpSAtan<ATANK_ASIN>>(in, out, n, s, flags, st, v, g);
    case CR_ACOSF: return launch_variant<OpSAtan<ATANK_ACOS>>(in, out, n, s, flags, st, v, g);
    case CR_ATANF: return launch_variant<OpSAtan<ATANK_ATAN>>(in, out, n, s, flags, st, v, g);
    case CR_SINHF: return launch_variant<OpSHyp<HYPK_SINH>>(in, out, n, s, flags, st, v, g);
    case CR_COSHF: return launch_variant<OpSHyp<HYPK_COSH>>(in, out, n, s, flags, st, v, g);
    case CR_TANHF: return launch_variant<OpSHyp<HYPK_TANH>>(in, out, n, s, flags, st, v, g);
  }
  return CR_E_IMPL;
}

int dispatch_f32(int f, const float* in, float* out, size_t n, hipStream_t s, unsigned flags,
                 DevStats* st, int v, int g) {
  switch (f) {
    case CR_EXPF: return launch_variant<OpExp<EXPK_E>>(in, out, n, s, flags, st, v, g);
    case CR_EXP2F: return launch_variant<OpExp<EXPK_2>>(in, out, n, s, flags, st, v, g);
    case CR_EXP10F: return launch_variant<OpExp<EXPK_10>>(in, out, n, s, flags, st, v, g);
    case CR_EXPM1F: return launch_variant<OpExp<EXPK_EM1>>(in, out, n, s, flags, st, v, g);
    case CR_LOGF: return launch_variant<OpLog<LOGK_E>>(in, out, n, s, flags, st, v, g);
    case CR_LOG2F: return launch_variant<OpLog<LOGK_2>>(in, out, n, s, flags, st, v, g);
    case CR_LOG10F: return launch_variant<OpLog<LOGK_10>>(in, out, n, s, flags, st, v, g);
    case CR_LOG1PF: return launch_variant<OpLog<LOGK_1P>>(in, out, n, s, flags, st, v, g);
    case CR_RSQRTF: return launch_variant<OpRsqrt>(in, out, n, s, flags, st, v, g);
    case CR_SINF: return launch_variant<OpTrig<TRIGK_SIN>>(in, out, n, s, flags, st, v, g);
    case CR_COSF: return launch_variant<OpTrig<TRIGK_COS>>(in, out, n, s, flags, st, v, g);
    case CR_TANF: return launch_variant<OpTrig<TRIGK_TAN>>(in, out, n, s, flags, st, v, g);
    case CR_SINCOSF: return launch_sincos<SinCosF64>(in, out, n, s, flags, st, g);
    case CR_ASINF: return launch_variant<OpAtan<ATANK_ASIN>>(in, out, n, s, flags, st, v, g);
    case CR_ACOSF: return launch_variant<OpAtan<ATANK_ACOS>>(in, out, n, s, flags, st, v, g);
    case CR_ATANF: return launch_variant<OpAtan<ATANK_ATAN>>(in, out, n, s, flags, st, v, g);
    case CR_SINHF: return launch_variant<OpHyp<HYPK_SINH>>(in, out, n, s, flags, st, v, g);
    case CR_COSHF: return launch_variant<OpHyp<HYPK_COSH>>(in, out, n, s, flags, st, v, g);
    case CR_TANHF: return launch_variant<OpHyp<HYPK_TANH>>(in, out, n, s, flags, st, v, g);
  }
  return CR_E_FUNC;
}


// Directed rounding modes: one grid-stride kernel per (function, mode).
template <class Op, int RM>
int launch_dir(const float* in, float* out, size_t n, hipStream_t s, DevStats* st, int grid) {
  size_t g = (n + BLOCK - 1) / BLOCK;
  if (g > (size_t)grid) g = grid;
  hipLaunchKernelGGL((k_map_f32_dir<Op, RM>), dim3((unsigned)g), dim3(BLOCK), 0, s, in, out,
                     (long long)n, st, 0LL);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? CR_OK : hip_fail(e);
}

template <int RM>
int dispatch_f32_dir(int f, const float* in, float* out, size_t n, hipStream_t s, DevStats* st,
                     int g) {
  switch (f) {
    case CR_EXPF: return launch_dir<OpExp<EXPK_E>, RM>(in, out, n, s, st, g);
    case CR_EXP2F: return launch_dir<OpExp<EXPK_2>, RM>(in, out, n, s, st, g);
    case CR_EXP10F: return launch_dir<OpExp<EXPK_10>, RM>(in, out, n, s, st, g);
    case CR_EXPM1F: return launch_dir<OpExp<EXPK_EM1>, RM>(in, out, n, s, st, g);
    case CR_LOGF: return launch_dir<OpLog<LOGK_E>, RM>(in, out, n, s, st, g);
    case CR_LOG2F: return launch_dir<OpLog<LOGK_2>, RM>(in, out, n, s, st, g);
    case CR_LOG10F: return launch_dir<OpLog<LOGK_10>, RM>(in, out, n, s, st, g);
    case CR_LOG1PF: return launch_dir<OpLog<LOGK_1P>, RM>(in, out, n, s, st, g);
    case CR_RSQRTF: return launch_dir<OpRsqrt, RM>(in, out, n, s, st, g);
    case CR_SINF: return launch_dir<OpTrig<TRIGK_SIN>, RM>(in, out, n, s, st, g);
    case CR_COSF: return launch_dir<OpTrig<TRIGK_COS>, RM>(in, out, n, s, st, g);
    case CR_TANF: return launch_dir<OpTrig<TRIGK_TAN>, RM>(in, out, n, s, st, g);
    case CR_ASINF: return launch_dir<OpAtan<ATANK_ASIN>, RM>(in, out, n, s, st, g);
    case CR_ACOSF: return launch_dir<OpAtan<ATANK_ACOS>, RM>(in, out, n, s, st, g);
    case CR_ATANF: return launch_dir<OpAtan<ATANK_ATAN>, RM>(in, out, n, s, st, g);
    case CR_SINHF: return launch_dir<OpHyp<HYPK_SINH>, RM>(in, out, n, s, st, g);
    case CR_COSHF: return launch_dir<OpHyp<HYPK_COSH>, RM>(in, out, n, s, st, g);
    case CR_TANHF: return launch_dir<OpHyp<HYPK_TANH>, RM>(in, out, n, s, st, g);
    case CR_SINCOSF: {
      size_t gg = (n + BLOCK - 1) / BLOCK;
      if (gg > (size_t)g) gg = g;
      hipLaunchKernelGGL((k_sincos_dir<SinCosF64, RM>), dim3((unsigned)gg), dim3(BLOCK), 0, s, in,
                         out, out + n, (long long)n, st, 0LL);
      hipError_t e = hipGetLastError();
      return e == hipSuccess ? CR_OK : hip_fail(e);
    }
  }
  return CR_E_FUNC;
}

int dispatch_dir(int mode, int f, const float* in, float* out, size_t n, hipStream_t s,
                 DevStats* st, int g) {
  switch (mode) {
    case RM_RZ: return dispatch_f32_dir<RM_RZ>(f, in, out, n, s, st, g);
    case RM_RU: return dispatch_f32_dir<RM_RU>(f, in, out, n, s, st, g);
    case RM_RD: return dispatch_f32_dir<RM_RD>(f, in, out, n, s, st, g);
  }
  return CR_E_IMPL;
}

// ------------------------------------------------------------ tuning table
// One launch configuration per (implementation, function): a k_map_f32
// variant and the persistent grid in workgroups per compute unit.  Index 0 of
// the first dimension is the binary64-internal implementation (and AUTO), 1
// the split one; functions 0..18, then the ids of EXTRA_FUNCS.
constexpr int EXTRA_FUNCS[] = {CR_EXP, CR_LOG, CR_EXP2, CR_CEXPF, CR_CLOGF, CR_CSINF};
constexpr int NFUNC_IDX = CR_NUM_F32 + (int)(sizeof(EXTRA_FUNCS) / sizeof(EXTRA_FUNCS[0]));
std::atomic<int> g_cfg_variant[2][NFUNC_IDX];
std::atomic<int> g_cfg_bpc[2][NFUNC_IDX];  // 0: the default

int fidx(int f) {
  if (f < CR_NUM_F32) return f;
  for (int i = 0; i < NFUNC_IDX - CR_NUM_F32; i++)
    if (EXTRA_FUNCS[i] == f) return CR_NUM_F32 + i;
  return 0;  // not reached: callers validate f first
}
int iidx(int impl) { return impl == CR_IMPL_SPLIT_F32 ? 1 : 0; }
// sincos and the complex functions have one kernel shape (variant 0 only),
// the binary64 functions NVARIANT64
int num_variants_of(int f) {
  return (f == CR_SINCOSF || func_complex(f)) ? 1 : f >= 64 ? NVARIANT64 : NVARIANT;
}

int eval_cfg(int func_id, int impl, unsigned flags, const void* in, void* out, size_t n,
             hipStream_t s, int variant, int bpc) {
  DevStats* st = nullptr;
  int rc = get_stats(&st);
  if (rc) return rc;
  const int g = num_cus() * (bpc > 0 ? bpc : default_bpc());
  const int mode = (int)((flags & CR_FLAG_ROUND_MASK) >> CR_FLAG_ROUND_SHIFT);
  if (mode != RM_RN)
    rc = dispatch_dir(mode, func_id, (const float*)in, (float*)out, n, s, st, g);
  else if (func_id < CR_NUM_F32 && impl == CR_IMPL_SPLIT_F32)
    rc = dispatch_f32_split(func_id, (const float*)in, (float*)out, n, s, flags, st, variant, g);
  else if (func_id < CR_NUM_F32)
    rc = dispatch_f32(func_id, (const float*)in, (float*)out, n, s, flags, st, variant, g);
  else if (func_id == CR_EXP)
    rc = launch_variant64<OpExp64>((const double*)in, (double*)out, n, s, flags, st, variant, g);
  else if (func_id == CR_EXP2)
    rc = launch_variant64<OpExp2_64>((const double*)in, (double*)out, n, s, flags, st, variant, g);
  else if (func_id == CR_LOG && impl == CR_IMPL_LOG128)
    rc = launch_variant64<OpLog128>((const double*)in, (double*)out, n, s, flags, st, variant, g);
  else if (func_id == CR_CEXPF)
    rc = launch_complex<CExpF>((const float*)in, (float*)out, n, s, flags, st, g);
  else if (func_id == CR_CLOGF)
    rc = launch_complex<CLogF>((const float*)in, (float*)out, n, s, flags, st, g);
  else if (func_id == CR_CSINF)
    rc = launch_complex<CSinF>((const float*)in, (float*)out, n, s, flags, st, g);
  else
    rc = launch_variant64<OpLog64>((const double*)in, (double*)out, n, s, flags, st, variant, g);
  if (rc == CR_OK) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    g_elems[dev] += n;
  }
  return rc;
}

const char* const FUNC_NAMES[NFUNC_IDX] = {
    "expf", "exp2f", "exp10f", "expm1f", "logf", "log2f", "log10f", "log1pf", "rsqrtf",
    "sinf", "cosf", "sincosf", "tanf", "asinf", "acosf", "atanf", "sinhf", "coshf", "tanhf",
    "exp", "log", "exp2", "cexpf", "clogf", "csinf"};

int func_of_idx(int i) { return i < CR_NUM_F32 ? i : EXTRA_FUNCS[i - CR_NUM_F32]; }

// ------------------------------------------------------------ batch plans
}  // namespace

struct cr_batch_plan {
  int device;
  BReq* d_reqs;
  BTile* d_tiles;
  long long ntiles;
  int grid;
  unsigned flags;
  hipGraphExec_t exec;
  hipEvent_t done;
  bool launched;
  long long elems;
};

namespace {

// Validate requests and build the request and tile tables (host side).
int build_tables(const cr_request* reqs, int32_t num, std::vector<BReq>& hr,
                 std::vector<BTile>& ht, long long& elems) {
  if (num < 0) return CR_E_SIZE;
  if (num > 0 && !reqs) return CR_E_NULL;
  hr.clear();
  ht.clear();
  elems = 0;
  std::vector<int> order(num);
  for (int i = 0; i < num; i++) {
    const cr_request& r = reqs[i];
    if (r.func_id < 0 || r.func_id >= CR_NUM_F32) return CR_E_FUNC;
    if (r.impl != CR_IMPL_AUTO && r.impl != CR_IMPL_F64_INTERNAL && r.impl != CR_IMPL_SPLIT_F32)
      return CR_E_IMPL;
    if (r.n < 0 || r.n >= ((int64_t)1 << 31)) return CR_E_SIZE;
    if (r.n == 0) continue;
    if (!r.in || !r.out) return CR_E_NULL;
    uintptr_t a = (uintptr_t)r.in, b = (uintptr_t)r.out;
    if ((a & 3) || (b & 3)) return CR_E_ALIGN;
    size_t nout = r.func_id == CR_SINCOSF ? 2 * (size_t)r.n : (size_t)r.n;
    bool same = a == b && nout == (size_t)r.n;
    if (!same && a < b + nout * 4 && b < a + (size_t)r.n * 4) return CR_E_OVERLAP;
    if (!cr_available(r.func_id, r.impl)) return CR_E_IMPL;
  }
  // order requests by (implementation, function) so that tiles sharing tables
  // are adjacent
  auto key = [&](int i) {
    return reqs[i].func_id + (reqs[i].impl == CR_IMPL_SPLIT_F32 ? BSPLIT : 0);
  };
  for (int i = 0; i < num; i++) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return key(x) < key(y); });
  for (int oi = 0; oi < num; oi++) {
    const cr_request& r = reqs[order[oi]];
    if (r.n == 0) continue;
    BReq q;
    q.in = r.in;
    q.out = r.out;
    q.n = r.n;
    q.func = r.func_id;
    q.key = key(order[oi]);
    q.orig = order[oi];
    uintptr_t a = (uintptr_t)r.in, b = (uintptr_t)r.out;
    uintptr_t c = b + 4 * (uintptr_t)r.n;
    q.aligned = ((a | b) & 15) == 0 && (r.func_id != CR_SINCOSF || (c & 15) == 0);
    int ri = (int)hr.size();
    hr.push_back(q);
    for (long long s = 0; s < r.n; s += TILE) {
      BTile t;
      t.req = ri;
      t.start = s;
      t.count = (int)((r.n - s) < TILE ? (r.n - s) : TILE);
      ht.push_back(t);
    }
    elems += r.n;
  }
  return CR_OK;
}

// Contiguous tile ranges of one key (function + BSPLIT for the split
// implementation) in the sorted tile table.
struct BRange {
  int key;
  long long t0, t1;
};

std::vector<BRange> key_ranges(const std::vector<BReq>& hr, const std::vector<BTile>& ht) {
  std::vector<BRange> rs;
  for (long long t = 0; t < (long long)ht.size(); t++) {
    int key = hr[ht[t].req].key;
    if (rs.empty() || rs.back().key != key) rs.push_back({key, t, t});
    rs.back().t1 = t + 1;
  }
  return rs;
}

template <class Op>
void launch_tiles_op(const BReq* r, const BTile* t, const BRange& g, int grid, DevStats* st,
                     unsigned flags, hipStream_t s) {
  hipLaunchKernelGGL(k_tiles<Op>, dim3(grid), dim3(BLOCK), 0, s, r, t, g.t0, g.t1, st, flags);
}

// Workgroups per compute unit of each batch kernel, per implementation
// (binary64-internal, binary32-only): a tuned setting (cr_tune_batch_set, the
// "batch" lines of the tuning file).  The plan's graph runs up to four kernels
// at a time (parallel branches), so together they hold about four times as
// many workgroups per CU; the default, 4, was the best of {1, 2, 4, 8, 16, 32}
// on the 4096-request workload when it was chosen (1 -> 361, 2 -> 413,
// 4 -> 428, 8 -> 422, 16 -> 411, 32 -> 385 Gelem/s).
constexpr int BATCH_BPC_DEFAULT = 4;
std::atomic<int> g_batch_bpc[2] = {BATCH_BPC_DEFAULT, BATCH_BPC_DEFAULT};

// Launch the kernel of one key range (at most one workgroup per tile).
int launch_tiles(const BReq* r, const BTile* t, const BRange& g, DevStats* st, unsigned flags,
                 hipStream_t s) {
  long long grid = (long long)num_cus() * g_batch_bpc[g.key >= BSPLIT ? 1 : 0].load();
  if (grid > g.t1 - g.t0) grid = g.t1 - g.t0;
  const int G = (int)grid;
  switch (g.key) {
    case CR_EXPF: launch_tiles_op<OpExp<EXPK_E>>(r, t, g, G, st, flags, s); break;
    case CR_EXP2F: launch_tiles_op<OpExp<EXPK_2>>(r, t, g, G, st, flags, s); break;
    case CR_EXP10F: launch_tiles_op<OpExp<EXPK_10>>(r, t, g, G, st, flags, s); break;
    case CR_EXPM1F: launch_tiles_op<OpExp<EXPK_EM1>>(r, t, g, G, st, flags, s); break;
    case CR_LOGF: launch_tiles_op<OpLog<LOGK_E>>(r, t, g, G, st, flags, s); break;
    case CR_LOG2F: launch_tiles_op<OpLog<LOGK_2>>(r, t, g, G, st, flags, s); break;
    case CR_LOG10F: launch_tiles_op<OpLog<LOGK_10>>(r, t, g, G, st, flags, s); break;
    case CR_LOG1PF: launch_tiles_op<OpLog<LOGK_1P>>(r, t, g, G, st, flags, s); break;
    case CR_RSQRTF: launch_tiles_op<OpRsqrt>(r, t, g, G, st, flags, s); break;
    case CR_SINF: launch_tiles_op<OpTrig<TRIGK_SIN>>(r, t, g, G, st, flags, s); break;
    case CR_COSF: launch_tiles_op<OpTrig<TRIGK_COS>>(r, t, g, G, st, flags, s); break;
    case CR_TANF: launch_tiles_op<OpTrig<TRIGK_TAN>>(r, t, g, G, st, flags, s); break;
    case CR_SINCOSF:
      hipLaunchKernelGGL(k_tiles_sincos<SinCosF64>, dim3(G), dim3(BLOCK), 0, s, r, t, g.t0, g.t1,
                         st, flags);
      break;
    case CR_ASINF: launch_tiles_op<OpAtan<ATANK_ASIN>>(r, t, g, G, st, flags, s); break;
    case CR_ACOSF: launch_tiles_op<OpAtan<ATANK_ACOS>>(r, t, g, G, st, flags, s); break;
    case CR_ATANF: launch_tiles_op<OpAtan<ATANK_ATAN>>(r, t, g, G, st, flags, s); break;
    case CR_SINHF: launch_tiles_op<OpHyp<HYPK_SINH>>(r, t, g, G, st, flags, s); break;
    case CR_COSHF: launch_tiles_op<OpHyp<HYPK_COSH>>(r, t, g, G, st, flags, s); break;
    case CR_TANHF: launch_tiles_op<OpHyp<HYPK_TANH>>(r, t, g, G, st, flags, s); break;
    case BSPLIT + CR_EXPF: launch_tiles_op<OpSExp<EXPK_E>>(r, t, g, G, st, flags, s); break;
    case BSPLIT + CR_EXP2F: launch_tiles_op<OpSExp<EXPK_2>>(r, t, g, G, st, flags, s); break;
    case BSPLIT + CR_EXP10F: launch_tiles_op<OpSExp<EXPK_10>>(r, t, g, G, st, flags, s); break;
    case BSPLIT + CR_EXPM1F: launch_tiles_op<OpSExp<EXPK_EM1>>(r, t, g, G, st, flags, s); break;
    case BSPLIT + CR_LOGF: launch_tiles_op<OpSLog<LOGK_E>>(r, t, g, G, st, flags, s); break;
    case BSPLIT + CR_LOG2F: launch_tiles_op<OpSLog<LOGK_2>>(r, t, g, G, st, flags, s); break;
    case BSPLIT + CR_LOG10F: launch_tiles_op<OpSLog<LOGK_10>>(r, t, g, G, st, flags, s); break;
    case BSPLIT + CR_LOG1PF: launch_tiles_op<OpSLog<LOGK_1P>>(r, t, g, G, st, flags, s); break;
    case BSPLIT + CR_RSQRTF: launch_tiles_op<OpSRsqrt>(r, t, g, G, st, flags, s); break;
    case BSPLIT + CR_SINF: launch_tiles_op<OpSTrig<TRIGK_SIN>>(r, t, g, G, st, flags, s); break;
    case BSPLIT + CR_COSF: launch_tiles_op<OpSTrig<TRIGK_COS>>(r, t, g, G, st, flags, s); break;
    case BSPLIT + CR_TANF: launch_tiles_op<OpSTrig<TRIGK_TAN>>(r, t, g, G, st, flags, s); break;
    case BSPLIT + CR_SINCOSF:
      hipLaunchKernelGGL(k_tiles_sincos<SinCosSplit>, dim3(G), dim3(BLOCK), 0, s, r, t, g.t0,
                         g.t1, st, flags);
      break;
    case BSPLIT + CR_ASINF: launch_tiles_op<OpSAtan<ATANK_ASIN>>(r, t, g, G, st, flags, s); break;
    case BSPLIT + CR_ACOSF: launch_tiles_op<OpSAtan<ATANK_ACOS>>(r, t, g, G, st, flags, s); break;
    case BSPLIT + CR_ATANF: launch_tiles_op<OpSAtan<ATANK_ATAN>>(r, t, g, G, st, flags, s); break;
    case BSPLIT + CR_SINHF: launch_tiles_op<OpSHyp<HYPK_SINH>>(r, t, g, G, st, flags, s); break;
    case BSPLIT + CR_COSHF: launch_tiles_op<OpSHyp<HYPK_COSH>>(r, t, g, G, st, flags, s); break;
    case BSPLIT + CR_TANHF: launch_tiles_op<OpSHyp<HYPK_TANH>>(r, t, g, G, st, flags, s); break;
    default: return CR_E_FUNC;
  }
  return CR_OK;
}

}  // namespace

extern "C" int cr_batch_plan_destroy(cr_batch_plan* plan);

namespace {
}  // namespace

extern "C" {

int cr_available(int func_id, int impl);

int cr_eval_ex(int func_id, int impl, unsigned flags, const void* in, void* out, size_t n,
               void* stream) {
  if (!func_valid(func_id)) return CR_E_FUNC;
  if (!impl_valid(impl)) return CR_E_IMPL;
  if (n == 0) return CR_OK;
  if (!in || !out) return CR_E_NULL;
  const size_t es = elem_bytes(func_id), al = func_complex(func_id) ? 4 : es;
  const size_t nout = func_id == CR_SINCOSF ? 2 * n : n;
  if (n > ((size_t)1 << 60)) return CR_E_SIZE;
  uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
  if ((a % al) || (b % al)) return CR_E_ALIGN;
  bool same = a == b && nout == n;
  if (!same && a < b + nout * es && b < a + n * es) return CR_E_OVERLAP;
  if (!cr_available(func_id, impl)) return CR_E_IMPL;
  if ((flags & CR_FLAG_ROUND_MASK) &&
      (func_id >= CR_NUM_F32 || impl == CR_IMPL_SPLIT_F32 || impl == CR_IMPL_LOG128))
    return CR_E_IMPL;  // directed modes: the binary32 functions, binary64-internal
  const int ii = iidx(impl), fi = fidx(func_id);
  return eval_cfg(func_id, impl, flags, in, out, n, (hipStream_t)stream,
                  g_cfg_variant[ii][fi].load(), g_cfg_bpc[ii][fi].load());
}

// ------------------------------------------------------------------ tuning
int cr_tune_num_variants(void) { return NVARIANT; }

int cr_tune_variant_info(int variant, int* elems_per_thread, int* prefetch, int* table_in_lds) {
  if (variant < 0 || variant >= NVARIANT) return CR_E_TUNE;
  if (elems_per_thread) *elems_per_thread = 4 * VARIANTS[variant][0];
  if (prefetch) *prefetch = VARIANTS[variant][1];
  if (table_in_lds) *table_in_lds = VARIANTS[variant][2] ? 0 : 1;
  return CR_OK;
}

static int tune_check(int func_id, int impl, const cr_tune_cfg* cfg) {
  if (!func_valid(func_id)) return CR_E_FUNC;
  if (!impl_valid(impl)) return CR_E_IMPL;
  if (!cfg) return CR_E_NULL;
  if (cfg->variant < 0 || cfg->variant >= num_variants_of(func_id)) return CR_E_TUNE;
  if (cfg->blocks_per_cu < 0 || cfg->blocks_per_cu > 64) return CR_E_TUNE;
  return CR_OK;
}

int cr_tune_get(int func_id, int impl, cr_tune_cfg* cfg) {
  if (!func_valid(func_id)) return CR_E_FUNC;
  if (!impl_valid(impl)) return CR_E_IMPL;
  if (!cfg) return CR_E_NULL;
  const int ii = iidx(impl), fi = fidx(func_id);
  cfg->variant = g_cfg_variant[ii][fi].load();
  int b = g_cfg_bpc[ii][fi].load();
  cfg->blocks_per_cu = b > 0 ? b : default_bpc();
  return CR_OK;
}

int cr_tune_set(int func_id, int impl, const cr_tune_cfg* cfg) {
  int rc = tune_check(func_id, impl, cfg);
  if (rc) return rc;
  const int ii = iidx(impl), fi = fidx(func_id);
  g_cfg_variant[ii][fi] = cfg->variant;
  g_cfg_bpc[ii][fi] = cfg->blocks_per_cu;
  return CR_OK;
}

int cr_tune_reset(void) {
  for (int i = 0; i < 2; i++) {
    for (int f = 0; f < NFUNC_IDX; f++) {
      g_cfg_variant[i][f] = 0;
      g_cfg_bpc[i][f] = 0;
    }
    g_batch_bpc[i] = BATCH_BPC_DEFAULT;
  }
  return CR_OK;
}

int cr_tune_batch_get(int impl, int32_t* blocks_per_cu) {
  if (!impl_valid(impl) || impl == CR_IMPL_LOG128) return CR_E_IMPL;
  if (!blocks_per_cu) return CR_E_NULL;
  *blocks_per_cu = g_batch_bpc[iidx(impl)].load();
  return CR_OK;
}

int cr_tune_batch_set(int impl, int32_t blocks_per_cu) {
  if (!impl_valid(impl) || impl == CR_IMPL_LOG128) return CR_E_IMPL;
  if (blocks_per_cu < 1 || blocks_per_cu > 64) return CR_E_TUNE;
  g_batch_bpc[iidx(impl)] = blocks_per_cu;
  return CR_OK;
}

int cr_tune_save(const char* path) {
  if (!path) return CR_E_NULL;
  FILE* fp = fopen(path, "w");
  if (!fp) return CR_E_TUNE;
  fprintf(fp, "# libcr launch configurations: function implementation variant blocks_per_cu\n");
  for (int i = 0; i < 2; i++)
    for (int f = 0; f < NFUNC_IDX; f++) {
      int b = g_cfg_bpc[i][f].load();
      fprintf(fp, "%s %s %d %d\n", FUNC_NAMES[f], i ? "split" : "f64", g_cfg_variant[i][f].load(),
              b > 0 ? b : default_bpc());
    }
  for (int i = 0; i < 2; i++)
    fprintf(fp, "batch %s 0 %d\n", i ? "split" : "f64", g_batch_bpc[i].load());
  int bad = ferror(fp);
  if (fclose(fp) != 0 || bad) return CR_E_TUNE;
  return CR_OK;
}

int cr_tune_load(const char* path) {
  if (!path) return CR_E_NULL;
  FILE* fp = fopen(path, "r");
  if (!fp) return CR_E_TUNE;
  struct Entry { int impl, func, variant, bpc; };
  std::vector<Entry> es;
  char line[512];
  int rc = CR_OK;
  while (fgets(line, sizeof line, fp)) {
    char* p = line;
    while (*p == ' ' || *p == '\t') p++;
    if (*p == '#' || *p == '\n' || *p == '\r' || *p == 0) continue;
    char fname[64], iname[16];
    int v = -1, b = -1;
    if (sscanf(p, "%63s %15s %d %d", fname, iname, &v, &b) != 4) {
      rc = CR_E_TUNE;
      break;
    }
    int f = -1;
    for (int k = 0; k < NFUNC_IDX; k++)
      if (!strcmp(fname, FUNC_NAMES[k])) f = func_of_idx(k);
    int impl = !strcmp(iname, "f64") ? CR_IMPL_F64_INTERNAL
               : !strcmp(iname, "split") ? CR_IMPL_SPLIT_F32 : -1;
    if (!strcmp(fname, "batch")) {  // the batch kernels' grid: variant 0 only
      if (impl < 0 || v != 0 || b < 1 || b > 64) {
        rc = CR_E_TUNE;
        break;
      }
      es.push_back({impl, -1, v, b});
      continue;
    }
    cr_tune_cfg c = {v, b};
    if (f < 0 || impl < 0 || tune_check(f, impl, &c) != CR_OK) {
      rc = CR_E_TUNE;
      break;
    }
    es.push_back({impl, f, v, b});
  }
  fclose(fp);
  if (rc) return rc;  // nothing applied from a malformed file
  for (const Entry& e : es) {
    if (e.func < 0) {
      g_batch_bpc[iidx(e.impl)] = e.bpc;
      continue;
    }
    g_cfg_variant[iidx(e.impl)][fidx(e.func)] = e.variant;
    g_cfg_bpc[iidx(e.impl)][fidx(e.func)] = e.bpc;
  }
  return CR_OK;
}

int cr_autotune(int func_id, int impl, const void* in, void* out, size_t n, int reps,
                void* stream, double* best_gelem_s) {
  if (!func_valid(func_id)) return CR_E_FUNC;
  if (!impl_valid(impl)) return CR_E_IMPL;
  if (n == 0 || !in || !out) return CR_E_NULL;
  const size_t es = elem_bytes(func_id), al = func_complex(func_id) ? 4 : es;
  const size_t nout = func_id == CR_SINCOSF ? 2 * n : n;
  if (n > ((size_t)1 << 60)) return CR_E_SIZE;
  uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
  if ((a % al) || (b % al)) return CR_E_ALIGN;
  bool same = a == b && nout == n;
  if (!same && a < b + nout * es && b < a + n * es) return CR_E_OVERLAP;
  if (!cr_available(func_id, impl)) return CR_E_IMPL;
  if (reps <= 0) reps = 10;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(e);
  }
  static const int BPCS[] = {2, 4, 8, 16, 32};
  constexpr int NB = sizeof(BPCS) / sizeof(BPCS[0]);
  const int nv = num_variants_of(func_id);
  // time reps launches of one configuration (after one untimed launch)
  auto time_cfg = [&](int v, int bpc, float& ms) -> int {
    int r0 = eval_cfg(func_id, impl, 0u, in, out, n, s, v, bpc);
    if (r0) return r0;
    hipError_t he = hipEventRecord(e0, s);
    for (int r = 0; r < reps && he == hipSuccess && r0 == CR_OK; r++)
      r0 = eval_cfg(func_id, impl, 0u, in, out, n, s, v, bpc);
    if (r0) return r0;
    if (he == hipSuccess) he = hipEventRecord(e1, s);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    return he == hipSuccess ? CR_OK : hip_fail(he);
  };
  // Let the clocks settle under this load (about 100 ms of it) before
  // timing: the first milliseconds of work run at lower clocks and would
  // favour whichever configuration is timed last.
  int rc = CR_OK;
  for (float busy = 0.0f; busy < 100.0f && rc == CR_OK;) {
    float ms = 0.0f;
    rc = time_cfg(0, 0, ms);
    busy += ms > 0.0f ? ms : 100.0f;
  }
  // three passes over the space, alternating in order; the median counts
  constexpr int NPASS = 3;
  std::vector<float> times((size_t)nv * NB * NPASS, 0.0f);
  for (int pass = 0; pass < NPASS && rc == CR_OK; pass++) {
    for (int c = 0; c < nv * NB && rc == CR_OK; c++) {
      const int idx = (pass & 1) ? nv * NB - 1 - c : c;
      float ms = 0.0f;
      rc = time_cfg(idx / NB, BPCS[idx % NB], ms);
      times[(size_t)idx * NPASS + pass] = ms;
    }
  }
  std::vector<float> best_of(nv * NB, 0.0f);
  for (int idx = 0; idx < nv * NB && rc == CR_OK; idx++) {
    float* t = &times[(size_t)idx * NPASS];
    std::sort(t, t + NPASS);
    best_of[idx] = t[NPASS / 2];
  }
  float best_ms = 0.0f;
  int best_v = 0, best_b = 0;
  for (int idx = 0; idx < nv * NB && rc == CR_OK; idx++) {
    if (best_ms == 0.0f || best_of[idx] < best_ms) {
      best_ms = best_of[idx];
      best_v = idx / NB;
      best_b = BPCS[idx % NB];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  const int ii = iidx(impl), fi = fidx(func_id);
  g_cfg_variant[ii][fi] = best_v;
  g_cfg_bpc[ii][fi] = best_b;
  if (best_gelem_s) *best_gelem_s = best_ms > 0 ? (double)n * reps / (best_ms * 1e-3) / 1e9 : 0.0;
  return CR_OK;
}

int cr_available(int func_id, int impl) {
  if (!func_valid(func_id)) return 0;
  if (impl == CR_IMPL_SPLIT_F32) return split_built(func_id) ? 1 : 0;
  if (impl == CR_IMPL_LOG128) return func_id == CR_LOG ? 1 : 0;
  if (impl != CR_IMPL_AUTO && impl != CR_IMPL_F64_INTERNAL) return 0;
  return func_built(func_id) ? 1 : 0;
}

int cr_eval(int func_id, const void* in, void* out, size_t n, void* stream) {
  return cr_eval_ex(func_id, CR_IMPL_AUTO, 0u, in, out, n, stream);
}

int cr_dft(const float* x, int64_t n, const float* w, int64_t m, double* X, unsigned flags,
           void* stream) {
  if (n < 0 || m < 0 || n > ((int64_t)1 << 24) || m > ((int64_t)1 << 31)) return CR_E_SIZE;
  if (m == 0) return CR_OK;
  if (!w || !X || (n > 0 && !x)) return CR_E_NULL;
  if (((uintptr_t)x % 4) || ((uintptr_t)w % 4) || ((uintptr_t)X % 16)) return CR_E_ALIGN;
  const uintptr_t xo = (uintptr_t)X, xe = xo + (uintptr_t)m * 16;
  if ((n > 0 && (uintptr_t)x < xe && xo < (uintptr_t)x + (uintptr_t)n * 4) ||
      ((uintptr_t)w < xe && xo < (uintptr_t)w + (uintptr_t)m * 4))
    return CR_E_OVERLAP;
  DevStats* st = nullptr;
  int rc = get_stats(&st);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  // samples per block: enough blocks to fill the chip (8 per CU) but at least
  // 8 samples per thread
  const long long target = (long long)num_cus() * 8;
  long long S = (target + m - 1) / m;
  const long long smax = (n + BLOCK * 8 - 1) / (BLOCK * 8);
  if (S > smax) S = smax;
  if (S < 1) S = 1;
  long long slice = (n + S - 1) / S;
  slice = (slice + BLOCK - 1) / BLOCK * BLOCK;
  if (slice < BLOCK) slice = BLOCK;
  S = n > 0 ? (n + slice - 1) / slice : 1;
  double4* part = nullptr;
  hipError_t e = hipMallocAsync((void**)&part, (size_t)m * S * sizeof(double4), s);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? CR_E_NOMEM : hip_fail(e);
  for (long long k0 = 0; k0 < m; k0 += 65535) {  // grid.y is at most 65535
    const long long mk = m - k0 < 65535 ? m - k0 : 65535;
    hipLaunchKernelGGL(k_dft, dim3((unsigned)S, (unsigned)mk), dim3(BLOCK), 0, s, x,
                       (long long)n, w + k0, slice, part + k0 * S, (int)S, st, flags, k0);
  }
  hipLaunchKernelGGL(k_dft_finish, dim3((unsigned)((m + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s,
                     part, (int)S, (long long)m, reinterpret_cast<double2*>(X));
  e = hipGetLastError();
  hipError_t e2 = hipFreeAsync(part, s);
  if (e != hipSuccess) return hip_fail(e);
  if (e2 != hipSuccess) return hip_fail(e2);
  int dev = 0;
  (void)hipGetDevice(&dev);
  g_elems[dev] += (unsigned long long)n * (unsigned long long)m;
  return CR_OK;
}


int cr_batch_plan_create(const cr_request* reqs, int32_t num, unsigned flags,
                         cr_batch_plan** plan) {
  if (!plan) return CR_E_NULL;
  *plan = nullptr;
  if (flags & CR_FLAG_ROUND_MASK) return CR_E_IMPL;  // batches round to nearest
  std::vector<BReq> hr;
  std::vector<BTile> ht;
  long long elems = 0;
  int rc = build_tables(reqs, num, hr, ht, elems);
  if (rc) return rc;
  DevStats* st = nullptr;
  rc = get_stats(&st);
  if (rc) return rc;
  cr_batch_plan* p = new cr_batch_plan();
  (void)hipGetDevice(&p->device);
  p->flags = flags;
  p->ntiles = (long long)ht.size();
  p->elems = elems;
  p->grid = (int)(p->ntiles < grid_blocks() ? p->ntiles : grid_blocks());
  hipError_t e = hipSuccess;
  if (!hr.empty()) e = hipMalloc(&p->d_reqs, hr.size() * sizeof(BReq));
  if (e == hipSuccess && !ht.empty()) e = hipMalloc(&p->d_tiles, ht.size() * sizeof(BTile));
  if (e != hipSuccess) {
    t_last_hip = (int)e;
    cr_batch_plan_destroy(p);
    return CR_E_NOMEM;
  }
  if (!hr.empty()) e = hipMemcpy(p->d_reqs, hr.data(), hr.size() * sizeof(BReq), hipMemcpyHostToDevice);
  if (e == hipSuccess && !ht.empty())
    e = hipMemcpy(p->d_tiles, ht.data(), ht.size() * sizeof(BTile), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming);
  // Capture the launches in a graph (private streams at default priority).
  // The per-function kernels are spread over NBRANCH parallel branches (a
  // fork from the origin stream and a join back to it) so that one kernel's
  // tail overlaps the next kernel's start.
  if (e == hipSuccess && p->grid > 0) {
    constexpr int NBRANCH = 4;
    hipStream_t cs = nullptr, side[NBRANCH] = {};
    hipEvent_t fork = nullptr, join[NBRANCH] = {};
    hipGraph_t g = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    for (int b = 0; b < NBRANCH && e == hipSuccess; b++) {
      e = hipStreamCreateWithFlags(&side[b], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&join[b], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t ec = hipEventRecord(fork, cs);
      for (int b = 0; b < NBRANCH && ec == hipSuccess; b++)
        ec = hipStreamWaitEvent(side[b], fork, 0);
      int rc2 = CR_OK, i = 0;
      if (ec == hipSuccess)
        for (const BRange& g2 : key_ranges(hr, ht))
          if (rc2 == CR_OK)
            rc2 = launch_tiles(p->d_reqs, p->d_tiles, g2, st, flags, side[i++ % NBRANCH]);
      for (int b = 0; b < NBRANCH && ec == hipSuccess; b++) {
        ec = hipEventRecord(join[b], side[b]);
        if (ec == hipSuccess) ec = hipStreamWaitEvent(cs, join[b], 0);
      }
      hipError_t e2 = hipStreamEndCapture(cs, &g);
      e = hipGetLastError();
      if (e == hipSuccess) e = ec;
      if (e == hipSuccess) e = e2;
      if (e == hipSuccess && rc2 != CR_OK) e = hipErrorInvalidValue;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (fork) (void)hipEventDestroy(fork);
    for (int b = 0; b < NBRANCH; b++) {
      if (join[b]) (void)hipEventDestroy(join[b]);
      if (side[b]) (void)hipStreamDestroy(side[b]);
    }
    if (cs) (void)hipStreamDestroy(cs);
  }
  if (e != hipSuccess) {
    t_last_hip = (int)e;
    cr_batch_plan_destroy(p);
    return CR_E_HIP;
  }
  *plan = p;
  return CR_OK;
}

int cr_batch_plan_launch(cr_batch_plan* plan, void* stream) {
  if (!plan) return CR_E_NULL;
  hipStream_t s = (hipStream_t)stream;
  if (plan->exec) {
    hipError_t e = hipGraphLaunch(plan->exec, s);
    if (e == hipSuccess) e = hipEventRecord(plan->done, s);
    if (e != hipSuccess) return hip_fail(e);
    plan->launched = true;
    g_elems[plan->device] += plan->elems;
  }
  return CR_OK;
}

int cr_batch_plan_destroy(cr_batch_plan* plan) {
  if (!plan) return CR_OK;
  if (plan->launched && plan->done) (void)hipEventSynchronize(plan->done);
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->done) (void)hipEventDestroy(plan->done);
  if (plan->d_reqs) (void)hipFree(plan->d_reqs);
  if (plan->d_tiles) (void)hipFree(plan->d_tiles);
  delete plan;
  return CR_OK;
}

int cr_eval_batch(const cr_request* reqs, int32_t num, void* stream) {
  std::vector<BReq> hr;
  std::vector<BTile> ht;
  long long elems = 0;
  int rc = build_tables(reqs, num, hr, ht, elems);
  if (rc) return rc;
  if (ht.empty()) return CR_OK;
  DevStats* st = nullptr;
  rc = get_stats(&st);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  BReq* dr = nullptr;
  BTile* dt = nullptr;
  hipError_t e = hipMallocAsync((void**)&dr, hr.size() * sizeof(BReq), s);
  if (e == hipSuccess) e = hipMallocAsync((void**)&dt, ht.size() * sizeof(BTile), s);
  if (e != hipSuccess) {
    if (dt) (void)hipFreeAsync(dt, s);
    if (dr) (void)hipFreeAsync(dr, s);
    t_last_hip = (int)e;
    return CR_E_NOMEM;
  }
  e = hipMemcpyAsync(dr, hr.data(), hr.size() * sizeof(BReq), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dt, ht.data(), ht.size() * sizeof(BTile), hipMemcpyHostToDevice, s);
  // the host vectors are freed on return: make sure the copies have read them
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) {
    for (const BRange& g : key_ranges(hr, ht)) (void)launch_tiles(dr, dt, g, st, 0u, s);
    e = hipGetLastError();
  }
  (void)hipFreeAsync(dt, s);
  (void)hipFreeAsync(dr, s);
  if (e != hipSuccess) return hip_fail(e);
  int dev = 0;
  (void)hipGetDevice(&dev);
  g_elems[dev] += elems;
  return CR_OK;
}

int cr_eval_batch_noalloc(const cr_request* reqs, int32_t num, void* stream) {
  if (num > CR_NOALLOC_MAX_REQUESTS) return CR_E_SCRATCH;
  std::vector<BReq> hr;
  std::vector<BTile> ht;
  long long elems = 0;
  int rc = build_tables(reqs, num, hr, ht, elems);
  if (rc) return rc;
  if (ht.empty()) return CR_OK;
  if (hr.size() > (size_t)CR_NOALLOC_MAX_REQUESTS || ht.size() > (size_t)CR_NOALLOC_MAX_TILES)
    return CR_E_SCRATCH;
  DevState* ds = nullptr;
  rc = get_state(&ds);
  if (rc) return rc;
  BReq* dr = reinterpret_cast<BReq*>(ds->scratch);
  BTile* dt = reinterpret_cast<BTile*>(ds->scratch + NOALLOC_REQ_BYTES);
  hipStream_t s = (hipStream_t)stream;
  // stream-ordered after earlier work on s (including an earlier call's
  // kernels still reading the tables); the host vectors are freed on return,
  // so wait until the copies have read them
  hipError_t e = hipMemcpyAsync(dr, hr.data(), hr.size() * sizeof(BReq), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dt, ht.data(), ht.size() * sizeof(BTile), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) {
    for (const BRange& g : key_ranges(hr, ht)) (void)launch_tiles(dr, dt, g, ds->stats, 0u, s);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return hip_fail(e);
  int dev = 0;
  (void)hipGetDevice(&dev);
  g_elems[dev] += elems;
  return CR_OK;
}

int cr_stats_reset(void* stream) {
  DevStats* st = nullptr;
  int rc = get_stats(&st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_zero_stats, dim3(1), dim3(256), 0, (hipStream_t)stream, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e);
  int dev = 0;
  (void)hipGetDevice(&dev);
  g_elems[dev] = 0;
  return CR_OK;
}

int cr_stats_read(void* stream, cr_stats* out) {
  if (!out) return CR_E_NULL;
  DevStats* st = nullptr;
  int rc = get_stats(&st);
  if (rc) return rc;
  DevStats* h = new DevStats;
  hipError_t e = hipMemcpyAsync(h, st, sizeof(DevStats), hipMemcpyDeviceToHost,
                                (hipStream_t)stream);
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e);
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  out->elems = g_elems[dev];
  out->fallback_lanes = out->fallback_waves = 0;
  for (int i = 0; i < NSLOT; i++) {
    out->fallback_lanes += h->slot[i].fallback_lanes;
    out->fallback_waves += h->slot[i].fallback_waves;
  }
  out->escapes = h->escapes;
  for (int i = 0; i < 16; i++) out->escape_index[i] = h->escape_index[i];
  delete h;
  return CR_OK;
}

const char* cr_status_str(int status) {
  switch (status) {
    case CR_OK: return "ok";
    case CR_E_FUNC: return "unknown function id";
    case CR_E_NULL: return "null pointer";
    case CR_E_OVERLAP: return "input and output overlap";
    case CR_E_ALIGN: return "pointer not aligned to its element size";
    case CR_E_IMPL: return "implementation not available";
    case CR_E_HIP: return "HIP runtime error";
    case CR_E_NOMEM: return "device allocation failed";
    case CR_E_SIZE: return "size too large";
    case CR_E_TUNE: return "invalid launch configuration or tuning file";
    case CR_E_SCRATCH: return "batch exceeds the static scratch of cr_eval_batch_noalloc";
  }
  return "unknown status";
}

int cr_last_hip_error(void) { return t_last_hip; }

}  // extern "C"
