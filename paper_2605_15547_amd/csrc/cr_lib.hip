// cr_lib.hip -- kernels and the C ABI of libcr (gfx950).
//
// One elementwise map kernel per function (a template over the function's
// evaluator).  Each workgroup stages the function's <= 16-entry tables in LDS
// once, then each thread loads U float4 vectors (128-bit, coalesced: lane i of
// a wave touches bytes [16 i, 16 i + 16) of a contiguous 1 KiB span), evaluates
// the 4U elements and stores U float4 vectors.  Pointers that are not 16-byte
// aligned, and ragged tails, go through a scalar grid-stride kernel.
#include <hip/hip_runtime.h>

#include <stdlib.h>

#include <atomic>
#include <mutex>

#include "../../include/cr.h"
#include "cr_f32_exp.h"
#include "cr_f32_log.h"
#include "cr_f32_rsqrt.h"
#include "cr_f32_trig.h"
#include "cr_f32_atan.h"
#include "cr_f32_hyp.h"

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
constexpr int TILE_U = CR_TILE_U;           // float4 vectors per thread per tile
constexpr int TILE = BLOCK * 4 * TILE_U;    // 2048 elements per tile
constexpr int QCAP = 512;                   // deferred elements held in LDS
constexpr int QCHECK = 8;                   // tiles between two looks at the queue
constexpr int QFLUSH = QCAP / 2;            // flush when the queue is fuller than this

// ------------------------------------------------------------ evaluators
// Op::fast(x, tab, ok): binary64 fast path and rounding test (inlined).
// Op::accurate(x, tab): double-double path from x alone (out of line).
template <int K>
struct OpExp {
  using Tab = ExpTab;
  static __device__ __forceinline__ void load(Tab& t, int tid) { exp_tab_load(t, tid); }
  static __device__ __forceinline__ float fast(float x, const Tab& t, bool& ok) {
    return exp_fast<K>(x, t, ok);
  }
  static __device__ __forceinline__ AccResult accurate(float x, const Tab& t) {
    return exp_accurate<K>(x, t);
  }
};

template <int K>
struct OpLog {
  using Tab = LogTab;
  static __device__ __forceinline__ void load(Tab& t, int tid) { log_tab_load<K>(t, tid); }
  static __device__ __forceinline__ float fast(float x, const Tab& t, bool& ok) {
    return log_fast<K>(x, t, ok);
  }
  static __device__ __forceinline__ AccResult accurate(float x, const Tab& t) {
    return log_accurate<K>(x, t);
  }
};

// rsqrtf decides its rounding exactly in the fast path: nothing is deferred.
struct OpRsqrt {
  using Tab = NoTab;
  static __device__ __forceinline__ void load(Tab&, int) {}
  static __device__ __forceinline__ float fast(float x, const Tab&, bool& ok) {
    return rsqrt_fast(x, ok);
  }
  static __device__ __noinline__ AccResult accurate(float x, const Tab&) {
    bool ok;
    return {rsqrt_fast(x, ok), 1};
  }
};

template <int KIND>
struct OpTrig {
  using Tab = TrigTab;
  static __device__ __forceinline__ void load(Tab& t, int tid) { trig_tab_load(t, tid); }
  static __device__ __forceinline__ float fast(float x, const Tab& t, bool& ok) {
    return trig_fast<KIND>(x, t, ok);
  }
  static __device__ __forceinline__ AccResult accurate(float x, const Tab& t) {
    return trig_accurate<KIND>(x, t);
  }
};

template <int KIND>
struct OpAtan {
  using Tab = AtanTab;
  static __device__ __forceinline__ void load(Tab& t, int tid) { atan_tab_load(t, tid); }
  static __device__ __forceinline__ float fast(float x, const Tab& t, bool& ok) {
    return atan_fast<KIND>(x, t, ok);
  }
  static __device__ __forceinline__ AccResult accurate(float x, const Tab& t) {
    return atan_accurate<KIND>(x, t);
  }
};

template <int KIND>
struct OpHyp {
  using Tab = ExpTab;
  static __device__ __forceinline__ void load(Tab& t, int tid) { exp_tab_load(t, tid); }
  static __device__ __forceinline__ float fast(float x, const Tab& t, bool& ok) {
    return hyp_fast<KIND>(x, t, ok);
  }
  static __device__ __forceinline__ AccResult accurate(float x, const Tab& t) {
    return hyp_accurate<KIND>(x, t);
  }
};

// Block-level bookkeeping of the accurate path, kept in LDS.
struct Deferred {
  unsigned n;                 // entries in the queue
  unsigned lanes, waves, esc; // counters of this workgroup
  unsigned idx[QCAP];         // element index (relative to the launch)
  float x[QCAP];              // the input value (the output may alias it)
};

__device__ __forceinline__ void note_escape(DevStats* st, long long idx) {
  unsigned long long slot = atomicAdd(&st->escapes, 1ull);
  if (slot < 16) st->escape_index[slot] = (unsigned long long)idx;
}

// Run the accurate path on every queued element, 256 at a time (whole waves),
// then empty the queue.  Called by all threads of the block.
template <class Op>
__device__ __noinline__ void flush_queue(Deferred& q, const typename Op::Tab& tab, float* out,
                                         DevStats* st, long long elem_base) {
  // q.n counts every enqueue attempt; entries past QCAP were never stored
  // (those elements took the accurate path in place), so only QCAP are valid
  unsigned n = q.n < QCAP ? q.n : QCAP;
  for (unsigned k = threadIdx.x; k < n; k += BLOCK) {
    AccResult a = Op::accurate(q.x[k], tab);
    out[q.idx[k]] = a.r;
    if (!a.ok) {
      atomicAdd(&q.esc, 1u);
      note_escape(st, elem_base + q.idx[k]);
    }
  }
  if (threadIdx.x == 0) {
    q.lanes += n;
    q.waves += (n + 63) / 64;
  }
  __syncthreads();
  if (threadIdx.x == 0) q.n = 0;
  __syncthreads();
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
template <class Op>
__global__ void __launch_bounds__(BLOCK)
    k_map_f32(const float4* in, float4* out, long long n4, DevStats* st,
              unsigned flags, long long elem_base) {
  __shared__ typename Op::Tab tab;
  __shared__ Deferred q;
  Op::load(tab, threadIdx.x);
  if (threadIdx.x == 0) {
    q.n = 0;
    q.lanes = q.waves = q.esc = 0;
  }
  __syncthreads();
  const bool force = flags & CR_FLAG_FORCE_FALLBACK;
  float* outf = reinterpret_cast<float*>(out);
  const long long ntiles = (n4 + BLOCK * TILE_U - 1) / (BLOCK * TILE_U);
  // software pipelining: the next tile's vectors are loaded while this tile
  // is evaluated
  float4 nxt[TILE_U];
  if (CR_PREFETCH) {
    long long base = (long long)blockIdx.x * (BLOCK * TILE_U) + threadIdx.x;
#pragma unroll
    for (int u = 0; u < TILE_U; u++) {
      long long i = base + (long long)u * BLOCK;
      if (i < n4) nxt[u] = in[i];
    }
  }
  int iter = 0;
  for (long long t = blockIdx.x; t < ntiles; t += gridDim.x, iter++) {
    long long base = t * (BLOCK * TILE_U) + threadIdx.x;
    float4 v[TILE_U];
    if (CR_PREFETCH) {
#pragma unroll
      for (int u = 0; u < TILE_U; u++) v[u] = nxt[u];
    } else {
#pragma unroll
      for (int u = 0; u < TILE_U; u++) {
        long long i = base + (long long)u * BLOCK;
        if (i < n4) v[u] = in[i];
      }
    }
    if (CR_PREFETCH) {
      long long nb = (t + gridDim.x) * (BLOCK * TILE_U) + threadIdx.x;
#pragma unroll
      for (int u = 0; u < TILE_U; u++) {
        long long i = nb + (long long)u * BLOCK;
        if (i < n4) nxt[u] = in[i];
      }
    }
#pragma unroll
    for (int u = 0; u < TILE_U; u++) {
      long long i = base + (long long)u * BLOCK;
      if (i < n4) {
        float* e = reinterpret_cast<float*>(&v[u]);
#pragma unroll
        for (int c = 0; c < 4; c++) {
          bool ok;
          float x = e[c];
          e[c] = Op::fast(x, tab, ok);
          if (!ok || force) {
            unsigned pos = atomicAdd(&q.n, 1u);
            if (pos < QCAP) {
              q.idx[pos] = (unsigned)(4 * i + c);
              q.x[pos] = x;
            } else {  // queue full (only with pathological inputs or force)
              AccResult a = Op::accurate(x, tab);
              e[c] = a.r;
              atomicAdd(&q.lanes, 1u);
              if (!a.ok) {
                atomicAdd(&q.esc, 1u);
                note_escape(st, elem_base + 4 * i + c);
              }
            }
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < TILE_U; u++) {
      long long i = base + (long long)u * BLOCK;
      if (i < n4) out[i] = v[u];
    }
    if (iter % QCHECK == QCHECK - 1) {
      // every thread must see the same fill level: read it between two
      // barriers (no thread can queue more elements before all have read it)
      __syncthreads();
      const unsigned nq = q.n;
      __syncthreads();
      if (nq > QFLUSH) flush_queue<Op>(q, tab, outf, st, elem_base);
    }
  }
  __syncthreads();
  // after the barrier above nothing else changes q.n: uniform
  if (q.n) flush_queue<Op>(q, tab, outf, st, elem_base);
  if (threadIdx.x == 0 && q.lanes) {
    CounterSlot& c = st->slot[blockIdx.x % NSLOT];
    atomicAdd(&c.fallback_lanes, (unsigned long long)q.lanes);
    atomicAdd(&c.fallback_waves, (unsigned long long)q.waves);
  }
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

// sincosf: the map kernel with two planar outputs (sin block, cos block), both
// 16-byte aligned (the host checks; otherwise the scalar form below runs).
__device__ __noinline__ void flush_queue_sincos(Deferred& q, const TrigTab& tab, float* os,
                                                float* oc, DevStats* st, long long elem_base) {
  unsigned n = q.n < QCAP ? q.n : QCAP;
  for (unsigned k = threadIdx.x; k < n; k += BLOCK) {
    AccResult2 a = sincos_accurate(q.x[k], tab);
    os[q.idx[k]] = a.s;
    oc[q.idx[k]] = a.c;
    if (!a.ok) {
      atomicAdd(&q.esc, 1u);
      note_escape(st, elem_base + q.idx[k]);
    }
  }
  if (threadIdx.x == 0) {
    q.lanes += n;
    q.waves += (n + 63) / 64;
  }
  __syncthreads();
  if (threadIdx.x == 0) q.n = 0;
  __syncthreads();
}

__global__ void __launch_bounds__(BLOCK)
    k_map_sincos(const float4* in, float4* outs, float4* outc, long long n4, DevStats* st,
                 unsigned flags, long long elem_base) {
  __shared__ TrigTab tab;
  __shared__ Deferred q;
  trig_tab_load(tab, threadIdx.x);
  if (threadIdx.x == 0) {
    q.n = 0;
    q.lanes = q.waves = q.esc = 0;
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
      if (i < n4) v[u] = in[i];
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
          e[c] = sincos_fast(x, tab, ec[c], ok);
          if (!ok || force) {
            unsigned pos = atomicAdd(&q.n, 1u);
            if (pos < QCAP) {
              q.idx[pos] = (unsigned)(4 * i + c);
              q.x[pos] = x;
            } else {
              AccResult2 a = sincos_accurate(x, tab);
              e[c] = a.s;
              ec[c] = a.c;
              atomicAdd(&q.lanes, 1u);
              if (!a.ok) {
                atomicAdd(&q.esc, 1u);
                note_escape(st, elem_base + 4 * i + c);
              }
            }
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < TILE_U; u++) {
      long long i = base + (long long)u * BLOCK;
      if (i < n4) {
        outs[i] = v[u];
        outc[i] = c4[u];
      }
    }
    if (iter % QCHECK == QCHECK - 1) {
      __syncthreads();
      const unsigned nq = q.n;
      __syncthreads();
      if (nq > QFLUSH)
        flush_queue_sincos(q, tab, reinterpret_cast<float*>(outs), reinterpret_cast<float*>(outc),
                           st, elem_base);
    }
  }
  __syncthreads();
  if (q.n)
    flush_queue_sincos(q, tab, reinterpret_cast<float*>(outs), reinterpret_cast<float*>(outc), st,
                       elem_base);
  if (threadIdx.x == 0 && q.lanes) {
    CounterSlot& c = st->slot[blockIdx.x % NSLOT];
    atomicAdd(&c.fallback_lanes, (unsigned long long)q.lanes);
    atomicAdd(&c.fallback_waves, (unsigned long long)q.waves);
  }
}

__global__ void __launch_bounds__(BLOCK)
    k_map_sincos_scalar(const float* in, float* outs, float* outc, long long n, DevStats* st,
                        unsigned flags, long long elem_base) {
  __shared__ TrigTab tab;
  trig_tab_load(tab, threadIdx.x);
  __syncthreads();
  const bool force = flags & CR_FLAG_FORCE_FALLBACK;
  unsigned lanes = 0;
  for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n;
       i += (long long)gridDim.x * BLOCK) {
    bool ok;
    float x = in[i], c;
    float s = sincos_fast(x, tab, c, ok);
    if (!ok || force) {
      AccResult2 a = sincos_accurate(x, tab);
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

__global__ void k_zero_stats(DevStats* st) {
  unsigned long long* p = reinterpret_cast<unsigned long long*>(st);
  for (int i = threadIdx.x; i < (int)(sizeof(DevStats) / 8); i += blockDim.x) p[i] = 0;
}

// ------------------------------------------------------------- host side
constexpr int MAX_DEV = 64;
std::mutex g_mu;
DevStats* g_stats[MAX_DEV];
std::atomic<unsigned long long> g_elems[MAX_DEV];
thread_local int t_last_hip = 0;

int hip_fail(hipError_t e) {
  t_last_hip = (int)e;
  return CR_E_HIP;
}

int get_stats(DevStats** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e);
  if (dev < 0 || dev >= MAX_DEV) return CR_E_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_stats[dev]) {
    DevStats* p = nullptr;
    e = hipMalloc(&p, sizeof(DevStats));
    if (e != hipSuccess) {
      t_last_hip = (int)e;
      return CR_E_NOMEM;
    }
    e = hipMemset(p, 0, sizeof(DevStats));
    if (e != hipSuccess) return hip_fail(e);
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e);
    g_stats[dev] = p;
  }
  *out = g_stats[dev];
  return CR_OK;
}

int g_grid_blocks = 0;  // persistent grid size (workgroups), set on first use

int grid_blocks() {
  if (!g_grid_blocks) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int per = CR_BLOCKS_PER_CU;
    if (const char* e = getenv("CR_BLOCKS_PER_CU")) per = atoi(e);
    if (per < 1) per = 1;
    if (per > 64) per = 64;
    g_grid_blocks = cus * per;
  }
  return g_grid_blocks;
}

template <class Op>
int launch_map_f32(const float* in, float* out, size_t n, hipStream_t s, unsigned flags,
                   DevStats* st) {
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
    size_t tiles = (chunk4 + BLOCK * TILE_U - 1) / (BLOCK * TILE_U);
    size_t g = tiles < (size_t)grid_blocks() ? tiles : (size_t)grid_blocks();
    size_t off = head + 4 * done;
    hipLaunchKernelGGL(k_map_f32<Op>, dim3((unsigned)g), dim3(BLOCK), 0, s,
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

int launch_sincos(const float* in, float* out, size_t n, hipStream_t s, unsigned flags,
                  DevStats* st) {
  float* outc = out + n;
  uintptr_t ai = (uintptr_t)in, ao = (uintptr_t)out, ac = (uintptr_t)outc;
  bool vec = (ai & 15) == 0 && (ao & 15) == 0 && (ac & 15) == 0;
  size_t body4 = vec ? n / 4 : 0;
  size_t done4 = 0;
  while (done4 < body4) {
    size_t chunk4 = body4 - done4;
    if (chunk4 > ((size_t)1 << 29)) chunk4 = (size_t)1 << 29;
    size_t tiles = (chunk4 + BLOCK * TILE_U - 1) / (BLOCK * TILE_U);
    size_t g = tiles < (size_t)grid_blocks() ? tiles : (size_t)grid_blocks();
    size_t off = 4 * done4;
    hipLaunchKernelGGL(k_map_sincos, dim3((unsigned)g), dim3(BLOCK), 0, s,
                       reinterpret_cast<const float4*>(in + off),
                       reinterpret_cast<float4*>(out + off), reinterpret_cast<float4*>(outc + off),
                       (long long)chunk4, st, flags, (long long)off);
    done4 += chunk4;
  }
  size_t off = 4 * body4;
  if (off < n) {
    size_t rest = n - off;
    size_t g = (rest + BLOCK - 1) / BLOCK;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_map_sincos_scalar, dim3((unsigned)g), dim3(BLOCK), 0, s, in + off,
                       out + off, outc + off, (long long)rest, st, flags, (long long)off);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e);
  return CR_OK;
}

bool func_valid(int f) { return (f >= 0 && f < CR_NUM_F32) || f == CR_EXP || f == CR_LOG; }
bool func_built(int f) { return f >= CR_EXPF && f <= CR_TANHF; }

int dispatch_f32(int f, const float* in, float* out, size_t n, hipStream_t s, unsigned flags,
                 DevStats* st) {
  switch (f) {
    case CR_EXPF: return launch_map_f32<OpExp<EXPK_E>>(in, out, n, s, flags, st);
    case CR_EXP2F: return launch_map_f32<OpExp<EXPK_2>>(in, out, n, s, flags, st);
    case CR_EXP10F: return launch_map_f32<OpExp<EXPK_10>>(in, out, n, s, flags, st);
    case CR_EXPM1F: return launch_map_f32<OpExp<EXPK_EM1>>(in, out, n, s, flags, st);
    case CR_LOGF: return launch_map_f32<OpLog<LOGK_E>>(in, out, n, s, flags, st);
    case CR_LOG2F: return launch_map_f32<OpLog<LOGK_2>>(in, out, n, s, flags, st);
    case CR_LOG10F: return launch_map_f32<OpLog<LOGK_10>>(in, out, n, s, flags, st);
    case CR_LOG1PF: return launch_map_f32<OpLog<LOGK_1P>>(in, out, n, s, flags, st);
    case CR_RSQRTF: return launch_map_f32<OpRsqrt>(in, out, n, s, flags, st);
    case CR_SINF: return launch_map_f32<OpTrig<TRIGK_SIN>>(in, out, n, s, flags, st);
    case CR_COSF: return launch_map_f32<OpTrig<TRIGK_COS>>(in, out, n, s, flags, st);
    case CR_TANF: return launch_map_f32<OpTrig<TRIGK_TAN>>(in, out, n, s, flags, st);
    case CR_SINCOSF: return launch_sincos(in, out, n, s, flags, st);
    case CR_ASINF: return launch_map_f32<OpAtan<ATANK_ASIN>>(in, out, n, s, flags, st);
    case CR_ACOSF: return launch_map_f32<OpAtan<ATANK_ACOS>>(in, out, n, s, flags, st);
    case CR_ATANF: return launch_map_f32<OpAtan<ATANK_ATAN>>(in, out, n, s, flags, st);
    case CR_SINHF: return launch_map_f32<OpHyp<HYPK_SINH>>(in, out, n, s, flags, st);
    case CR_COSHF: return launch_map_f32<OpHyp<HYPK_COSH>>(in, out, n, s, flags, st);
    case CR_TANHF: return launch_map_f32<OpHyp<HYPK_TANH>>(in, out, n, s, flags, st);
  }
  return CR_E_FUNC;
}

}  // namespace

extern "C" {

int cr_available(int func_id, int impl);

int cr_eval_ex(int func_id, int impl, unsigned flags, const void* in, void* out, size_t n,
               void* stream) {
  if (!func_valid(func_id)) return CR_E_FUNC;
  if (impl != CR_IMPL_AUTO && impl != CR_IMPL_F64_INTERNAL && impl != CR_IMPL_SPLIT_F32)
    return CR_E_IMPL;
  if (n == 0) return CR_OK;
  if (!in || !out) return CR_E_NULL;
  const size_t es = func_id >= 64 ? 8 : 4;
  const size_t nout = func_id == CR_SINCOSF ? 2 * n : n;
  if (n > ((size_t)1 << 60)) return CR_E_SIZE;
  uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
  if ((a % es) || (b % es)) return CR_E_ALIGN;
  bool same = a == b && nout == n;
  if (!same && a < b + nout * es && b < a + n * es) return CR_E_OVERLAP;
  if (!cr_available(func_id, impl)) return CR_E_IMPL;
  DevStats* st = nullptr;
  int rc = get_stats(&st);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (func_id < CR_NUM_F32)
    rc = dispatch_f32(func_id, (const float*)in, (float*)out, n, s, flags, st);
  else
    rc = CR_E_IMPL;
  if (rc == CR_OK) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    g_elems[dev] += n;
  }
  return rc;
}

int cr_available(int func_id, int impl) {
  if (!func_valid(func_id)) return 0;
  if (impl != CR_IMPL_AUTO && impl != CR_IMPL_F64_INTERNAL) return 0;
  return func_built(func_id) ? 1 : 0;
}

int cr_eval(int func_id, const void* in, void* out, size_t n, void* stream) {
  return cr_eval_ex(func_id, CR_IMPL_AUTO, 0u, in, out, n, stream);
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
  }
  return "unknown status";
}

int cr_last_hip_error(void) { return t_last_hip; }

}  // extern "C"
