/*
 * cr.h -- correctly rounded elementwise math on AMD Instinct MI355X (gfx950).
 *
 * The library evaluates one-input functions correctly rounded to nearest
 * (ties to even), element by element, on the GPU: the 19 single precision
 * functions the paper lists (Sec. II-A: acosf, asinf, atanf, cosf, coshf,
 * expf, exp2f, exp10f, expm1f, log10f, log1pf, log2f, logf, sincosf, sinf,
 * sinhf, rsqrtf, tanf, tanhf) and double precision exp2 and log (the
 * functions the paper studies in Sec. II-B; exp2 with the paper's three
 * 16-entry tables) plus double precision exp.  "Correctly rounded" means the
 * result is RN(f(x)) for the exact real f(x) (paper, Sec. I).  Only round-to-nearest-even is provided,
 * as in the paper's GPU experiments (Sec. III-C).
 *
 * Conventions shared by every entry point:
 *  - in/out are DEVICE pointers owned by the caller, on the current HIP
 *    device; the stream argument is a hipStream_t (NULL = default stream).
 *  - element type follows func_id: float for ids 0..18, double for 64..66,
 *    complex float pairs for 80..82; n counts input elements.  sincosf
 *    writes 2n floats, planar: out[0..n) = sin(in), out[n..2n) = cos(in).
 *  - n == 0 returns CR_OK without launching anything.
 *  - in == out (in place) is allowed for single-output functions; any other
 *    overlap of the input and output ranges is CR_E_OVERLAP.
 *  - pointers must be aligned to their element size (CR_E_ALIGN); 16-byte
 *    alignment is not required.
 *  - calls are asynchronous and stream-ordered: the return code reports
 *    argument and launch errors only; device faults surface at stream
 *    synchronisation as usual in HIP.  Entry points never abort or set errno.
 *  - special inputs follow IEEE 754-2019 Sec. 9.2: NaN inputs return the same
 *    NaN quieted (sign and payload kept); invalid operations on non-NaN
 *    inputs return the default quiet NaN 0x7fc00000 / 0x7ff8000000000000.
 *    Subnormal inputs and outputs are fully supported (no flush to zero).
 *  - no floating-point status flags are raised (the paper's SIMD libraries
 *    do not aim to set them either, Sec. II-A).
 */
#ifndef CR_H
#define CR_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum cr_func {
  CR_EXPF = 0, CR_EXP2F = 1, CR_EXP10F = 2, CR_EXPM1F = 3,
  CR_LOGF = 4, CR_LOG2F = 5, CR_LOG10F = 6, CR_LOG1PF = 7,
  CR_RSQRTF = 8,
  CR_SINF = 9, CR_COSF = 10, CR_SINCOSF = 11, CR_TANF = 12,
  CR_ASINF = 13, CR_ACOSF = 14, CR_ATANF = 15,
  CR_SINHF = 16, CR_COSHF = 17, CR_TANHF = 18,
  CR_NUM_F32 = 19,
  CR_EXP = 64, CR_LOG = 65, /* binary64 */
  /* binary64 exp2 (paper, Sec. II-B): x = (4096 m + 256 i1 + 16 i2 + i3)/4096 + R,
   * 2^x = 2^m T1[i1] T2[i2] T3[i3] 2^R with three 16-entry double-double tables */
  CR_EXP2 = 66,
  /* Complex binary32 functions accurate to 2 ulps on valid inputs, built from
   * the correctly rounded real functions (the paper's second application
   * benchmark, Sec. III-A).  Elements are complex numbers stored as
   * interleaved (re, im) float pairs; n counts complex numbers; in and out
   * need 4-byte alignment.  Each part is computed as stated, every correctly
   * rounded ingredient bit-exact and every other step one IEEE operation:
   *   cexpf: re = RN32(expf(x) cosf(y)), im = RN32(expf(x) sinf(y));
   *          valid for finite x < 88.7 and finite y
   *   csinf: re = RN32(sinf(x) coshf(y)), im = RN32(cosf(x) sinhf(y));
   *          valid for finite x and |y| < 89.4
   *   clogf: re = log|z| from logf or log1pf (near |z| = 1) plus a binary64
   *          correction, im = atan2(y, x) from atanf(min/max) and binary64
   *          reflections by pi/2 and pi; valid for finite z with
   *          2^-63 <= |z| < 2^63 (below 1.5 ulps).
   * Outside the valid inputs the results are those of the same IEEE
   * operations (NaN signs and payloads unspecified).  CR_IMPL_AUTO or
   * CR_IMPL_F64_INTERNAL only. */
  CR_CEXPF = 80, CR_CLOGF = 81, CR_CSINF = 82
};

/* Implementation choice for the binary32 functions (paper, Sec. II-A: the
 * paper's kernels compute in binary64 internally; Sec. II-A and IV propose a
 * single precision fast path for GPUs with weak binary64). */
enum cr_impl {
  CR_IMPL_AUTO = 0,         /* library default (currently F64_INTERNAL) */
  CR_IMPL_F64_INTERNAL = 1, /* binary64 fast path + double-double accurate path */
  CR_IMPL_SPLIT_F32 = 2,    /* binary32 arithmetic only, no binary64 operation: a
                             * float-float fast path, and a triple-float accurate step
                             * for the lanes that fail its rounding test (same results
                             * as F64_INTERNAL).  Round to nearest only.  Built for the
                             * functions where cr_available(f, CR_IMPL_SPLIT_F32) is 1;
                             * the others give CR_E_IMPL */
  CR_IMPL_LOG128 = 3        /* CR_LOG only: the paper's cr_log main path (Sec. II-B) with
                             * one 128-entry table of scaled 64-bit integers, T_j =
                             * log1p(r_j)/r_j - 1 for the 128 reciprocals r_j + 1 of 8
                             * significant bits; failing lanes take the same accurate path
                             * as the default (16-entry) log.  Same results, another
                             * speed; the launch configuration is the default log's. */
};

enum cr_flag {
  /* every element also takes the accurate path (testing aid); results are
   * identical by construction, only slower */
  CR_FLAG_FORCE_FALLBACK = 1u,
  /* Rounding mode of the results (IEEE 754-2019 Sec. 4.3; the paper's CPU
   * library supports every mode, Sec. II-A, its GPU runs were round to
   * nearest only, Sec. III-C).  Default (none of these): to nearest, ties to
   * even.  Toward zero / +infinity / -infinity are available for the binary32
   * functions (ids 0..18) with CR_IMPL_AUTO or CR_IMPL_F64_INTERNAL through
   * cr_eval_ex; other functions and implementations, and batch plans, return
   * CR_E_IMPL.  Overflow gives +-infinity or +-FLT_MAX as the mode
   * says (Sec. 7.4); results that round to zero keep their sign.  Each
   * element takes a double-double evaluation (about 2^-100 relative) with
   * both ends of its error interval rounded in the mode, so these modes run
   * at the accurate path's speed. */
  CR_FLAG_ROUND_TOWARD_ZERO = 1u << 4,
  CR_FLAG_ROUND_UP = 2u << 4,
  CR_FLAG_ROUND_DOWN = 3u << 4
};
#define CR_FLAG_ROUND_SHIFT 4
#define CR_FLAG_ROUND_MASK (3u << CR_FLAG_ROUND_SHIFT)

enum cr_status {
  CR_OK = 0,
  CR_E_FUNC = -1,    /* unknown func_id */
  CR_E_NULL = -2,    /* NULL pointer with n > 0 */
  CR_E_OVERLAP = -3, /* input and output overlap (other than exact in-place) */
  CR_E_ALIGN = -4,   /* pointer not aligned to its element size */
  CR_E_IMPL = -5,    /* unknown or unavailable implementation */
  CR_E_HIP = -6,     /* a HIP runtime call failed; see cr_last_hip_error() */
  CR_E_NOMEM = -7,   /* device allocation of library state failed */
  CR_E_SIZE = -9,    /* n too large */
  CR_E_TUNE = -10,   /* invalid launch configuration, or unreadable/malformed tuning file */
  CR_E_SCRATCH = -11 /* batch larger than the static scratch of cr_eval_batch_noalloc */
};

/* out[i] = RN(f(in[i])) for i < n, func = func_id, default implementation.
 * Paper, Sec. II-A (binary32) and Sec. II-B (binary64). */
int cr_eval(int func_id, const void *in, void *out, size_t n, void *stream);

/* As cr_eval, with an explicit implementation (enum cr_impl) and flags
 * (enum cr_flag). */
int cr_eval_ex(int func_id, int impl, unsigned flags, const void *in, void *out, size_t n,
               void *stream);

/* 1 if func_id is provided with implementation impl (enum cr_impl) by this
 * build of the library, else 0. */
int cr_available(int func_id, int impl);

/* Spectral interpolation by a brute-force discrete Fourier transform of real
 * samples (the paper's first application benchmark, Sec. III-A, which spends
 * its time in sincosf): for k < m,
 *   X[k] = sum_{j < n} x[j] (cos t_kj - i sin t_kj),  t_kj = RN32(w[k] j),
 * with sinf/cosf of t_kj correctly rounded.  Each product x[j] cos t_kj is
 * exact in binary64 and the sums are accumulated as double-doubles in a fixed
 * order, so X[k] (re, im) is the binary64 rounding of a value within about
 * n 2^-104 sum_j |x[j] cos t_kj| (resp. sin) of the exact sum, and the same on
 * every run.  Device pointers: x (n floats), w (m floats: w[k] = 2 pi f_k / N
 * for a frequency f_k in bins, any finite value allowed), X (m pairs of
 * doubles, 16-byte aligned, caller-owned).  0 <= n <= 2^24 (sample indices
 * exact in binary32; else CR_E_SIZE); m == 0 returns CR_OK.  flags: enum
 * cr_flag.  X may not overlap x or w (CR_E_OVERLAP).  The call allocates and
 * frees a stream-ordered workspace of m * S * 32 bytes (S = number of sample
 * slices, at most n / 2048 + 1); asynchronous and stream-ordered like
 * cr_eval.  Errors: CR_E_SIZE, CR_E_NULL, CR_E_ALIGN, CR_E_OVERLAP,
 * CR_E_NOMEM, CR_E_HIP. */
int cr_dft(const float *x, int64_t n, const float *w, int64_t m, double *X, unsigned flags,
           void *stream);

/* ------------------------------------------------------------------ batches
 * Many requests of mixed function and uneven length evaluated by ONE graph
 * launch (captured once, replayed on every launch; the batched form of
 * the elementwise map; the paper's SIMD functions are called on vectors of
 * arbitrary length, Sec. III-A).  Requests follow the conventions above
 * (device pointers, element alignment, sincosf planar within its own output,
 * in place allowed except for sincosf); binary32 functions only (ids 0..18);
 * each request holds fewer than 2^31 elements.  Requests may not overlap
 * each other's outputs (not checked across requests).
 */
typedef struct {
  int32_t func_id; /* enum cr_func, 0..18 */
  int32_t impl;    /* enum cr_impl */
  const void *in;  /* device pointer, n elements */
  void *out;       /* device pointer, n (2n for sincosf) elements */
  int64_t n;
} cr_request;

typedef struct cr_batch_plan cr_batch_plan; /* opaque, owned by the library */

/* Validate the requests, upload the tile table and capture the launch in a
 * HIP graph.  The plan keeps the request pointers: the buffers must stay
 * valid while the plan is launched.  flags: enum cr_flag (applied to every
 * request).  On success *plan receives a new plan (free it with
 * cr_batch_plan_destroy); on error *plan is NULL and nothing is allocated.
 * Errors: CR_E_NULL (reqs or plan NULL, or a NULL pointer in a request with
 * n > 0), CR_E_FUNC, CR_E_IMPL, CR_E_ALIGN, CR_E_OVERLAP (within a request),
 * CR_E_SIZE (num < 0 or a request with n < 0 or n >= 2^31), CR_E_NOMEM,
 * CR_E_HIP. */
int cr_batch_plan_create(const cr_request *reqs, int32_t num, unsigned flags,
                         cr_batch_plan **plan);
/* Launch the plan's graph on the stream (asynchronous, stream-ordered).  The
 * graph holds one persistent kernel per (implementation, function) present,
 * each over its own contiguous range of 4096-element tiles (requests are
 * sorted by implementation and function when the plan is made), spread over
 * four parallel branches that join before the launch completes. */
int cr_batch_plan_launch(cr_batch_plan *plan, void *stream);
/* Release the plan (synchronises with its last launch first). */
int cr_batch_plan_destroy(cr_batch_plan *plan);
/* Evaluate the requests with one launch on the stream, without a graph.  The
 * request and tile tables are allocated and freed stream-ordered; the call
 * synchronises the stream once, after copying the tables from host memory
 * and before the launch. */
int cr_eval_batch(const cr_request *reqs, int32_t num, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as cr_eval_batch, with the same request conventions, results
 * and errors, but the request and tile tables go into a fixed scratch array
 * in the library's static device memory instead of stream-ordered
 * allocations.  The call makes no hipMalloc/hipFree or other allocating
 * device call.  The scratch holds at most CR_NOALLOC_MAX_REQUESTS requests and
 * CR_NOALLOC_MAX_TILES tiles, where a request of n elements takes
 * ceil(n / 4096) tiles (about 2 10^9 elements in all); larger batches return
 * CR_E_SCRATCH before anything is copied or launched.  Each device holds one
 * scratch (about 8.4 MiB, kept until the process ends) shared by every call
 * on that device: calls on one stream are ordered, but calls that overlap in
 * time on different streams of one device race on the tables and must not
 * be made.  Copies the tables from host memory and synchronises the stream
 * once before launching, as cr_eval_batch does. */
#define CR_NOALLOC_MAX_REQUESTS 8192
#define CR_NOALLOC_MAX_TILES (1 << 19)
int cr_eval_batch_noalloc(const cr_request *reqs, int32_t num, void *stream);

/* Per-device counters of the current device, cumulative since the last reset
 * (paper, Sec. III-B: the cost of lanes sent to the accurate path).
 *   elems          elements submitted through cr_eval / cr_eval_ex
 *   fallback_lanes elements that failed the fast-path rounding test (or all,
 *                  with CR_FLAG_FORCE_FALLBACK) and took the accurate path
 *   fallback_waves wave-level executions of the accurate path (one wave of
 *                  64 lanes pays once per element slot in which any lane fails)
 *   escapes        elements whose accurate path could not certify the
 *                  rounding (expected 0; their output is still the accurate
 *                  path's result); escape_index[] holds the first ones, as
 *                  element indices within their call (for a batch:
 *                  (request index << 32) | element index within the
 *                  request, the request index counted in the caller's
 *                  array). */
typedef struct {
  uint64_t elems;
  uint64_t fallback_lanes;
  uint64_t fallback_waves;
  uint64_t escapes;
  uint64_t escape_index[16];
} cr_stats;

/* Zero the current device's counters (stream-ordered). */
int cr_stats_reset(void *stream);
/* Copy the current device's counters to *out; synchronises the stream. */
int cr_stats_read(void *stream, cr_stats *out);

/* ---- Launch configurations and the autotuner --------------------------------
 * The project's own addition beside the paper's kernels: how a function's
 * elementwise kernel is laid out on the GPU.  Each (function, implementation)
 * pair has one configuration: a kernel variant -- elements per thread (4, 8
 * or 16 binary32 values, i.e. 1, 2 or 4 float4 loads per tile), whether the
 * next tile is loaded while the current one is evaluated (software
 * pipelining), and where the function's <= 16-entry tables live (staged in
 * LDS per workgroup, or read from one device-global copy through the vector
 * caches) -- and the persistent grid size in workgroups per compute unit.
 * Results never depend on the configuration, only speed does.  sincosf and
 * the complex functions have variant 0 only (their grid is tunable).  The
 * binary64 functions have variants 0..3 of their own kernel: 0 = 8 doubles
 * per thread (4 double2 loads per tile), each element evaluated and queued
 * before the next; 1, 2, 3 = 2, 4, 8 doubles per thread, all elements of the
 * tile evaluated in straight-line code before the failing ones are queued.
 * cr_tune_variant_info describes the binary32 variants.
 * Configurations are process-wide host state shared by all devices. */
typedef struct {
  int32_t variant;       /* 0 .. cr_tune_num_variants()-1; 0 is the default */
  int32_t blocks_per_cu; /* 1..64; 0 (set only) = the library default (16) */
} cr_tune_cfg;

int cr_tune_num_variants(void);
/* Shape of a variant; any output pointer may be NULL.  CR_E_TUNE if out of range. */
int cr_tune_variant_info(int variant, int *elems_per_thread, int *prefetch, int *table_in_lds);
/* Current configuration of (func_id, impl); CR_IMPL_AUTO means F64_INTERNAL. */
int cr_tune_get(int func_id, int impl, cr_tune_cfg *cfg);
/* Install a configuration.  CR_E_FUNC / CR_E_IMPL / CR_E_NULL / CR_E_TUNE on bad input. */
int cr_tune_set(int func_id, int impl, const cr_tune_cfg *cfg);
/* All configurations back to the defaults. */
int cr_tune_reset(void);
/* Grid of the batch kernels (cr_batch_plan_create, cr_eval_batch,
 * cr_eval_batch_noalloc): workgroups per compute unit of each per-function
 * kernel of a batch, one setting per implementation (CR_IMPL_AUTO means
 * F64_INTERNAL), 1..64, default 4.  A plan keeps the value in force when it is
 * created.  Results never depend on it.  CR_E_IMPL / CR_E_NULL / CR_E_TUNE on
 * bad input. */
int cr_tune_batch_get(int impl, int32_t *blocks_per_cu);
int cr_tune_batch_set(int impl, int32_t blocks_per_cu);
/* Text file, one line per entry: "<function> <f64|split> <variant> <blocks_per_cu>",
 * and "batch <f64|split> 0 <blocks_per_cu>" for the batch grid; '#' starts a
 * comment line.  Load applies nothing unless the whole file is valid
 * (CR_E_TUNE otherwise); save writes every entry. */
int cr_tune_load(const char *path);
int cr_tune_save(const char *path);
/* Time every variant x grid size {2, 4, 8, 16, 32 workgroups per CU} of
 * (func_id, impl) on the caller's device buffers in/out (n elements, the same
 * conventions as cr_eval_ex; out is overwritten): about 100 ms of launches
 * first so the clocks settle, then three passes over the space (reps timed
 * launches per configuration after one untimed one, reps <= 0: 10), keeping
 * each configuration's median pass, and install the fastest.  Synchronizes the
 * stream; adds its launches to the statistics counters.  best_gelem_s (may be
 * NULL) receives the winner's rate in 10^9 elements per second. */
int cr_autotune(int func_id, int impl, const void *in, void *out, size_t n, int reps,
                void *stream, double *best_gelem_s);

/* Human-readable text for a status code (static storage). */
const char *cr_status_str(int status);
/* The last hipError_t seen by this thread inside the library (0 if none). */
int cr_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif
