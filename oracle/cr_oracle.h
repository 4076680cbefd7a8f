/*
 * cr_oracle.h -- CPU oracle for correctly rounded elementwise functions.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, rigorous reference
 * that the GPU library is checked against.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it; the product
 * path never does.
 *
 * What it computes (paper, Sec. I and Sec. II-A): for an input encoding x
 * and a function f, the correctly rounded value RN_even(f(x)) in binary32
 * (single precision functions) or binary64 (exp, log, exp2), where f(x) is the
 * exact real value.  The evaluation is a Ziv loop (Sec. I): f(x) is
 * enclosed in an interval with a from-scratch fixed-point multiprecision
 * ball arithmetic; when both ends of the interval round to the same
 * floating-point number that number is returned, otherwise the working
 * precision is doubled.
 *
 * Function ids (shared numbering convention with the GPU library, each side
 * defines its own constants):
 *   0 expf   1 exp2f   2 exp10f  3 expm1f  4 logf   5 log2f  6 log10f
 *   7 log1pf 8 rsqrtf  9 sinf   10 cosf   11 sincosf 12 tanf 13 asinf
 *  14 acosf 15 atanf  16 sinhf  17 coshf  18 tanhf  64 exp (binary64)
 *  65 log (binary64)  66 exp2 (binary64; the paper's binary64 exp2, Sec. II-B)
 *
 * Conventions: in/out are HOST pointers.  Element type follows the id
 * (float for 0..18, double for 64, 65, 66).  sincosf writes 2n floats, planar:
 * out[0..n) = sin, out[n..2n) = cos.
 * Return value: 0 on success, negative on a bad id / null pointer, or -9 if
 * some element did not resolve within the precision cap (its output is then
 * a NaN with payload 0xdead).
 */
#ifndef CR_ORACLE_H
#define CR_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int cr_oracle_eval(int func_id, const void *in, void *out, size_t n, int nthreads);

/* Hardness of each input: -log2(distance from f(x) to the nearest rounding
 * boundary of the destination format, in units of the result's ulp).  A
 * value of 1 means f(x) is exactly representable or as far as possible from
 * a midpoint; large values mean hard to round.  Special/exact cases and
 * NaN results report 0.  For sincosf the larger of the two is reported. */
int cr_oracle_hardness(int func_id, const void *in, double *h, size_t n, int nthreads);

/* As cr_oracle_eval in a given IEEE 754 rounding mode (Sec. 4.3): 0 = to
 * nearest, ties to even (the same results as cr_oracle_eval), 1 = toward
 * zero, 2 = toward +infinity, 3 = toward -infinity.  Overflow gives infinity
 * or the largest finite number as the mode says; values that round to zero
 * keep their sign.  Returns -3 for an unknown mode. */
int cr_oracle_eval_mode(int func_id, int mode, const void *in, void *out, size_t n,
                        int nthreads);

/* Exhaustive hard-case scan of binary32 encodings [lo, hi): a cheap double
 * precision estimate (libm) selects candidates whose estimate lies within
 * 2^-h_prefilter ulp of a midpoint; each candidate is then measured with
 * cr_oracle_hardness and kept if its hardness is >= h_keep.  Writes up to
 * max_out (input bits, hardness) pairs and returns how many were found
 * (which may exceed max_out).  For sincosf the sin and cos tests are ORed. */
int64_t cr_oracle_scan_f32(int func_id, uint32_t lo, uint64_t hi, double h_prefilter,
                           double h_keep, uint32_t *out_bits, double *out_h,
                           int64_t max_out, int nthreads);

/* Sampled hard-case scan for binary64 exp (64) / log (65) / exp2 (66) over the n given
 * inputs: a quad-precision estimate preselects candidates, the oracle keeps
 * those with hardness >= h_keep.  Same output convention as the f32 scan. */
int64_t cr_oracle_scan_f64(int func_id, const double *x, size_t n, double h_prefilter,
                           double h_keep, double *out_x, double *out_h, int64_t max_out,
                           int nthreads);

/* Independent check for rsqrtf: decides RN(1/sqrt(x)) for a binary32 x by
 * exact integer comparisons of m^2 * x against 1 at the neighbouring
 * midpoints m (no approximation of the function at all). */
int cr_oracle_rsqrtf_exact(const float *in, float *out, size_t n);

/* Constants evaluated two independent ways at the given precision (bits):
 * which = 0: ln2 = 2 atanh(1/3)      which = 1: ln2 = sum 1/(k 2^k)
 * which = 2: pi (Machin formula)     which = 3: pi (Euler: 4(atan 1/2 + atan 1/3))
 * which = 4: ln10 = 3 ln2 + 2 atanh(1/9)
 * Writes the enclosure midpoint as nbits fraction bits big-endian hex into
 * buf (hex digits of floor(c * 2^nbits)) and returns the radius bound in
 * units of 2^-nbits (as a double). */
double cr_oracle_constant(int which, int nbits, char *buf, size_t buflen);

/* Maximum working precision (bits) the Ziv loop reached during the last
 * cr_oracle_eval call on this thread group (diagnostic). */
int cr_oracle_last_max_prec(void);

#ifdef __cplusplus
}
#endif
#endif
