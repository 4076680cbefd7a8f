/*
 * cr_oracle.c -- slow, rigorous CPU oracle for correctly rounded functions.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark.  The GPU library never links or calls it,
 * and it shares no code, tables or constants with the GPU library.
 *
 * Definition followed (paper, Sec. I; Sec. II-A, validation paragraph): the
 * correctly rounded result is RN_even(f(x)) of the exact real value f(x).
 * cr_oracle_eval_mode also gives the results in the directed rounding modes
 * the paper's CPU library supports (Sec. II-A: round toward zero, up, down):
 * the same enclosures, with both ends rounded in that mode.
 * Method (paper, Sec. I, Ziv's iterative approach): enclose f(x) in an
 * interval; if both ends round to the same floating-point number, that number
 * is the answer; otherwise double the precision and try again.
 *
 * The enclosures use a fixed-point "ball" arithmetic written here from
 * scratch: a value is W * 2^-F (W a two's-complement integer of IL+FL 64-bit
 * limbs, F = 64*FL) together with a radius (in units of 2^-F) that bounds the
 * distance to the exact quantity.  Every operation widens the radius by a
 * proven bound on its own truncation error; every series adds a proven bound
 * on its tail.  Nothing here relies on the host floating-point unit for
 * correctness: libm is only used to pick the working precision.
 */
#define _GNU_SOURCE
#include "cr_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define IL 3     /* integer limbs: |value| < 2^191 */
#define MAXFL 40 /* up to 2560 fraction bits */
#define MAXL (IL + MAXFL)
#define PMAX 2048

static __thread int FL = 2;
static __thread int L = IL + 2;

typedef struct {
  uint64_t w[MAXL];
  double rad; /* radius, in units of 2^-(64*FL) */
} ball;

/* -------------------------------------------------------------------------
 * Upward-rounded arithmetic on non-negative doubles (radius bookkeeping).
 * A computed sum/product of non-negative doubles is within a factor
 * (1 +- 2^-53) of the exact one; scaling by (1 + 2^-50) and adding a tiny
 * absolute term makes it an upper bound, also through underflow.
 * ---------------------------------------------------------------------- */
static double up(double v) { return v * (1.0 + 0x1p-50) + 0x1p-1060; }
static double addu(double a, double b) { return up(a + b); }
static double mulu(double a, double b) { return up(a * b); }

static int set_fbits(int fbits) {
  int fl = (fbits + 63) / 64;
  if (fl < 1) fl = 1;
  if (fl > MAXFL) return -1;
  FL = fl;
  L = IL + fl;
  return 0;
}
#define FB (64 * FL)

/* ---------------- multi-limb integer helpers (L limbs) ---------------- */
static int w_isneg(const uint64_t *a) { return (int64_t)a[L - 1] < 0; }

static void w_negate(uint64_t *r, const uint64_t *a) {
  uint64_t carry = 1;
  for (int i = 0; i < L; i++) {
    uint64_t t = ~a[i] + carry;
    carry = carry && t == 0;
    r[i] = t;
  }
}

static int w_abs(uint64_t *r, const uint64_t *a) {
  int s = w_isneg(a);
  if (s)
    w_negate(r, a);
  else if (r != a)
    memcpy(r, a, sizeof(uint64_t) * L);
  return s;
}

static void w_add(uint64_t *r, const uint64_t *a, const uint64_t *b) {
  u128 c = 0;
  for (int i = 0; i < L; i++) {
    c += (u128)a[i] + b[i];
    r[i] = (uint64_t)c;
    c >>= 64;
  }
}

static void w_sub(uint64_t *r, const uint64_t *a, const uint64_t *b) {
  uint64_t borrow = 0;
  for (int i = 0; i < L; i++) {
    u128 t = (u128)a[i] - b[i] - borrow;
    r[i] = (uint64_t)t;
    borrow = (uint64_t)(t >> 64) & 1;
  }
}

static int w_iszero(const uint64_t *a) {
  for (int i = 0; i < L; i++)
    if (a[i]) return 0;
  return 1;
}

/* number of significant bits of an unsigned magnitude */
static int w_bitlen(const uint64_t *m) {
  for (int i = L - 1; i >= 0; i--)
    if (m[i]) return 64 * i + (64 - __builtin_clzll(m[i]));
  return 0;
}

/* bits [pos, pos+cnt) of an unsigned magnitude, cnt <= 64, pos >= 0 */
static uint64_t w_getbits(const uint64_t *m, int64_t pos, int cnt) {
  uint64_t r = 0;
  for (int k = 0; k < cnt; k++) {
    int64_t b = pos + k;
    if (b >= 64 * (int64_t)L) break;
    if ((m[b >> 6] >> (b & 63)) & 1) r |= (uint64_t)1 << k;
  }
  return r;
}

/* is any bit below position pos set? */
static int w_anybelow(const uint64_t *m, int64_t pos) {
  if (pos <= 0) return 0;
  int64_t full = pos >> 6;
  for (int64_t i = 0; i < full && i < L; i++)
    if (m[i]) return 1;
  if (full < L && (pos & 63)) {
    uint64_t mask = ((uint64_t)1 << (pos & 63)) - 1;
    if (m[full] & mask) return 1;
  }
  return 0;
}

/* |m| * 2^-F as a double: approximate, upper bound and lower bound */
static double w_val_approx(const uint64_t *m) {
  int i = L - 1;
  while (i > 0 && !m[i]) i--;
  double v = (double)m[i];
  if (i > 0) v = v * 0x1p64 + (double)m[i - 1];
  return ldexp(v, 64 * (i > 0 ? i - 1 : 0) - FB);
}
static double w_val_up(const uint64_t *m) {
  int i = L - 1;
  while (i > 0 && !m[i]) i--;
  double v = (double)m[i];
  if (i > 0) v = v * 0x1p64 + (double)m[i - 1] + 1.0;
  return up(up(ldexp(v, 64 * (i > 0 ? i - 1 : 0) - FB)));
}
static double w_val_down(const uint64_t *m) {
  int i = L - 1;
  while (i > 0 && !m[i]) i--;
  double v = (double)m[i];
  if (i > 0) v = v * 0x1p64 + (double)m[i - 1];
  return ldexp(v, 64 * (i > 0 ? i - 1 : 0) - FB) * (1.0 - 0x1p-50);
}
/* |m| as a double in units of 2^-F (upper bound) */
static double w_ulps_up(const uint64_t *m) {
  int i = L - 1;
  while (i > 0 && !m[i]) i--;
  double v = (double)m[i];
  if (i > 0) v = v * 0x1p64 + (double)m[i - 1] + 1.0;
  return up(up(ldexp(v, 64 * (i > 0 ? i - 1 : 0))));
}

static void fail_overflow(const char *where) {
  fprintf(stderr, "cr_oracle: fixed-point overflow in %s\n", where);
  abort();
}

/* ------------------------------ balls -------------------------------- */
static void b_set_si(ball *r, int64_t v) {
  memset(r->w, 0, sizeof(uint64_t) * L);
  uint64_t mag = v < 0 ? (uint64_t)(-(v + 1)) + 1 : (uint64_t)v;
  r->w[FL] = mag;
  if (v < 0) w_negate(r->w, r->w);
  r->rad = 0;
}

/* 2^e as a ball (exact when representable) */
static void b_set_2exp(ball *r, int e) {
  memset(r->w, 0, sizeof(uint64_t) * L);
  r->rad = 0;
  int64_t pos = (int64_t)e + FB;
  if (pos < 0) {
    r->rad = 1;
    return;
  }
  if (pos >= 64 * L - 1) fail_overflow("b_set_2exp");
  r->w[pos >> 6] = (uint64_t)1 << (pos & 63);
}

/* exact conversion of a finite double (radius 1 ulp if bits fall below 2^-F) */
static void b_set_d(ball *r, double x) {
  memset(r->w, 0, sizeof(uint64_t) * L);
  r->rad = 0;
  if (x == 0) return;
  int ex;
  double f = frexp(fabs(x), &ex); /* |x| = f 2^ex, f in [0.5,1) */
  uint64_t M = (uint64_t)ldexp(f, 53);
  int64_t sh = (int64_t)ex - 53 + FB; /* |x| = M 2^(ex-53) = M 2^sh 2^-F */
  if (sh >= 0) {
    if (sh + 53 >= 64 * L - 1) fail_overflow("b_set_d");
    int64_t limb = sh >> 6, bit = sh & 63;
    r->w[limb] |= M << bit;
    if (bit && limb + 1 < L) r->w[limb + 1] |= M >> (64 - bit);
  } else {
    int64_t s = -sh;
    uint64_t q = s >= 64 ? 0 : M >> s;
    if (s >= 64 || (q << s) != M) r->rad = 1;
    r->w[0] = q;
  }
  if (x < 0) w_negate(r->w, r->w);
}

static double b_mid(const ball *a) {
  uint64_t m[MAXL];
  int s = w_abs(m, a->w);
  double v = w_val_approx(m);
  return s ? -v : v;
}
/* upper bound of |value| over the ball (value units) */
static double b_abs_hi(const ball *a) {
  uint64_t m[MAXL];
  w_abs(m, a->w);
  return addu(w_val_up(m), ldexp(up(a->rad), -FB));
}
/* lower bound of |value| over the ball (value units), >= 0 */
static double b_abs_lo(const ball *a) {
  uint64_t m[MAXL];
  w_abs(m, a->w);
  double v = w_val_down(m) - ldexp(up(a->rad), -FB) * (1 + 0x1p-50);
  return v > 0 ? v * (1 - 0x1p-50) : 0;
}
/* upper bound of |value| over the ball, in units of 2^-F */
static double b_ulps_hi(const ball *a) {
  uint64_t m[MAXL];
  w_abs(m, a->w);
  return addu(w_ulps_up(m), a->rad);
}

static void b_add(ball *r, const ball *a, const ball *b) {
  w_add(r->w, a->w, b->w);
  r->rad = addu(a->rad, b->rad);
}
static void b_sub(ball *r, const ball *a, const ball *b) {
  w_sub(r->w, a->w, b->w);
  r->rad = addu(a->rad, b->rad);
}
static void b_neg(ball *r, const ball *a) {
  w_negate(r->w, a->w);
  r->rad = a->rad;
}
static void b_add_si(ball *r, const ball *a, int64_t v) {
  ball t;
  b_set_si(&t, v);
  b_add(r, a, &t);
}

/* r = a * b; the product is truncated toward zero (< 1 ulp) */
static void b_mul(ball *r, const ball *a, const ball *b) {
  uint64_t A[MAXL], B[MAXL], P[2 * MAXL];
  int sa = w_abs(A, a->w), sb = w_abs(B, b->w);
  double rad = addu(mulu(w_val_up(A), b->rad), mulu(w_val_up(B), a->rad));
  rad = addu(rad, ldexp(mulu(a->rad, b->rad), -FB));
  rad = addu(rad, 2.0);
  int la = L, lb = L;
  while (la > 0 && !A[la - 1]) la--;
  while (lb > 0 && !B[lb - 1]) lb--;
  memset(P, 0, sizeof(uint64_t) * 2 * L);
  for (int i = 0; i < la; i++) {
    u128 c = 0;
    for (int j = 0; j < lb; j++) {
      c += (u128)A[i] * B[j] + P[i + j];
      P[i + j] = (uint64_t)c;
      c >>= 64;
    }
    P[i + lb] = (uint64_t)c;
  }
  for (int i = FL + L; i < 2 * L; i++)
    if (P[i]) fail_overflow("b_mul");
  memcpy(r->w, P + FL, sizeof(uint64_t) * L);
  if (w_isneg(r->w)) fail_overflow("b_mul");
  if (sa ^ sb) w_negate(r->w, r->w);
  r->rad = rad;
}

/* r = a * k exactly (k a small integer) */
static void b_mul_si(ball *r, const ball *a, int64_t k) {
  uint64_t A[MAXL];
  int sa = w_abs(A, a->w);
  uint64_t km = k < 0 ? (uint64_t)(-(k + 1)) + 1 : (uint64_t)k;
  u128 c = 0;
  for (int i = 0; i < L; i++) {
    c += (u128)A[i] * km;
    r->w[i] = (uint64_t)c;
    c >>= 64;
  }
  if (c || w_isneg(r->w)) fail_overflow("b_mul_si");
  if (sa ^ (k < 0)) w_negate(r->w, r->w);
  r->rad = mulu(a->rad, (double)km);
}

/* r = a / d, d a positive integer; truncated toward zero (< 1 ulp) */
static void b_div_ui(ball *r, const ball *a, uint64_t d) {
  uint64_t A[MAXL];
  int sa = w_abs(A, a->w);
  u128 rem = 0;
  for (int i = L - 1; i >= 0; i--) {
    u128 cur = (rem << 64) | A[i];
    r->w[i] = (uint64_t)(cur / d);
    rem = cur % d;
  }
  if (sa) w_negate(r->w, r->w);
  r->rad = addu(up(a->rad / (double)d), 1.0);
}

/* r = a * 2^s for s >= 0 (exact) or s < 0 (truncated, < 1 ulp) */
static void b_mul2exp(ball *r, const ball *a, int s) {
  uint64_t A[MAXL], R[MAXL];
  int sa = w_abs(A, a->w);
  memset(R, 0, sizeof(uint64_t) * L);
  if (s >= 0) {
    if (w_bitlen(A) + s >= 64 * L - 1) fail_overflow("b_mul2exp");
    int ls = s >> 6, bs = s & 63;
    for (int i = L - 1; i >= ls; i--) {
      uint64_t v = A[i - ls] << bs;
      if (bs && i - ls - 1 >= 0) v |= A[i - ls - 1] >> (64 - bs);
      R[i] = v;
    }
    r->rad = ldexp(a->rad, s);
  } else {
    int t = -s, ls = t >> 6, bs = t & 63;
    for (int i = 0; i + ls < L; i++) {
      uint64_t v = A[i + ls] >> bs;
      if (bs && i + ls + 1 < L) v |= A[i + ls + 1] << (64 - bs);
      R[i] = v;
    }
    r->rad = addu(ldexp(a->rad, s), 1.0);
  }
  memcpy(r->w, R, sizeof(uint64_t) * L);
  if (sa) w_negate(r->w, r->w);
}

/* r = 1 / b.  Newton's iteration y <- y + y (1 - b y) on the midpoint, then
 * the enclosure |1/B - y| <= |1 - B y| / |B| over the whole ball B. */
static int b_inv(ball *r, const ball *b) {
  double lo = b_abs_lo(b);
  if (!(lo > 0)) return -1;
  ball y, t, e, bm = *b;
  bm.rad = 0;
  b_set_d(&y, 1.0 / b_mid(b));
  for (int bits = 48; bits < FB + 16; bits *= 2) {
    b_mul(&t, &bm, &y);
    b_set_si(&e, 1);
    b_sub(&e, &e, &t);
    b_mul(&t, &y, &e);
    b_add(&y, &y, &t);
    y.rad = 0;
  }
  b_mul(&t, b, &y);
  b_set_si(&e, 1);
  b_sub(&e, &e, &t);
  *r = y;
  r->rad = up(b_ulps_hi(&e) / lo);
  return 0;
}

static int b_div(ball *r, const ball *a, const ball *b) {
  ball ib;
  if (b_inv(&ib, b)) return -1;
  b_mul(r, a, &ib);
  return 0;
}

/* r = sqrt(a) for a > 0.  Newton on 1/sqrt for the midpoint y, then
 * |sqrt(A) - y| = |A - y^2| / (sqrt(A) + y) <= |A - y^2| / y. */
static int b_sqrt(ball *r, const ball *a) {
  double am = b_mid(a);
  if (!(am > 0) || !(b_abs_lo(a) > 0)) return -1;
  ball z, t, e, am_b = *a, y;
  am_b.rad = 0;
  b_set_d(&z, 1.0 / sqrt(am));
  for (int bits = 48; bits < FB + 16; bits *= 2) {
    b_mul(&t, &z, &z);
    b_mul(&e, &am_b, &t);
    b_set_si(&t, 1);
    b_sub(&e, &t, &e);  /* 1 - a z^2 */
    b_mul(&t, &z, &e);
    b_mul2exp(&t, &t, -1);
    b_add(&z, &z, &t);
    z.rad = 0;
  }
  b_mul(&y, &am_b, &z);
  y.rad = 0;
  double ylo = b_abs_lo(&y);
  if (!(ylo > 0)) return -1;
  b_mul(&t, &y, &y);
  b_sub(&e, a, &t);
  *r = y;
  r->rad = up(b_ulps_hi(&e) / ylo);
  return 0;
}

/* ---------------------------- series ---------------------------------- */

/* The loop below stops once a bound on the next term, lg2 in log2 units,
 * is below 2^-(F+2), i.e. a quarter of an ulp. */
static int tail_small(double lg2) { return lg2 < -(double)FB - 2.0; }

/* e^r for |r| <= 1 (Taylor).  Terms |r|^i/i! decrease with ratio <= 1/2
 * from i = 1 on, so the tail after the last term kept is at most twice the
 * first omitted term. */
static void b_exp_small(ball *y, const ball *r) {
  double rmax = b_abs_hi(r);
  ball term, t;
  b_set_si(y, 1);
  b_set_si(&term, 1);
  double lr = log2(rmax), lt = 0;
  for (int i = 1; i < 100000; i++) {
    b_mul(&t, &term, r);
    b_div_ui(&term, &t, (uint64_t)i);
    b_add(y, y, &term);
    lt += lr - log2((double)i);
    if (tail_small(lt + lr - log2((double)i + 1) + 1)) break;
  }
  y->rad = addu(y->rad, 1.0);
}

/* sum_{i>=1} r^i / i!  (= e^r - 1) for |r| <= 1/2, same tail argument */
static void b_expm1_small(ball *y, const ball *r) {
  double rmax = b_abs_hi(r);
  ball term, t;
  *y = *r;
  term = *r;
  double lr = log2(rmax), lt = lr;
  for (int i = 2; i < 100000; i++) {
    b_mul(&t, &term, r);
    b_div_ui(&term, &t, (uint64_t)i);
    b_add(y, y, &term);
    lt += lr - log2((double)i);
    if (tail_small(lt + lr - log2((double)i + 1) + 1)) break;
  }
  y->rad = addu(y->rad, 1.0);
}

/* atanh(u) = sum u^(2i+1)/(2i+1) for |u| <= 1/2; the tail after the term of
 * index N is at most |u|^(2N+3) / ((2N+3)(1-u^2)) <= 2 |u|^(2N+3)/(2N+3). */
static void b_atanh_series(ball *s, const ball *u) {
  double umax = b_abs_hi(u);
  ball u2, pw, t;
  b_mul(&u2, u, u);
  *s = *u;
  pw = *u;
  double lu = log2(umax);
  for (int i = 1; i < 100000; i++) {
    b_mul(&t, &pw, &u2);
    pw = t;
    b_div_ui(&t, &pw, (uint64_t)(2 * i + 1));
    b_add(s, s, &t);
    if (tail_small(lu * (2 * i + 3) - log2(2.0 * i + 3) + 1)) break;
  }
  s->rad = addu(s->rad, 1.0);
}

/* atan(u) = sum (-1)^i u^(2i+1)/(2i+1) for |u| < 1: alternating with
 * decreasing terms, so the tail is bounded by the first omitted term. */
static void b_atan_series(ball *s, const ball *u) {
  double umax = b_abs_hi(u);
  ball u2, pw, t;
  b_mul(&u2, u, u);
  *s = *u;
  pw = *u;
  double lu = log2(umax);
  for (int i = 1; i < 100000; i++) {
    b_mul(&t, &pw, &u2);
    pw = t;
    b_div_ui(&t, &pw, (uint64_t)(2 * i + 1));
    if (i & 1)
      b_sub(s, s, &t);
    else
      b_add(s, s, &t);
    if (tail_small(lu * (2 * i + 3) - log2(2.0 * i + 3))) break;
  }
  s->rad = addu(s->rad, 1.0);
}

/* sin r and cos r for |r| <= 1 (alternating Taylor series, tail bounded by
 * the first omitted term). */
static void b_sincos_small(ball *s, ball *c, const ball *r) {
  double rmax = b_abs_hi(r);
  double lr = log2(rmax);
  ball r2, term, t;
  b_mul(&r2, r, r);
  /* sin */
  *s = *r;
  term = *r;
  for (int i = 1; i < 100000; i++) {
    b_mul(&t, &term, &r2);
    b_div_ui(&term, &t, (uint64_t)(2 * i) * (uint64_t)(2 * i + 1));
    if (i & 1)
      b_sub(s, s, &term);
    else
      b_add(s, s, &term);
    if (tail_small(lr * (2 * i + 3) - lgamma(2.0 * i + 4) / M_LN2)) break;
  }
  s->rad = addu(s->rad, 1.0);
  /* cos */
  b_set_si(c, 1);
  b_set_si(&term, 1);
  for (int i = 1; i < 100000; i++) {
    b_mul(&t, &term, &r2);
    b_div_ui(&term, &t, (uint64_t)(2 * i - 1) * (uint64_t)(2 * i));
    if (i & 1)
      b_sub(c, c, &term);
    else
      b_add(c, c, &term);
    if (tail_small(lr * (2 * i + 2) - lgamma(2.0 * i + 3) / M_LN2)) break;
  }
  c->rad = addu(c->rad, 1.0);
}

/* sinh and cosh Taylor series for |r| <= 1/2 (positive terms, ratio < 1/2,
 * tail <= twice the first omitted term). */
static void b_sinhcosh_small(ball *sh, ball *ch, const ball *r) {
  double lr = log2(b_abs_hi(r));
  ball r2, term, t;
  b_mul(&r2, r, r);
  *sh = *r;
  term = *r;
  for (int i = 1; i < 100000; i++) {
    b_mul(&t, &term, &r2);
    b_div_ui(&term, &t, (uint64_t)(2 * i) * (uint64_t)(2 * i + 1));
    b_add(sh, sh, &term);
    if (tail_small(lr * (2 * i + 3) - lgamma(2.0 * i + 4) / M_LN2 + 1)) break;
  }
  sh->rad = addu(sh->rad, 1.0);
  b_set_si(ch, 1);
  b_set_si(&term, 1);
  for (int i = 1; i < 100000; i++) {
    b_mul(&t, &term, &r2);
    b_div_ui(&term, &t, (uint64_t)(2 * i - 1) * (uint64_t)(2 * i));
    b_add(ch, ch, &term);
    if (tail_small(lr * (2 * i + 2) - lgamma(2.0 * i + 3) / M_LN2 + 1)) break;
  }
  ch->rad = addu(ch->rad, 1.0);
}

/* ---------------------------- constants ------------------------------- */

/* ln 2 = 2 atanh(1/3) */
static void c_ln2_atanh(ball *r) {
  ball u;
  b_set_si(&u, 1);
  b_div_ui(&u, &u, 3);
  b_atanh_series(r, &u);
  b_mul2exp(r, r, 1);
}
/* ln 2 = sum_{k>=1} 1/(k 2^k); tail after k = N is below 2^-N/(N+1) */
static void c_ln2_series(ball *r) {
  ball t;
  b_set_si(r, 0);
  for (int k = 1;; k++) {
    b_set_2exp(&t, -k);
    b_div_ui(&t, &t, (uint64_t)k);
    b_add(r, r, &t);
    if (tail_small(-(double)k - log2((double)k + 1))) break;
  }
  r->rad = addu(r->rad, 1.0);
}
/* atan(1/n) by its alternating series in 1/n^2 */
static void c_atan_inv(ball *r, uint64_t n) {
  ball pw, t;
  b_set_si(&pw, 1);
  b_div_ui(&pw, &pw, n);
  *r = pw;
  double ln = log2((double)n);
  for (int i = 1;; i++) {
    b_div_ui(&pw, &pw, n * n);
    b_div_ui(&t, &pw, (uint64_t)(2 * i + 1));
    if (i & 1)
      b_sub(r, r, &t);
    else
      b_add(r, r, &t);
    if (tail_small(-ln * (2 * i + 3))) break;
  }
  r->rad = addu(r->rad, 1.0);
}
/* pi = 16 atan(1/5) - 4 atan(1/239) (Machin) */
static void c_pi_machin(ball *r) {
  ball a, b;
  c_atan_inv(&a, 5);
  c_atan_inv(&b, 239);
  b_mul_si(&a, &a, 16);
  b_mul_si(&b, &b, 4);
  b_sub(r, &a, &b);
}
/* pi = 4 (atan(1/2) + atan(1/3)) (Euler) */
static void c_pi_euler(ball *r) {
  ball a, b;
  c_atan_inv(&a, 2);
  c_atan_inv(&b, 3);
  b_add(r, &a, &b);
  b_mul_si(r, r, 4);
}
/* ln 10 = 3 ln 2 + ln(5/4), ln(5/4) = 2 atanh(1/9) */
static void c_ln10(ball *r) {
  ball l2, u, s;
  c_ln2_atanh(&l2);
  b_set_si(&u, 1);
  b_div_ui(&u, &u, 9);
  b_atanh_series(&s, &u);
  b_mul2exp(&s, &s, 1);
  b_mul_si(&l2, &l2, 3);
  b_add(r, &l2, &s);
}

/* per-thread cache, keyed by the fraction limb count */
static __thread ball k_ln2, k_ln10, k_pi;
static __thread int k_ln2_fl = -1, k_ln10_fl = -1, k_pi_fl = -1;
static const ball *LN2(void) {
  if (k_ln2_fl != FL) {
    c_ln2_atanh(&k_ln2);
    k_ln2_fl = FL;
  }
  return &k_ln2;
}
static const ball *LN10(void) {
  if (k_ln10_fl != FL) {
    c_ln10(&k_ln10);
    k_ln10_fl = FL;
  }
  return &k_ln10;
}
static const ball *PI(void) {
  if (k_pi_fl != FL) {
    c_pi_machin(&k_pi);
    k_pi_fl = FL;
  }
  return &k_pi;
}

/* ----------------------- function building blocks --------------------- */

/* e^X = y * 2^k for a ball X with |X| < 1100: k = nearest(X/ln2),
 * r = X - k ln2, |r| < 0.35, y = e^r. */
static void b_exp_scaled(ball *y, int64_t *k, const ball *X) {
  int64_t kk = (int64_t)nearbyint(b_mid(X) / M_LN2);
  ball t, r;
  b_mul_si(&t, LN2(), kk);
  b_sub(&r, X, &t);
  b_exp_small(y, &r);
  *k = kk;
}

/* natural log of a positive ball: X = m 2^e with m in [sqrt(1/2), sqrt(2)),
 * log m = 2 atanh((m-1)/(m+1)).  Returns log(m) in *lm and e in *e. */
static int b_log_parts(ball *lm, int64_t *e, const ball *X) {
  double xm = b_mid(X);
  if (!(xm > 0) || !(b_abs_lo(X) > 0)) return -1;
  int ex;
  double f = frexp(xm, &ex); /* xm = f 2^ex, f in [0.5,1) */
  int64_t ee = f < M_SQRT1_2 ? ex - 1 : ex;
  ball m, num, den, u, s;
  b_mul2exp(&m, X, (int)-ee);
  b_add_si(&num, &m, -1);
  b_add_si(&den, &m, 1);
  if (b_div(&u, &num, &den)) return -1;
  if (b_abs_hi(&u) > 0.25) return -1;
  b_atanh_series(&s, &u);
  b_mul2exp(lm, &s, 1);
  *e = ee;
  return 0;
}

/* atan of a ball z (any real).  |z| > 1 uses atan z = sign(z) pi/2 - atan(1/z);
 * then the argument is halved with atan a = 2 atan(a / (1 + sqrt(1 + a^2)))
 * until |a| < 1/64, and the alternating series finishes. */
static int b_atan(ball *r, const ball *z) {
  double zm = b_mid(z);
  int neg = zm < 0;
  ball a, t, u;
  if (neg)
    b_neg(&a, z);
  else
    a = *z;
  int inv = fabs(zm) > 1.0;
  if (inv) {
    if (b_inv(&t, &a)) return -1;
    a = t;
  }
  int j = 0;
  while (b_abs_hi(&a) > 1.0 / 64) {
    b_mul(&t, &a, &a);
    b_add_si(&t, &t, 1);
    if (b_sqrt(&u, &t)) return -1;
    b_add_si(&u, &u, 1);
    if (b_div(&t, &a, &u)) return -1;
    a = t;
    j++;
  }
  b_atan_series(&t, &a);
  b_mul2exp(&t, &t, j);
  if (inv) {
    ball h;
    b_mul2exp(&h, PI(), -1);
    b_sub(&t, &h, &t);
  }
  if (neg)
    b_neg(r, &t);
  else
    *r = t;
  return 0;
}

/* -------------------------- function evaluators ----------------------- */
/* Each evaluator encloses f(x) in y * 2^e2, working with about p bits of
 * relative accuracy plus guard bits; the Ziv driver checks the result. */

enum {
  F_EXPF = 0, F_EXP2F, F_EXP10F, F_EXPM1F, F_LOGF, F_LOG2F, F_LOG10F, F_LOG1PF, F_RSQRTF,
  F_SINF, F_COSF, F_SINCOSF, F_TANF, F_ASINF, F_ACOSF, F_ATANF, F_SINHF, F_COSHF, F_TANHF,
  F_NUM32,
  F_EXP = 64, F_LOG = 65, F_EXP2 = 66
};
/* internal kinds (sincosf is evaluated as sin and as cos) */
enum { K_EXP, K_EXP2, K_EXP10, K_EXPM1, K_LOG, K_LOG2, K_LOG10, K_LOG1P, K_RSQRT,
       K_SIN, K_COS, K_TAN, K_ASIN, K_ACOS, K_ATAN, K_SINH, K_COSH, K_TANH };

#define GUARD 64

/* extra fraction bits so that a result of magnitude about 2^-t keeps p bits */
static int tiny_extra(double est) {
  if (!(est != 0) || !isfinite(est)) return 0;
  int t = -ilogb(est);
  if (t < 0) t = 0;
  if (t > 1200) t = 1200;
  return t;
}

static int ev(int kind, double x, int p, ball *y, int64_t *e2) {
  ball X, t, u, v;
  *e2 = 0;
  switch (kind) {
    case K_EXP: {
      if (set_fbits(p + GUARD + 16)) return -1;
      b_set_d(&X, x);
      b_exp_scaled(y, e2, &X);
      return 0;
    }
    case K_EXP2: {
      if (set_fbits(p + GUARD + 16)) return -1;
      double k = nearbyint(x);
      b_set_d(&X, x - k); /* exact: |x| < 2^24 here */
      b_mul(&t, &X, LN2());
      b_exp_small(y, &t);
      *e2 = (int64_t)k;
      return 0;
    }
    case K_EXP10: {
      if (set_fbits(p + GUARD + 16)) return -1;
      b_set_d(&X, x);
      b_mul(&t, &X, LN10());
      b_exp_scaled(y, e2, &t);
      return 0;
    }
    case K_EXPM1: {
      if (fabs(x) < 0.5) {
        if (set_fbits(p + GUARD + tiny_extra(x))) return -1;
        b_set_d(&X, x);
        b_expm1_small(y, &X);
        return 0;
      }
      if (set_fbits(p + GUARD + 16)) return -1;
      b_set_d(&X, x);
      int64_t k;
      b_exp_scaled(&t, &k, &X);
      if (x > 0) { /* e^x - 1 = 2^k (y - 2^-k) */
        b_set_2exp(&u, (int)-k);
        b_sub(y, &t, &u);
        *e2 = k;
      } else { /* e^x - 1 = y 2^k - 1, k < 0 */
        b_mul2exp(&u, &t, (int)k);
        b_add_si(y, &u, -1);
      }
      return 0;
    }
    case K_LOG:
    case K_LOG2:
    case K_LOG10: {
      double est = kind == K_LOG ? log(x) : kind == K_LOG2 ? log2(x) : log10(x);
      if (set_fbits(p + GUARD + 8 + tiny_extra(est))) return -1;
      /* x = m 2^e exactly, m in [sqrt(1/2), sqrt(2)); log m = 2 atanh((m-1)/(m+1)) */
      int ex;
      double f = frexp(x, &ex);
      int64_t e = f < M_SQRT1_2 ? ex - 1 : ex;
      b_set_d(&X, f < M_SQRT1_2 ? 2 * f : f);
      b_add_si(&u, &X, -1);
      b_add_si(&v, &X, 1);
      if (b_div(&t, &u, &v)) return -1;
      b_atanh_series(&u, &t);
      b_mul2exp(&t, &u, 1);
      if (kind == K_LOG2) {
        if (b_div(&u, &t, LN2())) return -1;
        b_add_si(y, &u, e);
        return 0;
      }
      b_mul_si(&u, LN2(), e);
      b_add(&v, &t, &u);
      if (kind == K_LOG) {
        *y = v;
        return 0;
      }
      return b_div(y, &v, LN10());
    }
    case K_LOG1P: {
      if (x >= -0.5 && x <= 1.0) {
        if (set_fbits(p + GUARD + 8 + tiny_extra(x))) return -1;
        b_set_d(&X, x);
        b_add_si(&t, &X, 2);
        if (b_div(&u, &X, &t)) return -1; /* u = x/(2+x), |u| <= 1/3 */
        b_atanh_series(&v, &u);
        b_mul2exp(y, &v, 1);
        return 0;
      }
      if (set_fbits(p + GUARD + 8)) return -1;
      b_set_d(&X, x);
      b_add_si(&X, &X, 1); /* exact: 1 + x with x >= 1 or x in (-1,-1/2) */
      int64_t e;
      if (b_log_parts(&t, &e, &X)) return -1;
      b_mul_si(&u, LN2(), e);
      b_add(y, &t, &u);
      return 0;
    }
    case K_RSQRT: {
      /* x = m 4^e with m in [1,4): 1/sqrt(x) = 2^-e / sqrt(m) */
      if (set_fbits(p + GUARD + 8)) return -1;
      int ex;
      double f = frexp(x, &ex); /* x = f 2^ex */
      int e = (ex - 1) >> 1;    /* floor((ex-1)/2) */
      double m = ldexp(x, -2 * e);
      b_set_d(&X, m);
      if (b_sqrt(&t, &X)) return -1;
      if (b_inv(y, &t)) return -1;
      *e2 = -e;
      (void)f;
      return 0;
    }
    case K_SIN:
    case K_COS:
    case K_TAN: {
      double est = kind == K_SIN ? sin(x) : kind == K_COS ? cos(x) : tan(x);
      int red = ilogb(x) > 0 ? ilogb(x) : 0;
      if (set_fbits(p + GUARD + 16 + red + tiny_extra(est))) return -1;
      ball s, c;
      int q = 0;
      b_set_d(&X, x);
      if (fabs(x) <= 0.75) {
        b_sincos_small(&s, &c, &X);
      } else {
        /* x (2/pi) = k + f with k integer, |f| <= 1/2; x = (k + f) pi/2 */
        ball twoopi, Y, fr, r, hp;
        if (b_inv(&twoopi, PI())) return -1;
        b_mul2exp(&twoopi, &twoopi, 1);
        b_mul(&Y, &X, &twoopi);
        /* nearest integer: add 2^(F-1), the integer part is W >> F */
        uint64_t W[MAXL], half[MAXL];
        memset(half, 0, sizeof(uint64_t) * L);
        half[(FB - 1) >> 6] = (uint64_t)1 << ((FB - 1) & 63);
        w_add(W, Y.w, half);
        q = (int)(W[FL] & 3);
        /* fraction: keep the low F bits of W, then subtract 1/2 */
        for (int i = FL; i < L; i++) W[i] = 0;
        w_sub(fr.w, W, half);
        fr.rad = Y.rad;
        b_mul2exp(&hp, PI(), -1);
        b_mul(&r, &fr, &hp);
        b_sincos_small(&s, &c, &r);
      }
      ball qs, qc; /* sin and cos of x from the quadrant */
      switch (q) {
        case 0: qs = s; qc = c; break;
        case 1: qs = c; b_neg(&qc, &s); break;
        case 2: b_neg(&qs, &s); b_neg(&qc, &c); break;
        default: b_neg(&qs, &c); qc = s; break;
      }
      if (kind == K_SIN) *y = qs;
      else if (kind == K_COS) *y = qc;
      else return b_div(y, &qs, &qc);
      return 0;
    }
    case K_ATAN: {
      if (set_fbits(p + GUARD + 16 + tiny_extra(x))) return -1;
      if (isinf(x)) {
        b_mul2exp(y, PI(), -1);
        if (x < 0) b_neg(y, y);
        return 0;
      }
      b_set_d(&X, x);
      return b_atan(y, &X);
    }
    case K_ASIN: {
      if (set_fbits(p + GUARD + 16 + tiny_extra(x))) return -1;
      if (fabs(x) == 1.0) {
        b_mul2exp(y, PI(), -1);
        if (x < 0) b_neg(y, y);
        return 0;
      }
      /* asin x = atan(x / sqrt((1-x)(1+x))) */
      b_set_d(&X, x);
      b_set_si(&t, 1);
      b_sub(&u, &t, &X);
      b_add(&v, &t, &X);
      b_mul(&t, &u, &v);
      if (b_sqrt(&u, &t)) return -1;
      if (b_div(&v, &X, &u)) return -1;
      return b_atan(y, &v);
    }
    case K_ACOS: {
      double est = acos(x);
      if (set_fbits(p + GUARD + 16 + tiny_extra(est))) return -1;
      if (x == -1.0) {
        *y = *PI();
        return 0;
      }
      /* acos x = 2 atan(sqrt((1-x)/(1+x))) */
      b_set_d(&X, x);
      b_set_si(&t, 1);
      b_sub(&u, &t, &X);
      b_add(&v, &t, &X);
      if (b_div(&t, &u, &v)) return -1;
      if (b_sqrt(&u, &t)) return -1;
      if (b_atan(&v, &u)) return -1;
      b_mul2exp(y, &v, 1);
      return 0;
    }
    case K_SINH:
    case K_COSH:
    case K_TANH: {
      double ax = fabs(x);
      if (ax < 0.5) {
        if (set_fbits(p + GUARD + 8 + (kind == K_COSH ? 0 : tiny_extra(x)))) return -1;
        ball sh, ch;
        b_set_d(&X, x);
        b_sinhcosh_small(&sh, &ch, &X);
        if (kind == K_SINH) *y = sh;
        else if (kind == K_COSH) *y = ch;
        else return b_div(y, &sh, &ch);
        return 0;
      }
      if (set_fbits(p + GUARD + 16)) return -1;
      /* w = e^(-2|x|) shifted into fixed point; e^|x| = y0 2^k */
      ball A, w, y0;
      int64_t k, k2;
      b_set_d(&A, ax);
      b_exp_scaled(&y0, &k, &A);
      b_mul_si(&t, &A, -2);
      b_exp_scaled(&u, &k2, &t);
      b_mul2exp(&w, &u, (int)k2); /* k2 <= -1 */
      if (kind == K_TANH) {
        /* tanh|x| = (1 - w)/(1 + w) */
        b_set_si(&t, 1);
        b_sub(&u, &t, &w);
        b_add(&v, &t, &w);
        if (b_div(y, &u, &v)) return -1;
      } else {
        /* sinh|x| = e^|x| (1 - w)/2, cosh x = e^|x| (1 + w)/2 */
        b_set_si(&t, 1);
        if (kind == K_SINH)
          b_sub(&u, &t, &w);
        else
          b_add(&u, &t, &w);
        b_mul(y, &y0, &u);
        *e2 = k - 1;
      }
      if (x < 0 && kind != K_COSH) b_neg(y, y);
      return 0;
    }
  }
  return -1;
}

/* --------------------------- final rounding --------------------------- */
/* Rounding mode of the current evaluation (IEEE 754-2019, Sec. 4.3):
 * 0 = to nearest, ties to even; 1 = toward zero; 2 = toward +infinity;
 * 3 = toward -infinity. */
enum { RM_RN = 0, RM_RZ = 1, RM_RU = 2, RM_RD = 3 };
static __thread int t_mode = RM_RN;

/* The result of an overflow (Sec. 7.4): infinity when the mode rounds away
 * from zero in the result's direction (or to nearest), else the largest
 * finite number. */
static uint64_t overflow_enc(int fmt, int neg) {
  const uint64_t sign = neg ? (fmt ? (uint64_t)1 << 63 : (uint64_t)1 << 31) : 0;
  const uint64_t inf = fmt ? 0x7ff0000000000000ull : 0x7f800000ull;
  const uint64_t max = inf - 1;
  int to_inf = t_mode == RM_RN || (t_mode == RM_RU && !neg) || (t_mode == RM_RD && neg);
  return sign | (to_inf ? inf : max);
}

/* Round the exact real value M * 2^s (M an unsigned magnitude) to binary32
 * (fmt 0) or binary64 (fmt 1) in the current rounding mode, with gradual
 * underflow and overflow as above (IEEE 754-2019, Sec. 4.3.1, 4.3.2, 7.4).
 * If dist is non-null it receives the distance of the value from the
 * nearest round-to-nearest boundary, in units of the result's quantum. */
static uint64_t round_mag(const uint64_t *M, int64_t s, int fmt, int neg, double *dist) {
  const int P = fmt ? 53 : 24;
  const int emin = fmt ? -1022 : -126, emax = fmt ? 1023 : 127, bias = fmt ? 1023 : 127;
  const uint64_t sign = neg ? (fmt ? (uint64_t)1 << 63 : (uint64_t)1 << 31) : 0;
  int nb = w_bitlen(M);
  if (dist) *dist = 0.5;
  if (nb == 0) return sign;
  int64_t E = nb - 1 + s; /* exponent of the leading bit */
  if (E > emax) return overflow_enc(fmt, neg);
  int64_t q = (E < emin ? emin : E) - (P - 1); /* exponent of the quantum */
  int64_t sh = q - s;                          /* bits below the quantum */
  uint64_t mant;
  if (sh <= 0) {
    mant = w_getbits(M, 0, 64) << (-sh);
  } else {
    mant = w_getbits(M, sh, P + 1);
    int rbit = (int)w_getbits(M, sh - 1, 1);
    int sticky = w_anybelow(M, sh - 1);
    if (dist) {
      /* |(M mod 2^sh) - 2^(sh-1)| / 2^sh, from the top 64 bits below the
       * quantum (exact enough for a hardness measure) */
      int take = sh < 63 ? (int)sh : 63;
      uint64_t low = w_getbits(M, sh - take, take);
      uint64_t half = (uint64_t)1 << (take - 1);
      uint64_t diff = low >= half ? low - half : half - low; /* exact */
      *dist = ldexp((double)diff, -take);
      if (diff == 0 && w_anybelow(M, sh - take)) *dist = ldexp(1.0, -take - 1);
    }
    if (t_mode == RM_RN) {
      if (rbit && (sticky || (mant & 1))) mant++;
    } else if (rbit || sticky) { /* inexact: step away from zero if the mode says so */
      if ((t_mode == RM_RU && !neg) || (t_mode == RM_RD && neg)) mant++;
    }
  }
  if (mant == ((uint64_t)1 << P)) {
    mant >>= 1;
    q++;
  }
  uint64_t enc;
  if (mant >> (P - 1)) {
    int64_t ex = q + P - 1;
    if (ex > emax) return overflow_enc(fmt, neg);
    enc = ((uint64_t)(ex + bias) << (P - 1)) | (mant & (((uint64_t)1 << (P - 1)) - 1));
  } else {
    enc = mant; /* subnormal */
  }
  return sign | enc;
}

/* Round both ends of y * 2^e2; returns 1 and the encoding when they agree. */
static int round_ball(const ball *y, int64_t e2, int fmt, uint64_t *enc, double *dist) {
  if (!(y->rad < 0x1p900)) return 0;
  /* R = an integer >= rad: rad = M 2^(ex-53) with M < 2^53, rounded up */
  uint64_t R[MAXL], lo[MAXL], hi[MAXL], mag[MAXL];
  memset(R, 0, sizeof(uint64_t) * L);
  {
    int ex;
    double f = frexp(y->rad, &ex);
    uint64_t M = (uint64_t)ldexp(f, 53) + 1;
    int64_t sh = (int64_t)ex - 53;
    if (sh <= 0) {
      R[0] = (M >> (-sh >= 64 ? 63 : -sh)) + 1;
    } else {
      if (sh + 54 >= 64 * L - 1) return 0;
      int64_t limb = sh >> 6, bit = sh & 63;
      R[limb] = M << bit;
      if (bit && limb + 1 < L) R[limb + 1] = M >> (64 - bit);
    }
  }
  w_sub(lo, y->w, R);
  w_add(hi, y->w, R);
  int nlo = w_isneg(lo), nhi = w_isneg(hi);
  if (nlo != nhi || w_iszero(lo) || w_iszero(hi)) return 0;
  int64_t s = e2 - FB;
  w_abs(mag, lo);
  uint64_t a = round_mag(mag, s, fmt, nlo, NULL);
  w_abs(mag, hi);
  uint64_t b = round_mag(mag, s, fmt, nhi, NULL);
  if (a != b) return 0;
  if (dist) {
    w_abs(mag, y->w);
    round_mag(mag, s, fmt, w_isneg(y->w), dist);
  }
  *enc = a;
  return 1;
}

/* ------------------------------ specials ------------------------------ */
#define QNAN32 0x7fc00000u
#define QNAN64 0x7ff8000000000000ull
#define ONE32 0x3f800000u
#define ONE64 0x3ff0000000000000ull
#define INF32 0x7f800000u
#define INF64 0x7ff0000000000000ull
#define NEG32 0x80000000u
#define NEG64 0x8000000000000000ull

/* Special inputs and results that are not decided by the Ziv loop
 * (IEEE 754-2019 Sec. 9.2 conventions for zeros, infinities, NaN and
 * domain errors; exact zero results; the one exact midpoint exp2f(-150)).
 * Also cheap saturation bounds where the result is certainly an infinity,
 * a zero or +-1.  Returns 1 when the result is decided. */
/* The rounding of +-(1 - d) for 0 < d below a quarter of an ulp of 1:
 * +-1 to nearest, else 1 or its predecessor by the mode. */
static uint64_t below_one(int fmt, int neg) {
  const uint64_t one = fmt ? ONE64 : ONE32, sign = neg ? (fmt ? NEG64 : NEG32) : 0;
  int mag_one = t_mode == RM_RN || (t_mode == RM_RU && !neg) || (t_mode == RM_RD && neg);
  return sign | (mag_one ? one : one - 1);
}

/* The rounding of a positive value below half the smallest subnormal: +0,
 * or the smallest subnormal when rounding up. */
static uint64_t tiny_positive(void) { return t_mode == RM_RU ? 1 : 0; }

static int special(int kind, int fmt, double x, uint64_t *r) {
  const uint64_t one = fmt ? ONE64 : ONE32, inf = fmt ? INF64 : INF32,
                 qnan = fmt ? QNAN64 : QNAN32, neg = fmt ? NEG64 : NEG32;
  int sn = signbit(x) != 0;
  uint64_t szero = sn ? neg : 0; /* signed zero like x */
  switch (kind) {
    case K_EXP:
    case K_EXP2:
    case K_EXP10: {
      if (x == 0) { *r = one; return 1; }
      if (isinf(x)) { *r = x > 0 ? inf : 0; return 1; }
      double hiT, loT;
      /* binary64 exp2: 2^1024 overflows; 2^-1075 is exactly the midpoint
       * between 0 and the smallest subnormal (ties to even give +0) and
       * anything below rounds to 0 */
      if (fmt && kind == K_EXP2) { hiT = 1024; loT = -1075; }
      else if (fmt) { hiT = 710; loT = -746; }
      else if (kind == K_EXP) { hiT = 100; loT = -110; }
      else if (kind == K_EXP2) { hiT = 128; loT = -151; }
      else { hiT = 40; loT = -47; }
      if (x >= hiT) { *r = overflow_enc(fmt, 0); return 1; }
      if (x <= loT) { *r = tiny_positive(); return 1; }
      /* binary32: 2^-150 is exactly the midpoint between 0 and 2^-149 (ties
       * to even give +0); in binary64 it is an ordinary representable value */
      if (!fmt && kind == K_EXP2 && x == -150) { *r = tiny_positive(); return 1; }
      return 0;
    }
    case K_EXPM1:
      if (x == 0) { *r = szero; return 1; }
      if (isinf(x)) { *r = x > 0 ? inf : (one | neg); return 1; }
      if (x >= 100) { *r = overflow_enc(fmt, 0); return 1; }
      if (x <= -40) { *r = below_one(fmt, 1); return 1; }
      return 0;
    case K_LOG:
    case K_LOG2:
    case K_LOG10:
      if (x == 0) { *r = inf | neg; return 1; }
      if (x < 0) { *r = qnan; return 1; }
      if (isinf(x)) { *r = inf; return 1; }
      if (x == 1) { *r = 0; return 1; }
      return 0;
    case K_LOG1P:
      if (x == 0) { *r = szero; return 1; }
      if (x == -1) { *r = inf | neg; return 1; }
      if (x < -1) { *r = qnan; return 1; }
      if (isinf(x)) { *r = inf; return 1; }
      return 0;
    case K_RSQRT:
      if (x == 0) { *r = inf | szero; return 1; }
      if (x < 0) { *r = qnan; return 1; }
      if (isinf(x)) { *r = 0; return 1; }
      return 0;
    case K_SIN:
    case K_TAN:
      if (x == 0) { *r = szero; return 1; }
      if (isinf(x)) { *r = qnan; return 1; }
      return 0;
    case K_COS:
      if (x == 0) { *r = one; return 1; }
      if (isinf(x)) { *r = qnan; return 1; }
      return 0;
    case K_ASIN:
      if (x == 0) { *r = szero; return 1; }
      if (fabs(x) > 1) { *r = qnan; return 1; }
      return 0;
    case K_ACOS:
      if (x == 1) { *r = 0; return 1; }
      if (fabs(x) > 1) { *r = qnan; return 1; }
      return 0;
    case K_ATAN:
      if (x == 0) { *r = szero; return 1; }
      return 0; /* +-inf: +-RN(pi/2) from the Ziv loop */
    case K_SINH:
      if (x == 0) { *r = szero; return 1; }
      if (isinf(x)) { *r = inf | (sn ? neg : 0); return 1; }
      if (fabs(x) >= 100) { *r = overflow_enc(fmt, sn); return 1; }
      return 0;
    case K_COSH:
      if (x == 0) { *r = one; return 1; }
      if (isinf(x)) { *r = inf; return 1; }
      if (fabs(x) >= 100) { *r = overflow_enc(fmt, 0); return 1; }
      return 0;
    case K_TANH:
      if (x == 0) { *r = szero; return 1; }
      if (isinf(x)) { *r = sn ? (one | neg) : one; return 1; }
      if (fabs(x) >= 50) { *r = below_one(fmt, sn); return 1; }
      return 0;
  }
  return 0;
}

/* Non-special inputs whose result is a representable number (the only ones:
 * the exact values of exp2 at integers, exp10 at 1..10, log2 at powers of 2,
 * log10 at 10..10^10, rsqrt at powers of 4; every other finite result of
 * these functions at a non-zero algebraic argument is transcendental).  In a
 * directed mode an enclosure of such a value always straddles it, so the Ziv
 * loop could not finish; the exact value is returned instead.  (To nearest,
 * the Ziv loop decides them: an exact value is never a midpoint.) */
static int exact_case(int kind, int fmt, double x, uint64_t *r) {
  static const double P10[11] = {1e0, 1e1, 1e2, 1e3, 1e4, 1e5, 1e6, 1e7, 1e8, 1e9, 1e10};
  int e;
  double m;
  switch (kind) {
    case K_EXP2:
      if (x != nearbyint(x)) return 0;
      e = (int)x;
      if (!fmt) {
        if (e < -149 || e > 127) return 0;
        *r = e >= -126 ? (uint64_t)(e + 127) << 23 : (uint64_t)1 << (e + 149);
      } else {
        if (e < -1074 || e > 1023) return 0;
        *r = e >= -1022 ? (uint64_t)(e + 1023) << 52 : (uint64_t)1 << (e + 1074);
      }
      return 1;
    case K_EXP10:
      if (fmt || x != nearbyint(x) || x < 1 || x > 10) return 0;
      {
        float v = (float)P10[(int)x]; /* 10^k < 2^34 with at most 24 significant bits */
        uint32_t b;
        memcpy(&b, &v, 4);
        *r = b;
      }
      return 1;
    case K_LOG2:
    case K_RSQRT:
      if (!(x > 0) || isinf(x)) return 0;
      m = frexp(x, &e); /* x = m 2^e, m in [1/2, 1) */
      if (m != 0.5) return 0;
      e -= 1; /* x = 2^e */
      if (kind == K_RSQRT) {
        if (e & 1) return 0;
        e = -e / 2; /* rsqrt(2^(2k)) = 2^-k, a normal binary32 number */
        *r = (uint64_t)(e + 127) << 23;
      } else {
        float v = (float)e; /* exact: |e| <= 149 */
        uint32_t b;
        memcpy(&b, &v, 4);
        *r = b;
      }
      return 1;
    case K_LOG10:
      if (fmt) return 0;
      for (int k = 1; k <= 10; k++)
        if (x == P10[k]) {
          float v = (float)k;
          uint32_t b;
          memcpy(&b, &v, 4);
          *r = b;
          return 1;
        }
      return 0;
  }
  return 0;
}

/* --------------------------- Ziv driver -------------------------------- */
static __thread int t_maxp = 0;

/* Returns 1 and the encoding on success; 0 if unresolved below PMAX. */
static int ziv(int kind, int fmt, double x, uint64_t *enc, double *hard) {
  if (special(kind, fmt, x, enc) || (t_mode != RM_RN && exact_case(kind, fmt, x, enc))) {
    if (hard) *hard = 0;
    return 1;
  }
  int p0 = fmt ? 128 : 64;
  for (int p = p0; p <= PMAX; p *= 2) {
    ball y;
    int64_t e2;
    if (p > t_maxp) t_maxp = p;
    if (ev(kind, x, p, &y, &e2)) continue;
    if (round_ball(&y, e2, fmt, enc, NULL)) {
      if (hard) {
        /* measure the distance to the nearest midpoint with 64 more bits */
        double d = 0.5;
        uint64_t e3;
        if (!(ev(kind, x, p + 64, &y, &e2) == 0 && round_ball(&y, e2, fmt, &e3, &d)))
          round_ball(&y, e2, fmt, &e3, &d);
        *hard = d > 0 ? -log2(d) : 999.0;
      }
      return 1;
    }
  }
  return 0;
}

static int kind_of(int f) {
  static const int map[F_NUM32] = {K_EXP, K_EXP2, K_EXP10, K_EXPM1, K_LOG, K_LOG2, K_LOG10,
                                   K_LOG1P, K_RSQRT, K_SIN, K_COS, -1, K_TAN, K_ASIN, K_ACOS,
                                   K_ATAN, K_SINH, K_COSH, K_TANH};
  if (f >= 0 && f < F_NUM32) return map[f];
  if (f == F_EXP) return K_EXP;
  if (f == F_LOG) return K_LOG;
  if (f == F_EXP2) return K_EXP2;
  return -2;
}

/* one binary32 element; NaN inputs return themselves, quieted */
static int eval32(int kind, uint32_t xb, uint32_t *out, double *hard) {
  if ((xb & 0x7fffffffu) > 0x7f800000u) {
    *out = xb | 0x00400000u;
    if (hard) *hard = 0;
    return 0;
  }
  float xf;
  memcpy(&xf, &xb, 4);
  uint64_t enc;
  if (!ziv(kind, 0, (double)xf, &enc, hard)) {
    *out = 0x7fc0deadu;
    return -1;
  }
  *out = (uint32_t)enc;
  return 0;
}

static int eval64(int kind, uint64_t xb, uint64_t *out, double *hard) {
  if ((xb & 0x7fffffffffffffffull) > 0x7ff0000000000000ull) {
    *out = xb | 0x0008000000000000ull;
    if (hard) *hard = 0;
    return 0;
  }
  double x;
  memcpy(&x, &xb, 8);
  uint64_t enc;
  if (!ziv(kind, 1, x, &enc, hard)) {
    *out = 0x7ff800000000deadull;
    return -1;
  }
  *out = enc;
  return 0;
}

/* ---------------------------- thread pool ----------------------------- */
typedef struct {
  int func;
  const void *in;
  void *out;
  double *hard;
  size_t n, lo, hi;
  int status, maxp, mode;
} job_t;

static void *job_run(void *arg) {
  job_t *j = (job_t *)arg;
  t_maxp = 0;
  t_mode = j->mode;
  int f = j->func, st = 0;
  for (size_t i = j->lo; i < j->hi; i++) {
    if (f == F_SINCOSF) {
      uint32_t xb = ((const uint32_t *)j->in)[i], s, c;
      double hs, hc;
      st |= eval32(K_SIN, xb, &s, j->hard ? &hs : NULL);
      st |= eval32(K_COS, xb, &c, j->hard ? &hc : NULL);
      if (j->out) {
        ((uint32_t *)j->out)[i] = s;
        ((uint32_t *)j->out)[j->n + i] = c;
      }
      if (j->hard) j->hard[i] = hs > hc ? hs : hc;
    } else if (f < F_NUM32) {
      uint32_t xb = ((const uint32_t *)j->in)[i], r;
      st |= eval32(kind_of(f), xb, &r, j->hard ? &j->hard[i] : NULL);
      if (j->out) ((uint32_t *)j->out)[i] = r;
    } else {
      uint64_t xb = ((const uint64_t *)j->in)[i], r;
      st |= eval64(kind_of(f), xb, &r, j->hard ? &j->hard[i] : NULL);
      if (j->out) ((uint64_t *)j->out)[i] = r;
    }
  }
  j->status = st;
  j->maxp = t_maxp;
  return NULL;
}

static int g_last_maxp = 0;

static int run_jobs(int func, const void *in, void *out, double *hard, size_t n, int nthreads,
                    int mode) {
  if (kind_of(func) == -2) return -1;
  if (mode < RM_RN || mode > RM_RD) return -3;
  if (n == 0) return 0;
  if (!in || (!out && !hard)) return -2;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  if ((size_t)nthreads > n) nthreads = (int)n;
  job_t jobs[256];
  pthread_t th[256];
  for (int t = 0; t < nthreads; t++) {
    jobs[t] = (job_t){func, in, out, hard, n, n * t / nthreads, n * (t + 1) / nthreads, 0, 0,
                      mode};
  }
  for (int t = 1; t < nthreads; t++) pthread_create(&th[t], NULL, job_run, &jobs[t]);
  job_run(&jobs[0]);
  for (int t = 1; t < nthreads; t++) pthread_join(th[t], NULL);
  int st = 0, mp = 0;
  for (int t = 0; t < nthreads; t++) {
    st |= jobs[t].status;
    if (jobs[t].maxp > mp) mp = jobs[t].maxp;
  }
  g_last_maxp = mp;
  return st ? -9 : 0;
}

int cr_oracle_eval(int func_id, const void *in, void *out, size_t n, int nthreads) {
  return run_jobs(func_id, in, out, NULL, n, nthreads, RM_RN);
}

int cr_oracle_eval_mode(int func_id, int mode, const void *in, void *out, size_t n,
                        int nthreads) {
  return run_jobs(func_id, in, out, NULL, n, nthreads, mode);
}

int cr_oracle_hardness(int func_id, const void *in, double *h, size_t n, int nthreads) {
  return run_jobs(func_id, in, NULL, h, n, nthreads, RM_RN);
}

int cr_oracle_last_max_prec(void) { return g_last_maxp; }

/* ------------------------- rsqrtf, exact decision ----------------------- */
/* For positive binary32 x = X 2^a (X odd or zero-free integer) and a positive
 * candidate z with neighbouring midpoints m = M 2^b, decide whether
 * 1/sqrt(x) > m by the sign of 1 - m^2 x, computed exactly with integers. */
static int above_mid(uint64_t X, int a, uint64_t M, int b) {
  /* 1/sqrt(x) > m  <=>  m^2 x < 1  <=>  M^2 X 2^(2b+a) < 1 */
  u128 v = (u128)M * M * X; /* < 2^(2*25+24) */
  int e = 2 * b + a;
  if (v == 0) return 1;
  int bl = 0;
  for (u128 t = v; t; t >>= 1) bl++;
  /* v 2^e < 1 <=> bl + e <= 0 unless v is a power of two with bl + e == 1 */
  if (bl + e <= 0) return 1;
  if (bl + e >= 2) return 0;
  /* bl + e == 1: v 2^e in [1, 2): equals 1 only if v is a power of two */
  return 0;
}

int cr_oracle_rsqrtf_exact(const float *in, float *out, size_t n) {
  if (n && (!in || !out)) return -2;
  for (size_t i = 0; i < n; i++) {
    float x = in[i];
    uint32_t xb;
    memcpy(&xb, &x, 4);
    uint64_t enc;
    if (special(K_RSQRT, 0, (double)x, &enc) || isnan(x)) {
      uint32_t r = isnan(x) ? (xb | 0x00400000u) : (uint32_t)enc;
      memcpy(&out[i], &r, 4);
      continue;
    }
    int ex;
    double fx = frexp((double)x, &ex);
    uint64_t X = (uint64_t)ldexp(fx, 24); /* x = X 2^(ex-24) */
    int a = ex - 24;
    float z = (float)(1.0 / sqrt((double)x));
    for (int it = 0; it < 4; it++) {
      /* midpoints around z: z = Z 2^c with Z in [2^23, 2^24) */
      int ez;
      double fz = frexp((double)z, &ez);
      uint64_t Z = (uint64_t)ldexp(fz, 24);
      int c = ez - 24;
      /* upper midpoint: (2Z+1) 2^(c-1) */
      if (above_mid(X, a, 2 * Z + 1, c - 1)) {
        z = nextafterf(z, INFINITY);
        continue;
      }
      /* lower midpoint: (2Z-1) 2^(c-1), or (4Z-1) 2^(c-2) at a power of two */
      uint64_t Ml = Z == ((uint64_t)1 << 23) ? 4 * Z - 1 : 2 * Z - 1;
      int bl = Z == ((uint64_t)1 << 23) ? c - 2 : c - 1;
      if (!above_mid(X, a, Ml, bl)) {
        z = nextafterf(z, 0.0f);
        continue;
      }
      break;
    }
    out[i] = z;
  }
  return 0;
}

/* ------------------------------ constants ------------------------------ */
double cr_oracle_constant(int which, int nbits, char *buf, size_t buflen) {
  if (set_fbits(nbits) || nbits % 4) return -1;
  ball c;
  switch (which) {
    case 0: c_ln2_atanh(&c); break;
    case 1: c_ln2_series(&c); break;
    case 2: c_pi_machin(&c); break;
    case 3: c_pi_euler(&c); break;
    case 4: c_ln10(&c); break;
    default: return -1;
  }
  /* value floor(c 2^nbits) = W >> (F - nbits) as hex, integer part included */
  uint64_t m[MAXL];
  w_abs(m, c.w);
  int shift = FB - nbits;
  int total = 64 * L - shift; /* bits available */
  int ndig = (total + 3) / 4;
  if ((size_t)ndig + 1 > buflen) return -1;
  int started = 0, k = 0;
  for (int d = ndig - 1; d >= 0; d--) {
    unsigned v = (unsigned)w_getbits(m, shift + 4 * d, 4);
    if (!v && !started && d > nbits / 4) continue;
    started = 1;
    buf[k++] = "0123456789abcdef"[v];
  }
  buf[k] = 0;
  return ldexp(c.rad, nbits - FB) + 1.0;
}

/* --------------------------- hard-case scan ---------------------------- */
/* Cheap double-precision estimate used ONLY to preselect candidates. */
static double estimate(int kind, double x) {
  switch (kind) {
    case K_EXP: return exp(x);
    case K_EXP2: return exp2(x);
    case K_EXP10: return exp10(x);
    case K_EXPM1: return expm1(x);
    case K_LOG: return log(x);
    case K_LOG2: return log2(x);
    case K_LOG10: return log10(x);
    case K_LOG1P: return log1p(x);
    case K_RSQRT: return 1.0 / sqrt(x);
    case K_SIN: return sin(x);
    case K_COS: return cos(x);
    case K_TAN: return tan(x);
    case K_ASIN: return asin(x);
    case K_ACOS: return acos(x);
    case K_ATAN: return atan(x);
    case K_SINH: return sinh(x);
    case K_COSH: return cosh(x);
    case K_TANH: return tanh(x);
  }
  return NAN;
}

/* distance of a double y from the nearest binary32 rounding boundary, in
 * units of the binary32 quantum at y */
static double mid_dist32(double y) {
  y = fabs(y);
  if (!(y < 0x1p128) || y == 0) return 0.5;
  int e = ilogb(y);
  int q = (e < -126 ? -126 : e) - 23;
  double s = ldexp(y, -q); /* in units of the quantum */
  double fr = s - floor(s);
  return fabs(fr - 0.5);
}

typedef struct {
  int func;
  uint64_t lo, hi;
  double pre, keep;
  uint32_t *bits;
  double *h;
  int64_t max, count;
  pthread_mutex_t *mu;
  int64_t *shared;
} scan_t;

static void *scan_run(void *arg) {
  scan_t *s = (scan_t *)arg;
  double thr = pow(2.0, -s->pre);
  int k1 = s->func == F_SINCOSF ? K_SIN : kind_of(s->func);
  int k2 = s->func == F_SINCOSF ? K_COS : -1;
  for (uint64_t u = s->lo; u < s->hi; u++) {
    uint32_t xb = (uint32_t)u;
    if ((xb & 0x7f800000u) == 0x7f800000u) continue;
    float xf;
    memcpy(&xf, &xb, 4);
    double x = xf, r;
    uint64_t enc;
    int cand = 0;
    if (!special(k1, 0, x, &enc)) {
      double y = estimate(k1, x);
      if (isfinite(y) && mid_dist32(y) < thr) cand = 1;
    }
    if (!cand && k2 >= 0 && !special(k2, 0, x, &enc)) {
      double y = estimate(k2, x);
      if (isfinite(y) && mid_dist32(y) < thr) cand = 1;
    }
    if (!cand) continue;
    double h = 0;
    if (s->func == F_SINCOSF) {
      double h1 = 0, h2 = 0;
      uint32_t o;
      eval32(K_SIN, xb, &o, &h1);
      eval32(K_COS, xb, &o, &h2);
      h = h1 > h2 ? h1 : h2;
    } else {
      uint32_t o;
      eval32(k1, xb, &o, &h);
    }
    (void)r;
    if (h >= s->keep) {
      pthread_mutex_lock(s->mu);
      int64_t idx = (*s->shared)++;
      if (idx < s->max) {
        s->bits[idx] = xb;
        s->h[idx] = h;
      }
      pthread_mutex_unlock(s->mu);
    }
  }
  return NULL;
}

int64_t cr_oracle_scan_f32(int func_id, uint32_t lo, uint64_t hi, double h_prefilter,
                           double h_keep, uint32_t *out_bits, double *out_h, int64_t max_out,
                           int nthreads) {
  if (func_id < 0 || func_id >= F_NUM32) return -1;
  if (hi > 0x100000000ull || hi < lo) return -1;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  pthread_mutex_t mu = PTHREAD_MUTEX_INITIALIZER;
  int64_t shared = 0;
  scan_t jobs[256];
  pthread_t th[256];
  uint64_t span = hi - lo;
  for (int t = 0; t < nthreads; t++) {
    jobs[t] = (scan_t){func_id, lo + span * t / nthreads, lo + span * (t + 1) / nthreads,
                       h_prefilter, h_keep, out_bits, out_h, max_out, 0, &mu, &shared};
  }
  for (int t = 1; t < nthreads; t++) pthread_create(&th[t], NULL, scan_run, &jobs[t]);
  scan_run(&jobs[0]);
  for (int t = 1; t < nthreads; t++) pthread_join(th[t], NULL);
  return shared;
}

/* Sampled hard-case scan for binary64 exp/log/exp2: a quad-precision estimate
 * (libquadmath) preselects candidates within 2^-h_prefilter ulp of a
 * binary64 midpoint; the oracle then measures each candidate's hardness. */
#include <quadmath.h>

static double mid_dist64q(__float128 y) {
  y = fabsq(y);
  if (!(y < 0x1p1024Q) || y == 0) return 0.5;
  int e = ilogbq(y);
  int q = (e < -1022 ? -1022 : e) - 52;
  __float128 s = ldexpq(y, -q);
  __float128 fr = s - floorq(s);
  return (double)fabsq(fr - 0.5Q);
}

typedef struct {
  int kind;
  const double *x;
  size_t lo, hi;
  double pre, keep;
  double *ox, *oh;
  int64_t max;
  pthread_mutex_t *mu;
  int64_t *shared;
} scan64_t;

static void *scan64_run(void *arg) {
  scan64_t *s = (scan64_t *)arg;
  double thr = pow(2.0, -s->pre);
  for (size_t i = s->lo; i < s->hi; i++) {
    double x = s->x[i];
    uint64_t enc;
    if (isnan(x) || special(s->kind, 1, x, &enc)) continue;
    __float128 y = s->kind == K_EXP    ? expq((__float128)x)
                   : s->kind == K_EXP2 ? exp2q((__float128)x)
                                       : logq((__float128)x);
    if (!(mid_dist64q(y) < thr)) continue;
    uint64_t xb, o;
    double h = 0;
    memcpy(&xb, &x, 8);
    eval64(s->kind, xb, &o, &h);
    if (h >= s->keep) {
      pthread_mutex_lock(s->mu);
      int64_t idx = (*s->shared)++;
      if (idx < s->max) {
        s->ox[idx] = x;
        s->oh[idx] = h;
      }
      pthread_mutex_unlock(s->mu);
    }
  }
  return NULL;
}

int64_t cr_oracle_scan_f64(int func_id, const double *x, size_t n, double h_prefilter,
                           double h_keep, double *out_x, double *out_h, int64_t max_out,
                           int nthreads) {
  if (func_id != F_EXP && func_id != F_LOG && func_id != F_EXP2) return -1;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  pthread_mutex_t mu = PTHREAD_MUTEX_INITIALIZER;
  int64_t shared = 0;
  scan64_t jobs[256];
  pthread_t th[256];
  for (int t = 0; t < nthreads; t++)
    jobs[t] = (scan64_t){kind_of(func_id), x, n * t / nthreads, n * (t + 1) / nthreads,
                         h_prefilter, h_keep, out_x, out_h, max_out, &mu, &shared};
  for (int t = 1; t < nthreads; t++) pthread_create(&th[t], NULL, scan64_run, &jobs[t]);
  scan64_run(&jobs[0]);
  for (int t = 1; t < nthreads; t++) pthread_join(th[t], NULL);
  return shared;
}
