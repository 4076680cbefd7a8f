"""Oracle of the paper's application workloads (paper, Sec. III-A).

TEST INFRASTRUCTURE ONLY: imported by the test suite and the benchmark's CPU
baseline; the GPU library never imports it.

The paper runs two synthetic applications on top of its correctly rounded
binary32 functions:

1. Spectral interpolation at a non-integer frequency by a brute-force
   discrete Fourier transform of the original time samples, which spends its
   time in sin and cos (or sincos).
2. Complex expf, logf and sinf accurate to 2 ulps on valid inputs, built from
   the correctly rounded real functions (cexpf from expf, sinf and cosf;
   clogf from logf, log1pf and atanf plus division; csinf from coshf, sinhf,
   cosf and sinf), with real and imaginary parts in [-40, 40].

The paper gives the ingredients, not the formulas; the compositions below are
this project's (the GPU library evaluates the same compositions).  Each
function states what it computes; every correctly rounded step is the
oracle's own RN(f(x)) (oracle.evaluate), every other step is one IEEE 754
operation in the stated format (numpy float32 / float64 arithmetic rounds to
nearest even).

Error bounds (pinned against mpmath in tests/test_apps_oracle.py):
  * cexpf, csinf: each component is RN32(A B) with A, B correctly rounded;
    with a, b the significands of A, B in [1, 2), the two input errors add at
    most (1/a + 1/b)/2 ulp of the product's significand scale, i.e. at most
    1.5 ulp of the result, and the product's rounding 0.5 ulp: 2 ulps.
  * clogf: below 1.5 ulp for both components (see clogf).
  * dft: the transform is a sum in binary64 of exact products; its oracle is
    the correctly rounded sum of those products (math.fsum).
"""
import math

import numpy as np

from . import oracle as O

f32 = np.float32
f64 = np.float64

PI_D = f64(math.pi)        # RN64(pi)
PI2_D = f64(math.pi / 2)   # RN64(pi/2): pi/2 in binary64 is exactly math.pi / 2


def _split(z):
    z = np.ascontiguousarray(z, dtype=np.float32).reshape(-1, 2)
    return z[:, 0].copy(), z[:, 1].copy()


def _join(re, im):
    out = np.empty((re.size, 2), dtype=np.float32)
    out[:, 0] = re
    out[:, 1] = im
    return out.reshape(-1)


def cexpf(z, nthreads=None):
    """exp(x + iy) = e^x cos y + i e^x sin y for interleaved binary32 pairs
    (x, y): re = RN32(expf(x) cosf(y)), im = RN32(expf(x) sinf(y)), with
    expf, sinf, cosf correctly rounded.  Valid inputs: finite x below 88.7
    (no overflow of e^x) and any finite y."""
    x, y = _split(z)
    E = O.evaluate("expf", x, nthreads)
    S, C = O.evaluate("sincosf", y, nthreads)
    return _join(E * C, E * S)


def csinf(z, nthreads=None):
    """sin(x + iy) = sin x cosh y + i cos x sinh y: re = RN32(sinf(x)
    coshf(y)), im = RN32(cosf(x) sinhf(y)), each factor correctly rounded.
    Valid inputs: finite x, |y| below 89.4 (cosh y finite)."""
    x, y = _split(z)
    S, C = O.evaluate("sincosf", x, nthreads)
    Ch = O.evaluate("coshf", y, nthreads)
    Sh = O.evaluate("sinhf", y, nthreads)
    return _join(S * Ch, C * Sh)


def clogf(z, nthreads=None):
    """log(x + iy) = log|z| + i atan2(y, x) for interleaved binary32 pairs.

    Valid inputs: finite, 2^-63 <= |z| < 2^63 (so x^2 + y^2 stays a normal
    binary32 number when rounded).

    Imaginary part: a = max(|x|, |y|), b = min(|x|, |y|), t = RN32(b / a),
    A = atanf(t) (correctly rounded, in [0, pi/4]); in binary64,
    v = A, then v = RN64(pi/2) - v if |y| > |x|, then v = RN64(pi) - v if
    x < 0 (sign bit clear compares false for -0, as atan2 wants); the result
    is RN32(v) with the sign of y.  Error: t carries 2^-24 t, which moves
    atan by at most 2^-24 t/(1 + t^2); with atanf's own half ulp and the
    final rounding this stays below 1.5 ulp.

    Real part, with s = RN64(a^2 + b^2) (the squares are exact in binary64):
      * 0.5 <= s < 2 (|z| near 1, where log|z| is small): d = RN64((a^2 - 1)
        + b^2) (a^2 - 1 is exact since a^2 is in [0.25, 2)), d_hi = RN32(d),
        d_lo = d - d_hi (exact), L = log1pf(d_hi), re = RN32(0.5 (L + RN64(
        d_lo / (1 + d_hi)))) -- log1p(d) = log1p(d_hi) + log1p(d_lo/(1 + d_hi));
      * otherwise: s_hi = RN32(s), s_lo = s - s_hi (exact), L = logf(s_hi),
        re = RN32(0.5 (L + RN64(s_lo / s_hi))) -- log s = log s_hi + log1p(s_lo/s_hi).
    The correction term leaves a second-order error below 2^-46 relative, so
    the error is L's half ulp (at most one ulp of the result after halving,
    binade changes included) plus the final rounding: below 1.5 ulp.
    All binary64 sums are evaluated left to right as written.
    """
    x, y = _split(z)
    ax, ay = np.abs(x), np.abs(y)
    a = np.maximum(ax, ay)
    b = np.minimum(ax, ay)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = (b / a).astype(f32)
    A = O.evaluate("atanf", t, nthreads)
    v = A.astype(f64)
    v = np.where(ay > ax, PI2_D - v, v)
    v = np.where(x < 0, PI_D - v, v)
    im = np.copysign(v.astype(f32), y)

    a64, b64 = a.astype(f64), b.astype(f64)
    s = a64 * a64 + b64 * b64
    near = (s >= 0.5) & (s < 2.0)
    d = (a64 * a64 - 1.0) + b64 * b64
    d_hi = d.astype(f32)
    d_lo = d - d_hi.astype(f64)
    s_hi = s.astype(f32)
    s_lo = s - s_hi.astype(f64)
    arg = np.where(near, d_hi, s_hi)
    L1 = O.evaluate("log1pf", np.where(near, arg, f32(0)), nthreads)
    L0 = O.evaluate("logf", np.where(near, f32(1), arg), nthreads)
    with np.errstate(divide="ignore", invalid="ignore"):
        corr_near = d_lo / (1.0 + d_hi.astype(f64))
        corr_far = s_lo / s_hi.astype(f64)
    re_near = (0.5 * (L1.astype(f64) + corr_near)).astype(f32)
    re_far = (0.5 * (L0.astype(f64) + corr_far)).astype(f32)
    re = np.where(near, re_near, re_far)
    return _join(re, im)


COMPLEX = {"cexpf": cexpf, "clogf": clogf, "csinf": csinf}


def evaluate_complex(func, z, nthreads=None):
    return COMPLEX[func](z, nthreads)


def dft_phases(w, n0, n1):
    """theta[k, n] = RN32(w[k] n) for n in [n0, n1) (binary32 product of the
    per-sample angle w[k] and the exact sample index n < 2^24)."""
    w = np.asarray(w, dtype=np.float32)
    n = np.arange(n0, n1, dtype=np.float32)
    return (w[:, None] * n[None, :]).astype(f32)


def dft(x, w, nthreads=None):
    """Brute-force DFT of the real samples x at per-sample angles w (one per
    output frequency: w_k = 2 pi f_k / N for a frequency f_k in bins, rounded
    to binary32):

        X_k = sum_n x[n] (cos theta_kn - i sin theta_kn),  theta_kn = RN32(w_k n),

    with sin and cos correctly rounded (sincosf).  Each product x[n] cos
    theta_kn of two binary32 numbers is exact in binary64; X_k here is the
    correctly rounded binary64 sum of those exact products (math.fsum).

    Returns (X, mag) with X of shape (M, 2) binary64 (re, im) and mag[k] =
    (sum |x c|, sum |x s|), the scale of each sum's rounding error.
    """
    x = np.asarray(x, dtype=np.float32)
    w = np.asarray(w, dtype=np.float32)
    N = x.size
    if N >= (1 << 24):
        raise ValueError("sample indices must be exact in binary32")
    X = np.zeros((w.size, 2), dtype=np.float64)
    mag = np.zeros((w.size, 2), dtype=np.float64)
    xd = x.astype(np.float64)
    for k in range(w.size):
        th = dft_phases(w[k:k + 1], 0, N)[0]
        s, c = O.evaluate("sincosf", th, nthreads)
        pc = xd * c.astype(np.float64)   # exact
        ps = xd * s.astype(np.float64)   # exact
        X[k, 0] = math.fsum(pc.tolist())
        X[k, 1] = -math.fsum(ps.tolist())
        mag[k, 0] = math.fsum(np.abs(pc).tolist())
        mag[k, 1] = math.fsum(np.abs(ps).tolist())
    return X, mag
