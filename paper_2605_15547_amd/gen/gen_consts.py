"""Generates paper_2605_15547_amd/csrc/cr_consts.h: tables and polynomial
coefficients of the GPU kernels.

Everything is computed here with mpmath at high precision and rounded to
binary64 (or to double-double pairs hi + lo).  Polynomial coefficients come
from a weighted minimax fit (Lawson's iteratively reweighted least squares);
each approximation's error bound is measured on a dense grid with the ROUNDED
coefficients to choose the degree; the bound written next to the coefficients
(for the kernels' rounding tests to budget for) is a proven one: Taylor's
theorem with the Lagrange remainder on subintervals (gen/bounds.py).

The paper prints no coefficients (its listings elide them); these are this
project's own.  Run:  python paper_2605_15547_amd/gen/gen_consts.py
"""
import os
import sys

import mpmath as mp

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import bounds as B  # noqa: E402

mp.mp.prec = 200
HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(os.path.dirname(HERE), "csrc", "cr_consts.h")


# ------------------------------------------------------------ rounding utils
def d(x):
    """round to binary64 (RN)"""
    return float(mp.mpf(x))


def dd(x):
    """double-double (hi, lo) with hi = RN(x), lo = RN(x - hi)"""
    x = mp.mpf(x)
    hi = float(x)
    lo = float(x - mp.mpf(hi))
    return hi, lo


def td(x):
    hi = float(x)
    r = x - mp.mpf(hi)
    mid = float(r)
    lo = float(r - mp.mpf(mid))
    return hi, mid, lo


def split_bits(x, bits):
    """x rounded to `bits` significant bits, as a double"""
    x = mp.mpf(x)
    e = int(mp.floor(mp.log(abs(x), 2)))
    q = mp.mpf(2) ** (e - bits + 1)
    return float(mp.nint(x / q) * q)


def hexd(v):
    return float(v).hex()


# --------------------------------------------------------- minimax fitting
def cheb_nodes(a, b, n):
    a, b = mp.mpf(a), mp.mpf(b)
    return [(a + b) / 2 + (b - a) / 2 * mp.cos(mp.pi * (2 * i + 1) / (2 * n)) for i in range(n)]


def lawson_fit(g, w, a, b, powers, npts=500, iters=40):
    """Coefficients c_k (mp) minimising max |w(x) (g(x) - sum c_k x^p_k)| on [a,b].
    The fit runs in the scaled variable u = x / max(|a|, |b|) (bounded powers,
    well-conditioned normal equations) at 400 bits."""
    with mp.workprec(400):
        sc = max(abs(mp.mpf(a)), abs(mp.mpf(b)))
        xs = cheb_nodes(a, b, npts) + [mp.mpf(a), mp.mpf(b)]
        gs = [g(x) for x in xs]
        ws = [w(x) for x in xs]
        wmax = max(abs(v) for v in ws)
        ws = [v / wmax for v in ws]
        us = [x / sc for x in xs]
        W = [mp.mpf(1)] * len(xs)
        m = len(powers)
        c = None
        for _ in range(iters):
            A = mp.matrix(m, m)
            B = mp.matrix(m, 1)
            for u, gx, wx, Wi in zip(us, gs, ws, W):
                s2 = Wi * wx * wx
                pw = [u ** p for p in powers]
                for k in range(m):
                    B[k] += s2 * gx * pw[k]
                    for l in range(m):
                        A[k, l] += s2 * pw[k] * pw[l]
            c = mp.lu_solve(A, B)
            errs = [abs(wx * (gx - sum(c[k] * u ** powers[k] for k in range(m))))
                    for u, gx, wx in zip(us, gs, ws)]
            tot = sum(Wi * e for Wi, e in zip(W, errs))
            W = [Wi * e / tot for Wi, e in zip(W, errs)]
        return [c[k] / sc ** powers[k] for k in range(m)]


def max_err(fn, a, b, n=4000):
    """max |fn(x)| on a dense grid of [a,b] (plus Chebyshev points)"""
    a, b = mp.mpf(a), mp.mpf(b)
    pts = [a + (b - a) * i / n for i in range(n + 1)] + cheb_nodes(a, b, 1000)
    return max(abs(fn(x)) for x in pts)


def log2_of(x):
    return float(mp.log(x, 2)) if x > 0 else -9999.0


# ------------------------------------------------------------- header text
lines = []


def emit(s=""):
    lines.append(s)


def emit_dd_table(name, vals, comment):
    emit("// " + comment)
    emit("__device__ __constant__ const double2 %s[%d] = {" % (name, len(vals)))
    for v in vals:
        hi, lo = dd(v)
        emit("  {%s, %s}," % (hexd(hi), hexd(lo)))
    emit("};")


def emit_td_table(name, vals, comment):
    emit("// " + comment)
    emit("__device__ __constant__ const double4 %s[%d] = {" % (name, len(vals)))
    for v in vals:
        a, b, c = td(mp.mpf(v))
        emit("  {%s, %s, %s, 0.0}," % (hexd(a), hexd(b), hexd(c)))
    emit("};")


def emit_arr(name, vals, comment, ctype="double"):
    """Coefficient arrays are left non-const on purpose: the compiler then
    loads them once per kernel into scalar registers (uniform loads) and feeds
    them to v_fma_f64 as its scalar operand, instead of rebuilding each 64-bit
    constant in vector registers at every use."""
    emit("// " + comment)
    emit("__device__ __constant__ %s %s[%d] = {%s};" %
         (ctype, name, len(vals), ", ".join(hexd(v) for v in vals)))


def emit_const(name, v, comment=""):
    emit("#define %s (%s)%s" % (name, hexd(v), ("  /* " + comment + " */") if comment else ""))


# =================================================================== exp family
def gen_exp():
    ln2 = mp.log(2)
    emit("// ---- exponential family (expf, exp2f, exp10f, expm1f, sinhf, coshf, tanhf) ----")
    emit_dd_table("EXP_T16", [mp.power(2, mp.mpf(j) / 16) for j in range(16)],
                  "2^(j/16), j = 0..15, as double-double (hi, lo)")
    # Cody-Waite split of ln2/16: C1 has 41 significant bits so that k*C1 is
    # exact for |k| < 2^12 and x - k*C1 is exact (see kernel comment).
    c = ln2 / 16
    c1 = split_bits(c, 41)
    r1 = c - mp.mpf(c1)
    c2 = float(r1)
    c3 = float(r1 - mp.mpf(c2))
    emit_const("LN2_16_C1", c1, "ln2/16 rounded to 41 bits")
    emit_const("LN2_16_C2", c2, "next 53 bits of ln2/16")
    emit_const("LN2_16_C3", c3, "next 53 bits of ln2/16")
    emit_const("INV_LN2_16", d(16 / ln2), "16/ln2")
    h, l = dd(ln2 / 16)
    emit_const("LN2_16_HI", h, "ln2/16 hi")
    emit_const("LN2_16_LO", l, "ln2/16 lo")
    h, l = dd(16 * mp.log(10) / ln2)
    emit_const("LOG2_10_16_HI", h, "16 log2(10) hi")
    emit_const("LOG2_10_16_LO", l, "16 log2(10) lo")
    # exp10f fast reduction: C = 16 log2(10) = C1 + C2 with C1 on 28 bits, so
    # that x C1 is exact for binary32 x; C2 enters pre-multiplied by ln2/16
    c = 16 * mp.log(10) / ln2
    c1 = split_bits(c, 28)
    emit_const("LOG2_10_16_C1", c1, "16 log2(10) rounded to 28 bits")
    emit_const("EXP10_C2_LN2_16", d((c - mp.mpf(c1)) * ln2 / 16), "(16 log2(10) - C1) ln2/16")
    h, l = dd(mp.log(10))
    emit_const("LN10_HI", h, "ln 10 hi")
    emit_const("LN10_LO", l, "ln 10 lo")
    h, l = dd(ln2)
    emit_const("LN2_HI", h, "ln 2 hi")
    emit_const("LN2_LO", l, "ln 2 lo")

    # fast path: e^r - 1 = r + r^2 P(r), |r| <= RHO
    rho = mp.mpf("0.02167")  # (1/2 + 2^-40) ln2/16 < 0.02167
    for deg in range(3, 9):
        powers = list(range(deg + 1))
        cs = lawson_fit(lambda r: (mp.expm1(r) - r) / (r * r) if r != 0 else mp.mpf(0.5),
                        lambda r: r * r, -rho, rho, powers)
        cd = [d(v) for v in cs]
        err = max_err(lambda r: mp.expm1(r) - r - r * r * sum(mp.mpf(cd[k]) * r ** k
                                                              for k in range(len(cd))),
                      -rho, rho)
        if err < mp.mpf(2) ** -63:
            break
    bound = B.sup_bound(B.expm1_minus_r([mp.mpf(v) for v in cd], rho))
    emit("// e^r - 1 = r + r^2 (P0 + P1 r + ...), |r| <= %s; |error| <= 2^%.2f (absolute, proven)"
         % (mp.nstr(rho, 6), log2_of(bound)))
    emit_arr("EXPM1_P", cd, "minimax coefficients P0.. (degree %d)" % (len(cd) - 1))
    emit("#define EXPM1_P_DEG %d" % (len(cd) - 1))
    emit_const("EXPM1_P_ERR", d(bound), "bound on the approximation error")

    # accurate path: Taylor series of e^r - 1 to degree N in double-double
    N = 14
    rem = rho ** (N + 1) / mp.factorial(N + 1) * 2
    emit("// 1/k!, k = 0..%d, double-double (Taylor series of e^r, |r| <= %s: "
         "remainder <= 2^%.1f)" % (N, mp.nstr(rho, 6), log2_of(rem)))
    emit("#define EXP_TAYLOR_N %d" % N)
    emit_dd_table("INV_FACT", [1 / mp.factorial(k) for k in range(N + 1)], "1/k!")
    emit()


# =================================================================== log family
def log_intervals():
    """The 16 intervals of the reduced mantissa and their reciprocals c_j.

    m in [1,2) is indexed by its top 4 fraction bits j; for j >= 8 the kernel
    uses m' = m/2 in [0.75, 1) (and e' = e + 1), so the value range is
    [0.75, 1.5).  c_j ~ 1/center rounded to 9 significant bits (so m * c_j is
    exact for 24-bit m), and c_j = 1 on the two intervals next to 1 so that
    log(x) near x = 1 is t + ... with no cancellation."""
    out = []
    for j in range(16):
        if j < 8:
            lo, hi = 1 + mp.mpf(j) / 16, 1 + mp.mpf(j + 1) / 16
        else:
            lo, hi = (1 + mp.mpf(j) / 16) / 2, (1 + mp.mpf(j + 1) / 16) / 2
        if j in (0, 15):
            c = mp.mpf(1)
        else:
            c = mp.mpf(split_bits(2 / (lo + hi), 9))
        out.append((lo, hi, c))
    return out


def gen_log():
    emit("// ---- logarithm family (logf, log2f, log10f, log1pf) ----")
    iv = log_intervals()
    tmin = min(lo * c - 1 for lo, hi, c in iv)
    tmax = max(hi * c - 1 for lo, hi, c in iv)
    emit("// reduced argument t = m c_j - 1 lies in [%s, %s]" % (mp.nstr(tmin, 8), mp.nstr(tmax, 8)))
    emit_arr("LOG_C", [float(c) for _, _, c in iv], "c_j (9 significant bits)")
    # K = 1/ln b on 20 bits: K t is exact for the <= 33-bit t of binary32
    # inputs, and Q(0) = 1/ln b - K is tiny, so rounding Q's coefficients costs
    # nothing measurable
    bases = [("E", mp.mpf(1), mp.mpf(1)),
             ("2", 1 / mp.log(2), mp.mpf(split_bits(1 / mp.log(2), 20))),
             ("10", 1 / mp.log(10), mp.mpf(split_bits(1 / mp.log(10), 20)))]
    # -log_b(c_j) in three parts: hi a multiple of 2^-44 (2^-45 for b = 10), so
    # that e' C_hi + hi is exact (both multiples of that quantum, the sum below
    # 2^8), then lo = RN(rest) and z = RN(rest - lo) (for the accurate paths)
    for name, inv_ln, K in bases:
        q = mp.mpf(2) ** (-45 if name == "10" else -44)
        his, los, zs = [], [], []
        for _, _, c in iv:
            v = -mp.log(c) * inv_ln
            hi = float(mp.nint(v / q) * q)
            r = v - mp.mpf(hi)
            lo = float(r)
            his.append(hi)
            los.append(lo)
            zs.append(float(r - mp.mpf(lo)))
        b = "e" if name == "E" else name
        emit("// -log_b(c_j), b = %s: {hi (a multiple of 2^%d), lo}" % (b, -45 if name == "10" else -44))
        emit("__device__ __constant__ const double2 LOG%s_L[16] = {" % name)
        for hi, lo in zip(his, los):
            emit("  {%s, %s}," % (hexd(hi), hexd(lo)))
        emit("};")
        emit_arr("LOG%s_LZ" % name, zs, "-log_b(c_j) - hi - lo, b = %s" % b)
    # e' * C with C_hi on 44 bits so that e' C_hi is exact for |e'| < 2^9
    for name, v in (("E", mp.log(2)), ("10", mp.log10(2))):
        hi = split_bits(v, 44)
        emit_const("LOG%s_C_HI" % name, hi, "log_b(2), 44 bits")
        emit_const("LOG%s_C_LO" % name, d(v - mp.mpf(hi)), "log_b(2) - C_HI")
    a, b = tmin * mp.mpf("1.0001"), tmax * mp.mpf("1.0001")
    for name, inv_ln, K in bases:
        g = (lambda il, KK: (lambda t: (mp.log1p(t) * il / t - KK) if t != 0 else il - KK))(inv_ln, K)
        # the fast path's test allows 8 ulps; Q within 2^-57 keeps the whole
        # fast-path error below about 2.5 ulps (see cr_f32_log.h)
        for deg in range(6, 16):
            cs = lawson_fit(g, lambda t: mp.mpf(1), a, b, list(range(deg + 1)), npts=160, iters=16)
            cd = [d(v) for v in cs]
            err = max_err(lambda t: g(t) - sum(mp.mpf(cd[k]) * t ** k for k in range(len(cd))), a, b)
            if err < mp.mpf(2) ** -57:
                break
        bound = B.sup_bound(B.log_b_quotient([mp.mpf(v) for v in cd],
                                             {"E": "e", "2": "2", "10": "10"}[name],
                                             mp.mpf(d(K)), a, b))
        emit("// log_b(1+t) = K t + t Q(t), K = %s, t in [%s, %s]; |Q error| <= 2^%.2f (proven)"
             % (mp.nstr(K, 5), mp.nstr(a, 6), mp.nstr(b, 6), log2_of(bound)))
        emit_arr("LOG%s_Q" % name, cd, "Q coefficients (degree %d)" % (len(cd) - 1))
        emit("#define LOG%s_Q_DEG %d" % (name, len(cd) - 1))
        emit_const("LOG%s_K" % name, d(K))
    # accurate path
    for name, inv_ln, K in bases[1:]:
        h, l = dd(inv_ln)
        emit_const("INV_LN%s_HI" % name, h)
        emit_const("INV_LN%s_LO" % name, l)
    h, l = dd(mp.log10(2))
    emit_const("LOG10_2_HI", h)
    emit_const("LOG10_2_LO", l)
    emit()


# =================================================================== trig family
def gen_trig():
    emit("// ---- trigonometric family (sinf, cosf, sincosf, tanf) ----")
    # 2/pi = sum g_i 2^-i; word k (k >= 2) holds bits 32(k-2)+1 .. 32(k-1); words
    # 0 and 1 are zero so that windows may start up to 64 bits before the binary
    # point (arguments down to 2^-37 reduce correctly)
    words = [0, 0]
    with mp.workprec(800):  # 288 table bits need far more than the default precision
        two_over_pi = 2 / mp.pi
        for k in range(1, 10):
            words.append(int(mp.floor(two_over_pi * mp.mpf(2) ** (32 * k))) & 0xFFFFFFFF)
    emit("// bits of 2/pi: word k (k >= 2) = bits 32(k-2)+1 .. 32(k-1); words 0, 1 = 0")
    emit("__device__ __constant__ const unsigned TWO_OVER_PI_W[11] = {%s};"
         % ", ".join("0x%08xu" % w for w in words))
    h, m1, l = td(mp.pi / 32)
    emit_const("PI32_HI", h, "pi/32")
    emit_const("PI32_MID", m1)
    emit_const("PI32_LO", l)
    emit_const("PI64", d(mp.pi / 64), "pi/64 (small-argument threshold)")
    # Cody-Waite form of the reduction for |x| < 2^23 (|k| < 2^26.4): pi/32 in
    # three parts, the first on 26 bits so that k CW1 is exact
    with mp.workprec(800):
        c = mp.pi / 32
        c1 = split_bits(c, 26)
        rem = c - mp.mpf(c1)
        c2 = float(rem)
        c3 = float(rem - mp.mpf(c2))
    emit_const("PI32_CW1", c1, "pi/32 rounded to 26 bits")
    emit_const("PI32_CW2", c2)
    emit_const("PI32_CW3", c3)
    emit_const("INV_PI32", d(32 / mp.pi), "32/pi")
    emit("// sin(j pi/32), cos(j pi/32) for j = 0..15, double-double: {s_hi, s_lo, c_hi, c_lo}")
    emit("__device__ __constant__ const double4 SINCOS_T[16] = {")
    for j in range(16):
        sh, sl = dd(mp.sin(j * mp.pi / 32))
        ch, cl = dd(mp.cos(j * mp.pi / 32))
        emit("  {%s, %s, %s, %s}," % (hexd(sh), hexd(sl), hexd(ch), hexd(cl)))
    emit("};")
    rho = mp.pi / 64 * mp.mpf("1.0001")
    # fast path: sin r = r + r^3 S2(r^2), cos r - 1 = r^2 C2(r^2), degree 2 in
    # r^2, for the fast path's error budget (its rounding test allows 2^-45
    # relative)
    for name, g, w in (
            ("SIN_S2", lambda u: (mp.sin(mp.sqrt(u)) / mp.sqrt(u) - 1) / u if u != 0 else mp.mpf(-1) / 6,
             lambda u: u * mp.sqrt(u)),
            ("COS_C2", lambda u: (mp.cos(mp.sqrt(u)) - 1) / u if u != 0 else mp.mpf(-1) / 2,
             lambda u: u)):
        cs = lawson_fit(g, w, mp.mpf(0), rho * rho, [0, 1, 2], npts=120, iters=16)
        cd = [d(v) for v in cs]
        mk = B.sin_minus_r if name == "SIN_S2" else B.cos_minus_1
        bound = B.sup_bound(mk([mp.mpf(v) for v in cd], rho))
        emit("// %s (fast path): |r| <= pi/64; |approximation error| <= 2^%.2f (absolute, proven)"
             % ("sin r = r + r^3 S2(r^2)" if name == "SIN_S2" else "cos r - 1 = r^2 C2(r^2)",
                log2_of(bound)))
        emit_arr(name, cd, "coefficients (degree 2 in r^2)")
    # accurate path: Taylor coefficients (-1)^k / (2k+1)! and (-1)^k / (2k)!
    N = 9
    emit("#define TRIG_TAYLOR_N %d" % N)
    emit_dd_table("SIN_TAYLOR", [(-1) ** k / mp.factorial(2 * k + 1) for k in range(N + 1)],
                  "(-1)^k/(2k+1)!  (|r| <= pi/64: the omitted terms are below 2^-120 |r|)")
    emit_dd_table("COS_TAYLOR", [(-1) ** k / mp.factorial(2 * k) for k in range(N + 1)],
                  "(-1)^k/(2k)!")
    emit()


# ============================================================= inverse trig family
def gen_atan():
    emit("// ---- inverse trigonometric family (atanf, asinf, acosf) ----")
    emit("// {atan(j/16) hi, lo, (pi/2 - atan(j/16)) hi, lo}, j = 0..15")
    emit("__device__ __constant__ const double4 ATAN_T[16] = {")
    for j in range(16):
        a = mp.atan(mp.mpf(j) / 16)
        ah, al = dd(a)
        bh, bl = dd(mp.pi / 2 - a)
        emit("  {%s, %s, %s, %s}," % (hexd(ah), hexd(al), hexd(bh), hexd(bl)))
    emit("};")
    h, l = dd(mp.pi)
    emit_const("PI_HI", h)
    emit_const("PI_LO", l)
    h, l = dd(mp.pi / 2)
    emit_const("PIO2_HI", h)
    emit_const("PIO2_LO", l)
    # |t| <= (1/2)/(16 + 15/16) < 0.0296 for y <= x; the other branch is
    # symmetric; 1/31 covers both with margin
    rho = mp.mpf(1) / 31
    for deg in range(3, 8):
        cs = lawson_fit(lambda u: (mp.atan(mp.sqrt(u)) / mp.sqrt(u) - 1) / u if u != 0 else mp.mpf(-1) / 3,
                        lambda u: u * mp.sqrt(u), mp.mpf(0), rho * rho, list(range(deg + 1)),
                        npts=120, iters=16)
        cd = [d(v) for v in cs]
        err = max_err(lambda t: mp.atan(t) - t - t ** 3 * sum(mp.mpf(cd[k]) * t ** (2 * k)
                                                               for k in range(len(cd))),
                      mp.mpf(0), rho)
        if err < mp.mpf(2) ** -66:
            break
    emit("// atan t = t + t^3 P(t^2), |t| <= 1/31; |error| <= 2^%.2f (absolute, proven)"
         % log2_of(B.sup_bound(B.atan_minus_t([mp.mpf(v) for v in cd], rho))))
    emit_arr("ATAN_P", cd, "coefficients (degree %d in t^2)" % (len(cd) - 1))
    emit("#define ATAN_P_DEG %d" % (len(cd) - 1))
    N = 12
    emit("#define ATAN_TAYLOR_N %d" % N)
    emit_dd_table("ATAN_TAYLOR", [mp.mpf(-1) ** k / (2 * k + 1) for k in range(N + 1)],
                  "(-1)^k/(2k+1)  (|t| <= 1/31: omitted terms below 2^-125 |t|)")
    emit()


# ============================================================ binary64 exp / log
def gen_f64():
    emit("// ---- binary64 exp and log ----")
    with mp.workprec(600):
        ln2 = mp.log(2)
        emit_td_table("EXP64_T1", [mp.power(2, mp.mpf(i) / 16) for i in range(16)],
                      "2^(i/16) as triple-double {hi, mid, lo, 0}")
        emit_td_table("EXP64_T2", [mp.power(2, mp.mpf(i) / 256) for i in range(16)],
                      "2^(i/256) as triple-double {hi, mid, lo, 0}")
        # ln2/256 in four parts; C1 on 34 bits: k C1 exact for |k| < 2^19
        c = ln2 / 256
        c1 = split_bits(c, 34)
        r = c - mp.mpf(c1)
        c2 = float(r)
        r -= mp.mpf(c2)
        c3 = float(r)
        r -= mp.mpf(c3)
        c4 = float(r)
        emit_const("EXP64_C1", c1, "ln2/256 rounded to 34 bits")
        emit_const("EXP64_C2", c2)
        emit_const("EXP64_C3", c3)
        emit_const("EXP64_C4", c4)
        emit_const("EXP64_INV", d(256 / ln2), "256/ln2")
        emit_td_table("INV_FACT_TD", [1 / mp.factorial(k) for k in range(8)],
                      "1/k! as triple-double, k = 0..7")
        emit_td_table("LN2_TD", [ln2], "ln 2 as triple-double")
        iv = log_intervals()
        emit_td_table("LOG64_L", [-mp.log(c) for _, _, c in iv], "-ln(c_j) as triple-double")
        emit_td_table("INV_ODD_TD", [mp.mpf(1) / (2 * k + 1) for k in range(8)],
                      "1/(2k+1) as triple-double, k = 0..7")
        h, l = dd(mp.mpf(1) / 3)
        emit_const("THIRD_HI", h)
        emit_const("THIRD_LO", l)
    # fast exp: e^r - 1 - r = r^2 P(r), |r| <= rho
    rho = mp.log(2) / 512 * mp.mpf("1.0001")
    for deg in range(3, 8):
        cs = lawson_fit(lambda r: (mp.expm1(r) - r) / (r * r) if r != 0 else mp.mpf(0.5),
                        lambda r: r * r, -rho, rho, list(range(deg + 1)), npts=120, iters=16)
        cd = [d(v) for v in cs]
        err = max_err(lambda r: mp.expm1(r) - r - r * r * sum(mp.mpf(cd[k]) * r ** k
                                                              for k in range(len(cd))), -rho, rho)
        if err < mp.mpf(2) ** -80:
            break
    emit("// e^r - 1 = r + r^2 P(r), |r| <= ln2/512; |error| <= 2^%.2f (absolute, proven)"
         % log2_of(B.sup_bound(B.expm1_minus_r([mp.mpf(v) for v in cd], rho))))
    emit_arr("EXP64_P", cd, "coefficients (degree %d)" % (len(cd) - 1))
    emit("#define EXP64_P_DEG %d" % (len(cd) - 1))
    # fast log: log1p(t) = t - t^2/2 + t^3/3 + t^4 S(t), t in [-1/32, 1/16]
    iv = log_intervals()
    a = min(lo * c - 1 for lo, hi, c in iv) * mp.mpf("1.0001")
    b = max(hi * c - 1 for lo, hi, c in iv) * mp.mpf("1.0001")
    g = lambda t: (mp.log1p(t) - t + t * t / 2 - t ** 3 / 3) / t ** 4 if t != 0 else mp.mpf(-1) / 4
    for deg in range(9, 18):
        cs = lawson_fit(g, lambda t: t ** 4, a, b, list(range(deg + 1)), npts=160, iters=14)
        cd = [d(v) for v in cs]
        err = max_err(lambda t: mp.log1p(t) - t + t * t / 2 - t ** 3 / 3
                      - t ** 4 * sum(mp.mpf(cd[k]) * t ** k for k in range(len(cd))), a, b)
        if err < mp.mpf(2) ** -78:
            break
    Sm = [mp.mpf(v) for v in cd]
    emit("// log1p t = t - t^2/2 + t^3/3 + t^4 S(t), t in [%s, %s]; |error| <= 2^%.2f (absolute), "
         "|S - (log1p t - t + t^2/2 - t^3/3)/t^4| <= 2^%.2f (both proven)"
         % (mp.nstr(a, 6), mp.nstr(b, 6), log2_of(B.sup_bound(B.log64_absolute(Sm, a, b))),
            log2_of(B.sup_bound(B.log64_quotient(Sm, a, b)))))
    emit_arr("LOG64_S", cd, "coefficients (degree %d)" % (len(cd) - 1))
    emit("#define LOG64_S_DEG %d" % (len(cd) - 1))
    emit("#define ATANH64_N 16")
    emit_dd_table("INV_ODD_DD", [mp.mpf(1) / (2 * k + 1) for k in range(17)], "1/(2k+1), k = 0..16")
    emit()
    gen_exp2_64()
    gen_log128()


def gen_log128():
    """binary64 log with the paper's 128-entry scaled-integer table (Sec. II-B):
    rcp_j = the binary32 value with encoding (0x3F2B + j) << 16 (8 significant
    bits, 0.66796875 .. 1.328125), r_j = rcp_j - 1 (exact) and the entry
    T_j = log1p(r_j)/r_j - 1 stored as the 64-bit integer nearest to T_j 2^65."""
    emit("// ---- binary64 log, 128-entry scaled-integer table ----")
    vals = []
    with mp.workprec(400):
        for j in range(128):
            enc = (0x3F2B + j) << 16
            sign, ex, man = enc >> 31, (enc >> 23) & 0xFF, enc & 0x7FFFFF
            rcp = (1 + mp.mpf(man) / 2 ** 23) * mp.mpf(2) ** (ex - 127)
            r = rcp - 1
            T = mp.mpf(0) if r == 0 else mp.log1p(r) / r - 1
            vals.append(int(mp.nint(T * mp.mpf(2) ** 65)))
    assert all(abs(v) < 2 ** 63 for v in vals)
    emit("// T_j = log1p(r_j)/r_j - 1 scaled by 2^65 (r_j = rcp_j - 1, rcp_j = binary32 with "
         "encoding (0x3F2B + j) << 16)")
    emit("__device__ __constant__ const long long LOG128_T[128] = {")
    for i in range(0, 128, 4):
        emit("  " + " ".join("%dll," % v for v in vals[i:i + 4]))
    emit("};")
    # log1p t = t - t^2/2 + t^3/3 + t^4 S(t), |t| <= 2^-8 (1 + 2^-12)
    rho = mp.mpf(2) ** -8 * (1 + mp.mpf(2) ** -12)
    g = lambda t: (mp.log1p(t) - t + t * t / 2 - t ** 3 / 3) / t ** 4 if t != 0 else mp.mpf(-1) / 4
    for deg in range(1, 8):
        cs = lawson_fit(g, lambda t: t ** 4, -rho, rho, list(range(deg + 1)), npts=100, iters=12)
        cd = [d(v) for v in cs]
        err = max_err(lambda t: mp.log1p(t) - t + t * t / 2 - t ** 3 / 3
                      - t ** 4 * sum(mp.mpf(cd[k]) * t ** k for k in range(len(cd))), -rho, rho)
        if err < mp.mpf(2) ** -88:
            break
    Sm = [mp.mpf(v) for v in cd]
    emit("// log1p t = t - t^2/2 + t^3/3 + t^4 S(t), |t| <= 2^-8 (1 + 2^-12); |error| <= 2^%.2f "
         "(absolute, proven)" % log2_of(B.sup_bound(B.log64_absolute(Sm, -rho, rho))))
    emit_arr("LOG128_S", cd, "coefficients (degree %d)" % (len(cd) - 1))
    emit("#define LOG128_S_DEG %d" % (len(cd) - 1))
    emit()


def gen_exp2_64():
    """binary64 exp2 (paper, Sec. II-B): 2^x = 2^m T1[i1] T2[i2] T3[i3] 2^R with
    x = (4096 m + 256 i1 + 16 i2 + i3)/4096 + R, |R| <= 2^-13, and three
    16-entry tables: the main path reads each entry as a double-double
    (hi, mid); the third word serves the accurate path."""
    emit("// ---- binary64 exp2 ----")
    with mp.workprec(600):
        for name, den in (("EXP2_64_T1", 16), ("EXP2_64_T2", 256), ("EXP2_64_T3", 4096)):
            emit_td_table(name, [mp.power(2, mp.mpf(i) / den) for i in range(16)],
                          "2^(i/%d) as triple-double {hi, mid, lo, 0}" % den)
    # e^r - 1 - r = r^2 P(r) on |r| <= ln2 / 8192 (r = R ln2)
    rho = mp.log(2) / 8192 * mp.mpf("1.0001")
    for deg in range(1, 6):
        cs = lawson_fit(lambda r: (mp.expm1(r) - r) / (r * r) if r != 0 else mp.mpf(0.5),
                        lambda r: r * r, -rho, rho, list(range(deg + 1)), npts=80, iters=12)
        cd = [d(v) for v in cs]
        err = max_err(lambda r: mp.expm1(r) - r - r * r * sum(mp.mpf(cd[k]) * r ** k
                                                              for k in range(len(cd))), -rho, rho)
        if err < mp.mpf(2) ** -88:
            break
    emit("// e^r - 1 = r + r^2 P(r), |r| <= ln2/8192; |error| <= 2^%.2f (absolute, proven)"
         % log2_of(B.sup_bound(B.expm1_minus_r([mp.mpf(v) for v in cd], rho))))
    emit_arr("EXP2_64_P", cd, "coefficients (degree %d)" % (len(cd) - 1))
    emit("#define EXP2_64_P_DEG %d" % (len(cd) - 1))
    emit()


def main():
    emit("// Generated by paper_2605_15547_amd/gen/gen_consts.py -- do not edit.")
    emit("// Tables and polynomial coefficients of the correctly rounded kernels.")
    emit("#pragma once")
    emit("#include <hip/hip_runtime.h>")
    emit()
    gen_exp()
    gen_log()
    gen_trig()
    gen_atan()
    gen_f64()
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
