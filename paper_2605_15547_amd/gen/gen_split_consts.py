"""Generates paper_2605_15547_amd/csrc/cr_split_consts.h: the tables and
constants of the binary32-only ("split", float-float) kernels.

Every value is computed with mpmath at high precision and rounded directly to
binary32 (never through binary64, which would round twice); a float-float
entry is the pair hi = RN32(v), lo = RN32(v - hi).  Run:
    python paper_2605_15547_amd/gen/gen_split_consts.py
"""
import os

import mpmath as mp

mp.mp.prec = 300
HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(os.path.dirname(HERE), "csrc", "cr_split_consts.h")


def f32(x, mode="n"):
    """x rounded to binary32 (normal range): mode n = nearest-even, z = toward 0"""
    x = mp.mpf(x)
    if x == 0:
        return 0.0
    e = int(mp.floor(mp.log(abs(x), 2)))
    q = mp.mpf(2) ** (e - 23)
    while abs(x) / q >= 2 ** 24:
        q *= 2
    while abs(x) / q < 2 ** 23:
        q /= 2
    t = x / q
    n = mp.nint(t) if mode == "n" else (mp.floor(t) if t > 0 else mp.ceil(t))
    if mode == "n" and abs(t - mp.floor(t) - mp.mpf(0.5)) == 0:  # tie: even
        n = mp.floor(t) if int(mp.floor(t)) % 2 == 0 else mp.ceil(t)
    v = n * q
    return float(v)  # exact: v has 24 bits


def bits(x, nb, mode="z"):
    """x rounded to nb significant bits (toward zero by default)"""
    x = mp.mpf(x)
    e = int(mp.floor(mp.log(abs(x), 2)))
    q = mp.mpf(2) ** (e - nb + 1)
    t = x / q
    n = (mp.floor(t) if t > 0 else mp.ceil(t)) if mode == "z" else mp.nint(t)
    return float(n * q)


def ff(x):
    x = mp.mpf(x)
    hi = f32(x)
    lo = f32(x - mp.mpf(hi)) if x != mp.mpf(hi) else 0.0
    return hi, lo


def tf(x):
    """x as a triple-float h + m + l, each part the binary32 rounding of what
    the previous parts leave (about 72 significant bits)"""
    x = mp.mpf(x)
    h = f32(x)
    r = x - mp.mpf(h)
    m = f32(r) if r != 0 else 0.0
    r -= mp.mpf(m)
    l = f32(r) if r != 0 else 0.0
    return h, m, l


def fx(v):
    v = float(v)
    if v == 0.0:
        return "0.0f"
    return v.hex() + "f"


lines = []


def emit(s=""):
    lines.append(s)


def emit_ff_table(name, vals, comment):
    emit("// " + comment)
    emit("__device__ __constant__ const float2 %s[%d] = {" % (name, len(vals)))
    for v in vals:
        hi, lo = ff(v)
        emit("  {%s, %s}," % (fx(hi), fx(lo)))
    emit("};")


def emit_tf_table(name, vals, comment):
    emit("// " + comment + ", triple-float {h, m, l, 0}")
    emit("__device__ __constant__ const float4 %s[%d] = {" % (name, len(vals)))
    for v in vals:
        h, m, l = tf(v)
        emit("  {%s, %s, %s, 0.0f}," % (fx(h), fx(m), fx(l)))
    emit("};")


def emit_tf(name, v, comment=""):
    h, m, l = tf(v)
    emit_f(name + "_H", h, comment)
    emit_f(name + "_M", m)
    emit_f(name + "_L", l)


def emit_f(name, v, comment=""):
    emit("#define %s (%s)%s" % (name, fx(v), ("  /* " + comment + " */") if comment else ""))


def gen_exp():
    emit("// ---- exponential family, binary32-only ----")
    emit_ff_table("SEXP_T1", [mp.power(2, mp.mpf(j) / 16) for j in range(-8, 8)],
                  "2^(j/16), j = -8..7 (index j + 8), float-float")
    emit_ff_table("SEXP_T2", [mp.power(2, mp.mpf(j) / 256) for j in range(-8, 8)],
                  "2^(j/256), j = -8..7 (index j + 8), float-float")
    emit_ff_table("SEXP_D1", [mp.power(2, mp.mpf(j) / 16) - 1 for j in range(-8, 8)],
                  "2^(j/16) - 1, j = -8..7, float-float")
    emit_ff_table("SEXP_D2", [mp.power(2, mp.mpf(j) / 256) - 1 for j in range(-8, 8)],
                  "2^(j/256) - 1, j = -8..7, float-float")
    ln2 = mp.log(2)
    C = ln2 / 256
    c1 = bits(C, 8, "z")  # rounded toward zero: k c1 exact and x - k c1 exact
    assert mp.mpf(c1) <= C * (1 - mp.mpf(2) ** -20)
    c2 = f32(C - c1)
    c3 = f32(C - c1 - c2)
    emit_f("SEXP_INV_LN2_256", f32(256 / ln2), "256/ln2")
    emit_f("SEXP_C1", c1, "ln2/256 truncated to 8 bits")
    emit_f("SEXP_C2", c2, "next 24 bits of ln2/256")
    emit_f("SEXP_C3", c3, "next 24 bits of ln2/256")
    h, l = ff(ln2 / 256)
    emit_f("SEXP_LN2_256_H", h, "ln2/256 hi")
    emit_f("SEXP_LN2_256_L", l, "ln2/256 lo")
    L = 256 * mp.log(10, 2)
    a = f32(L)
    b = f32(L - a)
    c = f32(L - a - b)
    emit_f("SEXP_L10_H", a, "256 log2(10), three parts")
    emit_f("SEXP_L10_M", b)
    emit_f("SEXP_L10_L", c)
    emit_f("SEXP_INV6", f32(mp.mpf(1) / 6), "1/6")
    emit_f("SEXP_INV24", f32(mp.mpf(1) / 24), "1/24")
    emit()


def gen_log():
    emit("// ---- logarithm family, binary32-only ----")
    # first level: 16 intervals of the mantissa fold m in [0.75, 1.5)
    c1s = []
    for j in range(16):
        if j < 8:
            lo, hi = 1 + mp.mpf(j) / 16, 1 + mp.mpf(j + 1) / 16
        else:
            lo, hi = (1 + mp.mpf(j) / 16) / 2, (1 + mp.mpf(j + 1) / 16) / 2
        c = 1.0 if j in (0, 15) else bits(2 / (lo + hi), 9, "n")
        c1s.append(c)
        SLOG_C1S.append(c)
        t_lo, t_hi = lo * c - 1, hi * c - 1
        assert -0.0313 <= t_lo and t_hi <= 0.0626, (j, t_lo, t_hi)
    c2s = [1.0 if i == 0 else bits(1 / (1 + mp.mpf(i) / SLOG_S), 12, "n") for i in range(-8, 8)]
    SLOG_C2S.extend(c2s)
    emit("// first level: c1 ~ 1/m, 9 bits (1 for the two intervals next to 1)")
    emit("__device__ __constant__ const float SLOG_C1[16] = {%s};" % ", ".join(fx(c) for c in c1s))
    emit("// second level: c2 ~ 1/(1 + i/%d), i = -8..7, 12 bits" % SLOG_S)
    emit("__device__ __constant__ const float SLOG_C2[16] = {%s};" % ", ".join(fx(c) for c in c2s))
    emit_ff_table("SLOG_L1", [-mp.log(c) for c in c1s], "-log(c1), float-float")
    emit_ff_table("SLOG_L2", [-mp.log(c) for c in c2s], "-log(c2), float-float")
    emit_f("SLOG_S", SLOG_S, "second-level index scale")
    ln2 = mp.log(2)
    for name, v in (("SLOG_LN2", ln2), ("SLOG_LG2", mp.log(2, 10))):
        a = bits(v, 16, "n")
        b = f32(v - a)
        c = f32(v - a - b)
        emit_f(name + "_H", a, "16 bits (e times it is exact)")
        emit_f(name + "_M", b)
        emit_f(name + "_L", c)
    for name, v in (("SLOG_INV_LN2", 1 / ln2), ("SLOG_INV_LN10", 1 / mp.log(10)),
                    ("SLOG_THIRD", mp.mpf(1) / 3)):
        h, l = ff(v)
        emit_f(name + "_H", h)
        emit_f(name + "_L", l)
    for k in range(4, 8):
        emit_f("SLOG_P%d" % k, f32(mp.mpf((-1) ** (k + 1)) / k), "(-1)^(k+1)/k")
    emit()


def gen_trig():
    emit("// ---- trigonometric family, binary32-only ----")
    emit("// sin(j pi/32), cos(j pi/32), j = 0..15: {sin hi, sin lo, cos hi, cos lo}")
    emit("__device__ __constant__ const float4 STRIG_T[16] = {")
    for j in range(16):
        a = mp.pi * j / 32
        sh, sl = ff(mp.sin(a))
        ch, cl = ff(mp.cos(a))
        emit("  {%s, %s, %s, %s}," % (fx(sh), fx(sl), fx(ch), fx(cl)))
    emit("};")
    h, l = ff(mp.pi / 32)
    emit_f("STRIG_PI32_H", h, "pi/32 hi")
    emit_f("STRIG_PI32_L", l, "pi/32 lo")
    emit_f("STRIG_PI64", f32(mp.pi / 64, "z"), "pi/64 rounded down")
    for name, v in (("STRIG_S3", -mp.mpf(1) / 6), ("STRIG_C4", mp.mpf(1) / 24)):
        h, l = ff(v)
        emit_f(name + "_H", h)
        emit_f(name + "_L", l)
    emit_f("STRIG_S5", f32(mp.mpf(1) / 120), "1/5!")
    emit_f("STRIG_S7", f32(-mp.mpf(1) / 5040), "-1/7!")
    emit_f("STRIG_S9", f32(mp.mpf(1) / 362880), "1/9!")
    emit_f("STRIG_C6", f32(-mp.mpf(1) / 720), "-1/6!")
    emit_f("STRIG_C8", f32(mp.mpf(1) / 40320), "1/8!")
    emit()


def gen_atan():
    emit("// ---- inverse trigonometric family, binary32-only ----")
    emit("// {atan(j/16) hi, lo, (pi/2 - atan(j/16)) hi, lo}, j = 0..15")
    emit("__device__ __constant__ const float4 SATAN_T[16] = {")
    for j in range(16):
        a = mp.atan(mp.mpf(j) / 16)
        h, l = ff(a)
        h2, l2 = ff(mp.pi / 2 - a)
        emit("  {%s, %s, %s, %s}," % (fx(h), fx(l), fx(h2), fx(l2)))
    emit("};")
    for name, v in (("SATAN_PI", mp.pi), ("SATAN_THIRD", mp.mpf(1) / 3)):
        h, l = ff(v)
        emit_f(name + "_H", h)
        emit_f(name + "_L", l)
    for k in (5, 7, 9, 11, 13):
        emit_f("SATAN_P%d" % k, f32(mp.mpf((-1) ** ((k - 1) // 2)) / k), "(-1)^((k-1)/2)/k")
    emit()


def gen_tf():
    """Tables and constants of the triple-float accurate step."""
    emit("// ---- triple-float accurate step ----")
    emit_tf_table("TFEXP_T1", [mp.power(2, mp.mpf(j) / 16) for j in range(-8, 8)],
                  "2^(j/16), j = -8..7 (index j + 8)")
    emit_tf_table("TFEXP_T2", [mp.power(2, mp.mpf(j) / 256) for j in range(-8, 8)],
                  "2^(j/256), j = -8..7")
    emit_tf_table("TFEXP_D1", [mp.power(2, mp.mpf(j) / 16) - 1 for j in range(-8, 8)],
                  "2^(j/16) - 1, j = -8..7")
    emit_tf_table("TFEXP_D2", [mp.power(2, mp.mpf(j) / 256) - 1 for j in range(-8, 8)],
                  "2^(j/256) - 1, j = -8..7")
    ln2 = mp.log(2)
    C = ln2 / 256
    c1 = bits(C, 8, "z")
    c2 = f32(C - c1)
    c3 = f32(C - c1 - c2)
    c4 = f32(C - c1 - c2 - c3)
    emit_f("TFEXP_C4", c4, "fourth part of ln2/256 (after the three of the fast path)")
    emit_tf("TFEXP_LN2_256", C, "ln2/256")
    L = 256 * mp.log(10, 2)
    a = f32(L)
    b = f32(L - a)
    c = f32(L - a - b)
    d = f32(L - a - b - c)
    emit_f("TFEXP_L10_LL", d, "fourth part of 256 log2(10)")
    for k in range(3, 8):
        emit_f("TF_INVFACT%d" % k, f32(1 / mp.factorial(k)), "1/%d!" % k)
    emit_tf("TF_SIXTH", mp.mpf(1) / 6, "1/6")
    emit_tf("TF_THIRD", mp.mpf(1) / 3, "1/3")
    h, l = ff(mp.mpf(1) / 120)
    emit_f("TF_INV120_H", h, "1/120 hi")
    emit_f("TF_INV120_L", l, "1/120 lo")
    h, l = ff(mp.mpf(1) / 24)
    emit_f("TF_INV24_H", h, "1/24 hi")
    emit_f("TF_INV24_L", l, "1/24 lo")
    h, l = ff(mp.mpf(1) / 5)
    emit_f("TF_FIFTH_H", h, "1/5 hi")
    emit_f("TF_FIFTH_L", l, "1/5 lo")
    for k in range(5, 10):
        emit_f("TF_RECIP%d" % k, f32(mp.mpf(1) / k), "1/%d" % k)
    # log: -log c1, -log c2 of the split reduction, ln 2 and log10(2) in four
    # parts (the first 16 bits wide: e times it is exact)
    c1s, c2s = SLOG_C1S, SLOG_C2S
    emit_tf_table("TFLOG_L1", [-mp.log(c) for c in c1s], "-log(c1)")
    emit_tf_table("TFLOG_L2", [-mp.log(c) for c in c2s], "-log(c2)")
    for name, v in (("TFLOG_LN2", ln2), ("TFLOG_LG2", mp.log(2, 10))):
        a = bits(v, 16, "n")
        b = f32(v - a)
        c = f32(v - a - b)
        d = f32(v - a - b - c)
        emit_f(name + "_H", a, "16 bits (e times it is exact)")
        emit_f(name + "_M", b)
        emit_f(name + "_L", c)
        emit_f(name + "_LL", d)
    emit_tf("TFLOG_INV_LN2", 1 / ln2, "1/ln2")
    emit_tf("TFLOG_INV_LN10", 1 / mp.log(10), "1/ln10")
    # trig
    emit_tf_table("TFTRIG_S", [mp.sin(mp.pi * j / 32) for j in range(16)], "sin(j pi/32), j = 0..15")
    emit_tf_table("TFTRIG_C", [mp.cos(mp.pi * j / 32) for j in range(16)], "cos(j pi/32), j = 0..15")
    emit_tf("TFTRIG_PI32", mp.pi / 32, "pi/32")
    for k in (7, 9, 11, 13):
        emit_f("TFTRIG_S%d" % k, f32(mp.mpf((-1) ** ((k - 1) // 2)) / mp.factorial(k)),
               "(-1)^((k-1)/2)/%d!" % k)
    for k in (6, 8, 10, 12):
        emit_f("TFTRIG_C%d" % k, f32(mp.mpf((-1) ** (k // 2)) / mp.factorial(k)),
               "(-1)^(k/2)/%d!" % k)
    # inverse trig
    emit_tf_table("TFATAN_A", [mp.atan(mp.mpf(j) / 16) for j in range(16)], "atan(j/16)")
    emit_tf_table("TFATAN_B", [mp.pi / 2 - mp.atan(mp.mpf(j) / 16) for j in range(16)],
                  "pi/2 - atan(j/16)")
    emit_tf("TFATAN_PI", mp.pi, "pi")
    for k in (7, 9, 11, 13):
        emit_f("TFATAN_P%d" % k, f32(mp.mpf((-1) ** ((k - 1) // 2)) / k), "(-1)^((k-1)/2)/%d" % k)
    emit()


SLOG_S = 112
SLOG_C1S = []
SLOG_C2S = []


def main():
    emit("// Generated by paper_2605_15547_amd/gen/gen_split_consts.py -- do not edit.")
    emit("// Tables and constants of the binary32-only (float-float) kernels.")
    emit("#pragma once")
    emit("#include <hip/hip_runtime.h>")
    emit()
    gen_exp()
    gen_log()
    gen_trig()
    gen_atan()
    gen_tf()
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
