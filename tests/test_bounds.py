"""Proven approximation-error bounds of every polynomial a fast-path rounding
test relies on (CPU).

The coefficients are read back from the generated header the kernels
compile (paper_2605_15547_amd/csrc/cr_consts.h), and a rigorous upper bound
of the approximation error is derived for each by Taylor's theorem with the
Lagrange remainder on subintervals (paper_2605_15547_amd/gen/bounds.py).  Each
bound must lie below the figure the kernel's error budget uses (stated in the
kernel sources next to the rounding test) and below the bound printed in the
header.  (Paper, Sec. II-B: the correct-rounding test on the main path is only
as good as the error bound it is given.)
"""
import os
import re

import mpmath as mp
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2605_15547_amd", "csrc", "cr_consts.h")

from paper_2605_15547_amd.gen import bounds as B  # noqa: E402


@pytest.fixture(scope="module")
def hdr():
    with open(HDR) as f:
        return f.read()


def arr(txt, name):
    m = re.search(r"\b%s\[\d+\] = \{([^}]*)\}" % re.escape(name), txt)
    assert m, name
    return [mp.mpf(float.fromhex(v.strip())) for v in m.group(1).split(",")]


def const(txt, name):
    m = re.search(r"#define %s \(([^)]*)\)" % re.escape(name), txt)
    assert m, name
    return mp.mpf(float.fromhex(m.group(1)))


def printed_bound(txt, marker):
    """The bound the header prints on the comment line containing marker."""
    for line in txt.splitlines():
        if marker in line and "2^-" in line:
            return float(re.findall(r"2\^(-[\d.]+)", line)[-1])
    raise AssertionError(marker)


def t_range(txt):
    c = arr(txt, "LOG_C")
    lo = [1 + mp.mpf(j) / 16 if j < 8 else (1 + mp.mpf(j) / 16) / 2 for j in range(16)]
    hi = [1 + mp.mpf(j + 1) / 16 if j < 8 else (1 + mp.mpf(j + 1) / 16) / 2 for j in range(16)]
    return min(l * cj - 1 for l, cj in zip(lo, c)), max(h * cj - 1 for h, cj in zip(hi, c))


def proven(spec):
    return B.log2b(B.sup_bound(spec))


# (kernel budget in log2, where the budget is stated)
def test_exp64_main_path_polynomial(hdr):
    """binary64 exp main path (cr_f64.h): P's approximation error <= 2^-83.9 on
    |r| <= ln2/512 (1 + 2^-13 for the rounding of k)."""
    rho = mp.log(2) / 512 * (1 + mp.mpf(2) ** -13)
    b = proven(B.expm1_minus_r(arr(hdr, "EXP64_P"), rho))
    assert b <= -83.9, b
    assert b <= printed_bound(hdr, "|r| <= ln2/512") + 0.01, b


def test_log64_main_path_polynomial(hdr):
    """binary64 log main path (cr_f64.h): sup |g - S| <= 2^-57 for the exact
    quotient g(t) = (log1p t - t + t^2/2 - t^3/3)/t^4, over the t of every
    table row; and the absolute error t^4 |g - S| against the header."""
    a, b = t_range(hdr)
    S = arr(hdr, "LOG64_S")
    q = proven(B.log64_quotient(S, a, b))
    assert q <= -57, q
    ab = proven(B.log64_absolute(S, a, b))
    assert ab <= printed_bound(hdr, "log1p t = t - t^2/2 + t^3/3 + t^4 S(t)") + 0.01, ab


def test_expm1_polynomial_binary32(hdr):
    """binary32 exp family fast path (cr_f32_exp.h): polynomial error
    <= 2^-64.8 on |r| <= 0.02167."""
    b = proven(B.expm1_minus_r(arr(hdr, "EXPM1_P"), mp.mpf("0.02167")))
    assert b <= -64.8, b
    assert mp.mpf(2) ** b <= const(hdr, "EXPM1_P_ERR")


@pytest.mark.parametrize("base", ["E", "2", "10"])
def test_log_polynomials_binary32(hdr, base):
    """binary32 log family fast path (cr_f32_log.h): Q's approximation error
    below 2^-57.6 over the t of every table row."""
    a, b = t_range(hdr)
    K = const(hdr, "LOG%s_K" % base)
    bnd = proven(B.log_b_quotient(arr(hdr, "LOG%s_Q" % base), base.lower(), K, a, b))
    assert bnd <= -57.6, bnd


def test_sin_cos_polynomials(hdr):
    """binary32 trig fast path (cr_f32_trig.h): on |r| <= pi/64 (1 + 2^-20) the
    degree-2 corrections are within 2^-57.6 (sin r) and 2^-50.1 (cos r - 1),
    the figures of the fast path's 2^-45 |y| + 2^-57 error budget."""
    rho = mp.pi / 64 * (1 + mp.mpf(2) ** -20)
    s = proven(B.sin_minus_r(arr(hdr, "SIN_S2"), rho))
    c = proven(B.cos_minus_1(arr(hdr, "COS_C2"), rho))
    assert s <= -57.6 and c <= -50.1, (s, c)


def test_atan_polynomial(hdr):
    """binary32 inverse-trig fast path (cr_f32_atan.h): P within 2^-66 on
    |t| <= 1/31."""
    b = proven(B.atan_minus_t(arr(hdr, "ATAN_P"), mp.mpf(1) / 31))
    assert b <= -66, b


def test_bound_method_is_tight_and_sound():
    """The method on a case with a known answer: the degree-2 Taylor
    polynomial of e^r - 1 - r on |r| <= 2^-4 (P = [1/2, 1/6]) has error
    sup = e^rho - 1 - rho - rho^2/2 - rho^3/6 at r = rho (all remaining terms
    positive there).  The bound must not be below it and within 2% above."""
    rho = mp.mpf(2) ** -4
    exact = mp.exp(rho) - 1 - rho - rho ** 2 / 2 - rho ** 3 / 6
    got = B.sup_bound(B.expm1_minus_r([mp.mpf(1) / 2, mp.mpf(1) / 6], rho), pieces=128)
    assert exact <= got <= exact * mp.mpf("1.02"), (exact, got)


def test_exp2_64_main_path_polynomial(hdr):
    """binary64 exp2 main path (cr_f64.h): r = R ln2 with |R| <= 2^-13 (exact),
    so |r| <= ln2/8192; the budget takes P's approximation error as 2^-91.95
    of an error total of 2^-78.5 (the rounding test allows 2^-77)."""
    rho = mp.log(2) / 8192 * (1 + mp.mpf(2) ** -40)
    b = proven(B.expm1_minus_r(arr(hdr, "EXP2_64_P"), rho))
    assert b <= -91.9, b
    assert b <= printed_bound(hdr, "|r| <= ln2/8192") + 0.01, b


def test_log128_main_path_polynomial(hdr):
    """binary64 log with the 128-entry table (cr_f64.h): |t| <= 2^-8 (1 + 2^-12);
    the budget takes t^4 S as within 2^-75 |t| (2^-83 absolute at the ends)."""
    rho = mp.mpf(2) ** -8 * (1 + mp.mpf(2) ** -12)
    S = arr(hdr, "LOG128_S")
    ab = proven(B.log64_absolute(S, -rho, rho))
    assert ab <= -83, ab
    assert ab <= printed_bound(hdr, "|t| <= 2^-8 (1 + 2^-12)") + 0.01, ab


def test_log128_table_entries(hdr):
    """The 128 scaled integers are log1p(r)/r - 1 for the reciprocals of 8
    significant bits, to within half a unit of 2^-65."""
    m = re.search(r"LOG128_T\[128\] = \{([^}]*)\}", hdr)
    vals = [int(v.strip().rstrip("l")) for v in m.group(1).replace("ll", "").split(",")
            if v.strip()]
    assert len(vals) == 128
    with mp.workprec(200):
        for j, v in enumerate(vals):
            enc = (0x3F2B + j) << 16
            rcp = (1 + mp.mpf(enc & 0x7FFFFF) / 2 ** 23) * mp.mpf(2) ** (((enc >> 23) & 0xFF) - 127)
            r = rcp - 1
            T = mp.mpf(0) if r == 0 else mp.log1p(r) / r - 1
            assert abs(T * mp.mpf(2) ** 65 - v) <= 0.5, j
    # rcp = 1 (j = 85) has T = 0
    assert abs(vals[85]) == 0  # rcp = 1
