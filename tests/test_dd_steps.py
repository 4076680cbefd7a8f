"""Error bounds of two double-double steps of the binary64 main paths,
checked on the CPU by replaying their operation sequences with exactly rounded
binary64 operations (each operation computed exactly as a fraction and rounded
to nearest once, fma included) on random operands:

* dd_mul_1p (binary64 exp and exp2): B (1 + q) for a double-double table
  entry B and |q| < 2^-9, within 2^-104 relative;
* the binary64 log main path's t^3/3 from t2 = t^2 (TwoProd plus the cross
  term) by two TwoProds and fmas, within 10 u^2 = 10 2^-106 relative.

The sequences are the ones in csrc/cr_f64.h, restated operation by operation.
"""
import random
from fractions import Fraction as F

import pytest

U = F(1, 2 ** 53)


def rn(x):
    """x rounded to the nearest binary64 (ties to even), as a Fraction"""
    return F(float(x))


def add(a, b):
    return rn(a + b)


def mul(a, b):
    return rn(a * b)


def fma(a, b, c):
    return rn(a * b + c)


def two_prod(a, b):
    p = mul(a, b)
    return p, fma(a, b, -p)


def fast_two_sum(a, b):
    s = add(a, b)
    return s, add(b, -add(s, -a))


def dd_of(x):
    """a real as a normalised double-double"""
    hi = rn(x)
    return hi, rn(x - hi)


def dd_mul_1p(B, q):
    p_hi, p_lo = two_prod(B[0], q[0])
    pl = fma(B[0], q[1], fma(B[1], q[0], p_lo))
    s_hi, s_lo = fast_two_sum(B[0], p_hi)
    return fast_two_sum(s_hi, add(s_lo, add(B[1], pl)))


def third_of_cube(t_hi, t_lo):
    t2_hi, t2_lo = two_prod(t_hi, t_hi)
    t2_lo = fma(2 * t_hi, t_lo, t2_lo)
    p3_hi, p3_lo = two_prod(t2_hi, t_hi)
    p3l = fma(t2_lo, t_hi, fma(t2_hi, t_lo, p3_lo))
    third_hi = F(float.fromhex("0x1.5555555555555p-2"))  # THIRD_HI, THIRD_LO of cr_consts.h
    third_lo = F(float.fromhex("0x1.5555555555555p-56"))
    b_hi, b_lo = two_prod(p3_hi, third_hi)
    b_lo = fma(p3l, third_hi, fma(p3_hi, third_lo, b_lo))
    return b_hi, b_lo


def rand_dd(rng, lo, hi):
    x = F(rng.uniform(lo, hi)) + F(rng.uniform(-1, 1)) * F(2) ** -60 * F(rng.uniform(lo, hi))
    return dd_of(x)


@pytest.mark.parametrize("seed", range(4))
def test_dd_mul_1p_within_2_to_minus_104(seed):
    rng = random.Random(1000 + seed)
    worst = F(0)
    for _ in range(1500):
        B = rand_dd(rng, 1.0, 2.0)  # a table entry 2^(j/256) or 2^(i/4096) lies in [1, 2)
        q = rand_dd(rng, -2 ** -9, 2 ** -9)
        exact = (B[0] + B[1]) * (1 + q[0] + q[1])
        hi, lo = dd_mul_1p(B, q)
        err = abs(hi + lo - exact) / exact
        worst = max(worst, err)
        assert abs(lo) <= abs(hi) * U  # normalised
    assert worst < F(2) ** -104, float(worst)


@pytest.mark.parametrize("seed", range(4))
def test_log64_third_of_cube_within_10u2(seed):
    rng = random.Random(2000 + seed)
    worst = F(0)
    for k in range(1500):
        if k % 2:
            # c_j = 1 rows: t exact in binary64 (t.lo = 0), |t| up to 1/16
            t = (rn(F(rng.uniform(-1 / 32, 1 / 16))), F(0))
        else:
            t = rand_dd(rng, -1 / 32, 1 / 16)
        if t[0] == 0:
            continue
        tt = t[0] + t[1]
        exact = tt ** 3 / 3
        hi, lo = third_of_cube(*t)
        worst = max(worst, abs(hi + lo - exact) / abs(exact))
    assert worst < 10 * U * U, float(worst / (U * U))
