"""Pins of the CPU oracle to things other than itself (no GPU needed).

Each test checks the oracle against what the mathematics or the paper fixes:
closed forms and exact results, IEEE special values, two independent
derivations of each constant, an exact integer decision for rsqrtf, symmetry
and monotonicity invariants, brute force against an independent
multiprecision library (mpmath) at 400 bits, and the paper's statements about
the accuracy each function needs.
"""
import json
import os
import zlib

import numpy as np
import pytest

mp = pytest.importorskip("mpmath")

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
F32 = ["expf", "exp2f", "exp10f", "expm1f", "logf", "log2f", "log10f", "log1pf", "rsqrtf",
       "sinf", "cosf", "tanf", "asinf", "acosf", "atanf", "sinhf", "coshf", "tanhf"]


def u32(a):
    return np.asarray(a, dtype=np.float32).view(np.uint32)


def u64(a):
    return np.asarray(a, dtype=np.float64).view(np.uint64)


# ------------------------------------------------------- mpmath reference
MPF = {"expf": mp.exp, "exp2f": lambda x: mp.power(2, x), "exp10f": lambda x: mp.power(10, x),
       "expm1f": mp.expm1, "logf": mp.log, "log2f": lambda x: mp.log(x, 2),
       "log10f": mp.log10, "log1pf": mp.log1p, "rsqrtf": lambda x: 1 / mp.sqrt(x),
       "sinf": mp.sin, "cosf": mp.cos, "tanf": mp.tan, "asinf": mp.asin, "acosf": mp.acos,
       "atanf": mp.atan, "sinhf": mp.sinh, "coshf": mp.cosh, "tanhf": mp.tanh,
       "exp": mp.exp, "log": mp.log, "exp2": lambda x: mp.power(2, x)}
F64 = ("exp", "log", "exp2")


def mp_round(v, P, emin, emax):
    """RN-even of an mpf into a binary format with P bits (independent code path)."""
    if v == 0:
        return 0.0
    s = -1 if v < 0 else 1
    a = abs(v)
    e = int(mp.floor(mp.log(a, 2)))
    while mp.ldexp(1, e) > a:
        e -= 1
    while mp.ldexp(1, e + 1) <= a:
        e += 1
    q = max(e, emin) - (P - 1)
    m = a / mp.ldexp(1, q)
    fl = int(mp.floor(m))
    fr = m - fl
    if fr > 0.5 or (fr == 0.5 and fl % 2 == 1):
        fl += 1
    if fl >= 2 ** P:
        fl //= 2
        q += 1
    if q + P - 1 > emax:
        return s * float("inf")
    return s * float(mp.ldexp(fl, q))


def mp_ref(func, x):
    mp.mp.prec = 400
    v = MPF[func](mp.mpf(float(x)))
    if func in F64:
        return mp_round(v, 53, -1022, 1023)
    return np.float32(mp_round(v, 24, -126, 127))


def sample(func, n, seed):
    rng = np.random.default_rng(seed)
    if func in ("logf", "log2f", "log10f", "rsqrtf"):
        b = rng.integers(0x00000001, 0x7F800000, n, dtype=np.uint64).astype(np.uint32)
        return b.view(np.float32)
    if func == "log1pf":
        return np.concatenate([(rng.random(n // 2) * 3 - 0.999).astype(np.float32),
                               rng.integers(1, 0x7F000000, n - n // 2, dtype=np.uint64)
                               .astype(np.uint32).view(np.float32)])
    if func in ("asinf", "acosf"):
        return (rng.random(n) * 2 - 1).astype(np.float32)
    if func in ("sinf", "cosf", "tanf", "atanf"):
        sign = rng.integers(0, 2, n, dtype=np.uint64).astype(np.uint32) << 31
        b = sign | rng.integers(0x00000001, 0x7F800000, n, dtype=np.uint64).astype(np.uint32)
        return b.view(np.float32)
    if func in ("sinhf", "coshf"):
        return (rng.random(n) * 190 - 95).astype(np.float32)
    if func == "tanhf":
        return (rng.random(n) * 24 - 12).astype(np.float32)
    if func == "exp2f":
        return (rng.random(n) * 290 - 155).astype(np.float32)
    if func == "exp10f":
        return (rng.random(n) * 90 - 47).astype(np.float32)
    if func == "exp":
        return rng.random(n) * (712 + 750) - 750
    if func == "log":
        return np.ldexp(1 + rng.random(n), rng.integers(-1074, 1024, n))
    if func == "exp2":
        # half over the whole range (overflow and the subnormal results included),
        # half on [-20, 20], where the paper measures binary64 exp2
        return np.concatenate([rng.random(n - n // 2) * (1030 + 1080) - 1080,
                               rng.random(n // 2) * 40 - 20])
    return (rng.random(n) * 220 - 110).astype(np.float32)


@pytest.mark.parametrize("func", F32 + list(F64))
def test_brute_force_vs_mpmath(oracle, func):
    """Random inputs across the whole domain: oracle == mpmath (400 bits)."""
    x = sample(func, 160, 11 + (zlib.crc32(func.encode()) % 1000))
    got = oracle.evaluate(func, x)
    for xi, gi in zip(x, got):
        ref = mp_ref(func, xi)
        if func in F64:
            assert u64(gi) == u64(ref), (func, float(xi), gi, ref)
        else:
            assert u32(gi) == u32(ref), (func, float(xi), gi, ref)


@pytest.mark.parametrize("func", F32 + list(F64))
def test_hard_set_vs_mpmath(oracle, func):
    """The hardest inputs found by the exhaustive scan: oracle == mpmath."""
    path = os.path.join(GOLD, "hard", func + (".u64" if func in F64 else ".u32"))
    if not os.path.exists(path):
        pytest.skip("hard set not generated")
    dt = (np.uint64, np.float64) if func in F64 else (np.uint32, np.float32)
    x = np.fromfile(path, dtype=dt[0]).view(dt[1])[:24]
    got = oracle.evaluate(func, x)
    for xi, gi in zip(x, got):
        assert np.asarray(gi).view(dt[0]) == np.asarray(mp_ref(func, xi), dtype=dt[1]).view(dt[0])


def test_sincosf_is_sin_and_cos(oracle):
    x = sample("sinf", 2000, 5)
    sc = oracle.evaluate("sincosf", x)
    assert np.array_equal(u32(sc[0]), u32(oracle.evaluate("sinf", x)))
    assert np.array_equal(u32(sc[1]), u32(oracle.evaluate("cosf", x)))


# ---------------------------------------------------------- exact results
def test_exact_powers(oracle):
    k = np.arange(-149, 128)
    x = k.astype(np.float32)
    assert np.array_equal(u32(oracle.evaluate("exp2f", x)), u32(np.ldexp(np.float32(1), k)))
    assert np.array_equal(u32(oracle.evaluate("log2f", np.ldexp(np.float32(1), k))),
                          u32(x))
    # exp2f(-150) = 2^-150 is exactly the midpoint between 0 and 2^-149: ties to even
    assert u32(oracle.evaluate("exp2f", np.float32([-150.0])))[0] == 0
    # just above -150 rounds up to the smallest subnormal, just below rounds to 0
    x = np.array([np.nextafter(np.float32(-150), np.float32(0)),
                  np.nextafter(np.float32(-150), np.float32(-200))], dtype=np.float32)
    assert list(u32(oracle.evaluate("exp2f", x))) == [1, 0]
    p10 = np.array([10.0 ** i for i in range(11)], dtype=np.float32)  # exact up to 10^10
    assert np.array_equal(u32(oracle.evaluate("exp10f", np.arange(11, dtype=np.float32))),
                          u32(p10))
    assert np.array_equal(u32(oracle.evaluate("log10f", p10)),
                          u32(np.arange(11, dtype=np.float32)))
    k = np.arange(-74, 64)
    assert np.array_equal(u32(oracle.evaluate("rsqrtf", np.ldexp(np.float32(1), 2 * k))),
                          u32(np.ldexp(np.float32(1), -k)))


def rn53_root(num, n):
    """RN to 53 bits of num^(1/n) for an integer num in [1, 2^n), decided with
    exact integer comparisons (the root is irrational for the num used, so no
    tie can occur): M in [2^52, 2^53) with M^n <= num 2^(52 n) < (M+1)^n, then
    up when the midpoint (2M+1)/2 lies below the root."""
    t = num << (52 * n)
    lo, hi = 1 << 52, 1 << 53
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if mid ** n <= t:
            lo = mid
        else:
            hi = mid
    M = lo
    if (2 * M + 1) ** n < (num << (53 * n)):
        M += 1
    return M


def test_exact_powers_binary64(oracle):
    """binary64 exp2 (paper, Sec. II-B): exp2(k) = 2^k for every integer k with
    a representable result, the one exact midpoint exp2(-1075) = +0 (ties to
    even) and its neighbours, overflow at 1024, and exp2(k + 1/2),
    exp2(k + 1/4), exp2(k + 3/4) against 2^k times the correctly rounded
    roots of 2, 2 and 8, decided in integer arithmetic."""
    k = np.arange(-1074, 1024)
    got = u64(oracle.evaluate("exp2", k.astype(np.float64)))
    assert np.array_equal(got, u64(np.ldexp(1.0, k)))
    x = np.array([-1075.0, np.nextafter(-1075.0, 0), np.nextafter(-1075.0, -2000), 1024.0,
                  np.nextafter(1024.0, 0), -1e300, 1e300], dtype=np.float64)
    r = oracle.evaluate("exp2", x)
    assert u64(r[:3]).tolist() == [0, 1, 0]
    assert np.isinf(r[3]) and np.isfinite(r[4]) and r[4] > 1.7e308
    assert u64(r[5:]).tolist() == [0, 0x7FF0000000000000]
    for frac, num, n in ((0.5, 2, 2), (0.25, 2, 4), (0.75, 8, 4)):
        M = rn53_root(num, n)
        k = np.arange(-1022, 1023)
        got = oracle.evaluate("exp2", k + frac)
        assert np.array_equal(u64(got), u64(np.ldexp(float(M) * 2.0 ** -52, k))), frac
    sp = np.array([0.0, -0.0, np.inf, -np.inf], dtype=np.float64)
    assert u64(oracle.evaluate("exp2", sp)).tolist() == [u64(1.0)] * 2 + [0x7FF0000000000000, 0]
    nans = np.array([0x7FF8000000000000, 0xFFF8000000000000, 0x7FF0000000000001],
                    dtype=np.uint64)
    assert u64(oracle.evaluate("exp2", nans.view(np.float64))).tolist() == \
        (nans | np.uint64(0x0008000000000000)).tolist()


def test_exp2_binary64_monotone(oracle):
    rng = np.random.default_rng(17)
    x = np.sort(np.concatenate([rng.uniform(-1080, 1030, 4000), rng.uniform(-20, 20, 4000)]))
    y = oracle.evaluate("exp2", x)
    assert np.all(y[1:] >= y[:-1])


def test_exact_scalars(oracle):
    one32, zero32 = u32(np.float32(1)), u32(np.float32(0))
    for f in ("expf", "exp2f", "exp10f", "coshf", "cosf"):
        assert u32(oracle.evaluate(f, np.float32([0.0, -0.0]))).tolist() == [one32] * 2
    for f in ("logf", "log2f", "log10f", "acosf"):
        assert u32(oracle.evaluate(f, np.float32([1.0])))[0] == zero32
    assert u64(oracle.evaluate("exp", np.array([0.0, -0.0]))).tolist() == [u64(1.0)] * 2
    assert u64(oracle.evaluate("log", np.array([1.0])))[0] == 0


def test_special_values(oracle):
    inf, nan = np.float32(np.inf), np.float32(np.nan)
    QN = 0x7FC00000
    cases = {  # func: [(input, expected bits)]
        "expf": [(inf, 0x7F800000), (-inf, 0), (np.float32(100), 0x7F800000)],
        "expm1f": [(inf, 0x7F800000), (-inf, 0xBF800000), (np.float32(-0.0), 0x80000000)],
        "logf": [(np.float32(0), 0xFF800000), (np.float32(-0.0), 0xFF800000),
                 (np.float32(-1), QN), (-inf, QN), (inf, 0x7F800000)],
        "log1pf": [(np.float32(-1), 0xFF800000), (np.float32(-2), QN), (inf, 0x7F800000),
                   (np.float32(-0.0), 0x80000000)],
        "rsqrtf": [(np.float32(0), 0x7F800000), (np.float32(-0.0), 0xFF800000),
                   (np.float32(-4), QN), (inf, 0)],
        "sinf": [(inf, QN), (-inf, QN), (np.float32(-0.0), 0x80000000)],
        "cosf": [(inf, QN), (np.float32(-0.0), 0x3F800000)],
        "tanf": [(-inf, QN), (np.float32(-0.0), 0x80000000)],
        "asinf": [(np.float32(1.5), QN), (np.float32(-0.0), 0x80000000)],
        "acosf": [(np.float32(-1.5), QN), (np.float32(1.0), 0)],
        "atanf": [(np.float32(-0.0), 0x80000000)],
        "sinhf": [(-inf, 0xFF800000), (np.float32(-0.0), 0x80000000)],
        "coshf": [(-inf, 0x7F800000)],
        "tanhf": [(-inf, 0xBF800000), (inf, 0x3F800000), (np.float32(-0.0), 0x80000000)],
    }
    for f, lst in cases.items():
        x = np.array([c[0] for c in lst], dtype=np.float32)
        assert u32(oracle.evaluate(f, x)).tolist() == [c[1] for c in lst], f
    # NaN inputs come back quieted with sign and payload kept
    nans = np.array([0x7FC00000, 0xFFC00000, 0x7F800001, 0x7FC12345], dtype=np.uint32)
    for f in F32:
        got = u32(oracle.evaluate(f, nans.view(np.float32)))
        assert got.tolist() == (nans | 0x00400000).tolist(), f
    got = u64(oracle.evaluate("log", np.array([-1.0, 0.0, np.inf])))
    assert got.tolist() == [0x7FF8000000000000, 0xFFF0000000000000, 0x7FF0000000000000]
    # atan(+-inf) = +-RN(pi/2)
    pi2 = np.float32(mp_round(mp.pi / 2, 24, -126, 127))
    assert u32(oracle.evaluate("atanf", np.float32([inf, -inf]))).tolist() == \
        [int(u32(pi2)), int(u32(-pi2))]


# --------------------------------------------------------------- constants
def test_constants_two_ways(oracle):
    """pi by Machin and by Euler, ln2 by atanh(1/3) and by sum 1/(k 2^k): each
    pair agrees to 2048 bits within the computed radii, and agrees with
    mpmath's constants."""
    nb = 2048
    mp.mp.prec = nb + 64
    for a, b, ref in ((2, 3, mp.pi), (0, 1, mp.log(2))):
        ha, ra = oracle.constant(a, nb)
        hb, rb = oracle.constant(b, nb)
        va, vb = int(ha, 16), int(hb, 16)
        assert abs(va - vb) <= ra + rb + 2
        assert abs(va - int(mp.floor(ref * mp.mpf(2) ** nb))) <= ra + 2
    h10, r10 = oracle.constant(4, nb)
    assert abs(int(h10, 16) - int(mp.floor(mp.log(10) * mp.mpf(2) ** nb))) <= r10 + 2


# -------------------------------------------------------- exact decision
def test_rsqrtf_exact_integer_decision(oracle):
    """rsqrtf by the Ziv loop == rsqrtf decided with exact integer comparisons
    of m^2 x against 1 at the neighbouring midpoints (no approximation)."""
    rng = np.random.default_rng(3)
    b = rng.integers(1, 0x7F800000, 1 << 15, dtype=np.uint64).astype(np.uint32)
    x = np.concatenate([b.view(np.float32),
                        np.fromfile(os.path.join(GOLD, "hard", "rsqrtf.u32"), dtype="<u4")
                        .view(np.float32) if os.path.exists(os.path.join(GOLD, "hard",
                                                                         "rsqrtf.u32"))
                        else np.zeros(0, np.float32)])
    assert np.array_equal(u32(oracle.evaluate("rsqrtf", x)), u32(oracle.rsqrtf_exact(x)))


# ---------------------------------------------------------------- invariants
@pytest.mark.parametrize("func,lo,hi,sign", [
    ("expf", -104, 89, 1), ("exp2f", -150, 128, 1), ("exp10f", -46, 39, 1),
    ("expm1f", -20, 89, 1), ("logf", 1e-38, 3e38, 1), ("log2f", 1e-38, 3e38, 1),
    ("log10f", 1e-38, 3e38, 1), ("log1pf", -0.999, 1e30, 1), ("atanf", -1e6, 1e6, 1),
    ("asinf", -1, 1, 1), ("sinhf", -90, 90, 1), ("tanhf", -10, 10, 1), ("acosf", -1, 1, -1),
    ("rsqrtf", 1e-40, 3e38, -1), ("coshf", 0, 90, 1)])
def test_monotone(oracle, func, lo, hi, sign):
    rng = np.random.default_rng(7)
    if lo > 0:
        x = np.exp(rng.uniform(np.log(lo), np.log(hi), 6000)).astype(np.float32)
    else:
        x = rng.uniform(lo, hi, 6000).astype(np.float32)
    x = np.sort(x)
    y = oracle.evaluate(func, x).astype(np.float64)
    ok = (y[1:] >= y[:-1]) if sign > 0 else (y[1:] <= y[:-1])
    assert np.all(ok), func


@pytest.mark.parametrize("func,parity", [("sinf", -1), ("tanf", -1), ("asinf", -1),
                                         ("atanf", -1), ("sinhf", -1), ("tanhf", -1),
                                         ("cosf", 1), ("coshf", 1)])
def test_symmetry(oracle, func, parity):
    x = np.abs(sample(func, 3000, 9))
    if func in ("sinhf", "coshf"):
        x = np.abs(x)
    a = oracle.evaluate(func, x)
    b = oracle.evaluate(func, -x)
    if parity < 0:
        assert np.array_equal(u32(b), u32(-a))
    else:
        assert np.array_equal(u32(b), u32(a))


def test_trig_bounds(oracle):
    x = sample("sinf", 4000, 13)
    s, c = oracle.evaluate("sincosf", x)
    assert np.all(np.abs(s) <= 1) and np.all(np.abs(c) <= 1)
    assert np.all(np.abs(oracle.evaluate("tanhf", sample("tanhf", 2000, 1))) <= 1)


# ------------------------------------------------------------- hardness
def test_hardness_closed_form(oracle):
    """exp(x) for x = 2^-53: 1 + x is the midpoint between 1 and 1 + 2^-52 and
    exp(x) - (1 + x) = x^2/2 (1 + x/3 + ...), i.e. 2^-55 ulp: h = 55."""
    h = oracle.hardness("exp", np.array([2.0 ** -53]))[0]
    assert abs(h - 55.0) < 1e-6
    # exp(3 * 2^-53): distance 9 x 2^-55 ulp -> h = 55 - log2(9)
    h = oracle.hardness("exp", np.array([3 * 2.0 ** -53]))[0]
    assert abs(h - (55.0 - np.log2(9.0))) < 1e-6
    # an exactly representable result is as far as possible from a midpoint
    assert oracle.hardness("exp2f", np.float32([3.0]))[0] == 1.0


def test_paper_accuracy_statements():
    """Paper, Sec. II-A: most binary32 functions need slightly more than double
    precision to round correctly, while log2f needs less.  The exhaustive scan
    measures h_max, so the precision needed is 24 + 1 + h_max bits."""
    path = os.path.join(GOLD, "hard", "index.json")
    if not os.path.exists(path):
        pytest.skip("hard sets not generated")
    idx = json.load(open(path))
    need = {f: 25 + idx[f]["max_h"] for f in F32 if f in idx}
    assert need["log2f"] < 53
    assert sum(1 for f, v in need.items() if v > 53) > len(need) / 2
