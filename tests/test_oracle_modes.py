"""Pins of the oracle's directed rounding modes (IEEE 754-2019 Sec. 4.3:
toward zero, toward +infinity, toward -infinity), which the paper's CPU
library supports and its GPU runs leave out (paper, Sec. II-A, III-C).
No GPU needed.

* An independent rounding: mpmath at 400 bits, the float neighbours of the
  exact value found by comparing exact rationals, on random inputs over each
  domain and on the hard-to-round sets.
* Invariants: RD <= RN <= RU with RU and RD equal (exact) or adjacent; RZ is
  RD for positive results and RU for negative ones; RN is one of RD, RU.
* Exact results in every mode: exp2f(k), exp10f(k), log2f(2^k), log10f(10^k),
  rsqrtf(4^k), binary64 exp2(k).
* Saturation and underflow: overflow gives the largest finite number toward
  zero, tiny positive results round up to the smallest subnormal, tanh and
  expm1 stop one ulp short of +-1 toward zero.
* Tiny arguments: sin x just below x, tan x just above, and so on.
"""
import os
import sys

import numpy as np
import pytest

mp = pytest.importorskip("mpmath")

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
from test_oracle_pins import F32, MPF, sample  # noqa: E402

MODES = ("rz", "ru", "rd")
FMAX = np.float32(3.4028234663852886e38)


def bits32(a):
    return np.asarray(a, dtype=np.float32).view(np.uint32)


def neighbours32(v):
    """(RD, RU) of the exact mpf v in binary32 (gradual underflow, overflow to
    +-FLT_MAX / +-inf), by exact comparisons."""
    if v == 0:
        return np.float32(0.0), np.float32(0.0)
    if v > mp.mpf(float(FMAX)):
        return FMAX, np.float32(np.inf)
    if v < -mp.mpf(float(FMAX)):
        return np.float32(-np.inf), -FMAX
    c = np.float32(float(v))  # near v; corrected below
    if np.isinf(c):
        c = FMAX if v > 0 else -FMAX
    while mp.mpf(float(c)) > v:
        c = np.nextafter(c, np.float32(-np.inf))
    while mp.mpf(float(np.nextafter(c, np.float32(np.inf)))) <= v:
        c = np.nextafter(c, np.float32(np.inf))
    lo = c
    hi = lo if mp.mpf(float(lo)) == v else np.nextafter(lo, np.float32(np.inf))
    # zero results keep the sign of the value
    if lo == 0 and v < 0:
        lo = np.float32(-0.0)
    if hi == 0 and v < 0:
        hi = np.float32(-0.0)
    return lo, hi


def mp_mode(func, x, mode):
    mp.mp.prec = 400
    v = MPF[func](mp.mpf(float(x)))
    lo, hi = neighbours32(v)
    if mode == "rd":
        return lo
    if mode == "ru":
        return hi
    return lo if v >= 0 else hi


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("func", F32)
def test_directed_modes_against_mpmath(oracle, func, mode):
    """Random inputs over the domain and the 16 hardest-to-round inputs."""
    x = sample(func, 120, seed=9000 + F32.index(func))
    x = x[np.isfinite(MPF_ok(func, x))]
    hard = oracle_hard(func)
    if hard is not None:
        x = np.concatenate([x, hard[:16]])
    got = oracle.evaluate(func, x, mode=mode)
    for xi, gi in zip(x, got):
        want = mp_mode(func, xi, mode)
        assert bits32(gi) == bits32(want), (func, mode, float(xi), float(gi), float(want))


def MPF_ok(func, x):
    """Mask out inputs outside the real domain (NaN results)."""
    x = np.asarray(x, dtype=np.float64)
    if func in ("logf", "log2f", "log10f", "rsqrtf"):
        return np.where(x > 0, x, np.nan)
    if func == "log1pf":
        return np.where(x > -1, x, np.nan)
    if func in ("asinf", "acosf"):
        return np.where(np.abs(x) <= 1, x, np.nan)
    if func in ("sinf", "cosf", "tanf"):
        return np.where(np.abs(x) < 1e10, x, np.nan)  # mpmath's own reduction stays cheap
    return x


def oracle_hard(func):
    from paper_2605_15547_amd import inputs
    return inputs.hard_set(func)


@pytest.mark.parametrize("func", F32 + ["sincosf"])
def test_mode_invariants(oracle, func):
    """RD <= RN <= RU, RU - RD in {0, 1 ulp}, RZ by the sign of the result."""
    base = "sinf" if func == "sincosf" else func
    x = np.concatenate([sample(base, 4000, seed=9100 + len(func)),
                        np.array([0.0, -0.0, np.inf, -np.inf, 1.0, -1.0, 1e-40, -1e-40,
                                  3e38, -3e38], np.float32)]).astype(np.float32)
    rn = oracle.evaluate(func, x).ravel()
    rz, ru, rd = (oracle.evaluate(func, x, mode=m).ravel() for m in ("rz", "ru", "rd"))
    nan = np.isnan(rn)
    assert np.array_equal(np.isnan(ru), nan) and np.array_equal(np.isnan(rd), nan)
    ok = ~nan
    rn, rz, ru, rd = rn[ok], rz[ok], ru[ok], rd[ok]
    assert np.all(rd <= rn) and np.all(rn <= ru)
    exact = ru == rd
    step = np.nextafter(rd, np.float32(np.inf))
    assert np.all(exact | (ru == step) | (np.isinf(ru) & (rd == FMAX)))
    assert np.all((rn == rd) | (rn == ru))
    pos = (rd > 0) | ((rd == 0) & (ru > 0)) | ((rd == 0) & (ru == 0) & ~np.signbit(rd))
    assert np.all(np.where(pos, rz == rd, rz == ru) | ((rz == 0) & (rd == 0) & (ru == 0)))


def test_exact_results_in_every_mode(oracle):
    k = np.arange(-149, 128, dtype=np.float32)
    for m in ("rn",) + MODES:
        assert np.array_equal(oracle.evaluate("exp2f", k, mode=m), np.ldexp(1.0, k.astype(int))
                              .astype(np.float32))
        p2 = np.ldexp(np.float32(1), np.arange(-149, 128)).astype(np.float32)
        assert np.array_equal(oracle.evaluate("log2f", p2, mode=m),
                              np.arange(-149, 128).astype(np.float32))
        t = np.arange(1, 11, dtype=np.float32)
        assert np.array_equal(oracle.evaluate("exp10f", t, mode=m),
                              np.array([10.0 ** i for i in range(1, 11)], np.float32))
        assert np.array_equal(oracle.evaluate("log10f", np.array([10.0 ** i for i in range(1, 11)],
                                                                 np.float32), mode=m), t)
        q = np.ldexp(np.float32(1), np.arange(-148, 128, 2)).astype(np.float32)
        assert np.array_equal(oracle.evaluate("rsqrtf", q, mode=m),
                              np.ldexp(np.float32(1), -np.arange(-148, 128, 2) // 2)
                              .astype(np.float32))
        kk = np.arange(-1074, 1024, dtype=np.float64)
        assert np.array_equal(oracle.evaluate("exp2", kk, mode=m), np.ldexp(1.0, kk.astype(int)))


def _one(oracle, func, x, mode):
    return oracle.evaluate(func, np.array([x], np.float32), mode=mode)[0]


def test_saturation_and_underflow(oracle):
    one_m = np.nextafter(np.float32(1), np.float32(0))
    tiny = np.float32(2.0 ** -149)
    cases = [
        ("expf", 100.0, {"rz": FMAX, "ru": np.inf, "rd": FMAX}),
        ("expf", -200.0, {"rz": 0.0, "ru": tiny, "rd": 0.0}),
        ("exp2f", -150.0, {"rz": 0.0, "ru": tiny, "rd": 0.0}),
        ("exp2f", 128.0, {"rz": FMAX, "ru": np.inf, "rd": FMAX}),
        ("expm1f", -50.0, {"rz": -one_m, "ru": -one_m, "rd": -1.0}),
        ("tanhf", 60.0, {"rz": one_m, "ru": 1.0, "rd": one_m}),
        ("tanhf", -60.0, {"rz": -one_m, "ru": -one_m, "rd": -1.0}),
        ("tanhf", np.inf, {"rz": 1.0, "ru": 1.0, "rd": 1.0}),
        ("sinhf", 100.0, {"rz": FMAX, "ru": np.inf, "rd": FMAX}),
        ("sinhf", -100.0, {"rz": -FMAX, "ru": -FMAX, "rd": -np.inf}),
        ("coshf", -100.0, {"rz": FMAX, "ru": np.inf, "rd": FMAX}),
        ("sinhf", np.inf, {"rz": np.inf, "ru": np.inf, "rd": np.inf}),
    ]
    for func, x, want in cases:
        for m, w in want.items():
            got = _one(oracle, func, x, m)
            assert bits32(got) == bits32(np.float32(w)), (func, x, m, got, w)


def test_tiny_arguments(oracle):
    """For tiny x the exact value lies strictly between x (or 1) and the next
    float on the side of the correction term."""
    a = np.float32(2.0 ** -100)
    dn = np.nextafter(a, np.float32(0))
    up_ = np.nextafter(a, np.float32(1))
    one_m = np.nextafter(np.float32(1), np.float32(0))
    one_p = np.nextafter(np.float32(1), np.float32(2))
    cases = [
        ("sinf", a, {"rz": dn, "ru": a, "rd": dn}),       # x - x^3/6
        ("sinf", -a, {"rz": -dn, "ru": -dn, "rd": -a}),
        ("tanf", a, {"rz": a, "ru": up_, "rd": a}),       # x + x^3/3
        ("atanf", a, {"rz": dn, "ru": a, "rd": dn}),
        ("asinf", -a, {"rz": -a, "ru": -a, "rd": -up_}),
        ("sinhf", a, {"rz": a, "ru": up_, "rd": a}),
        ("tanhf", a, {"rz": dn, "ru": a, "rd": dn}),
        ("expm1f", -a, {"rz": -dn, "ru": -dn, "rd": -a}),  # x + x^2/2
        ("log1pf", a, {"rz": dn, "ru": a, "rd": dn}),     # x - x^2/2
        ("cosf", a, {"rz": one_m, "ru": 1.0, "rd": one_m}),
        ("coshf", a, {"rz": 1.0, "ru": one_p, "rd": 1.0}),
        ("expf", -a, {"rz": one_m, "ru": 1.0, "rd": one_m}),
        ("exp10f", a, {"rz": 1.0, "ru": one_p, "rd": 1.0}),
    ]
    for func, x, want in cases:
        for m, w in want.items():
            got = _one(oracle, func, x, m)
            assert bits32(got) == bits32(np.float32(w)), (func, x, m, got, w)
