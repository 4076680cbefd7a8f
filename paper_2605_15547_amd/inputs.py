"""Seeded synthetic input generators, shared by the tests and the benchmark.

This module holds no arithmetic of the functions themselves: it only draws
input encodings.  Random numbers come from SplitMix64 (Steele, Lea, Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014) in its
counter form z_i = mix(seed + (i+1) * 0x9E3779B97F4A7C15), vectorised with
numpy so both sides of every comparison see identical arrays.

Workload recipes (paper, Sec. III; the paper prints no input distribution for
its GPU tables, so these are synthetic stand-ins of the shapes it names):
  * expf correctness set: 64 special/edge encodings, then 2^20 values uniform
    in [-103.9, 88.7] (the full range where expf is neither 0 nor Inf).
  * exp/log family: per function 90% uniform over the finite domain, 5% raw
    32-bit patterns (NaN/Inf/subnormal/negative), 5% drawn from the
    function's hard-to-round set, categories mixed at random positions.
  * trig/hyperbolic family: random sign and exponent field uniform in
    [97, 254] (|x| in 2^-30 .. 2^127) for sin/cos/sincos/tan/atan; uniform
    in the domain for the others.
  * binary64 exp/log/exp2: exp uniform in [-745, 709.7]; log = ldexp(1+f, E)
    with E uniform in [-1074, 1023]; exp2 uniform in [-20, 20]; 1e-4 of the
    elements from the hard set.
  * ragged batch: 4096 requests, function uniform over the 19 binary32
    functions, length floor(2^(20 u)) capped at 2^20.
"""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "tests", "golden")

FUNCS32 = ["expf", "exp2f", "exp10f", "expm1f", "logf", "log2f", "log10f", "log1pf",
           "rsqrtf", "sinf", "cosf", "sincosf", "tanf", "asinf", "acosf", "atanf",
           "sinhf", "coshf", "tanhf"]
FUNC_ID = {name: i for i, name in enumerate(FUNCS32)}
FUNC_ID["exp"] = 64
FUNC_ID["log"] = 65
FUNC_ID["exp2"] = 66
F64_FUNCS = ("exp", "log", "exp2")
EXPLOG_FAMILY = FUNCS32[:9]
TRIG_FAMILY = FUNCS32[9:]

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, n, offset=0):
    """n outputs of SplitMix64 started at `seed`, counter form (uint64)."""
    with np.errstate(over="ignore"):
        i = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


class Stream:
    """A seeded stream of SplitMix64 words consumed in blocks."""

    def __init__(self, seed):
        self.seed = seed
        self.pos = 0

    def u64(self, n):
        z = splitmix64(self.seed, n, self.pos)
        self.pos += n
        return z

    def uniform(self, n):
        """doubles uniform in [0, 1) with 53 random bits"""
        return (self.u64(n) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53

    def u32(self, n):
        return (self.u64(n) >> np.uint64(32)).astype(np.uint32)

    def below(self, n, m):
        """integers uniform in [0, m) (m < 2^32, negligible bias)"""
        return ((self.u64(n) >> np.uint64(32)) * np.uint64(m) >> np.uint64(32)).astype(np.int64)


def f32_bits(bits):
    return np.asarray(bits, dtype=np.uint32).view(np.float32)


def uniform_f32(st, n, a, b):
    """RN_f32(a + (b - a) u), u uniform in [0,1)"""
    return (a + (b - a) * st.uniform(n)).astype(np.float32)


def encoding_uniform_f32(st, n, lo_bits, hi_bits):
    """float32 values with encodings uniform in [lo_bits, hi_bits]"""
    span = hi_bits - lo_bits + 1
    return f32_bits(np.uint32(lo_bits) + st.below(n, span).astype(np.uint32))


# ---------------------------------------------------------------- hard sets
def hard_set(func):
    """The function's hard-to-round inputs found by the oracle's exhaustive scan
    (tests/golden/hard/<func>.u32, written by tests/golden/make_hard_sets.py)."""
    path = os.path.join(GOLDEN, "hard", func + (".u64" if func in F64_FUNCS else ".u32"))
    if not os.path.exists(path):
        # the workloads' hard-input share depends on it: fail rather than
        # silently generating a different workload
        raise FileNotFoundError("hard set of %s missing: %s" % (func, path))
    dt = np.uint64 if func in F64_FUNCS else np.uint32
    a = np.fromfile(path, dtype=dt)
    return a.view(np.float64 if func in F64_FUNCS else np.float32)


def edge_inputs_expf():
    """The 64 special and edge encodings that open the expf correctness set
    (tests/golden/expf_edges.json, written by tests/golden/make_edges.py)."""
    with open(os.path.join(GOLDEN, "expf_edges.json")) as f:
        d = json.load(f)
    return f32_bits(np.array([int(b, 16) for b in d["bits"]], dtype=np.uint32))


# ------------------------------------------------------------ domain draws
def domain_f32(func, st, n):
    """Inputs uniform over the function's finite domain (see module doc)."""
    if func in ("expf", "expm1f"):
        return uniform_f32(st, n, -103.9, 88.7)
    if func == "exp2f":
        return uniform_f32(st, n, -150.0, 128.0)
    if func == "exp10f":
        return uniform_f32(st, n, -45.15, 38.53)
    if func in ("logf", "log2f", "log10f", "rsqrtf"):
        return encoding_uniform_f32(st, n, 0x00800000, 0x7F7FFFFF)
    if func == "log1pf":
        # normals in (-1, FLT_MAX]: positive normal encodings plus negative
        # normal encodings above -1, uniform over the union
        npos = 0x7F7FFFFF - 0x00800000 + 1
        nneg = 0xBF7FFFFF - 0x80800000 + 1
        k = st.below(n, npos + nneg).astype(np.uint64)
        bits = np.where(k < npos, np.uint64(0x00800000) + k,
                        np.uint64(0x80800000) + (k - np.uint64(npos)))
        return f32_bits(bits.astype(np.uint32))
    if func in ("sinf", "cosf", "sincosf", "tanf", "atanf"):
        sign = st.u32(n) & np.uint32(0x80000000)
        expo = (np.uint32(97) + st.below(n, 254 - 97 + 1).astype(np.uint32)) << np.uint32(23)
        mant = st.u32(n) & np.uint32(0x007FFFFF)
        return f32_bits(sign | expo | mant)
    if func in ("asinf", "acosf"):
        return uniform_f32(st, n, -1.0, 1.0)
    if func in ("sinhf", "coshf"):
        return uniform_f32(st, n, -89.4, 89.4)
    if func == "tanhf":
        return uniform_f32(st, n, -10.0, 10.0)
    raise ValueError(func)


def explog_family(func, n, seed=None):
    """Exp/log family workload: 90% domain, 5% raw bits, 5% hard set."""
    st = Stream(2000 + FUNC_ID[func] if seed is None else seed)
    cat = st.below(n, 100)
    x = domain_f32(func, st, n)
    raw = f32_bits(st.u32(n))
    x = np.where((cat >= 90) & (cat < 95), raw, x)
    hs = hard_set(func)
    if hs.size:
        pick = hs[st.below(n, hs.size)]
        x = np.where(cat >= 95, pick, x)
    return np.ascontiguousarray(x, dtype=np.float32)


def trig_family(func, n, seed=None):
    st = Stream(3000 + FUNC_ID[func] if seed is None else seed)
    return np.ascontiguousarray(domain_f32(func, st, n), dtype=np.float32)


def workload_f32(func, n, seed=None):
    """The binary32 workload of `func` (exp/log family or trig/hyperbolic)."""
    if func in EXPLOG_FAMILY:
        return explog_family(func, n, seed)
    return trig_family(func, n, seed)


def expf_correctness_set(n_uniform=1 << 20):
    """64 specials and edges, then n_uniform values uniform in [-103.9, 88.7]."""
    st = Stream(0)
    return np.concatenate([edge_inputs_expf(), uniform_f32(st, n_uniform, -103.9, 88.7)])


def workload_f64(func, n, seed=None):
    """binary64 exp/log/exp2 workload with 1e-4 of the elements from the hard
    set.  exp2: uniform in [-20, 20], the range of the paper's binary64 exp2
    measurements (Sec. III, Table IV)."""
    st = Stream(4000 + FUNC_ID[func] if seed is None else seed)
    if func == "exp":
        x = -745.0 + (709.7 + 745.0) * st.uniform(n)
    elif func == "exp2":
        x = -20.0 + 40.0 * st.uniform(n)
    elif func == "log":
        E = -1074 + st.below(n, 1023 + 1074 + 1)
        f = (st.u64(n) >> np.uint64(12)).astype(np.float64) * 2.0 ** -52
        x = np.ldexp(1.0 + f, E)
    else:
        raise ValueError(func)
    hs = hard_set(func)
    k = max(1, int(round(n * 1e-4))) if n >= 1000 else 0
    if hs.size and k:
        pos = st.below(k, n)
        x[pos] = hs[st.below(k, hs.size)]
    return np.ascontiguousarray(x, dtype=np.float64)


def batch_requests(num=4096, seed=5000, max_log2=20):
    """(func names, lengths, per-request seeds) of the ragged batch workload."""
    st = Stream(seed)
    funcs = [FUNCS32[i] for i in st.below(num, len(FUNCS32))]
    u = st.uniform(num)
    lens = np.minimum(2 ** max_log2, np.floor(2.0 ** (max_log2 * u))).astype(np.int64)
    seeds = (st.u64(num) >> np.uint64(1)).astype(np.int64)
    return funcs, lens, seeds


# ------------------------------------------------------- application workloads
COMPLEX_FUNCS = ("cexpf", "clogf", "csinf")


def complex_workload(n, seed=6000, lo=-40.0, hi=40.0):
    """n binary32 complex numbers, interleaved (re, im), both parts uniform in
    [lo, hi] (the paper's range for its complex expf/logf/sinf runs is
    [-40, 40], Sec. III-A)."""
    st = Stream(seed)
    return uniform_f32(st, 2 * n, lo, hi)


def dft_workload(n_samples, n_freqs, seed=7000):
    """Spectral interpolation inputs: n_samples binary32 time samples uniform
    in [-1, 1], and one binary32 per-sample angle w_k = RN32(2 pi f_k / N)
    per output frequency, f_k uniform in [0, N/2) in bins (non-integer, so
    between the bins an FFT would compute)."""
    st = Stream(seed)
    x = uniform_f32(st, n_samples, -1.0, 1.0)
    f = st.uniform(n_freqs) * (n_samples / 2.0)
    w = (2.0 * np.pi * f / n_samples).astype(np.float32)
    return x, w
