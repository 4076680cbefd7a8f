"""ctypes wrapper around the CPU oracle (oracle/libcr_oracle.so).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark.  The GPU library never imports it.

The oracle returns RN_even(f(x)) for binary32 functions (ids 0..18) and
binary64 exp/log/exp2 (ids 64, 65, 66), or f(x) rounded in a directed mode
(toward zero, +infinity or -infinity), computed by a Ziv loop over a
from-scratch fixed-point ball arithmetic (see cr_oracle.c for the method and
citations).
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcr_oracle.so")

FUNCS32 = ["expf", "exp2f", "exp10f", "expm1f", "logf", "log2f", "log10f", "log1pf",
           "rsqrtf", "sinf", "cosf", "sincosf", "tanf", "asinf", "acosf", "atanf",
           "sinhf", "coshf", "tanhf"]
FUNC_ID = {name: i for i, name in enumerate(FUNCS32)}
FUNC_ID["exp"] = 64
FUNC_ID["log"] = 65
FUNC_ID["exp2"] = 66


def build(force=False):
    """Compile the oracle with gcc (plain C, no GPU)."""
    src = os.path.join(HERE, "cr_oracle.c")
    if not force and os.path.exists(LIB_PATH) and \
            os.path.getmtime(LIB_PATH) >= os.path.getmtime(src):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-pthread",
                           src, "-o", tmp, "-lquadmath", "-lm"])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.cr_oracle_eval.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_size_t, ctypes.c_int]
        L.cr_oracle_hardness.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_size_t, ctypes.c_int]
        L.cr_oracle_eval_mode.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        L.cr_oracle_scan_f32.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]
        L.cr_oracle_scan_f32.restype = ctypes.c_int64
        L.cr_oracle_scan_f64.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]
        L.cr_oracle_scan_f64.restype = ctypes.c_int64
        L.cr_oracle_rsqrtf_exact.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]
        L.cr_oracle_constant.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_char_p,
                                         ctypes.c_size_t]
        L.cr_oracle_constant.restype = ctypes.c_double
        _lib = L
    return _lib


def default_threads():
    return max(1, min(16, os.cpu_count() or 1))


def _fid(func):
    return FUNC_ID[func] if isinstance(func, str) else int(func)


def in_dtype(func):
    return np.float64 if _fid(func) >= 64 else np.float32


# IEEE 754 rounding modes (Sec. 4.3) of evaluate(): to nearest (ties to
# even), toward zero, toward +infinity, toward -infinity
MODES = {"rn": 0, "rz": 1, "ru": 2, "rd": 3}


def evaluate(func, x, nthreads=None, mode="rn"):
    """Correctly rounded f(x) for a numpy array x (float32 or float64), in the
    rounding mode `mode` (a key of MODES).  sincosf returns an array of shape
    (2, n): (sin, cos)."""
    fid = _fid(func)
    x = np.ascontiguousarray(x, dtype=in_dtype(fid))
    n = x.size
    out = np.empty(2 * n if fid == FUNC_ID["sincosf"] else n, dtype=x.dtype)
    if mode == "rn":
        st = lib().cr_oracle_eval(fid, x.ctypes.data, out.ctypes.data, n,
                                  nthreads or default_threads())
    else:
        st = lib().cr_oracle_eval_mode(fid, MODES[mode], x.ctypes.data, out.ctypes.data, n,
                                       nthreads or default_threads())
    if st != 0:
        raise RuntimeError("cr_oracle_eval(%s, %s) returned %d" % (func, mode, st))
    return out.reshape(2, n) if fid == FUNC_ID["sincosf"] else out


def hardness(func, x, nthreads=None):
    fid = _fid(func)
    x = np.ascontiguousarray(x, dtype=in_dtype(fid))
    h = np.empty(x.size, dtype=np.float64)
    st = lib().cr_oracle_hardness(fid, x.ctypes.data, h.ctypes.data, x.size,
                                  nthreads or default_threads())
    if st != 0:
        raise RuntimeError("cr_oracle_hardness(%s) returned %d" % (func, st))
    return h


def scan_f32(func, lo, hi, h_prefilter, h_keep, max_out=1 << 20, nthreads=None):
    bits = np.empty(max_out, dtype=np.uint32)
    hs = np.empty(max_out, dtype=np.float64)
    cnt = lib().cr_oracle_scan_f32(_fid(func), lo, hi, h_prefilter, h_keep, bits.ctypes.data,
                                   hs.ctypes.data, max_out, nthreads or default_threads())
    if cnt < 0:
        raise RuntimeError("scan failed")
    k = min(cnt, max_out)
    return bits[:k].copy(), hs[:k].copy(), cnt


def scan_f64(func, x, h_prefilter, h_keep, max_out=1 << 20, nthreads=None):
    x = np.ascontiguousarray(x, dtype=np.float64)
    ox = np.empty(max_out, dtype=np.float64)
    oh = np.empty(max_out, dtype=np.float64)
    cnt = lib().cr_oracle_scan_f64(_fid(func), x.ctypes.data, x.size, h_prefilter, h_keep,
                                   ox.ctypes.data, oh.ctypes.data, max_out,
                                   nthreads or default_threads())
    if cnt < 0:
        raise RuntimeError("scan failed")
    k = min(cnt, max_out)
    return ox[:k].copy(), oh[:k].copy(), cnt


def rsqrtf_exact(x):
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty_like(x)
    lib().cr_oracle_rsqrtf_exact(x.ctypes.data, out.ctypes.data, x.size)
    return out


def constant(which, nbits):
    """(hex digits of floor(c 2^nbits), radius bound in units of 2^-nbits)"""
    buf = ctypes.create_string_buffer(nbits // 4 + 64)
    rad = lib().cr_oracle_constant(which, nbits, buf, len(buf))
    if rad < 0:
        raise ValueError("bad constant request")
    return buf.value.decode(), rad
