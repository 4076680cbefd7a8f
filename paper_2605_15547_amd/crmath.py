"""Thin ctypes binding of libcr (include/cr.h): argument marshalling only.

Every step of the computation runs in the library's HIP kernels; PyTorch is
used only for device memory and streams.  Importing this module loads the
in-tree paper_2605_15547_amd/libcr.so and fails loudly if it is missing.
"""
import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libcr.so")

FUNCS32 = ["expf", "exp2f", "exp10f", "expm1f", "logf", "log2f", "log10f", "log1pf",
           "rsqrtf", "sinf", "cosf", "sincosf", "tanf", "asinf", "acosf", "atanf",
           "sinhf", "coshf", "tanhf"]
FUNC_ID = {name: i for i, name in enumerate(FUNCS32)}
FUNC_ID["exp"] = 64
FUNC_ID["log"] = 65
FUNC_ID["exp2"] = 66
FUNCS64 = ["exp", "log", "exp2"]
# complex binary32 functions (interleaved re, im pairs; n counts complex numbers)
FUNC_ID["cexpf"] = 80
FUNC_ID["clogf"] = 81
FUNC_ID["csinf"] = 82
COMPLEX = ["cexpf", "clogf", "csinf"]

IMPL_AUTO, IMPL_F64_INTERNAL, IMPL_SPLIT_F32, IMPL_LOG128 = 0, 1, 2, 3
FLAG_FORCE_FALLBACK = 1
# rounding modes (enum cr_flag): to nearest is the default
FLAG_ROUND_TOWARD_ZERO, FLAG_ROUND_UP, FLAG_ROUND_DOWN = 1 << 4, 2 << 4, 3 << 4
ROUND_FLAGS = {"rn": 0, "rz": FLAG_ROUND_TOWARD_ZERO, "ru": FLAG_ROUND_UP,
               "rd": FLAG_ROUND_DOWN}

CR_OK = 0
STATUS = {0: "CR_OK", -1: "CR_E_FUNC", -2: "CR_E_NULL", -3: "CR_E_OVERLAP", -4: "CR_E_ALIGN",
          -5: "CR_E_IMPL", -6: "CR_E_HIP", -7: "CR_E_NOMEM", -9: "CR_E_SIZE", -10: "CR_E_TUNE",
          -11: "CR_E_SCRATCH"}
NOALLOC_MAX_REQUESTS = 8192
NOALLOC_MAX_TILES = 1 << 19

EXPORTED = ["cr_eval", "cr_eval_ex", "cr_available", "cr_batch_plan_create",
            "cr_batch_plan_launch", "cr_batch_plan_destroy", "cr_eval_batch", "cr_eval_batch_noalloc",
            "cr_dft",
            "cr_stats_reset",
            "cr_stats_read", "cr_status_str", "cr_last_hip_error", "cr_tune_num_variants",
            "cr_tune_variant_info", "cr_tune_get", "cr_tune_set", "cr_tune_reset", "cr_tune_load",
            "cr_tune_save", "cr_autotune", "cr_tune_batch_get", "cr_tune_batch_set"]


class CrError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__("%s: %s (%d)" % (what, STATUS.get(status, "?"), status))


class Request(ctypes.Structure):
    """cr_request: one entry of a batch (device pointers as integers)."""
    _fields_ = [("func_id", ctypes.c_int32), ("impl", ctypes.c_int32),
                ("in_", ctypes.c_void_p), ("out", ctypes.c_void_p), ("n", ctypes.c_int64)]


class TuneCfg(ctypes.Structure):
    """cr_tune_cfg: a kernel variant and the grid in workgroups per compute unit."""
    _fields_ = [("variant", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("elems", ctypes.c_uint64), ("fallback_lanes", ctypes.c_uint64),
                ("fallback_waves", ctypes.c_uint64), ("escapes", ctypes.c_uint64),
                ("escape_index", ctypes.c_uint64 * 16)]


_lib = None


def lib():
    """Load libcr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libcr.so not built: run python -c 'import __graft_entry__ as g; "
                              "g.build()' (expected at %s)" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        L.cr_eval.argtypes = [ctypes.c_int, vp, vp, sz, vp]
        L.cr_eval.restype = ctypes.c_int
        L.cr_eval_ex.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint, vp, vp, sz, vp]
        L.cr_eval_ex.restype = ctypes.c_int
        L.cr_available.argtypes = [ctypes.c_int, ctypes.c_int]
        L.cr_available.restype = ctypes.c_int
        L.cr_dft.argtypes = [vp, ctypes.c_int64, vp, ctypes.c_int64, vp, ctypes.c_uint, vp]
        L.cr_dft.restype = ctypes.c_int
        L.cr_batch_plan_create.argtypes = [ctypes.POINTER(Request), ctypes.c_int32, ctypes.c_uint,
                                           ctypes.POINTER(ctypes.c_void_p)]
        L.cr_batch_plan_launch.argtypes = [vp, vp]
        L.cr_batch_plan_destroy.argtypes = [vp]
        L.cr_eval_batch.argtypes = [ctypes.POINTER(Request), ctypes.c_int32, vp]
        L.cr_eval_batch_noalloc.argtypes = [ctypes.POINTER(Request), ctypes.c_int32, vp]
        L.cr_stats_reset.argtypes = [vp]
        L.cr_stats_read.argtypes = [vp, ctypes.POINTER(Stats)]
        L.cr_status_str.argtypes = [ctypes.c_int]
        L.cr_status_str.restype = ctypes.c_char_p
        L.cr_last_hip_error.restype = ctypes.c_int
        ip = ctypes.POINTER(ctypes.c_int)
        L.cr_tune_num_variants.restype = ctypes.c_int
        L.cr_tune_variant_info.argtypes = [ctypes.c_int, ip, ip, ip]
        L.cr_tune_get.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(TuneCfg)]
        L.cr_tune_set.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(TuneCfg)]
        L.cr_tune_batch_get.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int32)]
        L.cr_tune_batch_set.argtypes = [ctypes.c_int, ctypes.c_int32]
        L.cr_tune_load.argtypes = [ctypes.c_char_p]
        L.cr_tune_save.argtypes = [ctypes.c_char_p]
        L.cr_autotune.argtypes = [ctypes.c_int, ctypes.c_int, vp, vp, sz, ctypes.c_int, vp,
                                  ctypes.POINTER(ctypes.c_double)]
        _lib = L
    return _lib


def _fid(func):
    return FUNC_ID[func] if isinstance(func, str) else int(func)


def available(func, impl=IMPL_AUTO):
    return bool(lib().cr_available(_fid(func), impl))


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def eval_ptr(func, in_ptr, out_ptr, n, impl=IMPL_AUTO, flags=0, stream_ptr=None):
    """Raw call: device pointers (ints), element count, HIP stream pointer."""
    rc = lib().cr_eval_ex(_fid(func), impl, flags, ctypes.c_void_p(in_ptr),
                          ctypes.c_void_p(out_ptr), n, stream_ptr)
    if rc != CR_OK:
        raise CrError(rc, "cr_eval_ex(%s)" % func)


def evaluate(func, x, out=None, impl=IMPL_AUTO, flags=0, stream=None):
    """Correctly rounded func(x) for a contiguous CUDA tensor x (float32 for the
    binary32 functions, float64 for exp/log/exp2; complex functions take
    interleaved (re, im) float32 pairs).  sincosf returns shape (2, n)."""
    import torch
    fid = _fid(func)
    want = torch.float64 if 64 <= fid < 80 else torch.float32
    if x.dtype != want or not x.is_cuda or not x.is_contiguous():
        raise ValueError("expected a contiguous CUDA %s tensor" % want)
    n = x.numel() // 2 if fid >= 80 else x.numel()
    nout = 2 * n if fid == FUNC_ID["sincosf"] or fid >= 80 else n
    if out is None:
        out = torch.empty(nout, dtype=want, device=x.device)
    eval_ptr(fid, x.data_ptr(), out.data_ptr(), n, impl, flags, _stream_ptr(stream))
    return out.view(2, n) if fid == FUNC_ID["sincosf"] else out.view(x.shape)


def dft_ptr(x_ptr, n, w_ptr, m, out_ptr, flags=0, stream_ptr=None):
    """Raw cr_dft call: device pointers (ints), sample and frequency counts."""
    rc = lib().cr_dft(ctypes.c_void_p(x_ptr), n, ctypes.c_void_p(w_ptr), m,
                      ctypes.c_void_p(out_ptr), flags, stream_ptr)
    if rc != CR_OK:
        raise CrError(rc, "cr_dft")


def dft(x, w, out=None, flags=0, stream=None):
    """cr_dft on CUDA float32 tensors x (samples) and w (angles per output):
    returns an (m, 2) float64 tensor of (re, im)."""
    import torch
    for t in (x, w):
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("expected contiguous CUDA float32 tensors")
    m = w.numel()
    if out is None:
        out = torch.empty((m, 2), dtype=torch.float64, device=w.device)
    dft_ptr(x.data_ptr(), x.numel(), w.data_ptr(), m, out.data_ptr(), flags, _stream_ptr(stream))
    return out


def _requests(reqs):
    """reqs: list of (func, in_ptr, out_ptr, n[, impl]) -> ctypes array"""
    arr = (Request * max(1, len(reqs)))()
    for i, r in enumerate(reqs):
        func, ip, op, n = r[:4]
        impl = r[4] if len(r) > 4 else IMPL_AUTO
        arr[i] = Request(_fid(func), impl, ip, op, n)
    return arr


class BatchPlan:
    """A cr_batch_plan: requests captured into one graph launch."""

    def __init__(self, reqs, flags=0):
        self._arr = _requests(reqs)
        self.handle = ctypes.c_void_p()
        rc = lib().cr_batch_plan_create(self._arr, len(reqs), flags, ctypes.byref(self.handle))
        if rc != CR_OK:
            raise CrError(rc, "cr_batch_plan_create")

    def launch(self, stream=None):
        rc = lib().cr_batch_plan_launch(self.handle, _stream_ptr(stream))
        if rc != CR_OK:
            raise CrError(rc, "cr_batch_plan_launch")

    def destroy(self):
        if self.handle:
            lib().cr_batch_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def eval_batch(reqs, stream=None):
    arr = _requests(reqs)
    rc = lib().cr_eval_batch(arr, len(reqs), _stream_ptr(stream))
    if rc != CR_OK:
        raise CrError(rc, "cr_eval_batch")


def eval_batch_noalloc(reqs, stream=None):
    """cr_eval_batch_noalloc: the batch with its tables in static scratch."""
    arr = _requests(reqs)
    rc = lib().cr_eval_batch_noalloc(arr, len(reqs), _stream_ptr(stream))
    if rc != CR_OK:
        raise CrError(rc, "cr_eval_batch_noalloc")


def stats_reset(stream=None):
    rc = lib().cr_stats_reset(_stream_ptr(stream))
    if rc != CR_OK:
        raise CrError(rc, "cr_stats_reset")


def stats_read(stream=None):
    s = Stats()
    rc = lib().cr_stats_read(_stream_ptr(stream), ctypes.byref(s))
    if rc != CR_OK:
        raise CrError(rc, "cr_stats_read")
    return {"elems": s.elems, "fallback_lanes": s.fallback_lanes,
            "fallback_waves": s.fallback_waves, "escapes": s.escapes,
            "escape_index": list(s.escape_index)[:min(16, s.escapes)]}


# ------------------------------------------------------------------ tuning
def tune_variants():
    """[(elems_per_thread, prefetch, table_in_lds)] of every kernel variant."""
    L = lib()
    out = []
    for v in range(L.cr_tune_num_variants()):
        e, p, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        rc = L.cr_tune_variant_info(v, ctypes.byref(e), ctypes.byref(p), ctypes.byref(t))
        if rc != CR_OK:
            raise CrError(rc, "cr_tune_variant_info")
        out.append((e.value, p.value, t.value))
    return out


def tune_get(func, impl=IMPL_AUTO):
    c = TuneCfg()
    rc = lib().cr_tune_get(_fid(func), impl, ctypes.byref(c))
    if rc != CR_OK:
        raise CrError(rc, "cr_tune_get")
    return c.variant, c.blocks_per_cu


def tune_set(func, impl, variant, blocks_per_cu):
    c = TuneCfg(variant, blocks_per_cu)
    rc = lib().cr_tune_set(_fid(func), impl, ctypes.byref(c))
    if rc != CR_OK:
        raise CrError(rc, "cr_tune_set")


def tune_reset():
    lib().cr_tune_reset()


def tune_batch_get(impl=IMPL_AUTO):
    """Workgroups per CU of the batch kernels of one implementation."""
    b = ctypes.c_int32()
    rc = lib().cr_tune_batch_get(impl, ctypes.byref(b))
    if rc != CR_OK:
        raise CrError(rc, "cr_tune_batch_get")
    return b.value


def tune_batch_set(impl, blocks_per_cu):
    rc = lib().cr_tune_batch_set(impl, blocks_per_cu)
    if rc != CR_OK:
        raise CrError(rc, "cr_tune_batch_set")


def tune_load(path):
    rc = lib().cr_tune_load(os.fsencode(path))
    if rc != CR_OK:
        raise CrError(rc, "cr_tune_load")


def tune_save(path):
    rc = lib().cr_tune_save(os.fsencode(path))
    if rc != CR_OK:
        raise CrError(rc, "cr_tune_save")


def autotune(func, impl, in_ptr, out_ptr, n, reps=5, stream_ptr=None):
    """Time every launch configuration on the given device buffers, install
    the fastest and return its rate (Gelem/s)."""
    best = ctypes.c_double()
    rc = lib().cr_autotune(_fid(func), impl, in_ptr, out_ptr, n, reps, stream_ptr,
                           ctypes.byref(best))
    if rc != CR_OK:
        raise CrError(rc, "cr_autotune")
    return best.value
