"""The C-ABI library loads, exports every entry point its header declares, and
rejects bad arguments on the host before touching the GPU (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2605_15547_amd import build, crmath
    if not os.path.exists(crmath.LIB_PATH):
        build.build()
    return crmath.lib()


def declared_functions():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"^[A-Za-z_][\w \*]*?\b(cr_\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert "cr_eval" in names and "cr_eval_ex" in names
    for n in names:
        assert hasattr(L, n), n


def test_status_strings(L):
    from paper_2605_15547_amd import crmath
    for code in crmath.STATUS:
        assert L.cr_status_str(code)


def test_argument_validation(L):
    from paper_2605_15547_amd import crmath as C
    ev = L.cr_eval_ex
    vp = ctypes.c_void_p
    # n == 0: nothing to do
    assert ev(0, 0, 0, None, None, 0, None) == C.CR_OK
    # unknown function ids
    for f in (-1, 19, 63, 67, 79, 83, 1000):
        assert ev(f, 0, 0, vp(0x1000), vp(0x2000), 8, None) == -1
    # null pointers
    assert ev(0, 0, 0, None, vp(0x2000), 8, None) == -2
    assert ev(0, 0, 0, vp(0x1000), None, 8, None) == -2
    # misaligned (not a multiple of the element size)
    assert ev(0, 0, 0, vp(0x1001), vp(0x2000), 8, None) == -4
    assert ev(64, 0, 0, vp(0x1004), vp(0x2000), 8, None) == -4
    # overlapping ranges (in-place itself is allowed)
    assert ev(0, 0, 0, vp(0x1000), vp(0x1004), 8, None) == -3
    assert ev(11, 0, 0, vp(0x1000), vp(0x1000), 8, None) in (-3, -5)  # sincosf in place
    # unknown implementation
    assert ev(0, 7, 0, vp(0x1000), vp(0x2000), 8, None) == -5
    assert L.cr_available(0, 7) == 0
    assert L.cr_available(99, 0) == 0
    # binary64 exp2 takes 8-byte elements
    assert ev(66, 0, 0, vp(0x1004), vp(0x2000), 8, None) == -4
    # complex functions: float pairs, 4-byte alignment, no binary32-only form
    assert ev(80, 0, 0, vp(0x1002), vp(0x2000), 8, None) == -4
    assert ev(81, 0, 0, vp(0x1000), vp(0x1008), 8, None) == -3  # 8 pairs = 64 bytes
    assert ev(82, 2, 0, vp(0x1000), vp(0x2000), 8, None) == -5
    for f in (80, 81, 82, 66):
        assert L.cr_available(f, 0) == 1
        assert L.cr_available(f, 2) == 0


def test_rounding_mode_validation(L):
    """Directed modes: binary32 functions with the binary64-internal
    implementation only; batches round to nearest."""
    from paper_2605_15547_amd import crmath as C
    vp = ctypes.c_void_p
    ev = L.cr_eval_ex
    for fl in (C.FLAG_ROUND_TOWARD_ZERO, C.FLAG_ROUND_UP, C.FLAG_ROUND_DOWN):
        assert ev(64, 0, fl, vp(0x1000), vp(0x2000), 8, None) == -5   # binary64 exp
        assert ev(80, 0, fl, vp(0x1000), vp(0x2000), 8, None) == -5   # complex
        assert ev(65, 3, fl, vp(0x1000), vp(0x2000), 8, None) == -5   # log, 128-entry table
        assert ev(0, 2, fl, vp(0x1000), vp(0x2000), 8, None) == -5    # split implementation
        plan = vp()
        arr = C._requests([("expf", 0x1000, 0x2000, 8)])
        assert L.cr_batch_plan_create(arr, 1, fl, ctypes.byref(plan)) == -5
        assert plan.value is None


def test_dft_validation(L):
    """cr_dft rejects bad arguments before launching anything."""
    vp = ctypes.c_void_p
    d = L.cr_dft
    assert d(vp(0x1000), 8, vp(0x2000), 0, vp(0x3000), 0, None) == 0   # m == 0
    assert d(vp(0x1000), (1 << 24) + 1, vp(0x2000), 4, vp(0x3000), 0, None) == -9
    assert d(vp(0x1000), -1, vp(0x2000), 4, vp(0x3000), 0, None) == -9
    assert d(None, 8, vp(0x2000), 4, vp(0x3000), 0, None) == -2
    assert d(vp(0x1000), 8, None, 4, vp(0x3000), 0, None) == -2
    assert d(vp(0x1000), 8, vp(0x2000), 4, None, 0, None) == -2
    assert d(vp(0x1000), 8, vp(0x2000), 4, vp(0x3008), 0, None) == -4
    assert d(vp(0x1002), 8, vp(0x2000), 4, vp(0x3000), 0, None) == -4
    assert d(vp(0x3010), 8, vp(0x2000), 4, vp(0x3000), 0, None) == -3  # x inside X
    assert d(vp(0x1000), 8, vp(0x3030), 4, vp(0x3000), 0, None) == -3  # w inside X


def test_batch_validation(L):
    """Batch requests are validated on the host before anything touches a GPU."""
    from paper_2605_15547_amd import crmath as C
    vp = ctypes.c_void_p
    plan = vp()

    def create(reqs):
        arr = C._requests(reqs)
        return L.cr_batch_plan_create(arr, len(reqs), 0, ctypes.byref(plan))

    assert L.cr_batch_plan_create(None, 1, 0, ctypes.byref(plan)) == -2
    assert create([("expf", 0x1000, 0x2000, 8), (64, 0x3000, 0x4000, 8)]) == -1  # binary64
    assert create([(19, 0x1000, 0x2000, 8)]) == -1
    assert create([("expf", 0x1000, 0x2000, -1)]) == -9
    assert create([("expf", 0x1000, 0x2000, 1 << 31)]) == -9
    assert create([("expf", 0, 0x2000, 8)]) == -2
    assert create([("expf", 0x1002, 0x2000, 8)]) == -4
    assert create([("logf", 0x1000, 0x1008, 8)]) == -3
    assert create([("sincosf", 0x1000, 0x1000, 8)]) == -3
    assert create([("expf", 0x1000, 0x2000, 8, 9)]) == -5
    assert plan.value is None
    assert L.cr_batch_plan_launch(None, None) == -2
    assert L.cr_batch_plan_destroy(None) == 0


def test_tuning_table(L, tmp_path):
    """Launch configurations: defaults, set/get, validation, save/load round
    trip, and a malformed file applying nothing (host only, no GPU)."""
    from paper_2605_15547_amd import crmath as C
    C.tune_reset()
    vs = C.tune_variants()
    assert len(vs) == L.cr_tune_num_variants() >= 2
    assert vs[0] == (8, 1, 1)  # the default: 8 elements per thread, prefetch, LDS tables
    assert {e for e, _, _ in vs} == {4, 8, 16} and {t for _, _, t in vs} == {0, 1}
    assert C.tune_get("expf") == (0, 16)
    C.tune_set("logf", C.IMPL_F64_INTERNAL, 2, 8)
    assert C.tune_get("logf", C.IMPL_AUTO) == (2, 8)  # AUTO is the binary64-internal table
    assert C.tune_get("logf", C.IMPL_SPLIT_F32) == (0, 16)
    for func, impl, v, b in (("expf", 1, len(vs), 16), ("expf", 1, -1, 16), ("expf", 1, 0, 65),
                             ("sincosf", 1, 1, 16), ("exp", 1, 4, 16), ("cexpf", 1, 1, 16)):
        with pytest.raises(C.CrError) as e:
            C.tune_set(func, impl, v, b)
        assert e.value.status == -10
    with pytest.raises(C.CrError):
        C.tune_set("expf", 7, 0, 16)
    p = str(tmp_path / "tune.txt")
    C.tune_save(p)
    C.tune_reset()
    assert C.tune_get("logf") == (0, 16)
    C.tune_load(p)
    assert C.tune_get("logf") == (2, 8)
    bad = tmp_path / "bad.txt"
    bad.write_text("# header\nexpf f64 3 4\nnosuchf f64 0 16\n")
    with pytest.raises(C.CrError):
        C.tune_load(str(bad))
    assert C.tune_get("expf") == (0, 16)  # nothing applied
    for text in ("expf f64 0\n", "expf f32 0 16\n", "sincosf split 2 16\n", "log f64 0 99\n"):
        bad.write_text(text)
        with pytest.raises(C.CrError):
            C.tune_load(str(bad))
    with pytest.raises(C.CrError):
        C.tune_load(str(tmp_path / "missing.txt"))
    ok = tmp_path / "ok.txt"
    # the batch grid: one setting per implementation, in the same file
    assert C.tune_batch_get() == 4 and C.tune_batch_get(C.IMPL_SPLIT_F32) == 4
    C.tune_batch_set(C.IMPL_SPLIT_F32, 9)
    assert C.tune_batch_get(C.IMPL_SPLIT_F32) == 9 and C.tune_batch_get(C.IMPL_F64_INTERNAL) == 4
    for impl, b in ((C.IMPL_F64_INTERNAL, 0), (C.IMPL_F64_INTERNAL, 65), (C.IMPL_LOG128, 4),
                    (7, 4)):
        with pytest.raises(C.CrError):
            C.tune_batch_set(impl, b)
    C.tune_save(p)
    assert "batch split 0 9" in open(p).read().splitlines()
    C.tune_reset()
    assert C.tune_batch_get(C.IMPL_SPLIT_F32) == 4
    C.tune_load(p)
    assert C.tune_batch_get(C.IMPL_SPLIT_F32) == 9
    for text in ("batch f64 1 4\n", "batch f64 0 0\n", "batch f32 0 4\n", "batch f64 0\n"):
        bad.write_text(text)
        with pytest.raises(C.CrError):
            C.tune_load(str(bad))
    assert C.tune_batch_get(C.IMPL_SPLIT_F32) == 9  # nothing applied
    C.tune_reset()
    ok.write_text("  # comment\n\nexpf split 6 4\nexp f64 3 2\nbatch f64 0 2\n")
    C.tune_load(str(ok))
    # the binary64 functions have variants 0..3 of their own kernel
    assert C.tune_get("expf", C.IMPL_SPLIT_F32) == (6, 4) and C.tune_get("exp") == (3, 2)
    assert C.tune_batch_get() == 2
    C.tune_reset()
    # the autotuner validates its arguments before touching the GPU
    vp = ctypes.c_void_p
    at = L.cr_autotune
    assert at(0, 0, None, vp(0x2000), 8, 1, None, None) == -2
    assert at(99, 0, vp(0x1000), vp(0x2000), 8, 1, None, None) == -1
    assert at(0, 5, vp(0x1000), vp(0x2000), 8, 1, None, None) == -5
    assert at(0, 0, vp(0x1001), vp(0x2000), 8, 1, None, None) == -4
    assert at(0, 0, vp(0x1000), vp(0x1004), 8, 1, None, None) == -3


def test_committed_tuning_file_is_valid(L):
    """The launch configurations shipped for MI355X load cleanly and cover
    every function of both implementations."""
    from paper_2605_15547_amd import crmath as C
    path = os.path.join(ROOT, "paper_2605_15547_amd", "tuning", "mi355x.txt")
    assert os.path.exists(path)
    C.tune_reset()
    try:
        C.tune_load(path)
        seen = set()
        for line in open(path):
            if line.strip() and not line.lstrip().startswith("#"):
                f, impl, v, b = line.split()
                seen.add((f, impl))
                im = C.IMPL_SPLIT_F32 if impl == "split" else C.IMPL_F64_INTERNAL
                if f == "batch":
                    assert C.tune_batch_get(im) == int(b) and int(v) == 0
                else:
                    assert C.tune_get(f, im) == (int(v), int(b))
        for f in C.FUNCS32:
            assert (f, "f64") in seen and (f, "split") in seen, f
        assert ("exp", "f64") in seen and ("log", "f64") in seen
        assert ("batch", "f64") in seen and ("batch", "split") in seen
    finally:
        C.tune_reset()
