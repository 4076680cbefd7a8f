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
    for f in (-1, 19, 63, 66, 1000):
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
