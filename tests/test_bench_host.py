"""Host-side helpers of bench.py (CPU only): the kernel source hash that ties
the committed counter summaries to the code they were taken with."""
import importlib.util
import json
import os
import shutil
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    argv = sys.argv
    sys.argv = ["bench.py"]
    try:
        spec.loader.exec_module(b)
    finally:
        sys.argv = argv
    return b


def copy_tree(tmp_path):
    dst = tmp_path / "paper_2605_15547_amd" / "csrc"
    shutil.copytree(os.path.join(ROOT, "paper_2605_15547_amd", "csrc"), dst,
                    ignore=shutil.ignore_patterns("*.so", "*.o"))
    shutil.copytree(os.path.join(ROOT, "profiles"), tmp_path / "profiles")
    return dst


def test_source_hash_ignores_comments_but_not_code(tmp_path):
    b = load_bench()
    h0 = b.kernel_source_hash()
    csrc = copy_tree(tmp_path)
    b.ROOT = str(tmp_path)
    assert b.kernel_source_hash() == h0
    f = csrc / "cr_f32_log.h"
    text = f.read_text()
    f.write_text(text.replace("namespace cr {", "// a new comment\n/* and\n another */\nnamespace cr {", 1))
    assert b.kernel_source_hash() == h0
    f.write_text(text.replace("constexpr unsigned LOG_TEST_E = 1;", "constexpr unsigned LOG_TEST_E = 2;"))
    assert b.kernel_source_hash() != h0


def test_committed_summaries_match_the_code():
    """profiles/traffic.json, valu.json and flops.json were taken with the
    current kernel code (bench.py reads them only then)."""
    b = load_bench()
    h = b.kernel_source_hash()
    for name in ("traffic.json", "valu.json", "flops.json"):
        with open(os.path.join(ROOT, "profiles", name)) as fh:
            assert json.load(fh)["source_hash"] == h, name
    n = 1 << 26
    assert b.measured_traffic("log1pf", n) and b.measured_valu("log1pf", n)
    assert b.measured_flops("log1pf", n)["fp64_per_elem"] > 0
