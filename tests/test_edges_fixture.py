"""The regime-edge fixture (tests/golden/func_edges.json) against a fresh
oracle bisection for a few functions (CPU only)."""
import json
import os
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))


@pytest.mark.parametrize("func", ["expf", "tanhf", "atanf", "exp2"])
def test_edges_fixture_reproduces(oracle, func):
    import make_func_edges as ME
    with open(os.path.join(HERE, "golden", "func_edges.json")) as f:
        doc = json.load(f)["functions"][func]
    edges, fm = ME.edges_of(func)
    assert [e["edge"] for e in doc] == [n for n, _ in edges]
    for e, (name, k) in zip(doc, edges):
        assert int(e["bits"][2], 16) == fm.enc(k), (func, name)
