"""Writes tests/golden/expf_edges.json: the 64 special and edge inputs that open
the expf correctness workload.  Edges are located with the oracle (bisection
over binary32 encodings); the set is filled up with the hardest expf inputs of
tests/golden/hard/expf.u32.  Calls only oracle/.

Usage: python tests/golden/make_edges.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
from oracle import oracle as O  # noqa: E402


def f32(b):
    return np.array([b], dtype=np.uint32).view(np.float32)[0]


def bits(x):
    return int(np.array([x], dtype=np.float32).view(np.uint32)[0])


def order(b):
    """monotone integer key of a binary32 encoding (value order)"""
    return b if b < 0x80000000 else -(b & 0x7FFFFFFF)


def from_order(k):
    return k if k >= 0 else (0x80000000 | (-k))


def expf(b):
    return O.evaluate("expf", np.array([f32(b)], dtype=np.float32), 1)[0]


def last_true(pred, lo, hi):
    """largest order key k in [lo, hi] with pred(k) true (pred monotone: true then false)"""
    assert pred(lo) and not pred(hi)
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if pred(mid):
            lo = mid
        else:
            hi = mid
    return lo


def around(k, w=2):
    return [from_order(k + d) for d in range(-w, w + 1)]


def main():
    O.build()
    fmax = np.finfo(np.float32).max
    fixed = [0x00000000, 0x80000000, 0x7F800000, 0xFF800000,
             0x7FC00000, 0xFFC00000, 0x7F800001, 0x7FC12345,   # +-qNaN, sNaN, payload NaN
             0x00000001, 0x80000001, 0x007FFFFF, 0x807FFFFF,   # +-min/max subnormal
             0x00800000, 0x80800000, 0x7F7FFFFF, 0xFF7FFFFF,   # +-FLT_MIN, +-FLT_MAX
             bits(1.0), bits(-1.0), bits(np.float32(np.log(2.0))), bits(-np.float32(np.log(2.0)))]
    edges = []
    # overflow: largest x with expf(x) finite
    k = last_true(lambda k: np.isfinite(expf(from_order(k))), order(bits(80.0)), order(bits(100.0)))
    edges += around(k)
    # underflow to zero: largest x with expf(x) == 0
    k = last_true(lambda k: expf(from_order(k)) == 0.0, order(bits(-120.0)), order(bits(-90.0)))
    edges += around(k)
    # subnormal/normal result edge: largest x with expf(x) < FLT_MIN
    tiny = np.finfo(np.float32).tiny
    k = last_true(lambda k: expf(from_order(k)) < tiny, order(bits(-100.0)), order(bits(-80.0)))
    edges += around(k)
    # largest x > 0 and smallest x < 0 with expf(x) == 1
    k = last_true(lambda k: expf(from_order(k)) == 1.0, 0, order(bits(1e-3)))
    edges.append(from_order(k))
    k = last_true(lambda k: expf(from_order(-k)) == 1.0, 0, order(bits(1e-3)))
    edges.append(from_order(-k))
    allb = fixed + edges
    hard = np.fromfile(os.path.join(HERE, "hard", "expf.u32"), dtype="<u4")
    for b in hard:
        if len(allb) >= 64:
            break
        if int(b) not in allb:
            allb.append(int(b))
    assert len(allb) == 64
    with open(os.path.join(HERE, "expf_edges.json"), "w") as f:
        json.dump({"command": "python tests/golden/make_edges.py",
                   "bits": ["%08x" % b for b in allb],
                   "n_fixed": len(fixed), "n_edges": len(edges)}, f, indent=1)
    print("wrote", len(allb), "edge inputs")


if __name__ == "__main__":
    main()
