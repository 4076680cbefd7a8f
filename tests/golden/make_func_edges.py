"""Writes tests/golden/func_edges.json: for every function of the library, the
inputs around the places where its correctly rounded result changes regime --
overflow to infinity, underflow to zero, the first subnormal result,
saturation (tanh to 1, expm1 to -1, atan to pi/2), and the last input whose
result is still exactly x, 1 or -x (odd functions near 0, cos/cosh/exp near
0).  Each edge is located with the oracle by bisection over encodings in
value order and stored with the 2 encodings on either side.  Calls only
oracle/.

Usage: python tests/golden/make_func_edges.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
from oracle import oracle as O  # noqa: E402

OUT = os.path.join(HERE, "func_edges.json")
F64 = ("exp", "log", "exp2")


class Fmt:
    """binary32 or binary64 encodings as monotone integer keys (value order)."""

    def __init__(self, wide):
        self.wide = wide
        self.ut = np.uint64 if wide else np.uint32
        self.ft = np.float64 if wide else np.float32
        self.sign = 1 << (63 if wide else 31)

    def key(self, x):
        b = int(np.array([x], dtype=self.ft).view(self.ut)[0])
        return b if b < self.sign else -(b & (self.sign - 1))

    def enc(self, k):
        return k if k >= 0 else (self.sign | (-k))

    def val(self, k):
        return np.array([self.enc(k)], dtype=self.ut).view(self.ft)[0]


def f_of(func, fmt, k):
    y = O.evaluate(func, np.array([fmt.val(k)], dtype=fmt.ft), 1)
    return y[:, 0] if func == "sincosf" else y[0]


def boundary(pred, lo, hi):
    """largest key k in [lo, hi) with pred(k) true, given pred(lo) and not pred(hi)"""
    assert pred(lo) and not pred(hi), (lo, hi)
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if pred(mid):
            lo = mid
        else:
            hi = mid
    return lo


def edges_of(func):
    """(name, key of the last input on the 'true' side, format) of each edge"""
    wide = func in F64
    fm = Fmt(wide)
    K = fm.key
    f = lambda k: f_of(func, fm, k)  # noqa: E731
    tiny = np.finfo(fm.ft).tiny
    out = []

    def add(name, pred, a, b):
        out.append((name, boundary(pred, K(a), K(b))))

    def add_neg(name, pred, a, b):
        """pred over keys k of |x| in [a, b], the edge stored at x < 0"""
        out.append((name, -boundary(pred, K(a), K(b))))

    def same_as_x(a, b):
        add("f(x) == x", lambda k: f(k) == fm.val(k), a, b)
        add_neg("f(x) == x (x < 0)", lambda k: f(-k) == fm.val(-k), a, b)

    if func in ("expf", "exp2f", "exp10f", "exp", "exp2"):
        hi = {"expf": 100.0, "exp2f": 140.0, "exp10f": 45.0, "exp": 720.0, "exp2": 1030.0}[func]
        lo = {"expf": -120.0, "exp2f": -160.0, "exp10f": -50.0, "exp": -760.0,
              "exp2": -1090.0}[func]
        add("overflow", lambda k: np.isfinite(f(k)), 0.0, hi)
        add("underflow to zero", lambda k: f(k) == 0.0, lo, 0.0)
        add("subnormal result", lambda k: f(k) < tiny, lo, 0.0)
        add("f(x) == 1 (x > 0)", lambda k: f(k) == 1.0, 0.0, 1e-3)
        add_neg("f(x) == 1 (x < 0)", lambda k: f(-k) == 1.0, 0.0, 1e-3)
    elif func == "expm1f":
        add("overflow", lambda k: np.isfinite(f(k)), 0.0, 100.0)
        add("saturation to -1", lambda k: f(k) == -1.0, -100.0, 0.0)
        same_as_x(0.0, 1e-3)
    elif func in ("logf", "log2f", "log10f", "log"):
        # the result is 0 only at 1: the encodings around 1, the subnormal and
        # normal ends of the domain
        out.append(("x == 1", K(1.0)))
        out.append(("smallest normal", K(tiny)))
        out.append(("largest finite", K(np.finfo(fm.ft).max)))
    elif func == "log1pf":
        same_as_x(0.0, 1e-3)
        out.append(("x == -1", K(-1.0)))
    elif func == "rsqrtf":
        out.append(("x == 1", K(1.0)))
        out.append(("smallest normal", K(tiny)))
        out.append(("largest finite", K(np.finfo(fm.ft).max)))
    elif func in ("sinf", "tanf", "asinf", "atanf", "sinhf", "tanhf"):
        same_as_x(0.0, 0.5)
        if func == "atanf":
            add("saturation to RN(pi/2)", lambda k: f(k) < f(K(3.0e38)), 1.0, 3.0e38)
        if func == "tanhf":
            add("saturation to 1", lambda k: f(k) < 1.0, 0.0, 100.0)
            add("saturation to -1", lambda k: f(k) == -1.0, -100.0, 0.0)
        if func == "sinhf":
            add("overflow", lambda k: np.isfinite(f(k)), 0.0, 100.0)
            add_neg("overflow (x < 0)", lambda k: np.isfinite(f(-k)), 0.0, 100.0)
        if func == "asinf":
            out.append(("x == 1", K(1.0)))
            out.append(("x == -1", K(-1.0)))
    elif func in ("cosf", "coshf"):
        add("f(x) == 1", lambda k: f(k) == 1.0, 0.0, 0.5)
        add_neg("f(x) == 1 (x < 0)", lambda k: f(-k) == 1.0, 0.0, 0.5)
        if func == "coshf":
            add("overflow", lambda k: np.isfinite(f(k)), 0.0, 100.0)
    elif func == "sincosf":
        add("sin(x) == x", lambda k: f(k)[0] == fm.val(k), 0.0, 0.5)
        add("cos(x) == 1", lambda k: f(k)[1] == 1.0, 0.0, 0.5)
    elif func == "acosf":
        add("f(x) == RN(pi/2) (x > 0)", lambda k: f(k) == f(0), 0.0, 0.5)
        add_neg("f(x) == RN(pi/2) (x < 0)", lambda k: f(-k) == f(0), 0.0, 0.5)
        out.append(("x == 1", K(1.0)))
        out.append(("x == -1", K(-1.0)))
    else:
        raise ValueError(func)
    return out, fm


def main():
    O.build()
    doc = {"command": "python tests/golden/make_func_edges.py", "width": 2, "functions": {}}
    for func in O.FUNCS32 + list(F64):
        edges, fm = edges_of(func)
        ents = []
        for name, k in edges:
            enc = [fm.enc(k + d) for d in range(-2, 3)]
            ents.append({"edge": name, "bits": ["%0*x" % (16 if fm.wide else 8, e) for e in enc]})
        doc["functions"][func] = ents
        print(func, [(e["edge"], e["bits"][2]) for e in ents], flush=True)
    with open(OUT, "w") as fh:
        json.dump(doc, fh, indent=1)
        fh.write("\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
