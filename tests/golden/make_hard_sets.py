"""Writes the hard-to-round input sets used by the workloads and the tests.

Every value written here comes from the oracle (oracle/): candidate inputs are
preselected by a cheap estimate inside the oracle's scan and their hardness
  h(x) = -log2(distance of f(x) to the nearest rounding boundary / ulp)
is measured by the oracle's Ziv evaluator.  Nothing here touches the GPU
library.

binary32 functions: exhaustive scan of all 2^32 encodings; the 2048 inputs
with the largest h are kept (tests/golden/hard/<func>.u32, little endian).
binary64 exp/log/exp2: a quad-precision-prefiltered scan of 2^26 seeded
samples of the binary64 workload (exp2: half on [-20, 20], half over the whole
range) plus, for exp and log, two constructed families near the points where the
Taylor expansion puts f(x) next to a midpoint (exp near 0, log near 1); 1024
of each kind are kept (tests/golden/hard/<func>.u64).

Usage: python tests/golden/make_hard_sets.py [--threads N] [--only f1,f2]
(all binary32 functions and binary64 exp, log by default; exp2 with --only exp2)
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
from oracle import oracle as O  # noqa: E402
from paper_2605_15547_amd import inputs as I  # noqa: E402

OUT = os.path.join(HERE, "hard")
K32 = 2048
K64 = 1024


def sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def scan32(func, threads):
    t = time.time()
    bits, h, cnt = O.scan_f32(func, 0, 1 << 32, 18.0, 19.0, max_out=1 << 22, nthreads=threads)
    order = np.lexsort((bits, -h))[:K32]
    bits, h = bits[order], h[order]
    path = os.path.join(OUT, func + ".u32")
    bits.astype("<u4").tofile(path)
    return {"count_h_ge_19": int(cnt), "kept": int(bits.size), "max_h": float(h.max()),
            "min_h_kept": float(h.min()), "hardest_bits": "%08x" % int(bits[0]),
            "seconds": round(time.time() - t, 1), "sha256": sha(path)}


def constructed64(func):
    k = np.arange(1, 20001, dtype=np.float64)
    if func == "exp":
        # 1 + x is a binary64 midpoint for these x; exp(x) - (1 + x) ~ x^2/2
        return np.concatenate([k * 2.0 ** -53, -k * 2.0 ** -54])
    # log(1 + t) = t - t^2/2 + t^3/3 ...; t^2/2 lands on a midpoint for some t
    return np.concatenate([1.0 + k * 2.0 ** -52, 1.0 - k * 2.0 ** -53])


def scan64(func, threads):
    t = time.time()
    n = 1 << 26
    st = I.Stream(7000 + I.FUNC_ID[func])
    if func == "exp":
        x = -745.0 + (709.7 + 745.0) * st.uniform(n)
    elif func == "exp2":
        # half on [-20, 20] (where the paper measures binary64 exp2), half over
        # the whole range with a finite nonzero result
        x = np.concatenate([-20.0 + 40.0 * st.uniform(n // 2),
                            -1075.0 + (1024.0 + 1075.0) * st.uniform(n - n // 2)])
    else:
        E = -1074 + st.below(n, 1023 + 1074 + 1)
        f = (st.u64(n) >> np.uint64(12)).astype(np.float64) * 2.0 ** -52
        x = np.ldexp(1.0 + f, E)
    rx, rh, cnt = O.scan_f64(func, x, 15.0, 16.0, max_out=1 << 20, nthreads=threads)
    o = np.lexsort((rx, -rh))[:K64]
    rx, rh = rx[o], rh[o]
    if func == "exp2":  # no constructed family: the sampled scan only
        cx = ch = np.zeros(0)
    else:
        cx = constructed64(func)
        ch = O.hardness(func, cx, threads)
        o = np.lexsort((cx, -ch))[:K64]
        cx, ch = cx[o], ch[o]
    allx = np.concatenate([rx, cx])
    path = os.path.join(OUT, func + ".u64")
    allx.view(np.uint64).astype("<u8").tofile(path)
    return {"sampled": n, "sample_count_h_ge_16": int(cnt), "kept_sampled": int(rx.size),
            "sampled_max_h": float(rh.max()), "sampled_min_h_kept": float(rh.min()),
            "kept_constructed": int(cx.size),
            "constructed_max_h": float(ch.max()) if ch.size else None,
            "constructed_min_h_kept": float(ch.min()) if ch.size else None,
            "seconds": round(time.time() - t, 1), "sha256": sha(path)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=O.default_threads())
    ap.add_argument("--only", default="")
    a = ap.parse_args()
    O.build()
    os.makedirs(OUT, exist_ok=True)
    idx_path = os.path.join(OUT, "index.json")
    idx = json.load(open(idx_path)) if os.path.exists(idx_path) else {}
    funcs = a.only.split(",") if a.only else I.FUNCS32 + ["exp", "log"]
    for func in funcs:
        r = scan64(func, a.threads) if func in ("exp", "log", "exp2") else scan32(func, a.threads)
        idx[func] = r
        print(func, r, flush=True)
        idx["_command"] = "python tests/golden/make_hard_sets.py"
        with open(idx_path, "w") as f:
            json.dump(idx, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
