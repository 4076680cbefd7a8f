"""Oracle digests of every full-size workload and of exhaustive binary32 sweeps.

Correct rounding has one right answer per input, so a GPU result array can be
checked against the oracle through digests of the oracle's own results: this
script evaluates the CPU oracle (oracle/) on the seeded workloads of
paper_2605_15547_amd/inputs.py, or on every binary32 encoding, and stores an
xxh3-64 digest of the result bytes of each block of 2^20 consecutive
elements.  A GPU test recomputes the same digests from the library's output;
where a block's digest differs, only that block has to be evaluated element by
element with the oracle.  Nothing here touches the GPU library: the only
imports are the oracle and the input generators.

Targets (one JSON file each under tests/golden/digests/):
  expf_correctness          64 specials/edges + 2^20 uniform in [-103.9, 88.7]
  explog_2p26.<func>        exp/log family, 2^26 elements per function
  trig_2p26.<func>          trig/inverse/hyperbolic family, 2^26 per function
  binary64_2p24.<func>      binary64 exp/log/exp2, 2^24 elements per function
  batch_4096                the 4096-request ragged batch, one digest per request
  exhaustive.<func>         all 2^32 binary32 encodings of expf, logf, sinf
                            (paper, Sec. II-A: binary32 functions are validated
                            by exhaustive testing against an independent
                            reference)

Block digest: xxh3_64 of the little-endian result bytes of the block; for
sincosf the sine block's bytes followed by the cosine block's bytes.  A
digest of the input array is stored too, so a change of the input generators
shows as such rather than as a result mismatch.

Long targets checkpoint to <file>.partial and resume from it.

Usage: python tests/golden/make_digests.py [--threads N] [targets...]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np
import xxhash

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
from oracle import oracle as O  # noqa: E402
from paper_2605_15547_amd import inputs as I  # noqa: E402

OUT = os.path.join(HERE, "digests")
BLOCK = 1 << 20
SWEEP_FUNCS = ("expf", "logf", "sinf")


def block_digests(func, y, block=BLOCK):
    """Digest of each block of consecutive results (sincosf: shape (2, n))."""
    if func == "sincosf":
        n = y.shape[1]
        out = []
        for s in range(0, n, block):
            h = xxhash.xxh3_64()
            h.update(memoryview(np.ascontiguousarray(y[0, s:s + block])))
            h.update(memoryview(np.ascontiguousarray(y[1, s:s + block])))
            out.append(h.hexdigest())
        return out
    n = y.size
    return [xxhash.xxh3_64_hexdigest(memoryview(np.ascontiguousarray(y[s:s + block])))
            for s in range(0, n, block)]


def input_digest(x):
    return xxhash.xxh3_128_hexdigest(memoryview(np.ascontiguousarray(x)))


def oracle_sha():
    with open(os.path.join(ROOT, "oracle", "cr_oracle.c"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def write(name, doc):
    os.makedirs(OUT, exist_ok=True)
    path = os.path.join(OUT, name + ".json")
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=0)
        f.write("\n")
    os.replace(tmp, path)
    print("wrote", path, flush=True)


def exists(name):
    return os.path.exists(os.path.join(OUT, name + ".json"))


def evaluate(func, x, threads, step=1 << 23):
    """Oracle results of x, evaluated in slices so progress can be reported."""
    parts = []
    for s in range(0, x.size, step):
        parts.append(O.evaluate(func, x[s:s + step], threads))
    if func == "sincosf":
        return np.concatenate(parts, axis=1)
    return np.concatenate(parts)


def run_array(name, func, x, threads, recipe):
    t = time.time()
    y = evaluate(func, x, threads)
    doc = {"target": name, "func": func, "n": int(x.size), "block": BLOCK,
           "recipe": recipe, "input_xxh3_128": input_digest(x),
           "digests": block_digests(func, y), "oracle_sha256_16": oracle_sha(),
           "oracle_threads": threads, "oracle_seconds": round(time.time() - t, 1)}
    write(name, doc)


def t_expf_correctness(threads):
    if exists("expf_correctness"):
        return
    x = I.expf_correctness_set()
    run_array("expf_correctness", "expf", x, threads,
              "inputs.expf_correctness_set(): 64 specials/edges, then 2^20 uniform "
              "in [-103.9, 88.7], seed 0")


def t_family(fam, funcs, threads):
    for f in funcs:
        name = "%s.%s" % (fam, f)
        if exists(name):
            continue
        n = 1 << 24 if fam == "binary64_2p24" else 1 << 26
        x = I.workload_f64(f, n) if fam == "binary64_2p24" else I.workload_f32(f, n)
        run_array(name, f, x, threads, "inputs.workload_%s(%r, %d), default seed"
                  % ("f64" if fam == "binary64_2p24" else "f32", f, n))


def t_batch(threads):
    funcs, lens, seeds = I.batch_requests()
    t = time.time()
    digests, ind = [], []
    for f, n, sd in zip(funcs, lens, seeds):
        x = I.workload_f32(f, int(n), seed=int(sd) % (1 << 62))
        ind.append(input_digest(x))
        if n == 0:
            digests.append(None)
            continue
        y = O.evaluate(f, x, threads)
        d = block_digests(f, y, block=1 << 21)
        assert len(d) == 1
        digests.append(d[0])
    write("batch_4096", {"target": "batch_4096", "num": len(funcs), "funcs": list(funcs),
                         "lens": [int(v) for v in lens],
                         "recipe": "inputs.batch_requests(): 4096 requests, seed 5000; request k "
                                   "has inputs.workload_f32(func, len, seed=seed_k % 2^62); one "
                                   "digest per request over its whole result",
                         "input_xxh3_128": ind, "digests": digests,
                         "oracle_sha256_16": oracle_sha(), "oracle_threads": threads,
                         "oracle_seconds": round(time.time() - t, 1)})


def t_sweep(func, threads, chunk=1 << 23):
    """All 2^32 encodings in ascending order, checkpointed per chunk."""
    name = "exhaustive." + func
    if exists(name):
        return
    part = os.path.join(OUT, name + ".partial")
    digests, secs = [], 0.0
    if os.path.exists(part):
        with open(part) as fh:
            st = json.load(fh)
        digests, secs = st["digests"], st["seconds"]
    nblk = (1 << 32) // BLOCK
    per = chunk // BLOCK
    while len(digests) < nblk:
        c0 = len(digests) * BLOCK
        t = time.time()
        x = np.arange(c0, c0 + chunk, dtype=np.uint64).astype(np.uint32).view(np.float32)
        y = O.evaluate(func, x, threads)
        digests += block_digests(func, y)
        secs += time.time() - t
        with open(part + ".tmp", "w") as fh:
            json.dump({"digests": digests, "seconds": secs}, fh)
        os.replace(part + ".tmp", part)
        if len(digests) % (per * 32) == 0:
            print("%s: %d/%d blocks, %.0f s" % (func, len(digests), nblk, secs), flush=True)
    write(name, {"target": name, "func": func, "n": 1 << 32, "block": BLOCK,
                 "recipe": "every binary32 encoding 0x00000000..0xffffffff in ascending order; "
                           "block b holds encodings [b 2^20, (b+1) 2^20)",
                 "digests": digests, "oracle_sha256_16": oracle_sha(),
                 "oracle_threads": threads, "oracle_seconds": round(secs, 1)})
    os.remove(part)


TARGETS = ["expf_correctness", "explog", "binary64", "batch", "trig"] + \
    ["sweep_" + f for f in SWEEP_FUNCS]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=O.default_threads())
    ap.add_argument("targets", nargs="*", default=TARGETS)
    a = ap.parse_args()
    O.build()
    for tg in a.targets:
        t = time.time()
        if tg == "expf_correctness":
            t_expf_correctness(a.threads)
        elif tg == "explog":
            t_family("explog_2p26", I.EXPLOG_FAMILY, a.threads)
        elif tg == "trig":
            t_family("trig_2p26", I.TRIG_FAMILY, a.threads)
        elif tg == "binary64":
            t_family("binary64_2p24", ["exp", "log", "exp2"], a.threads)
        elif tg == "batch":
            if not exists("batch_4096"):
                t_batch(a.threads)
        elif tg.startswith("sweep_"):
            t_sweep(tg[len("sweep_"):], a.threads)
        else:
            raise SystemExit("unknown target " + tg)
        print("target %s done in %.0f s" % (tg, time.time() - t), flush=True)


if __name__ == "__main__":
    main()
