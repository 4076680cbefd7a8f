"""Benchmark: correctly rounded Gelem/s and % of the HBM roofline on one MI355X.

One step = one pass of the hot path over the exp/log-family workload: each of
expf, exp2f, exp10f, expm1f, logf, log2f, log10f, log1pf, rsqrtf evaluated on
its own 2^26 binary32 inputs (90% uniform over the domain, 5% raw bit
patterns, 5% hard-to-round inputs; paper_2605_15547_amd/inputs.py), inputs
resident in HBM before the timed region.  Functions the library does not
provide yet are listed in config.missing and left out.

Output: one JSON line.  value = total elements / total time (Gelem/s).  The
roofline object describes the kernel with the largest share of the step:
algorithmic bytes (4 B in + 4 B out per element) over its average launch
time, measured with HIP events on the stream it runs on.  cpu_baseline times
the CPU oracle (oracle/) on a bounded sample of the same inputs.

other_workloads (left out with --headline-only) reports, outside the headline
value: expf on its 2^20 + 64-element correctness set (launch-bound: the median
launch), the trig/inverse-trig/hyperbolic family at the same size, binary64
exp/log/exp2 on 2^24 inputs each (exp2 uniform in [-20, 20], the paper's
range), the paper's GPU metric (correctly rounded over the platform's ~1-ulp
library functions for expf, logf, sincosf, exp, log, exp2),
the ragged batch of 4096 mixed requests evaluated by one graph launch per step
(plan creation timed separately), the binary32-only implementation on the
same workloads, and the paper's application workloads (complex expf/logf/sinf
on 2^24 complex numbers, a 2^20-sample brute-force DFT at 256 frequencies).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n LOG2N]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

# binary64 functions (16 bytes per element)
F64 = ("exp", "log", "exp2")

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALU_PEAK = 256 * 64 * 2.4e9  # lane-instructions/s: one wave64 VALU instruction per CU per cycle
FAMILY = ["expf", "exp2f", "exp10f", "expm1f", "logf", "log2f", "log10f", "log1pf", "rsqrtf"]
TRIG = ["sinf", "cosf", "sincosf", "tanf", "asinf", "acosf", "atanf", "sinhf", "coshf", "tanhf"]
OTHER_LEGS = ("correctness", "trig", "binary64", "vsulp", "complex", "dft", "batch", "split")


def bytes_per_elem(func):
    return 16 if func in F64 else (12 if func == "sincosf" else 8)


def sample_sclk(result):
    """The shader clock while the settle phase keeps the GPU busy: one
    `rocm-smi --showclocks` (a child process), its sclk lines parsed (MHz; the
    largest if several GPUs are listed).  Stores the value, or None and why."""
    import re
    import subprocess
    try:
        out = subprocess.run(["rocm-smi", "--showclocks"], capture_output=True, text=True,
                             timeout=15).stdout
        mhz = [int(m) for m in re.findall(r"sclk clock level:\s*\d+:\s*\((\d+)\s*Mhz\)", out,
                                          flags=re.I)]
        result["sclk_mhz"] = max(mhz) if mhz else None
        if not mhz:
            result["why"] = "no sclk line in rocm-smi --showclocks"
    except (OSError, subprocess.SubprocessError) as e:
        result["sclk_mhz"] = None
        result["why"] = str(e)[:120]


def settle(fn, seconds, torch):
    """Untimed launches for `seconds` so the clocks settle under this load."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        fn()
        torch.cuda.synchronize()


def bench_family(torch, crmath, inputs, funcs, n, impl, steps, warmup, stream, settle_s=0.5):
    """Gelem/s and HBM fraction per function (inputs resident in HBM), plus the
    accurate-path share, for a family workload of n elements per function."""
    sp = crmath._stream_ptr(stream)
    res = {}
    bufs = {}
    for f in funcs:
        if not crmath.available(f, impl):
            res[f] = None
            continue
        x = inputs.workload_f64(f, n) if f in F64 else inputs.workload_f32(f, n)
        xt = torch.from_numpy(x).cuda()
        ot = torch.empty(2 * n if f == "sincosf" else n, dtype=xt.dtype, device="cuda")
        bufs[f] = (xt, ot)

    def launch(f):
        xt, ot = bufs[f]
        crmath.eval_ptr(f, xt.data_ptr(), ot.data_ptr(), n, impl, 0, sp)

    settle(lambda: [launch(f) for f in bufs], settle_s, torch)
    for f in bufs:
        for _ in range(warmup):
            launch(f)
        torch.cuda.synchronize()
        crmath.stats_reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            launch(f)
        e1.record(stream)
        torch.cuda.synchronize()
        st = crmath.stats_read()
        ms = e0.elapsed_time(e1) / steps
        gbs = bytes_per_elem(f) * n / (ms * 1e-3) / 1e9
        res[f] = {"ms": round(ms, 4), "gelem_s": round(n / (ms * 1e-3) / 1e9, 2),
                  "gb_s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                  "fallback_lane_rate": st["fallback_lanes"] / (n * steps),
                  "escapes": st["escapes"], "launch": list(crmath.tune_get(f, impl))}
    del bufs
    torch.cuda.empty_cache()
    log("bench: family", funcs[0], "...", {k: v and v["gelem_s"] for k, v in res.items()})
    return {"elems_per_function": n, "impl": "split_f32" if impl == 2 else "f64_internal",
            "per_func": res}


PAPER_GPU_FUNCS = ["expf", "logf", "sincosf", "exp", "log", "exp2"]


def bench_vs_ulp(torch, crmath, inputs, n, steps, warmup, stream):
    """The paper's GPU metric (Sec. III-C, Tables III, IV): correctly rounded
    throughput over the platform's ~1-ulp library functions (HIP's device math
    library, in a map kernel of the same launch shape), on the same inputs."""
    import ctypes
    path = os.path.join(ROOT, "paper_2605_15547_amd", "libcr_ulpref.so")
    if not os.path.exists(path):
        return None
    R = ctypes.CDLL(path)
    R.cr_ref_eval.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                              ctypes.c_void_p]
    sp = crmath._stream_ptr(stream)
    out = {}
    for f in PAPER_GPU_FUNCS:
        m = n >> 2 if f in F64 else n
        x = inputs.workload_f64(f, m) if f in F64 else inputs.workload_f32(f, m)
        xt = torch.from_numpy(x).cuda()
        ot = torch.empty(2 * m if f == "sincosf" else m, dtype=xt.dtype, device="cuda")
        fid = crmath.FUNC_ID[f]
        runs = {"cr": lambda: crmath.eval_ptr(f, xt.data_ptr(), ot.data_ptr(), m, 1, 0, sp),
                "ulp": lambda: R.cr_ref_eval(fid, xt.data_ptr(), ot.data_ptr(), m, sp)}
        settle(lambda: (runs["cr"](), runs["ulp"]()), 0.3, torch)
        rate = {}
        for k, fn in runs.items():
            for _ in range(warmup):
                fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            rate[k] = m / (e0.elapsed_time(e1) / steps * 1e-3) / 1e9
        out[f] = {"cr_gelem_s": round(rate["cr"], 2), "ulp_gelem_s": round(rate["ulp"], 2),
                  "ratio": round(rate["cr"] / rate["ulp"], 3)}
        del xt, ot
    torch.cuda.empty_cache()
    log("bench: vs 1-ulp library", out)
    return out


def bench_log_tables(torch, crmath, inputs, n, steps, warmup, stream):
    """binary64 log, the 16-entry build against the paper's 128-entry
    scaled-integer table (Sec. II-B), on the log workload and on the paper's
    range [0.125, 8] (Tables II, IV); the platform's ~1-ulp log on the same
    inputs for the paper's ratio."""
    import ctypes
    sp = crmath._stream_ptr(stream)
    st = inputs.Stream(4100)
    sets = {"workload": inputs.workload_f64("log", n),
            "uniform_0.125_8": (0.125 + 7.875 * st.uniform(n)).astype(np.float64)}
    ref = None
    path = os.path.join(ROOT, "paper_2605_15547_amd", "libcr_ulpref.so")
    if os.path.exists(path):
        ref = ctypes.CDLL(path)
        ref.cr_ref_eval.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_size_t, ctypes.c_void_p]
    out = {}
    for name, x in sets.items():
        xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
        ot = torch.empty_like(xt)
        runs = {"t16": lambda: crmath.eval_ptr("log", xt.data_ptr(), ot.data_ptr(), n, 1, 0, sp),
                "t128": lambda: crmath.eval_ptr("log", xt.data_ptr(), ot.data_ptr(), n,
                                                crmath.IMPL_LOG128, 0, sp)}
        if ref is not None:
            runs["ulp"] = lambda: ref.cr_ref_eval(65, xt.data_ptr(), ot.data_ptr(), n, sp)
        settle(lambda: [fn() for fn in runs.values()], 0.3, torch)
        r = {}
        for k, fn in runs.items():
            for _ in range(warmup):
                fn()
            torch.cuda.synchronize()
            crmath.stats_reset()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            s_ = crmath.stats_read()
            ms = e0.elapsed_time(e1) / steps
            r[k] = {"ms": round(ms, 4), "gelem_s": round(n / (ms * 1e-3) / 1e9, 2),
                    "hbm_frac": round(16 * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            if k != "ulp":
                r[k]["fallback_lane_rate"] = s_["fallback_lanes"] / (n * steps)
        if "ulp" in r:
            for k in ("t16", "t128"):
                r[k]["ratio_vs_ulp"] = round(r[k]["gelem_s"] / r["ulp"]["gelem_s"], 3)
        out[name] = r
        del xt, ot
    torch.cuda.empty_cache()
    log("bench: log tables", out)
    return {"elems": n, "t16": "16-entry reciprocal table, triple-double -ln c_j",
            "t128": "128-entry scaled-integer table (CR_IMPL_LOG128)", "per_input_set": out}


def bench_complex(torch, crmath, inputs, n, steps, warmup, stream):
    """The paper's complex expf/logf/sinf application (Sec. III-A): n complex
    numbers per function, parts uniform in [-40, 40]; 16 bytes per element."""
    sp = crmath._stream_ptr(stream)
    z = inputs.complex_workload(n)
    zt = torch.from_numpy(z).cuda()
    ot = torch.empty_like(zt)
    res = {}
    for f in crmath.COMPLEX:
        def run():
            crmath.eval_ptr(f, zt.data_ptr(), ot.data_ptr(), n, 0, 0, sp)
        settle(run, 0.2, torch)
        for _ in range(warmup):
            run()
        torch.cuda.synchronize()
        crmath.stats_reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        st = crmath.stats_read()
        ms = e0.elapsed_time(e1) / steps
        gbs = 16 * n / (ms * 1e-3) / 1e9
        res[f] = {"ms": round(ms, 4), "gelem_s": round(n / (ms * 1e-3) / 1e9, 2),
                  "gb_s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                  "fallback_lane_rate": st["fallback_lanes"] / (n * steps),
                  "escapes": st["escapes"]}
    del zt, ot
    torch.cuda.empty_cache()
    log("bench: complex", {k: v["gelem_s"] for k, v in res.items()})
    return {"elems_per_function": n, "unit": "10^9 complex numbers per second",
            "bytes_per_elem": 16, "inputs": "re, im uniform in [-40, 40]", "per_func": res}


def bench_dft(torch, crmath, inputs, n, m, steps, warmup, stream):
    """Spectral interpolation by brute-force DFT (Sec. III-A): m outputs of n
    samples each, one correctly rounded sincosf per (output, sample)."""
    x, w = inputs.dft_workload(n, m)
    xt, wt = torch.from_numpy(x).cuda(), torch.from_numpy(w).cuda()
    out = torch.empty((m, 2), dtype=torch.float64, device="cuda")
    sp = crmath._stream_ptr(stream)

    def run():
        crmath.dft_ptr(xt.data_ptr(), n, wt.data_ptr(), m, out.data_ptr(), 0, sp)
    settle(run, 0.3, torch)
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        run()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    r = {"samples": n, "outputs": m, "ms": round(ms, 4),
         "gsincos_s": round(n * m / (ms * 1e-3) / 1e9, 2),
         "what": "terms x[j] (cos t - i sin t), t = RN32(w_k j), per second; sincosf "
                 "correctly rounded, double-double sums"}
    log("bench: dft", r)
    return r


def bench_correctness_set(torch, crmath, inputs, steps, warmup, stream):
    """expf on its correctness set (64 specials and edges, then 2^20 values
    uniform in [-103.9, 88.7]), binary64-internal: 8.4 MB, about a
    microsecond of HBM time, so the launch dominates.  Per-launch events; the
    median launch is reported."""
    x = inputs.expf_correctness_set()
    xt = torch.from_numpy(x).cuda()
    out = torch.empty_like(xt)
    sp = crmath._stream_ptr(stream)
    n = x.size

    def run():
        crmath.eval_ptr("expf", xt.data_ptr(), out.data_ptr(), n, 1, 0, sp)

    settle(run, 0.2, torch)
    for _ in range(warmup):
        run()
    reps = max(steps, 20)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    torch.cuda.synchronize()
    for e0, e1 in evs:
        e0.record(stream)
        run()
        e1.record(stream)
    torch.cuda.synchronize()
    ms = sorted(e0.elapsed_time(e1) for e0, e1 in evs)[reps // 2]
    r = {"func": "expf", "impl": "f64_internal", "elements": int(n), "us_per_launch": round(ms * 1e3, 2),
         "gelem_s": round(n / (ms * 1e-3) / 1e9, 2),
         "hbm_frac": round(8 * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
         "note": "launch-bound (about 1 us of HBM time at 8 TB/s); not a roofline figure"}
    log("bench: correctness set", r)
    return r


def bench_batch(torch, crmath, inputs, steps, warmup, stream, impl=1):
    """The ragged batch: 4096 requests of mixed binary32 functions, lengths
    log-uniform in [1, 2^20], evaluated by one graph launch per step."""
    funcs, lens, seeds = inputs.batch_requests()
    bufs, reqs = [], []
    total, nbytes = 0, 0
    for f, n, sd in zip(funcs, lens, seeds):
        n = int(n)
        x = inputs.workload_f32(f, n, seed=int(sd) % (1 << 62))
        xt = torch.from_numpy(x).cuda()
        ot = torch.empty(2 * n if f == "sincosf" else n, dtype=torch.float32, device="cuda")
        bufs.append((xt, ot))
        reqs.append((f, xt.data_ptr(), ot.data_ptr(), n, impl))
        total += n
        nbytes += bytes_per_elem(f) * n
    t0 = time.perf_counter()
    plan = crmath.BatchPlan(reqs)
    create_s = time.perf_counter() - t0
    settle(lambda: plan.launch(stream), 0.3, torch)
    for _ in range(warmup):
        plan.launch(stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        plan.launch(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    plan.destroy()
    gbs = nbytes / (ms * 1e-3) / 1e9
    r = {"impl": "split_f32" if impl == 2 else "f64_internal",
         "requests": len(reqs), "elements": total, "ms": round(ms, 3),
         "gelem_s": round(total / (ms * 1e-3) / 1e9, 2), "gb_s": round(gbs, 1),
         "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "plan_create_s": round(create_s, 3),
         "blocks_per_cu": crmath.tune_batch_get(impl)}
    log("bench: batch", r)
    del bufs
    torch.cuda.empty_cache()
    return r


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """sha256 (first 16 hex digits) of the kernel sources csrc/cr_* with their
    comments removed and whitespace runs collapsed: a change of code
    invalidates the committed counter summaries, a change of comments or
    layout does not."""
    import glob
    import hashlib
    import re
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2605_15547_amd", "csrc", "cr_*"))):
        with open(f, encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())  # whitespace runs as one space
    return h.hexdigest()[:16]


def measured_traffic(func, n):
    """HBM bytes per launch of func's kernel from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE runs (calibrated against a plain copy), or None when
    the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_hash") != kernel_source_hash() or t.get("elems_per_launch") != n:
        return None
    return t["hbm_bytes_per_launch"].get(func)


def measured_valu(func, n):
    """VALU instructions per element of func's kernel from the committed
    rocprofv3 SQ_INSTS_VALU run, or None when the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", "valu.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_hash") != kernel_source_hash() or t.get("elems_per_launch") != n:
        return None
    return t["valu_per_elem"].get(func)


def measured_flops(func, n):
    """binary64 and binary32 floating-point operations per element of func's
    kernel from the committed per-type VALU counter run, or None when the
    kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", "flops.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_hash") != kernel_source_hash() or t.get("elems_per_launch") != n:
        return None
    return t["flops_per_elem"].get(func)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(funcs, host, gpu_head, seconds):
    """The oracle as it is, on a bounded sample: consecutive 2^14-element
    slices of each function's workload, round robin, for about `seconds` on
    every host thread; then one thread on 2^17 elements per function (2^20
    in all, about 1.2 million).  The multi-threaded results are compared bit for bit with
    the GPU's outputs of the timed step."""
    from oracle import oracle as O
    O.build()
    threads = O.default_threads()
    m, cnt, rounds = 1 << 14, 0, 0
    limit = min(v.size for v in gpu_head.values())
    ref = {f: [] for f in funcs}
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds and (rounds + 1) * m <= limit:
        for f in funcs:
            ref[f].append(O.evaluate(f, host[f][rounds * m:(rounds + 1) * m], threads))
            cnt += m
        rounds += 1
    dt = time.perf_counter() - t0
    compared, mismatches, first = 0, 0, None
    for f in funcs:
        if not ref[f]:
            continue
        r = np.concatenate(ref[f]).view(np.uint32)
        g = gpu_head[f][:r.size].view(np.uint32)
        bad = np.nonzero(r != g)[0]
        compared += r.size
        mismatches += int(bad.size)
        if bad.size and first is None:
            first = {"func": f, "index": int(bad[0]), "x": hex(int(host[f].view(np.uint32)[bad[0]])),
                     "gpu": hex(int(g[bad[0]])), "oracle": hex(int(r[bad[0]]))}
    m1 = 1 << 17
    t1 = time.perf_counter()
    for f in funcs:
        O.evaluate(f, host[f][:m1], 1)
    dt1 = time.perf_counter() - t1
    cpu = {"value": round(cnt / dt / 1e9, 6), "unit": "Gelem/s", "cores": threads,
           "kind": "oracle", "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
           "per_core_melem_s": round(cnt / dt / 1e6 / threads, 4),
           "one_thread": {"melem_s": round(m1 * len(funcs) / dt1 / 1e6, 4),
                          "elements": m1 * len(funcs), "seconds": round(dt1, 2)},
           "sample": "first %d inputs of each of the %d functions' workloads (%d elements, "
                     "%.1f s on %d threads); one thread: first 2^17 of each (%.1f s); Ziv "
                     "loop over fixed-point ball arithmetic"
                     % (rounds * m, len(funcs), cnt, dt, threads, dt1)}
    parity = {"against": "oracle", "compared": compared, "mismatches": mismatches,
              "first_mismatch": first,
              "what": "the cpu_baseline sample's oracle results vs the GPU outputs of the last "
                      "timed step, bit for bit"}
    return cpu, parity


def split_vs_f64(per, extra, n):
    """Throughput of the binary32-only implementation over the binary64-internal
    one, per family (harmonic: total elements over total time)."""
    out = {}
    pairs = [("exp_log_family", {"per_func": per}, extra.get("exp_log_family_split_f32")),
             ("trig_hyperbolic_family", extra.get("trig_hyperbolic_family"),
              extra.get("trig_hyperbolic_family_split_f32"))]
    for name, f64, spl in pairs:
        if not f64 or not spl:
            continue
        both = [f for f in f64["per_func"] if f64["per_func"].get(f) and spl["per_func"].get(f)]
        if not both:
            continue
        t_s = sum(spl["per_func"][f]["ms"] for f in both)
        t_d = sum(f64["per_func"][f]["ms"] for f in both)
        out[name] = {"functions": both,
                     "split_gelem_s": round(len(both) * n / (t_s * 1e-3) / 1e9, 2),
                     "f64_gelem_s": round(len(both) * n / (t_d * 1e-3) / 1e9, 2),
                     "ratio": round(t_d / t_s, 3)}
    b1, b2 = extra.get("ragged_batch"), extra.get("ragged_batch_split_f32")
    if b1 and b2:
        out["ragged_batch"] = {"split_gelem_s": b2["gelem_s"], "f64_gelem_s": b1["gelem_s"],
                               "ratio": round(b2["gelem_s"] / b1["gelem_s"], 3)}
    return out or None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=26, help="log2 of elements per function")
    ap.add_argument("--impl", type=int, default=1)
    ap.add_argument("--settle", type=float, default=1.0,
                    help="seconds of untimed steps before the warm-up (clock settling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--tuning", default=os.path.join(ROOT, "paper_2605_15547_amd", "tuning",
                                                      "mi355x.txt"),
                    help="launch configurations written by paper_2605_15547_amd/autotune.py")
    ap.add_argument("--no-tuning", action="store_true", help="library default configurations")
    ap.add_argument("--only", default=None,
                    help="comma-separated subset of the other workloads to measure: "
                         + ",".join(OTHER_LEGS) + " (default: all)")
    ap.add_argument("--headline-only", action="store_true",
                    help="measure only the exp/log-family step (profiling runs)")
    ap.add_argument("--copy-ref", action="store_true",
                    help="also time a plain copy of one input (profiler calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the method is an elementwise map with no "
              "exchange between GPUs, and this build runs on a single MI355X.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_15547_amd import crmath, inputs

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    crmath.lib()
    tuning = None
    if not a.no_tuning and os.path.exists(a.tuning):
        crmath.tune_load(a.tuning)
        tuning = os.path.relpath(a.tuning, ROOT)
    dev = torch.device("cuda:0")
    n = 1 << a.n
    funcs = [f for f in FAMILY if crmath.available(f, a.impl)]
    missing = [f for f in FAMILY if f not in funcs]
    log("bench: functions", funcs, "missing", missing, "n", n)

    xs, outs, host = {}, {}, {}
    for f in funcs:
        t0 = time.time()
        x = inputs.workload_f32(f, n)
        host[f] = x
        xs[f] = torch.from_numpy(x).to(dev)
        outs[f] = torch.empty_like(xs[f])
        log("bench: generated %s in %.1fs" % (f, time.time() - t0))
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    sp = crmath._stream_ptr(stream)

    def run(f):
        crmath.eval_ptr(f, xs[f].data_ptr(), outs[f].data_ptr(), n, a.impl, 0, sp)

    # let the clocks settle under this load before the warm-up steps (the first
    # ~100 ms of work run at lower clocks)
    # the shader clock is sampled once, half-way through, while the loop keeps
    # the GPU busy (the loop runs until the sample is in)
    import threading
    sclk = {"sclk_mhz": None, "when": "rocm-smi --showclocks during the settle launches"}
    sampler = threading.Thread(target=lambda: (time.sleep(min(0.5, a.settle / 2)),
                                               sample_sclk(sclk)), daemon=True)
    t_settle = time.perf_counter()
    if a.settle > 0:
        sampler.start()
    while time.perf_counter() - t_settle < a.settle or (a.settle > 0 and sampler.is_alive()
                                                       and time.perf_counter() - t_settle < 20):
        for f in funcs:
            run(f)
        torch.cuda.synchronize()
    for _ in range(a.warmup):
        for f in funcs:
            run(f)
    torch.cuda.synchronize()
    crmath.stats_reset()

    # per-function events on the launch stream
    ev = {f: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(a.steps)] for f in funcs}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(a.steps):
        for f in funcs:
            ev[f][s][0].record(stream)
            run(f)
            ev[f][s][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = crmath.stats_read()

    per = {}
    for f in funcs:
        ms = float(np.mean([b.elapsed_time(e) for b, e in ev[f]]))
        gbs = 8.0 * n / (ms * 1e-3) / 1e9
        per[f] = {"ms": round(ms, 4), "gelem_s": round(n / (ms * 1e-3) / 1e9, 2),
                  "gb_s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    total_elems = n * len(funcs) * a.steps
    value = total_elems / wall / 1e9
    dom = max(funcs, key=lambda f: per[f]["ms"])
    roof = {"bound": "hbm", "kernel": "k_map_f32<%s>" % dom,
            "achieved": per[dom]["gb_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(per[dom]["gb_s"] / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(dom, n),
            "bytes_per_elem": 8, "elems_per_launch": n}
    # the issue side of the same kernel: VALU instructions per element (from the
    # committed counter run) x elements per second against the issue rate of
    # one wave-level VALU instruction per CU per cycle (256 x 64 lanes x 2.4 GHz
    # = 39.3 T lane-instructions/s, the rate of the 78.6 TFLOP/s binary64 FMA
    # peak and half the packed binary32 peak of 157.3 TFLOP/s)
    vpe = measured_valu(dom, n)
    if vpe is not None:
        rate = vpe * n / (per[dom]["ms"] * 1e-3)
        roof["valu"] = {"instr_per_elem": vpe, "achieved_lane_instr_s": round(rate / 1e12, 2),
                        "peak_lane_instr_s": round(VALU_PEAK / 1e12, 2), "unit": "T/s",
                        "frac": round(rate / VALU_PEAK, 4)}
        # the same against the issue rate at the shader clock seen under this
        # load (sampled during the settle phase), when it was read
        if sclk.get("sclk_mhz"):
            at = 256 * 64 * sclk["sclk_mhz"] * 1e6
            roof["valu"]["frac_at_measured_clock"] = round(rate / at, 4)
            roof["valu"]["measured_clock_mhz"] = sclk["sclk_mhz"]
    else:
        roof["valu"] = None
    # the same kernel's floating-point rate against the vector peaks (binary64
    # 78.6, binary32 157.3 TFLOP/s), from the committed per-type counter run
    fl = measured_flops(dom, n)
    if fl is not None:
        eps = n / (per[dom]["ms"] * 1e-3)
        roof["flops"] = {"fp64_per_elem": fl["fp64_per_elem"],
                         "fp64_tflop_s": round(fl["fp64_per_elem"] * eps / 1e12, 2),
                         "fp64_peak": 78.6, "fp64_frac": round(fl["fp64_per_elem"] * eps / 78.6e12, 4),
                         "fp32_per_elem": fl["fp32_per_elem"],
                         "fp32_tflop_s": round(fl["fp32_per_elem"] * eps / 1e12, 2),
                         "fp32_peak": 157.3,
                         "fp32_frac": round(fl["fp32_per_elem"] * eps / 157.3e12, 4)}
    else:
        roof["flops"] = None

    # the leading outputs of the last timed step, for the check against the
    # oracle results the cpu_baseline leg computes
    check_n = min(n, 1 << 23)
    gpu_head = {f: outs[f][:check_n].cpu().numpy() for f in funcs}

    copy_ms = None
    if a.copy_ref:
        # a plain device-to-device copy of the same size: the reference used to
        # calibrate the HBM byte counters of the profiler (FETCH_SIZE/WRITE_SIZE)
        src, dst = xs[funcs[0]], outs[funcs[0]]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(a.steps):
            dst.copy_(src)
        e1.record(stream)
        torch.cuda.synchronize()
        copy_ms = e0.elapsed_time(e1) / a.steps

    extra = {}
    legs = set(OTHER_LEGS if a.only is None else a.only.split(","))
    if not a.headline_only:
        # free the headline buffers, then measure the other workloads
        del xs, outs
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        if "correctness" in legs:
            extra["expf_correctness_set"] = bench_correctness_set(torch, crmath, inputs, a.steps,
                                                                  a.warmup, stream)
        if "trig" in legs:
            extra["trig_hyperbolic_family"] = bench_family(
                torch, crmath, inputs, TRIG, n, a.impl, a.steps, a.warmup, stream)
        if "binary64" in legs:
            extra["binary64_exp_log"] = bench_family(
                torch, crmath, inputs, list(F64), 1 << 24, 0, a.steps, a.warmup, stream)
            extra["binary64_log_tables"] = bench_log_tables(torch, crmath, inputs, 1 << 24,
                                                            a.steps, a.warmup, stream)
        if "vsulp" in legs:
            extra["vs_ulp_library"] = bench_vs_ulp(torch, crmath, inputs, n, a.steps, a.warmup,
                                                   stream)
        if "complex" in legs:
            extra["complex_functions"] = bench_complex(torch, crmath, inputs, 1 << 24, a.steps,
                                                       a.warmup, stream)
        if "dft" in legs:
            extra["spectral_interpolation_dft"] = bench_dft(torch, crmath, inputs, 1 << 20, 256,
                                                            a.steps, a.warmup, stream)
        if "batch" in legs:
            extra["ragged_batch"] = bench_batch(torch, crmath, inputs, a.steps, a.warmup, stream)
            extra["ragged_batch_split_f32"] = bench_batch(torch, crmath, inputs, a.steps,
                                                          a.warmup, stream, impl=2)
        if "split" in legs:
            # the binary32-only (float-float) implementation beside the binary64-internal one
            extra["exp_log_family_split_f32"] = bench_family(
                torch, crmath, inputs, FAMILY, n, 2, a.steps, a.warmup, stream)
            extra["trig_hyperbolic_family_split_f32"] = bench_family(
                torch, crmath, inputs, TRIG, n, 2, a.steps, a.warmup, stream)

    cpu, parity = None, None
    if not a.no_cpu_baseline:
        cpu, parity = cpu_baseline(funcs, host, gpu_head, a.cpu_seconds)

    rec = {"metric": "correctly rounded Gelem/s (exp/log family, binary32), bit-exact",
           "value": round(value, 2), "unit": "Gelem/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": round(wall / a.steps * 1e3, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "exp/log family, 2^%d binary32 inputs per function" % a.n,
                      "functions": funcs, "missing": missing, "elems_per_function": n,
                      "impl": "f64_internal" if a.impl in (0, 1) else "split_f32",
                      "tuning": tuning,
                      "launch": {f: list(crmath.tune_get(f, a.impl)) for f in funcs}},
           "per_func": per,
           "fallback": {"lanes": st["fallback_lanes"], "waves": st["fallback_waves"],
                        "escapes": st["escapes"],
                        "lane_rate": st["fallback_lanes"] / max(1, total_elems)},
           "roofline": roof, "cpu_baseline": cpu, "parity_vs_oracle": parity,
           "other_workloads": extra}
    rec["split_f32_vs_f64"] = split_vs_f64(per, extra, n)
    rec["clock_under_load"] = sclk
    if copy_ms is not None:
        rec["copy_ref"] = {"ms": round(copy_ms, 4), "bytes": 8 * n,
                           "gb_s": round(8 * n / (copy_ms * 1e-3) / 1e9, 1)}
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
