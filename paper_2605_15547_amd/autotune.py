"""Tune the launch configuration of every function on this GPU and write the
tuning file the benchmark loads (paper_2605_15547_amd/tuning/mi355x.txt).

For each function and implementation the library's autotuner (cr_autotune)
times every kernel variant x grid size on that function's synthetic workload
(the benchmark's inputs, resident in device memory) and keeps the fastest.
Usage:  python -m paper_2605_15547_amd.autotune [--out PATH] [--log2n 26]
                                               [--funcs f1,f2 [--impls f64,split]]
With --funcs only the listed functions (and implementations) are retuned; the
other entries are kept from the file at --out.  The grid of the batch kernels
(workgroups per CU) is tuned last, on the 4096-request batch workload, unless
--funcs is given without "batch".
"""
import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tuning", "mi355x.txt")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--log2n", type=int, default=26)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--funcs", default=None, help="comma-separated subset to retune")
    ap.add_argument("--impls", default="f64,split", help="implementations to retune")
    a = ap.parse_args()
    import torch
    from paper_2605_15547_amd import crmath, inputs
    F64 = crmath.FUNCS64
    if not torch.cuda.is_available():
        raise SystemExit("autotune needs a GPU")
    crmath.tune_reset()
    sp = crmath._stream_ptr(None)
    funcs = crmath.FUNCS32 + F64
    if a.funcs:
        if os.path.exists(a.out):
            crmath.tune_load(a.out)
        funcs = [f for f in funcs if f in a.funcs.split(",")]
    impls = [i for i, nm in ((crmath.IMPL_F64_INTERNAL, "f64"), (crmath.IMPL_SPLIT_F32, "split"))
             if nm in a.impls.split(",")]
    for f in funcs:
        n = 1 << (a.log2n - 2 if f in F64 else a.log2n)
        x = inputs.workload_f64(f, n) if f in F64 else inputs.workload_f32(f, n)
        xt = torch.from_numpy(x).cuda()
        out = torch.empty(2 * n if f == "sincosf" else n, dtype=xt.dtype, device="cuda")
        for impl in impls:
            if not crmath.available(f, impl):
                continue
            t0 = time.time()
            rate = crmath.autotune(f, impl, xt.data_ptr(), out.data_ptr(), n, a.reps, sp)
            v, b = crmath.tune_get(f, impl)
            print("%-8s %-5s variant %d  %2d WG/CU  %7.1f Gelem/s  (%.1f s)"
                  % (f, "split" if impl == 2 else "f64", v, b, rate, time.time() - t0), flush=True)
        del xt, out
        torch.cuda.empty_cache()
    if not a.funcs or "batch" in a.funcs.split(","):
        tune_batch(torch, crmath, inputs, impls, a.reps)
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    crmath.tune_save(a.out)
    print("wrote", a.out, flush=True)


def tune_batch(torch, crmath, inputs, impls, reps, bpcs=(1, 2, 4, 8, 16), passes=3):
    """Workgroups per CU of the batch kernels: every candidate timed on the
    4096-request batch (one plan per candidate, reps graph launches after one
    untimed), three interleaved passes, each candidate's median pass kept."""
    funcs, lens, seeds = inputs.batch_requests()
    bufs = []
    for f, n, sd in zip(funcs, lens, seeds):
        n = int(n)
        xt = torch.from_numpy(inputs.workload_f32(f, n, seed=int(sd) % (1 << 62))).cuda()
        ot = torch.empty(2 * n if f == "sincosf" else n, dtype=torch.float32, device="cuda")
        bufs.append((f, n, xt, ot))
    total = sum(n for _, n, _, _ in bufs)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for impl in impls:
        t0 = time.time()
        reqs = [(f, xt.data_ptr(), ot.data_ptr(), n, impl) for f, n, xt, ot in bufs]
        times = {b: [] for b in bpcs}
        for p in range(passes):
            for b in bpcs:
                crmath.tune_batch_set(impl, b)
                plan = crmath.BatchPlan(reqs)
                for _ in range(3 if p == 0 else 1):  # the first pass also settles the clocks
                    plan.launch(stream)
                e0.record(stream)
                for _ in range(reps):
                    plan.launch(stream)
                e1.record(stream)
                torch.cuda.synchronize()
                times[b].append(e0.elapsed_time(e1) / reps)
                plan.destroy()
        med = {b: sorted(v)[len(v) // 2] for b, v in times.items()}
        best = min(med, key=med.get)
        crmath.tune_batch_set(impl, best)
        print("%-8s %-5s %2d WG/CU per kernel  %7.1f Gelem/s  (%s; %.1f s)"
              % ("batch", "split" if impl == crmath.IMPL_SPLIT_F32 else "f64", best,
                 total / (med[best] * 1e-3) / 1e9,
                 ", ".join("%d: %.1f" % (b, total / (med[b] * 1e-3) / 1e9) for b in bpcs),
                 time.time() - t0), flush=True)
    del bufs
    torch.cuda.empty_cache()


if __name__ == "__main__":
    sys.exit(main())
