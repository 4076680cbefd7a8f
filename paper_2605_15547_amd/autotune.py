"""Tune the launch configuration of every function on this GPU and write the
tuning file the benchmark loads (paper_2605_15547_amd/tuning/mi355x.txt).

For each function and implementation the library's autotuner (cr_autotune)
times every kernel variant x grid size on that function's synthetic workload
(the benchmark's inputs, resident in device memory) and keeps the fastest.
Usage:  python -m paper_2605_15547_amd.autotune [--out PATH] [--log2n 26]
                                               [--funcs f1,f2 [--impls f64,split]]
With --funcs only the listed functions (and implementations) are retuned; the
other entries are kept from the file at --out.
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
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    crmath.tune_save(a.out)
    print("wrote", a.out, flush=True)


if __name__ == "__main__":
    sys.exit(main())
