"""Summarise rocprofv3 SQLite output (kernel-trace stats, or one PMC counter per
dispatch) into a short text table, or turn a FETCH_SIZE and a WRITE_SIZE run of
the same workload into HBM bytes per launch.  Usage:
  python -m paper_2605_15547_amd.rocpd_summary stats   <results.db>
  python -m paper_2605_15547_amd.rocpd_summary counter <results.db>
  python -m paper_2605_15547_amd.rocpd_summary traffic <fetch.db> <write.db> <copy_bytes>
         <elems_per_launch> <source_hash>
  python -m paper_2605_15547_amd.rocpd_summary valu <valu.db> <elems_per_launch> <source_hash>
  python -m paper_2605_15547_amd.rocpd_summary valu_table <counter.txt> <stats.txt>
  python -m paper_2605_15547_amd.rocpd_summary flops_table <counter.txt>... <stats.txt>...
  python -m paper_2605_15547_amd.rocpd_summary flops_json <counter.txt> <elems_per_launch> <source_hash>
traffic calibrates both counters on the largest dispatch of the runtime's
plain copy kernel (copy_bytes read and written) and prints the text summary,
then one JSON line (the content of profiles/traffic.json).  valu reads a run
with SQ_INSTS_VALU and GRBM_GUI_ACTIVE and prints, per map kernel of
elems_per_launch elements, VALU instructions per element and the fraction of
the issue rate used (a CU issues one wave-level VALU instruction per cycle;
GRBM_GUI_ACTIVE sums the 8 XCDs' busy cycles), then one JSON line (the
content of profiles/valu.json).  valu_table turns the text printed by
"counter" for a SQ_INSTS_VALU + GRBM_GUI_ACTIVE run of bench.py's other
workloads, and the text printed by "stats" for a kernel trace of the same
workloads, into VALU instructions per element, issue-rate fraction and average
duration per kernel; elements per dispatch follow bench.py's workloads (2^26
binary32 map elements, 2^24 binary64 and complex, 2^20 samples x 256 outputs
for the DFT, each function's share of the 4096-request batch for the batch
kernels).  flops_table does the same for runs of the per-type VALU counters
(SQ_INSTS_VALU_{FMA,ADD,MUL,TRANS}_{F32,F64}, _INT32, _INT64, _CVT): the
instruction mix per element and the binary64 and binary32 floating-point rates
(an FMA counts two operations, every lane of a wave-level instruction one)
against MI355X's vector peaks, 78.6 TFLOP/s binary64 and 157.3 TFLOP/s binary32.
flops_json prints, per map kernel of elems_per_launch elements, the binary64
and binary32 floating-point operations per element (the content of
profiles/flops.json, read by bench.py for the headline's roofline).
"""
import json
import os
import re
import sqlite3
import sys
from collections import defaultdict


FUNCS = {"OpExp<0>": "expf", "OpExp<1>": "exp2f", "OpExp<2>": "exp10f", "OpExp<3>": "expm1f",
         "OpLog<0>": "logf", "OpLog<1>": "log2f", "OpLog<2>": "log10f", "OpLog<3>": "log1pf",
         "OpRsqrt": "rsqrtf", "OpTrig<0>": "sinf", "OpTrig<1>": "cosf", "OpTrig<2>": "tanf",
         "SinCosF64": "sincosf", "OpAtan<0>": "atanf", "OpAtan<1>": "asinf",
         "OpAtan<2>": "acosf", "OpHyp<0>": "sinhf", "OpHyp<1>": "coshf", "OpHyp<2>": "tanhf",
         "OpExp64": "exp", "OpLog64": "log", "OpExp2_64": "exp2", "CExpF": "cexpf",
         "CLogF": "clogf", "CSinF": "csinf"}
for _k in list(FUNCS):
    if _k.startswith("Op") and not _k.endswith("64") and _k[2:3] != "S":
        FUNCS["OpS" + _k[2:]] = FUNCS[_k] + " split"
FUNCS["SinCosSplit"] = "sincosf split"
FUNCS["OpLog128"] = "log, 128-entry table"
# the platform's ~1-ulp functions timed for the paper's ratio (libcr_ulpref.so)
REF_IDS = {"0": "HIP expf", "4": "HIP logf", "11": "HIP sincosf", "64": "HIP exp", "65": "HIP log",
           "66": "HIP exp2"}


def short(name):
    """k_map_f32<OpLog<3>> (log1pf) style names for the library's kernels."""
    name = name.replace("(anonymous namespace)::", "")
    m = re.match(r"void (k_\w+)<(\w+(?:<\d+>)?)[ ,>]", name)
    if m:
        op = m.group(2)
        what = REF_IDS.get(op, "?") if m.group(1).startswith("k_ref") else FUNCS.get(op, "?")
        return "%s<%s> (%s)" % (m.group(1), op, what)
    return name.split("(")[0][:60]


def stats(db):
    rows = db.execute("select name, duration from kernels").fetchall()
    agg = defaultdict(list)
    for n, d in rows:
        agg[short(n)].append(d)
    print("%-44s %6s %12s %10s %10s %10s" % ("kernel", "calls", "total_ns", "avg_ns", "min_ns",
                                             "max_ns"))
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        print("%-44s %6d %12d %10.0f %10d %10d" % (k, len(v), sum(v), sum(v) / len(v), min(v),
                                                    max(v)))


def counter(db):
    cols = [r[1] for r in db.execute("pragma table_info(counters_collection)")]
    q = "select * from counters_collection"
    agg = defaultdict(list)
    for r in db.execute(q):
        d = dict(zip(cols, r))
        agg[(short(d.get("kernel_name", "?")), d.get("counter_name"))].append(d.get("value"))
    print("%-44s %-20s %6s %16s" % ("kernel", "counter", "calls", "avg_per_dispatch"))
    for (k, c), v in sorted(agg.items()):
        print("%-44s %-20s %6d %16.1f" % (k, c, len(v), sum(v) / len(v)))


def per_dispatch(db):
    """{kernel name: [value per dispatch]} of a one-counter run, in KiB"""
    cols = [r[1] for r in db.execute("pragma table_info(counters_collection)")]
    agg = defaultdict(list)
    for r in db.execute("select * from counters_collection"):
        d = dict(zip(cols, r))
        agg[d.get("kernel_name", "?")].append(d.get("value"))
    return agg


def traffic(fetch_db, write_db, copy_bytes, elems, source_hash):
    f, w = per_dispatch(fetch_db), per_dispatch(write_db)
    copy = [k for k in f if "copyBuffer" in k]
    if not copy:
        raise SystemExit("no copy kernel in the fetch run")
    kib = copy_bytes / 1024.0
    fscale = kib / max(max(f[k]) for k in copy)
    wscale = kib / max(max(w[k]) for k in copy if k in w)
    print("calibration: the largest plain-copy dispatch moves %d bytes each way" % copy_bytes)
    print("  FETCH_SIZE scale %.3f, WRITE_SIZE scale %.3f" % (fscale, wscale))
    algo = 8.0 * elems / 1024.0
    out = {}
    print("per launch (%d elements, algorithmic 8 B per element = %.0f KiB):" % (elems, algo))
    for k in sorted(f):
        m = re.search(r"k_map_f32<(?:\(anonymous namespace\)::)?(\w+(?:<\d+>)?)", k)
        if not m or m.group(1) not in FUNCS or k not in w:
            continue
        fk = sum(f[k]) / len(f[k])
        wk = sum(w[k]) / len(w[k])
        tot = fk * fscale + wk * wscale
        name = FUNCS[m.group(1)]
        out[name] = int(round(tot * 1024))
        print("  %-14s %.3f x %.1f + %.3f x %.1f = %.1f KiB (%.4f x algorithmic)"
              % (name, fscale, fk, wscale, wk, tot, tot / algo))
    print(json.dumps({"source_hash": source_hash, "elems_per_launch": elems,
                      "fetch_scale": round(fscale, 4), "write_scale": round(wscale, 4),
                      "hbm_bytes_per_launch": out}))


def valu(db, elems, source_hash):
    cols = [r[1] for r in db.execute("pragma table_info(counters_collection)")]
    per = defaultdict(lambda: defaultdict(list))
    for r in db.execute("select * from counters_collection"):
        d = dict(zip(cols, r))
        per[d.get("kernel_name", "?")][d.get("counter_name")].append(d.get("value"))
    out = {}
    print("%-40s %10s %12s" % ("kernel (%d elements per dispatch)" % elems, "VALU/elem",
                               "issue_util"))
    for k in sorted(per):
        m = re.search(r"k_map_f32<(?:\(anonymous namespace\)::)?(\w+(?:<\d+>)?)", k)
        c = per[k]
        if not m or m.group(1) not in FUNCS or "SQ_INSTS_VALU" not in c:
            continue
        insts = sum(c["SQ_INSTS_VALU"]) / len(c["SQ_INSTS_VALU"])
        vpe = insts * 64.0 / elems
        util = None
        if "GRBM_GUI_ACTIVE" in c:
            cyc = sum(c["GRBM_GUI_ACTIVE"]) / len(c["GRBM_GUI_ACTIVE"]) / 8.0
            util = insts / (256.0 * cyc)
        name = FUNCS[m.group(1)]
        out[name] = round(vpe, 2)
        print("%-40s %10.1f %12s" % ("k_map_f32<%s> (%s)" % (m.group(1), name), vpe,
                                     "-" if util is None else "%.1f%%" % (100 * util)))
    print(json.dumps({"source_hash": source_hash, "elems_per_launch": elems,
                      "valu_per_elem": out}))


def _parse_rows(path, ncols):
    """(kernel, [last ncols fields]) of a text table printed above"""
    rows = []
    for line in open(path):
        f = line.split()
        if len(f) < ncols + 1 or f[0] == "kernel":
            continue
        try:
            vals = [float(v) for v in f[-ncols:]]
        except ValueError:
            continue
        rows.append((line[:line.rfind(f[-ncols])].split("  ")[0].strip(), vals, f))
    return rows


def _batch_elems():
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from paper_2605_15547_amd import inputs
    funcs, lens, _ = inputs.batch_requests()
    tot = defaultdict(int)
    for f, n in zip(funcs, lens):
        tot[f] += int(n)
    return tot


def elems_of(kernel, batch):
    """elements per dispatch of bench.py's workloads, by kernel"""
    m = re.match(r"(k_\w+)(?:<\S+>)? \((.+)\)$", kernel)
    if not m:
        return 268435456 if kernel == "k_dft" else None
    k, what = m.group(1), m.group(2)
    if k in ("k_map_f32", "k_map_sincos", "k_ref32"):
        return 1 << 26
    if k in ("k_map_f64", "k_complex", "k_ref64"):
        return 1 << 24
    if k in ("k_tiles", "k_tiles_sincos"):
        return batch.get(what.split()[0])
    return None


def valu_table(counter_txt, stats_txt):
    batch = _batch_elems()
    cnt = defaultdict(dict)
    for line in open(counter_txt):
        m = re.match(r"(.+?)\s+(SQ_\w+|GRBM_\w+)\s+(\d+)\s+([\d.]+)\s*$", line)
        if m:
            cnt[m.group(1).strip()][m.group(2)] = float(m.group(4))
    ns = {}
    for line in open(stats_txt):
        m = re.match(r"(.+?)\s+(\d+)\s+(\d+)\s+([\d.]+)\s+(\d+)\s+(\d+)\s*$", line)
        if m:
            ns[m.group(1).strip()] = float(m.group(4))
    print("%-46s %10s %10s %11s %10s" % ("kernel", "elements", "VALU/elem", "issue_util",
                                         "avg_ns"))
    for k in sorted(cnt):
        c = cnt[k]
        n = elems_of(k, batch)
        if not n or "SQ_INSTS_VALU" not in c:
            continue
        vpe = c["SQ_INSTS_VALU"] * 64.0 / n
        util = c["SQ_INSTS_VALU"] / (256.0 * c["GRBM_GUI_ACTIVE"] / 8.0) \
            if c.get("GRBM_GUI_ACTIVE") else None
        print("%-46s %10d %10.1f %11s %10s" % (k, n, vpe,
                                               "-" if util is None else "%.1f%%" % (100 * util),
                                               "%.0f" % ns[k] if k in ns else "-"))


def _load_counters(paths):
    cnt = defaultdict(dict)
    for path in paths:
        for line in open(path):
            m = re.match(r"(.+?)\s+(SQ_\w+|GRBM_\w+)\s+(\d+)\s+([\d.]+)\s*$", line)
            if m:
                cnt[m.group(1).strip()][m.group(2)] = float(m.group(4))
    return cnt


def _load_ns(paths):
    ns = {}
    for path in paths:
        for line in open(path):
            m = re.match(r"(.+?)\s+(\d+)\s+(\d+)\s+([\d.]+)\s+(\d+)\s+(\d+)\s*$", line)
            if m:
                ns[m.group(1).strip()] = float(m.group(4))
    return ns


FP64_PEAK, FP32_PEAK = 78.6, 157.3  # TFLOP/s, MI355X vector (non-matrix) peaks


def flops_table(counter_txts, stats_txts):
    batch = _batch_elems()
    cnt, ns = _load_counters(counter_txts), _load_ns(stats_txts)
    types = ["FMA_F64", "ADD_F64", "MUL_F64", "TRANS_F64", "FMA_F32", "ADD_F32", "MUL_F32",
             "TRANS_F32", "INT32", "INT64", "CVT"]
    print("instructions per element by type (wave-level counts x 64 / elements), and the")
    print("floating-point rates: TF64 = (2 FMA_F64 + ADD_F64 + MUL_F64) x 64 lanes / avg_ns,")
    print("TF32 likewise for binary32, against %.1f and %.1f TFLOP/s" % (FP64_PEAK, FP32_PEAK))
    print("%-40s" % "kernel" + "".join("%8s" % t.replace("_F", ".") for t in types)
          + "%8s %6s %8s %6s" % ("TF64", "%pk", "TF32", "%pk"))
    for k in sorted(cnt):
        c = cnt[k]
        n = elems_of(k, batch)
        if not n or "SQ_INSTS_VALU_FMA_F64" not in c:
            continue
        per = {t: c.get("SQ_INSTS_VALU_" + t, 0.0) * 64.0 / n for t in types}
        row = "%-40s" % k[:40] + "".join("%8.1f" % per[t] for t in types)
        if k in ns:
            f64 = (2 * per["FMA_F64"] + per["ADD_F64"] + per["MUL_F64"]) * n / ns[k] / 1e3
            f32 = (2 * per["FMA_F32"] + per["ADD_F32"] + per["MUL_F32"]) * n / ns[k] / 1e3
            row += "%8.2f %5.1f%% %8.2f %5.1f%%" % (f64, 100 * f64 / FP64_PEAK, f32,
                                                    100 * f32 / FP32_PEAK)
        print(row)


def flops_json(counter_txt, elems, source_hash):
    cnt = _load_counters([counter_txt])
    out = {}
    for k, c in cnt.items():
        m = re.search(r"k_map_f32<(\w+(?:<\d+>)?)>", k)
        if not m or m.group(1) not in FUNCS or "SQ_INSTS_VALU_FMA_F64" not in c:
            continue
        g = lambda t: c.get("SQ_INSTS_VALU_" + t, 0.0) * 64.0 / elems
        out[FUNCS[m.group(1)]] = {
            "fp64_per_elem": round(2 * g("FMA_F64") + g("ADD_F64") + g("MUL_F64"), 3),
            "fp32_per_elem": round(2 * g("FMA_F32") + g("ADD_F32") + g("MUL_F32"), 3)}
    print(json.dumps({"source_hash": source_hash, "elems_per_launch": elems,
                      "flops_per_elem": out}))


if __name__ == "__main__":
    mode, path = sys.argv[1], sys.argv[2]
    if mode == "flops_json":
        flops_json(path, int(sys.argv[3]), sys.argv[4])
    elif mode == "flops_table":
        args = sys.argv[2:]
        flops_table([a for a in args if "stats" not in os.path.basename(a)],
                    [a for a in args if "stats" in os.path.basename(a)])
    elif mode == "valu_table":
        valu_table(path, sys.argv[3])
    elif mode == "valu":
        valu(sqlite3.connect(path), int(sys.argv[3]), sys.argv[4])
    elif mode == "traffic":
        traffic(sqlite3.connect(path), sqlite3.connect(sys.argv[3]), int(sys.argv[4]),
                int(sys.argv[5]), sys.argv[6])
    else:
        db = sqlite3.connect(path)
        stats(db) if mode == "stats" else counter(db)
