"""Every full-size workload, and all 2^32 binary32 encodings of expf, logf and
sinf, against the oracle (needs a GPU).

The oracle's results are stored as digests of 2^20-element blocks
(tests/golden/digests/, written by tests/golden/make_digests.py from the
oracle alone).  Each test evaluates the same seeded inputs on the GPU in the
launch configuration the benchmark uses, digests the output blocks the same
way and compares every block, for both implementations of the binary32
functions.  Where a block differs, that block alone is evaluated with the
oracle and the first differing element is reported.  (Paper, Sec. II-A: the
binary32 functions are validated by exhaustive testing against an
independent reference.)
"""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_digests as MD  # noqa: E402

from paper_2605_15547_amd import crmath, inputs  # noqa: E402

F64 = crmath.FUNCS64

DIG = os.path.join(HERE, "golden", "digests")
IMPLS = [("f64", crmath.IMPL_F64_INTERNAL), ("split", crmath.IMPL_SPLIT_F32)]
TUNING = os.path.join(os.path.dirname(HERE), "paper_2605_15547_amd", "tuning", "mi355x.txt")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module", autouse=True)
def _tuned():
    """The launch configurations the benchmark times."""
    if torch.cuda.is_available() and os.path.exists(TUNING):
        crmath.tune_load(TUNING)
    yield
    if torch.cuda.is_available():
        crmath.tune_reset()


def _load(name):
    path = os.path.join(DIG, name + ".json")
    if not os.path.exists(path):
        pytest.skip("digest %s not generated" % name)
    with open(path) as f:
        return json.load(f)


def _gpu_eval(func, xt, impl):
    n = xt.numel()
    dt = torch.float64 if func in F64 else torch.float32
    out = torch.empty(2 * n if func == "sincosf" else n, dtype=dt, device="cuda")
    crmath.eval_ptr(func, xt.data_ptr(), out.data_ptr(), n, impl, 0, crmath._stream_ptr(None))
    return out


def _host(func, out):
    y = out.cpu().numpy()
    return y.reshape(2, -1) if func == "sincosf" else y


def _explain(func, x, y, blocks, block=MD.BLOCK):
    """First differing element of the first differing block, by the oracle."""
    from oracle import oracle as O
    b = blocks[0]
    xs = x[b * block:(b + 1) * block]
    ref = O.evaluate(func, xs)
    got = y[:, b * block:(b + 1) * block] if func == "sincosf" else y[b * block:(b + 1) * block]
    ib = np.uint64 if func in F64 else np.uint32
    gb, rb = np.asarray(got).view(ib).ravel(), np.asarray(ref).view(ib).ravel()
    bad = np.nonzero(gb != rb)[0]
    if not bad.size:
        return "block %d: digest differs but the oracle agrees element-wise" % b
    i = bad[0] % xs.size
    return ("%d blocks differ (first %s); block %d has %d mismatches, first x=0x%x gpu=0x%x "
            "oracle=0x%x" % (len(blocks), blocks[:8], b, bad.size, int(xs.view(ib)[i]),
                             int(gb[bad[0]]), int(rb[bad[0]])))


def _check_array(name, func, x, impl):
    doc = _load(name)
    assert MD.input_digest(x) == doc["input_xxh3_128"], \
        "%s: the input generator no longer reproduces the stored inputs" % name
    crmath.stats_reset()
    y = _host(func, _gpu_eval(func, torch.from_numpy(x).cuda(), impl))
    torch.cuda.synchronize()
    st = crmath.stats_read()
    got = MD.block_digests(func, y)
    bad = [i for i, (g, r) in enumerate(zip(got, doc["digests"])) if g != r]
    assert len(got) == len(doc["digests"])
    assert not bad, "%s: %s" % (name, _explain(func, x, y, bad))
    assert st["escapes"] == 0, st


@pytest.mark.parametrize("impl", IMPLS, ids=[i[0] for i in IMPLS])
def test_expf_correctness_set_digest(impl):
    _need_gpu()
    _check_array("expf_correctness", "expf", inputs.expf_correctness_set(), impl[1])


@pytest.mark.parametrize("impl", IMPLS, ids=[i[0] for i in IMPLS])
@pytest.mark.parametrize("func", inputs.EXPLOG_FAMILY)
def test_explog_family_2p26_digest(func, impl):
    _need_gpu()
    _check_array("explog_2p26." + func, func, inputs.workload_f32(func, 1 << 26), impl[1])


@pytest.mark.parametrize("impl", IMPLS, ids=[i[0] for i in IMPLS])
@pytest.mark.parametrize("func", inputs.TRIG_FAMILY)
def test_trig_family_2p26_digest(func, impl):
    _need_gpu()
    _check_array("trig_2p26." + func, func, inputs.workload_f32(func, 1 << 26), impl[1])


@pytest.mark.parametrize("func,impl", [(f, crmath.IMPL_AUTO) for f in F64]
                         + [("log", crmath.IMPL_LOG128)], ids=list(F64) + ["log-t128"])
def test_binary64_2p24_digest(func, impl):
    _need_gpu()
    _check_array("binary64_2p24." + func, func, inputs.workload_f64(func, 1 << 24), impl)


@pytest.fixture(scope="module")
def batch_inputs():
    doc = _load("batch_4096")
    funcs, lens, seeds = inputs.batch_requests()
    xs = [inputs.workload_f32(f, int(n), seed=int(sd) % (1 << 62))
          for f, n, sd in zip(funcs, lens, seeds)]
    return doc, list(funcs), xs


@pytest.mark.parametrize("impl", IMPLS, ids=[i[0] for i in IMPLS])
def test_batch_4096_digest(batch_inputs, impl):
    """The 4096-request ragged batch as one plan (graph) launch, every request
    compared with its oracle digest."""
    _need_gpu()
    doc, funcs, xs = batch_inputs
    assert [MD.input_digest(x) for x in xs] == doc["input_xxh3_128"]
    ins, outs, reqs = [], [], []
    for f, x in zip(funcs, xs):
        n = x.size
        xin = torch.from_numpy(x).cuda() if n else torch.empty(1, device="cuda")
        out = torch.empty(max(1, 2 * n if f == "sincosf" else n), device="cuda")
        ins.append(xin)
        outs.append(out)
        reqs.append((f, xin.data_ptr(), out.data_ptr(), n, impl[1]))
    crmath.stats_reset()
    plan = crmath.BatchPlan(reqs)
    plan.launch()
    torch.cuda.synchronize()
    plan.destroy()
    st = crmath.stats_read()
    bad = []
    for k, (f, x, out) in enumerate(zip(funcs, xs, outs)):
        if x.size == 0:
            assert doc["digests"][k] is None
            continue
        y = _host(f, out[:2 * x.size if f == "sincosf" else x.size])
        if MD.block_digests(f, y, block=1 << 21)[0] != doc["digests"][k]:
            bad.append(k)
    if bad:
        k = bad[0]
        f = funcs[k]
        y = _host(f, outs[k][:2 * xs[k].size if f == "sincosf" else xs[k].size])
        raise AssertionError("%d requests differ; request %d (%s, n=%d): %s"
                             % (len(bad), k, f, xs[k].size,
                                _explain(f, xs[k], y, [0], block=1 << 21)))
    assert st["escapes"] == 0, st


EXH_CHUNK = 1 << 28


@pytest.mark.parametrize("impl", IMPLS, ids=[i[0] for i in IMPLS])
@pytest.mark.parametrize("func", list(MD.SWEEP_FUNCS))
def test_exhaustive_2p32_digest(func, impl):
    """All 2^32 encodings, in 2^28-element launches, against the oracle."""
    _need_gpu()
    doc = _load("exhaustive." + func)
    per = EXH_CHUNK // MD.BLOCK
    crmath.stats_reset()
    bad = []
    for c in range((1 << 32) // EXH_CHUNK):
        xi = torch.arange(c * EXH_CHUNK, (c + 1) * EXH_CHUNK, dtype=torch.int64, device="cuda")
        xt = xi.to(torch.int32).view(torch.float32)
        del xi
        y = _host(func, _gpu_eval(func, xt, impl[1]))
        del xt
        got = MD.block_digests(func, y)
        ref = doc["digests"][c * per:(c + 1) * per]
        bad += [c * per + i for i, (g, r) in enumerate(zip(got, ref)) if g != r]
        if bad:
            b = bad[0] - c * per
            x = (np.arange(c * EXH_CHUNK, (c + 1) * EXH_CHUNK, dtype=np.uint64)
                 .astype(np.uint32).view(np.float32))
            raise AssertionError("exhaustive %s chunk %d: %s"
                                 % (func, c, _explain(func, x, y, [b])))
    torch.cuda.synchronize()
    assert crmath.stats_read()["escapes"] == 0
