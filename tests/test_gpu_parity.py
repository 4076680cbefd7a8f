"""Bit-exact parity of the HIP library against the CPU oracle (needs a GPU).

Inputs are the seeded synthetic workloads of paper_2605_15547_amd/inputs.py.
Correct rounding to nearest has exactly one right answer per input, so every
comparison is on the bit pattern of the result (NaN encodings included).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2605_15547_amd import crmath, inputs  # noqa: E402

F64 = crmath.FUNCS64

F32 = crmath.FUNCS32


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def built(func, impl=crmath.IMPL_AUTO):
    return crmath.available(func, impl)


def gpu_eval(func, x, impl=crmath.IMPL_AUTO, flags=0, offset_in=0, offset_out=0):
    """Run func on the GPU; offsets shift the device pointers by whole elements
    to exercise unaligned heads."""
    dt = torch.float64 if func in F64 else torch.float32
    n = x.size
    nout = 2 * n if func == "sincosf" else n
    xin = torch.empty(n + offset_in, dtype=dt, device="cuda")
    xin[offset_in:] = torch.from_numpy(np.ascontiguousarray(x))
    out = torch.full((nout + offset_out,), -7.0, dtype=dt, device="cuda")
    crmath.eval_ptr(func, xin[offset_in:].data_ptr(), out[offset_out:].data_ptr(), n, impl,
                    flags, crmath._stream_ptr(None))
    torch.cuda.synchronize()
    r = out[offset_out:].cpu().numpy()
    if offset_out:
        assert np.all(out[:offset_out].cpu().numpy() == -7.0), "wrote before the output range"
    return r.reshape(2, n) if func == "sincosf" else r


def bits(a):
    a = np.asarray(a)
    return a.view(np.uint64 if a.dtype == np.float64 else np.uint32)


def assert_same(func, x, got, ref):
    gb, rb = bits(got).ravel(), bits(ref).ravel()
    bad = np.nonzero(gb != rb)[0]
    if bad.size:
        i = bad[0] % x.size
        raise AssertionError("%s: %d mismatches; first at %d: x=%r (0x%x) gpu=0x%x oracle=0x%x"
                             % (func, bad.size, i, x[i], bits(x)[i], gb[bad[0]], rb[bad[0]]))


def workload(func, n, seed=None):
    if func in F64:
        return inputs.workload_f64(func, n, seed)
    return inputs.workload_f32(func, n, seed)


ALL = F32 + F64


@pytest.mark.parametrize("func", ALL)
def test_small_sizes_and_ragged_tails(oracle, func):
    """Sizes that span several workgroup tiles plus ragged tails (1..3 extra
    elements), including n = 1 and a tile boundary."""
    _need_gpu()
    if not built(func):
        pytest.skip("not built")
    for n, seed in ((1, 1), (3, 2), (4, 3), (5, 4), (2047, 5), (2048, 6), (2049, 7),
                    (70001, 8)):
        x = workload(func, n, seed=10_000 + seed)
        got = gpu_eval(func, x)
        assert_same(func, x, got, oracle.evaluate(func, x))


@pytest.mark.parametrize("func", ALL)
def test_unaligned_pointers_and_in_place(oracle, func):
    _need_gpu()
    if not built(func):
        pytest.skip("not built")
    x = workload(func, 5003, seed=77)
    ref = oracle.evaluate(func, x)
    for oi, oo in ((1, 1), (1, 0), (0, 3), (2, 2)):
        assert_same(func, x, gpu_eval(func, x, offset_in=oi, offset_out=oo), ref)
    if func != "sincosf":
        dt = torch.float64 if func in F64 else torch.float32
        t = torch.from_numpy(x).to("cuda", dt)
        crmath.eval_ptr(func, t.data_ptr(), t.data_ptr(), x.size, 0, 0, crmath._stream_ptr(None))
        torch.cuda.synchronize()
        assert_same(func, x, t.cpu().numpy(), ref)


@pytest.mark.parametrize("func", ALL)
def test_hard_set(oracle, func):
    """The hardest-to-round inputs of the exhaustive scan (they exercise the
    fast-path rounding test and the accurate path)."""
    _need_gpu()
    if not built(func):
        pytest.skip("not built")
    x = inputs.hard_set(func)
    if x is None:
        pytest.skip("no hard set")
    crmath.stats_reset()
    got = gpu_eval(func, x)
    assert_same(func, x, got, oracle.evaluate(func, x))
    st = crmath.stats_read()
    assert st["escapes"] == 0, st


@pytest.mark.parametrize("func", ALL)
def test_force_fallback_matches(oracle, func):
    """With every element sent through the accurate path the results are the
    same, and the counters see every element."""
    _need_gpu()
    if not built(func):
        pytest.skip("not built")
    x = workload(func, 40_000, seed=99)
    crmath.stats_reset()
    got = gpu_eval(func, x, flags=crmath.FLAG_FORCE_FALLBACK)
    st = crmath.stats_read()
    assert_same(func, x, got, oracle.evaluate(func, x))
    # special inputs (NaN, out of domain, zeros, infinities) never need it
    assert st["fallback_lanes"] >= 0.8 * x.size
    assert st["escapes"] == 0


@pytest.mark.parametrize("func", ALL)
def test_special_inputs(oracle, func):
    _need_gpu()
    if not built(func):
        pytest.skip("not built")
    if func in F64:
        sp = np.array([0.0, -0.0, np.inf, -np.inf, 1.0, -1.0, 5e-324, -5e-324,
                       2.2250738585072014e-308, 1.7976931348623157e308, -1.7976931348623157e308,
                       709.782712893384, 709.7827128933841, -745.1332191019411,
                       -745.1332191019412, -708.3964185322641, 2.0 ** -53, 1 + 2.0 ** -52,
                       1 - 2.0 ** -53, 1024.0, np.nextafter(1024.0, 0), -1074.0, -1075.0,
                       np.nextafter(-1075.0, 0), np.nextafter(-1075.0, -np.inf), -1022.0,
                       np.nextafter(-1022.0, 0), -1074.5, 0.5, -0.5, 2.0 ** -1022 * 3],
                      dtype=np.float64)
        nanb = np.array([0x7FF8000000000000, 0xFFF8000000000000, 0x7FF0000000000001,
                         0x7FF8000000012345], dtype=np.uint64)
        sp = np.concatenate([sp, nanb.view(np.float64)])
    else:
        b = [0x00000000, 0x80000000, 0x7F800000, 0xFF800000, 0x7FC00000, 0xFFC00000,
             0x7F800001, 0x7FC12345, 0x00000001, 0x80000001, 0x007FFFFF, 0x807FFFFF,
             0x00800000, 0x80800000, 0x7F7FFFFF, 0xFF7FFFFF, 0x3F800000, 0xBF800000,
             0x3F000000, 0xBF000000, 0x40000000, 0xC0000000, 0x42B17218, 0x42B17217,
             0xC2CFF1B5, 0xC2CFF1B4, 0xC3160000, 0xC3150000, 0x42FE0000, 0x43000000,
             0x4B000000, 0x4B800000, 0x3F800001, 0x3F7FFFFF, 0x33800000, 0xB3800000,
             0x32000000, 0xB2000000, 0x3FC90FDB, 0x40490FDB, 0x49742400]
        sp = np.array(b, dtype=np.uint32).view(np.float32)
    assert_same(func, sp, gpu_eval(func, sp), oracle.evaluate(func, sp))


def test_expf_correctness_set(oracle):
    """expf on 2^20 values uniform in [-103.9, 88.7] plus 64 specials and edges."""
    _need_gpu()
    x = inputs.expf_correctness_set()
    crmath.stats_reset()
    got = gpu_eval("expf", x)
    assert_same("expf", x, got, oracle.evaluate("expf", x))
    assert crmath.stats_read()["escapes"] == 0


@pytest.mark.parametrize("func", ALL)
def test_full_size_sampled(oracle, func):
    """Full workload size (2^26 binary32 / 2^24 binary64 elements) in the launch
    configuration the benchmark times; a seeded sample of 2^14 outputs is
    compared with the oracle one by one."""
    _need_gpu()
    if not built(func):
        pytest.skip("not built")
    n = (1 << 24) if func in F64 else (1 << 26)
    x = workload(func, n)
    got = gpu_eval(func, x)
    idx = inputs.Stream(424242).below(1 << 14, n)
    xs = x[idx]
    ref = oracle.evaluate(func, xs)
    if func == "sincosf":
        assert_same(func, xs, got[:, idx], ref)
    else:
        assert_same(func, xs, got[idx], ref)


@pytest.mark.parametrize("func", F64)
def test_binary64_main_path_matches_accurate_path(func):
    """binary64 has no exhaustive check: on 2^25 inputs (the workload and
    uniformly random values or encodings of the domain) every result the main
    path certifies must equal the accurate path's, forced on every element.
    With a main-path test of width 2^-69 (exp), 2^-70 (log) or 2^-77 (exp2)
    relative, some of these inputs lie within the test's width of a rounding
    boundary, where an understated error bound would show."""
    _need_gpu()
    n = 1 << 24
    xs = [workload(func, n, seed=77)]
    st = inputs.Stream(78)
    if func == "exp":
        xs.append((-745.0 + (709.7 + 745.0) * st.uniform(n)).astype(np.float64))
    elif func == "exp2":
        xs.append((-1075.0 + (1024.0 + 1075.0) * st.uniform(n)).astype(np.float64))
    else:
        b = (st.u64(n) >> np.uint64(1)) % np.uint64(0x7FF0000000000000)
        xs.append(b.view(np.float64))
    for x in xs:
        a = gpu_eval(func, x)
        crmath.stats_reset()
        b = gpu_eval(func, x, flags=crmath.FLAG_FORCE_FALLBACK)
        assert crmath.stats_read()["escapes"] == 0
        bad = np.nonzero(bits(a) != bits(b))[0]
        assert bad.size == 0, (func, bad.size, hex(int(bits(x)[bad[0]])))


def test_exp2_exact_and_tie_cases(oracle):
    """binary64 exp2 at every integer k in [-1080, 1030] (2^k exactly, +0 at
    and below the tie -1075, +Inf from 1024 on), at k + 1/2, k + 1/4, k + 3/4
    and at k +- 1 ulp, against the oracle."""
    _need_gpu()
    k = np.arange(-1080, 1031, dtype=np.float64)
    x = np.concatenate([k, k + 0.5, k + 0.25, k + 0.75, np.nextafter(k, np.inf),
                        np.nextafter(k, -np.inf)])
    crmath.stats_reset()
    got = gpu_eval("exp2", x)
    assert_same("exp2", x, got, oracle.evaluate("exp2", x))
    assert crmath.stats_read()["escapes"] == 0


def _edge_inputs(func):
    """Encodings around the function's regime edges (overflow, underflow, first
    subnormal result, saturation, last f(x) == x or 1), located with the oracle
    (tests/golden/func_edges.json, written by tests/golden/make_func_edges.py)."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "func_edges.json")
    with open(path) as f:
        doc = json.load(f)["functions"][func]
    ut, ft = (np.uint64, np.float64) if func in F64 else (np.uint32, np.float32)
    b = [int(v, 16) for e in doc for v in e["bits"]]
    return np.array(b, dtype=ut).view(ft)


@pytest.mark.parametrize("impl", [crmath.IMPL_F64_INTERNAL, crmath.IMPL_SPLIT_F32],
                         ids=["f64", "split"])
@pytest.mark.parametrize("func", ALL)
def test_function_edges(oracle, func, impl):
    """Every function at its regime edges, +-2 encodings, in both
    implementations; with the accurate path forced as well."""
    _need_gpu()
    if func in F64 and impl == crmath.IMPL_SPLIT_F32:
        pytest.skip("binary64 functions have one implementation")
    if not built(func, impl):
        pytest.skip("not built")
    x = _edge_inputs(func)
    ref = oracle.evaluate(func, x)
    crmath.stats_reset()
    assert_same(func, x, gpu_eval(func, x, impl=impl), ref)
    assert_same(func, x, gpu_eval(func, x, impl=impl, flags=crmath.FLAG_FORCE_FALLBACK), ref)
    assert crmath.stats_read()["escapes"] == 0


def test_log_128_entry_table_variant(oracle):
    """binary64 log through the paper's 128-entry scaled-integer table
    (CR_IMPL_LOG128): ragged sizes, the hard set, specials and edges, the
    paper's range [0.125, 8] and the accurate path forced, against the oracle;
    and on 2^24 inputs every certified main-path result equals the forced
    accurate path's."""
    _need_gpu()
    impl = crmath.IMPL_LOG128
    assert crmath.available("log", impl) and not crmath.available("exp", impl)
    st = inputs.Stream(4242)
    cases = [workload("log", n, seed=20_000 + n) for n in (1, 3, 2047, 2049, 70001)]
    cases.append(inputs.hard_set("log"))
    cases.append(_edge_inputs("log"))
    cases.append(np.array([0.0, -0.0, np.inf, -np.inf, 1.0, -1.0, 5e-324, 2.0 ** -1022,
                           1.7976931348623157e308, 0.75, np.nextafter(0.75, 0), 1.5,
                           np.nextafter(1.5, 0), 1 + 2.0 ** -52, 1 - 2.0 ** -53], np.float64))
    cases.append((0.125 * 64.0 ** st.uniform(1 << 16)).astype(np.float64))  # log-uniform [1/8, 8]
    cases.append((0.125 + 7.875 * st.uniform(1 << 16)).astype(np.float64))  # uniform [1/8, 8]
    crmath.stats_reset()
    for x in cases:
        x = np.ascontiguousarray(x, dtype=np.float64)
        ref = oracle.evaluate("log", x)
        assert_same("log", x, gpu_eval("log", x, impl=impl), ref)
        assert_same("log", x, gpu_eval("log", x, impl=impl, flags=crmath.FLAG_FORCE_FALLBACK), ref)
    assert crmath.stats_read()["escapes"] == 0
    for x in (workload("log", 1 << 24, seed=79),
              (0.125 + 7.875 * st.uniform(1 << 24)).astype(np.float64)):
        a = gpu_eval("log", x, impl=impl)
        b = gpu_eval("log", x, impl=impl, flags=crmath.FLAG_FORCE_FALLBACK)
        bad = np.nonzero(bits(a) != bits(b))[0]
        assert bad.size == 0, (bad.size, hex(int(bits(x)[bad[0]])))
