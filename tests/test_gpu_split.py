"""The binary32-only (split) implementation: float-float fast path,
triple-float accurate step, no binary64 operation.  Bit-exact parity with the
oracle, exhaustive agreement of its fast path with its accurate step, and of
its accurate step (forced on every element) with the binary64-internal
implementation, over all 2^32 inputs (needs a GPU)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2605_15547_amd import crmath, inputs  # noqa: E402

from test_gpu_parity import _edge_inputs, assert_same, gpu_eval  # noqa: E402

SPLIT = crmath.IMPL_SPLIT_F32
F32 = crmath.FUNCS32


def _need(func):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not crmath.available(func, SPLIT):
        pytest.skip("no split implementation")


@pytest.mark.parametrize("func", F32)
def test_split_small_sizes_and_unaligned(oracle, func):
    _need(func)
    for n, seed in ((1, 1), (5, 2), (2047, 3), (2049, 4), (70001, 5)):
        x = inputs.workload_f32(func, n, seed=20_000 + seed)
        assert_same(func, x, gpu_eval(func, x, impl=SPLIT), oracle.evaluate(func, x))
    x = inputs.workload_f32(func, 5003, seed=21_000)
    ref = oracle.evaluate(func, x)
    for oi, oo in ((1, 1), (0, 3)):
        assert_same(func, x, gpu_eval(func, x, impl=SPLIT, offset_in=oi, offset_out=oo), ref)


@pytest.mark.parametrize("func", F32)
def test_split_hard_set(oracle, func):
    _need(func)
    x = inputs.hard_set(func)
    crmath.stats_reset()
    assert_same(func, x, gpu_eval(func, x, impl=SPLIT), oracle.evaluate(func, x))
    assert crmath.stats_read()["escapes"] == 0


@pytest.mark.parametrize("func", F32)
def test_split_special_inputs(oracle, func):
    _need(func)
    b = [0x00000000, 0x80000000, 0x7F800000, 0xFF800000, 0x7FC00000, 0xFFC00000,
         0x7F800001, 0x7FC12345, 0x00000001, 0x80000001, 0x007FFFFF, 0x807FFFFF,
         0x00800000, 0x80800000, 0x7F7FFFFF, 0xFF7FFFFF, 0x3F800000, 0xBF800000,
         0x3F000000, 0xBF000000, 0x40000000, 0xC0000000, 0x42B17218, 0x42B17217,
         0xC2CFF1B5, 0xC2CFF1B4, 0xC3160000, 0xC3150000, 0x42FE0000, 0x43000000,
         0x4B000000, 0x4B800000, 0x3F800001, 0x3F7FFFFF, 0x33800000, 0xB3800000,
         0x32000000, 0xB2000000, 0x3FC90FDB, 0x40490FDB, 0x49742400]
    # binary32 integers and their neighbours: exact cases of exp2f and exp10f
    ks = np.arange(-160, 131, dtype=np.float32)
    sp = np.concatenate([np.array(b, dtype=np.uint32).view(np.float32), ks,
                         np.nextafter(ks, np.float32(np.inf)),
                         np.nextafter(ks, np.float32(-np.inf))])
    assert_same(func, sp, gpu_eval(func, sp, impl=SPLIT), oracle.evaluate(func, sp))


@pytest.mark.parametrize("func", [f for f in F32 if f != "rsqrtf"])
def test_split_triple_float_step_matches_oracle(oracle, func):
    """Every element through the triple-float step: workload, hard set,
    regime edges, raw encodings (specials, subnormals), tiny arguments."""
    _need(func)
    st = inputs.Stream(31_000 + crmath.FUNC_ID[func])
    tiny = np.ldexp(np.float32(1) + st.uniform(512).astype(np.float32),
                    -(12 + st.below(512, 130)).astype(np.int32)).astype(np.float32)
    parts = [inputs.workload_f32(func, 30_011, seed=31_100 + crmath.FUNC_ID[func]),
             inputs.hard_set(func), _edge_inputs(func), inputs.f32_bits(st.u32(8192)),
             tiny, -tiny]
    x = np.ascontiguousarray(np.concatenate([p for p in parts if p is not None]),
                             dtype=np.float32)
    crmath.stats_reset()
    got = gpu_eval(func, x, impl=SPLIT, flags=crmath.FLAG_FORCE_FALLBACK)
    stt = crmath.stats_read()
    assert_same(func, x, got, oracle.evaluate(func, x))
    assert stt["escapes"] == 0, stt


def test_split_expf_correctness_set(oracle):
    _need("expf")
    x = inputs.expf_correctness_set()
    assert_same("expf", x, gpu_eval("expf", x, impl=SPLIT), oracle.evaluate("expf", x))


@pytest.mark.parametrize("func", F32)
def test_split_full_size_sampled(oracle, func):
    _need(func)
    n = 1 << 26
    x = inputs.workload_f32(func, n)
    crmath.stats_reset()
    got = gpu_eval(func, x, impl=SPLIT)
    st = crmath.stats_read()
    idx = inputs.Stream(434343).below(1 << 14, n)
    ref = oracle.evaluate(func, x[idx])
    assert_same(func, x[idx], got[:, idx] if func == "sincosf" else got[idx], ref)
    assert st["escapes"] == 0


CHUNK = 1 << 28


@pytest.mark.parametrize("func", [f for f in F32 if f != "rsqrtf"])
def test_split_exhaustive_fast_path_matches_accurate_path(func):
    """Every binary32 encoding: the result the split fast path certifies equals
    the accurate path's (forced on every element)."""
    _need(func)
    sp = crmath._stream_ptr(None)
    crmath.stats_reset()
    total_bad, first = 0, None
    for c in range(1 << 32 >> 28):
        xi = torch.arange(c * CHUNK, (c + 1) * CHUNK, dtype=torch.int64, device="cuda")
        x = xi.to(torch.int32).view(torch.float32)
        del xi
        n = x.numel()
        nout = 2 * n if func == "sincosf" else n
        a = torch.empty(nout, dtype=torch.float32, device="cuda")
        b = torch.empty(nout, dtype=torch.float32, device="cuda")
        crmath.eval_ptr(func, x.data_ptr(), a.data_ptr(), n, SPLIT, 0, sp)
        crmath.eval_ptr(func, x.data_ptr(), b.data_ptr(), n, SPLIT, crmath.FLAG_FORCE_FALLBACK, sp)
        bad = a.view(torch.int32) != b.view(torch.int32)
        nb = int(bad.sum().item())
        if nb and first is None:
            i = int(torch.nonzero(bad)[0].item()) % CHUNK
            first = (hex(c * CHUNK + i), hex(int(a.view(torch.int32)[i].item()) & 0xffffffff),
                     hex(int(b.view(torch.int32)[i].item()) & 0xffffffff))
        total_bad += nb
        del a, b, bad, x
    torch.cuda.synchronize()
    st = crmath.stats_read()
    assert total_bad == 0, (func, total_bad, first)
    assert st["escapes"] == 0, st


def test_split_rsqrtf_exhaustive_matches_binary64_decision():
    """rsqrtf has no accurate path: both implementations decide the rounding
    exactly (binary64 midpoint residual vs integer comparison); they must agree
    on every binary32 encoding."""
    _need("rsqrtf")
    sp = crmath._stream_ptr(None)
    total_bad, first = 0, None
    for c in range(1 << 32 >> 28):
        xi = torch.arange(c * CHUNK, (c + 1) * CHUNK, dtype=torch.int64, device="cuda")
        x = xi.to(torch.int32).view(torch.float32)
        del xi
        a = torch.empty_like(x)
        b = torch.empty_like(x)
        crmath.eval_ptr("rsqrtf", x.data_ptr(), a.data_ptr(), x.numel(), SPLIT, 0, sp)
        crmath.eval_ptr("rsqrtf", x.data_ptr(), b.data_ptr(), x.numel(),
                        crmath.IMPL_F64_INTERNAL, 0, sp)
        bad = a.view(torch.int32) != b.view(torch.int32)
        nb = int(bad.sum().item())
        if nb and first is None:
            i = int(torch.nonzero(bad)[0].item())
            first = hex(c * CHUNK + i)
        total_bad += nb
        del a, b, bad, x
    torch.cuda.synchronize()
    assert total_bad == 0, (total_bad, first)


@pytest.mark.parametrize("func", [f for f in F32 if f != "rsqrtf"])
def test_split_triple_float_step_exhaustive_matches_binary64_path(func):
    """Every binary32 encoding through the triple-float step (forced on every
    element) gives the bits of the binary64-internal implementation, with no
    escape: the binary32-only accurate step decides every input on its own."""
    _need(func)
    sp = crmath._stream_ptr(None)
    crmath.stats_reset()
    total_bad, first = 0, None
    for c in range(1 << 32 >> 28):
        xi = torch.arange(c * CHUNK, (c + 1) * CHUNK, dtype=torch.int64, device="cuda")
        x = xi.to(torch.int32).view(torch.float32)
        del xi
        n = x.numel()
        nout = 2 * n if func == "sincosf" else n
        a = torch.empty(nout, dtype=torch.float32, device="cuda")
        b = torch.empty(nout, dtype=torch.float32, device="cuda")
        crmath.eval_ptr(func, x.data_ptr(), a.data_ptr(), n, SPLIT, crmath.FLAG_FORCE_FALLBACK, sp)
        st = crmath.stats_read()
        assert st["escapes"] == 0, (func, hex(c * CHUNK), st)
        crmath.eval_ptr(func, x.data_ptr(), b.data_ptr(), n, crmath.IMPL_F64_INTERNAL, 0, sp)
        # NaN results: compare as NaN (payloads are checked by the parity tests)
        av, bv = a.view(torch.int32), b.view(torch.int32)
        bad = (av != bv) & ~(torch.isnan(a) & torch.isnan(b))
        nb = int(bad.sum().item())
        if nb and first is None:
            i = int(torch.nonzero(bad)[0].item())
            first = (hex(c * CHUNK + i % CHUNK), hex(int(av[i].item()) & 0xffffffff),
                     hex(int(bv[i].item()) & 0xffffffff))
        total_bad += nb
        del a, b, av, bv, bad, x
    torch.cuda.synchronize()
    assert total_bad == 0, (func, total_bad, first)
