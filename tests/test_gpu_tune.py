"""Launch configurations and the autotuner (needs a GPU): every kernel variant
and grid size gives the same bits as the oracle, and the autotuner installs a
configuration that keeps them."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2605_15547_amd import crmath, inputs  # noqa: E402

F64 = crmath.FUNCS64

from test_gpu_parity import assert_same, gpu_eval  # noqa: E402


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(autouse=True)
def _reset_tuning():
    crmath.tune_reset()
    yield
    crmath.tune_reset()


CASES = [("expf", crmath.IMPL_F64_INTERNAL), ("log1pf", crmath.IMPL_F64_INTERNAL),
         ("sinf", crmath.IMPL_F64_INTERNAL), ("atanf", crmath.IMPL_F64_INTERNAL),
         ("logf", crmath.IMPL_SPLIT_F32), ("tanf", crmath.IMPL_SPLIT_F32)]


@pytest.mark.parametrize("func,impl", CASES)
def test_every_variant_is_bit_exact(oracle, func, impl):
    _need_gpu()
    if not crmath.available(func, impl):
        pytest.skip("not built")
    # several tiles per workgroup at the smallest grid, a ragged tail, an
    # unaligned head, and the forced accurate path on one variant
    x = inputs.workload_f32(func, 300_001, seed=31_000)
    ref = oracle.evaluate(func, x)
    for v in range(len(crmath.tune_variants())):
        for bpc in (1, 16):
            crmath.tune_set(func, impl, v, bpc)
            assert_same(func, x, gpu_eval(func, x, impl=impl), ref)
    crmath.tune_set(func, impl, len(crmath.tune_variants()) - 1, 2)
    assert_same(func, x, gpu_eval(func, x, impl=impl, offset_in=1, offset_out=1), ref)
    assert_same(func, x, gpu_eval(func, x, impl=impl, flags=crmath.FLAG_FORCE_FALLBACK), ref)


# the binary64 kernel's own variants (cr.h: 0..3)
N64_VARIANTS = 4


@pytest.mark.parametrize("func,impl", [("exp", crmath.IMPL_F64_INTERNAL),
                                       ("log", crmath.IMPL_F64_INTERNAL),
                                       ("exp2", crmath.IMPL_F64_INTERNAL),
                                       ("log", crmath.IMPL_LOG128)])
def test_every_binary64_variant_is_bit_exact(oracle, func, impl):
    _need_gpu()
    # several tiles per workgroup at the smallest grid, a ragged tail (odd n),
    # an unaligned head, and the forced accurate path on every variant
    x = inputs.workload_f64(func, 200_003, seed=31_500)
    ref = oracle.evaluate(func, x)
    for v in range(N64_VARIANTS):
        for bpc in (1, 16):
            crmath.tune_set(func, impl, v, bpc)
            assert_same(func, x, gpu_eval(func, x, impl=impl), ref)
        assert_same(func, x, gpu_eval(func, x, impl=impl, offset_in=1, offset_out=1), ref)
        assert_same(func, x, gpu_eval(func, x, impl=impl, flags=crmath.FLAG_FORCE_FALLBACK), ref)
    with pytest.raises(Exception):
        crmath.tune_set(func, impl, N64_VARIANTS, 16)


@pytest.mark.parametrize("func,impl", [("expf", 1), ("sincosf", 1), ("exp", 1), ("logf", 2)])
def test_autotune_installs_a_correct_configuration(oracle, func, impl):
    _need_gpu()
    n = 1 << 20
    if func in F64:
        x = inputs.workload_f64(func, n, seed=32_000)
        dt = torch.float64
    else:
        x = inputs.workload_f32(func, n, seed=32_000)
        dt = torch.float32
    xt = torch.from_numpy(x).to("cuda", dt)
    out = torch.empty(2 * n if func == "sincosf" else n, dtype=dt, device="cuda")
    rate = crmath.autotune(func, impl, xt.data_ptr(), out.data_ptr(), n, reps=2,
                           stream_ptr=crmath._stream_ptr(None))
    assert rate > 0
    v, b = crmath.tune_get(func, impl)
    nv = 1 if func == "sincosf" else N64_VARIANTS if func in F64 else len(crmath.tune_variants())
    assert 0 <= v < nv and b in (2, 4, 8, 16, 32)
    idx = inputs.Stream(5).below(4096, n)
    got = gpu_eval(func, x, impl=impl)
    ref = oracle.evaluate(func, x[idx])
    assert_same(func, x[idx], got[:, idx] if func == "sincosf" else got[idx], ref)
