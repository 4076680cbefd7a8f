"""The binary32 functions in the directed rounding modes (toward zero, +inf,
-inf) on the GPU against the oracle in the same mode (needs a GPU).

The paper's CPU library supports every IEEE 754 rounding mode; its GPU runs
were round to nearest only (Sec. II-A, III-C).  Each directed-mode result is
certified by the rounding of both ends of a ~2^-100 error interval; the
exhaustive test checks that this certification succeeds for every binary32
encoding (no escapes) in every mode, and the parity tests compare with the
oracle bit for bit on the workloads, the hard sets, the regime edges, tiny
arguments and the exact cases.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2605_15547_amd import crmath, inputs  # noqa: E402
from test_gpu_parity import _edge_inputs, assert_same, gpu_eval  # noqa: E402

MODES = ("rz", "ru", "rd")
F32 = crmath.FUNCS32


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _cases(func):
    st = inputs.Stream(8000 + crmath.FUNC_ID[func])
    parts = [inputs.workload_f32(func, 20_011, seed=8100 + crmath.FUNC_ID[func]),
             _edge_inputs(func),
             inputs.f32_bits(st.u32(4096))]  # raw encodings: specials, subnormals, negatives
    hs = inputs.hard_set(func)
    if hs is not None:
        parts.append(hs[:1024])
    tiny = np.ldexp(np.float32(1) + st.uniform(256).astype(np.float32),
                    -(26 + st.below(256, 120)).astype(np.int32)).astype(np.float32)
    parts += [tiny, -tiny]
    ints = np.arange(-160, 140, dtype=np.float32)
    parts += [ints, np.ldexp(np.float32(1), np.arange(-149, 128)).astype(np.float32),
              np.array([10.0 ** k for k in range(11)], np.float32),
              np.array([0.0, -0.0, np.inf, -np.inf, -1.0, 1.0, -18.0, -18.5, 20.0, 89.0, -89.0,
                        100.0, -104.0, -200.0, 3.0e38], np.float32)]
    return np.ascontiguousarray(np.concatenate(parts), dtype=np.float32)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("func", F32)
def test_directed_mode_matches_oracle(oracle, func, mode):
    _need_gpu()
    x = _cases(func)
    crmath.stats_reset()
    got = gpu_eval(func, x, impl=crmath.IMPL_F64_INTERNAL, flags=crmath.ROUND_FLAGS[mode])
    assert crmath.stats_read()["escapes"] == 0
    assert_same(func, x, got, oracle.evaluate(func, x, mode=mode))


CHUNK = 1 << 28


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("func", F32)
def test_directed_mode_certifies_every_encoding(func, mode):
    """All 2^32 binary32 inputs: every directed-mode result is certified (no
    escapes)."""
    _need_gpu()
    fl = crmath.ROUND_FLAGS[mode]
    crmath.stats_reset()
    for c in range((1 << 32) // CHUNK):
        xi = torch.arange(c * CHUNK, (c + 1) * CHUNK, dtype=torch.int64, device="cuda")
        x = xi.to(torch.int32).view(torch.float32)
        del xi
        n = x.numel()
        out = torch.empty(2 * n if func == "sincosf" else n, dtype=torch.float32, device="cuda")
        crmath.eval_ptr(func, x.data_ptr(), out.data_ptr(), n, crmath.IMPL_F64_INTERNAL, fl,
                        crmath._stream_ptr(None))
        del out, x
    torch.cuda.synchronize()
    st = crmath.stats_read()
    assert st["escapes"] == 0, (func, mode, st)
