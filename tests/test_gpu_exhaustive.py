"""Exhaustive checks over all 2^32 binary32 inputs (needs a GPU).

1. Fast path vs accurate path: for every encoding, the result the fast path
   certifies must equal the accurate path's result (forced on every element).
   This checks each fast path's error bound on every input; the accurate path
   itself is checked bit for bit against the oracle in test_gpu_parity.py.
2. No escapes: the accurate path certifies the rounding of every input.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2605_15547_amd import crmath  # noqa: E402

CHUNK = 1 << 28


def _run(func, x, flags):
    n = x.numel()
    out = torch.empty(2 * n if func == "sincosf" else n, dtype=torch.float32, device="cuda")
    crmath.eval_ptr(func, x.data_ptr(), out.data_ptr(), n, crmath.IMPL_F64_INTERNAL, flags,
                    crmath._stream_ptr(None))
    return out


@pytest.mark.parametrize("func", [f for f in crmath.FUNCS32 if f != "rsqrtf"])
def test_exhaustive_fast_path_matches_accurate_path(func):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not crmath.available(func, crmath.IMPL_F64_INTERNAL):
        pytest.skip("not built")
    crmath.stats_reset()
    total_bad = 0
    first = None
    for c in range(1 << 32 >> 28):
        xi = torch.arange(c * CHUNK, (c + 1) * CHUNK, dtype=torch.int64, device="cuda")
        x = xi.to(torch.int32).view(torch.float32)
        del xi
        a = _run(func, x, 0).view(torch.int32)
        b = _run(func, x, crmath.FLAG_FORCE_FALLBACK).view(torch.int32)
        bad = (a != b)
        nb = int(bad.sum().item())
        if nb and first is None:
            i = int(torch.nonzero(bad)[0].item()) % CHUNK
            first = (hex(c * CHUNK + i), hex(int(a[i].item()) & 0xffffffff),
                     hex(int(b[i].item()) & 0xffffffff))
        total_bad += nb
        del a, b, bad, x
    torch.cuda.synchronize()
    st = crmath.stats_read()
    assert total_bad == 0, (func, total_bad, first)
    assert st["escapes"] == 0, st
