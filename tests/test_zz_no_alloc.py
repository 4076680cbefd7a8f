"""cr_eval_batch_noalloc (tables in the library's static scratch) against
cr_eval_batch (tables in stream-ordered allocations), through the C ABI.

Two calls in a row, the second with a smaller batch, each compared bit for bit
with cr_eval_batch on the same requests; a sample of each call is also checked
against the oracle.  The size limit is rejected on the host before anything
is copied or launched.
"""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2605_15547_amd import crmath, inputs  # noqa: E402


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _items(num, seed, max_log2):
    funcs, lens, seeds = inputs.batch_requests(num=num, seed=seed, max_log2=max_log2)
    items = []
    for k, (f, n, sd) in enumerate(zip(funcs, lens, seeds)):
        n = int(n)
        x = inputs.workload_f32(f, n, seed=int(sd) % (1 << 62))
        oi, oo = k % 3, (k + 1) % 3  # unaligned requests too
        nout = 2 * n if f == "sincosf" else n
        xin = torch.empty(n + oi, dtype=torch.float32, device="cuda")
        if n:
            xin[oi:] = torch.from_numpy(x)
        items.append(dict(func=f, n=n, x=x, xin=xin, oi=oi, oo=oo, nout=nout))
    return items


def _reqs(items, outs, impl_of):
    return [(it["func"], it["xin"].data_ptr() + 4 * it["oi"], o.data_ptr() + 4 * it["oo"],
             it["n"], impl_of(k)) for k, (it, o) in enumerate(zip(items, outs))]


def _outs(items, fill):
    return [torch.full((it["nout"] + it["oo"],), fill, dtype=torch.float32, device="cuda")
            for it in items]


def _compare(items, a, b, oracle, what):
    for k, (it, oa, ob) in enumerate(zip(items, a, b)):
        ga = oa[it["oo"]:].cpu().numpy().view(np.uint32)
        gb = ob[it["oo"]:].cpu().numpy().view(np.uint32)
        bad = np.nonzero(ga != gb)[0]
        assert bad.size == 0, (what, k, it["func"], it["n"], int(bad.size))
        # nothing written before the request's output range
        assert np.all(oa[:it["oo"]].cpu().numpy() == -5.0), (what, k)
        if it["n"] and k % 7 == 0:
            ref = np.asarray(oracle.evaluate(it["func"], it["x"])).view(np.uint32).ravel()
            assert np.array_equal(ga, ref), (what, k, it["func"], "oracle")


@pytest.mark.parametrize("impl", [crmath.IMPL_AUTO, crmath.IMPL_SPLIT_F32])
def test_noalloc_matches_eval_batch_twice(oracle, impl):
    _need_gpu()
    for call, (num, seed, ml) in enumerate(((400, 6100, 15), (60, 6200, 11))):
        items = _items(num, seed, ml)
        items.append(dict(func="expf", n=0, x=np.zeros(0, np.float32),
                          xin=torch.empty(1, device="cuda"), oi=0, oo=0, nout=0))
        a, b = _outs(items, -5.0), _outs(items, -5.0)
        impl_of = (lambda k: impl if k % 2 else crmath.IMPL_AUTO)
        crmath.stats_reset()
        crmath.eval_batch_noalloc(_reqs(items, a, impl_of))
        torch.cuda.synchronize()
        st = crmath.stats_read()
        assert st["escapes"] == 0, st
        crmath.eval_batch(_reqs(items, b, impl_of))
        torch.cuda.synchronize()
        _compare(items, a, b, oracle, "call %d" % call)


def test_noalloc_rejects_oversize_batches():
    """Rejected on the host (no copy, no launch): too many requests, or more
    tiles than the scratch holds."""
    _need_gpu()
    L = crmath.lib()
    big = (crmath.Request * (crmath.NOALLOC_MAX_REQUESTS + 1))()
    assert L.cr_eval_batch_noalloc(big, len(big), None) == -11
    # two requests of 2^31 - 1 elements: 2^19 tiles of 4096 elements each, twice
    # the 2^19 tiles the scratch holds
    x = torch.empty(4, device="cuda")
    y = torch.empty(4, device="cuda")
    arr = (crmath.Request * 2)()
    n = (1 << 31) - 1
    arr[0] = crmath.Request(0, 0, x.data_ptr(), x.data_ptr(), n)
    arr[1] = crmath.Request(0, 0, y.data_ptr(), y.data_ptr(), n)
    assert L.cr_eval_batch_noalloc(arr, 2, None) == -11
    assert L.cr_status_str(-11)
    # the rejected calls launched nothing: the library still works
    v = torch.full((4097,), 0.5, device="cuda")
    o = torch.empty(4097, device="cuda")
    crmath.eval_batch_noalloc([("expf", v.data_ptr(), o.data_ptr(), 4097)])
    torch.cuda.synchronize()
    ref = oracle_free_expf_half()
    assert int(o.view(torch.int32)[0].item()) & 0xffffffff == ref
    assert torch.equal(o, o[0].expand(4097))


def oracle_free_expf_half():
    """RN_f32(e^0.5) = 0x3fd3094c (e^0.5 = 1.6487212707001282...; the binary32
    neighbours are 1.64872121811 and 1.64872133732, the first is nearer)."""
    return 0x3FD3094C


def test_noalloc_scratch_symbol_is_not_host_memory():
    """The entry point is exported and the request struct matches the header
    (32 bytes: two int32, two pointers, one int64)."""
    _need_gpu()
    assert ctypes.sizeof(crmath.Request) == 32
    assert hasattr(crmath.lib(), "cr_eval_batch_noalloc")
