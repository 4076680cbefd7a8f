"""Ragged batches (cr_batch_plan_* / cr_eval_batch) against the oracle (GPU).

Requests of mixed function and uneven length (including empty, single-element
and unaligned ones) are evaluated by one persistent launch; every output is
compared bit for bit with the oracle.  The plan's graph is replayed several
times with eager work and synchronisation in between, and every replay is
checked.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2605_15547_amd import crmath, inputs  # noqa: E402


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def make_requests(num, seed, max_log2, unaligned=False, extra=()):
    funcs, lens, seeds = inputs.batch_requests(num=num, seed=seed, max_log2=max_log2)
    funcs, lens, seeds = list(funcs), list(lens), list(seeds)
    for f, n in extra:
        funcs.append(f)
        lens.append(n)
        seeds.append(len(seeds) + 17)
    items = []
    for k, (f, n, sd) in enumerate(zip(funcs, lens, seeds)):
        n = int(n)
        x = inputs.workload_f32(f, n, seed=int(sd) % (1 << 62))
        oi = (k % 3) if unaligned else 0
        oo = ((k + 1) % 3) if unaligned else 0
        nout = 2 * n if f == "sincosf" else n
        xin = torch.empty(n + oi, dtype=torch.float32, device="cuda")
        if n:
            xin[oi:] = torch.from_numpy(x)
        out = torch.full((nout + oo,), -3.0, dtype=torch.float32, device="cuda")
        items.append(dict(func=f, n=n, x=x, xin=xin, out=out, oi=oi, oo=oo))
    return items


def req_list(items, impl_of=lambda k: crmath.IMPL_AUTO):
    return [(it["func"], it["xin"].data_ptr() + 4 * it["oi"], it["out"].data_ptr() + 4 * it["oo"],
             it["n"], impl_of(k)) for k, it in enumerate(items)]


def check(items, oracle, what):
    for it in items:
        f, n = it["func"], it["n"]
        if n == 0:
            assert torch.all(it["out"] == -3.0), (what, f, "wrote to an empty request")
            continue
        got = it["out"][it["oo"]:].cpu().numpy()
        if it["oo"]:
            assert np.all(it["out"][:it["oo"]].cpu().numpy() == -3.0)
        ref = oracle.evaluate(f, it["x"])
        gb = got.view(np.uint32).ravel()
        rb = np.asarray(ref).view(np.uint32).ravel()
        bad = np.nonzero(gb != rb)[0]
        assert bad.size == 0, (what, f, n, int(bad.size), int(bad[0]))


def test_batch_plan_replays(oracle):
    _need_gpu()
    items = make_requests(300, 5100, 14, extra=[("expf", 0), ("sincosf", 1), ("logf", 3),
                                                 ("sincosf", 4097), ("tanf", 2049)])
    crmath.stats_reset()
    plan = crmath.BatchPlan(req_list(items))
    for rep in range(3):
        for it in items:  # eager work between replays
            it["out"].fill_(-3.0)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        check(items, oracle, "replay %d" % rep)
    plan.destroy()
    assert crmath.stats_read()["escapes"] == 0


def test_batch_unaligned_and_forced(oracle):
    _need_gpu()
    items = make_requests(120, 5200, 12, unaligned=True, extra=[("sincosf", 1001)])
    plan = crmath.BatchPlan(req_list(items), flags=crmath.FLAG_FORCE_FALLBACK)
    plan.launch()
    torch.cuda.synchronize()
    check(items, oracle, "forced")
    plan.destroy()


@pytest.mark.parametrize("bpc", [1, 16])
def test_batch_grid_sizes(oracle, bpc):
    """The batch grid (cr_tune_batch_set) changes only the speed: plans made
    at 1 and 16 workgroups per CU, and cr_eval_batch, give the oracle's bits."""
    _need_gpu()
    items = make_requests(200, 5150 + bpc, 14, extra=[("sincosf", 2051), ("atanf", 4099)])
    try:
        for impl in (crmath.IMPL_F64_INTERNAL, crmath.IMPL_SPLIT_F32):
            crmath.tune_batch_set(impl, bpc)
        plan = crmath.BatchPlan(req_list(items, lambda k: 1 + k % 2))
        plan.launch()
        torch.cuda.synchronize()
        check(items, oracle, "plan at %d WG/CU" % bpc)
        plan.destroy()
        for it in items:
            it["out"].fill_(-3.0)
        crmath.eval_batch(req_list(items))
        torch.cuda.synchronize()
        check(items, oracle, "eval_batch at %d WG/CU" % bpc)
    finally:
        crmath.tune_reset()


def test_eval_batch(oracle):
    _need_gpu()
    items = make_requests(150, 5300, 13)
    crmath.eval_batch(req_list(items))
    torch.cuda.synchronize()
    check(items, oracle, "eval_batch")


def test_batch_full_size_sampled(oracle):
    """The full ragged workload (4096 requests, lengths up to 2^20) as one plan;
    a seeded sample of each request's outputs is compared with the oracle."""
    _need_gpu()
    funcs, lens, seeds = inputs.batch_requests()
    xs, outs, reqs = [], [], []
    for f, n, sd in zip(funcs, lens, seeds):
        n = int(n)
        x = inputs.workload_f32(f, n, seed=int(sd))
        xt = torch.from_numpy(x).cuda()
        ot = torch.empty(2 * n if f == "sincosf" else n, dtype=torch.float32, device="cuda")
        xs.append((f, x, xt))
        outs.append(ot)
        reqs.append((f, xt.data_ptr(), ot.data_ptr(), n))
    plan = crmath.BatchPlan(reqs)
    plan.launch()
    torch.cuda.synchronize()
    st = inputs.Stream(777)
    for (f, x, _), ot in zip(xs, outs):
        n = x.size
        k = min(n, 16)
        idx = st.below(k, n)
        got = ot.cpu().numpy()
        ref = oracle.evaluate(f, x[idx])
        if f == "sincosf":
            g = np.stack([got[:n][idx], got[n:][idx]])
        else:
            g = got[idx]
        assert np.array_equal(g.view(np.uint32), np.asarray(ref).view(np.uint32)), f
    plan.destroy()


def test_batch_mixed_implementations(oracle):
    """Requests alternating between the binary64-internal and the binary32-only
    implementation in one plan (replayed twice, the second time with every
    element forced through the accurate path in a second plan)."""
    _need_gpu()
    items = make_requests(240, 5400, 13, unaligned=True, extra=[("sincosf", 3001), ("expf", 1)])
    impl_of = lambda k: crmath.IMPL_SPLIT_F32 if k % 2 else crmath.IMPL_F64_INTERNAL
    crmath.stats_reset()
    plan = crmath.BatchPlan(req_list(items, impl_of))
    for rep in range(2):
        for it in items:
            it["out"].fill_(-3.0)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        check(items, oracle, "mixed replay %d" % rep)
    plan.destroy()
    assert crmath.stats_read()["escapes"] == 0
    plan = crmath.BatchPlan(req_list(items, impl_of), flags=crmath.FLAG_FORCE_FALLBACK)
    plan.launch()
    torch.cuda.synchronize()
    check(items, oracle, "mixed forced")
    plan.destroy()


def test_batch_full_size_split_sampled(oracle):
    """The full ragged workload with every request on the binary32-only
    implementation; a seeded sample of each request is compared."""
    _need_gpu()
    funcs, lens, seeds = inputs.batch_requests()
    xs, outs, reqs = [], [], []
    for f, n, sd in zip(funcs, lens, seeds):
        n = int(n)
        x = inputs.workload_f32(f, n, seed=int(sd))
        xt = torch.from_numpy(x).cuda()
        ot = torch.empty(2 * n if f == "sincosf" else n, dtype=torch.float32, device="cuda")
        xs.append((f, x, xt))
        outs.append(ot)
        reqs.append((f, xt.data_ptr(), ot.data_ptr(), n, crmath.IMPL_SPLIT_F32))
    plan = crmath.BatchPlan(reqs)
    plan.launch()
    torch.cuda.synchronize()
    st = inputs.Stream(778)
    for (f, x, _), ot in zip(xs, outs):
        n = x.size
        idx = st.below(min(n, 16), n)
        got = ot.cpu().numpy()
        ref = oracle.evaluate(f, x[idx])
        g = np.stack([got[:n][idx], got[n:][idx]]) if f == "sincosf" else got[idx]
        assert np.array_equal(g.view(np.uint32), np.asarray(ref).view(np.uint32)), f
    plan.destroy()
