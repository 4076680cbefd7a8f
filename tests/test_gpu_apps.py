"""The paper's application workloads on the GPU (paper, Sec. III-A) against the
oracle of oracle/apps.py (needs a GPU).

* cexpf, clogf, csinf: the oracle evaluates the same composition (correctly
  rounded ingredients from the oracle, every other step one IEEE operation),
  so the GPU results must agree bit for bit on valid inputs.
* cr_dft: the oracle sums the exact binary64 products correctly rounded
  (math.fsum); the library sums them as double-doubles, so each component
  must lie within one binary64 ulp plus n 2^-100 of the sum of magnitudes.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2605_15547_amd import crmath, inputs  # noqa: E402


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def apps(oracle):
    from oracle import apps as A
    return A


def _complex_gpu(func, z, flags=0, offset=0):
    zt = torch.empty(z.size + 2 * offset, dtype=torch.float32, device="cuda")
    zt[2 * offset:] = torch.from_numpy(z)
    out = torch.full((z.size + 2 * offset,), -7.0, dtype=torch.float32, device="cuda")
    crmath.eval_ptr(func, zt[2 * offset:].data_ptr(), out[2 * offset:].data_ptr(), z.size // 2,
                    crmath.IMPL_AUTO, flags, crmath._stream_ptr(None))
    torch.cuda.synchronize()
    return out[2 * offset:].cpu().numpy()


def _same(func, z, got, ref):
    gb, rb = got.view(np.uint32), ref.view(np.uint32)
    bad = np.nonzero(gb != rb)[0]
    if bad.size:
        i = bad[0] // 2
        raise AssertionError("%s: %d mismatching parts; first z=(%r, %r) gpu=0x%x oracle=0x%x"
                             % (func, bad.size, z[2 * i], z[2 * i + 1], gb[bad[0]], rb[bad[0]]))


def _adversarial(func):
    """Inputs near the places where each composition changes branch or loses
    digits: |z| near 1 (clogf's log1p branch), |x| == |y|, the axes, signed
    zeros in one part, and the edges of the valid range."""
    st = inputs.Stream(6100 + crmath.FUNC_ID[func])
    n = 1 << 12
    ang = st.uniform(n) * 2 * np.pi
    r = 1.0 + (st.uniform(n) - 0.5) * 2.0 ** -10
    ring = np.stack([r * np.cos(ang), r * np.sin(ang)], axis=1).astype(np.float32).ravel()
    v = inputs.uniform_f32(st, n, -40.0, 40.0)
    diag = np.stack([v, v * np.where(st.uniform(n) < 0.5, 1, -1)], axis=1).astype(np.float32)
    axes = np.stack([v, np.zeros(n, np.float32)], axis=1).astype(np.float32)
    axes2 = np.stack([np.float32(-0.0) * np.ones(n, np.float32), v], axis=1).astype(np.float32)
    near = np.stack([inputs.uniform_f32(st, n, 0.70, 0.72),
                     inputs.uniform_f32(st, n, 0.69, 0.71)], axis=1).astype(np.float32)
    parts = [ring, diag.ravel(), near.ravel()]
    if func == "clogf":
        # the axes only where |z| > 0; sqrt(0.5)-radius circle (s = 0.5 edge)
        parts += [axes.ravel()[np.repeat(v != 0, 2)], axes2.ravel()[np.repeat(v != 0, 2)]]
        big = np.stack([inputs.uniform_f32(st, n, -2.0 ** 62, 2.0 ** 62),
                        inputs.uniform_f32(st, n, -1e-15, 1e-15)], axis=1).astype(np.float32)
        parts.append(big.ravel())
    else:
        parts += [axes.ravel(), axes2.ravel()]
    return np.ascontiguousarray(np.concatenate(parts), dtype=np.float32)


@pytest.mark.parametrize("func", crmath.COMPLEX)
def test_complex_workload_matches_oracle(apps, func):
    """2^18 + 3 complex numbers with parts uniform in [-40, 40] (the paper's
    range), the ragged tail included, plus adversarial inputs."""
    _need_gpu()
    for z in (inputs.complex_workload((1 << 18) + 3), _adversarial(func)):
        crmath.stats_reset()
        got = _complex_gpu(func, z)
        assert crmath.stats_read()["escapes"] == 0
        _same(func, z, got, apps.evaluate_complex(func, z))


@pytest.mark.parametrize("func", crmath.COMPLEX)
def test_complex_sizes_offsets_and_forced_fallback(apps, func):
    _need_gpu()
    z = inputs.complex_workload(5003, seed=6200)
    ref = apps.evaluate_complex(func, z)
    for off in (0, 1, 3):
        _same(func, z, _complex_gpu(func, z, offset=off), ref)
    crmath.stats_reset()
    _same(func, z, _complex_gpu(func, z, flags=crmath.FLAG_FORCE_FALLBACK), ref)
    st = crmath.stats_read()
    assert st["escapes"] == 0 and st["fallback_lanes"] >= z.size // 2
    for n in (1, 2, 3, 2049):
        zz = inputs.complex_workload(n, seed=6300 + n)
        _same(func, zz, _complex_gpu(func, zz), apps.evaluate_complex(func, zz))


def _dft_gpu(x, w, flags=0):
    xt = torch.from_numpy(x).cuda()
    wt = torch.from_numpy(w).cuda()
    X = crmath.dft(xt, wt, flags=flags)
    torch.cuda.synchronize()
    return X.cpu().numpy()


def _dft_close(X, ref, mag, n):
    tol = np.spacing(np.abs(ref)) + n * 2.0 ** -100 * mag + 2.0 ** -1074
    err = np.abs(X - ref)
    bad = np.nonzero(err > tol)
    assert bad[0].size == 0, (bad[0][:4], X[bad][:4], ref[bad][:4])


@pytest.mark.parametrize("n,m", [(1, 1), (300, 7), (4099, 33), (70001, 5)])
def test_dft_matches_oracle(apps, n, m):
    """Spectral interpolation at non-integer frequencies: every component
    within one ulp (plus the summation bound) of the correctly rounded sum of
    the exact products."""
    _need_gpu()
    x, w = inputs.dft_workload(n, m, seed=7000 + n)
    ref, mag = apps.dft(x, w)
    crmath.stats_reset()
    X = _dft_gpu(x, w)
    assert crmath.stats_read()["escapes"] == 0
    _dft_close(X, ref, mag, n)
    # the same sums on every run, and with every sincosf through the accurate path
    assert np.array_equal(X.view(np.uint64), _dft_gpu(x, w).view(np.uint64))
    Xf = _dft_gpu(x, w, flags=crmath.FLAG_FORCE_FALLBACK)
    assert np.array_equal(X.view(np.uint64), Xf.view(np.uint64))


def test_dft_impulse_and_constant(apps):
    """An impulse at sample j gives one rotation RN(cos t) - i RN(sin t) per
    output; a constant signal at angle 0 sums exactly to n."""
    _need_gpu()
    n = 5000
    x = np.zeros(n, np.float32)
    x[1234] = 1.0
    w = np.array([0.001, 0.37, 2.5, 3.0], np.float32)
    X = _dft_gpu(x, w)
    ref, _ = apps.dft(x, w)
    assert np.array_equal(X.view(np.uint64), ref.view(np.uint64))
    X = _dft_gpu(np.ones(n, np.float32), np.zeros(3, np.float32))
    assert np.all(X[:, 0] == n) and np.all(X[:, 1] == 0.0)


def test_dft_full_size_sampled(apps):
    """The benchmark's DFT size (2^20 samples, 256 outputs) in its launch
    shape; 4 outputs checked against the oracle."""
    _need_gpu()
    n, m = 1 << 20, 256
    x, w = inputs.dft_workload(n, m)
    X = _dft_gpu(x, w)
    pick = np.array([0, 77, 128, 255])
    ref, mag = apps.dft(x, w[pick])
    _dft_close(X[pick], ref, mag, n)
