"""Pins of the application-workload oracle (oracle/apps.py) against mpmath and
closed forms (CPU).  Paper, Sec. III-A: complex expf, logf and sinf accurate
to 2 ulps on valid inputs with both parts in [-40, 40], and spectral
interpolation by a brute-force DFT that spends its time in sincos.

The compositions are this project's (the paper names only their
ingredients), so the pins check what the paper fixes -- the 2-ulp accuracy of
each component against the exact complex function, and the DFT's definition
against an independent high-precision evaluation -- not the formulas
themselves.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import apps as A
from paper_2605_15547_amd import inputs as I


def ulp32(v):
    """ulp of the binary32 format at the magnitude of the real v."""
    v = abs(v)
    if v < mp.mpf(2) ** -126:
        return mp.mpf(2) ** -149
    e = int(mp.floor(mp.log(v, 2)))
    return mp.mpf(2) ** (e - 23)


def exact(func, x, y):
    z = mp.mpc(mp.mpf(float(x)), mp.mpf(float(y)))
    if func == "cexpf":
        return mp.exp(z)
    if func == "csinf":
        return mp.sin(z)
    w = mp.log(z)
    if y == 0 and np.signbit(y):  # the branch cut: atan2(-0, x) = -atan2(+0, x)
        w = mp.mpc(w.real, -w.imag)
    return w


def max_ulp_err(func, z, out):
    zz = z.reshape(-1, 2)
    oo = out.reshape(-1, 2)
    worst = 0.0
    with mp.workprec(120):
        for (x, y), (r, i) in zip(zz, oo):
            e = exact(func, x, y)
            for got, want in ((r, e.real), (i, e.imag)):
                if want == 0:
                    assert got == 0, (func, x, y, got)
                    continue
                err = float(abs(mp.mpf(float(got)) - want) / ulp32(want))
                worst = max(worst, err)
    return worst


BOUND = {"cexpf": 2.0, "csinf": 2.0, "clogf": 1.5}


@pytest.mark.parametrize("func", I.COMPLEX_FUNCS)
def test_complex_within_bound_on_workload(func):
    z = I.complex_workload(3000, seed=6100)
    out = A.evaluate_complex(func, z)
    assert max_ulp_err(func, z, out) <= BOUND[func]


def adversarial_clog():
    """|z| near 1 (log|z| tiny), points near the axes and the diagonals,
    negative real parts, signed zeros."""
    st = I.Stream(6200)
    th = st.uniform(400) * 2 * np.pi
    r = 1.0 + (st.uniform(400) - 0.5) * 2.0 ** -10
    pts = [np.stack([r * np.cos(th), r * np.sin(th)], 1)]
    t = st.uniform(200) * 2.0 ** -20
    pts.append(np.stack([1.0 - t, t], 1))
    pts.append(np.stack([-(1.0 + t), t], 1))
    pts.append(np.stack([t, -(1.0 - t)], 1))
    a = (st.uniform(200) - 0.5) * 80
    pts.append(np.stack([a, a * (1 + 2.0 ** -22)], 1))
    pts.append(np.stack([a, np.full(200, 2.0 ** -60)], 1))
    pts.append(np.array([[1.0, 0.0], [-1.0, 0.0], [-1.0, -0.0], [0.0, 1.0], [-0.0, -1.0],
                         [40.0, 40.0], [-40.0, 2.0 ** -63], [2.0 ** -63, 0.0],
                         [0.6, 0.8], [-0.8, 0.6]]))
    return np.concatenate(pts).astype(np.float32).reshape(-1)


def test_clogf_adversarial():
    z = adversarial_clog()
    out = A.clogf(z)
    assert max_ulp_err("clogf", z, out) <= BOUND["clogf"]


@pytest.mark.parametrize("func", ["cexpf", "csinf"])
def test_products_adversarial(func):
    """Factors at the bottom and top of their binades and tiny cosines."""
    st = I.Stream(6300)
    x = np.concatenate([st.uniform(300) * 80 - 40, np.log(np.arange(1, 60))])
    y = np.concatenate([np.pi / 2 + (st.uniform(300) - 0.5) * 1e-3,
                        (st.uniform(59) - 0.5) * 80])
    z = np.stack([x, y], 1).astype(np.float32).reshape(-1)
    assert max_ulp_err(func, z, A.evaluate_complex(func, z)) <= BOUND[func]


def test_complex_exact_cases():
    z = np.array([0, 0, 0, -0.0], dtype=np.float32)
    e = A.cexpf(z).reshape(-1, 2)
    assert e.tolist() == [[1.0, 0.0], [1.0, -0.0]]
    assert np.signbit(e[1, 1])
    s = A.csinf(z).reshape(-1, 2)
    assert s.tolist() == [[0.0, 0.0], [0.0, -0.0]]
    l = A.clogf(np.array([1, 0, -1, 0, -1, -0.0, 0, 1], dtype=np.float32)).reshape(-1, 2)
    pi = np.float32(math.pi)
    assert l.tolist() == [[0.0, 0.0], [0.0, pi], [0.0, -pi], [0.0, np.float32(math.pi / 2)]]


def test_dft_impulse_is_one_rotation():
    """x = delta[n - n0]: X_k = cos(theta) - i sin(theta) with theta =
    RN32(w_k n0), correctly rounded -- fixes the phase and the sign
    convention."""
    N, n0 = 1000, 617
    x = np.zeros(N, dtype=np.float32)
    x[n0] = 1.0
    _, w = I.dft_workload(N, 16, seed=7100)
    X, _ = A.dft(x, w)
    with mp.workprec(100):
        for k in range(w.size):
            th = mp.mpf(float(np.float32(w[k]) * np.float32(n0)))
            assert X[k, 0] == float(np.float32(float(mp.cos(th))))
            assert X[k, 1] == -float(np.float32(float(mp.sin(th))))


def test_dft_constant_signal_at_zero_frequency():
    N = 4096
    X, _ = A.dft(np.full(N, 0.5, dtype=np.float32), np.zeros(2, dtype=np.float32))
    assert X.tolist() == [[N / 2, 0.0], [N / 2, 0.0]]


def test_dft_against_exact_transform():
    """The oracle's sum differs from the exact DFT of the same phases (true
    sin and cos of each binary32 phase) only by the half-ulp roundings of sin
    and cos and the final rounding of the sum."""
    N = 300
    x, w = I.dft_workload(N, 4, seed=7200)
    X, mag = A.dft(x, w)
    with mp.workprec(120):
        for k in range(w.size):
            re = mp.mpf(0)
            im = mp.mpf(0)
            for n in range(N):
                th = mp.mpf(float(np.float32(w[k]) * np.float32(n)))
                re += mp.mpf(float(x[n])) * mp.cos(th)
                im -= mp.mpf(float(x[n])) * mp.sin(th)
            bound = float(np.sum(np.abs(x.astype(np.float64)))) * 2.0 ** -25 * 1.0001
            assert abs(X[k, 0] - re) <= bound + abs(re) * 2.0 ** -52
            assert abs(X[k, 1] - im) <= bound + abs(im) * 2.0 ** -52
