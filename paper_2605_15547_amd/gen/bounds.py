"""Rigorous upper bounds on polynomial approximation errors.

For h = f - p on [a, b] with p a polynomial of degree d, split [a, b] into N
pieces [c - w, c + w].  By Taylor's theorem with the Lagrange remainder, on
each piece
    |h(x)| <= sum_{k <= d} |h^(k)(c)| w^k / k!  +  M w^(d+1) / (d+1)!,
where M bounds |f^(d+1)| on the piece (p^(d+1) = 0).  The derivatives at c
are evaluated at 320 bits: their rounding (relative 2^-310 of terms below 1)
is covered by adding 2^-250 to the result.  The bound of sup |h| over [a, b]
is the largest piece bound.  With N pieces the k >= 1 terms add about
pi (d + 2) / (2 N) of the true maximum, so N of a few hundred gives bounds
within a few percent of the true sup.

Each approximation the kernels' rounding tests rely on is described by a
Spec: the derivatives of f at a point, a bound of |f^(K)| on an interval, the
polynomial p (as coefficients of powers of x) and the interval.
"""
import mpmath as mp

PREC = 320


class Spec:
    """f - p on [a, b]; fder(c, k) = list of f^(j)(c), j < k; fbound(lo, hi, K)
    >= sup |f^(K)| on [lo, hi]; poly = {power: coefficient} (exact values)."""

    def __init__(self, name, fder, fbound, poly, a, b):
        self.name, self.fder, self.fbound = name, fder, fbound
        self.poly = {int(e): mp.mpf(c) for e, c in poly.items()}
        self.a, self.b = mp.mpf(a), mp.mpf(b)


def _poly_ders(poly, c, K):
    """p^(j)(c) for j < K."""
    out = []
    for j in range(K):
        s = mp.mpf(0)
        for e, co in poly.items():
            if e >= j:
                s += co * mp.ff(e, j) * c ** (e - j)
        out.append(s)
    return out


def sup_bound(spec, pieces=256):
    """Rigorous upper bound of sup |f - p| on [a, b]."""
    with mp.workprec(PREC):
        d = max(spec.poly)
        K = d + 1
        a, b = spec.a, spec.b
        worst = mp.mpf(0)
        for i in range(pieces):
            lo = a + (b - a) * i / pieces
            hi = a + (b - a) * (i + 1) / pieces
            c = (lo + hi) / 2
            w = (hi - lo) / 2
            fd = spec.fder(c, K)
            pd = _poly_ders(spec.poly, c, K)
            s = mp.mpf(0)
            for k in range(K):
                s += abs(fd[k] - pd[k]) * w ** k / mp.factorial(k)
            s += spec.fbound(lo, hi, K) * w ** K / mp.factorial(K)
            if s > worst:
                worst = s
        return worst + mp.mpf(2) ** -250


def log2b(v):
    return float(mp.log(v, 2))


# ---------------------------------------------------------- function families
def expm1_minus_r(poly_r2, rho):
    """e^r - 1 - r against r^2 P(r) on [-rho, rho]: poly_r2 = [P0, P1, ...]."""
    def fder(c, K):
        e = mp.exp(c)
        return [mp.expm1(c) - c, e - 1] + [e] * (K - 2)

    def fbound(lo, hi, K):
        return mp.exp(hi)
    poly = {k + 2: v for k, v in enumerate(poly_r2)}
    return Spec("e^r - 1 - r", fder, fbound, poly, -rho, rho)


def log1p_series_ders(c, K, shift, sign0, scale=1):
    """Derivatives of g(t) = scale * sum_{n>=0} s_n t^n / (n + shift) with
    s_n = sign0 (-1)^n, summed from the series until the terms fall below
    2^-340 (|c| <= 1/8 here, so they decrease geometrically)."""
    eps = mp.mpf(2) ** -340
    out = []
    for k in range(K):
        s = mp.mpf(0)
        coef = mp.factorial(k)  # n!/(n-k)! at n = k
        cp = mp.mpf(1)          # c^(n-k)
        sign = sign0 * (-1) ** k
        n = k
        while True:
            term = coef * cp / (n + shift)
            s += sign * term
            if n > k + 4 and abs(term) < eps:
                break
            n += 1
            coef = coef * n / (n - k)
            cp *= c
            sign = -sign
        out.append(scale * s)
    return out


def log1p_series_bound(lo, hi, K, shift, scale=1):
    """sup |g^(K)| for the series above: sum_j (j+K)!/j! |t|^j / (j+K+shift)
    <= K!/(K+shift) (1 - |t|)^-(K+1)."""
    t = max(abs(mp.mpf(lo)), abs(mp.mpf(hi)))
    return abs(scale) * mp.factorial(K) / (K + shift) / (1 - t) ** (K + 1)


def log64_quotient(S, a, b):
    """g(t) = (log1p t - t + t^2/2 - t^3/3) / t^4 = sum (-1)^(n+1) t^n/(n+4)
    against S(t) (unweighted)."""
    return Spec("(log1p t - t + t^2/2 - t^3/3)/t^4",
                lambda c, K: log1p_series_ders(c, K, 4, -1),
                lambda lo, hi, K: log1p_series_bound(lo, hi, K, 4),
                {k: v for k, v in enumerate(S)}, a, b)


def log64_absolute(S, a, b):
    """log1p t - t + t^2/2 - t^3/3 against t^4 S(t) (absolute)."""
    def fder(c, K):
        # f(t) = log1p t - t + t^2/2 - t^3/3
        out = [mp.log1p(c) - c + c * c / 2 - c ** 3 / 3,
               1 / (1 + c) - 1 + c - c * c, -1 / (1 + c) ** 2 + 1 - 2 * c,
               2 / (1 + c) ** 3 - 2]
        for k in range(4, K):
            out.append((-1) ** (k - 1) * mp.factorial(k - 1) / (1 + c) ** k)
        return out[:K]

    def fbound(lo, hi, K):
        return mp.factorial(K - 1) / (1 + min(mp.mpf(lo), mp.mpf(0))) ** K
    return Spec("log1p t - t + t^2/2 - t^3/3", fder, fbound,
                {k + 4: v for k, v in enumerate(S)}, a, b)


def log_b_quotient(Q, base, K0, a, b):
    """g(t) = log1p(t) / (t ln b) - K0 = sum (-1)^n t^n/(n+1) / ln b - K0
    against Q(t); 1/ln b is formed at the working precision."""
    def inv_ln():
        return mp.mpf(1) if base == "e" else 1 / mp.log(mp.mpf(base))

    def fder(c, K):
        v = log1p_series_ders(c, K, 1, +1, inv_ln())
        v[0] -= K0
        return v
    return Spec("log_b(1+t)/t - K", fder,
                lambda lo, hi, K: log1p_series_bound(lo, hi, K, 1, inv_ln()),
                {k: v for k, v in enumerate(Q)}, a, b)


def sin_minus_r(S, rho):
    """sin r - r against r^3 S(r^2), r in [0, rho] (both sides odd)."""
    def fder(c, K):
        cyc = [mp.sin(c), mp.cos(c), -mp.sin(c), -mp.cos(c)]
        out = [cyc[k % 4] for k in range(K)]
        out[0] -= c
        if K > 1:
            out[1] -= 1
        return out
    return Spec("sin r - r", fder, lambda lo, hi, K: mp.mpf(1),
                {2 * k + 3: v for k, v in enumerate(S)}, 0, rho)


def cos_minus_1(C, rho):
    """cos r - 1 against r^2 C(r^2), r in [0, rho] (both sides even)."""
    def fder(c, K):
        cyc = [mp.cos(c), -mp.sin(c), -mp.cos(c), mp.sin(c)]
        out = [cyc[k % 4] for k in range(K)]
        out[0] -= 1
        return out
    return Spec("cos r - 1", fder, lambda lo, hi, K: mp.mpf(1),
                {2 * k + 2: v for k, v in enumerate(C)}, 0, rho)


def atan_minus_t(P, rho):
    """atan t - t against t^3 P(t^2), t in [0, rho] (both sides odd).
    atan^(n)(t) = (-1)^(n-1) (n-1)! Im (t - i)^-n for n >= 1, so
    |atan^(n)| <= (n-1)!."""
    def fder(c, K):
        out = [mp.atan(c) - c]
        for n in range(1, K):
            v = (-1) ** (n - 1) * mp.factorial(n - 1) * mp.im(mp.mpc(c, -1) ** (-n))
            out.append(v - (1 if n == 1 else 0))
        return out
    return Spec("atan t - t", fder, lambda lo, hi, K: mp.factorial(K - 1),
                {2 * k + 3: v for k, v in enumerate(P)}, 0, rho)
