"""The FP64 transform schedule of the library, emulated exactly on the CPU.

The library runs transforms of primes below 2^50 in double precision
(van der Hoeven, Lecerf, Quintin, "Modular SIMD arithmetic in Mathemagix",
ACM TOMS 43(1), 2016): a residue is an integer-valued double, a product
y*w mod q is h = fl(y w), l = fma(y, w, -h), k = fl(y (w/q) + 1.5 2^52) -
1.5 2^52, r = fma(-k, q, h) + l, and transform values are re-centred
(x - q round(x / q)) on a fixed schedule: the forward Cooley-Tukey stages
re-centre X on stages s = 2 mod 3, the inverse Gentleman-Sande stages the
sum on every second executed stage, and the last inverse stage multiplies
both outputs by N^-1 and W^-1 N^-1. Twiddles are stored centred.

This file re-states that schedule independently of the library, executes
every double operation with exact rounding (Python floats are IEEE
doubles; an FMA is computed exactly with integers and rounded once), and
checks on the largest primes below 2^50 that
  * every value is an integer below 2^52 and every quotient takes the
    nearest integer (|y w/q| < 2^51),
  * the outputs equal the oracle's transform bit for bit,
and, separately, that a worst-case bound propagation over the schedule
(every product at its largest possible magnitude) stays inside the same
limits for every ring degree, for inputs below q and below 2q.
"""
import numpy as np
import pytest

import oracle as O

K_ROUND = 6755399441055744.0  # 1.5 * 2^52
TWO51 = float(2 ** 51)
TWO52 = float(2 ** 52)


def fma(a, b, c):
    """a * b + c rounded once to double (a, b, c doubles)"""
    na, da = a.as_integer_ratio()
    nb, db = b.as_integer_ratio()
    nc, dc = c.as_integer_ratio()
    return (na * nb * dc + nc * da * db) / (da * db * dc)


class Tracker:
    def __init__(self):
        self.max_abs = 0.0      # largest |value| seen
        self.max_quot = 0.0     # largest |y * (w/q)| before the rounding constant

    def see(self, v):
        a = abs(v)
        assert a == int(a) and a < TWO52, v
        if a > self.max_abs:
            self.max_abs = a


def mulmod(y, w, wq, q, tr):
    h = y * w
    l = fma(y, w, -h)
    tr.max_quot = max(tr.max_quot, abs(y * wq))
    k = fma(y, wq, K_ROUND) - K_ROUND
    r = fma(-k, q, h) + l
    # exactness: the double result is the integer y w - k q
    assert int(r) == int(y) * int(w) - int(k) * int(q), (y, w, k)
    tr.see(r)
    return r


def centre(x, q, qinv):
    k = fma(x, qinv, K_ROUND) - K_ROUND
    r = fma(-k, q, x)
    assert int(r) == int(x) - int(k) * int(q)
    return r


def centred(v, q):
    return float(v - q) if v > q // 2 else float(v)


def tables(q, logn):
    n = 1 << logn
    psi = O.min_psi(q, logn)
    pw = [pow(psi, k, q) for k in range(n)]
    brv = [int(format(k, "0%db" % logn)[::-1], 2) for k in range(n)]
    tw = [pw[brv[k]] for k in range(n)]
    itw = [pow(t, q - 2, q) for t in tw]
    qd = float(q)
    twf = [(centred(t, q), centred(t, q) / qd) for t in tw]
    itwf = [(centred(t, q), centred(t, q) / qd) for t in itw]
    ninv = pow(n, q - 2, q)
    last = itw[1] * ninv % q
    return twf, itwf, (centred(ninv, q), centred(ninv, q) / qd), (centred(last, q), centred(last, q) / qd)


def forward(a, q, logn, twf, tr):
    n = 1 << logn
    qd, qinv = float(q), 1.0 / float(q)
    r = [float(x) for x in a]
    for s in range(logn):
        half = n >> (s + 1)
        for g in range(1 << s):
            w, wq = twf[(1 << s) + g]
            for j in range(half):
                x = g * 2 * half + j
                y = x + half
                X = r[x]
                if s % 3 == 2:
                    X = centre(X, qd, qinv)
                T = mulmod(r[y], w, wq, qd, tr)
                r[x] = X + T
                r[y] = X - T
                tr.see(r[x])
                tr.see(r[y])
    out = []
    for v in r:
        c = centre(v, qd, qinv)
        assert abs(c) < qd
        out.append(int(c) % q)
    return out


def inverse(a, q, logn, itwf, ninv, last, tr):
    n = 1 << logn
    qd, qinv = float(q), 1.0 / float(q)
    r = [float(x) for x in a]
    for s in range(logn - 1, -1, -1):
        half = n >> (s + 1)
        rec = ((logn - 1 - s) & 1) == 1
        for g in range(1 << s):
            w, wq = itwf[(1 << s) + g]
            for j in range(half):
                x = g * 2 * half + j
                y = x + half
                X, Y = r[x], r[y]
                tr.see(X + Y)
                tr.see(X - Y)
                if s == 0:
                    r[x] = mulmod(X + Y, ninv[0], ninv[1], qd, tr)
                    r[y] = mulmod(X - Y, last[0], last[1], qd, tr)
                else:
                    U = X + Y
                    r[x] = centre(U, qd, qinv) if rec else U
                    r[y] = mulmod(X - Y, w, wq, qd, tr)
                    tr.see(r[x])
    out = []
    for v in r:
        assert abs(v) < qd  # the final conversion needs |v| < q
        out.append(int(v) % q)
    return out


def _largest_prime(logn):
    return O.find_primes(logn, [50])[0]


def _inputs(q, n):
    rng = np.random.default_rng(11)
    return {
        "all q-1": [q - 1] * n,
        "alternating": [(q - 1) if j % 2 else 0 for j in range(n)],
        "half blocks": [(q - 1) if j < n // 2 else (q - 1) // 2 for j in range(n)],
        "random": [int(v) for v in rng.integers(0, q, n, dtype=np.uint64)],
    }


@pytest.mark.parametrize("logn", [10, 12])
def test_fp64_schedule_exact_and_bit_identical(logn):
    q = _largest_prime(logn)
    assert q > 2 ** 50 - 2 ** 20
    n = 1 << logn
    orc = O.Oracle(logn, [q], [O.find_primes(logn, [60])[0]], 1)
    twf, itwf, ninv, last = tables(q, logn)
    for name, a in _inputs(q, n).items():
        tr = Tracker()
        f = forward(a, q, logn, twf, tr)
        assert np.array_equal(np.array(f, dtype=np.uint64), orc.ntt(np.array(a, dtype=np.uint64), 0)), name
        back = inverse(f, q, logn, itwf, ninv, last, tr)
        assert back == [x % q for x in a], name
        assert tr.max_quot < TWO51, (name, tr.max_quot / q)
        assert tr.max_abs < 4 * q, (name, tr.max_abs / q)


@pytest.mark.slow
def test_fp64_schedule_exact_at_n32768():
    logn = 15
    q = _largest_prime(logn)
    n = 1 << logn
    orc = O.Oracle(logn, [q], [O.find_primes(logn, [60])[0]], 1)
    twf, itwf, ninv, last = tables(q, logn)
    a = _inputs(q, n)["random"]
    tr = Tracker()
    f = forward(a, q, logn, twf, tr)
    assert np.array_equal(np.array(f, dtype=np.uint64), orc.ntt(np.array(a, dtype=np.uint64), 0))
    assert inverse(f, q, logn, itwf, ninv, last, tr) == a
    assert tr.max_quot < TWO51 and tr.max_abs < 4 * q


def _prod_bound(q, yb):
    """|y w - k q| for |y| <= yb: q (1/2 + |y| 2^-54) while |y| / 2 < 2^51
    (|w/q| <= 1/2 keeps the quotient rounding to nearest)"""
    assert yb / 2 < TWO51, "quotient may not round to nearest"
    return q * (0.5 + yb * 2.0 ** -54)


def _forward_worst(logn, q, in_bound):
    """Largest magnitude any forward value can reach when every product
    takes its worst rounding (re-centring gives <= q/2 + 1)."""
    b = peak = in_bound
    for s in range(logn):
        xb = q / 2 + 1 if s % 3 == 2 else b
        b = xb + _prod_bound(q, b)
        peak = max(peak, b)
    assert peak < TWO52
    return peak


def _inverse_worst(logn, q, in_bound):
    """The same for the inverse; also checks the last stage leaves |v| < q."""
    b = peak = in_bound
    for s in range(logn - 1, -1, -1):
        rec = ((logn - 1 - s) & 1) == 1
        sb = 2 * b
        peak = max(peak, sb)
        if s == 0:
            assert _prod_bound(q, sb) < q
        else:
            b = max(q / 2 + 1 if rec else sb, _prod_bound(q, sb))
    assert peak < TWO52
    return peak


@pytest.mark.parametrize("logn", range(10, 16))
def test_fp64_schedule_worst_case_bounds(logn):
    q = float(2 ** 50 - 1)  # every prime the engine takes is below this
    # plain inputs in [0, q); ModUp / ModDown sums enter the forward
    # transform below 2q; the inverse takes residues or products <= 0.75 q
    assert _forward_worst(logn, q, q) < 2.5 * q
    assert _forward_worst(logn, q, 2 * q) < 3.5 * q
    assert _inverse_worst(logn, q, q) <= 4 * q
