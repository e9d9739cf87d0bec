"""Pins for the oracle against facts that do not come from the oracle:
published known answers, closed forms, brute force on tiny inputs, exact
big-integer definitions and homomorphic invariants.

Each test names what pins it. All run on the CPU.
"""
import os

import numpy as np
import pytest
import sympy

import oracle as O
from oracle import encoding as E

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def brv(x, bits):
    return int(format(x, "0%db" % bits)[::-1], 2) if bits else 0


# ---------------------------------------------------------------------------
# randomness: Philox4x32-10 published known answers, sampler distributions
# ---------------------------------------------------------------------------
def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLD, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert O.philox4x32_10(v[0:4], v[4:6]) == v[6:10]


def test_samplers_distribution():
    n = 1 << 15
    t = O.sample_ternary(7, 0, O.TAG_SK, n)
    assert set(np.unique(t)) <= {-1, 0, 1}
    for v in (-1, 0, 1):
        assert abs(np.mean(t == v) - 1 / 3) < 0.02
    e = O.sample_cbd(7, 0, O.TAG_PK_E, n)
    # centred binomial with eta=21: mean 0, variance 21/2, |e| <= 21
    assert np.abs(e).max() <= 21
    assert abs(e.mean()) < 0.1
    assert abs(e.var() - 10.5) < 0.5
    q = 1125899904679937
    u = O.sample_uniform(7, 0, O.TAG_PK_A, 3, n, q)
    assert u.max() < q
    assert abs(float(u.astype(np.float64).mean()) / q - 0.5) < 0.01
    # different limbs / tags / objects give different streams
    assert not np.array_equal(u, O.sample_uniform(7, 0, O.TAG_PK_A, 4, n, q))
    assert not np.array_equal(t, O.sample_ternary(7, 1, O.TAG_SK, n))


# ---------------------------------------------------------------------------
# primes and roots (prime choice rule, smallest root), pinned with sympy's primality test
# ---------------------------------------------------------------------------
def _primes_by_rule_sympy(logn, bits):
    two_n = 2 << logn
    out = []
    for b in bits:
        c = ((2 ** b - 1) // two_n) * two_n + 1
        while not (sympy.isprime(c) and c not in out):
            c -= two_n
        out.append(c)
    return out


@pytest.mark.parametrize("logn,bits", [
    (13, [60, 40, 40, 60]),
    (14, [60] + [40] * 7 + [60]),
    (15, [50] * 16 + [60, 60]),
    (4, [30, 20, 20, 30]),
])
def test_prime_rule(logn, bits):
    got = O.find_primes(logn, bits)
    assert got == _primes_by_rule_sympy(logn, bits)
    for q, b in zip(got, bits):
        assert q % (2 << logn) == 1 and q.bit_length() == b


def test_min_psi_brute_force():
    # tiny primes: scan every candidate below psi
    for logn in (2, 3, 4):
        for q in O.find_primes(logn, [12, 14, 16]):
            psi = O.min_psi(q, logn)
            n = 1 << logn
            assert pow(psi, n, q) == q - 1
            assert all(pow(x, n, q) != q - 1 for x in range(2, psi))
    # a 60-bit prime at N=1024: minimum over all N odd powers of a root
    logn, n = 10, 1024
    q = O.find_primes(logn, [60])[0]
    psi = O.min_psi(q, logn)
    assert pow(psi, n, q) == q - 1
    assert psi == min(pow(psi, k, q) for k in range(1, 2 * n, 2))


# ---------------------------------------------------------------------------
# NTT: direct evaluation, schoolbook negacyclic convolution, inverse
# ---------------------------------------------------------------------------
def _tiny(logn, bits=(40, 30)):
    q = O.find_primes(logn, list(bits))
    return O.Oracle(logn, q[:1], q[1:], 1), q


@pytest.mark.parametrize("logn", [3, 4, 5, 6])
def test_ntt_direct_evaluation(logn):
    orc, q = _tiny(logn)
    n, qq = 1 << logn, q[0]
    rng = np.random.default_rng(logn)
    a = rng.integers(0, qq, n, dtype=np.uint64)
    got = orc.ntt(a, 0)
    psi = orc.psi(0)
    for k in range(n):
        x = pow(psi, 2 * brv(k, logn) + 1, qq)
        want = sum(int(a[j]) * pow(x, j, qq) for j in range(n)) % qq
        assert int(got[k]) == want


def _schoolbook_negacyclic(a, b, q):
    n = len(a)
    c = [0] * n
    for i in range(n):
        for j in range(n):
            k = i + j
            if k < n:
                c[k] += int(a[i]) * int(b[j])
            else:
                c[k - n] -= int(a[i]) * int(b[j])
    return [x % q for x in c]


@pytest.mark.parametrize("logn", [3, 4, 5, 6])
def test_ntt_convolution(logn):
    orc, q = _tiny(logn, (60, 50))
    n = 1 << logn
    rng = np.random.default_rng(100 + logn)
    for pi, qq in enumerate(q):
        a = rng.integers(0, qq, n, dtype=np.uint64)
        b = rng.integers(0, qq, n, dtype=np.uint64)
        fa, fb = orc.ntt(a, pi), orc.ntt(b, pi)
        prod = np.array([(int(x) * int(y)) % qq for x, y in zip(fa, fb)], dtype=np.uint64)
        assert [int(v) for v in orc.intt(prod, pi)] == _schoolbook_negacyclic(a, b, qq)


def test_ntt_roundtrip_large():
    q = O.find_primes(13, [60, 40, 60])
    orc = O.Oracle(13, q[:2], q[2:], 2)
    rng = np.random.default_rng(5)
    for pi in range(3):
        a = rng.integers(0, q[pi], 1 << 13, dtype=np.uint64)
        assert np.array_equal(orc.intt(orc.ntt(a, pi), pi), a)


# ---------------------------------------------------------------------------
# encoding: direct O(N^2) embedding, constants, conjugate symmetry
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("logn", [3, 4, 5])
def test_encode_direct_embedding(logn):
    n = 1 << logn
    scale = 2.0 ** 30
    rng = np.random.default_rng(logn)
    z = rng.uniform(-1, 1, n // 2) + 1j * rng.uniform(-1, 1, n // 2)
    m = E.encode(z, scale, n)
    zeta = np.exp(1j * np.pi / n)
    for j in range(n // 2):
        root = zeta ** pow(5, j, 2 * n)
        val = sum(float(m[i]) * root ** i for i in range(n))
        # rounding each coefficient moves each slot by at most n/2
        assert abs(val - scale * z[j]) <= n / 2 + 1e-6 * scale
    assert np.allclose(E.decode(m, scale, n), z, atol=n / scale)


def test_encode_constant_and_real():
    n, scale = 64, 2.0 ** 40
    m = E.encode(np.full(n // 2, 0.3125), scale, n)
    assert m[0] == round(0.3125 * scale) and not np.any(m[1:])
    # real slot values give a real polynomial whose decode has no imaginary part
    z = np.linspace(-1, 1, n // 2)
    d = E.decode(E.encode(z, scale, n), scale, n)
    assert np.max(np.abs(d.imag)) < 1e-9 and np.max(np.abs(d.real - z)) < 1e-9


def test_encode_rotation_is_galois():
    # rotating slots left by r equals X -> X^(5^r): pins the slot order
    n, scale = 32, 2.0 ** 20
    rng = np.random.default_rng(2)
    z = rng.uniform(-1, 1, n // 2)
    m = E.encode(z, scale, n)
    for r in (1, 3, 7):
        g = pow(5, r, 2 * n)
        mg = np.zeros(n, dtype=np.int64)
        for j in range(n):
            e = j * g % (2 * n)
            if e < n:
                mg[e] = m[j]
            else:
                mg[e - n] = -m[j]
        assert np.allclose(E.decode(mg, scale, n).real, np.roll(z, -r), atol=1e-4)


def test_crt_lift_roundtrip():
    q = O.find_primes(4, [60, 40, 40, 40])
    Q = 1
    for x in q:
        Q *= x
    rng = np.random.default_rng(3)
    xs = [int(rng.integers(-2 ** 62, 2 ** 62)) * int(rng.integers(1, 2 ** 60)) for _ in range(16)]
    xs[0], xs[1] = Q // 2, -(Q // 2) + 1
    res = [[x % qi for x in xs] for qi in q]
    assert E.crt_lift_centered(res, q) == xs


# ---------------------------------------------------------------------------
# residue-level ops against exact big-integer definitions
# ---------------------------------------------------------------------------
def _lift(res, primes):
    """non-centred CRT value in [0, Q)"""
    Q = 1
    for p in primes:
        Q *= p
    return [(x % Q) for x in E.crt_lift_centered(res, primes)], Q


def _coeff(orc, ct):
    """NTT-form [P][L][N] -> coefficient form"""
    out = np.zeros_like(ct)
    for p in range(ct.shape[0]):
        for i in range(ct.shape[1]):
            out[p, i] = orc.intt(ct[p, i], i)
    return out


def test_rescale_is_rounded_division():
    logn = 4
    q = O.find_primes(logn, [60, 40, 40, 60])
    orc = O.Oracle(logn, q[:3], q[3:], 3)
    n = 1 << logn
    rng = np.random.default_rng(4)
    for level in (1, 2):
        ct = np.stack([np.stack([rng.integers(0, q[i], n, dtype=np.uint64) for i in range(level + 1)])
                       for _ in range(2)])
        out = orc.rescale(ct)
        cin, cout = _coeff(orc, ct), _coeff(orc, out)
        ql = q[level]
        for p in range(2):
            vals, _ = _lift(cin[p], q[: level + 1])
            got, Qo = _lift(cout[p], q[:level])
            want = [((v + ql // 2) // ql) % Qo for v in vals]
            assert got == want


def test_modup_is_exact_lift_plus_small_multiple():
    logn = 3
    q = O.find_primes(logn, [50, 50, 50, 50, 60, 60])
    orc = O.Oracle(logn, q[:4], q[4:], 2)  # alpha = 2
    n = 1 << logn
    rng = np.random.default_rng(6)
    x = np.stack([rng.integers(0, q[i], n, dtype=np.uint64) for i in (2, 3)])
    QD = q[2] * q[3]
    X, _ = _lift(x, q[2:4])
    for t in (0, 1, 4, 5):
        got = orc.modup_digit(x, 2, 4, t)
        for j in range(n):
            # approximate conversion = X + u*Q_D with 0 <= u < alpha
            assert any((X[j] + u * QD) % q[t] == int(got[j]) for u in range(2))
    # on its own primes it is the identity
    got2 = orc.modup_digit(x, 2, 4, 2)
    assert np.array_equal(got2, x[0])


def test_moddown_is_division_by_P():
    logn = 3
    q = O.find_primes(logn, [50, 50, 60, 60])
    orc = O.Oracle(logn, q[:2], q[2:], 2)
    n = 1 << logn
    rng = np.random.default_rng(8)
    level = 1
    a = np.stack([rng.integers(0, q[i], n, dtype=np.uint64) for i in range(4)])
    a_ntt = np.stack([orc.ntt(a[i], i) for i in range(4)])
    out = orc.moddown(a_ntt, level)
    r = np.stack([orc.intt(out[i], i) for i in range(2)])
    A, QP = _lift(a, q)
    R, Qq = _lift(r, q[:2])
    P = q[2] * q[3]
    for j in range(n):
        # R*P + (A mod P) + v*P == A (mod Q) for some 0 <= v < k
        assert any((R[j] * P + A[j] % P + v * P - A[j]) % Qq == 0 for v in range(2))


def test_tensor_and_pointwise_exact():
    logn = 3
    q = O.find_primes(logn, [60, 50, 60])
    orc = O.Oracle(logn, q[:2], q[2:], 2)
    n = 1 << logn
    rng = np.random.default_rng(9)
    a = np.stack([np.stack([rng.integers(0, q[i], n, dtype=np.uint64) for i in range(2)]) for _ in range(2)])
    b = np.stack([np.stack([rng.integers(0, q[i], n, dtype=np.uint64) for i in range(2)]) for _ in range(2)])
    t = orc.tensor(a, b)
    s = orc.add(a, b)
    d = orc.sub(a, b)
    m = orc.mul_const(a, -12345)
    for i in range(2):
        for j in range(n):
            A0, A1, B0, B1 = (int(a[0, i, j]), int(a[1, i, j]), int(b[0, i, j]), int(b[1, i, j]))
            assert int(t[0, i, j]) == A0 * B0 % q[i]
            assert int(t[1, i, j]) == (A0 * B1 + A1 * B0) % q[i]
            assert int(t[2, i, j]) == A1 * B1 % q[i]
            assert int(s[1, i, j]) == (A1 + B1) % q[i]
            assert int(d[0, i, j]) == (A0 - B0) % q[i]
            assert int(m[1, i, j]) == (A1 * -12345) % q[i]


# ---------------------------------------------------------------------------
# scheme-level invariants: keys, encryption, key switching, rotation
# ---------------------------------------------------------------------------
class Scheme:
    def __init__(self, logn=5, bits=(60, 40, 40, 60), n_p=1, dnum=None, seed=11):
        q = O.find_primes(logn, list(bits))
        n_q = len(bits) - n_p
        self.orc = O.Oracle(logn, q[:n_q], q[n_q:], dnum or n_q)
        self.q = q
        self.n = 1 << logn
        self.s, self.sn = self.orc.keygen_secret(seed)
        self.pk = self.orc.keygen_public(self.sn, seed + 1)
        self.rk = self.orc.keygen_relin(self.sn, seed + 2)
        self.scale = 2.0 ** 40

    def enc(self, z, level, obj, scale=None):
        m = E.encode(z, scale or self.scale, self.n)
        return self.orc.encrypt(self.pk, self.orc.reduce_int(m, level), level, 99, obj)

    def dec(self, ct, scale):
        m = self.orc.decrypt(self.sn, ct)
        return E.decode_residues(m, self.q, scale, self.n)


@pytest.fixture(scope="module")
def sch():
    return Scheme()


def test_secret_and_public_key(sch):
    assert set(np.unique(sch.s)) <= {-1, 0, 1}
    # b + a*s = e, small (CBD bound 21) in the coefficient domain
    for i in range(sch.orc.n_q):
        qi = sch.q[i]
        v = np.array([(int(b) + int(a) * int(s)) % qi for b, a, s in
                      zip(sch.pk[0, i], sch.pk[1, i], sch.sn[i])], dtype=np.uint64)
        e = sch.orc.intt(v, i)
        cen = [int(x) if x <= qi // 2 else int(x) - qi for x in e]
        assert max(abs(x) for x in cen) <= 21


def test_encrypt_decrypt(sch):
    rng = np.random.default_rng(12)
    z = rng.uniform(-1, 1, sch.n // 2)
    for level in (0, 1, 2):
        ct = sch.enc(z, level, obj=level)
        m = sch.orc.decrypt(sch.sn, ct)
        want = E.encode(z, sch.scale, sch.n)
        got = E.crt_lift_centered(m, sch.q)
        noise = max(abs(g - int(w)) for g, w in zip(got, want))
        assert noise < 2 ** 16  # fresh noise: |v e + e0 + e1 s| << N * 21 * 3
        assert np.max(np.abs(sch.dec(ct, sch.scale) - z)) < 2 ** -20


def test_keyswitch_semantics():
    # <KS(d), (1, s)> - d s' is small for alpha = 2, k = 2 (valid noise)
    sc = Scheme(logn=4, bits=(50, 50, 50, 50, 60, 60), n_p=2, dnum=2)
    orc, n = sc.orc, sc.n
    rng = np.random.default_rng(13)
    level = 3
    d = np.stack([rng.integers(0, sc.q[i], n, dtype=np.uint64) for i in range(level + 1)])
    s2 = np.stack([np.array([int(x) * int(x) % sc.q[i] for x in sc.sn[i]], dtype=np.uint64)
                   for i in range(len(sc.q))])
    ks = orc.keyswitch(d, sc.rk)
    diff = np.zeros((level + 1, n), dtype=np.uint64)
    for i in range(level + 1):
        qi = sc.q[i]
        diff[i] = [(int(k0) + int(k1) * int(s) - int(dd) * int(t)) % qi for k0, k1, s, dd, t in
                   zip(ks[0, i], ks[1, i], sc.sn[i], d[i], s2[i])]
        diff[i] = orc.intt(diff[i], i)
    err = E.crt_lift_centered(diff, sc.q)
    # bound: alpha * N * 21 * (Q_D / P) + k N (Q_D ~ 2^100, P ~ 2^120)
    assert max(abs(x) for x in err) < 2 ** 16


def test_relin_and_mul_relin_rescale(sch):
    rng = np.random.default_rng(14)
    za = rng.uniform(-1, 1, sch.n // 2)
    zb = rng.uniform(-1, 1, sch.n // 2)
    a, b = sch.enc(za, 2, 1), sch.enc(zb, 2, 2)
    t = sch.orc.tensor(a, b)
    assert np.max(np.abs(sch.dec(t, sch.scale ** 2) - za * zb)) < 2 ** -18
    r = sch.orc.relinearize(t, sch.rk)
    assert np.max(np.abs(sch.dec(r, sch.scale ** 2) - za * zb)) < 2 ** -18
    out = sch.orc.mul_relin_rescale(a, b, sch.rk)
    assert np.array_equal(out, sch.orc.rescale(r))
    assert np.max(np.abs(sch.dec(out, sch.scale ** 2 / sch.q[2]) - za * zb)) < 2 ** -18


def test_rotation_and_composition(sch):
    rng = np.random.default_rng(15)
    z = rng.uniform(-1, 1, sch.n // 2)
    ct = sch.enc(z, 2, 3)
    for r in (1, 5, -1):
        g = sch.orc.galois_elt(r)
        gk = sch.orc.keygen_galois(sch.s, sch.sn, g, 77)
        rot = sch.orc.apply_galois(ct, g, gk)
        assert np.max(np.abs(sch.dec(rot, sch.scale).real - np.roll(z, -r))) < 2 ** -18
    g1, g2 = sch.orc.galois_elt(2), sch.orc.galois_elt(3)
    k1 = sch.orc.keygen_galois(sch.s, sch.sn, g1, 78)
    k2 = sch.orc.keygen_galois(sch.s, sch.sn, g2, 79)
    two = sch.orc.apply_galois(sch.orc.apply_galois(ct, g1, k1), g2, k2)
    assert np.max(np.abs(sch.dec(two, sch.scale).real - np.roll(z, -5))) < 2 ** -18
    # conjugation: g = 2N - 1 on complex slots
    zc = z + 1j * rng.uniform(-1, 1, sch.n // 2)
    ctc = sch.enc(zc, 2, 4)
    gc = 2 * sch.n - 1
    kc = sch.orc.keygen_galois(sch.s, sch.sn, gc, 80)
    conj = sch.orc.apply_galois(ctc, gc, kc)
    assert np.max(np.abs(sch.dec(conj, sch.scale) - np.conj(zc))) < 2 ** -18


def test_automorph_ntt_matches_coefficient_rule():
    # the NTT-domain automorphism composed with the NTT is the signed
    # coefficient permutation, checked here on Python integers
    logn = 4
    q = O.find_primes(logn, [60, 60])
    orc = O.Oracle(logn, q[:1], q[1:], 1)
    n = 1 << logn
    rng = np.random.default_rng(16)
    a = rng.integers(0, q[0], n, dtype=np.uint64)
    for g in (5, 25, 2 * n - 1):
        got = orc.intt(orc.automorph_ntt(orc.ntt(a, 0), 0, g), 0)
        want = [0] * n
        for j in range(n):
            e = j * g % (2 * n)
            if e < n:
                want[e] = int(a[j])
            else:
                want[e - n] = (-int(a[j])) % q[0]
        assert [int(x) for x in got] == want


def test_plain_ops_homomorphic(sch):
    rng = np.random.default_rng(17)
    z = rng.uniform(-1, 1, sch.n // 2)
    w = rng.uniform(-1, 1, sch.n // 2)
    ct = sch.enc(z, 2, 5)
    pt = sch.orc.reduce_int(E.encode(w, sch.scale, sch.n), 2)
    assert np.max(np.abs(sch.dec(sch.orc.mul_plain(ct, pt), sch.scale ** 2) - z * w)) < 2 ** -18
    assert np.max(np.abs(sch.dec(sch.orc.add_plain(ct, pt), sch.scale) - (z + w))) < 2 ** -18
    c = round(-0.75 * sch.scale)
    assert np.max(np.abs(sch.dec(sch.orc.mul_const(ct, c), sch.scale ** 2) + 0.75 * z)) < 2 ** -18
    assert np.max(np.abs(sch.dec(sch.orc.add_const(ct, c), sch.scale) - (z - 0.75))) < 2 ** -18
