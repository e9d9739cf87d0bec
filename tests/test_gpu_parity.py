"""GPU parity: every kernel path through the C ABI against the oracle,
bit-exact on residues, from the same seeded inputs and the same seeds for
the scheme's own randomness."""
import numpy as np
import pytest

import oracle as O
import synthetic as S
from oracle import encoding as OE
from oracle import nets as ON

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def ck():
    _gpu()
    from paper_2110_13638_amd import ckks
    return ckks


def _pair(ck, log_n, q_bits, p_bits, dnum, seed=3):
    primes = O.find_primes(log_n, list(q_bits) + list(p_bits))
    q, p = primes[: len(q_bits)], primes[len(q_bits):]
    ctx = ck.Context(log_n, q, p, dnum).keygen(seed)
    orc = O.Oracle(log_n, q, p, dnum)
    return ctx, orc


def _u(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("log_n", [10, 11, 12, 13, 14, 15])
def test_ntt_intt_bit_exact(ck, log_n):
    from paper_2110_13638_amd import _native as nat
    primes = O.find_primes(log_n, [60, 50, 40, 61 - 1, 36])
    orc = O.Oracle(log_n, primes[:4], primes[4:], 2)
    ctx = ck.Context(log_n, primes[:4], primes[4:], 2)
    n = 1 << log_n
    x = S.residues(log_n, primes, n)[0]
    print("ntt case log_n=%d primes=%s" % (log_n, primes), flush=True)
    dev = torch.from_numpy(x.view(np.int64)).cuda()
    ptrs = [dev[i].data_ptr() for i in range(len(primes))]
    ws, wb = ctx.ws_for(nat.CKKS_OP_NTT, len(primes))
    nat.ckks_ntt(ctx.h, ptrs, list(range(len(primes))), ws, wb, ctx.stream)
    torch.cuda.synchronize()
    got = _u(dev)
    for i in range(len(primes)):
        assert np.array_equal(got[i], orc.ntt(x[i], i)), "forward prime %d" % i
    nat.ckks_intt(ctx.h, ptrs, list(range(len(primes))), ws, wb, ctx.stream)
    torch.cuda.synchronize()
    assert np.array_equal(_u(dev), x)


@pytest.fixture(scope="module")
def small(ck):
    # the tiny configuration's chain at N = 2^12: [60, 40, 40 | 60], one prime per digit
    return _pair(ck, 12, [60, 40, 40], [60], 3)


@pytest.fixture(scope="module")
def wide(ck):
    # 50-bit chain with two special primes and four primes per digit
    return _pair(ck, 12, [50] * 16, [60, 60], 4)


def _keys_oracle(orc, seed):
    s, sn = orc.keygen_secret(seed)
    pk = orc.keygen_public(sn, seed + 1)
    rk = orc.keygen_relin(sn, seed + 2)
    return s, sn, pk, rk


@pytest.mark.parametrize("which", ["small", "wide"])
def test_keygen_bit_exact(request, which):
    ctx, orc = request.getfixturevalue(which)
    s, sn, pk, rk = _keys_oracle(orc, 3)
    assert np.array_equal(_u(ctx.sk), sn)
    assert np.array_equal(_u(ctx.pk), pk)
    assert np.array_equal(_u(ctx.rk), rk)
    g = ctx.galois_elt(3)
    assert g == orc.galois_elt(3)
    gk = ctx.add_galois_key(g, 41)
    assert np.array_equal(_u(gk), orc.keygen_galois(s, sn, g, 41))


def _enc_pair(ctx, orc, z, level, obj):
    m = ctx.encode_coeffs(z, ctx.default_scale)
    pt = ctx.pt_from_coeffs(m, level, ctx.default_scale)
    s, sn, pk, rk = _keys_oracle(orc, 3)
    pt_o = orc.reduce_int(m, level)
    assert np.array_equal(_u(pt.buf), pt_o)
    ct = ctx.encrypt(pt, seed=99, obj=obj)
    ct_o = orc.encrypt(pk, pt_o, level, 99, obj)
    return ct, ct_o, (s, sn, pk, rk)


def test_encode_matches_oracle_encoding(small):
    ctx, orc = small
    z = S.uniform_slots(5, ctx.N // 2) + 1j * S.uniform_slots(6, ctx.N // 2)
    m = ctx.encode_coeffs(z, ctx.default_scale)
    mo = OE.encode(z, ctx.default_scale, ctx.N)
    diff = np.abs(m - mo)
    # two independent FP64 embeddings may round a rare coefficient differently
    assert diff.max() <= 1 and np.mean(diff == 0) >= 0.999


@pytest.mark.parametrize("which", ["small", "wide"])
def test_encrypt_decrypt_bit_exact(request, which):
    ctx, orc = request.getfixturevalue(which)
    z = S.uniform_slots(7, ctx.N // 2)
    level = ctx.max_level
    ct, ct_o, keys = _enc_pair(ctx, orc, z, level, obj=5)
    assert np.array_equal(ct.residues(), ct_o)
    m = ctx.decrypt_residues(ct)
    assert np.array_equal(m, orc.decrypt(keys[1], ct_o))
    assert np.max(np.abs(ctx.decode(m, level, ct.scale).real - z)) < 2 ** -20


@pytest.mark.parametrize("which", ["small", "wide"])
def test_elementwise_bit_exact(request, which):
    ctx, orc = request.getfixturevalue(which)
    level = ctx.max_level
    a, ao, _ = _enc_pair(ctx, orc, S.uniform_slots(8, ctx.N // 2), level, 1)
    b, bo, _ = _enc_pair(ctx, orc, S.uniform_slots(9, ctx.N // 2), level, 2)
    assert np.array_equal(ctx.add(a, b).residues(), orc.add(ao, bo))
    assert np.array_equal(ctx.sub(a, b).residues(), orc.sub(ao, bo))
    t = ctx.multiply(a, b)
    assert t.n_poly == 3 and np.array_equal(t.residues(), orc.tensor(ao, bo))
    w = ctx.encode_coeffs(S.uniform_slots(10, ctx.N // 2), ctx.default_scale)
    pt = ctx.pt_from_coeffs(w, level, ctx.default_scale)
    pto = orc.reduce_int(w, level)
    assert np.array_equal(ctx.multiply_plain(a, pt).residues(), orc.mul_plain(ao, pto))
    assert np.array_equal(ctx.add_plain(a, pt).residues(), orc.add_plain(ao, pto))
    # expected constants from the oracle's own rounding (half away from zero)
    v = ON.round_half_away(-0.3 * ctx.default_scale)
    assert np.array_equal(ctx.multiply_scalar(a, -0.3).residues(), orc.mul_const(ao, v))
    v2 = ON.round_half_away(0.7 * a.scale)
    assert np.array_equal(ctx.add_scalar(a, 0.7).residues(), orc.add_const(ao, v2))


@pytest.mark.parametrize("which", ["small", "wide"])
def test_relin_rescale_rotate_bit_exact(request, which):
    ctx, orc = request.getfixturevalue(which)
    level = ctx.max_level
    za, zb = S.uniform_slots(11, ctx.N // 2), S.uniform_slots(12, ctx.N // 2)
    a, ao, keys = _enc_pair(ctx, orc, za, level, 1)
    b, bo, _ = _enc_pair(ctx, orc, zb, level, 2)
    rk = keys[3]
    t = ctx.multiply(a, b)
    to = orc.tensor(ao, bo)
    r = ctx.relinearize(t)
    ro = orc.relinearize(to, rk)
    assert np.array_equal(r.residues(), ro)
    rs = ctx.rescale(r)
    rso = orc.rescale(ro)
    assert np.array_equal(rs.residues(), rso)
    # rescale with a bias in the same pass: the oracle's rescale, then its
    # constant addition (a negative and a positive constant, two items)
    from paper_2110_13638_amd import _native as nat
    vs = [ON.round_half_away(-0.45 * rs.scale), ON.round_half_away(1.25 * rs.scale)]
    ins = [r, r]
    outs = [ctx.new_ct(2, r.level) for _ in ins]
    so = ctx._structs(outs)
    ws, wb = ctx.ws_for(nat.CKKS_OP_RESCALE, 2, [r.level, r.level])
    nat.ckks_rescale_add_scalar(ctx.h, ctx._structs(ins), vs, so, ws, wb, ctx.stream)
    for o, s_, v in zip(outs, so, vs):
        o.update(s_)
        assert o.level == rs.level and o.scale == rs.scale
        assert np.array_equal(o.residues(), orc.add_const(rso, v))
    # decoding is meaningful only where the special modulus exceeds a
    # digit's modulus (one prime per digit here); the wide chain (four
    # 50-bit primes per digit against two 60-bit special primes) is a
    # throughput configuration whose key-switch noise exceeds the message
    noise_valid = which == "small"
    if noise_valid:
        assert np.max(np.abs(ctx.decrypt(rs).real - za * zb)) < 2 ** -18
    # fused path equals the three calls
    f = ctx.hmult_relin_rescale([a], [b])[0]
    assert np.array_equal(f.residues(), rso)
    assert f.scale == rs.scale and f.level == rs.level
    # rotation and conjugation
    s, sn = keys[0], keys[1]
    for step in (1, -3):
        g = ctx.galois_elt(step)
        ctx.add_galois_key(g, 50 + step)
        rot = ctx.rotate(a, g=g)
        roto = orc.apply_galois(ao, g, orc.keygen_galois(s, sn, g, 50 + step))
        assert np.array_equal(rot.residues(), roto)
        if noise_valid:
            assert np.max(np.abs(ctx.decrypt(rot).real - np.roll(za, -step))) < 2 ** -18


def test_ragged_batched_hmult(wide):
    ctx, orc = wide
    levels = [l - 1 for l in S.ragged_limbs(13)]  # 4..16 limbs
    A, Bs, AO, BO = [], [], [], []
    for i, lv in enumerate(levels):
        res = S.residues(100 + i, ctx.q[: lv + 1], ctx.N, 4)
        AO.append(res[:2])
        BO.append(res[2:])
        A.append(ctx.ct_from_residues(res[:2]))
        Bs.append(ctx.ct_from_residues(res[2:]))
    outs = ctx.hmult_relin_rescale(A, Bs)
    _, _, _, rk = _keys_oracle(orc, 3)
    for i, lv in enumerate(levels):
        print("ragged case", i, "level", lv, flush=True)
        assert np.array_equal(outs[i].residues(), orc.mul_relin_rescale(AO[i], BO[i], rk)), i


# A 60-bit base prime as a ModUp source below N = 2^15: the FP64 engine
# splits such a source into two products in every ModUp kernel (generic and
# fixed digit size), for both transform shapes; one- and two-prime digits
# (one and two special primes), through HMult and a rotation.
@pytest.mark.parametrize("ntt_fp", [1, 0])
@pytest.mark.parametrize("wide", [0, 1])
@pytest.mark.parametrize("chain", ["one_prime_digits", "two_prime_digits"])
@pytest.mark.parametrize("log_n", [13, 14])
def test_hmult_60bit_modup_sources(ck, log_n, chain, wide, ntt_fp):
    if chain == "one_prime_digits":
        ctx, orc = _pair(ck, log_n, [60, 40, 40, 40], [60], 4)
    else:
        ctx, orc = _pair(ck, log_n, [60, 40, 40, 40], [60, 60], 2)
    ctx.set_tuning(ntt_wide=wide, ntt_fp=ntt_fp)
    s, sn, _, rk = _keys_oracle(orc, 3)
    lv = ctx.max_level
    A, Bs, AO, BO = [], [], [], []
    for i in range(3):
        res = S.residues(300 + i, ctx.q[: lv + 1], ctx.N, 4)
        AO.append(res[:2])
        BO.append(res[2:])
        A.append(ctx.ct_from_residues(res[:2]))
        Bs.append(ctx.ct_from_residues(res[2:]))
    print("60-bit source case log_n=%d %s wide=%d ntt_fp=%d" % (log_n, chain, wide, ntt_fp), flush=True)
    outs = ctx.hmult_relin_rescale(A, Bs)
    for i in range(3):
        assert np.array_equal(outs[i].residues(), orc.mul_relin_rescale(AO[i], BO[i], rk)), i
    # a rotation: key switch with the plain ModDown (one or two special primes)
    g = ctx.galois_elt(1)
    ctx.add_galois_key(g, 51)
    rot = ctx.rotate(A[0], g=g)
    assert np.array_equal(rot.residues(), orc.apply_galois(AO[0], g, orc.keygen_galois(s, sn, g, 51)))


def test_linear_bit_exact(small):
    ctx, orc = small
    level = ctx.max_level
    cts, cos = [], []
    for i in range(5):
        c, co, _ = _enc_pair(ctx, orc, S.uniform_slots(20 + i, ctx.N // 2), level, 10 + i)
        cts.append(c)
        cos.append(co)
    W = S.gaussian(3, (3, 5), 0.3)
    wants = []
    for j in range(3):
        want = None
        for i in range(5):
            term = orc.mul_const(cos[i], ON.round_half_away(W[j, i] * ctx.default_scale))
            want = term if want is None else orc.add(want, term)
        wants.append(want)
    # dense rows (matrix cores, then the VALU path), and ckks_linear with the
    # weights in device memory
    Wi = np.array([[ON.round_half_away(w * ctx.default_scale) for w in row] for row in W], dtype=np.int64)
    for mfma in (1, 0):
        ctx.set_tuning(lin_mfma=mfma)
        outs = ctx.linear(cts, W)
        for j in range(3):
            assert np.array_equal(outs[j].residues(), wants[j]), (mfma, j)
    ctx.set_tuning(lin_mfma=1)
    outs = ctx.linear_device_weights(cts, torch.from_numpy(Wi).to(ctx.device), ctx.default_scale)
    for j in range(3):
        assert np.array_equal(outs[j].residues(), wants[j]), j


def test_full_size_hmult_sampled(ck):
    # N = 2^15, 16 data primes of 50 bits + 2 special primes, dnum = 4:
    # the fused kernel at its benchmark shape, checked against the oracle
    ctx, orc = _pair(ck, 15, [50] * 16, [60, 60], 4, seed=5)
    _, _, _, rk = _keys_oracle(orc, 5)
    assert np.array_equal(_u(ctx.rk), rk)
    res = S.residues(77, ctx.q, ctx.N, 4)
    a, b = ctx.ct_from_residues(res[:2]), ctx.ct_from_residues(res[2:])
    out = ctx.hmult_relin_rescale([a, a], [b, b])
    want = orc.mul_relin_rescale(res[:2], res[2:], rk)
    assert np.array_equal(out[0].residues(), want)
    assert np.array_equal(out[1].residues(), want)


def test_wide_linear_no_accumulator_overflow(ck):
    # 2000 inputs with every residue q - 1 and weights -1 (= q - 1 mod q):
    # the exact sum of products exceeds 2^128 on the 60-bit prime, so the
    # kernel's running sums must be reduced along the way
    primes = O.find_primes(10, [60, 40, 60])
    q = primes[:2]
    ctx = ck.Context(10, q, primes[2:], 2)
    orc = O.Oracle(10, q, primes[2:], 2)
    n_in = 2000
    full = np.stack([np.full((1, ctx.N), qi - 1, dtype=np.uint64) for qi in q], axis=1)  # [1][2][N]
    one = np.concatenate([full, full])  # [2][2][N]
    cts = [ctx.ct_from_residues(one, 2.0 ** 40) for _ in range(n_in)]
    rows = np.zeros((2, n_in))
    rows[0, :] = -1.0 / 2 ** 40
    rows[1, ::2] = 3.0 / 2 ** 40
    wi = np.stack([np.full(n_in, -1), np.where(np.arange(n_in) % 2 == 0, 3, 0)]).astype(np.int64)
    for path in ("sparse", "dense", "device"):
        if path == "sparse":  # grouped VALU kernel (two different column lists)
            outs = ctx.linear_csr(cts, np.array([0, n_in, n_in + n_in // 2]),
                                  np.concatenate([np.arange(n_in), np.arange(0, n_in, 2)]),
                                  np.concatenate([np.full(n_in, -1), np.full(n_in // 2, 3)]).astype(np.int64), 2.0 ** 40)
        elif path == "dense":  # dense rows: the matrix cores
            outs = ctx.linear(cts, rows, w_scale=2.0 ** 40)
        else:  # weights in device memory: the VALU dense kernel
            outs = ctx.linear_device_weights(cts, torch.from_numpy(wi).to(ctx.device), 2.0 ** 40)
        for j, w in enumerate(([-1] * n_in, [3 if i % 2 == 0 else 0 for i in range(n_in)])):
            want = orc.lincomb([one] * n_in, w)
            assert np.array_equal(outs[j].residues(), want), (path, j)


def test_grouped_linear_row_groups(ck):
    # sparse rows whose column lists repeat in runs of 1..11 rows: the
    # grouped kernel's instantiations for groups of up to 2, 4, 5 and 8 rows
    # (runs above 8 split), on an FP64-engine prime and a 60-bit prime
    primes = O.find_primes(10, [60, 40, 60])
    q = primes[:2]
    ctx = ck.Context(10, q, primes[2:], 2).set_tuning(lin_mfma=0)
    orc = O.Oracle(10, q, primes[2:], 2)
    n_in = 40
    res = [S.residues(400 + i, q, ctx.N, 2) for i in range(n_in)]
    cts = [ctx.ct_from_residues(r, 2.0 ** 40) for r in res]
    rng = np.random.default_rng(5)
    for runs in ([1, 2, 1, 2], [3, 4, 1], [5, 5, 2], [7, 8, 11, 6]):
        rows = []
        for run in runs:
            cols = np.sort(rng.choice(n_in, size=int(rng.integers(1, 12)), replace=False))
            for _ in range(run):
                rows.append((cols, rng.integers(-(1 << 40), 1 << 40, size=len(cols))))
        row_ptr = np.concatenate([[0], np.cumsum([len(c) for c, _ in rows])])
        col = np.concatenate([c for c, _ in rows])
        w = np.concatenate([x for _, x in rows]).astype(np.int64)
        outs = ctx.linear_csr(cts, row_ptr, col, w, 2.0 ** 40)
        for j, (c, x) in enumerate(rows):
            want = orc.lincomb([res[i] for i in c], [int(v) for v in x])
            assert np.array_equal(outs[j].residues(), want), (runs, j)


@pytest.mark.parametrize("shape", [(845, 100), (37, 5), (64, 33)])
def test_dense_linear_matrix_cores_bit_exact(ck, shape):
    # dense rows (one shared column list) go to the int8-digit MFMA kernel:
    # bit-exact against the oracle's integer linear combination and against
    # the vector-ALU kernel, for odd sizes and negative weights
    n_in, n_out = shape
    primes = O.find_primes(12, [60, 40, 40, 60])
    ctx = ck.Context(12, primes[:3], primes[3:], 3)
    orc = O.Oracle(12, primes[:3], primes[3:], 3)
    ins = [S.residues(500 + i, ctx.q, ctx.N, 2) for i in range(n_in)]
    cts = [ctx.ct_from_residues(r, 2.0 ** 40) for r in ins]
    W = np.round(S.gaussian(7, (n_out, n_in), 0.1) * 2.0 ** 40).astype(np.int64)
    W[0, :] = -(2 ** 40)  # the largest weight magnitude the kernel takes
    row_ptr = np.arange(n_out + 1) * n_in
    col = np.tile(np.arange(n_in), n_out)
    outs = {}
    for mfma in (1, 0):
        ctx.set_tuning(lin_mfma=mfma)
        outs[mfma] = [o.residues().copy() for o in ctx.linear_csr(cts, row_ptr, col, W.reshape(-1), 2.0 ** 40)]
    ctx.set_tuning(lin_mfma=1)
    for j in range(n_out):
        want = orc.lincomb(ins, list(W[j]))
        assert np.array_equal(outs[1][j], want), j
        assert np.array_equal(outs[0][j], want), j


@pytest.mark.parametrize("ntt_fp", [1, 0])
def test_full_size_ragged_hmult(ck, ntt_fp):
    # N = 2^15, 16 x 50-bit + 2 x 60-bit primes, dnum 4 (four primes per
    # digit): a ragged batch of 13 pairs at 4..16 limbs, so the top digit
    # holds 1, 2, 3 or 4 primes and every fixed-size ModUp kernel runs;
    # both arithmetic engines, element-wise against the oracle
    ctx, orc = _pair(ck, 15, [50] * 16, [60, 60], 4, seed=5)
    _, _, _, rk = _keys_oracle(orc, 5)
    ctx.set_tuning(ntt_fp=ntt_fp)
    try:
        levels = [l - 1 for l in S.ragged_limbs(13)]
        A, Bs, AO, BO = [], [], [], []
        for i, lv in enumerate(levels):
            res = S.residues(300 + i, ctx.q[: lv + 1], ctx.N, 4)
            AO.append(res[:2])
            BO.append(res[2:])
            A.append(ctx.ct_from_residues(res[:2]))
            Bs.append(ctx.ct_from_residues(res[2:]))
        print("full-size ragged hmult ntt_fp=%d levels=%s" % (ntt_fp, levels), flush=True)
        outs = ctx.hmult_relin_rescale(A, Bs)
        for i, lv in enumerate(levels):
            assert np.array_equal(outs[i].residues(), orc.mul_relin_rescale(AO[i], BO[i], rk)), (i, lv)
    finally:
        ctx.set_tuning(ntt_fp=1)


@pytest.mark.parametrize("which", ["small", "wide"])
def test_conjugation_bit_exact(request, which):
    # Galois element 2N - 1 (complex conjugation of the slots)
    ctx, orc = request.getfixturevalue(which)
    level = ctx.max_level
    z = S.uniform_slots(13, ctx.N // 2) + 1j * S.uniform_slots(14, ctx.N // 2)
    m = ctx.encode_coeffs(z, ctx.default_scale)
    s, sn, pk, rk = _keys_oracle(orc, 3)
    ct = ctx.encrypt(ctx.pt_from_coeffs(m, level, ctx.default_scale), seed=99, obj=6)
    ct_o = orc.encrypt(pk, orc.reduce_int(m, level), level, 99, 6)
    g = 2 * ctx.N - 1
    ctx.add_galois_key(g, 77)
    got = ctx.rotate(ct, g=g)
    want = orc.apply_galois(ct_o, g, orc.keygen_galois(s, sn, g, 77))
    assert np.array_equal(got.residues(), want)
    if which == "small":
        dec = ctx.decode(ctx.decrypt_residues(got), level, got.scale)
        assert np.max(np.abs(dec - np.conj(z))) < 2 ** -18
