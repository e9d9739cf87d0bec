"""Serialisation round trips through host bytes: ciphertexts, plaintexts
and keys come back bit-identical, the payload of an encrypted ciphertext
equals the oracle's ciphertext of the same plaintext and seeds, and bytes of
one context are refused by another."""
import numpy as np
import pytest

import oracle as O
import synthetic as S
from oracle import encoding as E

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_13638_amd import ckks
    primes = O.find_primes(12, [60, 40, 40, 60])
    ctx = ckks.Context(12, primes[:3], primes[3:], 3).keygen(3)
    orc = O.Oracle(12, primes[:3], primes[3:], 3)
    return ckks, ctx, orc


def test_ciphertext_round_trip_matches_oracle(env):
    ckks, ctx, orc = env
    z = S.uniform_slots(1, ctx.N // 2)
    m = E.encode(z, 2.0 ** 40, ctx.N)
    ct = ctx.encrypt(ctx.pt_from_coeffs(m, 2, 2.0 ** 40), seed=9, obj=4)
    data = ctx.serialize(ct)
    assert len(data) == 64 + 2 * 3 * ctx.N * 8
    # payload = the oracle's ciphertext of the same plaintext and seeds
    _, sn = orc.keygen_secret(3)
    pk = orc.keygen_public(sn, 4)
    want = orc.encrypt(pk, orc.reduce_int(m, 2), 2, 9, 4)
    assert np.array_equal(np.frombuffer(data[64:], dtype=np.uint64).reshape(2, 3, ctx.N), want)
    back = ctx.deserialize(data)
    assert back.level == 2 and back.scale == ct.scale and back.n_poly == 2
    assert np.array_equal(back.residues(), ct.residues())
    assert np.max(np.abs(ctx.decrypt(back).real - z)) < 2 ** -18
    # into a buffer with a wider limb stride
    wide = ctx.deserialize(data, level=2)
    assert np.array_equal(wide.residues(), ct.residues())


def test_key_and_plaintext_round_trip(env):
    ckks, ctx, orc = env
    from paper_2110_13638_amd import _native as nat
    data = nat.ckks_serialize(ctx.h, nat.CKKS_OBJ_KEY, ctx.rk.data_ptr(), nat.CKKS_KEY_SWITCH, ctx.stream)
    rk2 = torch.zeros_like(ctx.rk)
    nat.ckks_deserialize(ctx.h, nat.CKKS_OBJ_KEY, data, rk2.data_ptr(), nat.CKKS_KEY_SWITCH, ctx.stream)
    assert torch.equal(rk2, ctx.rk)
    with pytest.raises(nat.CkksError):  # wrong key kind for these bytes
        nat.ckks_deserialize(ctx.h, nat.CKKS_OBJ_KEY, data, rk2.data_ptr(), nat.CKKS_KEY_PUBLIC, ctx.stream)
    m = E.encode(S.uniform_slots(2, ctx.N // 2), 2.0 ** 40, ctx.N)
    pt = ctx.pt_from_coeffs(m, 1, 2.0 ** 40)
    pdata = nat.ckks_serialize(ctx.h, nat.CKKS_OBJ_PT, pt.struct(), 0, ctx.stream)
    buf = torch.zeros_like(pt.buf)
    s = nat.ckks_pt(buf.data_ptr(), 0, 0, 0.0)
    nat.ckks_deserialize(ctx.h, nat.CKKS_OBJ_PT, pdata, s, 0, ctx.stream)
    assert s.level == 1 and s.scale == 2.0 ** 40 and torch.equal(buf, pt.buf)


def test_other_context_refuses_bytes(env):
    ckks, ctx, orc = env
    from paper_2110_13638_amd import _native as nat
    primes = O.find_primes(12, [60, 40, 36, 60])
    other = ckks.Context(12, primes[:3], primes[3:], 3)
    ct = ctx.encrypt(ctx.encode(S.uniform_slots(3, ctx.N // 2)), seed=1)
    data = ctx.serialize(ct)
    with pytest.raises(nat.CkksError) as e:
        other.deserialize(data)
    assert e.value.code == nat.CKKS_EPARAMS
