"""Pins of the oracle's linear layer (Sections 4.2.2-4.2.3: conv and dense
nodes are sums of ciphertext x weight products plus a bias).

* ``orc_lincomb`` against its definition written with Python big
  integers: out[t][i][j] = sum_k w_k ct_k[t][i][j] mod q_i, with negative
  weights, weights near 2^62 and 2000 inputs of residue q - 1 (whose exact
  sum of products is far beyond 128 bits).
* The oracle's vision lowering (``oracle.nets.linear`` for the strided conv
  and both dense layers, ``oracle.nets.square`` for x^2) at N = 2^10,
  decrypted and decoded against the FP64 network as written
  (``plainnet.vision_math``) within 2^-18 max(1, |y|): a wrong row, a
  dropped tap, a misplaced bias, a wrong rounding of a weight or a missing
  rescale all move the decoded logits far beyond that.
"""
import numpy as np

import oracle as O
import synthetic as S
from oracle import encoding as E
from oracle import nets as ON
from oracle import plainnet as PN

TOL = 2.0 ** -18


def _chain(logn, bits, n_p=1):
    primes = O.find_primes(logn, bits)
    return primes[: len(bits) - n_p], primes[len(bits) - n_p:]


def _bigint_lincomb(cts, weights, q):
    out = np.zeros_like(cts[0])
    for t in range(cts[0].shape[0]):
        for i, qi in enumerate(q):
            for j in range(cts[0].shape[2]):
                acc = 0
                for c, w in zip(cts, weights):
                    acc += int(w) * int(c[t, i, j])
                out[t, i, j] = acc % qi
    return out


def test_lincomb_matches_bigint_definition():
    q, p = _chain(6, [60, 40, 40, 60])
    orc = O.Oracle(6, q, p, 3)
    cts = [S.residues(30 + k, q, orc.N, 2) for k in range(7)]
    weights = [3, -1, 0, 2 ** 62 - 1, -(2 ** 62) + 5, -123456789012, 1 << 40]
    assert np.array_equal(orc.lincomb(cts, weights), _bigint_lincomb(cts, weights, q))
    # a single term is the plain product by a constant polynomial
    assert np.array_equal(orc.lincomb(cts[:1], [-7]), orc.mul_const(cts[0], -7))


def test_lincomb_extreme_inputs():
    q, p = _chain(4, [60, 50, 60])
    orc = O.Oracle(4, q, p, 2)
    full = np.stack([np.full(orc.N, qi - 1, dtype=np.uint64) for qi in q])[None]
    one = np.concatenate([full, full])  # [2][2][N], every residue q - 1
    n_in = 2000
    for w in (-1, 3, -(2 ** 40)):
        got = orc.lincomb([one] * n_in, [w] * n_in)
        for i, qi in enumerate(q):
            assert np.all(got[:, i] == (n_in * w * (qi - 1)) % qi), (w, i)


def _small_vision_inputs(n_images):
    """The vision network's shapes (5 filters 5x5 stride 2, 845 -> 100 -> 10)
    with the benchmark's seeded weights, on fewer images."""
    x, P = S.vision_inputs(n_images=n_images)
    return x, P


def test_vision_lowering_decodes_to_fp64_network():
    # slot-batched layout: image s in slot s, one ciphertext per pixel;
    # chain [60, 40 x 7 | 60] (one prime per digit) at N = 2^10 (512 images)
    logn = 10
    q, p = _chain(logn, [60] + [40] * 7 + [60])
    orc = O.Oracle(logn, q, p, 8)
    keys = ON.Keys(orc, 21)
    scale = 2.0 ** 40
    slots = orc.N // 2
    x, P = _small_vision_inputs(slots)
    pix = x.reshape(slots, -1).T  # [784][slots]
    level = len(q) - 1
    cts = []
    for i in range(pix.shape[0]):
        m = E.encode(pix[i], scale, orc.N)
        cts.append(orc.encrypt(keys.pk, orc.reduce_int(m, level), level, 9, i))
    rows, _ = PN.vision_conv_rows(P["conv_w"])
    F = P["conv_w"].shape[0]
    per = len(rows) // F
    conv_b = [P["conv_b"][j // per] for j in range(len(rows))]
    h, s = ON.linear(orc, cts, scale, rows, scale, conv_b)
    sq = [ON.square(orc, keys, c, s) for c in h]
    h, s = [c for c, _ in sq], sq[0][1]
    dense1 = [[(i, P["w1"][j, i]) for i in range(P["w1"].shape[1])] for j in range(P["w1"].shape[0])]
    h, s = ON.linear(orc, h, s, dense1, scale, list(P["b1"]))
    sq = [ON.square(orc, keys, c, s) for c in h]
    h, s = [c for c, _ in sq], sq[0][1]
    dense2 = [[(i, P["w2"][j, i]) for i in range(P["w2"].shape[1])] for j in range(P["w2"].shape[0])]
    out, s = ON.linear(orc, h, s, dense2, scale, list(P["b2"]))
    assert out[0].shape[1] == 3  # levels 7 -> 6 -> 5 -> 4 -> 3 -> 2 (limbs 8 -> 3)
    got = np.stack([E.decode_residues(orc.decrypt(keys.sn, c), orc.q, s, orc.N, slots).real for c in out]).T
    want = PN.vision_math(x, P)
    err = np.max(np.abs(got - want) / np.maximum(1.0, np.abs(want)))
    assert err <= TOL, err
    # the check is sensitive: one conv tap dropped moves the logits far away
    P2 = dict(P)
    P2["conv_w"] = P["conv_w"].copy()
    P2["conv_w"][2, 3, 1] = 0.0
    assert np.max(np.abs(PN.vision_math(x, P2) - want)) > 1e-3
