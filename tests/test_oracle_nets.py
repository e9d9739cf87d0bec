"""The oracle's encrypted lowerings decode to the FP64 plaintext networks
(the paper's own plaintext-vs-ciphertext check) within the tolerance
2^-18 * max(1, |y|)."""
import numpy as np
import pytest

import oracle as O
import synthetic as S
from oracle import encoding as E
from oracle import nets as ON
from oracle import plainnet as PN

TOL = 2.0 ** -18


def _encrypt(orc, keys, z, level, scale, seed, obj):
    m = E.encode(z, scale, orc.N)
    return orc.encrypt(keys.pk, orc.reduce_int(m, level), level, seed, obj)


def _decrypt(orc, keys, ct, scale, n):
    return E.decode_residues(orc.decrypt(keys.sn, ct), orc.q, scale, orc.N, n).real


def test_tiny_dense_network():
    # dense 16->8 by diagonals on 4096 slots, then x^2 (N = 8192, [60,40,40 | 60])
    logn = 13
    primes = O.find_primes(logn, [60, 40, 40, 60])
    orc = O.Oracle(logn, primes[:3], primes[3:], 3)
    x, W = S.tiny_dense_inputs()
    in_steps, post = PN.tiny_dense_steps()
    keys = ON.Keys(orc, 1, [orc.galois_elt(s) for s in in_steps[1:] + post])
    scale = 2.0 ** 40
    ct = _encrypt(orc, keys, x.reshape(-1), 2, scale, 7, 0)
    diags = PN.tiny_dense_diagonals(W)
    pts = [orc.reduce_int(E.encode(d, scale, orc.N), 2) for d in diags]
    y, s1 = ON.diag_dense(orc, keys, ct, scale, pts, scale, in_steps, post)
    z, s2 = ON.square(orc, keys, y, s1)
    got = _decrypt(orc, keys, z, s2, 4096)[: 8 * 256].reshape(8, 256)
    want = PN.tiny_dense_math(x, W)
    err = np.max(np.abs(got - want) / np.maximum(1.0, np.abs(want)))
    assert err <= TOL, err


def test_yield_network_small_ring():
    # the three rotation-based layers at N = 2^12 (8 windows per ciphertext)
    logn = 12
    primes = O.find_primes(logn, [60] + [40] * 5 + [60])
    orc = O.Oracle(logn, primes[:6], primes[6:], 6)
    x, ws, bs = S.yield_inputs(n_windows=8)
    slots = orc.N // 2
    Wn = PN.yield_layout(slots)
    periods = [256, 64, 16]
    steps = []
    for l in range(3):
        a, b = PN.yield_layer_plan(ws[l].shape[1], ws[l].shape[0], periods[l], Wn)
        steps += a + b
    elts = set(ON.naf_elements(orc, steps))
    keys = ON.Keys(orc, 2, sorted(elts))
    scale = 2.0 ** 40
    v = PN.yield_pack(x, slots)[0]
    ct = _encrypt(orc, keys, v, 5, scale, 9, 0)
    s = scale
    for l in range(3):
        M, b = ws[l], bs[l]
        in_steps, post = PN.yield_layer_plan(M.shape[1], M.shape[0], periods[l], Wn)
        lvl = ct.shape[1] - 1
        d = PN.yield_diagonals(M, periods[l], Wn)
        pts = [orc.reduce_int(E.encode(di, scale, orc.N), lvl) for di in d]
        out_scale = s * scale / orc.q[lvl]
        bias = orc.reduce_int(E.encode(PN.yield_bias_vector(b, Wn), out_scale, orc.N), lvl - 1)
        ct, s = ON.diag_dense(orc, keys, ct, s, pts, scale, in_steps, post, bias)
        if l < 2:
            ct, s = ON.square(orc, keys, ct, s)
    got = _decrypt(orc, keys, ct, s, slots)[:Wn]
    want = PN.yield_math(x, ws, bs)[:, 0]
    err = np.max(np.abs(got - want) / np.maximum(1.0, np.abs(want)))
    assert err <= TOL, err


@pytest.mark.parametrize("which", ["relu", "sigmoid"])
def test_polynomial_activation(which):
    # Section 4.4's approximations by Horner's rule at N = 2^12, [60, 40 x 4 | 60]
    logn = 12
    primes = O.find_primes(logn, [60] + [40] * 4 + [60])
    orc = O.Oracle(logn, primes[:5], primes[5:], 5)
    keys = ON.Keys(orc, 4)
    scale = 2.0 ** 40
    if which == "relu":
        rng_q = 4.0
        coeffs = PN.relu_approx_coeffs(rng_q)
        x = S.uniform_slots(5, orc.N // 2) * rng_q
    else:
        coeffs = PN.sigmoid_approx_coeffs()
        x = S.uniform_slots(6, orc.N // 2) * 5.0
    ct = _encrypt(orc, keys, x, 4, scale, 3, 0)
    y, s = ON.poly(orc, keys, ct, scale, coeffs, scale)
    assert y.shape[1] == 5 - (len(coeffs) - 1)
    got = _decrypt(orc, keys, y, s, orc.N // 2)
    want = PN.poly_eval(coeffs, x)
    err = np.max(np.abs(got - want) / np.maximum(1.0, np.abs(want)))
    assert err <= TOL, err


def _hoist_setup(steps):
    logn = 12
    primes = O.find_primes(logn, [60, 40, 40, 60])
    orc = O.Oracle(logn, primes[:3], primes[3:], 3)
    keys = ON.Keys(orc, 5, sorted({orc.galois_elt(s) for s in steps if s}))
    return orc, keys


def test_hoisted_identity_is_plaintext_product():
    # g = 1 only: ModDown(pt * P c) = pt * c exactly
    orc, keys = _hoist_setup([0])
    scale = 2.0 ** 40
    z = S.uniform_slots(7, orc.N // 2)
    ct = _encrypt(orc, keys, z, 2, scale, 3, 0)
    d = S.uniform_slots(8, orc.N // 2)
    m = E.encode(d, scale, orc.N)
    got = orc.hoisted_linear(ct, [1], [None], m[None, :])
    assert np.array_equal(got, orc.mul_plain(ct, orc.reduce_int(m, 2)))


def test_hoisted_sum_decodes_to_weighted_rotations():
    steps = [0, 1, 5, 100, 2047]
    orc, keys = _hoist_setup(steps)
    scale = 2.0 ** 40
    z = S.uniform_slots(9, orc.N // 2)
    ct = _encrypt(orc, keys, z, 2, scale, 3, 0)
    ds = [S.uniform_slots(20 + i, orc.N // 2) for i in range(len(steps))]
    coeffs = np.stack([E.encode(d, scale, orc.N) for d in ds])
    y, s = ON.diag_dense_hoisted(orc, keys, ct, scale, coeffs, scale, steps, [])
    got = _decrypt(orc, keys, y, s, orc.N // 2)
    want = sum(d * np.roll(z, -st) for d, st in zip(ds, steps))
    err = np.max(np.abs(got - want) / np.maximum(1.0, np.abs(want)))
    assert err <= TOL, err
    # a dropped or misplaced rotation term is caught
    bad = sum(d * np.roll(z, -st) for d, st in zip(ds, [0, 1, 5, 101, 2047]))
    assert np.max(np.abs(got - bad)) > 1e-3


def test_yield_network_hoisted_small_ring():
    logn = 12
    primes = O.find_primes(logn, [60] + [40] * 5 + [60])
    orc = O.Oracle(logn, primes[:6], primes[6:], 6)
    x, ws, bs = S.yield_inputs(n_windows=8)
    slots = orc.N // 2
    Wn = PN.yield_layout(slots)
    periods = [256, 64, 16]
    plans = [PN.yield_layer_plan(ws[l].shape[1], ws[l].shape[0], periods[l], Wn) for l in range(3)]
    steps = {st for a, b in plans for st in a + b if st}
    keys = ON.Keys(orc, 2, sorted(orc.galois_elt(st) for st in steps))
    scale = 2.0 ** 40
    packed = PN.yield_pack(x, slots)
    y = _encrypt(orc, keys, packed[0], 5, scale, 9, 0)
    s = scale
    for l in range(3):
        in_steps, post = plans[l]
        lv = y.shape[1] - 1
        coeffs = np.stack([E.encode(di, scale, orc.N) for di in PN.yield_diagonals(ws[l], periods[l], Wn)])
        out_scale = s * scale / orc.q[lv]
        bias = orc.reduce_int(E.encode(PN.yield_bias_vector(bs[l], Wn), out_scale, orc.N), lv - 1)
        y, s = ON.diag_dense_hoisted(orc, keys, y, s, coeffs, scale, in_steps, post, bias)
        if l < 2:
            y, s = ON.square(orc, keys, y, s)
    got = _decrypt(orc, keys, y, s, Wn)
    want = PN.yield_math(x, ws, bs)[:Wn, 0]
    err = np.max(np.abs(got[: len(want)] - want) / np.maximum(1.0, np.abs(want)))
    assert err <= TOL, err


def test_conv_slots_layer_small_ring():
    # the paper's image-in-slots conv (kernel masquerading, taps summed by
    # hoisted rotations) + x^2 at N = 2^12: two images per ciphertext
    logn = 12
    primes = O.find_primes(logn, [60] + [40] * 3 + [60])
    orc = O.Oracle(logn, primes[:4], primes[4:], 4)
    scale = 2.0 ** 40
    x, P = S.vision_inputs(n_images=2)
    slots = orc.N // 2
    steps, masks, bias = PN.conv_slots_layout(P["conv_w"], P["conv_b"], slots)
    keys = ON.Keys(orc, 7, sorted(orc.galois_elt(s) for s in steps if s))
    v = PN.conv_slots_pack(x, slots)
    ct = _encrypt(orc, keys, v[0], 3, scale, 5, 0)
    mcs = [np.stack([E.encode(masks[f, t], scale, orc.N) for t in range(len(steps))]) for f in range(masks.shape[0])]
    out_scale = scale * scale / orc.q[3]
    bps = [orc.reduce_int(E.encode(bias[f], out_scale, orc.N), 2) for f in range(masks.shape[0])]
    outs, s = ON.conv_slots(orc, keys, ct, scale, mcs, steps, bps, scale)
    got = np.stack([_decrypt(orc, keys, y, s, slots) for y in outs])[None]
    vals = PN.conv_slots_anchor_values(got, 2)
    want = PN.vision_conv_square_math(x, P)
    err = np.max(np.abs(vals - want) / np.maximum(1.0, np.abs(want)))
    assert err <= TOL, err


def test_conv_commuted_layout_fp64():
    # the commuted terms summed by the client equal the biased
    # cross-correlation, with the bias spread over each anchor's taps
    x, P = S.vision_inputs(n_images=3)
    slots = 2048
    terms = PN.conv_commuted_packed(x, P, slots)
    got = PN.conv_commuted_sum(terms, 3)
    want = PN.vision_conv_math(x, P)
    assert np.max(np.abs(got - want)) < 1e-12
    assert np.allclose(PN.vision_tail_math(want, P), PN.vision_math(x, P), rtol=0, atol=1e-9)
    # a dropped or misplaced tap shows: every anchor needs all of its taps
    offsets, masks, bias = PN.conv_commuted_layout(P["conv_w"], P["conv_b"], slots)
    assert len(offsets) == 25 and masks.shape == (5, 25, slots)
    broken = terms.copy()
    broken[:, :, 7] = 0
    assert np.max(np.abs(PN.conv_commuted_sum(broken, 3) - want)) > 1e-3


def test_conv_commuted_key_rotation_small_ring():
    # the oracle's commuted conv (masked products, no rotation) at N = 2^11
    # (one image per ciphertext), then the client's key rotation: decrypt,
    # sum over the kernel, re-encrypt one ciphertext per conv output
    # (slot-batched); decoded within tolerance of the FP64 conv
    logn = 11
    primes = O.find_primes(logn, [60, 40, 40, 40, 40, 60])
    orc = O.Oracle(logn, primes[:5], primes[5:], 5)
    scale = 2.0 ** 40
    x, P = S.vision_inputs(n_images=2)
    slots = orc.N // 2
    offsets, masks, bias = PN.conv_commuted_layout(P["conv_w"], P["conv_b"], slots)
    keys = ON.Keys(orc, 9)
    v = PN.conv_slots_pack(x, slots)
    cts = [_encrypt(orc, keys, v[c], 1, scale, 5, c) for c in range(v.shape[0])]
    mcs = [[E.encode(masks[f, t], scale, orc.N) for t in range(25)] for f in range(5)]
    out_scale = scale * scale / orc.q[1]
    bps = [[orc.reduce_int(E.encode(bias[f, t], out_scale, orc.N), 0) for t in range(25)] for f in range(5)]
    terms, scales = [], []
    for ct in cts:
        ys, s = ON.conv_commuted(orc, keys, ct, scale, mcs, bps, scale)
        assert s == out_scale and len(ys) == 125
        terms += ys
        scales += [s] * len(ys)

    def reform(vals):
        arr = np.array(vals).reshape(len(cts), 5, 25, slots)
        conv = PN.conv_commuted_sum(arr, 2).reshape(2, -1)  # [image][845]
        out = np.zeros((conv.shape[1], slots))
        out[:, :2] = conv.T  # slot-batched: image i at slot i
        return list(out)

    fresh, pts = ON.key_rotation(orc, keys, terms, scales, reform, 4, scale, 11)
    assert len(fresh) == 845 and fresh[0].shape == (2, 5, orc.N)
    want = PN.vision_conv_math(x, P).reshape(2, -1)
    for j in (0, 100, 423, 844):
        got = _decrypt(orc, keys, fresh[j], scale, 2)
        assert np.max(np.abs(got - want[:, j]) / np.maximum(1.0, np.abs(want[:, j]))) <= TOL, j


def test_slots_network_fp64_layout():
    # the whole vision network in the image-in-slots layout (masked taps,
    # masks + rotate-and-sum per dense neuron) equals the plain network
    x, P = S.vision_inputs(n_images=3)
    got = PN.slots_network_packed(x, P, 2048)
    assert np.max(np.abs(got - PN.vision_math(x, P))) < 1e-12
    # a rotate-and-sum missing one step sums half the block
    masks = PN.slots_dense_masks(P["w1"], 2048)
    assert masks.shape == (100, 5, 2048) and np.count_nonzero(masks[0, 0]) == 2 * 169
    assert PN.block_sum_steps() == [1 << k for k in range(10)]


def test_slots_network_encrypted_small_ring():
    # the oracle's lowering of the image-in-slots network with server-side
    # rotate-and-sum dense layers at N = 2^11 (one image per ciphertext),
    # decoded within tolerance of the FP64 network
    logn = 11
    primes = O.find_primes(logn, [60] + [40] * 5 + [60])
    orc = O.Oracle(logn, primes[:6], primes[6:], 6)
    scale = 2.0 ** 40
    x, P = S.vision_inputs(n_images=1)
    slots = orc.N // 2
    steps, masks, bias = PN.conv_slots_layout(P["conv_w"], P["conv_b"], slots)
    rs = PN.block_sum_steps()
    keys = ON.Keys(orc, 7, sorted({orc.galois_elt(s) for s in steps if s} | {orc.galois_elt(s) for s in rs}))
    ct = _encrypt(orc, keys, PN.conv_slots_pack(x, slots)[0], 5, scale, 5, 0)
    mcs = [np.stack([E.encode(masks[f, t], scale, orc.N) for t in range(25)]) for f in range(5)]
    s1 = scale * scale / orc.q[5]
    bps = [orc.reduce_int(E.encode(bias[f], s1, orc.N), 4) for f in range(5)]
    conv, s = ON.conv_slots(orc, keys, ct, scale, mcs, steps, bps, scale)  # level 3
    dm = PN.slots_dense_masks(P["w1"], slots)
    mpts = [[orc.reduce_int(E.encode(dm[j, f], scale, orc.N), 3) for f in range(5)] for j in range(100)]
    s2 = s * scale / orc.q[3]
    bvec = np.zeros((100, slots))
    bvec[:, ::1024] = P["b1"][:, None]
    bpts = [orc.reduce_int(E.encode(bvec[j], s2, orc.N), 2) for j in range(100)]
    h, s3 = ON.slots_dense(orc, keys, conv, s, mpts, scale, bpts, rs)
    assert s3 == s2 and h[0].shape[1] == 3
    sq = []
    for y in h:
        z, s4 = ON.square(orc, keys, y, s3)
        sq.append(z)
    rows = [[(j, P["w2"][k, j]) for j in range(100)] for k in range(10)]
    logits, s5 = ON.linear(orc, sq, s4, rows, scale, P["b2"])
    got = np.array([_decrypt(orc, keys, o, s5, 1)[0] for o in logits])
    want = PN.vision_math(x, P)[0]
    assert np.max(np.abs(got - want) / np.maximum(1.0, np.abs(want))) <= TOL
