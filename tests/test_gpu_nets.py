"""GPU graph runtime on the three network shapes: ciphertexts bit-exact
against the oracle's lowering from the same integer plaintexts and seeds,
decoded outputs within 2^-18 * max(1, |y|) of the FP64 network."""
import numpy as np
import pytest

import oracle as O
import synthetic as S
from oracle import encoding as E
from oracle import nets as ON
from oracle import plainnet as PN

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
TOL = 2.0 ** -18
SCALE = 2.0 ** 40


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_13638_amd import ckks, nets
    return ckks, nets


def _setup(ckks, logn, q_bits, p_bits, dnum, seed):
    primes = O.find_primes(logn, list(q_bits) + list(p_bits))
    q, p = primes[: len(q_bits)], primes[len(q_bits):]
    ctx = ckks.Context(logn, q, p, dnum).keygen(seed)
    orc = O.Oracle(logn, q, p, dnum)
    return ctx, orc


def _enc_both(ctx, orc, keys, z, level, seed, obj):
    m = E.encode(z, SCALE, ctx.N)
    ct = ctx.encrypt(ctx.pt_from_coeffs(m, level, SCALE), seed=seed, obj=obj)
    cto = orc.encrypt(keys.pk, orc.reduce_int(m, level), level, seed, obj)
    assert np.array_equal(ct.residues(), cto)
    return ct, cto


def _rel_err(got, want):
    return np.max(np.abs(got - want) / np.maximum(1.0, np.abs(want)))


def test_tiny_dense_full_size(mods):
    ckks, nets = mods
    ctx, orc = _setup(ckks, 13, [60, 40, 40], [60], 3, 1)
    x, W = S.tiny_dense_inputs()
    in_steps, post = PN.tiny_dense_steps()
    steps = in_steps[1:] + post
    elts = [orc.galois_elt(s) for s in steps]
    keys = ON.Keys(orc, 1, elts)
    assert sorted(elts) == nets.galois_for_steps(ctx, steps, direct=True)
    for g in elts:
        ctx.add_galois_key(g, nets.galois_key_seed(1 + 3, g))
    ct, cto = _enc_both(ctx, orc, keys, x.reshape(-1), 2, 7, 0)
    # the product computes the same diagonals as the oracle's plain network
    assert np.array_equal(nets.tiny_dense_diagonals(W, 256), PN.tiny_dense_diagonals(W))
    coeffs = np.stack([E.encode(d, SCALE, ctx.N) for d in PN.tiny_dense_diagonals(W)])
    g, _ = nets.build_tiny_dense(ctx, W, 256, 2, SCALE, diag_coeffs=coeffs)
    out = g.run([ct])[0]
    pts = [orc.reduce_int(c, 2) for c in coeffs]
    y, s1 = ON.diag_dense(orc, keys, cto, SCALE, pts, SCALE, in_steps, post)
    z, s2 = ON.square(orc, keys, y, s1)
    assert out.level == 0 and out.scale == s2
    assert np.array_equal(out.residues(), z)
    got = ctx.decrypt(out, 4096).real[: 8 * 256].reshape(8, 256)
    err = _rel_err(got, PN.tiny_dense_math(x, W))
    print("tiny dense: max relative error 2^%.1f" % np.log2(err))
    assert err <= TOL


def test_yield_small_ring(mods):
    ckks, nets = mods
    ctx, orc = _setup(ckks, 12, [60] + [40] * 5, [60], 6, 2)
    x, ws, bs = S.yield_inputs(n_windows=16)
    slots = ctx.N // 2
    Wn = nets.yield_windows(slots)
    steps = nets.yield_steps(ws, Wn)
    elts = nets.galois_for_steps(ctx, steps)
    assert elts == ON.naf_elements(orc, steps)
    keys = ON.Keys(orc, 2, elts)
    for g in elts:
        ctx.add_galois_key(g, nets.galois_key_seed(2 + 3, g))
    packed = PN.yield_pack(x, slots)
    assert np.array_equal(nets.yield_pack(x, slots), packed)
    n_ct = packed.shape[0]
    cts, ctos = zip(*[_enc_both(ctx, orc, keys, packed[c], 5, 9, c) for c in range(n_ct)])
    # integer plaintexts of every layer, encoded by the oracle
    dcs, bcs = [], []
    s, lvl = SCALE, 5
    periods = [256, 64, 16]
    for l in range(3):
        d = PN.yield_diagonals(ws[l], periods[l], Wn)
        assert np.array_equal(nets.yield_diagonals(ws[l], periods[l], Wn), d)
        dcs.append(np.stack([E.encode(di, SCALE, ctx.N) for di in d]))
        out_scale = s * SCALE / orc.q[lvl]
        bcs.append(E.encode(PN.yield_bias_vector(bs[l], Wn), out_scale, ctx.N))
        s, lvl = out_scale, lvl - 1
        if l < 2:
            s, lvl = s * s / orc.q[lvl], lvl - 1
    g = nets.build_yield(ctx, ws, bs, n_ct, 5, SCALE, diag_coeffs=dcs, bias_coeffs=bcs)
    outs = g.run(list(cts))
    # oracle lowering of the same layers
    s = SCALE
    ys = list(ctos)
    for l in range(3):
        M = ws[l]
        in_steps, post = PN.yield_layer_plan(M.shape[1], M.shape[0], periods[l], Wn)
        lv = ys[0].shape[1] - 1
        pts = [orc.reduce_int(c, lv) for c in dcs[l]]
        bias = orc.reduce_int(bcs[l], lv - 1)
        res = [ON.diag_dense(orc, keys, y, s, pts, SCALE, in_steps, post, bias) for y in ys]
        ys = [r[0] for r in res]
        s = res[0][1]
        if l < 2:
            res = [ON.square(orc, keys, y, s) for y in ys]
            ys = [r[0] for r in res]
            s = res[0][1]
    want = PN.yield_math(x, ws, bs)[:, 0]
    got = []
    for c in range(n_ct):
        assert outs[c].scale == s and np.array_equal(outs[c].residues(), ys[c]), c
        got.append(ctx.decrypt(outs[c], Wn).real)
    err = _rel_err(np.concatenate(got)[: len(want)], want)
    print("yield: max relative error 2^%.1f" % np.log2(err))
    assert err <= TOL


def test_vision_small_ring(mods):
    ckks, nets = mods
    logn = 10
    ctx, orc = _setup(ckks, logn, [60] + [40] * 7, [60], 8, 3)
    n_img = ctx.N // 2
    x, P = S.vision_inputs(n_images=n_img)
    keys = ON.Keys(orc, 3)
    pix = x.reshape(n_img, -1).T
    cts, ctos = zip(*[_enc_both(ctx, orc, keys, pix[i], 7, 11, i) for i in range(pix.shape[0])])
    g = nets.build_vision(ctx, P, 28, 7, SCALE)
    outs = g.run(list(cts))
    # oracle: conv (original row order) -> x^2 -> dense -> x^2 -> dense
    rows, _ = PN.vision_conv_rows(P["conv_w"])
    F = P["conv_w"].shape[0]
    per = len(rows) // F
    h, s = ON.linear(orc, list(ctos), SCALE, rows, SCALE, [P["conv_b"][j // per] for j in range(len(rows))])
    sq = [ON.square(orc, keys, c, s) for c in h]
    h, s = [c for c, _ in sq], sq[0][1]
    W1 = P["w1"]
    h, s = ON.linear(orc, h, s, [[(i, W1[j, i]) for i in range(W1.shape[1])] for j in range(W1.shape[0])], SCALE,
                     list(P["b1"]))
    sq = [ON.square(orc, keys, c, s) for c in h]
    h, s = [c for c, _ in sq], sq[0][1]
    W2 = P["w2"]
    h, s = ON.linear(orc, h, s, [[(i, W2[j, i]) for i in range(W2.shape[1])] for j in range(W2.shape[0])], SCALE,
                     list(P["b2"]))
    for j in range(10):
        assert outs[j].scale == s and np.array_equal(outs[j].residues(), h[j]), j
    got = np.stack([ctx.decrypt(outs[j], n_img).real for j in range(10)], axis=1)
    want = PN.vision_math(x, P)
    err = _rel_err(got, want)
    print("vision: max relative error 2^%.1f" % np.log2(err))
    assert err <= TOL


@pytest.mark.parametrize("which", ["relu", "sigmoid"])
def test_poly_activation(mods, which):
    # Section 4.4's activation approximations as a graph node, N = 2^12,
    # [60, 40 x 4 | 60]: bit-exact vs the oracle's Horner lowering, decoded
    # within tolerance of the FP64 polynomial
    ckks, nets = mods
    ctx, orc = _setup(ckks, 12, [60] + [40] * 4, [60], 5, 4)
    keys = ON.Keys(orc, 4)
    if which == "relu":
        coeffs = nets.relu_approx_coeffs(4.0)
        assert coeffs == PN.relu_approx_coeffs(4.0)
        x = S.uniform_slots(5, ctx.N // 2) * 4.0
    else:
        coeffs = nets.sigmoid_approx_coeffs()
        assert coeffs == PN.sigmoid_approx_coeffs()
        x = S.uniform_slots(6, ctx.N // 2) * 5.0
    cts, ctos = zip(*[_enc_both(ctx, orc, keys, x, 4, 13, i) for i in range(3)])
    from paper_2110_13638_amd.graph import Graph
    g = Graph(ctx)
    g.chain(g.input(3, 4, SCALE), g.poly(coeffs, SCALE), g.output())
    outs = g.run(list(cts))
    for i in range(3):
        y, s = ON.poly(orc, keys, ctos[i], SCALE, coeffs, SCALE)
        assert outs[i].level == y.shape[1] - 1 and outs[i].scale == s
        assert np.array_equal(outs[i].residues(), y), i
    got = ctx.decrypt(outs[0], ctx.N // 2).real
    want = PN.poly_eval(coeffs, x)
    err = _rel_err(got, want)
    print("%s approximation: max relative error 2^%.1f" % (which, np.log2(err)))
    assert err <= TOL


def test_conv_slots_layer(mods):
    # the paper's image-in-slots conv layout at N = 2^12 (two images per
    # ciphertext): bit-exact vs the oracle's lowering, decoded conv^2 at the
    # anchors within tolerance of the FP64 layers
    ckks, nets = mods
    ctx, orc = _setup(ckks, 12, [60] + [40] * 3, [60], 4, 7)
    slots = ctx.N // 2
    x, P = S.vision_inputs(n_images=4)
    steps, masks, bias = PN.conv_slots_layout(P["conv_w"], P["conv_b"], slots)
    s2, m2, b2 = nets.conv_slots_layout(P["conv_w"], P["conv_b"], slots)
    assert s2 == steps and np.array_equal(m2, masks) and np.array_equal(b2, bias)
    elts = nets.galois_for_steps(ctx, steps, direct=True)
    keys = ON.Keys(orc, 7, elts)
    for g in elts:
        ctx.add_galois_key(g, nets.galois_key_seed(7 + 3, g))
    v = PN.conv_slots_pack(x, slots)
    assert np.array_equal(nets.conv_slots_pack(x, slots), v)
    cts, ctos = zip(*[_enc_both(ctx, orc, keys, v[c], 3, 5, c) for c in range(v.shape[0])])
    mcs = [np.stack([E.encode(masks[f, t], SCALE, ctx.N) for t in range(len(steps))]) for f in range(5)]
    out_scale = SCALE * SCALE / orc.q[3]
    bcs = [E.encode(bias[f], out_scale, ctx.N) for f in range(5)]
    g = nets.build_conv_slots(ctx, P, len(cts), 3, SCALE, mask_coeffs=mcs, bias_coeffs=bcs)
    outs = g.run(list(cts))  # filter-major: outs[f * n_ct + c]
    n_ct = len(cts)
    got = np.zeros((n_ct, 5, slots))
    for c in range(n_ct):
        ys, s = ON.conv_slots(orc, keys, ctos[c], SCALE, mcs, steps,
                              [orc.reduce_int(b, 2) for b in bcs], SCALE)
        for f in range(5):
            o = outs[f * n_ct + c]
            assert o.scale == s and np.array_equal(o.residues(), ys[f]), (c, f)
            got[c, f] = ctx.decrypt(o, slots).real
    vals = PN.conv_slots_anchor_values(got, 4)
    err = _rel_err(vals, PN.vision_conv_square_math(x, P))
    print("conv in slots: max relative error 2^%.1f" % np.log2(err))
    assert err <= TOL


def test_conv_commuted_key_rotation_network(mods):
    # the paper's own route through the vision network at N = 2^12 (two
    # images per ciphertext): kernel-masquerading terms with the commuted
    # bias (no rotations) bit-exact vs the oracle; the client's key
    # rotation (decrypt, sum over the kernel, re-encrypt slot-batched)
    # gives the oracle's plaintext integers up to the encoder rule (+-1,
    # >= 99.9 % equal); the slot-batched rest of the network on the
    # re-encrypted ciphertexts decodes within tolerance of the FP64 network
    ckks, nets = mods
    ctx, orc = _setup(ckks, 12, [60, 40, 40, 40, 40], [60], 5, 7)
    keys = ON.Keys(orc, 7)
    slots = ctx.N // 2
    x, P = S.vision_inputs(n_images=4)
    offsets, masks, bias = PN.conv_commuted_layout(P["conv_w"], P["conv_b"], slots)
    o2, m2, b2 = nets.conv_commuted_layout(P["conv_w"], P["conv_b"], slots)
    assert o2 == offsets and np.array_equal(m2, masks) and np.allclose(b2, bias, rtol=1e-15, atol=0)
    v = PN.conv_slots_pack(x, slots)
    n_ct = v.shape[0]
    cts, ctos = zip(*[_enc_both(ctx, orc, keys, v[c], 1, 5, c) for c in range(n_ct)])
    mcs = [[E.encode(masks[f, t], SCALE, ctx.N) for t in range(25)] for f in range(5)]
    out_scale = SCALE * SCALE / orc.q[1]
    bcs = [[E.encode(bias[f, t], out_scale, ctx.N) for t in range(25)] for f in range(5)]
    g = nets.build_conv_commuted(ctx, P, n_ct, 1, SCALE, mask_coeffs=mcs, bias_coeffs=bcs)
    outs = g.run(list(cts))  # node-major: outs[(f * 25 + t) * n_ct + c]
    assert len(outs) == 125 * n_ct
    terms_g, terms_o = [], []
    for c in range(n_ct):
        ys, s = ON.conv_commuted(orc, keys, ctos[c], SCALE, mcs, [[orc.reduce_int(b, 0) for b in bf] for bf in bcs],
                                 SCALE)
        for k in range(125):
            o = outs[k * n_ct + c]
            assert o.scale == s and np.array_equal(o.residues(), ys[k]), (c, k)
            terms_g.append(o)
        terms_o += ys

    def reform(pn):
        def f(vals):
            arr = np.array(vals).reshape(n_ct, 5, 25, slots)
            conv = pn(arr, 4).reshape(4, -1)
            out = np.zeros((conv.shape[1], slots))
            out[:, :4] = conv.T
            return list(out)
        return f

    # key rotation: GPU client path vs the oracle's
    fresh_o, pts_o = ON.key_rotation(orc, keys, terms_o, [out_scale] * len(terms_o), reform(PN.conv_commuted_sum),
                                     4, SCALE, 11)
    vals_g = [ctx.decrypt(t).real for t in terms_g]
    ints_g = [ctx.encode_coeffs(v_, SCALE) for v_ in reform(nets.conv_commuted_sum)(vals_g)]
    diff = np.stack(ints_g).astype(np.int64) - np.stack(pts_o).astype(np.int64)
    assert np.max(np.abs(diff)) <= 1 and np.mean(diff == 0) >= 0.999
    fresh = nets.key_rotation(ctx, terms_g, reform(nets.conv_commuted_sum), 4, SCALE, 11)
    same = [np.array_equal(a.residues(), b) for a, b in zip(fresh, fresh_o)]
    print("re-encrypted ciphertexts identical to the oracle's: %d of %d" % (sum(same), len(same)))
    for k, (a, m) in enumerate(zip(fresh, ints_g)):
        if k % 97 == 0:  # from the same integers, encryption is bit-exact
            assert np.array_equal(a.residues(), orc.encrypt(keys.pk, orc.reduce_int(m, 4), 4, 11, k))
    # the rest of the network on the GPU, decoded vs FP64
    tail = nets.build_vision_tail(ctx, P, 4, SCALE)
    logits = tail.run(fresh)
    got = np.stack([ctx.decrypt(o, 4).real for o in logits], axis=1)
    err = _rel_err(got, PN.vision_math(x, P))
    print("commuted conv + key rotation + slot-batched tail: max relative error 2^%.1f" % np.log2(err))
    assert err <= TOL


def test_slots_network_rotate_and_sum(mods):
    # the vision network in the image-in-slots layout with its dense layers
    # summed on the server (masks + rotate-and-sum per neuron) at N = 2^12,
    # two images per ciphertext: conv, dense 1 and the head bit-exact vs
    # the oracle's lowering; logits within tolerance of the FP64 network
    ckks, nets = mods
    ctx, orc = _setup(ckks, 12, [60] + [40] * 5, [60], 6, 7)
    slots = ctx.N // 2
    x, P = S.vision_inputs(n_images=4)
    steps, masks, bias = PN.conv_slots_layout(P["conv_w"], P["conv_b"], slots)
    rs = PN.block_sum_steps()
    assert nets.block_sum_steps() == rs
    assert np.array_equal(nets.slots_dense_masks(P["w1"], slots), PN.slots_dense_masks(P["w1"], slots))
    elts = sorted(set(nets.galois_for_steps(ctx, steps, direct=True)) | set(nets.galois_for_steps(ctx, rs, direct=True)))
    keys = ON.Keys(orc, 7, elts)
    for g in elts:
        ctx.add_galois_key(g, nets.galois_key_seed(7 + 3, g))
    v = PN.conv_slots_pack(x, slots)
    n_ct = v.shape[0]
    cts, ctos = zip(*[_enc_both(ctx, orc, keys, v[c], 5, 5, c) for c in range(n_ct)])
    mcs = [np.stack([E.encode(masks[f, t], SCALE, ctx.N) for t in range(25)]) for f in range(5)]
    s1 = SCALE * SCALE / orc.q[5]
    bcs = [E.encode(bias[f], s1, ctx.N) for f in range(5)]
    g = nets.build_conv_slots(ctx, P, n_ct, 5, SCALE, mask_coeffs=mcs, bias_coeffs=bcs)
    outs = g.run(list(cts))
    conv = [[outs[f * n_ct + c] for c in range(n_ct)] for f in range(5)]
    conv_o = [ON.conv_slots(orc, keys, ctos[c], SCALE, mcs, steps, [orc.reduce_int(b, 4) for b in bcs], SCALE)
              for c in range(n_ct)]
    s = conv_o[0][1]
    for c in range(n_ct):
        for f in range(5):
            assert np.array_equal(conv[f][c].residues(), conv_o[c][0][f])
    dm = PN.slots_dense_masks(P["w1"], slots)
    mc = [[E.encode(dm[j, f], SCALE, ctx.N) for f in range(5)] for j in range(100)]
    s2 = s * SCALE / orc.q[3]
    bvec = np.zeros((100, slots))
    bvec[:, ::1024] = P["b1"][:, None]
    bc = [E.encode(bvec[j], s2, ctx.N) for j in range(100)]
    h = nets.slots_dense(ctx, conv, SCALE, P["w1"], P["b1"], mask_coeffs=mc, bias_coeffs=bc)
    want = PN.vision_math(x, P)
    for c in range(n_ct):
        print("rotate-and-sum dense, ciphertext %d" % c, flush=True)
        ho, s3 = ON.slots_dense(orc, keys, [conv_o[c][0][f] for f in range(5)], s, 
                                [[orc.reduce_int(m, 3) for m in mj] for mj in mc], SCALE,
                                [orc.reduce_int(b, 2) for b in bc], rs)
        for j in range(100):
            assert h[j][c].scale == s3 and np.array_equal(h[j][c].residues(), ho[j]), (c, j)
        head = nets.build_slots_head(ctx, P, 100, 2, s3)
        logits = head.run([h[j][c] for j in range(100)])
        sq = [ON.square(orc, keys, y, s3)[0] for y in ho]
        s4 = s3 * s3 / orc.q[2]
        lo, s5 = ON.linear(orc, sq, s4, [[(j, P["w2"][k, j]) for j in range(100)] for k in range(10)], SCALE,
                           P["b2"])
        got = np.zeros((2, 10))
        for k in range(10):
            assert logits[k].scale == s5 and np.array_equal(logits[k].residues(), lo[k]), (c, k)
            got[:, k] = ctx.decrypt(logits[k]).real[::1024][:2]
        err = _rel_err(got, want[2 * c:2 * c + 2])
        print("image-in-slots network, rotate-and-sum: max relative error 2^%.1f" % np.log2(err))
        assert err <= TOL
