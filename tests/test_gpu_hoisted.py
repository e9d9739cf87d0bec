"""Hoisted rotations with plaintext weights (one shared decomposition, one
ModDown): the C ABI call bit-exact against the oracle's definition for one-
and four-prime digits, and the yield network with hoisted layers bit-exact
against the oracle's hoisted lowering and decoded within tolerance."""
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


# rotation sets: arbitrary steps, and steps that are multiples of 8 slots at
# N = 2^12 (every Galois element is then 1 mod 2N / 256, so each aligned block
# of 256 NTT slots maps onto itself and the kernel keeps the digits in LDS)
STEPS = {"any_steps": [0, 1, 5, 100, 2047, 3], "block_steps": [0, 8, 64, 1000, 2040, 24]}


@pytest.mark.parametrize("ntt_fp", [1, 0])
@pytest.mark.parametrize("steps_kind", ["any_steps", "block_steps"])
@pytest.mark.parametrize("chain", ["one_prime_digits", "four_prime_digits", "eight_one_prime_digits",
                                   "ten_one_prime_digits"])
def test_hoisted_linear_bit_exact(mods, chain, steps_kind, ntt_fp):
    ckks, nets = mods
    from paper_2110_13638_amd import _native as nat
    if chain == "one_prime_digits":
        q_bits, p_bits, dnum, level = [60, 40, 40], [60], 3, 2
    elif chain == "four_prime_digits":
        q_bits, p_bits, dnum, level = [50] * 8, [60, 60], 2, 6
    elif chain == "eight_one_prime_digits":  # 3 ciphertexts per staged work item
        q_bits, p_bits, dnum, level = [50] * 8, [60], 8, 7
    else:  # 10 digits: two batches of key loads, 2 ciphertexts per staged work item
        q_bits, p_bits, dnum, level = [50] * 10, [60], 10, 9
    primes = O.find_primes(12, q_bits + p_bits)
    q, p = primes[: len(q_bits)], primes[len(q_bits):]
    ctx = ckks.Context(12, q, p, dnum).keygen(5)
    ctx.set_tuning(ntt_fp=ntt_fp)
    orc = O.Oracle(12, q, p, dnum)
    steps = STEPS[steps_kind]
    elts = [1 if s == 0 else orc.galois_elt(s) for s in steps]
    keys = ON.Keys(orc, 5, [g for g in elts if g != 1])
    for g in elts:
        if g != 1:
            ctx.add_galois_key(g, nets.galois_key_seed(5 + 3, g))
            assert np.array_equal(ctx.gk[g].cpu().numpy().view(np.uint64).reshape(-1), keys.gk[g].reshape(-1))
    coeffs = np.stack([E.encode(S.uniform_slots(40 + i, ctx.N // 2), SCALE, ctx.N) for i in range(len(steps))])
    B = 6  # more than one group of ciphertexts per item
    ins = [S.residues(60 + b, q[: level + 1], ctx.N, 2) for b in range(B)]
    cts = [ctx.ct_from_residues(r, SCALE) for r in ins]
    outs = [ctx.new_ct(2, level, 1.0) for _ in range(B)]
    so = ctx._structs(outs)
    dev = torch.from_numpy(coeffs).to(ctx.device)
    wb = nat.ckks_hoisted_linear_workspace_bytes(ctx.h, B, level, len(steps))
    ws, wbytes = ctx.workspace(wb)
    print("hoisted case", chain, steps_kind, "ntt_fp", ntt_fp, "B", B, "rotations", len(steps), flush=True)
    nat.ckks_hoisted_linear(ctx.h, ctx._structs(cts), so, elts, [ctx.gk[g].data_ptr() if g != 1 else None
                                                                 for g in elts], dev.data_ptr(), SCALE, ws, wbytes,
                            ctx.stream)
    outs = ctx._outs(so, outs)
    gks = [None if g == 1 else keys.gk[g] for g in elts]
    for b in range(B):
        want = orc.hoisted_linear(ins[b], elts, gks, coeffs)
        assert outs[b].scale == SCALE * SCALE and np.array_equal(outs[b].residues(), want), b


def test_yield_hoisted_small_ring(mods):
    ckks, nets = mods
    logn = 12
    primes = O.find_primes(logn, [60] + [40] * 5 + [60])
    ctx = ckks.Context(logn, primes[:6], primes[6:], 6).keygen(2)
    orc = O.Oracle(logn, primes[:6], primes[6:], 6)
    x, ws, bs = S.yield_inputs(n_windows=16)
    slots = ctx.N // 2
    Wn = nets.yield_windows(slots)
    steps = nets.yield_steps(ws, Wn)
    elts = nets.galois_for_steps(ctx, steps, direct=True)
    keys = ON.Keys(orc, 2, elts)
    for g in elts:
        ctx.add_galois_key(g, nets.galois_key_seed(2 + 3, g))
    packed = PN.yield_pack(x, slots)
    n_ct = packed.shape[0]
    ms = [E.encode(packed[c], SCALE, ctx.N) for c in range(n_ct)]
    cts = [ctx.encrypt(ctx.pt_from_coeffs(m, 5, SCALE), seed=9, obj=c) for c, m in enumerate(ms)]
    dcs, bcs = [], []
    s, lvl = SCALE, 5
    periods = [256, 64, 16]
    for l in range(3):
        dcs.append(np.stack([E.encode(di, SCALE, ctx.N) for di in PN.yield_diagonals(ws[l], periods[l], Wn)]))
        out_scale = s * SCALE / orc.q[lvl]
        bcs.append(E.encode(PN.yield_bias_vector(bs[l], Wn), out_scale, ctx.N))
        s, lvl = out_scale, lvl - 1
        if l < 2:
            s, lvl = s * s / orc.q[lvl], lvl - 1
    g = nets.build_yield(ctx, ws, bs, n_ct, 5, SCALE, diag_coeffs=dcs, bias_coeffs=bcs, hoisted=True)
    outs = g.run(cts)
    got = []
    for c in range(n_ct):
        y = orc.encrypt(keys.pk, orc.reduce_int(ms[c], 5), 5, 9, c)
        s = SCALE
        for l in range(3):
            in_steps, post = PN.yield_layer_plan(ws[l].shape[1], ws[l].shape[0], periods[l], Wn)
            lv = y.shape[1] - 1
            y, s = ON.diag_dense_hoisted(orc, keys, y, s, dcs[l], SCALE, in_steps, post,
                                         orc.reduce_int(bcs[l], lv - 1))
            if l < 2:
                y, s = ON.square(orc, keys, y, s)
        assert outs[c].scale == s and np.array_equal(outs[c].residues(), y), c
        got.append(ctx.decrypt(outs[c], Wn).real)
    want = PN.yield_math(x, ws, bs)[:, 0]
    err = np.max(np.abs(np.concatenate(got)[: len(want)] - want) / np.maximum(1.0, np.abs(want)))
    print("yield hoisted: max relative error 2^%.1f" % np.log2(err))
    assert err <= TOL
