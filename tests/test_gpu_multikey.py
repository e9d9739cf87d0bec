"""Key switching with per-item keys through the C ABI: one launch carries
ciphertexts of two clients (two key sets on the same ring, the paper's
threat model of Section 2.3: each client keeps its own secret and hands the
server its evaluation keys). Every output is checked element-wise against
the oracle with that item's own key."""
import numpy as np
import pytest

import oracle as O
import synthetic as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


CHAINS = {
    "small": (12, [60, 40, 40], [60], 3),
    "wide": (12, [50] * 16, [60, 60], 4),
}
SEEDS = (3, 11)
STEPS = (1, 5)


@pytest.fixture(scope="module", params=sorted(CHAINS))
def setup(request):
    _gpu()
    from paper_2110_13638_amd import ckks
    log_n, qb, pb, dnum = CHAINS[request.param]
    primes = O.find_primes(log_n, qb + pb)
    q, p = primes[: len(qb)], primes[len(qb):]
    ctx = ckks.Context(log_n, q, p, dnum)
    orc = O.Oracle(log_n, q, p, dnum)
    keys, okeys = [], []
    for sd in SEEDS:
        keys.append(ctx.client_keys(sd, galois_steps=STEPS))
        s, sn = orc.keygen_secret(sd)
        rk = orc.keygen_relin(sn, sd + 2)
        gk = {orc.galois_elt(st): orc.keygen_galois(s, sn, orc.galois_elt(st), sd + 3) for st in STEPS}
        okeys.append((s, sn, rk, gk))
    return ctx, orc, keys, okeys


def _u(t):
    return t.cpu().numpy().view(np.uint64)


def test_client_keys_bit_exact(setup):
    ctx, orc, keys, okeys = setup
    for k, (s, sn, rk, gk) in zip(keys, okeys):
        assert np.array_equal(_u(k.sk), sn)
        assert np.array_equal(_u(k.rk), rk)
        for g, key in gk.items():
            assert np.array_equal(_u(k.gk[g]), key)


def _batch(ctx, n, seed0, n_poly=2):
    levels = [max(1, ctx.max_level - (i % 3)) for i in range(n)]
    res = [S.residues(seed0 + i, ctx.q[: lv + 1], ctx.N, n_poly) for i, lv in enumerate(levels)]
    return levels, res


def test_hmult_two_clients_one_launch(setup):
    ctx, orc, keys, okeys = setup
    n = 6
    levels, res_a = _batch(ctx, n, 700)
    _, res_b = _batch(ctx, n, 800)
    owner = [i % 2 for i in range(n)]
    A = [ctx.ct_from_residues(r) for r in res_a]
    Bs = [ctx.ct_from_residues(r) for r in res_b]
    outs = ctx.hmult_relin_rescale(A, Bs, rk=[keys[o].rk for o in owner])
    for i in range(n):
        want = orc.mul_relin_rescale(res_a[i], res_b[i], okeys[owner[i]][2])
        assert np.array_equal(outs[i].residues(), want), i
    # the other client's key gives a different result (the keys are really per item)
    wrong = orc.mul_relin_rescale(res_a[0], res_b[0], okeys[1][2])
    assert not np.array_equal(outs[0].residues(), wrong)


def test_relinearize_two_clients_one_launch(setup):
    ctx, orc, keys, okeys = setup
    n = 4
    levels, res = _batch(ctx, n, 900, n_poly=3)
    owner = [1, 0, 0, 1]
    outs = ctx.relinearize([ctx.ct_from_residues(r) for r in res], rk=[keys[o].rk for o in owner])
    for i in range(n):
        assert np.array_equal(outs[i].residues(), orc.relinearize(res[i], okeys[owner[i]][2])), i


def test_rotate_per_item_steps_and_keys(setup):
    ctx, orc, keys, okeys = setup
    n = 6
    levels, res = _batch(ctx, n, 1000)
    owner = [i % 2 for i in range(n)]
    elts = [ctx.galois_elt(STEPS[(i // 2) % 2]) for i in range(n)]
    outs = ctx.rotate([ctx.ct_from_residues(r) for r in res], g=elts,
                      gk=[keys[o].gk[g] for o, g in zip(owner, elts)])
    for i in range(n):
        want = orc.apply_galois(res[i], elts[i], okeys[owner[i]][3][elts[i]])
        assert np.array_equal(outs[i].residues(), want), i
