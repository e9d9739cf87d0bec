"""Every launch-shape setting the autotuner may pick computes the same
residues: NTT / INTT against the oracle for each ring degree, and the
batched HMult + relinearise + rescale against the oracle under every
setting; the autotuner's pick and its cache round-trip."""
import itertools
import json

import numpy as np
import pytest

import oracle as O
import synthetic as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ck():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_13638_amd import ckks
    return ckks


def _u(t):
    return t.cpu().numpy().view(np.uint64)


SETTINGS = [dict(ntt_wide=w, ew_log=e, xcd_remap=x, fuse_tail=f, ip_cts=i, ntt_fp=p)
            for w, e, x, f, i, p in itertools.product((0, 1), (1, 2, 3), (0, 1), (0, 1), (2, 4, 16), (0, 1))]


@pytest.mark.parametrize("log_n", [11, 12, 13, 14, 15, 16])
def test_ntt_variants_bit_exact(ck, log_n):
    from paper_2110_13638_amd import _native as nat
    primes = O.find_primes(log_n, [60, 50, 40, 36])
    orc = O.Oracle(log_n, primes[:3], primes[3:], 1)
    ctx = ck.Context(log_n, primes[:3], primes[3:], 1)
    x = S.residues(9 + log_n, primes, 1 << log_n)[0]
    want = [orc.ntt(x[i], i) for i in range(len(primes))]
    # the 60-bit prime takes the integer engine, the others the FP64 one when enabled
    for wide, remap, fp in itertools.product((0, 1) if log_n <= 14 else (0,), (0, 1), (0, 1)):
        print("ntt variant log_n=%d wide=%d remap=%d fp=%d" % (log_n, wide, remap, fp), flush=True)
        ctx.set_tuning(ntt_wide=wide, xcd_remap=remap, ntt_fp=fp)
        dev = torch.from_numpy(x.view(np.int64)).cuda()
        ptrs = [dev[i].data_ptr() for i in range(len(primes))]
        ws, wb = ctx.ws_for(nat.CKKS_OP_NTT, len(primes))
        nat.ckks_ntt(ctx.h, ptrs, list(range(len(primes))), ws, wb, ctx.stream)
        torch.cuda.synchronize()
        got = _u(dev)
        for i in range(len(primes)):
            assert np.array_equal(got[i], want[i]), (wide, remap, i)
        nat.ckks_intt(ctx.h, ptrs, list(range(len(primes))), ws, wb, ctx.stream)
        torch.cuda.synchronize()
        assert np.array_equal(_u(dev), x)


@pytest.fixture(scope="module")
def hm(ck):
    primes = O.find_primes(12, [50] * 16 + [60, 60])
    ctx = ck.Context(12, primes[:16], primes[16:], 4).keygen(3)
    orc = O.Oracle(12, primes[:16], primes[16:], 4)
    _, sn = orc.keygen_secret(3)
    rk = orc.keygen_relin(sn, 3 + 2)
    levels = [l - 1 for l in S.ragged_limbs(6)]
    ins, want = [], []
    for i, lv in enumerate(levels):
        res = S.residues(300 + i, ctx.q[: lv + 1], ctx.N, 4)
        ins.append((ctx.ct_from_residues(res[:2]), ctx.ct_from_residues(res[2:])))
        want.append(orc.mul_relin_rescale(res[:2], res[2:], rk))
    return ctx, ins, want


@pytest.mark.parametrize("st", SETTINGS, ids=lambda d: "w%d_e%d_x%d_f%d_i%d_p%d" % (d["ntt_wide"], d["ew_log"], d["xcd_remap"],
                                                                              d["fuse_tail"], d["ip_cts"], d["ntt_fp"]))
def test_hmult_variants_bit_exact(hm, st):
    ctx, ins, want = hm
    print("hmult variant", st, flush=True)
    ctx.set_tuning(**st)
    outs = ctx.hmult_relin_rescale([a for a, _ in ins], [b for _, b in ins])
    for o, w in zip(outs, want):
        assert np.array_equal(o.residues(), w)
    ctx.set_tuning(ntt_wide=0, ew_log=2, xcd_remap=1, fuse_tail=0, ip_cts=4, ntt_fp=1)


def test_autotune_pick_and_cache(hm, tmp_path):
    from paper_2110_13638_amd import tune
    ctx, ins, want = hm
    A, B = [a for a, _ in ins], [b for _, b in ins]
    cache = str(tmp_path / "tune.json")
    best, times = tune.autotune(ctx, lambda: ctx.hmult_relin_rescale(A, B), "hmult-ragged", cache=cache,
                                space={"ntt_wide": (0, 1), "ew_log": (2, 3), "xcd_remap": (1,), "fuse_tail": (0,), "ip_cts": (4,)},
                                reps=2)
    assert len(times) == 4 and all(t > 0 for t in times.values())

    def applied():
        cur = ctx.tuning()
        return {k: cur[k] for k in best}

    assert applied() == best
    # the cached pick is applied without timing again
    ctx.set_tuning(ntt_wide=0, ew_log=2, xcd_remap=1, fuse_tail=0, ip_cts=4, ntt_fp=1)
    again, times2 = tune.autotune(ctx, None, "hmult-ragged", cache=cache)
    assert again == best and times2 == {} and applied() == best
    assert json.load(open(cache))
    outs = ctx.hmult_relin_rescale(A, B)
    for o, w in zip(outs, want):
        assert np.array_equal(o.residues(), w)
    ctx.set_tuning(ntt_wide=0, ew_log=2, xcd_remap=1, fuse_tail=0, ip_cts=4, ntt_fp=1)


def test_graph_replans_when_launch_shapes_change(ck):
    """A graph planned under one setting (fused HMult tail: fewer scratch
    limbs) runs under another (separate tail pass: more) without a workspace
    error, with identical results."""
    from paper_2110_13638_amd import graph as G
    primes = O.find_primes(11, [60, 40, 40, 40, 60])
    ctx = ck.Context(11, primes[:4], primes[4:], 4).keygen(8)
    ctx.set_tuning(fuse_tail=1)
    g = G.Graph(ctx)
    g.chain(g.input(6, 3, ctx.default_scale), g.square(), g.square(), g.output())
    g.plan()
    res = S.residues(90, ctx.q, ctx.N, 12)
    cts = [ctx.ct_from_residues(res[2 * i: 2 * i + 2], ctx.default_scale) for i in range(6)]
    want = [o.residues().copy() for o in g.run(cts)]
    for st in (dict(fuse_tail=0), dict(fuse_tail=0, ip_cts=2), dict(fuse_tail=1, ip_cts=16), dict(ntt_fp=0)):
        print("graph under", st, flush=True)
        ctx.set_tuning(**st)
        got = [o.residues() for o in g.run(cts)]
        for a, b in zip(got, want):
            assert np.array_equal(a, b), st
    ctx.set_tuning(ntt_wide=0, ew_log=2, xcd_remap=1, fuse_tail=0, ip_cts=4, ntt_fp=1)
