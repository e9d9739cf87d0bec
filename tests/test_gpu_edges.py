"""Edge cases of the device entry points: empty batches, the bench's exact
launch configuration (256 pairs at N = 2^15, autotuned launch shapes) with
sampled outputs against the oracle, and the error paths (no level left,
mismatched levels and scales, aliasing)."""
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


@pytest.fixture(scope="module")
def small(ck):
    primes = O.find_primes(12, [60, 40, 40, 60])
    ctx = ck.Context(12, primes[:3], primes[3:], 3).keygen(3)
    return ctx, O.Oracle(12, primes[:3], primes[3:], 3)


def test_empty_batches_are_no_ops(small):
    ctx, _ = small
    from paper_2110_13638_amd import _native as nat
    ws, wb = ctx.workspace(1 << 20)
    empty = (nat.ckks_ct * 0)()
    nat.ckks_hmult_relin_rescale(ctx.h, ctx.rk.data_ptr(), empty, empty, empty, ws, wb, ctx.stream)
    nat.ckks_add(ctx.h, empty, empty, empty, ws, wb, ctx.stream)
    nat.ckks_ntt(ctx.h, [], [], ws, wb, ctx.stream)
    torch.cuda.synchronize()


def test_error_paths(small):
    ctx, _ = small
    from paper_2110_13638_amd import _native as nat
    a = ctx.ct_from_residues(S.residues(1, ctx.q, ctx.N, 2), 2.0 ** 40)
    b = ctx.ct_from_residues(S.residues(2, ctx.q[:2], ctx.N, 2), 2.0 ** 40)
    with pytest.raises(nat.CkksError) as e:
        ctx.hmult_relin_rescale([a], [b])  # levels differ
    assert e.value.code == nat.CKKS_ELEVEL
    z = ctx.ct_from_residues(S.residues(3, ctx.q[:1], ctx.N, 2), 2.0 ** 40)
    with pytest.raises(nat.CkksError) as e:
        ctx.hmult_relin_rescale([z], [z])  # no prime left to rescale
    assert e.value.code == nat.CKKS_EDEPTH
    c = ctx.ct_from_residues(S.residues(4, ctx.q, ctx.N, 2), 2.0 ** 30)
    with pytest.raises(nat.CkksError) as e:
        ctx.add(a, c)  # scales differ
    assert e.value.code == nat.CKKS_ESCALE
    with pytest.raises(nat.CkksError) as e:
        ctx.hmult_relin_rescale([a], [a], outs=[a])  # output aliases an input
    assert e.value.code == nat.CKKS_EINVAL
    ws, wb = ctx.workspace(1 << 20)
    with pytest.raises(nat.CkksError) as e:  # workspace too small for the batch
        nat.ckks_hmult_relin_rescale(ctx.h, ctx.rk.data_ptr(), ctx._structs([a] * 64), ctx._structs([a] * 64),
                                     ctx._structs([ctx.new_ct(2, 1) for _ in range(64)]), ws, 4096, ctx.stream)
    assert e.value.code == nat.CKKS_ENOMEM
    # ciphertext and key buffers must be 16-byte aligned (residues move in pairs);
    # rejected on the host before anything is launched
    wsb, wbb = ctx.ws_for(nat.CKKS_OP_HMULT, 1, [a.level])
    sa = ctx._structs([a])
    sa[0].data += 8
    with pytest.raises(nat.CkksError) as e:
        nat.ckks_hmult_relin_rescale(ctx.h, ctx.rk.data_ptr(), sa, ctx._structs([a]),
                                     ctx._structs([ctx.new_ct(2, a.level - 1)]), wsb, wbb, ctx.stream)
    assert e.value.code == nat.CKKS_EINVAL and "aligned" in str(e.value)
    with pytest.raises(nat.CkksError) as e:
        nat.ckks_hmult_relin_rescale(ctx.h, ctx.rk.data_ptr() + 8, ctx._structs([a]), ctx._structs([a]),
                                     ctx._structs([ctx.new_ct(2, a.level - 1)]), wsb, wbb, ctx.stream)
    assert e.value.code == nat.CKKS_EINVAL and "aligned" in str(e.value)
    # the fused rescale + bias needs its constants
    wsr, wbr = ctx.ws_for(nat.CKKS_OP_RESCALE, 1, [a.level])
    with pytest.raises(nat.CkksError) as e:
        nat._call("ckks_rescale_add_scalar", ctx.h, ctx._structs([a]), None, ctx._structs([ctx.new_ct(2, a.level)]),
                  1, wsr, wbr, ctx.stream)
    assert e.value.code == nat.CKKS_EINVAL


def test_bench_configuration_sampled(ck):
    # the timed workload: 256 pairs at 16 limbs, N = 2^15, dnum 4, with the
    # launch shapes the autotuner picks; three outputs checked against the oracle
    from paper_2110_13638_amd import _native as nat, tune
    primes = O.find_primes(15, [50] * 16 + [60, 60])
    q, p = primes[:16], primes[16:]
    ctx = ck.Context(15, q, p, 4).keygen(1)
    orc = O.Oracle(15, q, p, 4)
    _, sn = orc.keygen_secret(1)
    rk = orc.keygen_relin(sn, 3)
    B, top = 256, 15
    res = S.residues_device(0, q, ctx.N, 4 * B, ctx.device).view(B, 2, 2, 16, ctx.N)
    A = [ck.Ciphertext(ctx, res[i, 0], 2, top, 1.0) for i in range(B)]
    Bc = [ck.Ciphertext(ctx, res[i, 1], 2, top, 1.0) for i in range(B)]
    outs = [ctx.new_ct(2, top - 1, 1.0) for _ in range(B)]
    best, _ = tune.autotune(ctx, lambda: ctx.hmult_relin_rescale(A, Bc, outs=outs), "edge-test", reps=1,
                            space={"ew_log": (1, 2), "fuse_tail": (0, 1), "ip_cts": (2, 4, 16)})
    print("bench configuration, launch shapes", best, flush=True)
    ctx.hmult_relin_rescale(A, Bc, outs=outs)
    torch.cuda.synchronize()
    for i in (0, 97, 255):
        a, b = A[i].residues(), Bc[i].residues()
        want = orc.mul_relin_rescale(a, b, rk)
        assert np.array_equal(outs[i].residues(), want), i


@pytest.mark.parametrize("log_n", [13, 15])
def test_fp64_engine_prime_boundary(ck, log_n):
    """Primes on both sides of the FP64 engine's 2^50 bound in one chain: the
    largest primes below 2^50 (the engine's tightest magnitude bounds), 51-
    and 60-bit primes (integer engine), digits that mix both classes (ModUp
    converts with the integer engine) and a special prime below 2^50.
    Transforms and the fused HMult are bit-exact against the oracle with the
    FP64 engine on and off."""
    from paper_2110_13638_amd import _native as nat
    bits_q = [51, 50, 50, 49, 50, 51, 50, 50]
    bits_p = [50, 60]
    primes = O.find_primes(log_n, bits_q + bits_p)
    assert any(p < (1 << 50) for p in primes) and any(p > (1 << 50) for p in primes)
    nq = len(bits_q)
    ctx = ck.Context(log_n, primes[:nq], primes[nq:], 4).keygen(5)
    orc = O.Oracle(log_n, primes[:nq], primes[nq:], 4)
    _, sn = orc.keygen_secret(5)
    rk = orc.keygen_relin(sn, 5 + 2)
    x = S.residues(70 + log_n, primes, 1 << log_n)[0]
    want = [orc.ntt(x[i], i) for i in range(len(primes))]
    levels = [nq - 1, 5, 3, 1]
    ins, outs_want = [], []
    for i, lv in enumerate(levels):
        res = S.residues(80 + i, ctx.q[: lv + 1], ctx.N, 4)
        ins.append((ctx.ct_from_residues(res[:2]), ctx.ct_from_residues(res[2:])))
        outs_want.append(orc.mul_relin_rescale(res[:2], res[2:], rk))
    for fp in (1, 0):
        print("engine boundary log_n=%d fp=%d" % (log_n, fp), flush=True)
        ctx.set_tuning(ntt_fp=fp)
        dev = torch.from_numpy(x.view(np.int64)).cuda()
        ptrs = [dev[i].data_ptr() for i in range(len(primes))]
        ws, wb = ctx.ws_for(nat.CKKS_OP_NTT, len(primes))
        nat.ckks_ntt(ctx.h, ptrs, list(range(len(primes))), ws, wb, ctx.stream)
        torch.cuda.synchronize()
        got = dev.cpu().numpy().view(np.uint64)
        for i in range(len(primes)):
            assert np.array_equal(got[i], want[i]), (fp, i, primes[i])
        nat.ckks_intt(ctx.h, ptrs, list(range(len(primes))), ws, wb, ctx.stream)
        torch.cuda.synchronize()
        assert np.array_equal(dev.cpu().numpy().view(np.uint64), x)
        outs = ctx.hmult_relin_rescale([a for a, _ in ins], [b for _, b in ins])
        for o, w in zip(outs, outs_want):
            assert np.array_equal(o.residues(), w), fp
    ctx.set_tuning(ntt_fp=1)


def test_ring_2_16_transforms_and_scope(ck):
    # N = 2^16: a batch of limbs of every prime class (FP64 and 64-bit
    # engines), forward and inverse each against the oracle from random
    # residues; operations beyond plain transforms and element-wise ones
    # are refused with CKKS_EPARAMS
    from paper_2110_13638_amd import _native as nat
    log_n = 16
    primes = O.find_primes(log_n, [60, 50, 49, 60])
    orc = O.Oracle(log_n, primes[:3], primes[3:], 3)
    ctx = ck.Context(log_n, primes[:3], primes[3:], 3)
    pidx = [0, 1, 2, 3, 1, 2, 0]
    x = np.stack([S.residues(70 + k, [primes[i]], 1 << log_n)[0, 0] for k, i in enumerate(pidx)])
    for fp in (1, 0):
        ctx.set_tuning(ntt_fp=fp)
        print("N=2^16 transforms ntt_fp=%d" % fp, flush=True)
        dev = torch.from_numpy(x.view(np.int64).copy()).cuda()
        ptrs = [dev[k].data_ptr() for k in range(len(pidx))]
        ws, wb = ctx.ws_for(nat.CKKS_OP_NTT, len(pidx))
        nat.ckks_ntt(ctx.h, ptrs, pidx, ws, wb, ctx.stream)
        torch.cuda.synchronize()
        got = dev.cpu().numpy().view(np.uint64)
        for k, i in enumerate(pidx):
            assert np.array_equal(got[k], orc.ntt(x[k], i)), (fp, k)
        dev = torch.from_numpy(x.view(np.int64).copy()).cuda()
        ptrs = [dev[k].data_ptr() for k in range(len(pidx))]
        nat.ckks_intt(ctx.h, ptrs, pidx, ws, wb, ctx.stream)
        torch.cuda.synchronize()
        got = dev.cpu().numpy().view(np.uint64)
        for k, i in enumerate(pidx):
            assert np.array_equal(got[k], orc.intt(x[k], i)), (fp, k)
    a = ctx.ct_from_residues(S.residues(5, primes[:3], 1 << log_n, 2), 2.0 ** 40)
    b = ctx.add(a, a)  # element-wise: runs
    assert np.array_equal(b.residues(), orc.add(a.residues(), a.residues()))
    with pytest.raises(nat.CkksError) as e:
        ctx.rescale(a)
    assert e.value.code == nat.CKKS_EPARAMS
