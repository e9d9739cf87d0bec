"""The allocation-free HMult + relinearise + rescale entry point, through
the C ABI: on two calls in a row (the second with a smaller, ragged batch
on another ring) its outputs equal those of ckks_hmult_relin_rescale with a
caller workspace residue for residue, and one output of each call is also
checked against the oracle. A batch whose scratch exceeds the fixed array
is refused before anything is launched."""
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
    from paper_2110_13638_amd import _native as nat
    return ckks, nat


def _run_pair(ckks, nat, log_n, qb, pb, dnum, levels, seed):
    primes = O.find_primes(log_n, qb + pb)
    q, p = primes[: len(qb)], primes[len(qb):]
    ctx = ckks.Context(log_n, q, p, dnum).keygen(seed)
    A = [ctx.ct_from_residues(S.residues(seed * 100 + 2 * k, q[: lv + 1], ctx.N, 2), 2.0 ** 40)
         for k, lv in enumerate(levels)]
    B = [ctx.ct_from_residues(S.residues(seed * 100 + 2 * k + 1, q[: lv + 1], ctx.N, 2), 2.0 ** 40)
         for k, lv in enumerate(levels)]
    want = ctx.hmult_relin_rescale(A, B)
    outs = [ctx.new_ct(2, lv - 1, 1.0) for lv in levels]
    # the outputs start as garbage, not zeros: nothing may rely on them
    for o in outs:
        o.buf.fill_(-1)
    so = ctx._structs(outs)
    nat.ckks_hmult_relin_rescale_noalloc(ctx.h, ctx.rk.data_ptr(), ctx._structs(A), ctx._structs(B), so,
                                         ctx.stream)
    ctx._outs(so, outs)
    torch.cuda.synchronize()
    for w, g in zip(want, outs):
        assert g.level == w.level and g.scale == w.scale
        assert np.array_equal(g.residues(), w.residues())
    # one item against the oracle (independent of both entry points)
    orc = O.Oracle(log_n, q, p, dnum)
    _, sn = orc.keygen_secret(seed)
    rk = orc.keygen_relin(sn, seed + 2)
    k = len(levels) - 1
    ref = orc.mul_relin_rescale(A[k].residues(), B[k].residues(), rk)
    assert np.array_equal(outs[k].residues(), ref)
    return ctx


def test_noalloc_matches_workspace_call_twice(ck):
    ckks, nat = ck
    # first call: two pairs on the 2^15 chain (16 x 50-bit + 2 x 60-bit, dnum 4), ragged levels
    _run_pair(ckks, nat, 15, [50] * 16, [60, 60], 4, [15, 12], seed=5)
    # second call, smaller: three ragged pairs on a 2^13 chain; the array keeps the first call's contents
    _run_pair(ckks, nat, 13, [60, 40, 40, 40], [60], 4, [3, 1, 2], seed=7)


def test_noalloc_refuses_oversized_batch(ck):
    ckks, nat = ck
    primes = O.find_primes(15, [50] * 16 + [60, 60])
    ctx = ckks.Context(15, primes[:16], primes[16:], 4).keygen(1)
    levels = [15] * 3
    need = nat.ckks_workspace_bytes(ctx.h, nat.CKKS_OP_HMULT, len(levels), levels)
    assert need > nat.CKKS_NOALLOC_SCRATCH_BYTES
    A = [ctx.new_ct(2, 15) for _ in levels]
    outs = [ctx.new_ct(2, 14) for _ in levels]
    with pytest.raises(nat.CkksError) as e:
        nat.ckks_hmult_relin_rescale_noalloc(ctx.h, ctx.rk.data_ptr(), ctx._structs(A), ctx._structs(A),
                                             ctx._structs(outs), ctx.stream)
    assert e.value.code == nat.CKKS_ENOMEM
    assert "fixed scratch" in str(e.value)
