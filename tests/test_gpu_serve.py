"""Serving engine: continuous batching gives every request the same result
it gets alone (bit-identical), and the same as the plain one-op-per-launch
path; admission by HBM footprint bounds what runs concurrently."""
import numpy as np
import pytest

import synthetic as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2110_13638_amd import ckks, serve, _native as nat
    ctxs = {}
    # HMult requests: 16 x 50-bit chain, two special primes, dnum 4 (two rings)
    for log_n in (11, 12):
        primes = nat.ckks_find_primes(log_n, [50] * 16 + [60, 60])
        ctxs[("hmult", log_n)] = ckks.Context(log_n, primes[:16], primes[16:], 4).keygen(5)
    # vision requests: [60, 40 x 7 | 60], one prime per digit
    primes = nat.ckks_find_primes(10, [60] + [40] * 7 + [60])
    vctx = ckks.Context(10, primes[:8], primes[8:], 8).keygen(6)
    ctxs[("vision", 10)] = vctx
    _, P = S.vision_inputs(n_images=4)
    vision = {10: serve.VisionModel(vctx, P)}
    return serve, ctxs, vision


def _requests(serve, ctxs, spec, rids=None):
    reqs = []
    for k, (kind, log_n, level, arrival) in enumerate(spec):
        rid = k if rids is None else rids[k]
        ctx = ctxs[(kind, log_n)]
        n_ct = 2 if kind == "hmult" else 784
        # inputs seeded by the request id: the same request has the same data alone and in a mix
        res = S.residues_device(100 + rid, ctx.q[: level + 1], ctx.N, 2 * n_ct, ctx.device).view(n_ct, 2, level + 1,
                                                                                                  ctx.N)
        from paper_2110_13638_amd.ckks import Ciphertext
        cts = [Ciphertext(ctx, res[i], 2, level, ctx.default_scale) for i in range(n_ct)]
        reqs.append(serve.Request(rid, kind, log_n, arrival, cts))
    return reqs


def _engine(serve, ctxs, vision, cap=64 << 30):
    return serve.Engine(ctxs, vision, hbm_cap=cap)


SPEC = [("hmult", 12, 15, 0.000), ("vision", 10, 7, 0.001), ("hmult", 11, 6, 0.001),
        ("hmult", 12, 9, 0.002), ("vision", 10, 6, 0.002), ("hmult", 11, 15, 0.003)]


def _res(r):
    return [c.residues() for c in r.result]


def test_alone_equals_mix_equals_plain(env):
    serve, ctxs, vision = env
    mix = _engine(serve, ctxs, vision).run(_requests(serve, ctxs, SPEC))
    mix = {r.rid: r for r in mix}
    assert len(mix) == len(SPEC)
    for rid, spec in enumerate(SPEC):
        print("request", rid, spec, flush=True)
        alone = _engine(serve, ctxs, vision).run(_requests(serve, ctxs, [spec[:3] + (0.0,)], rids=[rid]))[0]
        a, m = _res(alone), _res(mix[rid])
        assert len(a) == len(m) and all(np.array_equal(x, y) for x, y in zip(a, m)), rid
        assert alone.result[0].scale == mix[rid].result[0].scale
    plain = serve.run_plain(ctxs, vision, _requests(serve, ctxs, SPEC))
    for r in plain:
        m = _res(mix[r.rid])
        assert all(np.array_equal(x, y) for x, y in zip(_res(r), m)), r.rid
    st = serve.latency_stats(list(mix.values()))
    assert st["p99_ms"] >= st["p50_ms"] > 0


def test_admission_by_footprint(env):
    serve, ctxs, vision = env
    reqs = _requests(serve, ctxs, [("vision", 10, 7, 0.0), ("vision", 10, 7, 0.0)])
    eng = _engine(serve, ctxs, vision)
    one = eng.footprint(reqs[0])
    # room for one vision request at a time: both still finish, never together
    eng = _engine(serve, ctxs, vision, cap=one + one // 2)
    peak = [0]
    orig = eng.tick

    def tick(now, *rest):
        busy = orig(now, *rest)
        peak[0] = max(peak[0], len(eng.active))
        return busy

    eng.tick = tick
    done = eng.run(reqs)
    assert len(done) == 2 and peak[0] == 1
    from paper_2110_13638_amd import _native as nat
    small = _engine(serve, ctxs, vision, cap=one // 2)
    with pytest.raises(nat.CkksError):
        small.submit(_requests(serve, ctxs, [("vision", 10, 7, 0.0)])[0])


def test_clients_share_launches(env):
    """Requests of two clients (each with its own resident key set) in one
    mix: each result equals the request served alone and on the plain path
    with that client's keys, and an HMult result equals the fused call with
    the client's relinearisation key."""
    serve, ctxs, vision = env
    keys = {}
    for (kind, log_n), ctx in ctxs.items():
        for client in (0, 1):
            keys[(kind, log_n, client)] = ctx.client_keys(40 + 10 * client + log_n)
    spec = [("hmult", 12, 15, 0.000), ("hmult", 12, 11, 0.000), ("vision", 10, 7, 0.001),
            ("vision", 10, 7, 0.001), ("hmult", 11, 9, 0.002)]
    clients = [0, 1, 1, 0, 1]

    def reqs(sp, cl, rids=None):
        rs = _requests(serve, ctxs, sp, rids)
        for r, c in zip(rs, cl):
            r.client = c
        return rs

    eng = serve.Engine(ctxs, vision, hbm_cap=64 << 30, client_keys=keys)
    assert eng.used == eng.key_bytes > 0
    mix = {r.rid: r for r in eng.run(reqs(spec, clients))}
    assert eng.used == eng.key_bytes
    for rid, (sp, c) in enumerate(zip(spec, clients)):
        alone = serve.Engine(ctxs, vision, client_keys=keys).run(reqs([sp[:3] + (0.0,)], [c], rids=[rid]))[0]
        assert all(np.array_equal(x, y) for x, y in zip(_res(alone), _res(mix[rid]))), rid
    plain = serve.run_plain(ctxs, vision, reqs(spec, clients), client_keys=keys)
    for r in plain:
        assert all(np.array_equal(x, y) for x, y in zip(_res(r), _res(mix[r.rid]))), r.rid
    # the HMult requests really used their client's key
    for rid in (0, 1, 4):
        kind, log_n, level, _ = spec[rid]
        a, b = _requests(serve, ctxs, [spec[rid]], rids=[rid])[0].inputs
        ctx = ctxs[(kind, log_n)]
        want = ctx.hmult_relin_rescale([a], [b], rk=[keys[(kind, log_n, clients[rid])].rk])[0]
        assert np.array_equal(want.residues(), _res(mix[rid])[0])
        other = ctx.hmult_relin_rescale([a], [b], rk=[keys[(kind, log_n, 1 - clients[rid])].rk])[0]
        assert not np.array_equal(other.residues(), _res(mix[rid])[0])
