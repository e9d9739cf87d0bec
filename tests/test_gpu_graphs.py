"""Launch recording and HIP graph replay: a recorded batched HMult and a
recorded network run are captured into a HIP graph (torch.cuda.graph) and
replayed several times on new inputs written into the same buffers, with
eager work and synchronisations between replays; every replay is checked
bit-exact against the oracle (HMult) or against an eager run of the same
network on the same inputs."""
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


def test_recorded_hmult_graph_replays(ck):
    from paper_2110_13638_amd import _native as nat
    primes = O.find_primes(12, [50] * 16 + [60, 60])
    ctx = ck.Context(12, primes[:16], primes[16:], 4).keygen(3)
    orc = O.Oracle(12, primes[:16], primes[16:], 4)
    _, sn = orc.keygen_secret(3)
    rk = orc.keygen_relin(sn, 5)
    levels = [l - 1 for l in S.ragged_limbs(6)]
    bufs = [torch.zeros(4, lv + 1, ctx.N, dtype=torch.int64, device=ctx.device) for lv in levels]
    A = [ck.Ciphertext(ctx, b[:2], 2, lv, 1.0) for b, lv in zip(bufs, levels)]
    B = [ck.Ciphertext(ctx, b[2:], 2, lv, 1.0) for b, lv in zip(bufs, levels)]
    outs = [ctx.new_ct(2, lv - 1, 1.0) for lv in levels]

    def fill(seed):
        res = []
        for i, lv in enumerate(levels):
            r = S.residues(seed + i, ctx.q[: lv + 1], ctx.N, 4)
            bufs[i].copy_(torch.from_numpy(r.view(np.int64)))
            res.append(r)
        return res

    def check(res, tag):
        torch.cuda.synchronize()
        for i in range(len(levels)):
            want = orc.mul_relin_rescale(res[i][:2], res[i][2:], rk)
            assert np.array_equal(outs[i].residues(), want), (tag, i)

    ctx.ws_for(nat.CKKS_OP_HMULT, len(A), levels)  # size the workspace before recording
    res = fill(400)
    with ctx.record() as rec:
        ctx.hmult_relin_rescale(A, B, outs=outs)
    plan = rec.plan
    assert plan.n_launches >= 6 and plan.arena_used > 0
    check(res, "recorded run")
    # plain replay of the plan on new inputs
    res = fill(500)
    plan.launch()
    check(res, "plan replay")
    # HIP graph capture of the plan, replayed on new inputs with eager work between
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.launch()
    side = [ctx.new_ct(2, lv - 1, 1.0) for lv in levels]
    for k in range(3):
        print("graph replay", k, flush=True)
        res = fill(600 + 10 * k)
        g.replay()
        check(res, "graph replay %d" % k)
        # eager work of the program between replays: the same op into other buffers
        ctx.hmult_relin_rescale(A, B, outs=side)
        torch.cuda.synchronize()
        for i in range(len(levels)):
            assert torch.equal(side[i].buf[:, : levels[i]], outs[i].buf[:, : levels[i]])


def test_recorded_network_graph_replays(ck):
    from paper_2110_13638_amd import serve
    from paper_2110_13638_amd import graph as G
    logn = 10
    primes = O.find_primes(logn, [60] + [40] * 7 + [60])
    ctx = ck.Context(logn, primes[:8], primes[8:], 8).keygen(6)
    _, P = S.vision_inputs(n_images=4)
    model = serve.VisionModel(ctx, P)
    # the vision network as a graph: conv (sparse) -> x^2 -> dense -> x^2 -> dense
    g = G.Graph(ctx)
    x = g.input(784, 7, ctx.default_scale)
    prev = x
    for layer in model.layers:
        if layer == "square":
            nxt = g.square()
        else:
            rows = [[(int(c), float(w) / model.w_scale) for c, w in
                     zip(layer["col"][layer["row_ptr"][j]:layer["row_ptr"][j + 1]],
                         layer["w"][layer["row_ptr"][j]:layer["row_ptr"][j + 1]])] for j in range(layer["n_out"])]
            nxt = g.linear(rows, model.w_scale, bias=layer["bias"])
        g.edge(prev, nxt)
        prev = nxt
    g.edge(prev, g.output())
    g.plan()
    buf = torch.zeros(784, 2, 8, ctx.N, dtype=torch.int64, device=ctx.device)
    cts = [ck.Ciphertext(ctx, buf[i], 2, 7, ctx.default_scale) for i in range(784)]

    def fill(seed):
        buf.copy_(S.residues_device(seed, ctx.q, ctx.N, 784 * 2, ctx.device).view(784, 2, 8, ctx.N))

    fill(1)
    g.run(cts)  # allocate the graph workspace outside the recording
    ctx.workspace(1 << 24)
    fill(2)
    with ctx.record(256 << 20) as rec:
        outs = g.run(cts)
    plan = rec.plan
    first = [o.residues().copy() for o in outs]
    cap = torch.cuda.CUDAGraph()
    with torch.cuda.graph(cap):
        plan.launch()
    for k in range(3):
        print("network replay", k, flush=True)
        fill(10 + k)
        cap.replay()
        torch.cuda.synchronize()
        got = [o.residues().copy() for o in outs]
        # eager run of the same graph on the same inputs
        eager = g.run(cts)
        torch.cuda.synchronize()
        for a, b in zip(got, eager):
            assert np.array_equal(a, b.residues()), k
        assert not all(np.array_equal(a, b) for a, b in zip(got, first))
