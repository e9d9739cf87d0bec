"""The serving engine's scheduling and failure handling on the CPU, with a
fake device backend: admission by footprint, continuous batching that does
not change a request's result, cancellation, timeouts and injected launch
faults (CKKS_FAULT_INJECT), where only the faulty request fails and every
other result stays identical to a fault-free run.

The fake backend computes a deterministic function per ciphertext (so a
result never depends on which batch it ran in, as with the real kernels)
and completes its events after a fixed number of queries."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2110_13638_amd import _native as nat  # noqa: E402
from paper_2110_13638_amd import serve  # noqa: E402

class FakeCt:
    def __init__(self, level, data, scale=1.0):
        self.level, self.data, self.scale, self.n_poly = level, np.asarray(data, dtype=np.int64), scale, 2

class FakeKeys:
    def __init__(self, tag):
        self.rk = torch.tensor([tag])  # a one-word "key" (8 resident bytes)
        self.pk = None
        self.gk = {}

class FakeCtx:
    """the Context methods the engine calls, on numpy vectors"""

    def __init__(self):
        self.rk = torch.tensor([7])
        self.launches = []  # batch size of every launch

    def hmult_relin_rescale(self, A, B, rk=None):
        self.launches.append(len(A))
        keys = rk if rk is not None else [self.rk] * len(A)
        return [FakeCt(a.level - 1, (a.data * b.data + int(k)) % 1000003) for a, b, k in zip(A, B, keys)]

    def linear_csr(self, flat, row_ptr, col, w, w_scale):
        self.launches.append(len(row_ptr) - 1)
        out = []
        for j in range(len(row_ptr) - 1):
            acc = np.zeros_like(flat[0].data)
            for e in range(int(row_ptr[j]), int(row_ptr[j + 1])):
                acc = (acc + int(w[e]) * flat[int(col[e])].data) % 1000003
            out.append(FakeCt(flat[0].level, acc))
        return out

    def rescale_inplace(self, cts):
        for c in cts:
            c.level -= 1
        return cts

    def add_scalars_inplace(self, cts, values):
        for c, v in zip(cts, values):
            c.data = (c.data + int(round(v * 100))) % 1000003
        return cts

    def rescale_add_scalars_inplace(self, cts, values):
        return self.add_scalars_inplace(self.rescale_inplace(cts), values)

class FakeVision:
    """two tiny linear layers around a square, in the VisionModel shape"""
    n_pix = 3
    w_scale = 1.0

    def __init__(self):
        def layer(n_in, n_out, seed):
            rng = np.random.default_rng(seed)
            row_ptr = np.arange(n_out + 1) * n_in
            col = np.tile(np.arange(n_in), n_out)
            return dict(row_ptr=row_ptr, col=col, w=rng.integers(-50, 50, n_in * n_out), n_in=n_in, n_out=n_out,
                        bias=rng.normal(0, 1, n_out))
        self.layers = [layer(3, 2, 1), "square", layer(2, 1, 2)]

    def block(self, layer, R):
        L = self.layers[layer]
        nnz = int(L["row_ptr"][-1])
        row_ptr = np.concatenate([[0]] + [L["row_ptr"][1:] + r * nnz for r in range(R)])
        col = np.concatenate([L["col"] + r * L["n_in"] for r in range(R)])
        return row_ptr, col, np.tile(L["w"], R), np.tile(L["bias"], R)

class FakeEvent:
    """completes after `lag` queries (work still in flight until then)"""
    lag = 2

    def __init__(self):
        self.n = 0

    def record(self):
        pass

    def query(self):
        self.n += 1
        return self.n > self.lag

    def synchronize(self):
        self.n = self.lag + 1

class FakeEngine(serve.Engine):
    def __init__(self, ctxs, vision, **kw):
        kw.setdefault("event_factory", FakeEvent)
        kw.setdefault("sync", lambda: None)
        super().__init__(ctxs, vision, **kw)

    def footprint(self, req):
        return 100 * (len(req.inputs) if not callable(req.inputs) else 3)

def _env():
    ctxs = {("hmult", 12): FakeCtx(), ("vision", 10): FakeCtx()}
    return ctxs, {10: FakeVision()}

def _reqs(spec):
    out = []
    for rid, (kind, arrival, client) in enumerate(spec):
        rng = np.random.default_rng(100 + rid)
        n = 2 if kind == "hmult" else 3
        log_n = 12 if kind == "hmult" else 10
        cts = [FakeCt(9, rng.integers(0, 1000, 4)) for _ in range(n)]
        out.append(serve.Request(rid, kind, log_n, arrival, cts, level=9, client=client))
    return out

SPEC = [("hmult", 0.0, 0), ("vision", 0.0, 1), ("hmult", 0.0, 1), ("vision", 0.0, 0), ("hmult", 0.0, 2),
        ("vision", 0.0, 2)]

def _keys():
    return {(k, n, c): FakeKeys(11 + c) for (k, n) in (("hmult", 12), ("vision", 10)) for c in range(3)}

def _results(done):
    return {r.rid: [c.data.copy() for c in r.result] for r in done}

def _run(spec, **kw):
    ctxs, vision = _env()
    eng = FakeEngine(ctxs, vision, client_keys=_keys(), **kw)
    done = eng.run(_reqs(spec))
    return eng, ctxs, done

def test_batched_equals_alone():
    eng, ctxs, done = _run(SPEC)
    assert len(done) == len(SPEC) and not eng.failed
    assert all(r.status == "done" for r in done)
    # requests of several clients shared launches
    assert max(ctxs[("hmult", 12)].launches) == 3 and max(ctxs[("vision", 10)].launches) > 2
    mix = _results(done)
    for rid, sp in enumerate(SPEC):
        ctxs, vision = _env()
        alone = FakeEngine(ctxs, vision, client_keys=_keys()).run([_reqs(SPEC)[rid]])
        assert all(np.array_equal(a, b) for a, b in zip(_results(alone)[rid], mix[rid]))
    # each client's key entered its own results
    ctxs, vision = _env()
    other = {k: FakeKeys(99) for k in _keys()}
    swapped = _results(FakeEngine(ctxs, vision, client_keys=other).run(_reqs(SPEC)))
    assert not np.array_equal(swapped[0][0], mix[0][0])
    assert eng.used == eng.key_bytes

def test_admission_cap_one_at_a_time():
    ctxs, vision = _env()
    eng = FakeEngine(ctxs, vision, hbm_cap=350)
    assert eng.key_bytes == 0
    peak = [0]
    orig = eng.tick

    def tick(now, *rest):
        busy = orig(now, *rest)
        peak[0] = max(peak[0], len(eng.active))
        return busy

    eng.tick = tick
    done = eng.run(_reqs([("vision", 0.0, 0), ("vision", 0.0, 0)]))
    assert len(done) == 2 and peak[0] == 1
    with pytest.raises(nat.CkksError):
        FakeEngine(ctxs, vision, hbm_cap=250).submit(_reqs([("vision", 0.0, 0)])[0])

def test_fault_injection_isolates_the_request(monkeypatch):
    _, _, ref = _run(SPEC)
    ref = _results(ref)
    monkeypatch.setenv("CKKS_FAULT_INJECT", "3")
    eng, _, done = _run(SPEC)
    assert sorted(r.rid for r in done) == [0, 1, 2, 4, 5]
    assert [r.rid for r in eng.failed] == [3] and eng.failed[0].status == "error"
    assert "injected fault" in eng.failed[0].error
    got = _results(done)
    for rid in got:
        assert all(np.array_equal(a, b) for a, b in zip(got[rid], ref[rid])), rid
    assert eng.used == eng.key_bytes  # every footprint released

def test_fault_in_a_later_stage():
    # the faulty request fails after its first stage ran in a batch
    ctxs, vision = _env()

    class Late(FakeEngine):
        def _launch(self, log_n, kind, stage, rs):
            if stage == 2 and any(r.rid == 1 for r in rs):
                raise nat.CkksError(nat.CKKS_EDEVICE, "device error in stage 2")
            return super()._launch(log_n, kind, stage, rs)

    eng = Late(ctxs, vision, client_keys=_keys())
    done = eng.run(_reqs(SPEC))
    assert [r.rid for r in eng.failed] == [1] and "stage 2" in eng.failed[0].error
    _, _, ref = _run(SPEC)
    ref = _results(ref)
    for rid, res in _results(done).items():
        assert all(np.array_equal(a, b) for a, b in zip(res, ref[rid]))

def test_cancel_and_timeout():
    ctxs, vision = _env()
    eng = FakeEngine(ctxs, vision, hbm_cap=350)
    reqs = _reqs([("vision", 0.0, 0), ("vision", 0.0, 0), ("vision", 0.0, 0), ("hmult", 0.0, 0)])
    reqs[2].timeout = 0.0  # cannot be admitted before its deadline (the cap holds one vision request)
    eng.cancel(1)
    done = eng.run(reqs)
    st = {r.rid: r.status for r in done + eng.failed}
    assert st == {0: "done", 1: "cancelled", 2: "timeout", 3: "done"}
    assert eng.used == eng.key_bytes == 0
    # a request cancelled while in flight stops after its current stage
    ctxs, vision = _env()
    eng = FakeEngine(ctxs, vision)
    reqs = _reqs([("vision", 0.0, 0), ("hmult", 0.0, 0)])
    orig = eng.tick
    calls = [0]

    def tick(now, *rest):
        calls[0] += 1
        if calls[0] == 2:
            eng.cancel(0)
        return orig(now, *rest)

    eng.tick = tick
    done = eng.run(reqs)
    assert [r.rid for r in done] == [1] and eng.failed[0].status == "cancelled"
    assert eng.failed[0].stage < len(FakeVision().layers)

def test_fault_inject_parsing():
    assert serve.fault_inject_ids("3, 17,") == {3, 17}
    assert serve.fault_inject_ids("") == set()
