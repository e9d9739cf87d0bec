"""Continuous-batching server for encrypted inference requests.

Requests of different kinds, ring degrees and levels arrive over time. The
engine keeps evaluation keys resident per ring (one context each), admits a
waiting request only when its HBM footprint fits under the cap, and at every
tick groups all in-flight requests that sit at the same stage of the same
program on the same ring into ONE batched launch of the C ABI. Requests that
arrive while others are on the device join at the next tick, so their work
shares launches with the requests already running (continuous batching, not
a queue). Each request's result is computed ciphertext by ciphertext by the
same kernels whatever batch it lands in, so it is bit-identical alone and in
the mix.

Each request belongs to a client, whose evaluation keys (made from that
client's own secret, the threat model of Section 2.3) stay resident in HBM
for the whole run and are counted against the admission cap; requests of
different clients share launches through the per-item key arrays of the
batched key-switching calls.

Programs:
  * ``hmult``: one fused HMult + relinearise + rescale of a ciphertext pair;
  * ``vision``: the slot-batched vision network (conv -> x^2 -> dense ->
    x^2 -> dense) on one request's pixel ciphertexts; linear layers of the
    requests in a group run as one block-diagonal sparse layer, squares as
    one fused HMult batch.

Failure handling: a request can be cancelled (``Engine.cancel``) or carry
a timeout (seconds after arrival); either ends it at the next tick, waiting
or in flight, and releases its HBM share. A launch that fails for a group is
retried request by request, so only the request that fails is dropped (with
its error) and the others continue unchanged. ``CKKS_FAULT_INJECT`` (a comma
separated list of request ids) makes every launch that carries one of those
requests fail, to exercise that path.

The plain path (``run_plain``) serves the same requests first-in first-out,
one operation per launch (B = 1, unfused multiply / relinearize / rescale),
on the same kernels.
"""
import os
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _native as nat
from . import nets


@dataclass
class Request:
    rid: int
    kind: str            # "hmult" | "vision"
    log_n: int
    arrival: float       # seconds from the start of the run
    inputs: object       # device Ciphertexts (owned by the request), or a callable
                         # that creates them when the request is admitted
    level: int = -1      # input level (needed before a lazy request is admitted)
    client: int = 0      # whose keys relinearise this request's products
    timeout: float = None  # seconds after arrival by which it must finish, or None
    stage: int = 0
    state: list = field(default_factory=list)
    footprint: int = 0
    admitted: float = -1.0
    done_event: object = None
    finish: float = -1.0
    result: list = None
    status: str = "pending"  # done | cancelled | timeout | error
    error: str = None


class VisionModel:
    """Per-ring sparse rows of the vision network (weights as integers)."""

    def __init__(self, ctx, P, side=28, w_scale=None):
        self.ctx = ctx
        self.w_scale = w_scale or ctx.default_scale
        F = P["conv_w"].shape[0]
        rows, out_side = nets.conv_rows(P["conv_w"], side)
        rows, order = nets.reorder_conv_rows(rows, F)
        per = out_side * out_side
        self.n_pix = side * side
        self.layers = []
        conv_bias = [P["conv_b"][i // per] for i in order]
        self.layers.append(self._csr(rows, conv_bias))
        self.layers.append("square")
        W1 = P["w1"][:, order]
        self.layers.append(self._csr([[(i, W1[j, i]) for i in range(W1.shape[1])] for j in range(W1.shape[0])],
                                     P["b1"]))
        self.layers.append("square")
        W2 = P["w2"]
        self.layers.append(self._csr([[(i, W2[j, i]) for i in range(W2.shape[1])] for j in range(W2.shape[0])],
                                     P["b2"]))

    def _csr(self, rows, bias):
        ws = self.w_scale
        row_ptr = np.zeros(len(rows) + 1, dtype=np.int64)
        cols, vals = [], []
        for j, r in enumerate(rows):
            for c, x in r:
                cols.append(c)
                vals.append(x)
            row_ptr[j + 1] = len(cols)
        n_in = max(cols) + 1
        w = nat.ckks_encode_scalars(self.ctx.h, vals, ws)  # integer weights round(x * scale), in C
        return dict(row_ptr=row_ptr, col=np.array(cols, dtype=np.int64), w=w,
                    n_in=n_in, n_out=len(rows), bias=np.asarray(bias, dtype=np.float64))

    def block(self, layer, R):
        """block-diagonal CSR of one linear layer over R requests"""
        L = self.layers[layer]
        nnz = int(L["row_ptr"][-1])
        row_ptr = np.concatenate([[0]] + [L["row_ptr"][1:] + r * nnz for r in range(R)])
        col = np.concatenate([L["col"] + r * L["n_in"] for r in range(R)])
        w = np.tile(L["w"], R)
        return row_ptr, col, w, np.tile(L["bias"], R)


def key_set_bytes(keys):
    """device bytes of one client's server-resident keys (public,
    relinearisation, Galois; the secret stays with the client)"""
    t = [keys.pk, keys.rk] + list(keys.gk.values())
    return sum(x.numel() * x.element_size() for x in t if x is not None)


def fault_inject_ids(spec=None):
    """request ids named by CKKS_FAULT_INJECT (or ``spec``): "3,17" -> {3, 17}"""
    spec = os.environ.get("CKKS_FAULT_INJECT", "") if spec is None else spec
    return {int(x) for x in str(spec).replace(" ", "").split(",") if x}


class Engine:
    def __init__(self, contexts, vision=None, hbm_cap=64 << 30, square_chunk=1024, client_keys=None,
                 event_factory=None, sync=None, fault_inject=None):
        self.ctx = contexts          # (kind, log_n) -> Context
        self.vision = vision or {}   # log_n -> VisionModel
        # (kind, log_n, client) -> KeySet resident on the device; without it
        # every request uses its context's own key set
        self.keys = client_keys or {}
        self.cap = hbm_cap
        self.square_chunk = square_chunk
        # resident keys occupy HBM for the whole run: admission counts them
        self.key_bytes = sum(key_set_bytes(k) for k in self.keys.values())
        self.used = self.key_bytes
        self.waiting, self.active, self.done = [], [], []
        self.failed = []             # cancelled, timed out or failed requests
        self._cancel = set()
        self._event = event_factory or torch.cuda.Event
        self._sync = sync or torch.cuda.synchronize
        self.fault = fault_inject_ids(fault_inject)

    def _rk(self, r):
        k = self.keys.get((r.kind, r.log_n, r.client))
        return k.rk if k is not None else self.ctx[(r.kind, r.log_n)].rk

    # --- memory accounting ---------------------------------------------------
    def footprint(self, req):
        ctx = self.ctx[(req.kind, req.log_n)]
        lvl = req.level if callable(req.inputs) else req.inputs[0].level
        if req.kind == "hmult":
            levels = [lvl]
            return 2 * nat.ckks_ct_bytes(ctx.h, 2, lvl) + nat.ckks_workspace_bytes(ctx.h, nat.CKKS_OP_HMULT, 1, levels)
        m = self.vision[req.log_n]
        n1 = m.layers[0]["n_out"]
        # inputs, conv outputs, square outputs, fused-HMult scratch per ciphertext
        per = nat.ckks_ct_bytes(ctx.h, 2, lvl)
        n_in = m.n_pix if callable(req.inputs) else len(req.inputs)
        return (n_in + 2 * n1) * per + n1 * nat.ckks_workspace_bytes(ctx.h, nat.CKKS_OP_HMULT, 1, [lvl])

    # --- lifecycle -------------------------------------------------------------
    def submit(self, req):
        req.footprint = self.footprint(req)
        if req.footprint > self.cap - self.key_bytes:
            raise nat.CkksError(nat.CKKS_ENOMEM, "request %d needs %d bytes; the cap leaves %d beside the "
                                "resident keys" % (req.rid, req.footprint, self.cap - self.key_bytes))
        self.waiting.append(req)

    def cancel(self, rid):
        """end request ``rid`` at the next tick (waiting or in flight)"""
        self._cancel.add(rid)

    def _drop(self, r, status, stamp, msg=None, active=False):
        r.status, r.error = status, msg
        r.finish = stamp()
        if active:
            self.used -= r.footprint
        # its buffers are released; kernels already queued on the stream still
        # run before the allocator hands the memory to later work
        r.inputs = r.state = r.result = None
        self.failed.append(r)

    def _expire(self, now, stamp):
        def why(r):
            if r.rid in self._cancel:
                return "cancelled"
            if r.timeout is not None and now > r.arrival + r.timeout:
                return "timeout"
            return None

        keep = []
        for r in self.waiting:
            w = why(r) if r.arrival <= now or r.rid in self._cancel else None
            if w:
                self._drop(r, w, stamp)
            else:
                keep.append(r)
        self.waiting = keep
        keep = []
        for r in self.active:
            w = why(r) if r.done_event is None else None  # the last stage is queued: let it finish
            if w:
                self._drop(r, w, stamp, active=True)
            else:
                keep.append(r)
        self.active = keep

    def _admit(self, now):
        keep = []
        for r in self.waiting:
            if r.arrival <= now and self.used + r.footprint <= self.cap:
                self.used += r.footprint
                r.admitted = now
                if callable(r.inputs):
                    r.inputs = r.inputs()
                r.state = list(r.inputs)
                self.active.append(r)
            else:
                keep.append(r)
        self.waiting = keep

    def _retire(self, stamp):
        keep = []
        for r in self.active:
            if r.done_event is not None and r.done_event.query():
                r.finish = stamp()  # when the completion is observed, not when the tick began
                r.status = "done"
                self.used -= r.footprint
                r.inputs = r.state = None  # the result stays; inputs and intermediates are released
                self.done.append(r)
            else:
                keep.append(r)
        self.active = keep

    def _n_stages(self, r):
        return 1 if r.kind == "hmult" else len(self.vision[r.log_n].layers)

    def tick(self, now, stamp=None):
        stamp = stamp or (lambda: now)
        self._expire(now, stamp)
        self._admit(now)
        groups = {}
        for r in self.active:
            if r.done_event is None:
                # the fused HMult batch takes ragged levels; a block-diagonal
                # linear layer needs one level, so vision stages also group by level
                lvl = r.state[0].level if r.kind == "vision" else -1
                groups.setdefault((r.log_n, r.kind, r.stage, lvl), []).append(r)
        for (log_n, kind, stage, _), rs in groups.items():
            for r in self._launch_isolated(log_n, kind, stage, rs, stamp):
                r.stage += 1
                if r.stage == self._n_stages(r):
                    r.result = r.state
                    ev = self._event()
                    ev.record()
                    r.done_event = ev
        self._retire(stamp)
        return bool(groups)

    def _launch_isolated(self, log_n, kind, stage, rs, stamp):
        """Launch a group; if it fails, launch its requests one by one and
        drop the ones that still fail. Returns the requests that advanced."""
        try:
            self._launch(log_n, kind, stage, rs)
            return rs
        except nat.CkksError as e:
            if len(rs) == 1:
                self._fail(rs[0], e, stamp)
                return []
        ok = []
        for r in rs:
            try:
                self._launch(log_n, kind, stage, [r])
                ok.append(r)
            except nat.CkksError as e:
                self._fail(r, e, stamp)
        return ok

    def _fail(self, r, err, stamp):
        self.active.remove(r)
        self._drop(r, "error", stamp, str(err), active=True)

    def _launch(self, log_n, kind, stage, rs):
        bad = sorted(r.rid for r in rs if r.rid in self.fault)
        if bad:
            raise nat.CkksError(nat.CKKS_EDEVICE, "injected fault for request(s) %s (CKKS_FAULT_INJECT)" % bad)
        ctx = self.ctx[(kind, log_n)]
        if kind == "hmult":
            outs = ctx.hmult_relin_rescale([r.state[0] for r in rs], [r.state[1] for r in rs],
                                           rk=[self._rk(r) for r in rs])
            for r, o in zip(rs, outs):
                r.state = [o]
            return
        m = self.vision[log_n]
        layer = m.layers[stage]
        if layer == "square":
            flat = [c for r in rs for c in r.state]
            keys = [self._rk(r) for r in rs for _ in r.state]
            outs = []
            for k in range(0, len(flat), self.square_chunk):
                part = flat[k:k + self.square_chunk]
                outs += ctx.hmult_relin_rescale(part, part, rk=keys[k:k + self.square_chunk])
            k = 0
            for r in rs:
                n = len(r.state)
                r.state = outs[k:k + n]
                k += n
            return
        R = len(rs)
        row_ptr, col, w, bias = m.block(stage, R)
        flat = [c for r in rs for c in r.state]
        outs = ctx.linear_csr(flat, row_ptr, col, w, m.w_scale)
        ctx.rescale_add_scalars_inplace(outs, bias)
        n = layer["n_out"]
        for i, r in enumerate(rs):
            r.state = outs[i * n:(i + 1) * n]

    def run(self, requests, clock=time.perf_counter):
        """Serve requests whose ``arrival`` offsets are seconds from now."""
        for r in sorted(requests, key=lambda r: r.arrival):
            self.submit(r)
        t0 = clock()

        def stamp():
            return clock() - t0

        while self.waiting or self.active:
            now = stamp()
            busy = self.tick(now, stamp)
            if not busy:
                # nothing to launch: sleep until the next arrival or completion
                nxt = min([r.arrival for r in self.waiting], default=now)
                if self.active:
                    self.active[0].done_event.synchronize()
                elif nxt > now:
                    time.sleep(min(nxt - now, 0.002))
        self._sync()
        return self.done


# ---------------------------------------------------------------------------
# plain path: FIFO, one operation per launch
# ---------------------------------------------------------------------------
def _plain_square(ctx, c, rk):
    t = ctx.multiply(c, c)
    r = ctx.relinearize(t, rk=rk)
    return ctx.rescale(r)


def run_plain(contexts, vision, requests, clock=time.perf_counter, client_keys=None):
    keys = client_keys or {}
    t0 = clock()
    for req in sorted(requests, key=lambda r: r.arrival):
        while clock() - t0 < req.arrival:
            time.sleep(0.0005)
        if callable(req.inputs):
            req.inputs = req.inputs()
        ctx = contexts[(req.kind, req.log_n)]
        k = keys.get((req.kind, req.log_n, req.client))
        rk = [k.rk if k is not None else ctx.rk]
        if req.kind == "hmult":
            a, b = req.inputs
            t = ctx.multiply(a, b)
            req.result = [ctx.rescale(ctx.relinearize(t, rk=rk))]
        else:
            m = vision[req.log_n]
            state = list(req.inputs)
            for stage, layer in enumerate(m.layers):
                if layer == "square":
                    state = [_plain_square(ctx, c, rk) for c in state]
                    continue
                out = []
                rp, col, w = layer["row_ptr"], layer["col"], layer["w"]
                for j in range(layer["n_out"]):
                    a, b = int(rp[j]), int(rp[j + 1])
                    o = ctx.linear_csr(state, np.array([0, b - a]), col[a:b], w[a:b], m.w_scale)[0]
                    o = ctx.rescale(o)
                    o = ctx.add_scalar(o, layer["bias"][j])
                    out.append(o)
                state = out
            req.result = state
        torch.cuda.synchronize()
        req.finish = clock() - t0
    return requests


def latency_stats(requests):
    lat = np.array([r.finish - r.arrival for r in requests])
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3)}
