"""Python view of the C ABI graph runtime (the paper's Algorithms 1-5).

Nodes are created on a ``ckks_graph`` handle; ``run`` fires the graph on
device ciphertexts and returns the OUTPUT nodes' ciphertexts, which are
views into this object's workspace (valid until the next run).
"""
import ctypes

import numpy as np
import torch

from . import _native as nat
from .ckks import Ciphertext, _align


class Graph:
    def __init__(self, ctx):
        self.ctx = ctx
        self.g = nat.ckks_graph_create(ctx.h)
        self._ws = None
        self._ws_bytes = 0
        self._keep = []
        self.n_out = 0
        self.n_inputs = 0

    def __del__(self):
        g = getattr(self, "g", None)
        if g:
            # at interpreter exit the binding module may already be torn down
            destroy = getattr(nat, "ckks_graph_destroy", None)
            if destroy is not None:
                destroy(g)
            self.g = None

    # --- nodes -----------------------------------------------------------------
    def input(self, n_ct, level, scale):
        self.n_inputs += n_ct
        return nat.ckks_graph_add_node(self.g, nat.CKKS_NODE_INPUT, nat.ckks_input_attrs(n_ct, level, scale))

    def linear(self, rows, w_scale, bias=None):
        """rows[j] = [(input index, weight)] over the node's stacked inputs"""
        row_ptr = np.zeros(len(rows) + 1, dtype=np.uint32)
        cols, ws = [], []
        for j, r in enumerate(rows):
            cols += [int(c) for c, _ in r]
            ws += [float(w) for _, w in r]
            row_ptr[j + 1] = len(cols)
        col = np.ascontiguousarray(cols, dtype=np.uint32)
        w = np.ascontiguousarray(ws, dtype=np.float64)
        b = np.ascontiguousarray(bias, dtype=np.float64) if bias is not None else None
        P = ctypes.POINTER
        a = nat.ckks_linear_attrs(len(rows), row_ptr.ctypes.data_as(P(ctypes.c_uint32)),
                                  col.ctypes.data_as(P(ctypes.c_uint32)), w.ctypes.data_as(P(ctypes.c_double)),
                                  w_scale, b.ctypes.data_as(P(ctypes.c_double)) if b is not None else None)
        return nat.ckks_graph_add_node(self.g, nat.CKKS_NODE_LINEAR, a)

    def dense(self, W, w_scale, bias=None):
        W = np.asarray(W, dtype=np.float64)
        return self.linear([[(i, W[j, i]) for i in range(W.shape[1])] for j in range(W.shape[0])], w_scale, bias)

    def diag_dense(self, diag_coeffs, in_steps, pt_scale, post_steps=(), bias_slots=None, bias_coeffs=None,
                   hoisted=False):
        P = ctypes.POINTER
        d = np.ascontiguousarray(diag_coeffs, dtype=np.int64)
        st = np.ascontiguousarray(in_steps, dtype=np.int32)
        ps = np.ascontiguousarray(post_steps, dtype=np.int32) if len(post_steps) else None
        bs = np.ascontiguousarray(bias_slots, dtype=np.float64) if bias_slots is not None else None
        bc = np.ascontiguousarray(bias_coeffs, dtype=np.int64) if bias_coeffs is not None else None
        a = nat.ckks_diag_attrs(len(st), st.ctypes.data_as(P(ctypes.c_int32)), d.ctypes.data_as(P(ctypes.c_int64)),
                                pt_scale, len(post_steps), ps.ctypes.data_as(P(ctypes.c_int32)) if ps is not None
                                else None, bs.ctypes.data_as(P(ctypes.c_double)) if bs is not None else None,
                                len(bs) if bs is not None else 0,
                                bc.ctypes.data_as(P(ctypes.c_int64)) if bc is not None else None,
                                1 if hoisted else 0)
        return nat.ckks_graph_add_node(self.g, nat.CKKS_NODE_DIAG_DENSE, a)

    def square(self):
        return nat.ckks_graph_add_node(self.g, nat.CKKS_NODE_SQUARE)

    def poly(self, coeffs, w_scale=None):
        """polynomial activation sum_k coeffs[k] x^k (degree >= 1)"""
        c = np.ascontiguousarray(coeffs, dtype=np.float64)
        self._keep.append(c)
        a = nat.ckks_poly_attrs(len(c) - 1, c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                w_scale or self.ctx.default_scale)
        return nat.ckks_graph_add_node(self.g, nat.CKKS_NODE_POLY, a)

    def output(self):
        return nat.ckks_graph_add_node(self.g, nat.CKKS_NODE_OUTPUT)

    def edge(self, a, b):
        nat.ckks_graph_add_edge(self.g, a, b)
        return b

    def chain(self, *ids):
        for a, b in zip(ids, ids[1:]):
            self.edge(a, b)
        return ids[-1]

    # --- planning / execution ----------------------------------------------------------
    def plan(self):
        # workspace sizes depend on the context's launch shapes (e.g. the
        # fused HMult tail needs fewer scratch limbs): remember them
        self._planned_tuning = self.ctx.tuning()
        self._ws_bytes, self.n_out = nat.ckks_graph_plan(self.g)
        return self._ws_bytes, self.n_out

    def run(self, inputs, galois=None):
        if not self._ws_bytes or getattr(self, "_planned_tuning", None) != self.ctx.tuning():
            self.plan()
        ctx = self.ctx
        if self._ws is None or self._ws.numel() < self._ws_bytes + 256:
            self._ws = None
            self._ws = torch.empty(self._ws_bytes + 256, dtype=torch.uint8, device=ctx.device)
        ws = ctypes.c_void_p(_align(self._ws.data_ptr()))
        ins = (nat.ckks_ct * len(inputs))(*[c.struct() for c in inputs])
        outs = (nat.ckks_ct * self.n_out)()
        gk = ctx.gk if galois is None else galois
        elts = sorted(gk)
        nat.ckks_graph_run(self.g, ins, outs, ctx.rk.data_ptr() if ctx.rk is not None else None, elts,
                           [gk[e].data_ptr() for e in elts], ws, self._ws_bytes, ctx.stream)
        res = []
        base = self._ws
        for s in outs:
            # wrap the view: data pointer inside the workspace tensor
            off = s.data - base.data_ptr()
            stride = s.limb_stride
            n = 2 * stride * ctx.N
            buf = base[off: off + n * 8].view(torch.int64).view(2, stride, ctx.N)
            res.append(Ciphertext(ctx, buf, int(s.n_poly), int(s.level), float(s.scale)))
        return res
