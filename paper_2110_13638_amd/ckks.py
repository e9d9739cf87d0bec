"""Device-resident RNS-CKKS objects over the C ABI.

PyTorch provides device memory and the current stream only; every step of
the arithmetic runs in libckks_hip.so. ``Ciphertext`` follows the paper's
container semantics (Section 4.1): after a ciphertext product it
relinearises and rescales, and before a binary op it switches the higher
operand down the modulus chain so that levels match; scales must then be
equal (the lowering keeps branch depths equal).
"""
import ctypes

import numpy as np
import torch

from . import _native as nat


def _align(ptr, a=256):
    return (ptr + a - 1) // a * a


class Plaintext:
    def __init__(self, ctx, buf, level, scale):
        self.ctx, self.buf, self.level, self.scale = ctx, buf, level, scale

    def struct(self):
        return nat.ckks_pt(self.buf.data_ptr(), self.level, 0, self.scale)


class Ciphertext:
    """[n_poly][limb_stride][N] uint64 residues (stored as int64) in NTT form."""

    def __init__(self, ctx, buf, n_poly, level, scale):
        self.ctx, self.buf = ctx, buf
        self.n_poly, self.level, self.scale = n_poly, level, scale

    @property
    def limb_stride(self):
        return self.buf.shape[1]

    def struct(self):
        return nat.ckks_ct(self.buf.data_ptr(), self.n_poly, self.level, self.limb_stride, 0, self.scale)

    def update(self, s):
        self.n_poly, self.level, self.scale = int(s.n_poly), int(s.level), float(s.scale)
        return self

    def residues(self):
        """host uint64 array [n_poly][level+1][N]"""
        return self.buf[: self.n_poly, : self.level + 1].cpu().numpy().view(np.uint64)

    def copy(self):
        return Ciphertext(self.ctx, self.buf.clone(), self.n_poly, self.level, self.scale)

    # --- container semantics (Section 4.1) --------------------------------
    def _match(self, other):
        a, b = self, other
        if a.level > b.level:
            a = a.ctx.mod_switch(a, b.level)
        elif b.level > a.level:
            b = b.ctx.mod_switch(b, a.level)
        return a, b

    def __add__(self, other):
        if isinstance(other, Ciphertext):
            a, b = self._match(other)
            return self.ctx.add(a, b)
        return self.ctx.add_scalar(self, float(other))

    def __sub__(self, other):
        a, b = self._match(other)
        return self.ctx.sub(a, b)

    def __mul__(self, other):
        if isinstance(other, Ciphertext):
            a, b = self._match(other)
            return self.ctx.hmult_relin_rescale([a], [b])[0]
        if isinstance(other, Plaintext):
            return self.ctx.rescale(self.ctx.multiply_plain(self, other))
        return self.ctx.rescale(self.ctx.multiply_scalar(self, float(other)))


class Plan:
    """Recorded kernel launches of a sequence of calls on one context.

    ``launch()`` re-issues them on the current stream (no copies, no
    allocation), so it may run inside ``torch.cuda.graph`` capture. The
    buffers the recorded calls used must stay alive: the plan keeps the
    arena, and the caller keeps inputs, outputs and the context."""

    def __init__(self, ctx, handle, arena, used):
        self.ctx, self.h, self.arena, self.arena_used = ctx, handle, arena, used
        self.workspace = ctx._ws  # the recorded launches address this buffer

    @property
    def n_launches(self):
        return nat.ckks_plan_launch_count(self.h)

    def launch(self):
        nat.ckks_plan_launch(self.h, self.ctx.stream)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            nat.ckks_plan_destroy(h)
            self.h = None


class _Recording:
    def __init__(self, ctx, arena_bytes):
        self.ctx, self.arena_bytes, self.plan = ctx, arena_bytes, None

    def __enter__(self):
        self.arena = torch.empty(self.arena_bytes + 256, dtype=torch.uint8, device=self.ctx.device)
        self.ctx._recording = True
        nat.ckks_record_begin(self.ctx.h, _align(self.arena.data_ptr()), self.arena_bytes)
        return self

    def __exit__(self, *exc):
        self.ctx._recording = False
        h, used = nat.ckks_record_end(self.ctx.h)
        self.plan = Plan(self.ctx, h, self.arena, used)
        if exc[0] is not None:
            self.plan = None
        return False


class KeySet:
    """One client's keys on a ring: secret (client side only), public,
    relinearisation and Galois keys by element (server resident)."""

    def __init__(self):
        self.sk = self.pk = self.rk = None
        self.gk = {}


class Context:
    """Parameters, device tables, keys and a reusable workspace."""

    def __init__(self, log_n, q, p, dnum, device="cuda", default_scale=2.0 ** 40):
        self.log_n, self.N = log_n, 1 << log_n
        self.q, self.p, self.dnum = [int(x) for x in q], [int(x) for x in p], dnum
        self.primes = self.q + self.p
        self.device = torch.device(device)
        self.default_scale = default_scale
        self.h = nat.ckks_ctx_create(log_n, self.q, self.p, dnum)
        nb = nat.ckks_ctx_device_bytes(self.h)
        self._tables = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        nat.ckks_ctx_upload(self.h, _align(self._tables.data_ptr()), self.stream)
        self._ws = None
        self._recording = False
        self.sk = self.pk = self.rk = None
        self.gk = {}

    @classmethod
    def from_bits(cls, log_n, q_bits, p_bits, dnum, **kw):
        primes = nat.ckks_find_primes(log_n, list(q_bits) + list(p_bits))
        return cls(log_n, primes[: len(q_bits)], primes[len(q_bits):], dnum, **kw)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            try:
                torch.cuda.synchronize(self.device)
            except Exception:
                pass
            # at interpreter exit the binding module may already be torn down
            destroy = getattr(nat, "ckks_ctx_destroy", None)
            if destroy is not None:
                destroy(h)
            self.h = None

    # --- plumbing -----------------------------------------------------------
    @property
    def stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    @property
    def max_level(self):
        return len(self.q) - 1

    def digits(self, level):
        return nat.ckks_ctx_digits(self.h, level)

    TUNING_KNOBS = {"ntt_wide": nat.CKKS_TUNE_NTT_WIDE, "ew_log": nat.CKKS_TUNE_EW_LOG,
                    "xcd_remap": nat.CKKS_TUNE_XCD_REMAP, "fuse_tail": nat.CKKS_TUNE_FUSE_TAIL,
                    "ip_cts": nat.CKKS_TUNE_IP_CTS, "lin_mfma": nat.CKKS_TUNE_LIN_MFMA,
                    "ntt_fp": nat.CKKS_TUNE_NTT_FP}

    def tuning(self):
        return {k: nat.ckks_ctx_get_tuning(self.h, v) for k, v in self.TUNING_KNOBS.items()}

    def set_tuning(self, **knobs):
        for k, v in knobs.items():
            nat.ckks_ctx_set_tuning(self.h, self.TUNING_KNOBS[k], int(v))
        return self

    # --- serialisation (client <-> server transfer) ---------------------------
    def serialize(self, ct):
        return nat.ckks_serialize(self.h, nat.CKKS_OBJ_CT, ct.struct(), 0, self.stream)

    def deserialize(self, data, level=None):
        """a new ciphertext from bytes (room for ``level``, default the stored one)"""
        import struct as _st
        n_poly, lv = _st.unpack_from("<II", data, 28)
        out = self.new_ct(n_poly, lv if level is None else level)
        s = out.struct()
        nat.ckks_deserialize(self.h, nat.CKKS_OBJ_CT, data, s, 0, self.stream)
        return out.update(s)

    def record(self, arena_bytes=64 << 20):
        """``with ctx.record() as r: ...`` records the calls made in the
        block; ``r.plan`` replays their launches. The workspace must not be
        reallocated while recording (size it first with ``workspace``)."""
        return _Recording(self, arena_bytes)

    def workspace(self, nbytes):
        nbytes = max(int(nbytes), 1 << 20)
        if self._ws is None or self._ws.numel() < nbytes + 256:
            if self._recording and self._ws is not None:
                raise RuntimeError("workspace would move while recording: size it with ctx.workspace() first")
            self._ws = None
            self._ws = torch.empty(int(nbytes * 1.25) + 256, dtype=torch.uint8, device=self.device)
        return ctypes.c_void_p(_align(self._ws.data_ptr())), self._ws.numel() - 256

    def ws_for(self, op, B, levels=None):
        return self.workspace(nat.ckks_workspace_bytes(self.h, op, B, levels))

    def limbs(self, *shape):
        return torch.empty(*shape, self.N, dtype=torch.int64, device=self.device)

    def new_ct(self, n_poly, level, scale=1.0, stride=None):
        return Ciphertext(self, self.limbs(n_poly, stride or level + 1), n_poly, level, scale)

    def ct_from_residues(self, res, scale=1.0):
        """host uint64 [n_poly][L][N] -> device ciphertext"""
        res = np.ascontiguousarray(res, dtype=np.uint64)
        buf = torch.from_numpy(res.view(np.int64)).to(self.device)
        return Ciphertext(self, buf, res.shape[0], res.shape[1] - 1, scale)

    # --- keys -----------------------------------------------------------------
    def keygen(self, seed=1, galois_steps=()):
        """this context's default key set (secret seed, public seed + 1,
        relinearisation seed + 2, Galois seed + 3)"""
        k = self.client_keys(seed)
        self.sk, self.pk, self.rk = k.sk, k.pk, k.rk
        for s in galois_steps:
            self.add_galois_key(self.galois_elt(s), seed + 3)
        return self

    def client_keys(self, seed, galois_steps=()):
        """Another client's key set on the same ring (same seeds rule as
        keygen). Its rk / gk pointers go into the per-item key arrays of the
        batched key-switching calls, so requests of several clients share
        launches."""
        k = KeySet()
        k.sk = torch.empty(len(self.primes), self.N, dtype=torch.int64, device=self.device)
        ws, wb = self.ws_for(nat.CKKS_OP_KEYGEN, 1)
        nat.ckks_keygen_secret(self.h, seed, k.sk.data_ptr(), ws, wb, self.stream)
        k.pk = torch.empty(2, len(self.q), self.N, dtype=torch.int64, device=self.device)
        nat.ckks_keygen_public(self.h, k.sk.data_ptr(), seed + 1, k.pk.data_ptr(), ws, wb, self.stream)
        k.rk = self.new_switch_key()
        nat.ckks_keygen_relin(self.h, k.sk.data_ptr(), seed + 2, k.rk.data_ptr(), ws, wb, self.stream)
        for st in galois_steps:
            g = self.galois_elt(st)
            gk = self.new_switch_key()
            nat.ckks_keygen_galois(self.h, k.sk.data_ptr(), g, seed + 3, gk.data_ptr(), ws, wb, self.stream)
            k.gk[g] = gk
        return k

    def key_bytes(self):
        """device bytes of one switching key (relinearisation or Galois)"""
        return nat.ckks_key_bytes(self.h, nat.CKKS_KEY_SWITCH)

    def new_switch_key(self):
        return torch.empty(self.digits(self.max_level), 2, len(self.primes), self.N, dtype=torch.int64,
                           device=self.device)

    def galois_elt(self, step):
        return nat.ckks_galois_elt(self.h, step)

    def add_galois_key(self, g, seed):
        if g in self.gk:
            return self.gk[g]
        k = self.new_switch_key()
        ws, wb = self.ws_for(nat.CKKS_OP_KEYGEN, 1)
        nat.ckks_keygen_galois(self.h, self.sk.data_ptr(), g, seed, k.data_ptr(), ws, wb, self.stream)
        self.gk[g] = k
        return k

    # --- encoding -----------------------------------------------------------------
    def encode_coeffs(self, z, scale):
        z = np.asarray(z)
        re = np.ascontiguousarray(np.real(z), dtype=np.float64)
        im = np.ascontiguousarray(np.imag(z), dtype=np.float64) if np.iscomplexobj(z) else None
        out = np.zeros(self.N, dtype=np.int64)
        nat.ckks_encode(self.h, re.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        im.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if im is not None else None,
                        len(re), scale, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        return out

    def pt_from_coeffs(self, coeffs, level, scale):
        dev = torch.from_numpy(np.ascontiguousarray(coeffs, dtype=np.int64)).to(self.device)
        pt = Plaintext(self, self.limbs(level + 1), level, scale)
        ws, wb = self.ws_for(nat.CKKS_OP_NTT, level + 1)
        s = pt.struct()
        nat.ckks_pt_load(self.h, dev.data_ptr(), s, ws, wb, self.stream)
        return pt

    def encode(self, z, level=None, scale=None):
        level = self.max_level if level is None else level
        scale = scale or self.default_scale
        return self.pt_from_coeffs(self.encode_coeffs(z, scale), level, scale)

    def decode(self, residues, level, scale, n=None):
        n = n or self.N // 2
        res = np.ascontiguousarray(residues, dtype=np.uint64)
        re = np.zeros(n)
        im = np.zeros(n)
        dp = ctypes.POINTER(ctypes.c_double)
        nat._call("ckks_decode", self.h, res.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), level, scale,
                  re.ctypes.data_as(dp), im.ctypes.data_as(dp), n)
        return re + 1j * im

    # --- encryption ---------------------------------------------------------------
    def encrypt(self, pt, seed=7, obj=0, keys=None):
        ct = self.new_ct(2, pt.level, pt.scale)
        s = ct.struct()
        ws, wb = self.ws_for(nat.CKKS_OP_ENCRYPT, 1, [pt.level])
        pk = (keys or self).pk
        nat.ckks_encrypt(self.h, pk.data_ptr(), pt.struct(), seed, obj, s, ws, wb, self.stream)
        return ct.update(s)

    def decrypt_residues(self, ct, keys=None):
        m = self.limbs(ct.level + 1)
        ws, wb = self.ws_for(nat.CKKS_OP_NTT, ct.level + 1)
        sk = (keys or self).sk
        nat.ckks_decrypt(self.h, sk.data_ptr(), ct.struct(), m.data_ptr(), ws, wb, self.stream)
        return m.cpu().numpy().view(np.uint64)

    def decrypt(self, ct, n=None, keys=None):
        return self.decode(self.decrypt_residues(ct, keys), ct.level, ct.scale, n)

    # --- evaluation (batched: lists of ciphertexts) ----------------------------------
    @staticmethod
    def _structs(cts):
        return (nat.ckks_ct * len(cts))(*[c.struct() for c in cts])

    def _outs(self, structs, cts):
        for s, c in zip(structs, cts):
            c.update(s)
        return cts

    def _ew(self, fn, a, b, n_poly_out=None, extra=()):
        single = isinstance(a, Ciphertext)
        A = [a] if single else list(a)
        Bs = ([b] if single else list(b)) if b is not None else None
        outs = [self.new_ct(n_poly_out or x.n_poly, x.level, x.scale) for x in A]
        sa, so = self._structs(A), self._structs(outs)
        ws, wb = self.ws_for(nat.CKKS_OP_ELEMENTWISE, len(A), [x.level for x in A])
        if Bs is None:
            fn(self.h, sa, *extra, so, ws, wb, self.stream)
        else:
            sb = Bs if isinstance(Bs[0], ctypes.Array) else None
            fn(self.h, sa, self._structs(Bs) if sb is None else sb, so, ws, wb, self.stream)
        self._outs(so, outs)
        return outs[0] if single else outs

    def add(self, a, b):
        return self._ew(nat.ckks_add, a, b)

    def sub(self, a, b):
        return self._ew(nat.ckks_sub, a, b)

    def multiply(self, a, b):
        return self._ew(nat.ckks_multiply, a, b, n_poly_out=3)

    def _ptop(self, fn, a, pts):
        single = isinstance(a, Ciphertext)
        A = [a] if single else list(a)
        P = [pts] if single else list(pts)
        outs = [self.new_ct(x.n_poly, x.level, x.scale) for x in A]
        sp = (nat.ckks_pt * len(P))(*[p.struct() for p in P])
        so = self._structs(outs)
        ws, wb = self.ws_for(nat.CKKS_OP_ELEMENTWISE, len(A), [x.level for x in A])
        fn(self.h, self._structs(A), sp, so, ws, wb, self.stream)
        self._outs(so, outs)
        return outs[0] if single else outs

    def add_plain(self, a, pt):
        return self._ptop(nat.ckks_add_plain, a, pt)

    def multiply_plain(self, a, pt):
        return self._ptop(nat.ckks_multiply_plain, a, pt)

    def const_int(self, c, scale):
        """the constant polynomial round_half_away(c * scale), rounded in C"""
        return int(nat.ckks_encode_scalars(self.h, [c], scale)[0])

    def multiply_scalar(self, a, c, c_scale=None):
        c_scale = c_scale or self.default_scale
        v = self.const_int(c, c_scale)
        out = self.new_ct(a.n_poly, a.level, a.scale)
        so = self._structs([out])
        ws, wb = self.ws_for(nat.CKKS_OP_ELEMENTWISE, 1, [a.level])
        nat.ckks_multiply_scalar(self.h, self._structs([a]), [v], [c_scale], so, ws, wb, self.stream)
        return out.update(so[0])

    def add_scalar(self, a, c):
        v = self.const_int(c, a.scale)
        out = self.new_ct(a.n_poly, a.level, a.scale)
        so = self._structs([out])
        ws, wb = self.ws_for(nat.CKKS_OP_ELEMENTWISE, 1, [a.level])
        nat.ckks_add_scalar(self.h, self._structs([a]), [v], so, ws, wb, self.stream)
        return out.update(so[0])

    def _key_ptrs(self, keys, n, default):
        """per-item device key pointers: None = the context's key for all"""
        if keys is None:
            return default.data_ptr()
        keys = list(keys)
        if len(keys) != n:
            raise ValueError("need one key per item")
        return [k.data_ptr() for k in keys]

    def relinearize(self, a, rk=None):
        """rk: None (this context's key) or one relinearisation key per item"""
        single = isinstance(a, Ciphertext)
        A = [a] if single else list(a)
        outs = [self.new_ct(2, x.level, x.scale) for x in A]
        so = self._structs(outs)
        ws, wb = self.ws_for(nat.CKKS_OP_KEYSWITCH, len(A), [x.level for x in A])
        nat.ckks_relinearize(self.h, self._key_ptrs(rk, len(A), self.rk), self._structs(A), so, ws, wb, self.stream)
        self._outs(so, outs)
        return outs[0] if single else outs

    def rescale(self, a):
        single = isinstance(a, Ciphertext)
        A = [a] if single else list(a)
        outs = [self.new_ct(x.n_poly, x.level - 1, x.scale) for x in A]
        so = self._structs(outs)
        ws, wb = self.ws_for(nat.CKKS_OP_RESCALE, len(A), [x.level for x in A])
        nat.ckks_rescale(self.h, self._structs(A), so, ws, wb, self.stream)
        self._outs(so, outs)
        return outs[0] if single else outs

    def mod_switch(self, a, level):
        out = Ciphertext(self, a.buf, a.n_poly, a.level, a.scale)
        s = out.struct()
        nat.ckks_mod_switch_to(self.h, s, level)
        return out.update(s)

    def rotate(self, a, step=None, g=None, gk=None):
        """Left rotation of the slots by step (or Galois element g). With
        lists: g may be one element per item, and gk one key per item
        (several clients' keys in one launch); otherwise this context's key."""
        single = isinstance(a, Ciphertext)
        A = [a] if single else list(a)
        if g is None:
            g = [self.galois_elt(s) for s in step] if isinstance(step, (list, tuple)) else self.galois_elt(step)
        elts = list(g) if isinstance(g, (list, tuple)) else [g] * len(A)
        if gk is None:
            for e in set(elts):
                if e not in self.gk:
                    raise nat.CkksError(nat.CKKS_ENOKEY, "no Galois key for element %d" % e)
            keys = [self.gk[e].data_ptr() for e in elts]
        else:
            keys = [k.data_ptr() for k in gk]
        outs = [self.new_ct(2, x.level, x.scale) for x in A]
        so = self._structs(outs)
        ws, wb = self.ws_for(nat.CKKS_OP_KEYSWITCH, len(A), [x.level for x in A])
        nat.ckks_rotate(self.h, keys, elts, self._structs(A), so, ws, wb, self.stream)
        self._outs(so, outs)
        return outs[0] if single else outs

    def hmult_relin_rescale(self, A, Bs, outs=None, rk=None):
        """rk: None (this context's key) or one relinearisation key per item"""
        outs = outs or [self.new_ct(2, x.level - 1, x.scale) for x in A]
        so = self._structs(outs)
        ws, wb = self.ws_for(nat.CKKS_OP_HMULT, len(A), [x.level for x in A])
        nat.ckks_hmult_relin_rescale(self.h, self._key_ptrs(rk, len(A), self.rk), self._structs(A), self._structs(Bs),
                                     so, ws, wb, self.stream)
        return self._outs(so, outs)

    def linear(self, inputs, W, w_scale=None):
        """out[j] = sum_i round(W[j,i] * w_scale) * inputs[i]: dense rows through
        ckks_linear_csr (the matrix cores when the context enables them)"""
        w_scale = w_scale or self.default_scale
        W = np.asarray(W, dtype=np.float64)
        n_out, n_in = W.shape
        Wi = nat.ckks_encode_scalars(self.h, W, w_scale).reshape(-1)
        row_ptr = np.arange(n_out + 1, dtype=np.uint32) * n_in
        col = np.tile(np.arange(n_in, dtype=np.uint32), n_out)
        return self.linear_csr(inputs, row_ptr, col, Wi, w_scale)

    def linear_device_weights(self, inputs, W_int, w_scale):
        """the same product with the integer weights [n_out][n_in] already in
        device memory (ckks_linear, VALU)"""
        n_out, n_in = W_int.shape
        lvl = inputs[0].level
        outs = [self.new_ct(2, lvl, 1.0) for _ in range(n_out)]
        so = self._structs(outs)
        ws, wb = self.workspace(nat.ckks_workspace_bytes(self.h, nat.CKKS_OP_LINEAR, n_out, [lvl, n_in]))
        nat.ckks_linear(self.h, self._structs(inputs), W_int.data_ptr(), w_scale, so, ws, wb, self.stream)
        return self._outs(so, outs)

    # --- batched helpers used by the serving engine ---------------------------------
    def linear_csr(self, inputs, row_ptr, col, w_int, w_scale, outs=None):
        """rows over `inputs`: out[j] = sum_e w_int[e] * inputs[col[e]]"""
        lvl = inputs[0].level
        n_out = len(row_ptr) - 1
        outs = outs or [self.new_ct(2, lvl, 1.0) for _ in range(n_out)]
        so = self._structs(outs)
        nb = nat.ckks_linear_csr_workspace_bytes(self.h, len(inputs), n_out, int(row_ptr[-1]), lvl)
        ws, wb = self.workspace(nb)
        nat.ckks_linear_csr(self.h, self._structs(inputs), n_out, np.ascontiguousarray(row_ptr, dtype=np.uint32),
                            np.ascontiguousarray(col, dtype=np.uint32), np.ascontiguousarray(w_int, dtype=np.int64),
                            w_scale, so, ws, wb, self.stream)
        return self._outs(so, outs)

    def rescale_inplace(self, cts):
        s = self._structs(cts)
        ws, wb = self.ws_for(nat.CKKS_OP_RESCALE, len(cts), [c.level for c in cts])
        nat.ckks_rescale(self.h, s, s, ws, wb, self.stream)
        return self._outs(s, cts)

    def rescale_add_scalars_inplace(self, cts, values):
        """rescale, then cts[k] += values[k] at the scale after the rescale,
        in one pass (ckks_rescale_add_scalar)"""
        v = [self.const_int(x, c.scale / float(self.q[c.level])) for x, c in zip(values, cts)]
        s = self._structs(cts)
        ws, wb = self.ws_for(nat.CKKS_OP_RESCALE, len(cts), [c.level for c in cts])
        nat.ckks_rescale_add_scalar(self.h, s, v, s, ws, wb, self.stream)
        return self._outs(s, cts)

    def add_scalars_inplace(self, cts, values):
        """cts[k] += values[k] (floats, encoded at each ciphertext's scale)"""
        v = [self.const_int(x, c.scale) for x, c in zip(values, cts)]
        s = self._structs(cts)
        ws, wb = self.ws_for(nat.CKKS_OP_ELEMENTWISE, len(cts), [c.level for c in cts])
        nat.ckks_add_scalar(self.h, s, v, s, ws, wb, self.stream)
        return self._outs(s, cts)
