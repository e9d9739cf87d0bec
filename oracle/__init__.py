"""The oracle: a plain, slow, obviously correct CPU RNS-CKKS.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it. The product package
never imports, links or calls anything here, and nothing here imports the
product package: the two share no code. Seeded inputs come from the
separate ``synthetic`` module, which holds none of the method's arithmetic.

Layout:
  ckks_oracle.c  -- residue arithmetic, NTT, sampling, key switching,
                    rescale, encryption (plain C, 128-bit products, '%')
  encoding.py    -- canonical-embedding encode/decode in FP64 (numpy FFT
                    as the transform primitive) and the exact CRT lift
  plainnet.py    -- FP64 plaintext networks (packed-slot and unpacked)

Parity status per function is listed in the module headers; every function
here is pinned by a ``-m "not gpu"`` test in ``tests/test_oracle_*.py``.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_U64P = ctypes.POINTER(ctypes.c_uint64)
_I64P = ctypes.POINTER(ctypes.c_int64)
_U32P = ctypes.POINTER(ctypes.c_uint32)

_lib = None


def use_library(path):
    """Bind the oracle to another build of ckks_oracle.c (the benchmark's
    -O3 -march=native timing copy); call before creating any Oracle."""
    global _lib
    _lib = None
    return lib(path)


def lib(path=None):
    global _lib
    if _lib is None:
        if path is None:
            path = _build.LIB
            if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
                _build.build()
        L = ctypes.CDLL(path)
        u64, u32, i64, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, ctypes.c_void_p
        sig = {
            "orc_is_prime": (ctypes.c_int, [u64]),
            "orc_find_primes": (ctypes.c_int, [u32, _U32P, u32, _U64P]),
            "orc_min_psi": (u64, [u64, u32]),
            "orc_mulmod": (u64, [u64, u64, u64]),
            "orc_powmod": (u64, [u64, u64, u64]),
            "orc_ctx_create": (vp, [u32, _U64P, u32, u32, u32]),
            "orc_ctx_destroy": (None, [vp]),
            "orc_ctx_psi": (u64, [vp, u32]),
            "orc_digits": (u32, [vp, u32]),
            "orc_ntt": (None, [vp, u32, _U64P]),
            "orc_intt": (None, [vp, u32, _U64P]),
            "orc_philox4x32_10": (None, [_U32P, _U32P, _U32P]),
            "orc_sample_ternary": (None, [u64, u32, u32, u32, _I64P]),
            "orc_sample_cbd": (None, [u64, u32, u32, u32, _I64P]),
            "orc_sample_uniform": (None, [u64, u32, u32, u32, u32, u64, _U64P]),
            "orc_keygen_secret": (None, [vp, u64, _I64P, _U64P]),
            "orc_keygen_public": (None, [vp, _U64P, u64, _U64P]),
            "orc_keygen_switch": (None, [vp, _U64P, _U64P, u64, u32, _U64P]),
            "orc_keygen_relin": (None, [vp, _U64P, u64, _U64P]),
            "orc_keygen_galois": (None, [vp, _I64P, _U64P, u64, u64, _U64P]),
            "orc_automorph_ntt": (None, [vp, u32, u64, _U64P, _U64P]),
            "orc_encrypt": (None, [vp, _U64P, _U64P, u32, u64, u32, _U64P]),
            "orc_decrypt": (None, [vp, _U64P, _U64P, u32, u32, _U64P]),
            "orc_add": (None, [vp, _U64P, _U64P, u32, u32, _U64P]),
            "orc_sub": (None, [vp, _U64P, _U64P, u32, u32, _U64P]),
            "orc_add_plain": (None, [vp, _U64P, _U64P, u32, u32, _U64P]),
            "orc_mul_plain": (None, [vp, _U64P, _U64P, u32, u32, _U64P]),
            "orc_mul_const": (None, [vp, _U64P, i64, u32, u32, _U64P]),
            "orc_add_const": (None, [vp, _U64P, i64, u32, u32, _U64P]),
            "orc_tensor": (None, [vp, _U64P, _U64P, u32, _U64P]),
            "orc_rescale": (None, [vp, _U64P, u32, u32, _U64P]),
            "orc_mod_switch": (None, [vp, _U64P, u32, u32, u32, _U64P]),
            "orc_modup_digit": (None, [vp, _U64P, u32, u32, u32, _U64P]),
            "orc_moddown": (None, [vp, _U64P, u32, _U64P]),
            "orc_keyswitch": (None, [vp, _U64P, u32, _U64P, _U64P]),
            "orc_relinearize": (None, [vp, _U64P, u32, _U64P, _U64P]),
            "orc_apply_galois": (None, [vp, _U64P, u32, u64, _U64P, _U64P]),
            "orc_mul_relin_rescale": (None, [vp, _U64P, _U64P, u32, _U64P, _U64P]),
            "orc_lincomb": (None, [vp, ctypes.POINTER(_U64P), _I64P, u32, u32, u32, _U64P]),
            "orc_hoisted_linear": (None, [vp, _U64P, u32, u32, _U64P, ctypes.POINTER(_U64P), _I64P, _U64P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p64(a):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_U64P)


def _pi64(a):
    assert a.dtype == np.int64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_I64P)


def _u64(a):
    return np.ascontiguousarray(a, dtype=np.uint64)


# ---------------------------------------------------------------------------
# free functions
# ---------------------------------------------------------------------------
def is_prime(n: int) -> bool:
    return bool(lib().orc_is_prime(n))


def find_primes(logn: int, bits):
    """Prime choice: per requested bit size, in order, the largest unused
    prime below 2^bits that is 1 mod 2N."""
    b = (ctypes.c_uint32 * len(bits))(*bits)
    out = np.zeros(len(bits), dtype=np.uint64)
    rc = lib().orc_find_primes(logn, b, len(bits), _p64(out))
    if rc != 0:
        raise ValueError("no such primes")
    return [int(x) for x in out]


def min_psi(q: int, logn: int) -> int:
    return int(lib().orc_min_psi(q, logn))


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def sample_ternary(seed, obj, tag, n):
    out = np.zeros(n, dtype=np.int64)
    lib().orc_sample_ternary(seed, obj, tag, n, _pi64(out))
    return out


def sample_cbd(seed, obj, tag, n):
    out = np.zeros(n, dtype=np.int64)
    lib().orc_sample_cbd(seed, obj, tag, n, _pi64(out))
    return out


def sample_uniform(seed, obj, tag, limb, n, q):
    out = np.zeros(n, dtype=np.uint64)
    lib().orc_sample_uniform(seed, obj, tag, limb, n, q, _p64(out))
    return out


TAG_SK, TAG_PK_A, TAG_PK_E, TAG_SWK_A, TAG_SWK_E, TAG_ENC_V, TAG_ENC_E0, TAG_ENC_E1 = range(1, 9)


class Oracle:
    """Parameters plus the per-prime constants of the plain C oracle.

    ``q``: data primes q_0..q_L (q_0 the base prime that holds the final
    result); ``p``: key-switching special primes; ``dnum``: digits at the
    top level, alpha = ceil((L+1)/dnum) primes per digit (hybrid key switching).
    All arrays are numpy uint64 in [0, q), polys in NTT form unless a
    method says otherwise, layout [poly][limb][N].
    """

    def __init__(self, logn, q, p, dnum):
        self.logn = logn
        self.N = 1 << logn
        self.q = [int(x) for x in q]
        self.p = [int(x) for x in p]
        self.primes = self.q + self.p
        self.n_q, self.n_p, self.dnum = len(self.q), len(self.p), dnum
        self.alpha = -(-self.n_q // dnum)
        arr = _u64(self.primes)
        self._h = lib().orc_ctx_create(logn, _p64(arr), self.n_q, self.n_p, dnum)
        if not self._h:
            raise ValueError("bad oracle parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_ctx_destroy(h)
            self._h = None

    # -- transforms ---------------------------------------------------------
    def psi(self, i):
        return int(lib().orc_ctx_psi(self._h, i))

    def ntt(self, a, prime_idx):
        a = _u64(a).copy()
        lib().orc_ntt(self._h, prime_idx, _p64(a))
        return a

    def intt(self, a, prime_idx):
        a = _u64(a).copy()
        lib().orc_intt(self._h, prime_idx, _p64(a))
        return a

    def digits(self, level):
        return int(lib().orc_digits(self._h, level))

    # -- integer plaintexts -------------------------------------------------
    def reduce_int(self, coeffs, level, ntt=True):
        """Signed integer polynomial (int64 or Python ints) -> [l+1][N]
        residues (NTT form when ntt=True)."""
        out = np.zeros((level + 1, self.N), dtype=np.uint64)
        co = [int(x) for x in coeffs]
        for i in range(level + 1):
            qi = self.q[i]
            out[i] = np.array([c % qi for c in co], dtype=np.uint64)
            if ntt:
                out[i] = self.ntt(out[i], i)
        return out

    # -- keys ---------------------------------------------------------------
    def keygen_secret(self, seed):
        s = np.zeros(self.N, dtype=np.int64)
        sn = np.zeros((self.n_q + self.n_p, self.N), dtype=np.uint64)
        lib().orc_keygen_secret(self._h, seed, _pi64(s), _p64(sn))
        return s, sn

    def keygen_public(self, sk_ntt, seed):
        pk = np.zeros((2, self.n_q, self.N), dtype=np.uint64)
        lib().orc_keygen_public(self._h, _p64(_u64(sk_ntt)), seed, _p64(pk))
        return pk

    def key_shape(self):
        return (self.digits(self.n_q - 1), 2, self.n_q + self.n_p, self.N)

    def keygen_relin(self, sk_ntt, seed):
        rk = np.zeros(self.key_shape(), dtype=np.uint64)
        lib().orc_keygen_relin(self._h, _p64(_u64(sk_ntt)), seed, _p64(rk))
        return rk

    def keygen_galois(self, sk_coeff, sk_ntt, g, seed):
        gk = np.zeros(self.key_shape(), dtype=np.uint64)
        lib().orc_keygen_galois(self._h, _pi64(np.ascontiguousarray(sk_coeff, dtype=np.int64)),
                                _p64(_u64(sk_ntt)), g, seed, _p64(gk))
        return gk

    def keygen_switch(self, sk_ntt, sprime_ntt, seed, key_id):
        k = np.zeros(self.key_shape(), dtype=np.uint64)
        lib().orc_keygen_switch(self._h, _p64(_u64(sk_ntt)), _p64(_u64(sprime_ntt)), seed, key_id,
                                _p64(k))
        return k

    # -- encryption ---------------------------------------------------------
    def encrypt(self, pk, pt_ntt, level, seed, obj):
        ct = np.zeros((2, level + 1, self.N), dtype=np.uint64)
        lib().orc_encrypt(self._h, _p64(_u64(pk)), _p64(_u64(pt_ntt)), level, seed, obj, _p64(ct))
        return ct

    def decrypt(self, sk_ntt, ct):
        ct = _u64(ct)
        n_poly, L = ct.shape[0], ct.shape[1]
        m = np.zeros((L, self.N), dtype=np.uint64)
        lib().orc_decrypt(self._h, _p64(_u64(sk_ntt)), _p64(ct), n_poly, L - 1, _p64(m))
        return m

    # -- evaluation ---------------------------------------------------------
    def _binop(self, fn, a, b):
        a, b = _u64(a), _u64(b)
        out = np.zeros_like(a)
        fn(self._h, _p64(a), _p64(b), a.shape[0], a.shape[1] - 1, _p64(out))
        return out

    def add(self, a, b):
        return self._binop(lib().orc_add, a, b)

    def sub(self, a, b):
        return self._binop(lib().orc_sub, a, b)

    def add_plain(self, a, pt):
        return self._binop(lib().orc_add_plain, a, pt)

    def mul_plain(self, a, pt):
        return self._binop(lib().orc_mul_plain, a, pt)

    def mul_const(self, a, v):
        a = _u64(a)
        out = np.zeros_like(a)
        lib().orc_mul_const(self._h, _p64(a), int(v), a.shape[0], a.shape[1] - 1, _p64(out))
        return out

    def add_const(self, a, v):
        a = _u64(a)
        out = np.zeros_like(a)
        lib().orc_add_const(self._h, _p64(a), int(v), a.shape[0], a.shape[1] - 1, _p64(out))
        return out

    def tensor(self, a, b):
        a, b = _u64(a), _u64(b)
        L = a.shape[1]
        out = np.zeros((3, L, self.N), dtype=np.uint64)
        lib().orc_tensor(self._h, _p64(a), _p64(b), L - 1, _p64(out))
        return out

    def rescale(self, a):
        a = _u64(a)
        n_poly, L = a.shape[0], a.shape[1]
        out = np.zeros((n_poly, L - 1, self.N), dtype=np.uint64)
        lib().orc_rescale(self._h, _p64(a), n_poly, L - 1, _p64(out))
        return out

    def mod_switch(self, a, to_level):
        a = _u64(a)
        return a[:, : to_level + 1].copy()

    def modup_digit(self, x_coeff, lo, hi, target_prime):
        x = _u64(x_coeff)
        out = np.zeros(self.N, dtype=np.uint64)
        lib().orc_modup_digit(self._h, _p64(x), lo, hi, target_prime, _p64(out))
        return out

    def moddown(self, a, level):
        a = _u64(a)
        out = np.zeros((level + 1, self.N), dtype=np.uint64)
        lib().orc_moddown(self._h, _p64(a), level, _p64(out))
        return out

    def keyswitch(self, d, swk):
        d = _u64(d)
        L = d.shape[0]
        ks = np.zeros((2, L, self.N), dtype=np.uint64)
        lib().orc_keyswitch(self._h, _p64(d), L - 1, _p64(_u64(swk)), _p64(ks))
        return ks

    def relinearize(self, ct3, rk):
        ct3 = _u64(ct3)
        L = ct3.shape[1]
        out = np.zeros((2, L, self.N), dtype=np.uint64)
        lib().orc_relinearize(self._h, _p64(ct3), L - 1, _p64(_u64(rk)), _p64(out))
        return out

    def galois_elt(self, step):
        """Left rotation by r uses g = 5^(r mod N/2) mod 2N (slot j <-> zeta^(5^j))."""
        two_n = 2 * self.N
        return pow(5, step % (self.N // 2), two_n)

    def apply_galois(self, ct, g, gk):
        ct = _u64(ct)
        L = ct.shape[1]
        out = np.zeros((2, L, self.N), dtype=np.uint64)
        lib().orc_apply_galois(self._h, _p64(ct), L - 1, g, _p64(_u64(gk)), _p64(out))
        return out

    def automorph_ntt(self, a, prime_idx, g):
        a = _u64(a)
        out = np.zeros_like(a)
        lib().orc_automorph_ntt(self._h, prime_idx, g, _p64(a), _p64(out))
        return out

    def lincomb(self, cts, weights):
        """sum_k weights[k] * cts[k] (integer weights, one level)"""
        cts = [_u64(c) for c in cts]
        arr = (_U64P * len(cts))(*[_p64(c) for c in cts])
        w = np.ascontiguousarray(weights, dtype=np.int64)
        out = np.zeros_like(cts[0])
        lib().orc_lincomb(self._h, arr, _pi64(w), len(cts), cts[0].shape[0], cts[0].shape[1] - 1, _p64(out))
        return out

    def hoisted_linear(self, ct, galois, gks, pt_coeffs):
        """sum_i pt_i (x) rot_{g_i}(ct) with one shared decomposition and one
        ModDown; g = 1 is the identity (its key entry is ignored)"""
        ct = _u64(ct)
        L = ct.shape[1]
        g = np.ascontiguousarray(galois, dtype=np.uint64)
        keys = [_u64(k) if k is not None else np.zeros(1, dtype=np.uint64) for k in gks]
        arr = (_U64P * len(keys))(*[_p64(k) for k in keys])
        pc = np.ascontiguousarray(pt_coeffs, dtype=np.int64)
        out = np.zeros((2, L, self.N), dtype=np.uint64)
        lib().orc_hoisted_linear(self._h, _p64(ct), L - 1, len(g), _p64(g), arr, _pi64(pc), _p64(out))
        return out

    def mul_relin_rescale(self, a, b, rk):
        a, b = _u64(a), _u64(b)
        L = a.shape[1]
        out = np.zeros((2, L - 1, self.N), dtype=np.uint64)
        lib().orc_mul_relin_rescale(self._h, _p64(a), _p64(b), L - 1, _p64(_u64(rk)), _p64(out))
        return out
