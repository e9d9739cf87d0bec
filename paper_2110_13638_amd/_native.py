"""ctypes binding of libckks_hip.so: the C ABI declared in include/ckks.h.

Argument marshalling only: every function here has the name of the C entry
point it calls and does no arithmetic. Loading fails loudly when the HIP
library has not been built: there is no fallback path.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libckks_hip.so")

CKKS_OK = 0
CKKS_EINVAL, CKKS_ELEVEL, CKKS_ESCALE, CKKS_EDEPTH = -1, -2, -3, -4
CKKS_ENOKEY, CKKS_EPARAMS, CKKS_ENOMEM, CKKS_EDEVICE = -5, -6, -7, -8
ERROR_NAMES = {-1: "EINVAL", -2: "ELEVEL", -3: "ESCALE", -4: "EDEPTH", -5: "ENOKEY", -6: "EPARAMS",
               -7: "ENOMEM", -8: "EDEVICE"}

CKKS_KEY_SECRET, CKKS_KEY_PUBLIC, CKKS_KEY_SWITCH = 0, 1, 2
(CKKS_OP_NTT, CKKS_OP_ELEMENTWISE, CKKS_OP_KEYSWITCH, CKKS_OP_RESCALE, CKKS_OP_HMULT, CKKS_OP_KEYGEN,
 CKKS_OP_ENCRYPT, CKKS_OP_LINEAR) = range(8)
CKKS_OBJ_CT, CKKS_OBJ_PT, CKKS_OBJ_KEY = 0, 1, 2
CKKS_TUNE_NTT_WIDE, CKKS_TUNE_EW_LOG, CKKS_TUNE_XCD_REMAP, CKKS_TUNE_FUSE_TAIL, CKKS_TUNE_IP_CTS = 0, 1, 2, 3, 4
CKKS_TUNE_LIN_MFMA = 5
CKKS_TUNE_NTT_FP = 6
CKKS_NOALLOC_SCRATCH_BYTES = 80 << 20


class CkksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERROR_NAMES.get(code, "?"), code, msg))
        self.code = code


class ckks_params(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("n_q", ctypes.c_uint32), ("q", ctypes.POINTER(ctypes.c_uint64)),
                ("n_p", ctypes.c_uint32), ("p", ctypes.POINTER(ctypes.c_uint64)), ("dnum", ctypes.c_uint32)]


class ckks_ct(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("n_poly", ctypes.c_uint32), ("level", ctypes.c_uint32),
                ("limb_stride", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("scale", ctypes.c_double)]


class ckks_pt(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("level", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("scale", ctypes.c_double)]


class ckks_launch_record(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 56), ("items", ctypes.c_uint32), ("ms", ctypes.c_float)]


class ckks_input_attrs(ctypes.Structure):
    _fields_ = [("n_ct", ctypes.c_uint32), ("level", ctypes.c_uint32), ("scale", ctypes.c_double)]


class ckks_linear_attrs(ctypes.Structure):
    _fields_ = [("n_out", ctypes.c_uint32), ("row_ptr", ctypes.POINTER(ctypes.c_uint32)),
                ("col", ctypes.POINTER(ctypes.c_uint32)), ("w", ctypes.POINTER(ctypes.c_double)),
                ("w_scale", ctypes.c_double), ("bias", ctypes.POINTER(ctypes.c_double))]


class ckks_diag_attrs(ctypes.Structure):
    _fields_ = [("n_diag", ctypes.c_uint32), ("in_steps", ctypes.POINTER(ctypes.c_int32)),
                ("diag_coeffs", ctypes.POINTER(ctypes.c_int64)), ("pt_scale", ctypes.c_double),
                ("n_post", ctypes.c_uint32), ("post_steps", ctypes.POINTER(ctypes.c_int32)),
                ("bias_slots", ctypes.POINTER(ctypes.c_double)), ("n_bias_slots", ctypes.c_uint32),
                ("bias_coeffs", ctypes.POINTER(ctypes.c_int64)), ("hoisted", ctypes.c_uint32)]


CKKS_NODE_INPUT, CKKS_NODE_LINEAR, CKKS_NODE_DIAG_DENSE, CKKS_NODE_SQUARE, CKKS_NODE_OUTPUT, CKKS_NODE_POLY = range(6)


class ckks_poly_attrs(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_uint32), ("coeffs", ctypes.POINTER(ctypes.c_double)),
                ("w_scale", ctypes.c_double)]

_u32, _u64, _i32, _sz, _vp, _dbl = (ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_size_t,
                                    ctypes.c_void_p, ctypes.c_double)
_P = ctypes.POINTER
_SIGS = {
    "ckks_last_error": (ctypes.c_char_p, []),
    "ckks_find_primes": (ctypes.c_int, [_u32, _P(_u32), _u32, _P(_u64)]),
    "ckks_parameterise": (ctypes.c_int, [_u32, _u32, _dbl, _P(_u32), _u32, _P(_u32), _P(_u32)]),
    "ckks_ctx_create": (ctypes.c_int, [_P(ckks_params), _P(_vp)]),
    "ckks_ctx_destroy": (None, [_vp]),
    "ckks_ctx_device_bytes": (_sz, [_vp]),
    "ckks_ctx_upload": (ctypes.c_int, [_vp, _vp, _vp]),
    "ckks_ctx_log_n": (_u32, [_vp]),
    "ckks_ctx_max_level": (_u32, [_vp]),
    "ckks_ctx_digits": (_u32, [_vp, _u32]),
    "ckks_ctx_prime": (_u64, [_vp, _u32]),
    "ckks_ct_bytes": (_sz, [_vp, _u32, _u32]),
    "ckks_pt_bytes": (_sz, [_vp, _u32]),
    "ckks_key_bytes": (_sz, [_vp, ctypes.c_int]),
    "ckks_workspace_bytes": (_sz, [_vp, ctypes.c_int, _u32, _P(_u32)]),
    "ckks_ntt": (ctypes.c_int, [_vp, _P(_vp), _P(_u32), _u32, _vp, _sz, _vp]),
    "ckks_intt": (ctypes.c_int, [_vp, _P(_vp), _P(_u32), _u32, _vp, _sz, _vp]),
    "ckks_keygen_secret": (ctypes.c_int, [_vp, _u64, _vp, _vp, _sz, _vp]),
    "ckks_keygen_public": (ctypes.c_int, [_vp, _vp, _u64, _vp, _vp, _sz, _vp]),
    "ckks_keygen_relin": (ctypes.c_int, [_vp, _vp, _u64, _vp, _vp, _sz, _vp]),
    "ckks_keygen_galois": (ctypes.c_int, [_vp, _vp, _u32, _u64, _vp, _vp, _sz, _vp]),
    "ckks_galois_elt": (_u32, [_vp, _i32]),
    "ckks_encode": (ctypes.c_int, [_vp, _P(_dbl), _P(_dbl), _sz, _dbl, _P(ctypes.c_int64)]),
    "ckks_decode": (ctypes.c_int, [_vp, _P(_u64), _u32, _dbl, _P(_dbl), _P(_dbl), _sz]),
    "ckks_pt_load": (ctypes.c_int, [_vp, _vp, _P(ckks_pt), _vp, _sz, _vp]),
    "ckks_encrypt": (ctypes.c_int, [_vp, _vp, _P(ckks_pt), _u64, _u32, _P(ckks_ct), _vp, _sz, _vp]),
    "ckks_decrypt": (ctypes.c_int, [_vp, _vp, _P(ckks_ct), _vp, _vp, _sz, _vp]),
    "ckks_add": (ctypes.c_int, [_vp, _P(ckks_ct), _P(ckks_ct), _P(ckks_ct), _u32, _vp, _sz, _vp]),
    "ckks_sub": (ctypes.c_int, [_vp, _P(ckks_ct), _P(ckks_ct), _P(ckks_ct), _u32, _vp, _sz, _vp]),
    "ckks_add_plain": (ctypes.c_int, [_vp, _P(ckks_ct), _P(ckks_pt), _P(ckks_ct), _u32, _vp, _sz, _vp]),
    "ckks_multiply_plain": (ctypes.c_int, [_vp, _P(ckks_ct), _P(ckks_pt), _P(ckks_ct), _u32, _vp, _sz, _vp]),
    "ckks_multiply_scalar": (ctypes.c_int, [_vp, _P(ckks_ct), _P(ctypes.c_int64), _P(_dbl), _P(ckks_ct), _u32,
                                            _vp, _sz, _vp]),
    "ckks_add_scalar": (ctypes.c_int, [_vp, _P(ckks_ct), _P(ctypes.c_int64), _P(ckks_ct), _u32, _vp, _sz, _vp]),
    "ckks_multiply": (ctypes.c_int, [_vp, _P(ckks_ct), _P(ckks_ct), _P(ckks_ct), _u32, _vp, _sz, _vp]),
    "ckks_relinearize": (ctypes.c_int, [_vp, _P(_vp), _P(ckks_ct), _P(ckks_ct), _u32, _vp, _sz, _vp]),
    "ckks_rescale": (ctypes.c_int, [_vp, _P(ckks_ct), _P(ckks_ct), _u32, _vp, _sz, _vp]),
    "ckks_rescale_add_scalar": (ctypes.c_int, [_vp, _P(ckks_ct), _P(ctypes.c_int64), _P(ckks_ct), _u32, _vp, _sz,
                                               _vp]),
    "ckks_mod_switch_to": (ctypes.c_int, [_vp, _P(ckks_ct), _u32]),
    "ckks_rotate": (ctypes.c_int, [_vp, _P(_vp), _P(_u32), _P(ckks_ct), _P(ckks_ct), _u32, _vp, _sz, _vp]),
    "ckks_hmult_relin_rescale": (ctypes.c_int, [_vp, _P(_vp), _P(ckks_ct), _P(ckks_ct), _P(ckks_ct), _u32, _vp,
                                                _sz, _vp]),
    "ckks_hmult_relin_rescale_noalloc": (ctypes.c_int, [_vp, _P(_vp), _P(ckks_ct), _P(ckks_ct), _P(ckks_ct), _u32,
                                                        _vp]),
    "ckks_encode_scalars": (ctypes.c_int, [_vp, _P(_dbl), _sz, _dbl, _P(ctypes.c_int64)]),
    "ckks_encode_scalar": (ctypes.c_int, [_vp, _dbl, _dbl, _u32, _P(_u64)]),
    "ckks_linear": (ctypes.c_int, [_vp, _P(ckks_ct), _u32, _vp, _dbl, _P(ckks_ct), _u32, _vp, _sz, _vp]),
    "ckks_linear_csr_workspace_bytes": (_sz, [_vp, _u32, _u32, _sz, _u32]),
    "ckks_hoisted_linear_workspace_bytes": (_sz, [_vp, _u32, _u32, _u32]),
    "ckks_hoisted_linear": (ctypes.c_int, [_vp, _P(ckks_ct), _P(ckks_ct), _u32, _u32, _P(_u32), _P(_vp), _vp, _dbl,
                                          _vp, _sz, _vp]),
    "ckks_linear_csr": (ctypes.c_int, [_vp, _P(ckks_ct), _u32, _u32, _P(_u32), _P(_u32), _P(ctypes.c_int64), _dbl,
                                       _P(ckks_ct), _vp, _sz, _vp]),
    "ckks_graph_create": (ctypes.c_int, [_vp, _P(_vp)]),
    "ckks_graph_destroy": (None, [_vp]),
    "ckks_graph_add_node": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _P(_u32)]),
    "ckks_graph_add_edge": (ctypes.c_int, [_vp, _u32, _u32]),
    "ckks_graph_plan": (ctypes.c_int, [_vp, _P(_sz), _P(_u32)]),
    "ckks_graph_run": (ctypes.c_int, [_vp, _P(ckks_ct), _u32, _P(ckks_ct), _u32, _vp, _P(_u32), _P(_vp), _u32,
                                      _vp, _sz, _vp]),
    "ckks_graph_autohe": (ctypes.c_int, [_vp, _P(_u32), _P(_u32), _P(_u32), _u32]),
    "ckks_serialize": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int, _vp, _P(_sz), _vp]),
    "ckks_deserialize": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _sz, _vp, ctypes.c_int, _vp]),
    "ckks_record_begin": (ctypes.c_int, [_vp, _vp, _sz]),
    "ckks_record_end": (ctypes.c_int, [_vp, _P(_vp), _P(_sz)]),
    "ckks_plan_launch": (ctypes.c_int, [_vp, _vp]),
    "ckks_plan_launch_count": (_u32, [_vp]),
    "ckks_plan_destroy": (None, [_vp]),
    "ckks_ctx_set_tuning": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
    "ckks_ctx_get_tuning": (ctypes.c_int, [_vp, ctypes.c_int]),
    "ckks_profile_enable": (ctypes.c_int, [ctypes.c_int]),
    "ckks_profile_collect": (ctypes.c_int, [_P(ckks_launch_record), _u32, _P(_u32)]),
}

_lib = None


def lib():
    """The loaded library; raises when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libckks_hip.so is not built (run paper_2110_13638_amd/build.py); "
                              "there is no fallback implementation")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return sorted(_SIGS)


def check(rc):
    if rc != CKKS_OK:
        raise CkksError(rc, lib().ckks_last_error().decode())
    return rc


def _call(name, *args):
    return check(getattr(lib(), name)(*args))


# one wrapper per entry point, same names as the C ABI ------------------------
def ckks_last_error():
    return lib().ckks_last_error().decode()


def ckks_find_primes(log_n, bits):
    b = (ctypes.c_uint32 * len(bits))(*bits)
    out = (ctypes.c_uint64 * len(bits))()
    _call("ckks_find_primes", log_n, b, len(bits), out)
    return [int(x) for x in out]


def ckks_parameterise(cost, scale_bits=40, special_mult=1.5):
    cap = cost + 2
    bits = (ctypes.c_uint32 * cap)()
    nb, ln = ctypes.c_uint32(), ctypes.c_uint32()
    _call("ckks_parameterise", cost, scale_bits, special_mult, bits, cap, ctypes.byref(nb), ctypes.byref(ln))
    return [int(bits[i]) for i in range(nb.value)], 1 << ln.value


def ckks_ctx_create(log_n, q, p, dnum):
    qa = (ctypes.c_uint64 * len(q))(*q)
    pa = (ctypes.c_uint64 * len(p))(*p)
    prm = ckks_params(log_n, len(q), qa, len(p), pa, dnum)
    h = ctypes.c_void_p()
    _call("ckks_ctx_create", ctypes.byref(prm), ctypes.byref(h))
    return h


def ckks_ctx_destroy(h):
    lib().ckks_ctx_destroy(h)


def ckks_ctx_device_bytes(h):
    return int(lib().ckks_ctx_device_bytes(h))


def ckks_ctx_upload(h, dev_ptr, stream=None):
    _call("ckks_ctx_upload", h, dev_ptr, stream)


def ckks_ctx_digits(h, level):
    return int(lib().ckks_ctx_digits(h, level))


def ckks_ctx_prime(h, i):
    return int(lib().ckks_ctx_prime(h, i))


def ckks_ct_bytes(h, n_poly, level):
    return int(lib().ckks_ct_bytes(h, n_poly, level))


def ckks_key_bytes(h, kind):
    return int(lib().ckks_key_bytes(h, kind))


def ckks_workspace_bytes(h, op, B, levels=None):
    lv = (ctypes.c_uint32 * len(levels))(*levels) if levels is not None else None
    return int(lib().ckks_workspace_bytes(h, op, B, lv))


def _ptr_arrays(limb_ptrs, prime_idx):
    n = len(limb_ptrs)
    return (ctypes.c_void_p * n)(*limb_ptrs), (ctypes.c_uint32 * n)(*prime_idx), n


def ckks_ntt(h, limb_ptrs, prime_idx, ws, ws_bytes, stream=None):
    lp, pi, n = _ptr_arrays(limb_ptrs, prime_idx)
    _call("ckks_ntt", h, lp, pi, n, ws, ws_bytes, stream)


def ckks_intt(h, limb_ptrs, prime_idx, ws, ws_bytes, stream=None):
    lp, pi, n = _ptr_arrays(limb_ptrs, prime_idx)
    _call("ckks_intt", h, lp, pi, n, ws, ws_bytes, stream)


def ckks_keygen_secret(h, seed, sk, ws, ws_bytes, stream=None):
    _call("ckks_keygen_secret", h, seed, sk, ws, ws_bytes, stream)


def ckks_keygen_public(h, sk, seed, pk, ws, ws_bytes, stream=None):
    _call("ckks_keygen_public", h, sk, seed, pk, ws, ws_bytes, stream)


def ckks_keygen_relin(h, sk, seed, rk, ws, ws_bytes, stream=None):
    _call("ckks_keygen_relin", h, sk, seed, rk, ws, ws_bytes, stream)


def ckks_keygen_galois(h, sk, galois_elt, seed, gk, ws, ws_bytes, stream=None):
    _call("ckks_keygen_galois", h, sk, galois_elt, seed, gk, ws, ws_bytes, stream)


def ckks_galois_elt(h, step):
    return int(lib().ckks_galois_elt(h, step))


def ckks_encode(h, re, im, n, scale, coeffs_out):
    """re/im: pointers to n doubles (im may be None); coeffs_out: int64[N]"""
    _call("ckks_encode", h, re, im, n, scale, coeffs_out)


def ckks_decode(h, residues, level, scale, re_out, im_out):
    _call("ckks_decode", h, residues, level, scale, re_out, im_out, len(re_out))


def ckks_pt_load(h, coeffs_dev, pt, ws, ws_bytes, stream=None):
    _call("ckks_pt_load", h, coeffs_dev, ctypes.byref(pt), ws, ws_bytes, stream)


def ckks_encrypt(h, pk, pt, seed, obj, ct, ws, ws_bytes, stream=None):
    _call("ckks_encrypt", h, pk, ctypes.byref(pt), seed, obj, ctypes.byref(ct), ws, ws_bytes, stream)


def ckks_decrypt(h, sk, ct, m_dev, ws, ws_bytes, stream=None):
    _call("ckks_decrypt", h, sk, ctypes.byref(ct), m_dev, ws, ws_bytes, stream)


def _arr(T, xs):
    return (T * len(xs))(*xs)


def ckks_add(h, a, b, out, ws, ws_bytes, stream=None):
    _call("ckks_add", h, a, b, out, len(out), ws, ws_bytes, stream)


def ckks_sub(h, a, b, out, ws, ws_bytes, stream=None):
    _call("ckks_sub", h, a, b, out, len(out), ws, ws_bytes, stream)


def ckks_add_plain(h, a, p, out, ws, ws_bytes, stream=None):
    _call("ckks_add_plain", h, a, p, out, len(out), ws, ws_bytes, stream)


def ckks_multiply_plain(h, a, p, out, ws, ws_bytes, stream=None):
    _call("ckks_multiply_plain", h, a, p, out, len(out), ws, ws_bytes, stream)


def ckks_multiply_scalar(h, a, v, v_scale, out, ws, ws_bytes, stream=None):
    _call("ckks_multiply_scalar", h, a, _arr(ctypes.c_int64, v), _arr(ctypes.c_double, v_scale), out, len(out),
          ws, ws_bytes, stream)


def ckks_add_scalar(h, a, v, out, ws, ws_bytes, stream=None):
    _call("ckks_add_scalar", h, a, _arr(ctypes.c_int64, v), out, len(out), ws, ws_bytes, stream)


def ckks_multiply(h, a, b, out3, ws, ws_bytes, stream=None):
    _call("ckks_multiply", h, a, b, out3, len(out3), ws, ws_bytes, stream)


def _per_item(x, n):
    """one value for every item, or a sequence of n"""
    if isinstance(x, (list, tuple, np.ndarray)):
        if len(x) != n:
            raise ValueError("expected %d per-item values, got %d" % (n, len(x)))
        return [int(v) for v in x]
    return [int(x)] * n


def ckks_relinearize(h, rk, in3, out, ws, ws_bytes, stream=None):
    """rk: one key pointer for every item, or one per item"""
    _call("ckks_relinearize", h, _arr(_vp, _per_item(rk, len(out))), in3, out, len(out), ws, ws_bytes, stream)


def ckks_rescale(h, a, out, ws, ws_bytes, stream=None):
    _call("ckks_rescale", h, a, out, len(out), ws, ws_bytes, stream)


def ckks_rescale_add_scalar(h, a, v, out, ws, ws_bytes, stream=None):
    """rescale, then v[b] (integers at the output scale) added to every slot of out[b]'s first poly"""
    _call("ckks_rescale_add_scalar", h, a, _arr(ctypes.c_int64, v), out, len(out), ws, ws_bytes, stream)


def ckks_mod_switch_to(h, ct, level):
    _call("ckks_mod_switch_to", h, ctypes.byref(ct), level)


def ckks_rotate(h, gk, galois_elt, a, out, ws, ws_bytes, stream=None):
    """gk, galois_elt: one key pointer / element for every item, or one per item"""
    n = len(out)
    _call("ckks_rotate", h, _arr(_vp, _per_item(gk, n)), _arr(_u32, _per_item(galois_elt, n)), a, out, n, ws,
          ws_bytes, stream)


def ckks_hmult_relin_rescale(h, rk, a, b, out, ws, ws_bytes, stream=None):
    """rk: one relinearisation key pointer for every item, or one per item"""
    _call("ckks_hmult_relin_rescale", h, _arr(_vp, _per_item(rk, len(out))), a, b, out, len(out), ws, ws_bytes,
          stream)


def ckks_hmult_relin_rescale_noalloc(h, rk, a, b, out, stream=None):
    """The same call with the library's fixed scratch array instead of a workspace"""
    _call("ckks_hmult_relin_rescale_noalloc", h, _arr(_vp, _per_item(rk, len(out))), a, b, out, len(out), stream)


def ckks_encode_scalars(h, values, scale):
    """round_half_away(values[k] * scale) as an int64 array (computed in C)"""
    v = np.ascontiguousarray(values, dtype=np.float64).reshape(-1)
    out = np.zeros(v.size, dtype=np.int64)
    _call("ckks_encode_scalars", h, v.ctypes.data_as(_P(_dbl)), v.size, float(scale),
          out.ctypes.data_as(_P(ctypes.c_int64)))
    return out


def ckks_encode_scalar(h, value, scale, level):
    """per-limb residues of the constant polynomial round_half_away(value * scale)"""
    out = np.zeros(level + 1, dtype=np.uint64)
    _call("ckks_encode_scalar", h, float(value), float(scale), level, out.ctypes.data_as(_P(_u64)))
    return out


def ckks_linear(h, inp, W_dev, w_scale, out, ws, ws_bytes, stream=None):
    _call("ckks_linear", h, inp, len(inp), W_dev, w_scale, out, len(out), ws, ws_bytes, stream)


def ckks_linear_csr_workspace_bytes(h, n_in, n_out, nnz, level):
    return int(lib().ckks_linear_csr_workspace_bytes(h, n_in, n_out, nnz, level))


def ckks_hoisted_linear_workspace_bytes(h, B, level, n_rot):
    return lib().ckks_hoisted_linear_workspace_bytes(h, B, level, n_rot)


def ckks_hoisted_linear(h, inp, out, galois_elts, galois_keys, pt_coeffs_dev, pt_scale, ws, ws_bytes, stream=None):
    n = len(galois_elts)
    _call("ckks_hoisted_linear", h, inp, out, len(inp), n, _arr(_u32, galois_elts), _arr(_vp, galois_keys),
          pt_coeffs_dev, pt_scale, ws, ws_bytes, stream)


def ckks_linear_csr(h, inp, n_out, row_ptr, col, w, w_scale, out, ws, ws_bytes, stream=None):
    """row_ptr/col: uint32 numpy arrays, w: int64 numpy array (host)"""
    _call("ckks_linear_csr", h, inp, len(inp), n_out, row_ptr.ctypes.data_as(_P(_u32)),
          col.ctypes.data_as(_P(_u32)), w.ctypes.data_as(_P(ctypes.c_int64)), w_scale, out, ws, ws_bytes, stream)


def ckks_serialize(h, obj_kind, obj, key_kind=0, stream=None):
    """bytes of a ciphertext / plaintext (ctypes struct, passed by reference)
    or key (device pointer)"""
    ref = ctypes.byref(obj) if obj_kind != CKKS_OBJ_KEY else obj
    n = _sz()
    _call("ckks_serialize", h, obj_kind, ref, key_kind, None, ctypes.byref(n), stream)
    buf = ctypes.create_string_buffer(n.value)
    _call("ckks_serialize", h, obj_kind, ref, key_kind, buf, ctypes.byref(n), stream)
    return buf.raw[: n.value]


def ckks_deserialize(h, obj_kind, data, obj, key_kind=0, stream=None):
    ref = ctypes.byref(obj) if obj_kind != CKKS_OBJ_KEY else obj
    _call("ckks_deserialize", h, obj_kind, data, len(data), ref, key_kind, stream)
    return obj


def ckks_record_begin(h, arena, arena_bytes):
    _call("ckks_record_begin", h, arena, arena_bytes)


def ckks_record_end(h):
    plan, used = _vp(), _sz()
    _call("ckks_record_end", h, ctypes.byref(plan), ctypes.byref(used))
    return plan, used.value


def ckks_plan_launch(plan, stream=None):
    _call("ckks_plan_launch", plan, stream)


def ckks_plan_launch_count(plan):
    return lib().ckks_plan_launch_count(plan)


def ckks_plan_destroy(plan):
    lib().ckks_plan_destroy(plan)


def ckks_ctx_set_tuning(h, knob, value):
    _call("ckks_ctx_set_tuning", h, knob, value)


def ckks_ctx_get_tuning(h, knob):
    return lib().ckks_ctx_get_tuning(h, knob)


def ckks_profile_enable(on):
    _call("ckks_profile_enable", 1 if on else 0)


def ckks_profile_collect(cap=1 << 16):
    recs = (ckks_launch_record * cap)()
    n = ctypes.c_uint32()
    _call("ckks_profile_collect", recs, cap, ctypes.byref(n))
    return [(recs[i].name.decode(), int(recs[i].items), float(recs[i].ms)) for i in range(min(n.value, cap))]


def ckks_graph_create(h):
    g = ctypes.c_void_p()
    _call("ckks_graph_create", h, ctypes.byref(g))
    return g


def ckks_graph_destroy(g):
    lib().ckks_graph_destroy(g)


def ckks_graph_add_node(g, kind, attrs=None):
    nid = ctypes.c_uint32()
    _call("ckks_graph_add_node", g, kind, ctypes.byref(attrs) if attrs is not None else None, ctypes.byref(nid))
    return nid.value


def ckks_graph_add_edge(g, src, dst):
    _call("ckks_graph_add_edge", g, src, dst)


def ckks_graph_plan(g):
    ws = ctypes.c_size_t()
    nout = ctypes.c_uint32()
    _call("ckks_graph_plan", g, ctypes.byref(ws), ctypes.byref(nout))
    return ws.value, nout.value


def ckks_graph_run(g, inputs, outputs, rk, galois_elts, galois_keys, ws, ws_bytes, stream=None):
    n = len(galois_elts)
    ge = (ctypes.c_uint32 * max(n, 1))(*galois_elts)
    gk = (ctypes.c_void_p * max(n, 1))(*galois_keys)
    _call("ckks_graph_run", g, inputs, len(inputs), outputs, len(outputs), rk, ge, gk, n, ws, ws_bytes, stream)


def ckks_graph_autohe(g, n_nodes):
    ng = ctypes.c_uint32()
    gof = (ctypes.c_uint32 * max(n_nodes, 1))()
    cost = (ctypes.c_uint32 * max(n_nodes, 1))()
    _call("ckks_graph_autohe", g, ctypes.byref(ng), gof, cost, n_nodes)
    return ng.value, [int(gof[i]) for i in range(n_nodes)], [int(cost[i]) for i in range(ng.value)]
