"""Encrypted lowerings of the benchmark networks, on the oracle's
primitives.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper builds conv and dense nodes as sums of ciphertext x weight
products plus a bias (Sections 4.2.2-4.2.3; its Equation for the biased
cross-correlation), uses a polynomial activation, and lets the ciphertext
container rescale after every product (Section 4.1). The op sequence of
each layer below is fixed so that the GPU path can reproduce it bit for
bit:

  linear layer (integer weights round(w * 2^40)):
      acc = sum_k w_k ct_k ; acc = rescale(acc) ; acc = acc + round(b * scale)
  diagonal (rotation-based) dense layer:
      acc = sum_i diag_i (x) rot(x, in_steps[i]) ; acc = rescale(acc) ;
      for r in post_steps: acc = acc + rot(acc, r) ; acc = acc + bias_pt
  square activation: rescale(relinearise(x (x) x))
  polynomial activation p(x) = c0 + c1 x + ... + cd x^d (Horner's rule,
  constants round(c * 2^40) for the product, round(c * scale) for sums):
      h = rescale(x * c_d) ; for k = d-1 .. 1: h = h + c_k ;
      h = rescale(relinearise(x' (x) h)) with x' = x switched down to h's
      level ; h = h + c_0

Rotations by a step that has its own Galois key use it directly;
otherwise the step is composed from power-of-two keys in non-adjacent form,
least significant digit first.
"""
import numpy as np

from . import encoding as E
from . import plainnet as PN


def galois_seed(base, g):
    """seed of the Galois key for element g (both sides derive it so)"""
    return base + g


class Keys:
    """Oracle keys derived from one seed: secret (seed), public (seed + 1),
    relinearisation (seed + 2), Galois for element g (seed + 3 + g)."""

    def __init__(self, orc, seed, galois_elts=()):
        self.orc = orc
        self.s, self.sn = orc.keygen_secret(seed)
        self.pk = orc.keygen_public(self.sn, seed + 1)
        self.rk = orc.keygen_relin(self.sn, seed + 2)
        self.seed = seed
        self.gk = {}
        for g in galois_elts:
            self.add_galois(g)

    def add_galois(self, g):
        if g not in self.gk:
            self.gk[g] = self.orc.keygen_galois(self.s, self.sn, g, galois_seed(self.seed + 3, g))
        return self.gk[g]


def rotate(orc, keys, ct, step):
    half = orc.N // 2
    step %= half
    if step == 0:
        return ct
    g = orc.galois_elt(step)
    if g in keys.gk:
        return orc.apply_galois(ct, g, keys.gk[g])
    # signed step in (-N/4, N/4], composed in non-adjacent form
    s = step if step <= half // 2 else step - half
    for k, d in PN.naf(s):
        gk = orc.galois_elt(d * (1 << k))
        ct = orc.apply_galois(ct, gk, keys.gk[gk])
    return ct


def naf_elements(orc, steps):
    """Galois elements needed to compose the given steps from powers of two"""
    half = orc.N // 2
    out = set()
    for st in steps:
        st %= half
        if st == 0:
            continue
        s = st if st <= half // 2 else st - half
        for k, d in PN.naf(s):
            out.add(orc.galois_elt(d * (1 << k)))
    return sorted(out)


def linear(orc, cts, scale, rows, w_scale, biases):
    """rows[j] = [(input index, weight)], biases[j] float or None.
    Returns (output cts, output scale)."""
    level = cts[0].shape[1] - 1
    q_top = orc.q[level]
    out_scale = scale * w_scale / q_top
    outs = []
    for j, row in enumerate(rows):
        idx = [i for i, _ in row]
        w = [round_half_away(x * w_scale) for _, x in row]
        acc = orc.lincomb([cts[i] for i in idx], w)
        acc = orc.rescale(acc)
        if biases is not None and biases[j] is not None:
            acc = orc.add_const(acc, round_half_away(biases[j] * out_scale))
        outs.append(acc)
    return outs, out_scale


def square(orc, keys, ct, scale):
    return orc.mul_relin_rescale(ct, ct, keys.rk), scale * scale / orc.q[ct.shape[1] - 1]


def round_half_away(v):
    """integer nearest to v, halves away from zero (the encoding rounding)"""
    return int(np.sign(v) * np.floor(abs(v) + 0.5))


def poly(orc, keys, ct, scale, coeffs, w_scale):
    """Polynomial activation of degree d = len(coeffs) - 1 >= 1 (Section
    4.4's approximations of ReLU and sigmoid). Returns (ct, scale); uses d
    levels."""
    d = len(coeffs) - 1
    level = ct.shape[1] - 1
    h = orc.rescale(orc.mul_const(ct, round_half_away(coeffs[d] * w_scale)))
    hs = scale * w_scale / orc.q[level]
    for k in range(d - 1, 0, -1):
        h = orc.add_const(h, round_half_away(coeffs[k] * hs))
        lv = h.shape[1] - 1
        xs = orc.mod_switch(ct, lv)
        h = orc.mul_relin_rescale(xs, h, keys.rk)
        hs = scale * hs / orc.q[lv]
    h = orc.add_const(h, round_half_away(coeffs[0] * hs))
    return h, hs


def diag_dense_hoisted(orc, keys, ct, scale, diag_coeffs, pt_scale, in_steps, post_steps, bias_pt=None):
    """As diag_dense, with the in_steps rotations hoisted: one shared
    decomposition of the input and one ModDown for the whole weighted sum
    (orc.hoisted_linear); every nonzero step uses its own Galois key.
    diag_coeffs: integer plaintext coefficients [n_diag][N] at pt_scale."""
    elts = [1 if st % (orc.N // 2) == 0 else orc.galois_elt(st) for st in in_steps]
    gks = [None if g == 1 else keys.gk[g] for g in elts]
    acc = orc.hoisted_linear(ct, elts, gks, diag_coeffs)
    level = ct.shape[1] - 1
    acc = orc.rescale(acc)
    out_scale = scale * pt_scale / orc.q[level]
    for st in post_steps:
        acc = orc.add(acc, rotate(orc, keys, acc, st))
    if bias_pt is not None:
        acc = orc.add_plain(acc, bias_pt)
    return acc, out_scale


def diag_dense(orc, keys, ct, scale, diag_pts, pt_scale, in_steps, post_steps, bias_pt=None):
    """diag_pts: NTT-form plaintexts at the ciphertext's level (integer
    encodings at pt_scale); bias_pt: NTT-form plaintext at the level and
    scale after the rescale, or None."""
    acc = None
    for pt, st in zip(diag_pts, in_steps):
        t = orc.mul_plain(rotate(orc, keys, ct, st), pt)
        acc = t if acc is None else orc.add(acc, t)
    level = ct.shape[1] - 1
    acc = orc.rescale(acc)
    out_scale = scale * pt_scale / orc.q[level]
    for st in post_steps:
        acc = orc.add(acc, rotate(orc, keys, acc, st))
    if bias_pt is not None:
        acc = orc.add_plain(acc, bias_pt)
    return acc, out_scale


def conv_slots(orc, keys, ct, scale, mask_coeffs, steps, bias_pts, pt_scale):
    """The paper's conv layout on one image-in-slots ciphertext: per filter f
    the masked-kernel taps summed with hoisted rotations, rescale, + bias at
    the anchors, then x^2. mask_coeffs[f]: [k*k][N] integer plaintexts at
    pt_scale; bias_pts[f]: NTT-form plaintext at the level and scale after
    the rescale. Returns ([F] ciphertexts, scale)."""
    outs, s_out = [], None
    for f in range(len(mask_coeffs)):
        y, s = diag_dense_hoisted(orc, keys, ct, scale, mask_coeffs[f], pt_scale, steps, [], bias_pts[f])
        y, s_out = square(orc, keys, y, s)
        outs.append(y)
    return outs, s_out


def conv_commuted(orc, keys, ct, scale, mask_coeffs, bias_pts, pt_scale):
    """The paper's conv layer with the sum over the kernel commuted past a
    key rotation (Section 4.2.2): per filter f and tap t the masked product
    of the unrotated ciphertext, rescaled, plus the commuted bias terms.
    mask_coeffs[f][t]: integer plaintext at pt_scale; bias_pts[f][t]:
    NTT-form plaintext at the level and scale after the rescale. Returns
    ([F * k*k] ciphertexts, filter-major, scale)."""
    outs, s_out = [], None
    for f in range(len(mask_coeffs)):
        for t in range(len(mask_coeffs[f])):
            y, s_out = diag_dense(orc, keys, ct, scale, [orc.reduce_int(mask_coeffs[f][t], ct.shape[1] - 1)],
                                  pt_scale, [0], [], bias_pts[f][t])
            outs.append(y)
    return outs, s_out


def key_rotation(orc, keys, cts, scales, reform, level, scale, seed, obj0=0):
    """The client's key rotation (Sections 4.2.2 and 6): every ciphertext is
    sent back, decrypted and decoded; the client's plaintext function
    ``reform`` maps the list of decoded slot vectors to new slot vectors
    (here the sum over the kernel and a change of layout), which are
    encoded at ``scale`` and encrypted afresh at ``level`` (seed, object
    ids obj0, obj0 + 1, ...). Returns (ciphertexts, their integer
    plaintexts)."""
    vals = [E.decode_residues(orc.decrypt(keys.sn, ct), orc.q, s, orc.N).real for ct, s in zip(cts, scales)]
    new = reform(vals)
    pts = [E.encode(v, scale, orc.N) for v in new]
    outs = [orc.encrypt(keys.pk, orc.reduce_int(m, level), level, seed, obj0 + k) for k, m in enumerate(pts)]
    return outs, pts


def slots_dense(orc, keys, conv_cts, scale, mask_pts, pt_scale, bias_pts, steps):
    """Dense layer after the image-in-slots conv, summed on the server
    (Section 4.2.2 read with Galois rotations): for neuron j the filter
    outputs conv_cts[f] times the masks mask_pts[j][f] (NTT-form
    plaintexts at pt_scale, the layer's weights at the anchors), added, rescaled,
    rotate-and-summed over the image block (steps) and given the bias
    plaintext bias_pts[j] (at the level and scale after the rescale).
    Returns ([n] ciphertexts, scale)."""
    level = conv_cts[0].shape[1] - 1
    outs, s_out = [], None
    for j in range(len(mask_pts)):
        acc = None
        for f, ct in enumerate(conv_cts):
            t = orc.mul_plain(ct, mask_pts[j][f])
            acc = t if acc is None else orc.add(acc, t)
        acc = orc.rescale(acc)
        for st in steps:
            acc = orc.add(acc, rotate(orc, keys, acc, st))
        outs.append(orc.add_plain(acc, bias_pts[j]))
    return outs, scale * pt_scale / orc.q[level]
