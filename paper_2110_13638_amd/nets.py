"""Encrypted lowerings of the paper's network shapes onto the graph runtime.

Layer semantics follow the paper: conv ("biased cross-correlation",
Section 4.2.2) and dense (Section 4.2.3) are sums of ciphertext x weight
products plus a bias, the activation is a polynomial (x^2), and the
container rescales after every product (Section 4.1). Three packings:

  * tiny dense: features x samples in one ciphertext (feature-major),
    dense layer by the hybrid diagonal method (rotations + plaintext
    diagonals), then rotate-and-sum, then x^2;
  * vision: slot-batched, one ciphertext per pixel, image s in slot s;
    conv = sparse linear layer over pixels (stride 2, one zero row and
    column of padding), dense layers = linear layers over ciphertexts;
  * yield regressor: windows x 256 padded features per ciphertext,
    three hybrid-diagonal dense layers with power-of-two Galois keys.
"""
import math

import numpy as np

from .graph import Graph


def naf_digits(n):
    """signed binary digits of n, least significant first: [(position, +-1)]"""
    out, k = [], 0
    while n:
        if n & 1:
            d = 2 - (n & 3)
            out.append((k, d))
            n -= d
        n >>= 1
        k += 1
    return out


def galois_for_steps(ctx, steps, direct=False):
    """Galois elements needed for the steps: each step itself when
    direct, else the power-of-two factors of its non-adjacent form."""
    half = ctx.N // 2
    out = set()
    for s in steps:
        s %= half
        if s == 0:
            continue
        if direct:
            out.add(ctx.galois_elt(s))
            continue
        v = s if s <= half // 2 else s - half
        for k, d in naf_digits(v):
            out.add(ctx.galois_elt(d * (1 << k)))
    return sorted(out)


def galois_key_seed(base, g):
    return base + g


# ---------------------------------------------------------------------------
# tiny dense: dense n_in -> n_out by diagonals on n_in x S slots, then x^2
# ---------------------------------------------------------------------------
def diag_plan(n_in, n_out, block):
    """in_steps i * block (i < n_out), then rotate-and-sum by n_out * block,
    2 n_out block, ... while the span stays below n_in"""
    in_steps = [i * block for i in range(n_out)]
    post, span = [], n_out
    while span < n_in:
        post.append(span * block)
        span *= 2
    return in_steps, post


def tiny_dense_diagonals(W, block):
    """diag_i[f * block + w] = W[f mod n_out][(f + i) mod n_in]"""
    n_out, n_in = W.shape
    d = np.empty((n_out, n_in, block))
    for i in range(n_out):
        for f in range(n_in):
            d[i, f, :] = W[f % n_out, (f + i) % n_in]
    return d.reshape(n_out, n_in * block)


def build_tiny_dense(ctx, W, block, in_level, scale, diag_coeffs=None):
    n_out, n_in = W.shape
    in_steps, post = diag_plan(n_in, n_out, block)
    if diag_coeffs is None:
        diag_coeffs = np.stack([ctx.encode_coeffs(d, scale) for d in tiny_dense_diagonals(W, block)])
    g = Graph(ctx)
    x = g.input(1, in_level, scale)
    d = g.diag_dense(diag_coeffs, in_steps, scale, post)
    g.chain(x, d, g.square(), g.output())
    g.plan()
    return g, in_steps + post


# ---------------------------------------------------------------------------
# vision: slot-batched conv -> x^2 -> dense -> x^2 -> dense
# ---------------------------------------------------------------------------
def conv_rows(conv_w, side, stride=2):
    """rows of the strided cross-correlation over the pixel ciphertexts:
    output (o, y, x) = sum w_o[dy, dx] pix(2y + dy, 2x + dx); pixels in the
    zero padding (one bottom row, one right column) are dropped"""
    F, k, _ = conv_w.shape
    out_side = (side + 1 - k) // stride + 1
    rows = []
    for o in range(F):
        for y in range(out_side):
            for xx in range(out_side):
                r = []
                for dy in range(k):
                    for dx in range(k):
                        pr, pc = stride * y + dy, stride * xx + dx
                        if pr < side and pc < side:
                            r.append((pr * side + pc, conv_w[o, dy, dx]))
                rows.append(r)
    return rows, out_side


def reorder_conv_rows(rows, filters):
    """Group the filters of one output position next to each other (they
    share their pixel list, so the linear kernel loads it once): new row
    order is position-major; returns rows and the permutation back."""
    per = len(rows) // filters
    order = [o * per + p for p in range(per) for o in range(filters)]
    return [rows[i] for i in order], order


def build_vision(ctx, P, side, in_level, scale, w_scale=None):
    w_scale = w_scale or scale
    F = P["conv_w"].shape[0]
    rows, out_side = conv_rows(P["conv_w"], side)
    rows_g, order = reorder_conv_rows(rows, F)
    per = out_side * out_side
    conv_bias = [P["conv_b"][i // per] for i in order]
    # dense 1 consumes the conv outputs in their grouped order
    W1 = P["w1"][:, order]
    g = Graph(ctx)
    x = g.input(side * side, in_level, scale)
    c = g.linear(rows_g, w_scale, conv_bias)
    s1 = g.square()
    d1 = g.dense(W1, w_scale, P["b1"])
    s2 = g.square()
    d2 = g.dense(P["w2"], w_scale, P["b2"])
    g.chain(x, c, s1, d1, s2, d2, g.output())
    g.plan()
    return g


# ---------------------------------------------------------------------------
# yield regressor: 256 padded features x W windows per ciphertext
# ---------------------------------------------------------------------------
def yield_windows(slots, n_feat=256):
    return slots // n_feat


def yield_pack(x, slots, n_feat=256):
    """x [n][features] -> [n_ct][slots], slot f * W + w holds window w's
    feature f (zero padded to 256 features)"""
    W = yield_windows(slots, n_feat)
    n, f = x.shape
    n_ct = -(-n // W)
    v = np.zeros((n_ct, n_feat, W))
    for c in range(n_ct):
        blk = x[c * W:(c + 1) * W]
        v[c, :f, : blk.shape[0]] = blk.T
    return v.reshape(n_ct, n_feat * W)


def yield_diagonals(M, period, W, n_feat=256):
    """d_i[f * W + w] = M[f mod n_out][(f + i) mod period] (0 beyond n_in)"""
    n_out, n_in = M.shape
    d = np.zeros((n_out, n_feat, W))
    for i in range(n_out):
        for f in range(n_feat):
            c = (f + i) % period
            if c < n_in:
                d[i, f, :] = M[f % n_out, c]
    return d.reshape(n_out, n_feat * W)


def yield_bias(b, W, n_feat=256):
    n_out = len(b)
    return np.repeat(np.array([b[f % n_out] for f in range(n_feat)]), W)


YIELD_PERIODS = (256, 64, 16)


def yield_steps(ws, W):
    steps = []
    for l, M in enumerate(ws):
        a, b = diag_plan(YIELD_PERIODS[l], M.shape[0], W)
        steps += a + b
    return steps


def build_yield(ctx, ws, bs, n_ct, in_level, scale, diag_coeffs=None, bias_coeffs=None, hoisted=False):
    """diag_coeffs / bias_coeffs: optional pre-encoded integer plaintexts
    per layer (otherwise encoded here with the library's encoder). hoisted:
    each layer's rotations share one decomposition and one ModDown (every
    step then needs its own Galois key: galois_for_steps(..., direct=True))."""
    W = yield_windows(ctx.N // 2)
    g = Graph(ctx)
    prev = g.input(n_ct, in_level, scale)
    for l, (M, b) in enumerate(zip(ws, bs)):
        in_steps, post = diag_plan(YIELD_PERIODS[l], M.shape[0], W)
        if diag_coeffs is None:
            dc = np.stack([ctx.encode_coeffs(d, scale) for d in yield_diagonals(M, YIELD_PERIODS[l], W)])
        else:
            dc = diag_coeffs[l]
        if bias_coeffs is None:
            node = g.diag_dense(dc, in_steps, scale, post, bias_slots=yield_bias(b, W), hoisted=hoisted)
        else:
            node = g.diag_dense(dc, in_steps, scale, post, bias_coeffs=bias_coeffs[l], hoisted=hoisted)
        g.edge(prev, node)
        prev = node
        if l < len(ws) - 1:
            prev = g.edge(prev, g.square())
    g.edge(prev, g.output())
    g.plan()
    return g


# ---------------------------------------------------------------------------
# polynomial activations (Section 4.4; coefficients from the appendix
# equations), c_0 first
# ---------------------------------------------------------------------------
def relu_approx_coeffs(q):
    """R_a(x) = 4/(3 pi q) x^2 + x/2 + q/(3 pi) for the approximation range q"""
    return [q / (3.0 * math.pi), 0.5, 4.0 / (3.0 * math.pi * q)]


def sigmoid_approx_coeffs():
    """sigma_a(x) = 0.5 + 0.197 x - 0.004 x^3"""
    return [0.5, 0.197, 0.0, -0.004]


# ---------------------------------------------------------------------------
# the paper's conv layout (Section 4.2.2, kernel masquerading): each image in
# a block of `block` slots of one ciphertext (pixel p = 28 r + c), each
# filter a masked kernel per tap; the k*k taps are summed with hoisted
# rotations in one DIAG_DENSE node per filter
# ---------------------------------------------------------------------------
def conv_slots_layout(conv_w, conv_b, slots, side=28, block=1024, stride=2):
    """(steps [k*k], masks [F][k*k][slots], bias [F][slots]): tap t = (dy, dx)
    rotates by 28 dy + dx; its mask holds w_f[dy, dx] at every output anchor
    p = 2y * 28 + 2x whose tap pixel lies inside the image; the bias sits at
    the anchors."""
    F, k, _ = conv_w.shape
    out_side = (side + 1 - k) // stride + 1
    n_blk = slots // block
    taps = [(dy, dx) for dy in range(k) for dx in range(k)]
    steps = [dy * side + dx for dy, dx in taps]
    masks = np.zeros((F, len(taps), slots))
    bias = np.zeros((F, slots))
    anchors = [(y, xx, stride * y * side + stride * xx) for y in range(out_side) for xx in range(out_side)]
    for b in range(n_blk):
        base = b * block
        for y, xx, p in anchors:
            bias[:, base + p] = conv_b
            for t, (dy, dx) in enumerate(taps):
                if stride * y + dy < side and stride * xx + dx < side:
                    masks[:, t, base + p] = conv_w[:, dy, dx]
    return steps, masks, bias


def conv_slots_pack(x, slots, block=1024):
    """images [n][side][side] -> [n_ct][slots], image i in block i mod (slots / block)"""
    n = x.shape[0]
    per = slots // block
    flat = x.reshape(n, -1)
    v = np.zeros((-(-n // per), slots))
    for i in range(n):
        v[i // per, (i % per) * block:(i % per) * block + flat.shape[1]] = flat[i]
    return v


def build_conv_slots(ctx, P, n_ct, in_level, scale, mask_coeffs=None, bias_coeffs=None, block=1024):
    """input (image-in-slots ciphertexts) -> per filter: masked taps summed by
    hoisted rotations, rescale, + bias, x^2 -> one output node per filter
    (outputs filter-major). Every tap step needs its own Galois key."""
    slots = ctx.N // 2
    steps, masks, bias = conv_slots_layout(P["conv_w"], P["conv_b"], slots, block=block)
    g = Graph(ctx)
    x = g.input(n_ct, in_level, scale)
    for f in range(masks.shape[0]):
        dc = mask_coeffs[f] if mask_coeffs is not None else np.stack(
            [ctx.encode_coeffs(masks[f, t], scale) for t in range(len(steps))])
        if bias_coeffs is None:
            node = g.diag_dense(dc, steps, scale, (), bias_slots=bias[f], hoisted=True)
        else:
            node = g.diag_dense(dc, steps, scale, (), bias_coeffs=bias_coeffs[f], hoisted=True)
        g.edge(x, node)
        g.chain(node, g.square(), g.output())
    g.plan()
    return g


def conv_slots_steps(side=28, k=5):
    return [dy * side + dx for dy in range(k) for dx in range(k)]


# ---------------------------------------------------------------------------
# the paper's own route through its conv (Section 4.2.2): kernel masquerading
# without rotations, the sum over the kernel commuted past a client key
# rotation, then the rest of the network in the slot-batched layout
# ---------------------------------------------------------------------------
def conv_commuted_layout(conv_w, conv_b, slots, side=28, block=1024, stride=2):
    """(offsets [k*k], masks [F][k*k][slots], bias [F][k*k][slots]): the term
    of tap t = (dy, dx) of anchor p = 2y * side + 2x sits at the tap's pixel
    p + side dy + dx of the unrotated image block, weighted by w_f[dy, dx],
    with b_f / n(p) added there (n(p): the anchor's taps inside the image;
    the bias commuted into the sum). Taps outside the image have no term."""
    F, k, _ = conv_w.shape
    out_side = (side + 1 - k) // stride + 1
    ys, xs = np.meshgrid(np.arange(out_side), np.arange(out_side), indexing="ij")
    ys, xs = ys.ravel(), xs.ravel()
    anchor = stride * ys * side + stride * xs
    # taps inside the image per anchor
    inside = np.array([[(stride * y + dy < side) and (stride * x + dx < side) for dy in range(k) for dx in range(k)]
                       for y, x in zip(ys, xs)])  # [anchors][k*k]
    n_valid = inside.sum(axis=1)
    offsets = [dy * side + dx for dy in range(k) for dx in range(k)]
    masks = np.zeros((F, k * k, slots))
    bias = np.zeros((F, k * k, slots))
    for t, off in enumerate(offsets):
        dy, dx = divmod(t, k)
        a = np.nonzero(inside[:, t])[0]
        for base in range(0, slots - block + 1, block):
            pos = base + anchor[a] + off
            masks[:, t, pos] = conv_w[:, dy, dx][:, None]
            bias[:, t, pos] = conv_b[:, None] / n_valid[a][None, :]
    return offsets, masks, bias


def build_conv_commuted(ctx, P, n_ct, in_level, scale, mask_coeffs=None, bias_coeffs=None, block=1024):
    """input (image-in-slots ciphertexts) -> one DIAG_DENSE node per filter f
    and tap t (a single diagonal at step 0: masked product, rescale, commuted
    bias terms) -> one output node each; run() returns the F * k*k outputs
    node-major: outs[(f * k*k + t) * n_ct + c]. No Galois keys."""
    slots = ctx.N // 2
    offsets, masks, bias = conv_commuted_layout(P["conv_w"], P["conv_b"], slots, block=block)
    g = Graph(ctx)
    x = g.input(n_ct, in_level, scale)
    F, KK = masks.shape[0], masks.shape[1]
    for f in range(F):
        for t in range(KK):
            dc = (mask_coeffs[f][t] if mask_coeffs is not None else ctx.encode_coeffs(masks[f, t], scale))[None]
            if bias_coeffs is None:
                node = g.diag_dense(dc, [0], scale, (), bias_slots=bias[f, t])
            else:
                node = g.diag_dense(dc, [0], scale, (), bias_coeffs=bias_coeffs[f][t])
            g.edge(x, node)
            g.edge(node, g.output())
    g.plan()
    return g


def conv_commuted_sum(terms, n_img, side=28, block=1024, k=5, stride=2):
    """Client side of the key rotation: decoded terms [n_ct][F][k*k][slots]
    -> conv outputs [n_img][F * out_side^2] (filter, row, column order):
    each output sums its taps' terms at the taps' pixels."""
    n_ct, F, KK, slots = terms.shape
    out_side = (side + 1 - k) // stride + 1
    per = slots // block
    out = np.zeros((n_img, F, out_side, out_side))
    for t in range(KK):
        dy, dx = divmod(t, k)
        ny = sum(1 for y in range(out_side) if stride * y + dy < side)
        nx = sum(1 for x in range(out_side) if stride * x + dx < side)
        pos = (stride * np.arange(ny)[:, None] + dy) * side + (stride * np.arange(nx)[None, :] + dx)
        for i in range(n_img):
            c, b = divmod(i, per)
            out[i, :, :ny, :nx] += terms[c][:, t][:, b * block + pos]
    return out.reshape(n_img, -1)


def key_rotation(ctx, cts, reform, level, scale, seed, obj0=0, keys=None):
    """The client's key rotation (Sections 4.2.2 and 6): the ciphertexts go
    back to the key holder, who decrypts and decodes them (ckks_decrypt,
    ckks_decode), applies its plaintext function ``reform`` (list of slot
    vectors -> list of slot vectors) and encrypts the result afresh at
    ``level`` and ``scale`` (ckks_encode, ckks_encrypt; object ids obj0,
    obj0 + 1, ...). Returns the new ciphertexts."""
    vals = [ctx.decrypt(c, keys=keys).real for c in cts]
    return [ctx.encrypt(ctx.encode(v, level=level, scale=scale), seed=seed, obj=obj0 + k, keys=keys)
            for k, v in enumerate(reform(vals))]


def build_vision_tail(ctx, P, in_level, scale, w_scale=None):
    """The vision network after its conv, on slot-batched conv outputs
    (filter, row, column order; image s in slot s): x^2 -> dense -> x^2 ->
    dense; weights at w_scale (default the context's scale)."""
    w_scale = w_scale or ctx.default_scale
    g = Graph(ctx)
    x = g.input(P["w1"].shape[1], in_level, scale)
    g.chain(x, g.square(), g.dense(P["w1"], w_scale, P["b1"]), g.square(), g.dense(P["w2"], w_scale, P["b2"]),
            g.output())
    g.plan()
    return g


# ---------------------------------------------------------------------------
# the vision network's dense layers directly on the image-in-slots conv
# outputs, summed on the server by rotations (no key rotation)
# ---------------------------------------------------------------------------
def slots_dense_masks(W1, slots, block=1024, side=28, out_side=13, stride=2):
    """masks [n][F][slots]: neuron j's weight for filter f's output (y, x) at
    that output's anchor 2y * side + 2x in every image block"""
    n, n_in = W1.shape
    per_f = out_side * out_side
    F = n_in // per_f
    ys, xs = np.divmod(np.arange(per_f), out_side)
    anchors = stride * ys * side + stride * xs
    masks = np.zeros((n, F, slots))
    for base in range(0, slots - block + 1, block):
        for f in range(F):
            masks[:, f, base + anchors] = W1[:, f * per_f:(f + 1) * per_f]
    return masks


def block_sum_steps(block=1024):
    """steps 1, 2, ..., block / 2: rotate-and-sum of a block into its first slot"""
    return [1 << k for k in range(block.bit_length() - 1)]


def slots_dense(ctx, conv_outs, scale, W1, b1, mask_coeffs=None, bias_coeffs=None, block=1024):
    """Dense layer over the image-in-slots conv outputs conv_outs[f][c]
    (filter f, ciphertext c): for every neuron j and ciphertext c,
    sum_f conv_outs[f][c] (x) mask_{j,f}, rescale, rotate-and-sum over the
    image block (a Galois key per step 1, 2, ..., block/2), + b1[j] at
    each block's first slot. Batched: one call per operation over all
    neurons and ciphertexts. Returns outs[j][c] (neuron j's value at each
    block's first slot)."""
    F, n_ct = len(conv_outs), len(conv_outs[0])
    n = W1.shape[0]
    slots = ctx.N // 2
    c0 = conv_outs[0][0]
    level, s_in = c0.level, c0.scale
    if mask_coeffs is None:
        masks = slots_dense_masks(W1, slots, block)
        mask_coeffs = [[ctx.encode_coeffs(masks[j, f], scale) for f in range(F)] for j in range(n)]
    pts = [[ctx.pt_from_coeffs(mask_coeffs[j][f], level, scale) for f in range(F)] for j in range(n)]
    acc = None
    for f in range(F):
        t = ctx.multiply_plain([conv_outs[f][c] for j in range(n) for c in range(n_ct)],
                               [pts[j][f] for j in range(n) for c in range(n_ct)])
        acc = t if acc is None else ctx.add(acc, t)
    acc = ctx.rescale(acc)
    for st in block_sum_steps(block):
        acc = ctx.add(acc, ctx.rotate(acc, step=st))
    out_scale = acc[0].scale
    if bias_coeffs is None:
        bias = np.zeros((n, slots))
        bias[:, ::block] = np.asarray(b1)[:, None]
        bias_coeffs = [ctx.encode_coeffs(bias[j], out_scale) for j in range(n)]
    bpts = [ctx.pt_from_coeffs(bias_coeffs[j], level - 1, out_scale) for j in range(n)]
    acc = ctx.add_plain(acc, [bpts[j] for j in range(n) for c in range(n_ct)])
    return [acc[j * n_ct:(j + 1) * n_ct] for j in range(n)]


def build_slots_head(ctx, P, n, in_level, scale, w_scale=None):
    """x^2 -> dense (scalar weights at w_scale, default the context's scale)
    on the n neuron ciphertexts of slots_dense at (in_level, scale)"""
    w_scale = w_scale or ctx.default_scale
    g = Graph(ctx)
    x = g.input(n, in_level, scale)
    g.chain(x, g.square(), g.dense(P["w2"], w_scale, P["b2"]), g.output())
    g.plan()
    return g
