"""FP64 plaintext networks: the paper's validation method (Section 5:
the same graph is run on plain arrays and on ciphertexts and the results
are compared).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Each network exists twice:
  * ``*_math``: the plain network as written (matrix products, x^2);
  * ``*_packed``: the same computation on one FP64 slot vector laid out as
    the encrypted lowering lays it out, with np.roll for slot rotations
    (left rotation by r: slot j <- slot j + r). Agreement of the two to
    1e-12 pins the packing algebra (diagonals, rotate-and-sum) before any
    encryption is involved.
"""
import numpy as np


def naf(n):
    """Non-adjacent form of a signed integer, least significant digit
    first: list of (position, +1 / -1)."""
    out = []
    k = 0
    while n != 0:
        if n & 1:
            d = 2 - (n & 3)  # +1 or -1
            out.append((k, d))
            n -= d
        n >>= 1
        k += 1
    return out


# ---------------------------------------------------------------------------
# tiny dense: 16 features x 256 samples in 4096 slots, dense 16->8, x^2
# ---------------------------------------------------------------------------
def tiny_dense_math(x, W):
    """x [16][256], W [8][16] -> (W x)^2 [8][256]"""
    return (W @ x) ** 2


def tiny_dense_layout(n_in=16, n_samples=256):
    """feature-major: slot f * n_samples + w"""
    return n_in * n_samples


def tiny_dense_diagonals(W, n_samples=256):
    """d_i[f * S + w] = W[f mod n_out][(f + i) mod n_in] for i < n_out"""
    n_out, n_in = W.shape
    d = np.zeros((n_out, n_in * n_samples))
    for i in range(n_out):
        for f in range(n_in):
            d[i, f * n_samples:(f + 1) * n_samples] = W[f % n_out, (f + i) % n_in]
    return d


def tiny_dense_steps(n_in=16, n_out=8, n_samples=256):
    """input rotations (i * S for i < n_out) and the rotate-and-sum steps"""
    in_steps = [i * n_samples for i in range(n_out)]
    post = []
    span = n_out
    while span < n_in:
        post.append(span * n_samples)
        span *= 2
    return in_steps, post


def tiny_dense_packed(x, W):
    n_out, n_in = W.shape
    S = x.shape[1]
    v = x.reshape(-1)
    d = tiny_dense_diagonals(W, S)
    in_steps, post = tiny_dense_steps(n_in, n_out, S)
    y = sum(d[i] * np.roll(v, -in_steps[i]) for i in range(n_out))
    for r in post:
        y = y + np.roll(y, -r)
    y = y * y
    return y[: n_out * S].reshape(n_out, S)


# ---------------------------------------------------------------------------
# vision: slot-batched, one ciphertext per pixel
# ---------------------------------------------------------------------------
def vision_conv_rows(conv_w, side=28, stride=2):
    """Output (o, y, x) of the strided cross-correlation as a sparse row:
    [(pixel index, weight)], pixels outside the image (the zero padding of
    one bottom row and one right column) contribute nothing."""
    F, k, _ = conv_w.shape
    out_side = (side + 1 - k) // stride + 1
    rows = []
    for o in range(F):
        for y in range(out_side):
            for xx in range(out_side):
                row = []
                for dy in range(k):
                    for dx in range(k):
                        r, c = stride * y + dy, stride * xx + dx
                        if r < side and c < side:
                            row.append((r * side + c, conv_w[o, dy, dx]))
                rows.append(row)
    return rows, out_side


def vision_math(x, P):
    """x [n][28][28] -> logits [n][10]"""
    n, side, _ = x.shape
    F, k, _ = P["conv_w"].shape
    pad = np.zeros((n, side + 1, side + 1))
    pad[:, :side, :side] = x
    out_side = (side + 1 - k) // 2 + 1
    conv = np.zeros((n, F, out_side, out_side))
    for o in range(F):
        for y in range(out_side):
            for xx in range(out_side):
                patch = pad[:, 2 * y:2 * y + k, 2 * xx:2 * xx + k]
                conv[:, o, y, xx] = np.tensordot(patch, P["conv_w"][o], axes=([1, 2], [0, 1])) + P["conv_b"][o]
    h = (conv ** 2).reshape(n, -1)
    h = (h @ P["w1"].T + P["b1"]) ** 2
    return h @ P["w2"].T + P["b2"]


def vision_packed(x, P):
    """Same network on the per-pixel slot vectors (slot s = image s)."""
    n, side, _ = x.shape
    pix = x.reshape(n, -1).T  # [784][n]
    rows, _ = vision_conv_rows(P["conv_w"], side)
    F = P["conv_w"].shape[0]
    per = len(rows) // F
    conv = np.stack([sum(w * pix[i] for i, w in row) + P["conv_b"][j // per] for j, row in enumerate(rows)])
    h = conv ** 2
    h = np.stack([P["w1"][j] @ h + P["b1"][j] for j in range(P["w1"].shape[0])]) ** 2
    out = np.stack([P["w2"][j] @ h + P["b2"][j] for j in range(P["w2"].shape[0])])
    return out.T


# ---------------------------------------------------------------------------
# yield regressor: feature-major packing, rotation-based matvec
# ---------------------------------------------------------------------------
def yield_math(x, ws, bs):
    h = (x @ ws[0].T + bs[0]) ** 2
    h = (h @ ws[1].T + bs[1]) ** 2
    return h @ ws[2].T + bs[2]


def yield_layout(slots, n_feat=256):
    """windows per ciphertext W = slots / 256; slot f * W + w"""
    return slots // n_feat


def yield_pack(x, slots, n_feat=256):
    """x [n][147] -> slot vectors [n_ct][slots] (zero padded features)"""
    W = yield_layout(slots, n_feat)
    n = x.shape[0]
    n_ct = -(-n // W)
    v = np.zeros((n_ct, n_feat, W))
    for c in range(n_ct):
        blk = x[c * W:(c + 1) * W]
        v[c, : blk.shape[1], : blk.shape[0]] = blk.T
    return v.reshape(n_ct, -1)


def yield_layer_plan(n_in, n_out, period, W):
    """Hybrid diagonal layer on an input that is `period`-periodic in the
    feature index (period = 256 for the first layer): diagonals i < n_out
    with d_i[f] = M[f mod n_out][(f + i) mod period] (zero beyond n_in),
    input rotations i * W, then rotate-and-sum by n_out * W, 2 n_out W, ...
    until the span reaches the period."""
    in_steps = [i * W for i in range(n_out)]
    post = []
    span = n_out
    while span < period:
        post.append(span * W)
        span *= 2
    return in_steps, post


def yield_diagonals(M, period, W, n_feat=256):
    n_out, n_in = M.shape
    d = np.zeros((n_out, n_feat, W))
    for i in range(n_out):
        for f in range(n_feat):
            col = (f + i) % period
            if col < n_in:
                d[i, f, :] = M[f % n_out, col]
    return d.reshape(n_out, -1)


def yield_bias_vector(b, W, n_feat=256):
    """bias of output j at every feature block f with f mod n_out = j"""
    n_out = len(b)
    v = np.zeros((n_feat, W))
    for f in range(n_feat):
        v[f] = b[f % n_out]
    return v.reshape(-1)


def yield_packed(x, ws, bs, slots):
    W = yield_layout(slots)
    v = yield_pack(x, slots)
    periods = [256, 64, 16]
    outs = []
    for c in range(v.shape[0]):
        y = v[c]
        for layer in range(3):
            M, b = ws[layer], bs[layer]
            n_out = M.shape[0]
            in_steps, post = yield_layer_plan(M.shape[1], n_out, periods[layer], W)
            d = yield_diagonals(M, periods[layer], W)
            z = sum(d[i] * np.roll(y, -in_steps[i]) for i in range(n_out))
            for r in post:
                z = z + np.roll(z, -r)
            z = z + yield_bias_vector(b, W)
            y = z ** 2 if layer < 2 else z
        outs.append(y[:W])
    return np.concatenate(outs)[: x.shape[0]]


# ---------------------------------------------------------------------------
# polynomial activations (Section 4.4 and the appendix equations)
# ---------------------------------------------------------------------------
def relu_approx_coeffs(q):
    """R_a(x) = 4/(3 pi q) x^2 + x/2 + q/(3 pi): coefficients c0, c1, c2 for
    the approximation range q."""
    return [q / (3.0 * np.pi), 0.5, 4.0 / (3.0 * np.pi * q)]


def sigmoid_approx_coeffs():
    """sigma_a(x) = 0.5 + 0.197 x - 0.004 x^3: coefficients c0..c3."""
    return [0.5, 0.197, 0.0, -0.004]


def poly_eval(coeffs, x):
    """sum_k c_k x^k, term by term (no Horner), in FP64."""
    x = np.asarray(x, dtype=np.float64)
    return sum(c * x ** k for k, c in enumerate(coeffs))


# ---------------------------------------------------------------------------
# the paper's conv layout (Section 4.2.2, kernel masquerading): the image in
# the slots of one ciphertext (image b in the slot block [b*block, (b+1)*block),
# pixel p = 28 r + c), each filter a sparse masked kernel per tap
# ---------------------------------------------------------------------------
def conv_slots_layout(conv_w, conv_b, slots, side=28, block=1024, stride=2):
    """Rotation steps of the k*k taps, per filter and tap the mask (the tap
    weight at every output anchor whose tap pixel lies inside the image),
    and per filter the bias at the anchors; anchors are p = (2y) 28 + 2x.
    Returns (steps [k*k], masks [F][k*k][slots], bias [F][slots])."""
    F, k, _ = conv_w.shape
    out_side = (side + 1 - k) // stride + 1
    n_blk = slots // block
    steps = [dy * side + dx for dy in range(k) for dx in range(k)]
    masks = np.zeros((F, k * k, slots))
    bias = np.zeros((F, slots))
    for y in range(out_side):
        for xx in range(out_side):
            p = stride * y * side + stride * xx
            for b in range(n_blk):
                bias[:, b * block + p] = conv_b
            for t, (dy, dx) in enumerate((dy, dx) for dy in range(k) for dx in range(k)):
                if stride * y + dy < side and stride * xx + dx < side:
                    for b in range(n_blk):
                        masks[:, t, b * block + p] = conv_w[:, dy, dx]
    return steps, masks, bias


def conv_slots_pack(x, slots, block=1024):
    """images [n][side][side] -> slot vectors [n_ct][slots]"""
    n = x.shape[0]
    per = slots // block
    n_ct = -(-n // per)
    v = np.zeros((n_ct, slots))
    flat = x.reshape(n, -1)
    for i in range(n):
        v[i // per, (i % per) * block:(i % per) * block + flat.shape[1]] = flat[i]
    return v


def conv_slots_packed(x, P, slots, block=1024):
    """conv + bias + x^2 in the image-in-slots layout with np.roll for the
    rotations: [n_ct][F][slots] (values at the anchors, zero elsewhere)"""
    steps, masks, bias = conv_slots_layout(P["conv_w"], P["conv_b"], slots, block=block)
    v = conv_slots_pack(x, slots, block)
    out = np.zeros((v.shape[0], masks.shape[0], slots))
    for c in range(v.shape[0]):
        for f in range(masks.shape[0]):
            acc = sum(masks[f, t] * np.roll(v[c], -s) for t, s in enumerate(steps))
            out[c, f] = (acc + bias[f]) ** 2
    return out


def conv_slots_anchor_values(out, n, side=28, block=1024, out_side=13):
    """[n_ct][F][slots] -> [n][F][out_side][out_side] read at the anchors"""
    F, slots = out.shape[1], out.shape[2]
    per = slots // block
    res = np.zeros((n, F, out_side, out_side))
    for i in range(n):
        for y in range(out_side):
            for xx in range(out_side):
                res[i, :, y, xx] = out[i // per, :, (i % per) * block + 2 * y * side + 2 * xx]
    return res


def slots_dense_masks(W1, slots, block=1024, side=28, out_side=13, stride=2):
    """Dense 845 -> n after the image-in-slots conv, summed on the server
    by rotations: for neuron j and filter f a mask holding W1[j, f 169 +
    13 y + x] at the anchor 2y side + 2x of every image block; the masked
    filter outputs are added, and a rotate-and-sum over the block (steps 1,
    2, ..., block / 2) leaves the neuron's value at the block's first slot.
    Returns masks [n][F][slots]."""
    n, n_in = W1.shape
    F = n_in // (out_side * out_side)
    masks = np.zeros((n, F, slots))
    for b in range(slots // block):
        for f in range(F):
            for y in range(out_side):
                for xx in range(out_side):
                    masks[:, f, b * block + stride * y * side + stride * xx] = W1[:, f * out_side * out_side +
                                                                                   y * out_side + xx]
    return masks


def block_sum_steps(block=1024):
    """rotate-and-sum steps that sum a block of slots into its first slot"""
    return [1 << k for k in range(int(np.log2(block)))]


def slots_network_packed(x, P, slots, block=1024):
    """The whole vision network in the image-in-slots layout (FP64, np.roll):
    conv by masked taps, x^2, dense 1 by masks + rotate-and-sum per neuron,
    x^2, dense 2 by scalar weights; logits [n_img][classes] read at each
    block's first slot."""
    conv = conv_slots_packed(x, P, slots, block)  # [n_ct][F][slots], squared
    masks = slots_dense_masks(P["w1"], slots, block)
    n_ct = conv.shape[0]
    per = slots // block
    out = []
    for c in range(n_ct):
        h = []
        for j in range(masks.shape[0]):
            acc = (masks[j] * conv[c]).sum(axis=0)
            for st in block_sum_steps(block):
                acc = acc + np.roll(acc, -st)
            h.append((acc + P["b1"][j]) ** 2)
        h = np.stack(h)
        logits = P["w2"] @ h + P["b2"][:, None]  # [classes][slots]
        out.append(logits[:, ::block][:, :per].T)
    return np.concatenate(out)[: x.shape[0]]


def conv_commuted_layout(conv_w, conv_b, slots, side=28, block=1024, stride=2):
    """Kernel masquerading with the sum over the kernel left for after a
    key rotation (Section 4.2.2): per filter f and tap t = (dy, dx) one
    masked product of the unrotated image-in-slots vector, whose mask holds
    w_f[dy, dx] at the tap pixel q = p + side dy + dx of every output anchor
    p = stride y side + stride x with that pixel inside the image. The bias
    is commuted into the terms: b_f / n(p) at the same positions, n(p) the
    anchor's taps inside the image, so that the terms of an anchor sum to
    its biased cross-correlation. Every tap keeps its own ciphertext (a
    ciphertext cannot be folded onto itself without rotations).
    Returns (offsets [k*k], masks [F][k*k][slots], bias [F][k*k][slots])."""
    F, k, _ = conv_w.shape
    out_side = (side + 1 - k) // stride + 1
    n_blk = slots // block
    taps = [(dy, dx) for dy in range(k) for dx in range(k)]
    offsets = [dy * side + dx for dy, dx in taps]
    masks = np.zeros((F, k * k, slots))
    bias = np.zeros((F, k * k, slots))
    for y in range(out_side):
        for xx in range(out_side):
            p = stride * y * side + stride * xx
            valid = [t for t, (dy, dx) in enumerate(taps) if stride * y + dy < side and stride * xx + dx < side]
            for t in valid:
                dy, dx = taps[t]
                for b in range(n_blk):
                    q = b * block + p + offsets[t]
                    masks[:, t, q] = conv_w[:, dy, dx]
                    bias[:, t, q] = conv_b / len(valid)
    return offsets, masks, bias


def conv_commuted_sum(vals, n_img, side=28, block=1024, k=5, stride=2):
    """The client's side of the key rotation: decoded term vectors
    vals [n_ct][F][k*k][slots] -> conv outputs [n_img][F][13][13], each the
    sum over taps t of the term at the anchor's tap pixel."""
    n_ct, F, kk, slots = vals.shape
    per = slots // block
    out_side = (side + 1 - k) // stride + 1
    offsets = [dy * side + dx for dy in range(k) for dx in range(k)]
    out = np.zeros((n_img, F, out_side, out_side))
    for i in range(n_img):
        c, b = i // per, i % per
        for y in range(out_side):
            for xx in range(out_side):
                p = b * block + stride * y * side + stride * xx
                for t in range(kk):
                    if stride * y + t // k < side and stride * xx + t % k < side:
                        out[i, :, y, xx] += vals[c, :, t, p + offsets[t]]
    return out


def conv_commuted_packed(x, P, slots, block=1024):
    """the terms of the commuted conv on the packed images (FP64):
    [n_ct][F][k*k][slots] = mask (.) v + bias"""
    offsets, masks, bias = conv_commuted_layout(P["conv_w"], P["conv_b"], slots, block=block)
    v = conv_slots_pack(x, slots, block)
    return np.stack([masks * v[c][None, None, :] + bias for c in range(v.shape[0])])


def vision_conv_math(x, P):
    """the biased cross-correlation of vision_math: [n][F][13][13]"""
    n, side, _ = x.shape
    F, k, _ = P["conv_w"].shape
    pad = np.zeros((n, side + 1, side + 1))
    pad[:, :side, :side] = x
    out_side = (side + 1 - k) // 2 + 1
    conv = np.zeros((n, F, out_side, out_side))
    for o in range(F):
        for y in range(out_side):
            for xx in range(out_side):
                patch = pad[:, 2 * y:2 * y + k, 2 * xx:2 * xx + k]
                conv[:, o, y, xx] = np.tensordot(patch, P["conv_w"][o], axes=([1, 2], [0, 1])) + P["conv_b"][o]
    return conv


def vision_tail_math(conv, P):
    """the rest of vision_math after the conv: x^2 -> dense -> x^2 -> dense"""
    n = conv.shape[0]
    h = (conv ** 2).reshape(n, -1)
    h = (h @ P["w1"].T + P["b1"]) ** 2
    return h @ P["w2"].T + P["b2"]


def vision_conv_square_math(x, P):
    """the first two layers of vision_math: (conv + bias)^2 [n][F][13][13]"""
    n, side, _ = x.shape
    F, k, _ = P["conv_w"].shape
    pad = np.zeros((n, side + 1, side + 1))
    pad[:, :side, :side] = x
    out_side = (side + 1 - k) // 2 + 1
    conv = np.zeros((n, F, out_side, out_side))
    for o in range(F):
        for y in range(out_side):
            for xx in range(out_side):
                patch = pad[:, 2 * y:2 * y + k, 2 * xx:2 * xx + k]
                conv[:, o, y, xx] = np.tensordot(patch, P["conv_w"][o], axes=([1, 2], [0, 1])) + P["conv_b"][o]
    return conv ** 2
