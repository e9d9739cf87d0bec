"""Pins for the FP64 plaintext networks: the packed-slot circuits (the
layouts the encrypted lowerings use, with np.roll as slot rotation) agree
with the networks written as plain matrix algebra."""
import numpy as np

import synthetic as S
from oracle import plainnet as PN


def test_naf_reconstructs_and_is_non_adjacent():
    for n in list(range(-300, 300)) + [2047, 4095, 63 * 32]:
        digits = PN.naf(n)
        assert sum(d << k for k, d in digits) == n
        pos = [k for k, _ in digits]
        assert all(b - a >= 2 for a, b in zip(pos, pos[1:]))


def test_tiny_dense_packed_equals_math():
    x, W = S.tiny_dense_inputs()
    assert np.max(np.abs(PN.tiny_dense_packed(x, W) - PN.tiny_dense_math(x, W))) < 1e-12


def test_vision_packed_equals_math():
    x, P = S.vision_inputs(n_images=16)
    a, b = PN.vision_packed(x, P), PN.vision_math(x, P)
    assert a.shape == (16, 10)
    assert np.max(np.abs(a - b)) < 1e-10 * max(1.0, np.max(np.abs(b)))
    rows, side = PN.vision_conv_rows(P["conv_w"])
    assert side == 13 and len(rows) == 845
    assert sum(len(r) for r in rows) == 5 * (12 * 12 * 25 + 2 * 12 * 20 + 16)


def test_yield_packed_equals_math():
    x, ws, bs = S.yield_inputs(n_windows=40)
    for slots in (4096, 8192):
        a, b = PN.yield_packed(x, ws, bs, slots), PN.yield_math(x, ws, bs)
        assert np.max(np.abs(a[:, None] - b)) < 1e-10 * max(1.0, np.max(np.abs(b)))
