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


def test_relu_approx_closed_forms():
    # R_a(0) = q/(3 pi), R_a(+-q) = 5q/(3 pi) +- q/2; its largest distance
    # to ReLU on [-q, q] is q/(3 pi), at 0
    for q in (1.0, 4.0, 10.0):
        c = PN.relu_approx_coeffs(q)
        assert len(c) == 3
        assert abs(PN.poly_eval(c, 0.0) - q / (3 * np.pi)) < 1e-12 * q
        assert abs(PN.poly_eval(c, q) - (5 * q / (3 * np.pi) + q / 2)) < 1e-12 * q
        assert abs(PN.poly_eval(c, -q) - (5 * q / (3 * np.pi) - q / 2)) < 1e-12 * q
        xs = np.linspace(-q, q, 20001)
        gap = np.abs(PN.poly_eval(c, xs) - np.maximum(xs, 0))
        assert abs(gap.max() - q / (3 * np.pi)) < 1e-9 * q and abs(xs[gap.argmax()]) < 1e-9 * q
        # the paper's derivative of the approximation: 8x/(3 pi q) + 1/2
        h = 1e-6 * q
        for x0 in (-0.7 * q, 0.0, 0.3 * q):
            num = (PN.poly_eval(c, x0 + h) - PN.poly_eval(c, x0 - h)) / (2 * h)
            assert abs(num - (8 * x0 / (3 * np.pi * q) + 0.5)) < 1e-6


def test_sigmoid_approx_closed_forms():
    c = PN.sigmoid_approx_coeffs()
    assert PN.poly_eval(c, 0.0) == 0.5
    assert abs(PN.poly_eval(c, 1.0) - 0.693) < 1e-15
    # odd around 1/2: sigma_a(x) + sigma_a(-x) = 1
    xs = np.linspace(-5, 5, 1001)
    assert np.max(np.abs(PN.poly_eval(c, xs) + PN.poly_eval(c, -xs) - 1.0)) < 1e-15
    # derivative 0.197 - 0.012 x^2 (the paper's approximate derivative)
    h = 1e-6
    for x0 in (-3.0, 0.5, 2.0):
        num = (PN.poly_eval(c, x0 + h) - PN.poly_eval(c, x0 - h)) / (2 * h)
        assert abs(num - (0.197 - 0.012 * x0 * x0)) < 1e-8
    # it follows the sigmoid on the stated range [-5, 5] to within 0.06
    # (largest gap 0.051 near |x| = 3.83)
    assert np.max(np.abs(PN.poly_eval(c, xs) - 1 / (1 + np.exp(-xs)))) < 0.06


def test_conv_slots_packed_equals_math():
    # the image-in-slots layout (masked kernels, rotations) reproduces the
    # strided cross-correlation + bias + square at every anchor
    x, P = S.vision_inputs(n_images=5)
    slots = 2048  # two images per ciphertext
    out = PN.conv_slots_packed(x, P, slots)
    got = PN.conv_slots_anchor_values(out, 5)
    assert np.max(np.abs(got - PN.vision_conv_square_math(x, P))) < 1e-12
    # the first two layers of the full network agree with it
    steps, masks, bias = PN.conv_slots_layout(P["conv_w"], P["conv_b"], slots)
    assert steps == [dy * 28 + dx for dy in range(5) for dx in range(5)]
    # no weighted tap reads outside its image (rotations never mix images)
    for t, st in enumerate(steps):
        for b in range(2):
            for p in np.nonzero(masks[0, t, b * 1024:(b + 1) * 1024])[0]:
                assert p + st < 784
