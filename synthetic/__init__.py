"""Seeded synthetic inputs shared by the tests, the benchmark, the oracle
side and the GPU side.

This module holds none of the method's arithmetic: only numpy random draws
with fixed seeds and the shapes of the paper's workloads (no dataset item
is reproduced; every input is synthetic). Randomness that the scheme
itself draws (secrets, errors, masks) is NOT here: both sides derive it
from a counter-based generator keyed by a seed.
"""
import numpy as np


def residues(seed, primes, n, count=1):
    """``count`` polynomials of ``len(primes)`` limbs each, residues uniform
    in [0, q_i): array [count][limbs][n] of uint64."""
    rng = np.random.default_rng(seed)
    out = np.empty((count, len(primes), n), dtype=np.uint64)
    for c in range(count):
        for i, q in enumerate(primes):
            out[c, i] = rng.integers(0, int(q), n, dtype=np.uint64)
    return out


def residues_device(seed, primes, n, count, device):
    """Same role as ``residues`` for large batches, drawn on the device with
    a seeded torch generator: tensor [count][limbs][n] int64 holding values
    uniform in [0, q_i)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    out = torch.empty(count, len(primes), n, dtype=torch.int64, device=device)
    for i, q in enumerate(primes):
        out[:, i] = torch.randint(0, int(q), (count, n), generator=g, device=device, dtype=torch.int64)
    return out


def ragged_limbs(batch, lo=4, hi=16):
    """Limb counts lo + (i mod (hi - lo + 1)) for a ragged batch."""
    span = hi - lo + 1
    return [lo + (i % span) for i in range(batch)]


def uniform_slots(seed, n, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, n)


def gaussian(seed, shape, sigma):
    return np.random.default_rng(seed).normal(0.0, sigma, shape)


# ---------------------------------------------------------------------------
# workload inputs (shapes of the paper's two networks, synthetic values)
# ---------------------------------------------------------------------------
def tiny_dense_inputs(seed_x=0, seed_w=1, n_samples=256, n_in=16, n_out=8, sigma=0.3):
    """Dense 16->8 on 256 samples (4096 slots = 16 features x 256 samples):
    x uniform[-1, 1], W ~ N(0, sigma^2), no bias."""
    x = np.random.default_rng(seed_x).uniform(-1.0, 1.0, (n_in, n_samples))
    w = np.random.default_rng(seed_w).normal(0.0, sigma, (n_out, n_in))
    return x, w


def vision_inputs(seed_x=0, seed_w=1, n_images=8192, side=28, filters=5, k=5, hidden=100,
                  classes=10, sigma=0.1):
    """Slot-batched vision net: images uniform[0,1]; conv filters k x k,
    dense (filters*13*13)->hidden->classes, weights and biases N(0, sigma^2)."""
    x = np.random.default_rng(seed_x).uniform(0.0, 1.0, (n_images, side, side))
    rng = np.random.default_rng(seed_w)
    out_side = (side + 1 - k) // 2 + 1  # 13 with one row/column of zero padding
    conv_w = rng.normal(0.0, sigma, (filters, k, k))
    conv_b = rng.normal(0.0, sigma, filters)
    n1 = filters * out_side * out_side
    w1 = rng.normal(0.0, sigma, (hidden, n1))
    b1 = rng.normal(0.0, sigma, hidden)
    w2 = rng.normal(0.0, sigma, (classes, hidden))
    b2 = rng.normal(0.0, sigma, classes)
    return x, dict(conv_w=conv_w, conv_b=conv_b, w1=w1, b1=b1, w2=w2, b2=b2)


def yield_inputs(seed_x=0, seed_w=1, n_windows=4096, days=7, features=21, sigma=0.1,
                 dims=(64, 16, 1)):
    """Time-series regressor: windows of days x features ~ N(0, 1), dense
    147->64->16->1 with weights and biases N(0, sigma^2)."""
    x = np.random.default_rng(seed_x).normal(0.0, 1.0, (n_windows, days * features))
    rng = np.random.default_rng(seed_w)
    ws, bs = [], []
    n_in = days * features
    for d in dims:
        ws.append(rng.normal(0.0, sigma, (d, n_in)))
        bs.append(rng.normal(0.0, sigma, d))
        n_in = d
    return x, ws, bs
