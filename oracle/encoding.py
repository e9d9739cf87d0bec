"""Oracle encode/decode: the CKKS canonical embedding in FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Definitions (paper Section 2.1: a sequence of values is encoded into one
polynomial and only the whole can be operated on; CKKS slots = N/2):
  zeta = exp(i pi / N), a primitive 2N-th root of unity;
  slot j (0 <= j < N/2) is the evaluation point zeta^(5^j mod 2N)
  (slot order by powers of 5), its conjugate point zeta^(-5^j) carries conj(z_j);
  encode(z, Delta) = round_half_away(Delta * sigma^-1(z)) where
  sigma^-1(z)_i = (1/N) sum_{k odd} v(zeta^k) zeta^(-i k) (the inverse canonical embedding);
  decode(m, Delta) = m(zeta^(5^j)) / Delta.
Both directions use numpy's length-2N FFT as the transform primitive: the
value vector V (V[k] = value at zeta^k, zero at even k) gives
sum_k V[k] zeta^(-ik) = fft(V)[i], and m(zeta^k) = 2N * ifft(m)[k].
The CRT lift is Python big-integer arithmetic, written as its definition.
"""
import numpy as np


def slot_positions(N):
    """k_j = 5^j mod 2N for j < N/2 (the evaluation exponent of slot j)."""
    two_n = 2 * N
    out = np.empty(N // 2, dtype=np.int64)
    x = 1
    for j in range(N // 2):
        out[j] = x
        x = (x * 5) % two_n
    return out


def round_half_away(x):
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


def encode(z, scale, N):
    """z: up to N/2 real or complex values (zero-padded). Returns int64
    coefficients, or raises when a coefficient reaches 2^62 (round half away from zero)."""
    z = np.asarray(z, dtype=np.complex128)
    if z.size > N // 2:
        raise ValueError("too many slots")
    zz = np.zeros(N // 2, dtype=np.complex128)
    zz[: z.size] = z
    V = np.zeros(2 * N, dtype=np.complex128)
    pos = slot_positions(N)
    V[pos] = zz
    V[(2 * N - pos) % (2 * N)] = np.conj(zz)
    m = np.real(np.fft.fft(V))[:N] / N
    r = round_half_away(m * scale)
    if np.any(np.abs(r) >= 2.0 ** 62):
        raise ValueError("coefficient out of range")
    return r.astype(np.int64)


def decode(m, scale, N, n_slots=None):
    """m: N real coefficients (float64 or ints). Returns complex slots."""
    m = np.asarray([float(x) for x in m], dtype=np.float64)
    pad = np.zeros(2 * N, dtype=np.float64)
    pad[:N] = m
    vals = np.fft.ifft(pad) * (2 * N)
    z = vals[slot_positions(N)] / scale
    return z if n_slots is None else z[:n_slots]


def crt_lift_centered(residues, primes):
    """Exact centered CRT lift: residues [L][N] mod primes[0..L-1] ->
    Python ints in (-Q/2, Q/2]."""
    L = len(residues)
    Q = 1
    for q in primes[:L]:
        Q *= q
    terms = []
    for i in range(L):
        qi = primes[i]
        qhat = Q // qi
        terms.append((qhat, pow(qhat % qi, -1, qi), qi))
    N = len(residues[0])
    out = []
    for j in range(N):
        x = 0
        for i, (qhat, qinv, qi) in enumerate(terms):
            x += (int(residues[i][j]) * qinv % qi) * qhat
        x %= Q
        if x > Q // 2:
            x -= Q
        out.append(x)
    return out


def decode_residues(residues, primes, scale, N, n_slots=None):
    """Decrypted coefficient-form residues -> slots."""
    return decode(crt_lift_centered(residues, primes), scale, N, n_slots)
