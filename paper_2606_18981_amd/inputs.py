"""Seeded synthetic input generators (shared by tests, smoke and bench).

This module holds no arithmetic of the transform itself: it only draws input
arrays and request traces.  Both the GPU library and the oracle are fed from
here.

Two kinds of generators:
  * numpy ``default_rng(seed)`` generators for host-side inputs that are
    copied to the device (uniform, Gaussian, delta, tone, multi-tone);
  * a host implementation of the counter-based Philox-4x32-10 generator
    (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2,
    3", SC 2011) with the same amplitude mapping as the device generator in
    the library, so that device-generated inputs can be reproduced on the host
    without copying them back.

The tone and multi-tone inputs follow the paper's correctness inputs
(Sec. 4 experimental setup: a single complex exponential at a known bin).
"""

from __future__ import annotations

import math

import numpy as np

# ---------------------------------------------------------------------------
# numpy-based inputs
# ---------------------------------------------------------------------------


def uniform_pm1(n: int, seed: int) -> np.ndarray:
    """re, im i.i.d. uniform[-1, 1], complex128, length 2^n."""
    rng = np.random.default_rng(seed)
    N = 1 << n
    re = rng.uniform(-1.0, 1.0, N)
    im = rng.uniform(-1.0, 1.0, N)
    return re + 1j * im


def gaussian(n: int, seed: int, unit_norm: bool = False) -> np.ndarray:
    """re, im i.i.d. N(0, 1); optionally scaled to unit L2 norm."""
    rng = np.random.default_rng(seed)
    N = 1 << n
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    if unit_norm:
        x /= np.linalg.norm(x)
    return x


def delta(n: int, j: int = 0) -> np.ndarray:
    """Unit impulse at index j."""
    x = np.zeros(1 << n, dtype=np.complex128)
    x[j] = 1.0
    return x


def tone(n: int, k0: int) -> np.ndarray:
    """x_j = exp(+2 pi i k0 j / N): a unit-modulus tone at bin k0.

    The angle index (k0 j) mod N is reduced in integers first.
    """
    N = 1 << n
    j = np.arange(N, dtype=np.int64)
    m = (j * k0) % N
    return np.exp(2j * np.pi * m.astype(np.float64) / N)


def multi_tone(n: int, seed: int, count: int = 8, noise_var: float = 0.01):
    """Sum of ``count`` tones at seeded distinct bins plus complex noise.

    Amplitudes A ~ U[0.5, 2], phases phi ~ U[0, 2 pi), bins drawn without
    replacement from [0, N); noise re, im ~ N(0, noise_var) (variance, so
    sigma = sqrt(noise_var)).  Returns (x, bins, amplitudes, phases).
    """
    rng = np.random.default_rng(seed)
    N = 1 << n
    bins = rng.choice(N, size=count, replace=False)
    amp = rng.uniform(0.5, 2.0, count)
    ph = rng.uniform(0.0, 2.0 * np.pi, count)
    j = np.arange(N, dtype=np.int64)
    x = np.zeros(N, dtype=np.complex128)
    for b, a, p in zip(bins.tolist(), amp.tolist(), ph.tolist()):
        m = (j * b) % N
        x += a * np.exp(1j * p) * np.exp(2j * np.pi * m.astype(np.float64) / N)
    s = math.sqrt(noise_var)
    x += s * rng.standard_normal(N) + 1j * s * rng.standard_normal(N)
    return x, bins, amp, ph


# ---------------------------------------------------------------------------
# Philox-4x32-10 (host implementation from the published definition)
# ---------------------------------------------------------------------------

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
_U32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox-4x32 with 10 rounds.

    ctr: uint32 array of shape (4, M); key: two uint32 words.
    One round: (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 (64-bit products),
    c' = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key is bumped by the
    Weyl constants (W0, W1) between rounds.
    """
    c = [np.asarray(ctr[i], dtype=np.uint64) & _U32 for i in range(4)]
    k0 = int(key[0]) & 0xFFFFFFFF
    k1 = int(key[1]) & 0xFFFFFFFF
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    for r in range(10):
        if r > 0:
            k0 = (k0 + PHILOX_W0) & 0xFFFFFFFF
            k1 = (k1 + PHILOX_W1) & 0xFFFFFFFF
        p0 = m0 * c[0]
        p1 = m1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _U32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _U32
        c = [hi1 ^ c[1] ^ np.uint64(k0), lo1, hi0 ^ c[3] ^ np.uint64(k1), lo0]
    return np.stack([x.astype(np.uint32) for x in c])


def _philox_words(n: int, seed: int, stream: int, start: int = 0, count=None):
    N = 1 << n
    if count is None:
        count = N - start
    i = np.arange(start, start + count, dtype=np.uint64)
    ctr = np.stack([
        i & _U32,
        i >> np.uint64(32),
        np.full(count, stream & 0xFFFFFFFF, dtype=np.uint64),
        np.full(count, (stream >> 32) & 0xFFFFFFFF, dtype=np.uint64),
    ])
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    return philox4x32_10(ctr, key)


def _u53(lo, hi):
    a = (hi.astype(np.uint64) << np.uint64(32)) | lo.astype(np.uint64)
    return (a >> np.uint64(11)).astype(np.float64)


def philox_gaussian(n: int, seed: int, stream: int = 0, start: int = 0, count=None):
    """Amplitude i gets Box-Muller normals from Philox(ctr=(i, stream), key=seed).

    u1 = (w0w1 >> 11 + 1/2) 2^-53, u2 = (w2w3 >> 11 + 1/2) 2^-53,
    re = sqrt(-2 ln u1) cos(2 pi u2), im = sqrt(-2 ln u1) sin(2 pi u2).
    """
    w = _philox_words(n, seed, stream, start, count)
    u1 = (_u53(w[0], w[1]) + 0.5) * 2.0 ** -53
    u2 = (_u53(w[2], w[3]) + 0.5) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u1))
    th = 2.0 * np.pi * u2
    return r * np.cos(th) + 1j * r * np.sin(th)


def philox_uniform_pm1(n: int, seed: int, stream: int = 0, start: int = 0, count=None):
    """re = 2 u1 - 1, im = 2 u2 - 1 with u = (w >> 11) 2^-53 in [0, 1)."""
    w = _philox_words(n, seed, stream, start, count)
    u1 = _u53(w[0], w[1]) * 2.0 ** -53
    u2 = _u53(w[2], w[3]) * 2.0 ** -53
    return (2.0 * u1 - 1.0) + 1j * (2.0 * u2 - 1.0)


# ---------------------------------------------------------------------------
# workload shapes: batched uneven sizes and the served request stream
# ---------------------------------------------------------------------------


def batch_sizes(seed: int, count: int = 512, lo: int = 8, hi: int = 20,
                aqft_frac: float = 0.25, aqft_k: int = 8):
    """Sizes and cutoffs for the uneven batch.

    n = round(exp(U[ln lo, ln hi])) (log-uniform, integer, biased to small);
    a seeded permutation marks round(aqft_frac * count) entries AQFT with
    cutoff aqft_k, the rest exact (cutoff -1).
    """
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), count))).astype(np.int64)
    ns = np.clip(ns, lo, hi)
    cut = np.full(count, -1, dtype=np.int64)
    n_aqft = int(round(aqft_frac * count))
    cut[rng.permutation(count)[:n_aqft]] = aqft_k
    return ns, cut


def served_trace(seed: int, rate: float, duration: float, n_lo: int = 10, n_hi: int = 26,
                 aqft_frac: float = 0.3, k_lo: int = 6, k_hi: int = 16):
    """Poisson arrivals (exponential gaps) with per-request shape and seed.

    Returns a dict of equal-length arrays: arrival (s), n, dtype (0 = complex64,
    1 = complex128, 50/50), cutoff (-1 exact, else uniform in [k_lo, k_hi] for
    an aqft_frac share), seed (per-request input seed).
    """
    rng = np.random.default_rng(seed)
    expected = int(rate * duration * 1.2) + 16
    gaps = rng.exponential(1.0 / rate, expected)
    t = np.cumsum(gaps)
    while t[-1] < duration:
        more = rng.exponential(1.0 / rate, expected)
        t = np.concatenate([t, t[-1] + np.cumsum(more)])
    t = t[t < duration]
    m = t.size
    n = rng.integers(n_lo, n_hi + 1, m)
    dt = rng.integers(0, 2, m)
    is_aqft = rng.uniform(0.0, 1.0, m) < aqft_frac
    k = rng.integers(k_lo, k_hi + 1, m)
    cutoff = np.where(is_aqft, k, -1)
    seeds = rng.integers(1, 2 ** 62, m)
    return {"arrival": t, "n": n, "dtype": dt, "cutoff": cutoff, "seed": seeds}
