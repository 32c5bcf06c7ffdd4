"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds random-number draws and array shaping only: no transform
arithmetic.  Every generator uses numpy's PCG64 (``default_rng(seed)``), draws
in float64 and rounds once to float32, which is what the GPU consumes; the
oracle later widens those float32 values back to float64 exactly.  The FP64
path takes the float64 draws as they are (``dtype=np.float64``).

The five workloads (sizes, distributions and seeds):
  c1  N=1024, batch 16, split, re/im ~ U[-1, 1), seed 1
  c2  N=4096, batch 8192, re/im ~ N(0, 1), seed 2 (used in both layouts)
  c3  N=2^24, batch 1, split, N(0, 1) plus 8 cosines at distinct seeded
      integer frequencies in [1, N/2 - 1], seed 3
  c4  4096 transforms of size 2^k, k ~ U{6..16}, re/im ~ U[-1, 1), seed 4,
      packed back to back in draw order
  c5  batch 1024, N=4096, split, x ~ N(0, 1), weights w ~ U[0, 1), seed 5
"""
from __future__ import annotations

import numpy as np

SEEDS = {"c1": 1, "c2": 2, "c3": 3, "c4": 4, "c5": 5}


def uniform_complex(shape, seed: int, dtype=np.float32) -> tuple[np.ndarray, np.ndarray]:
    """(re, im) arrays (float32 unless dtype says otherwise) with entries i.i.d. U[-1, 1)."""
    rng = np.random.default_rng(seed)
    re = rng.uniform(-1.0, 1.0, size=shape).astype(dtype)
    im = rng.uniform(-1.0, 1.0, size=shape).astype(dtype)
    return re, im


def normal_complex(shape, seed: int, dtype=np.float32) -> tuple[np.ndarray, np.ndarray]:
    """(re, im) arrays (float32 unless dtype says otherwise) with entries i.i.d. N(0, 1)."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(size=shape).astype(dtype)
    im = rng.standard_normal(size=shape).astype(dtype)
    return re, im


def c1(seed: int = SEEDS["c1"]):
    """N=1024, batch 16, split layout, U[-1, 1)."""
    return uniform_complex((16, 1024), seed)


def c2(seed: int = SEEDS["c2"], batch: int = 8192, n: int = 4096):
    """N=4096, batch 8192, N(0, 1).  Smaller batches draw a prefix of other seeds' streams."""
    return normal_complex((batch, n), seed)


def c3_frequencies(n: int, seed: int = SEEDS["c3"], count: int = 8) -> np.ndarray:
    """Distinct integer frequencies in [1, n/2 - 1], drawn from the seed."""
    rng = np.random.default_rng(seed + 1000)
    hi = max(n // 2 - 1, 1)
    if hi < count:
        raise ValueError("too few frequencies available")
    return np.sort(rng.choice(np.arange(1, hi + 1), size=count, replace=False))


def c3(n: int = 1 << 24, seed: int = SEEDS["c3"]):
    """N(0, 1) noise plus 8 unit cosines; returns (re, im, noise_re, noise_im, freqs).

    The cosines are built in float64 from the exactly reduced phase (f*j mod n),
    summed with the noise, then the whole signal is rounded to float32 once.
    """
    rng = np.random.default_rng(seed)
    nr = rng.standard_normal(n)
    ni = rng.standard_normal(n)
    freqs = c3_frequencies(n, seed)
    j = np.arange(n, dtype=np.int64)
    tones = np.zeros(n)
    for f in freqs:
        tones += np.cos(2.0 * np.pi * ((int(f) * j) % n) / n)
    re = (nr + tones).astype(np.float32)
    im = ni.astype(np.float32)
    return re, im, nr, ni, freqs


def c4_sizes(count: int = 4096, seed: int = SEEDS["c4"], kmin: int = 6, kmax: int = 16) -> np.ndarray:
    """Transform sizes 2^k with k uniform on {kmin..kmax}, in draw order."""
    rng = np.random.default_rng(seed)
    k = rng.integers(kmin, kmax + 1, size=count)
    return (np.int64(1) << k.astype(np.int64))


def c4(count: int = 4096, seed: int = SEEDS["c4"], kmin: int = 6, kmax: int = 16):
    """Ragged batch: (sizes, offsets, re, im) with transforms packed in draw order."""
    sizes = c4_sizes(count, seed, kmin, kmax)
    offsets = np.zeros(count, dtype=np.int64)
    if count > 1:
        offsets[1:] = np.cumsum(sizes)[:-1]
    total = int(sizes.sum())
    re, im = uniform_complex((total,), seed + 1)
    return sizes, offsets, re, im


def c5(seed: int = SEEDS["c5"], batch: int = 1024, n: int = 4096):
    """(re, im, w): x ~ N(0, 1) split, weights ~ U[0, 1) of shape (batch, n)."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(size=(batch, n)).astype(np.float32)
    im = rng.standard_normal(size=(batch, n)).astype(np.float32)
    w = rng.uniform(0.0, 1.0, size=(batch, n)).astype(np.float32)
    return re, im, w


def interleave(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    """complex64 (complex128) array from float32 (float64) parts (layout change only)."""
    out = np.empty(re.shape, dtype=np.complex128 if re.dtype == np.float64 else np.complex64)
    out.real = re
    out.imag = im
    return out
