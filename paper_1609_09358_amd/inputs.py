"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module draws random numbers and nothing else: uniform information bits,
unit-variance Gaussian noise samples and per-frame Eb/N0 values.  It contains
none of the decoder's arithmetic (no encoding, no channel model, no CRC), so
the CPU oracle and the GPU library can both be fed from it without sharing
any code.  Every draw comes from numpy's Philox-4x32 counter generator keyed by
(seed, stream), so each stream is reproducible on its own.
"""
import numpy as np

# stream identifiers, so that bits, noise and SNR draws never overlap
_STREAM_BITS = 1
_STREAM_NOISE = 2
_STREAM_SNR = 3


def _gen(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[int(seed) & 0xFFFFFFFFFFFFFFFF, stream]))


def info_bits(B: int, K: int, seed: int) -> np.ndarray:
    """Uniform i.i.d. information bits, uint8 0/1, shape [B][K]."""
    return _gen(seed, _STREAM_BITS).integers(0, 2, size=(B, K), dtype=np.uint8)


def noise(B: int, N: int, seed: int, dtype=np.float64) -> np.ndarray:
    """Unit-variance Gaussian samples, shape [B][N]."""
    return _gen(seed, _STREAM_NOISE).standard_normal(size=(B, N)).astype(dtype, copy=False)


def ebn0_uniform(B: int, lo_db: float, hi_db: float, seed: int) -> np.ndarray:
    """Per-frame Eb/N0 in dB, uniform on [lo_db, hi_db]."""
    return _gen(seed, _STREAM_SNR).uniform(lo_db, hi_db, size=B)


def choice(B: int, options, seed: int, stream: int = 4) -> np.ndarray:
    """B indices drawn uniformly from range(len(options))."""
    return _gen(seed, stream).integers(0, len(options), size=B)
