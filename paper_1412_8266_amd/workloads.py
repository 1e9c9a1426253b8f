"""Seeded synthetic inputs of the MRG32k3a workloads.

Shared by the tests, the benchmark and the CPU oracle runs; it holds no
generator arithmetic -- only the shapes, seeds and input draws:

* C1: 64 streams spaced 2^127 apart from the seed (12345 x 6), 16384 outputs
  per stream as uint32, and the same again as FP64;
* C2: plain bulk fill, 2^20 streams (one per GPU lane), 4096 outputs each, as
  uint32 and as FP32, base state from a 64-bit master seed;
* C3: 2^16 streams, each jumped by a random offset drawn uniformly in
  [0, 2^64) plus one substream (2^76), then 1024 outputs;
* C4: a batch of 10,000 requests, stream counts and per-stream lengths
  log-uniform in [1, 4096] and [1, 2^20], dtypes uniform over u32/f32/f64;
* C5: Poisson arrivals at 20k requests/s for 60 s over 50,000 clients, sizes
  as C4, output admission capped at 64 GiB.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

C1_SEED = (12345, 12345, 12345, 12345, 12345, 12345)
C1_STREAMS = 64
C1_N = 16384

MASTER_SEED = 0x0123456789ABCDEF
C2_STREAMS = 1 << 20
C2_N = 4096

C3_STREAMS = 1 << 16
C3_N = 1024
C3_OFFSET_SEED = 3

C4_REQUESTS = 10_000
C4_MAX_STREAMS = 4096
C4_MAX_LEN = 1 << 20
C4_SEED = 4

C5_RATE = 20_000.0
C5_DURATION = 60.0
C5_CLIENTS = 50_000
C5_ARENA_BYTES = 64 << 30
C5_SEED = 5


def c3_offsets(n: int = C3_STREAMS, seed: int = C3_OFFSET_SEED) -> np.ndarray:
    """Per-stream offsets, uniform in [0, 2^64)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << 64, size=n, dtype=np.uint64, endpoint=False)


def c3_exponents(offsets: np.ndarray) -> np.ndarray:
    """[n, 3] little-endian 64-bit words of offset + 1 * 2^76 (word 1, bit 12)."""
    e = np.zeros((offsets.shape[0], 3), dtype=np.uint64)
    e[:, 0] = offsets
    e[:, 1] = np.uint64(1 << 12)
    return e


def random_exponents(n: int, bits: int, seed: int) -> np.ndarray:
    """[n, 3] words of exponents uniform in [0, 2^bits), bits <= 192."""
    rng = np.random.default_rng(seed)
    w = rng.integers(0, 1 << 64, size=(n, 3), dtype=np.uint64, endpoint=False)
    for i in range(3):
        lo = 64 * i
        if bits <= lo:
            w[:, i] = 0
        elif bits < lo + 64:
            w[:, i] &= np.uint64((1 << (bits - lo)) - 1)
    return w


def words_to_int(words) -> int:
    return int(words[0]) | (int(words[1]) << 64) | (int(words[2]) << 128)


def log_uniform_int(rng: np.random.Generator, hi: int, size: int) -> np.ndarray:
    """Integers in [1, hi], floor(exp(U * ln(hi + 1))) with U ~ U[0, 1)."""
    u = rng.random(size)
    v = np.floor(np.exp(u * math.log(hi + 1))).astype(np.int64)
    return np.clip(v, 1, hi)


@dataclass
class Requests:
    n_streams: np.ndarray   # int64 [R]
    length: np.ndarray      # int64 [R], outputs per stream
    dtype: np.ndarray       # int32 [R], 0 u32 / 1 f32 / 2 f64
    first_stream: np.ndarray  # int64 [R], global stream index of each request

    def __len__(self):
        return int(self.n_streams.shape[0])

    def samples(self) -> np.ndarray:
        return self.n_streams * self.length

    def bytes(self) -> np.ndarray:
        return self.samples() * np.where(self.dtype == 2, 8, 4)


def c4_requests(n: int = C4_REQUESTS, max_streams: int = C4_MAX_STREAMS,
                max_len: int = C4_MAX_LEN, seed: int = C4_SEED) -> Requests:
    """Requests over contiguous global streams from the master seed."""
    rng = np.random.default_rng(seed)
    k = log_uniform_int(rng, max_streams, n)
    L = log_uniform_int(rng, max_len, n)
    dt = rng.integers(0, 3, size=n).astype(np.int32)
    first = np.concatenate([[0], np.cumsum(k)[:-1]]).astype(np.int64)
    return Requests(k, L, dt, first)


@dataclass
class Arrivals:
    t: np.ndarray        # float64 [R] arrival times in seconds
    client: np.ndarray   # int64 [R]
    req: Requests


def c5_arrivals(rate: float = C5_RATE, duration: float = C5_DURATION,
                clients: int = C5_CLIENTS, max_streams: int = C4_MAX_STREAMS,
                max_len: int = C4_MAX_LEN, seed: int = C5_SEED) -> Arrivals:
    rng = np.random.default_rng(seed)
    n_expected = int(rate * duration * 1.2) + 16
    gaps = rng.exponential(1.0 / rate, size=n_expected)
    t = np.cumsum(gaps)
    t = t[t < duration]
    n = t.shape[0]
    client = rng.integers(0, clients, size=n).astype(np.int64)
    k = log_uniform_int(rng, max_streams, n)
    L = log_uniform_int(rng, max_len, n)
    dt = rng.integers(0, 3, size=n).astype(np.int32)
    return Arrivals(t, client, Requests(k, L, dt, np.zeros(n, dtype=np.int64)))
