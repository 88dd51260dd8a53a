"""Seeded synthetic inputs for the MMH-MH privacy-amplification hash.

This module holds no part of the hash's arithmetic: it only draws words from a
counter-based generator and lays them out the way the hash expects its inputs.
The caller supplies the plan shape (gamma, k) for a block; choosing gamma and k
is the plan rule's job, not this module's.

Generator: splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014).  Word i of the stream seeded with s is
``mix(s + (i + 1) * 0x9E3779B97F4A7C15 mod 2^64)`` with the published mixer.

Input model: the paper's security model takes the reconciled key x uniformly at
random (Sec. 3.2.1), so key bits are i.i.d. Bernoulli(0.5); the hash seeds a, b,
c are uniform in their ranges (Algorithm 1, REQUIRE line), with b forced odd.

Draw order for one block (one stream):
  1. key words, ceil(n/64) of them, bits >= n in the last word cleared;
  2. a_0 .. a_{k-1}, W = ceil(gamma/64) words each, bits >= gamma cleared;
  3. b, W words, bits >= gamma cleared, then b |= 1;
  4. c, W words, bits >= gamma cleared.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


class SplitMix64:
    """splitmix64 stream; ``words(m)`` returns the next m outputs as uint64."""

    def __init__(self, seed: int):
        self.state = int(seed) & _MASK64

    def words(self, m: int) -> np.ndarray:
        m = int(m)
        if m == 0:
            return np.zeros(0, dtype=np.uint64)
        with np.errstate(over="ignore"):
            idx = np.arange(1, m + 1, dtype=np.uint64)
            z = np.uint64(self.state) + idx * GOLDEN
            out = _mix(z)
        self.state = (self.state + m * int(GOLDEN)) & _MASK64
        return out

    def next_u64(self) -> int:
        return int(self.words(1)[0])

    def next_double(self) -> float:
        """Uniform double in [0, 1): top 53 bits of the next word times 2^-53."""
        return (self.next_u64() >> 11) * (2.0 ** -53)


def mask_tail(words: np.ndarray, nbits: int) -> np.ndarray:
    """Clear bits >= nbits of a little-endian word array (in place)."""
    rem = nbits % 64
    if rem and len(words):
        words[-1] &= np.uint64((1 << rem) - 1)
    return words


@dataclass
class Block:
    n: int
    r: int
    gamma: int
    k: int
    key: np.ndarray  # ceil(n/64) uint64, little-endian bit order
    a: np.ndarray    # k * W uint64, chunk i at [i*W, (i+1)*W)
    b: np.ndarray    # W uint64, odd
    c: np.ndarray    # W uint64

    @property
    def W(self) -> int:
        return (self.gamma + 63) // 64


def draw_block(rng: SplitMix64, n: int, r: int, gamma: int, k: int) -> Block:
    """Draw one block's key and seeds from ``rng`` in the fixed draw order."""
    W = (gamma + 63) // 64
    key = mask_tail(rng.words((n + 63) // 64), n)
    a = rng.words(k * W)
    if k:
        a = a.reshape(k, W)
        rem = gamma % 64
        if rem:
            a[:, -1] &= np.uint64((1 << rem) - 1)
        a = a.reshape(-1)
    b = mask_tail(rng.words(W), gamma)
    b[0] |= np.uint64(1)
    c = mask_tail(rng.words(W), gamma)
    return Block(n=n, r=r, gamma=gamma, k=k, key=key, a=a, b=b, c=c)


def single_block(seed: int, n: int, r: int, gamma: int, k: int) -> Block:
    """One block from a fresh stream seeded with ``seed``."""
    return draw_block(SplitMix64(seed), n, r, gamma, k)


def uneven_blocks(seed: int, count: int, plan_shape, n_lo_log2: int = 22,
                  n_hi_log2: int = 28, f_lo: float = 0.05, f_hi: float = 0.30):
    """Blocks of uneven size: n log-uniform in [2^lo, 2^hi], r/n uniform in
    [f_lo, f_hi].  All (n, r) pairs are drawn first (two doubles per block),
    then each block's key and seeds in block order.  ``plan_shape(n, r)``
    returns (gamma, k)."""
    rng = SplitMix64(seed)
    shapes = []
    for _ in range(count):
        u = rng.next_double()
        v = rng.next_double()
        n = int(math.floor(2.0 ** (n_lo_log2 + (n_hi_log2 - n_lo_log2) * u)))
        r = int(math.floor((f_lo + (f_hi - f_lo) * v) * n))
        r = max(1, r)
        shapes.append((n, r))
    blocks = []
    for n, r in shapes:
        g, k = plan_shape(n, r)
        blocks.append(draw_block(rng, n, r, g, k))
    return blocks


def poisson_requests(seed: int, count: int, sessions: int, rate_per_s: float,
                     n_lo_log2: int = 24, n_hi_log2: int = 28, ratio: float = 0.1):
    """Arrival schedule for the serving workload: exponential inter-arrival
    times at the aggregate rate, a uniformly chosen session, n log-uniform in
    [2^lo, 2^hi] and r = floor(ratio * n).  Returns a list of
    (t_arrival_s, session, n, r); keys and seeds are drawn separately."""
    rng = SplitMix64(seed)
    t = 0.0
    out = []
    for _ in range(count):
        u = rng.next_double()
        t += -math.log(1.0 - u) / rate_per_s
        s = rng.next_u64() % sessions
        w = rng.next_double()
        n = int(math.floor(2.0 ** (n_lo_log2 + (n_hi_log2 - n_lo_log2) * w)))
        out.append((t, int(s), n, max(1, int(math.floor(ratio * n)))))
    return out
