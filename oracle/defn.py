"""Python arbitrary-precision definition of the MMH-MH hash.

TEST INFRASTRUCTURE ONLY: the product path never imports this package.

Each function follows a passage of the paper (Yan, Li, Mao, Chen, "An
efficient hybrid hash based privacy amplification algorithm for quantum key
distribution", arXiv 2105.13678):

* MMH, Sec. 2.1 eq. (2): g_a(x) = sum_i a_i x_i mod p over Z_p^k.
* MH,  Sec. 2.2 eq. (4): h_{b,c}(x) = ((b x + c) mod 2^alpha) div 2^(alpha-beta),
  b odd.
* The combination, Algorithm 1 (REQUIRE/ENSURE lines, split, reload test, MMH
  sum, MH step), with p = M_gamma = 2^gamma - 1 and seeds b, c in Z_{2^gamma}.
* Parameter choice, Sec. 4 and Table 3: n = gamma * k, gamma > beta.

Readings where the paper is silent or ambiguous (each is also listed with the
design notes):
* gamma is the smallest Mersenne exponent strictly greater than r, unless the
  caller names one; k = ceil(n / gamma); the key is zero-padded to k*gamma bits.
* bit t of chunk x_i is key bit i*gamma + t (little-endian), likewise for the
  seeds and the output (output bit t is bit gamma - r + t of U).
* alpha in the MH step is gamma (b, c are gamma-bit numbers in Algorithm 1).
* a chunk equal to 2^gamma - 1 makes the block RELOAD: no output.
* a seed word with bits >= gamma set is an error (SEED_RANGE); an even b is an
  error (SEED_B_EVEN).  Precedence: SEED_RANGE, then SEED_B_EVEN, then RELOAD.
"""
from __future__ import annotations

# Exponents e for which 2^e - 1 is a known Mersenne prime, in increasing order.
# The paper points to the public list of Mersenne primes for this (Sec. 3.1).
MERSENNE_EXPONENTS = (
    2, 3, 5, 7, 13, 17, 19, 31, 61, 89, 107, 127, 521, 607, 1279, 2203, 2281,
    3217, 4253, 4423, 9689, 9941, 11213, 19937, 21701, 23209, 44497, 86243,
    110503, 132049, 216091, 756839, 859433, 1257787, 1398269, 2976221, 3021377,
    6972593, 13466917, 20996011, 24036583, 25964951, 30402457, 32582657,
    37156667, 42643801, 43112609, 57885161, 74207281, 77232917, 82589933,
    136279841,
)

OK, RELOAD = 0, 2
ERR_ARG, ERR_NO_GAMMA, ERR_GAMMA = -1, -2, -3
ERR_SEED_B_EVEN, ERR_SEED_RANGE = -5, -6


def plan_shape(n: int, r: int, gamma: int | None = None):
    """(status, gamma, k) by the parameter rule (Sec. 4, Table 3, Alg. 1)."""
    if n < 2 or r < 1 or r >= n:
        return ERR_ARG, 0, 0
    if gamma is None or gamma == 0:
        cands = [e for e in MERSENNE_EXPONENTS if e > r]
        if not cands:
            return ERR_NO_GAMMA, 0, 0
        gamma = cands[0]
    elif gamma not in MERSENNE_EXPONENTS or gamma <= r:
        return ERR_GAMMA, 0, 0
    k = -(-n // gamma)
    return OK, gamma, k


def words_to_int(words) -> int:
    """Little-endian uint64 words to a Python int."""
    return int.from_bytes(bytes(memoryview(_as_u64(words)).cast("B")), "little")


def int_to_words(v: int, nwords: int):
    import numpy as np
    return np.frombuffer(v.to_bytes(8 * nwords, "little"), dtype=np.uint64).copy()


def _as_u64(words):
    import numpy as np
    return np.ascontiguousarray(np.asarray(words, dtype=np.uint64))


def mod_mersenne(v: int, gamma: int) -> int:
    """v mod (2^gamma - 1) for v >= 0 by the identity of Sec. 3.1:
    x mod M_gamma = floor(x / 2^gamma) + x mod 2^gamma (a congruence), applied
    until the value is below 2^gamma, then 2^gamma - 1 itself maps to 0.
    Equal to Python's ``v % (2**gamma - 1)`` (checked in the pins), but linear
    time where CPython's long division is quadratic."""
    p = (1 << gamma) - 1
    while v >> gamma:
        v = (v & p) + (v >> gamma)
    return 0 if v == p else v


def mmh(a: list[int], x: list[int], p: int) -> int:
    """Sec. 2.1 eq. (2): sum_i a_i x_i mod p, with p = 2^gamma - 1."""
    gamma = p.bit_length()
    assert p == (1 << gamma) - 1
    return mod_mersenne(sum(ai * xi for ai, xi in zip(a, x)), gamma)


def mh(y: int, b: int, c: int, alpha: int, beta: int) -> int:
    """Sec. 2.2 eq. (4): ((b y + c) mod 2^alpha) div 2^(alpha - beta)."""
    return ((b * y + c) & ((1 << alpha) - 1)) >> (alpha - beta)


def split_key(K: int, n: int, gamma: int, k: int) -> list[int]:
    """Algorithm 1, split step: chunk i is key bits [i*gamma, (i+1)*gamma)."""
    K &= (1 << n) - 1
    mask = (1 << gamma) - 1
    return [(K >> (i * gamma)) & mask for i in range(k)]


def hash_ints(K: int, n: int, r: int, gamma: int, a: list[int], b: int, c: int):
    """Algorithm 1 on Python ints.  Returns (status, z, y, U)."""
    k = len(a)
    p = (1 << gamma) - 1
    if any(ai >> gamma for ai in a) or (b >> gamma) or (c >> gamma):
        return ERR_SEED_RANGE, None, None, None
    if b % 2 == 0:
        return ERR_SEED_B_EVEN, None, None, None
    x = split_key(K, n, gamma, k)
    if any(xi == p for xi in x):
        return RELOAD, None, None, None
    y = mmh(a, x, p)
    U = (b * y + c) & ((1 << gamma) - 1)
    z = mh(y, b, c, gamma, r)
    return OK, z, y, U


def hash_words(key, n: int, r: int, gamma: int, a_words, b_words, c_words):
    """Same as hash_ints, on the word layouts of the library's interface:
    key = ceil(n/64) words, a = k chunks of W = ceil(gamma/64) words, b and c
    W words each.  Returns (status, z, y, U) with Python ints."""
    import numpy as np
    W = (gamma + 63) // 64
    a_words = _as_u64(a_words)
    k = len(a_words) // W
    a = [words_to_int(a_words[i * W:(i + 1) * W]) for i in range(k)]
    K = words_to_int(key)
    return hash_ints(K, n, r, gamma, a, words_to_int(b_words), words_to_int(c_words))
