"""Exact model of the index algebra of the transform lengths N = 3 * 2^m.

A product of two L-limb numbers (2L - 1 <= N = 3M, M = 2^m) is computed as
one radix-3 decimation-in-frequency step over three length-M transforms,
each a four-step transform of N1 = 2^m1 rows by N2 = 2^m2 columns.  The
library picks omega_N = w^(3^-1 mod 2^m) * c (w the power-of-two root of its
host code, c a cube root of unity), applies the row part omega_N^(k0 r N2) of
the radix-3 twiddle where the column pass unpacks the limbs and the column
part omega_N^(k0 c) inside the four-step twiddle table of the row pass
(exponent (3 bitrev(r') + k0) c for stored row r' of transform k0), and
undoes the radix-3 step in the reconstruction kernel as
s0 + u1 + u2 and s0 - (u1 + u2)/2 +- h (u1 - u2), h = (omega_3^-1 - omega_3^-2)/2.

This test runs those formulas with plain modular integers (no Montgomery
form, no lazy reduction; the transforms inside the columns and rows as direct
DFTs) for small shapes and each prime of the 3 * 2^m prime table, and checks
that (a) the forward values are the length-N DFT with root omega_N at index
3 (k1 + N1 k2) + k0, and (b) the whole forward-multiply-inverse sequence is
the cyclic convolution of the two limb sequences.
"""
import os
import random
import re

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
INTERNAL = os.path.join(os.path.dirname(HERE), "paper_2105_13678_amd", "csrc", "pa_internal.hpp")


def primes_3():
    text = open(INTERNAL).read()
    body = re.search(r"PRIME_TRIPLES_3\[\]\s*=\s*\{(.*?)\};", text, flags=re.S).group(1)
    rows = re.findall(r"\{(\d+), \{(\d+)u, (\d+)u, (\d+)u\}\}", body)
    return [(int(r[0]), [int(x) for x in r[1:]]) for r in rows]


def root_of_unity(p, log2n):
    """As the library's host code: g^((p-1)/2^log2n) for the smallest
    quadratic non-residue g."""
    g = 2
    while pow(g, (p - 1) // 2, p) != p - 1:
        g += 1
    return pow(g, (p - 1) >> log2n, p)


def root_of_len3(p, log2n):
    """omega_N for N = 3 * 2^log2n: w^(3^-1 mod 2^log2n) * c, c the first
    h^((p-1)/3) != 1."""
    w = root_of_unity(p, log2n)
    a = pow(3, -1, 1 << log2n) if log2n else 0
    h = 2
    while pow(h, (p - 1) // 3, p) == 1:
        h += 1
    return pow(w, a, p) * pow(h, (p - 1) // 3, p) % p


def brev(x, bits):
    return int(format(x, f"0{bits}b")[::-1], 2) if bits else 0


def dft(v, root, p):
    n = len(v)
    return [sum(v[j] * pow(root, j * k, p) for j in range(n)) % p for k in range(n)]


def forward(x, p, m1, m2, wN):
    """Stored transform words: T[k0][rho][c2] for transform k0, stored row rho
    (column frequency k1 = bitrev(rho)) and row frequency k2 = c2 (rows kept
    in natural frequency order here)."""
    N1, N2 = 1 << m1, 1 << m2
    M = N1 * N2
    N = 3 * M
    assert all(v == 0 for v in x[2 * M:]), "limbs past 2M are padding"
    w1 = pow(wN, 3 * N2, p)  # omega_N1 (the column table's root: omega_N^(3 N2))
    w2 = pow(wN, 3 * N1, p)  # omega_N2
    out = []
    for k0 in range(3):
        cols = [[0] * N1 for _ in range(N2)]
        for c in range(N2):
            col = []
            for r in range(N1):
                n = r * N2 + c
                assert r < N1 // 2 or x[n + M] == 0, "x_(n+M) reaches only the upper half of the rows"
                g0 = pow(wN, k0 * r * N2, p)               # row part of the radix-3 twiddle
                g1 = pow(wN, k0 * (r * N2 + M), p)         # the same times omega_3^k0
                col.append((x[n] * g0 + x[n + M] * g1) % p)
            f = dft(col, w1, p)
            for k1 in range(N1):
                cols[c][brev(k1, m1)] = f[k1]              # bit-reversed row order, as stored
        rows = []
        for rho in range(N1):
            g = 3 * brev(rho, m1) + k0                      # four-step table exponent per column
            row = [cols[c][rho] * pow(wN, g * c, p) % p for c in range(N2)]
            rows.append(dft(row, w2, p))
        out.append(rows)
    return out


def inverse(T, p, m1, m2, wN):
    """Inverse rows (with the inverse four-step table and 1/N), inverse
    columns to natural order, then the inverse radix-3 step of the
    reconstruction kernel; returns the N coefficients."""
    N1, N2 = 1 << m1, 1 << m2
    M = N1 * N2
    N = 3 * M
    wi = pow(wN, -1, p)
    w1i = pow(wi, 3 * N2, p)
    w2i = pow(wi, 3 * N1, p)
    ninv = pow(N, -1, p)
    s = [[0] * M for _ in range(3)]
    for k0 in range(3):
        cols = [[0] * N1 for _ in range(N2)]
        for rho in range(N1):
            g = 3 * brev(rho, m1) + k0
            row = dft(T[k0][rho], w2i, p)
            for c in range(N2):
                cols[c][rho] = row[c] * ninv % p * pow(wi, g * c, p) % p
        for c in range(N2):
            nat = [cols[c][brev(k1, m1)] for k1 in range(N1)]
            col = dft(nat, w1i, p)
            for r in range(N1):
                s[k0][r * N2 + c] = col[r]
    w3 = pow(wN, M, p)                        # omega_3
    w3sq = w3 * w3 % p                        # omega_3^-1
    h = (w3sq - w3) * pow(2, -1, p) % p       # (omega_3^-1 - omega_3^-2) / 2
    neg_half = (p - 1) // 2                   # -1/2 mod p
    out = [0] * N
    for j1 in range(M):
        r = j1 >> m2
        u1 = s[1][j1] * pow(wi, 1 * r * N2, p) % p
        u2 = s[2][j1] * pow(wi, 2 * r * N2, p) % p
        a = (u1 + u2) * neg_half % p
        d = (u1 - u2) * h % p
        out[j1] = (s[0][j1] + u1 + u2) % p
        out[j1 + M] = (s[0][j1] + a + d) % p
        out[j1 + 2 * M] = (s[0][j1] + a - d) % p
    return out


SHAPES = [(1, 1), (2, 1), (1, 3), (3, 3), (2, 4), (4, 2)]


@pytest.mark.parametrize("m1,m2", SHAPES)
def test_radix3_index_algebra(m1, m2):
    rng = random.Random(m1 * 16 + m2)
    triples = primes_3()
    for max_lg, ps in (triples[0], triples[-1]):
        for p in ps:
            m = m1 + m2
            assert (p - 1) % (3 << max_lg) == 0 and m <= max_lg
            M = 1 << m
            N = 3 * M
            wN = root_of_len3(p, m)
            assert pow(wN, 3, p) == root_of_unity(p, m), "omega_N^3 is the power-of-two root"
            assert pow(wN, N, p) == 1 and pow(wN, N // 2, p) != 1 and pow(wN, N // 3, p) != 1
            L = (N + 1) // 2  # the longest limb sequences whose product fits
            xa = [rng.randrange(p) for _ in range(L)] + [0] * (N - L)
            xb = [rng.randrange(p) for _ in range(L)] + [0] * (N - L)
            Ta = forward(xa, p, m1, m2, wN)
            Tb = forward(xb, p, m1, m2, wN)
            X = dft(xa, wN, p)
            N1 = 1 << m1
            for k0 in range(3):
                for rho in range(N1):
                    k1 = brev(rho, m1)
                    for k2 in range(1 << m2):
                        assert Ta[k0][rho][k2] == X[3 * (k1 + N1 * k2) + k0], (p, m1, m2, k0, k1, k2)
            prod = [[[Ta[k0][r][c] * Tb[k0][r][c] % p for c in range(1 << m2)] for r in range(N1)]
                    for k0 in range(3)]
            got = inverse(prod, p, m1, m2, wN)
            want = [0] * N
            for i, u in enumerate(xa):
                if u:
                    for j, v in enumerate(xb):
                        want[(i + j) % N] = (want[(i + j) % N] + u * v) % p
            assert got == want, (p, m1, m2)


def _is_prime(n):
    """Deterministic Miller-Rabin for n < 3.4e14 (bases 2..17)."""
    if n < 2:
        return False
    for q in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % q == 0:
            return n == q
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17):
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def test_no_word_prime_has_power_of_two_roots_of_2():
    """The weighted (Crandall-Fagin) transform for products mod 2^gamma - 1
    needs, at length N = 2^m, an N-th root of 2 modulo each prime, i.e.
    2^((p-1)/2^m) = 1 mod p.  An exhaustive search over every prime
    p = c 2^m + 1 < 2^31 (c odd) with m >= 16 finds none, so no prime that
    fits the 32-bit lazy arithmetic can run weighted transforms of the
    lengths the hash needs (2^16 points and up); the 64-bit prime
    2^64 - 2^32 + 1 has them (2 has order 192 there)."""
    found, count = [], 0
    for m in range(16, 31):
        for c in range(1, 1 << (31 - m), 2):
            p = (c << m) | 1
            if not _is_prime(p):
                continue
            count += 1
            if pow(2, (p - 1) >> m, p) == 1:
                found.append((p, m))
    assert count > 3000 and found == []
    P = (1 << 64) - (1 << 32) + 1
    assert pow(2, 192, P) == 1 and pow(2, 96, P) != 1 and pow(2, 64, P) != 1
    assert pow(2, (P - 1) >> 26, P) == 1  # 2 is a 2^26-th power mod P
