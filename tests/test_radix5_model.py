"""Exact model of the index algebra of the transform lengths N = 5 * 2^m.

A product of two L-limb numbers (2L - 1 <= N = 5M, M = 2^m) is computed as
one radix-5 decimation-in-frequency step over five length-M transforms, each
a four-step transform of N1 = 2^m1 rows by N2 = 2^m2 columns.  Because
L <= 5M/2, the inputs x_(n+3M) and x_(n+4M) are padding and x_(n+2M) is
nonzero only for n < M/2 (the lower half of the column-pass rows).  The
library picks omega_N = w^(5^-1 mod 2^m) * c (w the power-of-two root of its
host code, c the first h^((p-1)/5) != 1), applies the row part of the
radix-5 twiddle where the column pass unpacks the limbs, as three tables
g_n0[r] = omega_N^(k0 (r N2 + n0 M)), n0 = 0, 1, 2 (the row part of
omega_N^(k0 n) times omega_5^(k0 n0)), the column part omega_N^(k0 c) inside
the four-step table of the row pass (exponent (5 bitrev(r') + k0) c for
stored row r' of transform k0), and undoes the radix-5 step in the
reconstruction kernel: u_k0 = s_k0 omega_N^(-k0 r N2), then
x_(j1 + n0 M) = sum_k0 u_k0 omega_5^(-k0 n0).

This test runs those formulas with plain modular integers (no Montgomery
form, no lazy reduction; the transforms inside the columns and rows as direct
DFTs) for small shapes and each prime of the 5 * 2^m prime table, and checks
that (a) the forward values are the length-N DFT with root omega_N at index
5 (k1 + N1 k2) + k0, and (b) the whole forward-multiply-inverse sequence is
the cyclic convolution of the two limb sequences.  It also checks the prime
table against a direct search: the three largest primes below 2^30 with
5 * 2^m | p - 1.
"""
import os
import random
import re

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
INTERNAL = os.path.join(os.path.dirname(HERE), "paper_2105_13678_amd", "csrc", "pa_internal.hpp")


def primes_5():
    text = open(INTERNAL).read()
    body = re.search(r"PRIME_TRIPLES_5\[\]\s*=\s*\{(.*?)\};", text, flags=re.S).group(1)
    rows = re.findall(r"\{(\d+), \{(\d+)u, (\d+)u, (\d+)u\}\}", body)
    return [(int(r[0]), [int(x) for x in r[1:]]) for r in rows]


def is_prime(n):
    """Deterministic Miller-Rabin for n < 3.3 * 10^24."""
    if n < 2:
        return False
    for q in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % q == 0:
            return n == q
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
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


def root_of_unity(p, log2n):
    """As the library's host code: g^((p-1)/2^log2n) for the smallest
    quadratic non-residue g."""
    g = 2
    while pow(g, (p - 1) // 2, p) != p - 1:
        g += 1
    return pow(g, (p - 1) >> log2n, p)


def root_of_len5(p, log2n):
    """omega_N for N = 5 * 2^log2n: w^(5^-1 mod 2^log2n) * c, c the first
    h^((p-1)/5) != 1 (h = 2, 3, ...)."""
    w = root_of_unity(p, log2n)
    a = pow(5, -1, 1 << log2n) if log2n else 0
    h = 2
    while pow(h, (p - 1) // 5, p) == 1:
        h += 1
    return pow(w, a, p) * pow(h, (p - 1) // 5, p) % p


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
    assert all(v == 0 for v in x[2 * M + M // 2:]), "limbs past 5M/2 are padding"
    w1 = pow(wN, 5 * N2, p)  # omega_N1 (the column table's root: omega_N^(5 N2))
    w2 = pow(wN, 5 * N1, p)  # omega_N2
    out = []
    for k0 in range(5):
        cols = [[0] * N1 for _ in range(N2)]
        for c in range(N2):
            col = []
            for r in range(N1):
                n = r * N2 + c
                assert r < N1 // 2 or x[n + 2 * M] == 0, "x_(n+2M) reaches only the lower half of the rows"
                g = [pow(wN, k0 * (r * N2 + n0 * M), p) for n0 in range(3)]  # tables g0, g1, g2
                col.append((x[n] * g[0] + x[n + M] * g[1] + x[n + 2 * M] * g[2]) % p)
            f = dft(col, w1, p)
            for k1 in range(N1):
                cols[c][brev(k1, m1)] = f[k1]  # bit-reversed row order, as stored
        rows = []
        for rho in range(N1):
            g = 5 * brev(rho, m1) + k0  # four-step table exponent per column
            row = [cols[c][rho] * pow(wN, g * c, p) % p for c in range(N2)]
            rows.append(dft(row, w2, p))
        out.append(rows)
    return out


def inverse(T, p, m1, m2, wN):
    """Inverse rows (with the inverse four-step table and 1/N), inverse
    columns to natural order, then the inverse radix-5 step of the
    reconstruction kernel; returns the N coefficients."""
    N1, N2 = 1 << m1, 1 << m2
    M = N1 * N2
    N = 5 * M
    wi = pow(wN, -1, p)
    w1i = pow(wi, 5 * N2, p)
    w2i = pow(wi, 5 * N1, p)
    ninv = pow(N, -1, p)
    s = [[0] * M for _ in range(5)]
    for k0 in range(5):
        cols = [[0] * N1 for _ in range(N2)]
        for rho in range(N1):
            g = 5 * brev(rho, m1) + k0
            row = dft(T[k0][rho], w2i, p)
            for c in range(N2):
                cols[c][rho] = row[c] * ninv % p * pow(wi, g * c, p) % p
        for c in range(N2):
            nat = [cols[c][brev(k1, m1)] for k1 in range(N1)]
            col = dft(nat, w1i, p)
            for r in range(N1):
                s[k0][r * N2 + c] = col[r]
    w5i = pow(wi, M, p)  # omega_5^-1
    out = [0] * N
    for j1 in range(M):
        r = j1 >> m2
        u = [s[k0][j1] * pow(wi, k0 * r * N2, p) % p for k0 in range(5)]
        for n0 in range(5):
            out[j1 + n0 * M] = sum(u[k0] * pow(w5i, k0 * n0, p) for k0 in range(5)) % p
    return out


SHAPES = [(1, 1), (2, 1), (1, 3), (3, 2), (2, 3)]


@pytest.mark.parametrize("m1,m2", SHAPES)
def test_radix5_index_algebra(m1, m2):
    rng = random.Random(m1 * 16 + m2 + 5)
    triples = primes_5()
    for max_lg, ps in (triples[0], triples[-1]):
        for p in ps:
            m = m1 + m2
            assert (p - 1) % (5 << max_lg) == 0 and m <= max_lg
            M = 1 << m
            N = 5 * M
            wN = root_of_len5(p, m)
            assert pow(wN, 5, p) == root_of_unity(p, m), "omega_N^5 is the power-of-two root"
            assert pow(wN, N, p) == 1 and pow(wN, N // 2, p) != 1 and pow(wN, N // 5, p) != 1
            L = (N + 1) // 2  # the longest limb sequences whose product fits
            xa = [rng.randrange(p) for _ in range(L)] + [0] * (N - L)
            xb = [rng.randrange(p) for _ in range(L)] + [0] * (N - L)
            Ta = forward(xa, p, m1, m2, wN)
            Tb = forward(xb, p, m1, m2, wN)
            X = dft(xa, wN, p)
            N1 = 1 << m1
            for k0 in range(5):
                for rho in range(N1):
                    k1 = brev(rho, m1)
                    for k2 in range(1 << m2):
                        assert Ta[k0][rho][k2] == X[5 * (k1 + N1 * k2) + k0], (p, m1, m2, k0, k1, k2)
            prod = [[[Ta[k0][r][c] * Tb[k0][r][c] % p for c in range(1 << m2)] for r in range(N1)]
                    for k0 in range(5)]
            got = inverse(prod, p, m1, m2, wN)
            want = [0] * N
            for i, u in enumerate(xa):
                if u:
                    for j, v in enumerate(xb):
                        want[(i + j) % N] = (want[(i + j) % N] + u * v) % p
            assert got == want, (p, m1, m2)


def test_prime_table_is_the_largest_triple_per_length():
    """Each row of the 5 * 2^m prime table holds, in decreasing order, the
    three largest primes below 2^30 with 5 * 2^m | p - 1."""
    for max_lg, ps in primes_5():
        step = 5 << max_lg
        found = []
        c = ((1 << 30) - 2) // step
        while len(found) < 3:
            if is_prime(c * step + 1):
                found.append(c * step + 1)
            c -= 1
        assert ps == found, (max_lg, ps, found)
