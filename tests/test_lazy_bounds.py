"""Worst-case model of the lazy modular reduction in the transform kernels.

The kernels keep residues modulo three primes below 2^30 only partially
reduced (forward values in [0, 2p), inverse values in [0, 4p), Montgomery
products with R = 2^32 and no final subtraction, raw products pending in 64
bits).  Random keys cannot reach the worst cases, so this test models every
arithmetic primitive with exact 32/64-bit integer semantics and drives each
composition the kernels use with residues at the top of their ranges:

* interval bounds: every Montgomery product's inputs satisfy a*b < 2^32 p,
  every 32-bit sum stays below 2^32, every pending 64-bit sum below
  2^64 - 2^32 p, and each composition's outputs stay in the range its
  consumer assumes, for every prime of both prime tables;
* exact values: at the extreme inputs the modelled results lie in range and
  are congruent to the mathematical value (the DFT of the inputs, the
  pointwise products, the Chinese-remainder value).

Compositions modelled (each named after its kernel): the unpacking step of
the forward column pass (all three length forms), the radix-2/4/8/16 forward DFTs
with and without the zero-upper-half first stage and fused step twiddles,
the inverse DFTs with and without fused step twiddles, the row passes'
multiply-accumulate (64-bit pending products reduced once per three pairs in
the 4096-point row kernel; Montgomery products accumulated per pair in the
generic one, whose pair groups are then summed), the four-step twiddles on
load and store, the canonicalisation at the end of the inverse column pass,
the inverse radix-3 and radix-5 steps of the lengths 3 * 2^m and 5 * 2^m and
Garner's reconstruction.
"""
import os
import random
import re

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
INTERNAL = os.path.join(os.path.dirname(HERE), "paper_2105_13678_amd", "csrc", "pa_internal.hpp")

M32 = 1 << 32
M64 = 1 << 64


def table_primes():
    """Every prime of the library's prime tables (lengths 2^m, 3 * 2^m, 5 * 2^m)."""
    text = open(INTERNAL).read()
    primes = set()
    for body in re.findall(r"PRIME_TRIPLES(?:_3|_5)?\[\]\s*=\s*\{(.*?)\};", text, flags=re.S):
        primes.update(int(x) for x in re.findall(r"(\d+)u", body))
    assert len(primes) >= 10
    return sorted(primes)


class V:
    """A modelled register: exact value v and exclusive upper bound hi (the
    worst case over every input the call site can see)."""
    __slots__ = ("v", "hi")

    def __init__(self, v, hi):
        assert 0 <= v < hi, (v, hi)
        self.v, self.hi = v, hi


class Field:
    def __init__(self, p):
        self.p = p
        assert 4 * p < M32 and p < (1 << 30)
        self.p2 = 2 * p
        self.pinv = (-pow(p, -1, M32)) % M32  # -p^-1 mod 2^32
        self.rinv = pow(M32, -1, p)
        self.one = M32 % p
        g = 2
        while pow(g, (p - 1) // 2, p) != p - 1:
            g += 1
        w16 = pow(g, (p - 1) // 16, p)
        self.w16_plain = [pow(w16, j, p) for j in range(8)]
        self.w16i_plain = [pow(w16, (16 - j) % 16, p) for j in range(8)]
        self.w16 = [V(x * M32 % p, p) for x in self.w16_plain]   # Montgomery form, canonical
        self.w16i = [V(x * M32 % p, p) for x in self.w16i_plain]

    # ---- primitives, exact 32/64-bit semantics -------------------------------
    def mont(self, a, b):
        p = self.p
        assert (a.hi - 1) * (b.hi - 1) < M32 * p, "Montgomery input bound a*b < 2^32 p"
        t = a.v * b.v
        m = (t % M32) * self.pinv % M32
        assert t + m * p < M64
        r = (t + m * p) >> 32
        hi = ((a.hi - 1) * (b.hi - 1) + (M32 - 1) * p) // M32 + 1
        assert hi <= 2 * p and r < hi
        assert r % p == a.v * b.v * self.rinv % p
        return V(r, hi)

    def redc64(self, T):
        p = self.p
        assert T.hi - 1 < M64 - M32 * p, "pending sum bound"
        m = (T.v % M32) * self.pinv % M32
        r = (T.v + m * p) >> 32
        hi = (T.hi - 1 + (M32 - 1) * p) // M32 + 1
        assert r < hi and r % p == T.v * self.rinv % p
        return V(r, hi)

    def red2(self, x):  # min(x, x - 2p) as 32-bit unsigned
        assert x.hi <= 4 * self.p, "red2 input must be below 4p"
        r = min(x.v, (x.v - self.p2) % M32)
        assert r % self.p == x.v % self.p
        return V(r, min(x.hi, self.p2))

    def csub(self, x):  # min(x, x - p) as 32-bit unsigned, for x < 2p
        assert x.hi <= self.p2, "one conditional subtraction needs x < 2p"
        r = min(x.v, (x.v - self.p) % M32)
        assert r < self.p and r == x.v % self.p
        return V(r, self.p)

    def canon(self, x):
        assert x.hi <= self.p2, "canon input must be below 2p"
        r = min(x.v, (x.v - self.p) % M32)
        assert r < self.p and r == x.v % self.p
        return V(r, self.p)

    def add(self, a, b):
        hi = a.hi + b.hi - 1
        assert hi <= M32, "32-bit sum overflows"
        return V(a.v + b.v, hi)

    def sub2p(self, u, x):  # u + 2p - x, must neither wrap below 0 nor above 2^32
        assert x.hi - 1 <= self.p2, "difference operand above 2p"
        hi = u.hi + self.p2
        assert hi <= M32
        return V(u.v + self.p2 - x.v, hi)

    def mul64(self, a, b):
        return V(a.v * b.v, (a.hi - 1) * (b.hi - 1) + 1)

    def add64(self, a, b):
        hi = a.hi + b.hi - 1
        assert hi <= M64
        return V(a.v + b.v, hi)

    def mmul(self, a, b):
        return self.canon(self.mont(a, b))

    def msub(self, a, b):  # canonical a - b
        assert a.hi <= self.p and b.hi <= self.p
        d = (a.v - b.v) % M32
        r = min(d, (d + self.p) % M32)
        assert r == (a.v - b.v) % self.p
        return V(r, self.p)

    # ---- small DFTs, as the device's dft_fwd_x / dft_inv_x --------------------
    def dft_fwd(self, v, R, lowhalf=False, tw=None):
        v = list(v)
        H = R // 2
        if lowhalf:
            for j in range(H):
                v[j + H] = self.mont(v[j], self.w16[j * (8 // H)]) if j else v[j]
        h = H // 2 if lowhalf else H
        while h >= 1:
            for blk in range(0, R, 2 * h):
                for j in range(h):
                    u, x = v[blk + j], v[blk + j + h]
                    s = self.add(u, x)
                    d = self.sub2p(u, x)
                    if tw is not None and h == 1:
                        v[blk] = self.mont(s, tw[blk]) if blk else self.red2(s)
                        v[blk + 1] = self.mont(d, tw[blk + 1])
                    else:
                        v[blk + j] = self.red2(s)
                        v[blk + j + h] = self.mont(d, self.w16[j * (8 // h)]) if j else self.red2(d)
            h //= 2
        return v

    def dft_inv(self, v, R, tw=None):
        v = list(v)
        h = 1
        while h < R:
            for blk in range(0, R, 2 * h):
                for j in range(h):
                    if tw is not None and h == 1:
                        a = self.mont(v[blk], tw[blk]) if blk else self.red2(v[blk])
                        q = self.mont(v[blk + 1], tw[blk + 1])
                    else:
                        a = self.red2(v[blk + j])
                        q = self.mont(v[blk + j + h], self.w16i[j * (8 // h)]) if j else self.red2(v[blk + j + h])
                    v[blk + j] = self.add(a, q)
                    v[blk + j + h] = self.sub2p(a, q)
            h *= 2
        return v


def brev(s, bits):
    return int(format(s, f"0{bits}b")[::-1], 2) if bits else 0


def dft_ref(F, x, R, tw=None, inverse=False):
    """Direct R-point DFT mod p of plain values (forward: slot s holds
    frequency bitrev(s), times tw_s; inverse: bit-reversed slots in, each
    first times tw_s, natural order out, times R)."""
    p = F.p
    w = pow(F.w16_plain[1], 16 // R, p)
    if inverse:
        w = pow(w, p - 2, p)
    lg = R.bit_length() - 1
    if not inverse:
        out = []
        for s in range(R):
            k = brev(s, lg)
            val = sum(x[n] * pow(w, n * k, p) for n in range(R)) % p
            out.append(val * tw[s] % p if tw is not None and s else val)
        return out
    xs = [(x[s] * tw[s] % p if tw is not None and s else x[s] % p) for s in range(R)]
    return [sum(xs[s] * pow(w, n * brev(s, lg), p) for s in range(R)) % p for n in range(R)]


PRIMES = table_primes()


def extreme_inputs(F, hi, R, rng):
    """Input vectors at the corners of [0, hi): all maximal, alternating
    maximal and zero, all zero, one maximal, and random."""
    top = hi - 1
    yield [top] * R
    yield [top if j % 2 == 0 else 0 for j in range(R)]
    yield [0 if j % 2 == 0 else top for j in range(R)]
    yield [0] * R
    yield [top] + [0] * (R - 1)
    for _ in range(3):
        yield [rng.randrange(hi) for _ in range(R)]


def tw_values(F, R, rng):
    """Step twiddles: canonical Montgomery-form words, the largest first."""
    yield [V(F.p - 1, F.p) for _ in range(R)]
    yield [V(rng.randrange(F.p), F.p) for _ in range(R)]


@pytest.mark.parametrize("p", PRIMES)
def test_primitive_corners(p):
    F = Field(p)
    corners = [0, 1, p - 1, p, 2 * p - 1]
    for a in corners + [3 * p, 4 * p - 1]:
        for b in corners[:3]:
            F.mont(V(a, 4 * p), V(b, p))  # inverse-side operand with a canonical twiddle
    for a in corners:
        for b in corners:
            F.mont(V(a, 2 * p), V(b, 2 * p))  # two forward-side values (generic row product)
    for a in (0, 1, M32 - 1, (1 << 31) + 5):
        F.mont(V(a, M32), V(F.one, p))  # raw 32-bit limb into Montgomery form
        F.mont(V(a, M32), V(p - 1, p))  # Garner: a word times a canonical constant
    for x in (0, 2 * p - 1, 2 * p, 4 * p - 1):
        F.red2(V(x, 4 * p))
    for x in (0, p - 1, p, 2 * p - 1):
        F.canon(V(x, 2 * p))


@pytest.mark.parametrize("p", PRIMES)
def test_forward_dfts_stay_below_2p(p):
    F = Field(p)
    rng = random.Random(p)
    for R in (2, 4, 8, 16):
        for lowhalf in ((False, True) if R >= 4 else (False,)):
            for use_tw in (False, True):
                for tws in (tw_values(F, R, rng) if use_tw else [None]):
                    for xs in extreme_inputs(F, 2 * p, R, rng):
                        if lowhalf:
                            xs = xs[:R // 2] + [0] * (R // 2)
                        out = F.dft_fwd([V(x, 2 * p) for x in xs], R, lowhalf, tws)
                        assert all(o.hi <= 2 * p for o in out)
                        plain_tw = [t.v * F.rinv % p for t in tws] if tws else None
                        assert [o.v % p for o in out] == dft_ref(F, xs, R, plain_tw)


@pytest.mark.parametrize("p", PRIMES)
def test_inverse_dfts_stay_below_4p(p):
    F = Field(p)
    rng = random.Random(p + 1)
    for R in (2, 4, 8, 16):
        for use_tw in (False, True):
            for tws in (tw_values(F, R, rng) if use_tw else [None]):
                for xs in extreme_inputs(F, 4 * p, R, rng):
                    out = F.dft_inv([V(x, 4 * p) for x in xs], R, tws)
                    assert all(o.hi <= 4 * p for o in out)
                    plain_tw = [t.v * F.rinv % p for t in tws] if tws else None
                    assert [o.v % p for o in out] == dft_ref(F, xs, R, plain_tw, inverse=True)


@pytest.mark.parametrize("p", PRIMES)
def test_column_unpack_and_row_passes(p):
    """The compositions around the DFTs, at their extreme inputs."""
    F = Field(p)
    rng = random.Random(p + 2)
    # forward column pass, N = 2^m: a 32-bit limb into Montgomery form, [0, 2p)
    for limb in (0, 1, M32 - 1):
        assert F.mont(V(limb, M32), V(F.one, p)).hi <= 2 * p
    # N = 3 * 2^m: two row-twiddled limbs (rows < N1/2), summed and reduced
    for x, x1 in ((M32 - 1, M32 - 1), (0, M32 - 1), (M32 - 1, 0)):
        for g0, g1 in ((p - 1, p - 1), (rng.randrange(p), rng.randrange(p))):
            s = F.red2(F.add(F.mont(V(x, M32), V(g0, p)), F.mont(V(x1, M32), V(g1, p))))
            assert s.hi <= 2 * p
    # N = 5 * 2^m: three row-twiddled limbs (the third on rows < N1/2), the
    # first two summed and reduced, then the third added and reduced
    for x, x1, x2 in ((M32 - 1, M32 - 1, M32 - 1), (0, M32 - 1, M32 - 1), (M32 - 1, 0, 0)):
        for g0, g1, g2 in ((p - 1, p - 1, p - 1), (rng.randrange(p), rng.randrange(p), rng.randrange(p))):
            s = F.red2(F.add(F.mont(V(x, M32), V(g0, p)), F.mont(V(x1, M32), V(g1, p))))
            s = F.red2(F.add(s, F.mont(V(x2, M32), V(g2, p))))
            assert s.hi <= 2 * p
            assert s.v % p == (x * g0 + x1 * g1 + x2 * g2) * F.rinv % p
    # 4096-point row kernel: four-step twiddle on load, three radix-16 steps
    # (two with step twiddles), raw products pending, reduced once per three pairs
    for xs in extreme_inputs(F, 2 * p, 16, rng):
        v = [F.mont(V(x, 2 * p), V(p - 1, p)) for x in xs]
        v = F.dft_fwd(v, 16, tw=[V(p - 1, p)] * 16)
        v = F.dft_fwd(v, 16, tw=[V(p - 1, p)] * 16)
        v = F.dft_fwd(v, 16)
        assert all(o.hi <= 2 * p for o in v)
    top = V(2 * p - 1, 2 * p)
    for npairs in (1, 2, 3, 4, 7):
        acc = V(0, 1)
        pend = V(0, 1)
        want = 0
        for i in range(npairs):
            pend = F.add64(pend, F.mul64(top, top))
            want = (want + top.v * top.v) % p
            if (i + 1) % 3 == 0 or i + 1 == npairs:
                acc = F.red2(F.add(acc, F.red2(F.redc64(pend))))
                pend = V(0, 1)
        assert acc.hi <= 2 * p and acc.v % p == want * F.rinv % p
    # pending bound with the largest possible pair count between reductions
    F.redc64(V(3 * (2 * p - 1) ** 2, 3 * (2 * p - 1) ** 2 + 1))
    # generic row kernel: Montgomery product per pair, accumulator below 2p,
    # then the pair groups' accumulators summed pairwise
    acc = V(0, 1)
    for _ in range(5):
        acc = F.red2(F.add(acc, F.mont(top, top)))
    grp = acc
    for _ in range(7):
        grp = F.red2(F.add(grp, acc))
    assert grp.hi <= 2 * p
    # inverse: DFT outputs below 4p, then the inverse four-step twiddle (with
    # 1/N and the Montgomery correction folded in, canonical) on store
    v = F.dft_inv([V(4 * p - 1, 4 * p)] * 16, 16, tw=[V(p - 1, p)] * 16)
    out = [F.mont(x, V(p - 1, p)) for x in v]
    assert all(o.hi <= 2 * p for o in out)
    # inverse column pass: inputs below 2p from the row pass, canonical at the end
    v = F.dft_inv([V(2 * p - 1, 2 * p)] * 8, 8, tw=[V(p - 1, p)] * 8)
    v = F.dft_inv(v, 8)
    assert all(F.canon(F.red2(x)).hi <= p for x in v)


@pytest.mark.parametrize("p", PRIMES)
def test_inverse_radix3_step(p):
    """The reconstruction kernel's inverse radix-3 step on canonical residues:
    s0 + u1 + u2, s0 - (u1 + u2)/2 +- h (u1 - u2), canonical at the end."""
    F = Field(p)
    for s0, s1, s2 in ((p - 1, p - 1, p - 1), (0, p - 1, 0), (p - 1, 0, p - 1), (0, 0, 0)):
        for gi1, gi2 in ((p - 1, p - 1), (1, p - 1)):
            S0, S1, S2 = V(s0, p), V(s1, p), V(s2, p)
            u1 = F.mont(S1, V(gi1, p))
            u2 = F.mont(S2, V(gi2, p))
            a = F.mont(F.add(u1, u2), V((p - 1) // 2 * M32 % p, p))
            d = F.mont(F.sub2p(u1, u2), V(p - 1, p))
            x0 = F.canon(F.red2(F.add(S0, F.red2(F.add(u1, u2)))))
            x1 = F.canon(F.red2(F.add(S0, F.red2(F.add(a, d)))))
            x2 = F.canon(F.red2(F.add(S0, F.red2(F.sub2p(a, d)))))
            assert max(x0.hi, x1.hi, x2.hi) <= p


@pytest.mark.parametrize("p", PRIMES)
def test_inverse_radix5_step(p):
    """The reconstruction kernel's inverse radix-5 step on canonical residues
    s_k0: u_0 = s_0, u_k0 = s_k0 * gi_k0 (Montgomery, k0 > 0), then
    x_n0 = u_0 + sum_(k0 > 0) u_k0 * w^(k0 n0 mod 5) (w^0 taken as u_k0 itself
    for n0 = 0), each partial sum reduced below 2p, canonical at the end."""
    F = Field(p)
    rng = random.Random(p + 5)
    for ss in ([p - 1] * 5, [0, p - 1, 0, p - 1, 0], [p - 1, 0, 0, 0, p - 1], [rng.randrange(p) for _ in range(5)]):
        for gi in ([p - 1] * 5, [rng.randrange(p) for _ in range(5)]):
            wi = [V(rng.randrange(p) if e else F.one, p) for e in range(5)]
            wi[1] = V(p - 1, p)
            S = [V(x, p) for x in ss]
            u = [S[0]] + [F.mont(S[k0], V(gi[k0], p)) for k0 in range(1, 5)]
            assert all(t.hi <= 2 * p for t in u)
            for n0 in range(5):
                acc = u[0]
                want = u[0].v
                for k0 in range(1, 5):
                    term = F.mont(u[k0], wi[(k0 * n0) % 5]) if n0 else u[k0]
                    acc = F.red2(F.add(acc, term))
                    want += term.v
                x = F.canon(acc)
                assert x.hi <= p and x.v == want % p


def test_garner_at_the_corners():
    """Garner's reconstruction (canonical residues -> the value below
    p0 p1 p2) for the corner residues of every prime triple."""
    text = open(INTERNAL).read()
    triples = [tuple(int(x) for x in t) for t in re.findall(r"\{\d+, \{(\d+)u, (\d+)u, (\d+)u\}\}", text)]
    assert len(triples) >= 10
    rng = random.Random(5)
    for p0, p1, p2 in triples:
        F1, F2 = Field(p1), Field(p2)
        inv_p0_mod_p1 = V(pow(p0, -1, p1) * M32 % p1, p1)
        inv_p0p1_mod_p2 = V(pow(p0 * p1, -1, p2) * M32 % p2, p2)
        inv_p1_mod_p2 = V(pow(p1, -1, p2) * M32 % p2, p2)
        one_sub = p0 < 2 * p1 and p0 < 2 * p2 and p1 < 2 * p2  # as the library's host code

        def reduce(F, x):  # a canonical value of a larger prime, reduced modulo F.p
            return F.csub(x) if one_sub else F.mmul(x, V(F.one, F.p))
        cases = [(p0 - 1, p1 - 1, p2 - 1), (0, 0, 0), (p0 - 1, 0, 0), (0, p1 - 1, 0), (0, 0, p2 - 1),
                 (p1, p1 - 1, p2), (p2, 0, p2 - 1)]
        cases = [(a % p0, b % p1, c % p2) for a, b, c in cases]
        cases += [(rng.randrange(p0), rng.randrange(p1), rng.randrange(p2)) for _ in range(20)]
        for r0, r1, r2 in cases:
            r0a, r0b = reduce(F1, V(r0, p0)), reduce(F2, V(r0, p0))
            v1 = F1.mmul(F1.msub(V(r1, p1), r0a), inv_p0_mod_p1)
            v1b = reduce(F2, V(v1.v, p1))
            T = F2.add64(F2.mul64(F2.msub(V(r2, p2), r0b), inv_p0p1_mod_p2),
                         F2.mul64(V(p2 - v1b.v, p2 + 1), inv_p1_mod_p2))
            v2 = F2.canon(F2.redc64(T))
            c = r0 + v1.v * p0 + v2.v * p0 * p1
            assert c < p0 * p1 * p2
            assert (c % p0, c % p1, c % p2) == (r0, r1, r2)
