"""CPU checks of the C interface: the library loads, exports every function
include/pa.h declares, and its host-side plan rule (its own copy of the
Mersenne table and the parameter rule of Sec. 4 / Table 3) agrees with the
oracle's.  No compute call is made here."""
import ctypes
import math
import random

import pytest

import oracle
from oracle import defn
from paper_2105_13678_amd import binding


def test_library_exports_every_header_function():
    names = binding.header_functions()
    assert {"pa_plan_create", "pa_hash", "pa_hash_async", "pa_plan_query", "pa_status_string"} <= set(names)
    lib = binding.lib()
    for name in names:
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_status_strings():
    for code, name in [(0, "PA_OK"), (2, "PA_RELOAD"), (-2, "PA_ERR_NO_GAMMA"), (-4, "PA_ERR_INEXACT"),
                       (-5, "PA_ERR_SEED_B_EVEN"), (-6, "PA_ERR_SEED_RANGE"), (-10, "PA_ERR_LIMIT")]:
        assert binding.status_string(code) == name
    assert binding.decode_status(0) == 0
    assert binding.decode_status(4) == binding.PA_RELOAD
    assert binding.decode_status(2 | 4) == binding.PA_ERR_SEED_B_EVEN
    assert binding.decode_status(1 | 2 | 4) == binding.PA_ERR_SEED_RANGE


def test_plan_rule_matches_oracle():
    rng = random.Random(3)
    for _ in range(3000):
        r = int(2 ** rng.uniform(0, 27.5))
        n = r + 1 + int(2 ** rng.uniform(0, 33))
        st_o, g_o, k_o = oracle.plan(n, r, 0)
        st, info = binding.plan_query(n, r)
        if st_o != 0:
            assert st == st_o
            continue
        if st == binding.PA_ERR_LIMIT:
            assert k_o > 4096 or (2 * math.ceil(g_o / 32) - 1) > 3 << 23
            continue
        assert st == 0, (n, r, st)
        assert (info["gamma"], info["k"]) == (g_o, k_o)


@pytest.mark.parametrize("n,r,flags,gamma,k,B,L,N", [
    (1 << 20, (1 << 20) // 10, 0, 110503, 10, 32, 3454, 1 << 13),
    (260_000_000, 26_000_000, 0, 30402457, 9, 32, 950077, 1 << 21),
    (10 * 25964951, 25237932, 0, 25964951, 10, 32, 811405, 1 << 21),
    # the paper's largest CV block (8e8 bits, r = n/10): 5 * 2^20 instead of 2^23 (or 3 * 2^21)
    (800_000_000, 80_000_000, 0, 82589933, 10, 32, 2580936, 5 << 20),
    (800_000_000, 80_000_000, 1, 82589933, 10, 32, 2580936, 1 << 23),
    (800_000_000, 80_000_000, 2, 82589933, 10, 32, 2580936, 3 << 21),
    # the largest block: 3 * 2^22 at B = 31 instead of 2^24 at B = 29
    (1 << 32, 1 << 27, 0, 136279841, 32, 31, 4396124, 3 << 22),
    (1 << 32, 1 << 27, 1, 136279841, 32, 29, 4699305, 1 << 24),
])
def test_derived_shapes(n, r, flags, gamma, k, B, L, N):
    st, info = binding.plan_query(n, r, flags=flags)
    assert st == 0
    assert (info["gamma"], info["k"], info["B"], info["L"], info["N"]) == (gamma, k, B, L, N)
    f = info["len_factor"]
    assert info["nprimes"] == 3 and info["log2N1"] + info["log2N2"] == info["log2N"]
    assert N == f << info["log2N"] and f in (1, 3, 5) and (flags == 0 or f == {1: 1, 2: 3, 4: 5}[flags])
    # the primes: the three largest below 2^30 with f * 2^max(log2N, 20 or 18) | p - 1
    assert sorted(info["primes"]) == sorted(largest_ntt_primes(max(info["log2N"], 20 if f == 1 else 18), f=f))
    # exactness: k L (2^B - 1)^2 below the product of the three NTT primes
    P3 = math.prod(info["primes"])
    assert k * L * (2 ** B - 1) ** 2 < P3
    assert info["exact_log2"] < math.log2(P3)
    assert info["out_words"] == (r + 63) // 64
    assert info["seed_words"] == (gamma + 63) // 64
    assert 2 * L - 1 <= N < 2 * (2 * L - 1) or N == 64


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 3.4e14 (bases 2, 3, 5, 7, 11, 13, 17)."""
    if n < 2:
        return False
    for q in (2, 3, 5, 7, 11, 13, 17):
        if n % q == 0:
            return n == q
    d, s = n - 1, 0
    while d % 2 == 0:
        d, s = d // 2, s + 1
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


def largest_ntt_primes(m: int, count: int = 3, f: int = 1) -> list[int]:
    """The `count` largest primes p < 2^30 with f * 2^m | p - 1, by search."""
    step = f << m
    out, c = [], ((1 << 30) - 2) // step
    while len(out) < count and c > 0:
        p = c * step + 1
        if is_prime(p):
            out.append(p)
        c -= 1
    return out


def test_prime_triples_are_the_largest_with_the_roots():
    """Every plan's primes are below 2^30 (so 4p < 2^32), prime, have the
    transform's roots of unity, and are the largest such (one triple serves
    every length up to 2^20, and every length 3 * 2^m up to 3 * 2^18)."""
    seen = set()
    rng = random.Random(5)
    for i in range(600):
        r = int(2 ** rng.uniform(0, 27.0))
        n = r + 1 + int(2 ** rng.uniform(0, 31))
        st, info = binding.plan_query(n, r, flags=binding.PA_FLAG_RADIX3_LENGTHS if i % 2 else 0)
        if st != 0:
            continue
        m, f = info["log2N"], info["len_factor"]
        for p in info["primes"]:
            assert p < (1 << 30) and (p - 1) % (f << m) == 0 and is_prime(p)
        if (m, f) not in seen:
            assert sorted(info["primes"]) == sorted(largest_ntt_primes(max(m, 20 if f == 1 else 18), f=f))
            seen.add((m, f))
    assert len({m for m, f in seen if f == 1}) >= 8 and len({m for m, f in seen if f == 3}) >= 6


def length_cost(info) -> float:
    """The plan rule's cost of a transform length: N log2 N butterflies, plus
    one pass over N for the radix-3 step of the lengths 3 * 2^m (three for
    the radix-5 step of 5 * 2^m), which count 1.6 (2.0) times below
    3 * 2^19 (5 * 2^19) (measured slower there)."""
    N, f = info["N"], info["len_factor"]
    extra = {1: 0.0, 3: 1.0, 5: 3.0}[f]
    small = 1.0 if f == 1 or info["log2N"] >= 19 else (1.6 if f == 3 else 2.0)
    return N * (math.log2(N) + extra) * small


def test_auto_limb_width_is_cheapest_exact():
    """B = 0 picks, over all limb widths, the cheapest exact transform
    length (each width with the shortest exact length of either form), the
    widest width among equal costs."""
    rng = random.Random(4)
    for _ in range(120):
        r = int(2 ** rng.uniform(0, 27.5))
        n = r + 1 + int(2 ** rng.uniform(0, 32.5))
        st, info = binding.plan_query(n, r)
        if st != 0:
            continue
        g, k, B = info["gamma"], info["k"], info["B"]
        assert k * -(-g // B) * (2 ** B - 1) ** 2 < math.prod(info["primes"])
        assert 2 * info["L"] - 1 <= info["N"]
        c = length_cost(info)
        for b in range(8, 33):
            if b == B:
                continue
            st_b, info_b = binding.plan_query(n, r, B=b)
            if st_b != 0:
                assert st_b in (binding.PA_ERR_INEXACT, binding.PA_ERR_LIMIT)
                continue
            assert length_cost(info_b) >= c if b < B else length_cost(info_b) > c, (n, r, b, B)


def test_power_of_two_flag():
    """PA_FLAG_POW2_LENGTHS restricts the plan to lengths 2^m; the old rule
    (widest exact B) then holds; unknown flag bits are rejected."""
    rng = random.Random(6)
    mixed = 0
    for _ in range(200):
        r = int(2 ** rng.uniform(0, 27.5))
        n = r + 1 + int(2 ** rng.uniform(0, 32.5))
        st, info = binding.plan_query(n, r, flags=binding.PA_FLAG_POW2_LENGTHS)
        st0, info0 = binding.plan_query(n, r)
        assert (st == 0) == (st0 == 0)
        if st != 0:
            continue
        mixed += info0["len_factor"] != 1
        assert info["len_factor"] == 1 and info["N"] == 1 << info["log2N"]
        assert length_cost(info0) <= length_cost(info)
        B = info["B"]
        if B < 32:
            assert binding.plan_query(n, r, B=B + 1, flags=binding.PA_FLAG_POW2_LENGTHS)[0] in (
                binding.PA_ERR_INEXACT, binding.PA_ERR_LIMIT)
    assert mixed >= 15  # the rule still takes lengths 3 * 2^m and 5 * 2^m (from 2^19 up) for many shapes
    assert binding.plan_query(1000, 10, flags=8)[0] == binding.PA_ERR_ARG  # unknown bit
    for two in (3, 5, 6, 7):  # at most one length flag
        assert binding.plan_query(1000, 10, flags=two)[0] == binding.PA_ERR_ARG


def test_radix5_flag():
    """PA_FLAG_RADIX5_LENGTHS: the shortest exact length 5 * 2^m (m <= 20,
    columns of at most 256 rows) with its own primes (5 * 2^m | p - 1)."""
    rng = random.Random(15)
    seen = 0
    for _ in range(300):
        r = int(2 ** rng.uniform(0, 26))
        n = r + 1 + int(2 ** rng.uniform(0, 30))
        st0, info0 = binding.plan_query(n, r)
        st, info = binding.plan_query(n, r, flags=binding.PA_FLAG_RADIX5_LENGTHS)
        if st0 == 0:
            assert info0["len_factor"] in (1, 3, 5)
        if st != 0:
            assert st in (binding.PA_ERR_LIMIT, binding.PA_ERR_INEXACT)
            continue
        seen += 1
        N, m = info["N"], info["log2N"]
        assert info["len_factor"] == 5 and N == 5 << m and m <= 20 and info["log2N1"] <= 8
        assert N >= 2 * info["L"] - 1 and (m == 6 or (5 << (m - 1)) < 2 * info["L"] - 1)
        assert all((p - 1) % N == 0 and p < 1 << 30 for p in info["primes"])
        assert info["k"] * info["L"] * (2 ** info["B"] - 1) ** 2 < math.prod(info["primes"])
    assert seen > 100
    # the paper's 8e8-bit CV block: 2L - 1 = 0.62 * 2^23 fits 5 * 2^20 (1.02x) instead of 3 * 2^21 (1.22x)
    st, info = binding.plan_query(800_000_000, 80_000_000, flags=binding.PA_FLAG_RADIX5_LENGTHS)
    assert st == 0 and info["N"] == 5 << 20 and info["log2N1"] == 8


def test_plan_errors():
    assert binding.plan_query(1 << 32, (1 << 32) // 10)[0] == binding.PA_ERR_NO_GAMMA
    assert binding.plan_query(100, 100)[0] == binding.PA_ERR_ARG
    assert binding.plan_query(100, 0)[0] == binding.PA_ERR_ARG
    assert binding.plan_query(100, 10, gamma=11)[0] == binding.PA_ERR_GAMMA
    assert binding.plan_query(100, 13, gamma=13)[0] == binding.PA_ERR_GAMMA
    assert binding.plan_query(1000, 10, B=7)[0] == binding.PA_ERR_ARG
    assert binding.plan_query(1000, 10, B=33)[0] == binding.PA_ERR_ARG
    # exactness bound k * L * (2^B - 1)^2 < p0 p1 p2
    st, info = binding.plan_query(260_000_000, 26_000_000, B=32)
    assert st == 0
    assert binding.plan_query(1 << 32, 1 << 27, B=32)[0] == binding.PA_ERR_INEXACT
    assert binding.plan_query(1 << 32, 200)[0] == binding.PA_ERR_LIMIT   # k > 4096


def test_length_form_flags_and_tile_width():
    """PA_FLAG_RADIX3_LENGTHS forces lengths 3 * 2^m, both flags together are
    rejected, as is a nonzero reserved word; col_lg fixes the key-chunk
    column-tile width within the tile limits (2^col_lg <= row length,
    log2N1 + col_lg <= 14) and is reported back; the automatic width widens
    short columns and narrows columns of 1024 rows to 8."""
    n, r = 18_802_622, 2_288_514  # gamma = 2,976,221, k = 7
    st, i3 = binding.plan_query(n, r, flags=binding.PA_FLAG_RADIX3_LENGTHS)
    assert st == 0 and i3["len_factor"] == 3 and i3["N"] == 3 << 16
    st, i2 = binding.plan_query(n, r, flags=binding.PA_FLAG_POW2_LENGTHS)
    assert st == 0 and i2["len_factor"] == 1 and i2["N"] == 1 << 18
    assert binding.plan_query(n, r, flags=3)[0] == binding.PA_ERR_ARG
    prm = binding.Params(n, r, 0, 0, 0, 0, 1)
    info = binding.PlanInfo()
    assert binding.lib().pa_plan_query(ctypes.byref(prm), ctypes.byref(info)) == binding.PA_ERR_ARG
    # automatic width: 2^16-point rows of 16 rows widen to 64 columns (14 arrays)
    assert (i3["log2N1"], i3["log2N2"], i3["col_lg"]) == (4, 12, 6)
    assert binding.plan_query(260_000_000, 26_000_000)[1]["col_lg"] == 4
    # columns of 1024 rows (the 2^32-bit block, N = 3 * 2^22; the 5e8-bit
    # block, N = 2^22): 8 columns
    i_big = binding.plan_query(1 << 32, 1 << 27)[1]
    assert (i_big["log2N1"], i_big["log2N2"], i_big["col_lg"]) == (10, 12, 3)
    i_5e8 = binding.plan_query(500_000_000, 50_000_000)[1]
    assert (i_5e8["N"], i_5e8["log2N1"], i_5e8["log2N2"], i_5e8["col_lg"]) == (1 << 22, 10, 12, 3)
    for c in (1, 3, 8, 10):
        st, info = binding.plan_query(n, r, flags=binding.PA_FLAG_RADIX3_LENGTHS, col_lg=c)
        assert st == 0 and info["col_lg"] == c
    assert binding.plan_query(n, r, flags=binding.PA_FLAG_RADIX3_LENGTHS, col_lg=11)[0] == binding.PA_ERR_ARG  # 4 + 11 > 14
    assert binding.plan_query(1 << 20, 1 << 16, col_lg=13)[0] == binding.PA_ERR_ARG  # wider than a row


def test_profile_digest_covers_code_only(tmp_path):
    """bench.py reports a kernel's HBM bytes only while the profile summary was
    taken on the current device sources: the digest covers their code, so an
    edit of comments or white space keeps it and any code edit changes it."""
    from paper_2105_13678_amd import build, profile_summary
    code = "__global__ void k(int *p) {\n    p[0] = 1;  // one\n}\n/* block\n   comment */\n"
    assert build._code_only(code) == build._code_only("__global__ void k(int *p) { p[0] = 1; }")
    assert build._code_only(code) != build._code_only(code.replace("p[0] = 1", "p[0] = 2"))
    digest = build.source_digest()
    summary = tmp_path / "hbm.md"
    summary.write_text(f"    traffic k_row16<0> fetch=10 write=20 sources={digest}\n"
                       f"    traffic k_other fetch=1 write=2 sources={'0' * 64}\n")
    assert profile_summary.read_traffic(str(summary), "k_row16<0>") == (10, 20)
    assert profile_summary.read_traffic(str(summary), "k_other") is None  # taken on other sources
    assert profile_summary.read_traffic(str(tmp_path / "absent.md"), "k_row16<0>") is None
