"""GPU parity: the HIP path (through the C interface) against the CPU oracle,
bit for bit, on seeded synthetic inputs.

Every case prints its name, seed and shape before it touches the GPU.
"""
import hashlib
import json
import math
import os
import random
import sys

import numpy as np
import pytest

import oracle
from oracle import defn
from paper_2105_13678_amd import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def pa():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2105_13678_amd as pa
    pa.lib()
    return pa


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def put(pa, words):
    return pa.to_device(np.asarray(words, dtype=np.uint64))


def run_gpu(pa, plan, blk, stages=False):
    key, a, b, c = (put(pa, x) for x in (blk.key, blk.a, blk.b, blk.c))
    if stages:
        st, out, y, U = plan.hash_stages(key, a, b, c)
        return st, pa.from_device(out), pa.from_device(y), pa.from_device(U)
    st, out = plan.hash(key, a, b, c)
    return st, pa.from_device(out)


def check_block(pa, blk, B=0, stages=True, label="", flags=0, col_lg=0):
    say(f"[case] {label} n={blk.n} r={blk.r} gamma={blk.gamma} k={blk.k} B={B} flags={flags} col_lg={col_lg}")
    plan = pa.Plan(blk.n, blk.r, gamma=blk.gamma, B=B, flags=flags, col_lg=col_lg)
    try:
        st_g, out_g, y_g, U_g = run_gpu(pa, plan, blk, stages=True)
    finally:
        plan.close()
    st_o, out_o, y_o, U_o = oracle.hash(blk.key, blk.n, blk.r, blk.gamma, blk.a, blk.b, blk.c, stages=True)
    assert st_g == st_o, (label, st_g, st_o)
    if st_o == 0:
        assert np.array_equal(out_g, out_o), label
        if stages:
            assert np.array_equal(y_g, y_o), label + " (y)"
            assert np.array_equal(U_g, U_o), label + " (U)"
    return st_g, out_g


def test_small_random_shapes(pa):
    rng = random.Random(2024)
    gammas = [e for e in defn.MERSENNE_EXPONENTS if 2 <= e <= 23209]
    for t in range(120):
        g = rng.choice(gammas)
        r = rng.randrange(1, g) if g > 2 else 1
        n = rng.randrange(r + 1, rng.choice([2, 5, 12]) * g + 2)
        st, g2, k = defn.plan_shape(n, r, g)
        blk = synth.single_block(1000 + t, n, r, g, k)
        check_block(pa, blk, label=f"random#{t}")


@pytest.mark.parametrize("gamma", [61, 521, 9689])
def test_maximum_chunk_count(pa, gamma):
    """k = 4096 chunks (the plan's limit) with a ragged last chunk: the
    multiply-accumulate runs over 4096 pairs, the column pass over 8192
    arrays, and the reload flag over 4096 chunks."""
    k = 4096
    n, r = k * gamma - 3, gamma // 2
    st, g, kk = defn.plan_shape(n, r, gamma)
    assert st == 0 and kk == k
    assert pa.plan_query(n, r, gamma)[0] == 0
    assert pa.plan_query(n + gamma, r, gamma)[0] == -10  # k = 4097: PA_ERR_LIMIT
    blk = synth.single_block(4096 + gamma, n, r, g, kk)
    check_block(pa, blk, label=f"k=4096 gamma={gamma}")


@pytest.mark.parametrize("gamma", [89, 127, 521, 4423, 110503])
def test_edge_shapes(pa, gamma):
    cases = [
        ("r=1", 3 * gamma, 1),
        ("r=gamma-1", 3 * gamma, gamma - 1),
        ("n=k*gamma", 7 * gamma, gamma // 3),
        ("n=k*gamma-1", 7 * gamma - 1, gamma // 3),
        ("n=gamma+1", gamma + 1, gamma // 2),
        ("k=1", gamma - 1, gamma // 2),
        ("n=k*gamma+1", 4 * gamma + 1, gamma // 5 + 1),
    ]
    for i, (label, n, r) in enumerate(cases):
        st, g, k = defn.plan_shape(n, r, gamma)
        assert st == 0
        blk = synth.single_block(7 * gamma + i, n, r, g, k)
        check_block(pa, blk, label=f"edge {label}")


@pytest.mark.parametrize("B", [8, 11, 16, 20, 24, 29, 31, 32])
def test_limb_width_invariance(pa, B):
    """The output is the same integer for every exact limb width (B is
    representation only, the 2^B-ary words of Sec. 2.1); B changes L, N and
    the transform tiling."""
    n, r = 1 << 20, (1 << 20) // 10
    st, g, k = defn.plan_shape(n, r)
    blk = synth.single_block(31, n, r, g, k)
    check_block(pa, blk, B=B, label=f"B={B}")


@pytest.mark.parametrize("gamma,k", [(756839, 3), (1257787, 2), (3021377, 4), (6972593, 2), (13466917, 2)])
def test_register_radix16_rows(pa, gamma, k):
    """Shapes whose transform length (2^16 .. 2^20) selects the 4096-word
    register radix-16 row pass (and columns of 2^4 .. 2^8 rows), with ragged n."""
    n = k * gamma - 12345
    r = gamma // 7
    st, g, kk = defn.plan_shape(n, r, gamma)
    assert st == 0 and kk == k
    blk = synth.single_block(gamma % 1000, n, r, g, kk)
    check_block(pa, blk, label=f"radix16 rows gamma={gamma}")


def test_two_to_the_21_transform_two_chunks(pa):
    """A 2^21-point transform (the shape of the 2.6e8-bit block) with k = 2
    and a ragged tail: exercises the fixed-shape 512-row column pass and the
    multiply-accumulate over two pairs."""
    gamma = 20996011
    n, r = 2 * gamma - 777, 2_000_001
    st, g, k = defn.plan_shape(n, r, gamma)
    assert st == 0 and k == 2
    blk = synth.single_block(21, n, r, g, k)
    check_block(pa, blk, label="N=2^21 k=2")


@pytest.mark.parametrize("gamma,variants", [
    (6972593, [(0, 1)]),                      # 2^19: 128-row columns
    (13466917, [(0, 1), (0, 2), (16, 2)]),    # 2^20 (256 rows), 3 * 2^19 (128 rows), 3 * 2^20 (256 rows)
])
def test_two_pass_column_shapes(pa, gamma, variants):
    """Columns of 128 and 256 rows (the forward pass's radix-16 last step,
    the 256-row tiles' radix-16 first step and the two-pass inverse), in both
    length forms and both stages, one chunk with a ragged tail, against the
    oracle's output and stage values (computed once per block)."""
    n, r = gamma - 1234, gamma // 9
    st, g, k = defn.plan_shape(n, r, gamma)
    assert st == 0 and k == 1
    blk = synth.single_block(gamma % 97, n, r, g, k)
    st_o, out_o, y_o, U_o = oracle.hash(blk.key, n, r, g, blk.a, blk.b, blk.c, stages=True)
    assert st_o == 0
    for B, flags in variants:
        info = pa.plan_query(n, r, g, B=B, flags=flags)[1]
        assert info["log2N1"] in (7, 8) and info["col_lg"] == 4, info
        say(f"[case] two-pass columns gamma={g} n={n} r={r} B={B} flags={flags} N={info['N']} "
            f"m1={info['log2N1']}")
        plan = pa.Plan(n, r, gamma=g, B=B, flags=flags)
        try:
            st_g, out_g, y_g, U_g = run_gpu(pa, plan, blk, stages=True)
        finally:
            plan.close()
        assert st_g == 0
        assert np.array_equal(y_g, y_o) and np.array_equal(U_g, U_o) and np.array_equal(out_g, out_o), info


@pytest.mark.parametrize("n,r,flags", [
    (1 << 20, (1 << 20) // 10, 0),        # 8192-point transforms: generic column and row kernels
    (3 * 44497 - 7, 44497 // 3, 2),       # 3 * 2^m: radix-3 column pass, coefficient planes, digit tiles
    (2 * 1257787 - 9, 1257787 // 5, 1),   # 2^17: 4096-point register rows, 32-row columns
    (6972593 - 1234, 6972593 // 9, 1),    # 2^19: two-pass 128-row columns
])
def test_poisoned_scratch_does_not_change_results(pa, n, r, flags):
    """Determinism against stale memory: the plan's scratch (everything but
    the twiddle tables) is filled with a pattern before each hash
    (pa_plan_fill_scratch); output and both stage values stay the oracle's
    for every pattern, so no kernel reads a scratch word it has not written."""
    st, g, k = defn.plan_shape(n, r)
    assert st == 0
    blk = synth.single_block(n % 1009, n, r, g, k)
    st_o, out_o, y_o, U_o = oracle.hash(blk.key, n, r, g, blk.a, blk.b, blk.c, stages=True)
    assert st_o == 0
    plan = pa.Plan(n, r, flags=flags)
    try:
        for word in (0x00000000, 0xFFFFFFFF, 0xA5A5A5A5, 0x3FFFFFFF, 0x80000001):
            say(f"[case] poisoned scratch n={n} r={r} gamma={g} k={k} flags={flags} word={word:#010x}")
            assert plan.fill_scratch(word) == 0
            st_g, out_g, y_g, U_g = run_gpu(pa, plan, blk, stages=True)
            assert st_g == 0
            assert np.array_equal(out_g, out_o) and np.array_equal(y_g, y_o) and np.array_equal(U_g, U_o), word
    finally:
        plan.close()


# (gamma, k) whose transform length is 3 * 2^m, m = 6 .. 16: column passes of
# 2^3 .. 2^7 rows (the 8-row one single-step), rows of 2^3 .. 2^12 words.
RADIX3_SHAPES = [(2203, 2), (4253, 3), (9689, 1), (19937, 2), (44497, 3), (86243, 2), (132049, 3),
                 (756839, 2), (1257787, 3), (2976221, 2)]


@pytest.mark.parametrize("gamma,k", RADIX3_SHAPES)
def test_radix3_lengths_against_oracle(pa, gamma, k):
    """Lengths N = 3 * 2^m (radix-3 step fused into the unpacking column
    pass and into the Chinese-remainder step), ragged n, against the oracle;
    then the same block on power-of-two lengths."""
    n, r = k * gamma - 7, gamma // 3
    st, g, kk = defn.plan_shape(n, r, gamma)
    assert st == 0 and kk == k
    info = pa.plan_query(n, r, gamma, flags=pa.PA_FLAG_RADIX3_LENGTHS)[1]
    assert info["len_factor"] == 3, info
    blk = synth.single_block(3 * gamma + k, n, r, g, kk)
    _, out3 = check_block(pa, blk, label=f"radix-3 N={info['N']} gamma={gamma} k={k}",
                          flags=pa.PA_FLAG_RADIX3_LENGTHS)
    _, out2 = check_block(pa, blk, label=f"power-of-two gamma={gamma} k={k}", flags=pa.PA_FLAG_POW2_LENGTHS)
    assert np.array_equal(out3, out2)


# (gamma, k) for lengths 5 * 2^m, m = 6 .. 20: column passes of 8 .. 256 rows
# (compile-time tiles and the generic kernel), rows of 8 .. 4096 words.
RADIX5_SHAPES = [(2203, 2), (4253, 3), (9689, 1), (19937, 2), (44497, 3), (86243, 2), (132049, 3),
                 (756839, 2), (1257787, 3), (2976221, 2), (6972593, 1), (13466917, 1)]


@pytest.mark.parametrize("gamma,k", RADIX5_SHAPES)
def test_radix5_lengths_against_oracle(pa, gamma, k):
    """Lengths N = 5 * 2^m (PA_FLAG_RADIX5_LENGTHS: radix-5 step fused into
    the unpacking column pass, five transforms per tile and prime, and the
    inverse radix-5 step fused into the reconstruction), ragged n, output and
    both stage values against the oracle."""
    n, r = k * gamma - 7, gamma // 3
    st, g, kk = defn.plan_shape(n, r, gamma)
    assert st == 0 and kk == k
    info = pa.plan_query(n, r, gamma, flags=pa.PA_FLAG_RADIX5_LENGTHS)[1]
    assert info["len_factor"] == 5, info
    blk = synth.single_block(5 * gamma + k, n, r, g, kk)
    check_block(pa, blk, label=f"radix-5 N={info['N']} m1={info['log2N1']} c={info['col_lg']} gamma={gamma} k={k}",
                flags=pa.PA_FLAG_RADIX5_LENGTHS)


@pytest.mark.parametrize("n,r", [(3 * 20996011 - 99, 14_000_000), (800_000_000, 80_000_000)])
def test_radix3_against_power_of_two_lengths(pa, n, r):
    """Larger radix-3 shapes (3 * 2^19 with 128-row columns and 4096-word
    register rows; the paper's 8e8-bit CV block at 3 * 2^21 with 512-row
    columns) against the same block on power-of-two lengths (2^21, 2^23),
    output and both stage values."""
    st, g, k = defn.plan_shape(n, r)
    assert st == 0
    i3 = pa.plan_query(n, r, flags=pa.PA_FLAG_RADIX3_LENGTHS)[1]
    i2 = pa.plan_query(n, r, flags=pa.PA_FLAG_POW2_LENGTHS)[1]
    assert i3["len_factor"] == 3 and i2["len_factor"] == 1 and i3["N"] < i2["N"]
    blk = synth.single_block(5, n, r, g, k)
    res = []
    for flags in (pa.PA_FLAG_RADIX3_LENGTHS, pa.PA_FLAG_POW2_LENGTHS):
        say(f"[case] radix-3 vs power-of-two n={n} r={r} gamma={g} k={k} flags={flags}")
        plan = pa.Plan(n, r, flags=flags)
        try:
            res.append(run_gpu(pa, plan, blk, stages=True))
        finally:
            plan.close()
    assert res[0][0] == res[1][0] == 0
    for a3, a2 in zip(res[0][1:], res[1][1:]):
        assert np.array_equal(a3, a2)


@pytest.mark.parametrize("gamma,k,flags", [(2976221, 7, 2), (2976221, 7, 1), (132049, 3, 2), (20996011, 2, 2),
                                           (44497, 5, 1)])
def test_column_tile_widths(pa, gamma, k, flags):
    """Every admissible column-tile width of the key-chunk column pass
    (2^1 .. 2^min(row, 14 - column) columns; 1 to 8 first-step tasks per
    thread, idle threads where a tile has fewer tasks than threads) gives the
    oracle's output, for both length forms."""
    n, r = k * gamma - 5, gamma // 5
    st, g, kk = defn.plan_shape(n, r, gamma)
    assert st == 0 and kk == k
    info = pa.plan_query(n, r, gamma, flags=flags)[1]
    blk = synth.single_block(11 * k + flags, n, r, g, kk)
    st_o, out_o = oracle.hash(blk.key, n, r, g, blk.a, blk.b, blk.c)
    hi = min(info["log2N2"], 14 - info["log2N1"])
    for c in sorted({1, 2, hi // 2, hi - 1, hi} - {0}):
        say(f"[case] tile width gamma={gamma} k={k} flags={flags} N={info['N']} col_lg={c}")
        plan = pa.Plan(n, r, gamma=gamma, flags=flags, col_lg=c)
        try:
            st_g, out = run_gpu(pa, plan, blk)
        finally:
            plan.close()
        assert st_g == st_o == 0
        assert np.array_equal(out, out_o), c


def test_tuned_plans_match(pa):
    """pa_plan_tune returns an exact shape (explicit B, length form, tile
    width) whose output equals the oracle's."""
    for n, r in ((18_802_622, 2_288_514), (5_000_000, 300_000)):
        st, g, k = defn.plan_shape(n, r)
        say(f"[case] tune n={n} r={r}")
        best, ms = pa.plan_tune(n, r, reps=2)
        assert best["B"] >= 8 and best["flags"] in (1, 2, 4) and best["col_lg"] >= 1 and ms > 0
        info = pa.plan_query(n, r, B=best["B"], flags=best["flags"], col_lg=best["col_lg"])[1]
        assert info["k"] * info["L"] * (2 ** info["B"] - 1) ** 2 < math.prod(info["primes"])
        blk = synth.single_block(77, n, r, g, k)
        check_block(pa, blk, B=best["B"], flags=best["flags"], stages=False, label="tuned", col_lg=best["col_lg"])


def test_config_one_mib_block(pa):
    n, r = 1 << 20, (1 << 20) // 10
    st, g, k = defn.plan_shape(n, r)
    blk = synth.single_block(1, n, r, g, k)
    check_block(pa, blk, label="2^20 block seed 1")


def _chunks_key(chunks, gamma, n):
    K = 0
    for i, x in enumerate(chunks):
        K |= x << (i * gamma)
    K &= (1 << n) - 1
    return defn.int_to_words(K, (n + 63) // 64)


def _blk(chunks, a, b, c, gamma, n, r):
    W = (gamma + 63) // 64
    return synth.Block(n=n, r=r, gamma=gamma, k=len(a), key=_chunks_key(chunks, gamma, n),
                       a=np.concatenate([defn.int_to_words(v, W) for v in a]),
                       b=defn.int_to_words(b, W), c=defn.int_to_words(c, W))


@pytest.mark.parametrize("flags", [1, 2])
@pytest.mark.parametrize("B", [0, 8, 13])
@pytest.mark.parametrize("gamma", [61, 89, 521, 4423, 44497, 110503])
def test_fold_canonical_cases(pa, gamma, B, flags):
    """S = p must fold to y = 0; S = p + 1 to 1; one-hot seeds rotate a chunk
    (2^gamma = 1 mod p); a_i = p - 1 complements.  Narrow limbs (B = 8, 13)
    spread the second fold's V mod p over up to 16 limbs; both length forms
    (flags 1: 2^m, 2: 3 * 2^m) reconstruct the coefficients differently."""
    p = (1 << gamma) - 1
    rng = random.Random(gamma)
    c = rng.randrange(1 << gamma)
    r = max(1, gamma // 3)
    for label, chunks, a in [("S=p", [p - 1, 1], [1, 1]), ("S=p+1", [p - 1, 2], [1, 1]),
                             ("S=2p", [p - 1, 1], [2, 2]), ("S=0", [0, 0], [5, 7]),
                             ("S=2^gamma", [p - 1, p - 1, 3], [1, 1, 1])]:
        blk = _blk(chunks, a, 1, c, gamma, len(chunks) * gamma, r)
        check_block(pa, blk, B=B, flags=flags, label=f"fold {label}")
    if gamma > 32 * (B or 32) + 64:  # V's carry into limb 32 of y, b odd and > 1
        R = rng.randrange(1 << (gamma - 32 * (B or 32) - 1))
        blk = _blk([p - 1, 1 + ((R + 1) << (32 * (B or 32)))], [1, 1], 3, c, gamma, 2 * gamma, r)
        check_block(pa, blk, B=B, flags=flags, label="fold carry into limb 32")
    x = rng.randrange(p)
    s = rng.randrange(gamma)
    blk = _blk([0, x, 0], [0, 1 << s, 0], 1, 0, gamma, 3 * gamma, r)
    check_block(pa, blk, B=B, flags=flags, label="rotate")
    blk = _blk([0, x, 0], [3, p - 1, 9], 1, 0, gamma, 3 * gamma, r)
    check_block(pa, blk, B=B, flags=flags, label="complement")
    # all-ones limbs everywhere except one bit: long carry chains in every scan
    blk = _blk([p - 1, p - 2, p ^ 1], [p - 1, p - 1, p - 1], (1 << gamma) - 1, (1 << gamma) - 1,
               gamma, 3 * gamma, r)
    check_block(pa, blk, B=B, flags=flags, label="long carries")


def _wrap_cases(gamma, B, rng, c):
    """(label, chunks, a, b, c) for the second fold's cases with a_i = 1:
    S = T_lo + (T >> gamma) equal to p (y = 0); T = 2^gamma (S = 1); the
    lowest 32 limbs of T_lo all ones and T >= 2^gamma, so that V's carry runs
    into limb 32 (upper limbs random: y = S; all ones: S = 2^gamma, y = 1);
    long carries with b = c = p."""
    p = (1 << gamma) - 1
    lo = 32 * B if B else 32 * 32
    R = rng.randrange(1 << (gamma - lo - 1))
    return [("S=p", [p - 1, 1], [1, 1], 1, c),
            ("S=p+1", [p - 1, 2], [1, 1], 1, c),
            ("carry into limb 32", [p - 1, 1 + ((R + 1) << lo)], [1, 1], 3, c),
            ("S=2^gamma", [p - 1, p - 1, 3], [1, 1, 1], 5, c),
            ("long carries", [p - 1, p - 2], [p - 1, p - 1], p, p)]


@pytest.mark.parametrize("flags", [1, 2])
def test_general_wrap_over_many_tiles(pa, flags):
    """The second fold's general case (S = p folds to 0, S = p + 1 to 1, long
    carries) on more carry tiles than the general wrap kernel has
    workgroups (gamma = 1,257,787 at B = 8: 154 tiles), so its workgroups
    take several tiles each."""
    gamma = 1257787
    p = (1 << gamma) - 1
    rng = random.Random(flags)
    c = rng.randrange(1 << gamma)
    r = gamma // 3
    info = pa.plan_query(2 * gamma, r, gamma, B=8, flags=flags)[1]
    assert -(-(info["L"] - 1) // 1024) > 128, info
    for label, chunks, a, b, cc in _wrap_cases(gamma, 8, rng, c):
        blk = _blk(chunks, a, b, cc, gamma, len(chunks) * gamma, r)
        check_block(pa, blk, B=8, flags=flags, label=f"general wrap {label}")


def test_status_codes_and_untouched_output(pa):
    import torch
    gamma = 4423
    p = (1 << gamma) - 1
    n, r = 3 * gamma, 100
    plan = pa.Plan(n, r, gamma=gamma)
    W = (gamma + 63) // 64
    try:
        cases = [
            ("reload", [5, p, 7], [1, 2, 3], 3, 4, pa.PA_RELOAD),
            ("b even", [5, 6, 7], [1, 2, 3], 4, 4, -5),
            ("seed range a", [5, 6, 7], [1, 1 << gamma, 3], 3, 4, -6),
            ("seed range c", [5, 6, 7], [1, 2, 3], 3, 1 << gamma, -6),
            ("range beats reload", [5, p, 7], [1 << gamma, 2, 3], 4, 4, -6),
        ]
        for label, chunks, a, b, c, want in cases:
            say(f"[case] status {label}")
            key = put(pa, _chunks_key(chunks, gamma, n))
            aw = np.concatenate([defn.int_to_words(v % (1 << (64 * W)), W) for v in a])
            bw = defn.int_to_words(b % (1 << (64 * W)), W)
            cw = defn.int_to_words(c % (1 << (64 * W)), W)
            # bits >= 64*W cannot be represented; 1 << gamma stays inside W words here
            out = torch.full((plan.out_words,), 0x5A5A, dtype=torch.int64, device=plan.device)
            st, _ = plan.hash(key, put(pa, aw), put(pa, bw), put(pa, cw), out=out)
            st_o, _ = oracle.hash(_chunks_key(chunks, gamma, n), n, r, gamma, aw, bw, cw)
            assert st == want == st_o, (label, st, want, st_o)
            assert bool((out == 0x5A5A).all()), label + ": output touched"
    finally:
        plan.close()


def test_repeat_runs_identical_and_plan_reuse(pa):
    n, r = 3_000_000, 400_000
    st, g, k = defn.plan_shape(n, r)
    plan = pa.Plan(n, r)
    try:
        outs = []
        for seed in (41, 42, 41):
            blk = synth.single_block(seed, n, r, g, k)
            say(f"[case] reuse seed={seed} n={n} r={r}")
            stg, out = run_gpu(pa, plan, blk)
            st_o, out_o = oracle.hash(blk.key, n, r, g, blk.a, blk.b, blk.c)
            assert stg == st_o == 0 and np.array_equal(out, out_o)
            outs.append(out)
        assert np.array_equal(outs[0], outs[2])
    finally:
        plan.close()


def test_mmh_stage_linear_in_key(pa):
    """Invariant checked without the oracle: with the seeds fixed, the MMH
    value is Z_p-linear in the chunk vector (eq. 2): y(x + x') = y(x) + y(x')
    mod p, where + adds chunks mod p."""
    gamma = 110503
    p = (1 << gamma) - 1
    k = 5
    n = k * gamma
    rng = random.Random(9)
    a = [rng.randrange(p) for _ in range(k)]
    b = rng.randrange(1 << gamma) | 1
    c = rng.randrange(1 << gamma)
    x1 = [rng.randrange(p) for _ in range(k)]
    x2 = [rng.randrange(p) for _ in range(k)]
    xs = [(u + v) % p for u, v in zip(x1, x2)]
    plan = pa.Plan(n, 1000, gamma=gamma)
    ys = []
    Us = []
    try:
        for label, x in (("x1", x1), ("x2", x2), ("x1+x2", xs)):
            say(f"[case] linearity {label}")
            blk = _blk(x, a, b, c, gamma, n, 1000)
            st, out, y, U = run_gpu(pa, plan, blk, stages=True)
            assert st == 0
            ys.append(defn.words_to_int(y))
            Us.append(defn.words_to_int(U))
    finally:
        plan.close()
    assert ys[2] == (ys[0] + ys[1]) % p
    # U is affine in y: U(y) = b*y + c mod 2^gamma
    for y, U in zip(ys, Us):
        assert U == (b * y + c) % (1 << gamma)


def _digest(words):
    return hashlib.sha256(np.ascontiguousarray(words, dtype=np.uint64).tobytes()).hexdigest()


@pytest.mark.parametrize("flags", [0, 1, 2, 4])
@pytest.mark.parametrize("name", ["single_block_2p20", "single_block_2p6e8", "paper_cv_block",
                                  "max_length_single_chunk", "len_2p22_single_chunk", "len_2p23_single_chunk",
                                  "cv_8e8_block", "corner_2p28_r03"])
def test_full_size_blocks_against_stored_oracle_digest(pa, name, flags):
    """Full-size blocks, in the launch configuration the benchmark times,
    against digests written by tests/golden/make_golden.py (oracle only);
    with flags = 1, 2 or 4 (PA_FLAG_POW2_LENGTHS, PA_FLAG_RADIX3_LENGTHS,
    PA_FLAG_RADIX5_LENGTHS) also on the length forms other than the plan
    rule's (5 * 2^m where one holds the product, m <= 20)."""
    gold = json.load(open(os.path.join(HERE, "golden", "full_size.json")))[name]
    n, r = gold["n"], gold["r"]
    st, g, k = defn.plan_shape(n, r)
    assert (g, k) == (gold["gamma"], gold["k"])
    if flags == 4 and pa.plan_query(n, r, flags=4)[0] != 0:
        pytest.skip("no length 5 * 2^m with m <= 20 holds this product")
    if flags and pa.plan_query(n, r)[1]["len_factor"] == {1: 1, 2: 3, 4: 5}[flags]:
        pytest.skip("the plan rule already picks this length form")
    blk = synth.single_block(gold["seed"], n, r, g, k)
    say(f"[case] full size {name} n={n} r={r} gamma={g} k={k} flags={flags}")
    plan = pa.Plan(n, r, flags=flags)
    try:
        st_g, out, y, U = run_gpu(pa, plan, blk, stages=True)
    finally:
        plan.close()
    assert st_g == gold["status"] == 0
    assert [int(v) for v in out[:4]] == gold["out_head"]
    assert _digest(y) == gold["y_sha256"]
    assert _digest(U) == gold["U_sha256"]
    assert _digest(out) == gold["out_sha256"]


def _chunk_int(key_bytes: bytes, lo_bit: int, nbits: int, n: int) -> int:
    """Key bits [lo_bit, lo_bit + nbits) as an int, zero at and above bit n."""
    hi_bit = min(lo_bit + nbits, n)
    if hi_bit <= lo_bit:
        return 0
    b0, b1 = lo_bit // 8, (hi_bit + 7) // 8
    v = int.from_bytes(key_bytes[b0:b1], "little") >> (lo_bit - 8 * b0)
    return v & ((1 << (hi_bit - lo_bit)) - 1)


def _rotation_closed_form(pa, n, r, seed, label):
    """Hash one block with seeds a_i = 2^(s_i) and b = 2^gamma - 1 on both
    length forms (the plan rule's and, flagged, the other) and check both
    against a closed form instead of the oracle: the MMH sum is
    y = sum_i rotl(x_i, s_i) mod p (2^gamma = 1 mod p turns a power-of-two
    product into a rotation) and, with b = -1 mod 2^gamma, the MH value is
    U = c - y mod 2^gamma.  The key and c are uniform; every chunk is active."""
    st, g, k = defn.plan_shape(n, r)
    assert st == 0
    rng = synth.SplitMix64(seed)
    key = rng.words((n + 63) // 64)
    W = (g + 63) // 64
    shifts = [int(v % g) for v in rng.words(k)]
    a = np.zeros(k * W, dtype=np.uint64)
    for i, s in enumerate(shifts):
        a[i * W + s // 64] = np.uint64(1) << np.uint64(s % 64)
    b = np.full(W, np.uint64(0xFFFFFFFFFFFFFFFF), dtype=np.uint64)
    b[-1] = np.uint64((1 << (g % 64)) - 1) if g % 64 else b[-1]
    c = rng.words(W)
    if g % 64:
        c[-1] &= np.uint64((1 << (g % 64)) - 1)
    runs = []
    for flags in (pa.PA_FLAG_RADIX3_LENGTHS, pa.PA_FLAG_POW2_LENGTHS):
        inf = pa.plan_query(n, r, flags=flags)[1]
        say(f"[case] {label} n={n} r={r} gamma={g} k={k} N={inf['N']} B={inf['B']} flags={flags}")
        plan = pa.Plan(n, r, flags=flags)
        try:
            runs.append(run_gpu(pa, plan, synth.Block(n, r, g, k, key, a, b, c), stages=True))
        finally:
            plan.close()
    assert runs[0][0] == runs[1][0] == 0
    for a3, a2 in zip(runs[0][1:], runs[1][1:]):
        assert np.array_equal(a3, a2)
    st_g, out, y, U = runs[0]
    p = (1 << g) - 1
    kb = key.tobytes()
    ysum = 0
    for i, s in enumerate(shifts):
        x = _chunk_int(kb, i * g, g, n)
        ysum += ((x << s) | (x >> (g - s))) & p
    y_want = defn.mod_mersenne(ysum, g)
    c_int = int.from_bytes(c.tobytes(), "little")
    U_want = (c_int - y_want) % (1 << g)
    assert int.from_bytes(y.tobytes(), "little") == y_want
    assert int.from_bytes(U.tobytes(), "little") == U_want
    assert int.from_bytes(out.tobytes(), "little") == U_want >> (g - r)


def test_largest_block_power_of_two_seeds(pa):
    """The largest block, n = 2^32 with r = 2^27 (gamma = 136,279,841, k = 32;
    B = 31 with 3 * 2^22-point transforms, and B = 29 with 2^24-point ones
    under PA_FLAG_POW2_LENGTHS), against the rotation closed form."""
    n, r = 1 << 32, 1 << 27
    assert defn.plan_shape(n, r) == (0, 136279841, 32)
    info = pa.plan_query(n, r)[1]
    info2 = pa.plan_query(n, r, flags=pa.PA_FLAG_POW2_LENGTHS)[1]
    assert (info["N"], info["B"], info2["N"], info2["B"]) == (3 << 22, 31, 1 << 24, 29)
    _rotation_closed_form(pa, n, r, 77, "largest block")


def test_power_of_two_seeds_1024_row_columns(pa):
    """n = 5e8, r = 5e7 (gamma = 57,885,161, k = 9): the plan rule's 2^22-point
    transforms have columns of 1024 rows (the 1024 x 8 column kernel) and
    rows of 4096; the radix-3 form 3 * 2^21 runs the 512-row kernels.  Both
    against the rotation closed form."""
    n, r = 500_000_000, 50_000_000
    assert defn.plan_shape(n, r) == (0, 57885161, 9)
    i2 = pa.plan_query(n, r, flags=pa.PA_FLAG_POW2_LENGTHS)[1]
    i3 = pa.plan_query(n, r, flags=pa.PA_FLAG_RADIX3_LENGTHS)[1]
    assert (i2["N"], i2["log2N1"], i2["log2N2"], i2["col_lg"]) == (1 << 22, 10, 12, 3)
    assert (i3["N"], i3["log2N1"]) == (3 << 21, 9)
    assert pa.plan_query(n, r)[1]["N"] == 1 << 22
    _rotation_closed_form(pa, n, r, 78, "1024-row columns")


@pytest.mark.parametrize("gamma,k,flags,B", [(4423, 5, 0, 0), (4423, 5, 0, 8), (44497, 3, 2, 0), (44497, 3, 1, 8),
                                             (110503, 10, 1, 0), (756839, 2, 2, 8)])
def test_key_bits_past_n_are_ignored(pa, gamma, k, flags, B):
    """Bits >= n of the key's last word are ignored (the split zero-pads the
    key past bit n, Alg. 1): with every such bit set, the output equals the
    oracle's for the same words and the output of the masked key; ragged n
    on both length forms, at the automatic limb width and at B = 8."""
    n = k * gamma - 1000 - (gamma % 61)
    assert n % 64 != 0
    r = gamma // 4
    st, g, kk = defn.plan_shape(n, r, gamma)
    assert st == 0 and kk == k
    blk = synth.single_block(9000 + gamma + B + flags, n, r, g, kk)
    masked = blk.key.copy()
    blk.key[-1] |= ~np.uint64((1 << (n % 64)) - 1)  # every bit >= n of the last word
    assert blk.key[-1] != masked[-1]
    label = f"tail bits set gamma={gamma} k={k} n%64={n % 64} flags={flags} B={B}"
    _, out_tail = check_block(pa, blk, B=B, flags=flags, label=label)
    blk.key = masked
    _, out_masked = check_block(pa, blk, B=B, flags=flags, label=label + " (masked)")
    assert np.array_equal(out_tail, out_masked)
