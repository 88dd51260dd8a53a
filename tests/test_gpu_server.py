"""GPU parity of the serving loop (pa_server_*): requests submitted in a mix
from several sessions give bit-for-bit the outputs of the single-block path
(and of the oracle), the same as when each runs alone; statuses, admission
under a tight memory budget and the error paths.  Every case prints its name,
seed and shapes before it touches the GPU."""
import sys

import numpy as np
import pytest

import oracle
from oracle import defn
from paper_2105_13678_amd import synth

pytestmark = pytest.mark.gpu

GAMMAS = (110503, 756839)  # two output classes
KMAX = 10


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


def session_seeds(seed, gamma, even_b=False):
    rng = synth.SplitMix64(seed)
    W = (gamma + 63) // 64
    a = rng.words(KMAX * W).reshape(KMAX, W)
    if gamma % 64:
        a[:, -1] &= np.uint64((1 << (gamma % 64)) - 1)
    a = a.reshape(-1).copy()
    b = synth.mask_tail(rng.words(W), gamma)
    b[0] |= np.uint64(1)
    if even_b:
        b[0] &= ~np.uint64(1)
    c = synth.mask_tail(rng.words(W), gamma)
    return a, b, c


def requests(seed, count, sessions):
    """(n, r, session, key) with r = n/10 and r in the range of one of the two
    output classes (so gamma is that class), k <= KMAX."""
    rng = synth.SplitMix64(seed)
    lows = {110503: 86244, 756839: 216092}
    out = []
    for i in range(count):
        g = GAMMAS[i % 2]
        u = rng.next_double()
        r = int(lows[g] + u * (g - 1 - lows[g]))
        n = 10 * r + int(rng.next_u64() % 10)
        assert defn.plan_shape(n, r)[1:] == (g, -(-n // g))
        key = synth.mask_tail(rng.words((n + 63) // 64), n)
        out.append((n, r, int(rng.next_u64() % sessions), key))
    return out


def single_block_out(pa, n, r, key, a, b, c):
    g = defn.plan_shape(n, r)[1]
    k = -(-n // g)
    W = (g + 63) // 64
    with pa.Plan(n, r) as plan:
        st, out = plan.hash(pa.to_device(key), pa.to_device(a[: k * W]), pa.to_device(b), pa.to_device(c))
    return st, pa.from_device(out)


def test_server_mix_equals_alone_and_single_block(pa):
    """Three sessions (session 2 has an even b), two output classes, 24
    requests submitted at once plus one all-ones key (RELOAD); then each
    request again on its own.  Outputs and statuses equal the single-block
    path's and the oracle's (every request, statuses included)."""
    seeds = {(s, g): session_seeds(100 + 10 * s + j, g, even_b=(s == 2)) for s in range(3)
             for j, g in enumerate(GAMMAS)}
    reqs = requests(41, 24, 3)
    n0, r0 = 950000, 95000
    ones = np.full((n0 + 63) // 64, np.uint64(0xFFFFFFFFFFFFFFFF), dtype=np.uint64)
    reqs.append((n0, r0, 0, synth.mask_tail(ones, n0)))
    say("[case] server mix:", [(n, r, s) for n, r, s, _ in reqs])
    with pa.Server(max_inflight=6, hbm_budget_bytes=4 << 30) as srv:
        for (s, g), (a, b, c) in seeds.items():
            assert srv.set_seeds(s, g, KMAX, a, b, c) == 0
        outs = [np.zeros((r + 63) // 64, dtype=np.uint64) for n, r, s, key in reqs]
        tickets = []
        for (n, r, s, key), out in zip(reqs, outs):
            st, t = srv.submit(n, r, s, key, out)
            assert st == 0
            tickets.append(t)
        mix = [srv.wait(t) for t in tickets]
        alone = []
        for n, r, s, key in reqs:
            out = np.zeros((r + 63) // 64, dtype=np.uint64)
            st, t = srv.submit(n, r, s, key, out)
            assert st == 0
            alone.append((srv.wait(t), out))
    for (n, r, s, key), out, (pst, res, tm), ((pst2, res2, _), out2) in zip(reqs, outs, mix, alone):
        assert pst == 0 and pst2 == 0
        g = defn.plan_shape(n, r)[1]
        st1, out1 = single_block_out(pa, n, r, key, *seeds[(s, g)])
        assert res == res2 == st1, (n, r, s, res, res2, st1)
        if res == 0:
            assert np.array_equal(out, out1) and np.array_equal(out2, out1), (n, r, s)
        assert tm["total_ms"] >= tm["queued_ms"] >= 0 and tm["device_ms"] > 0
    assert mix[-1][1] == 2  # the all-ones key reloads
    assert all(res == -5 for (n, r, s, key), (p, res, t) in zip(reqs, mix) if s == 2)
    for (n, r, s, key), out, (p, res, t) in zip(reqs, outs, mix):
        g = defn.plan_shape(n, r)[1]
        k = -(-n // g)
        a, b, c = seeds[(s, g)]
        st_o, out_o = oracle.hash(key, n, r, g, a[: k * ((g + 63) // 64)], b, c)
        assert st_o == res, (n, r, s, st_o, res)
        if st_o == 0:
            assert np.array_equal(out, out_o), (n, r, s)


def test_server_tight_budget_serialises_admission(pa):
    """A budget about the size of the largest request: admission waits for
    memory to free up, and every request still completes correctly (equal to
    the single-block path and to the oracle)."""
    seeds = {g: session_seeds(200 + j, g) for j, g in enumerate(GAMMAS)}
    reqs = requests(43, 8, 1)
    big = max(pa.plan_query(n, r)[1]["workspace_bytes"] for n, r, s, k in reqs)
    say("[case] server tight budget:", [(n, r) for n, r, s, _ in reqs], "budget", big)
    with pa.Server(max_inflight=4, hbm_budget_bytes=big) as srv:
        for g, (a, b, c) in seeds.items():
            assert srv.set_seeds(0, g, KMAX, a, b, c) == 0
        outs = [np.zeros((r + 63) // 64, dtype=np.uint64) for n, r, s, key in reqs]
        tickets = [srv.submit(n, r, 0, key, out)[1] for (n, r, s, key), out in zip(reqs, outs)]
        res = [srv.wait(t) for t in tickets]
    for (n, r, s, key), out, (p, st, tm) in zip(reqs, outs, res):
        g = defn.plan_shape(n, r)[1]
        st1, out1 = single_block_out(pa, n, r, key, *seeds[g])
        assert p == 0 and st == st1 == 0 and np.array_equal(out, out1)
        a, b, c = seeds[g]
        k = -(-n // g)
        st_o, out_o = oracle.hash(key, n, r, g, a[: k * ((g + 63) // 64)], b, c)
        assert st_o == 0 and np.array_equal(out, out_o), (n, r)


def test_server_errors(pa):
    say("[case] server error paths")
    a, b, c = session_seeds(300, GAMMAS[0])
    n, r = 1_000_000, 100_000
    key = np.zeros((n + 63) // 64, dtype=np.uint64)
    out = np.zeros((r + 63) // 64, dtype=np.uint64)
    with pa.Server(max_inflight=2, hbm_budget_bytes=64 << 20) as srv:
        assert srv.submit(n, r, 0, key, out)[0] == -1      # no seeds for (0, gamma): PA_ERR_ARG
        assert srv.set_seeds(0, 110501, KMAX, a, b, c) == -3  # not a Mersenne exponent: PA_ERR_GAMMA
        assert srv.set_seeds(0, GAMMAS[0], KMAX, a, b, c) == 0
        assert srv.set_seeds(0, GAMMAS[0], KMAX, a, b, c) == -9  # already resident: PA_ERR_BUSY
        assert srv.submit(n, 0, 0, key, out)[0] == -1      # r = 0: PA_ERR_ARG
        st, t = srv.submit(n, r, 0, key, out)
        assert st == 0
        assert srv.wait(t)[:2] == (0, 0)
        assert srv.poll(t)[0] == -1                         # reported once
        assert srv.poll(t + 1000)[0] == -1                  # unknown ticket
        big_n = 20 * 756839
        big_key = np.zeros((big_n + 63) // 64, dtype=np.uint64)
        big_out = np.zeros((big_n // 10 + 63) // 64, dtype=np.uint64)
        a2, b2, c2 = session_seeds(301, GAMMAS[1])
    with pa.Server(max_inflight=2, hbm_budget_bytes=1 << 20) as srv:
        assert srv.set_seeds(0, GAMMAS[1], KMAX, a2, b2, c2) == 0
        assert srv.submit(7_000_000, 700_000, 0, big_key, big_out)[0] == -10  # above the budget: PA_ERR_LIMIT
