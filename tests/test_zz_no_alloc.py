"""pa_hash_noalloc (the entry point that allocates nothing) against
pa_hash_async (the plan-based entry point) and the CPU oracle, bit for bit,
on consecutive calls that share the library's static device array: a block,
then a smaller one of another transform length, then two more of the first
length (the tables rebuilt once, then reused from the array).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2105_13678_amd import synth

pytestmark = pytest.mark.gpu


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


def _inputs(pa, seed, n, r):
    st, info = pa.plan_query(n, r)
    assert st == 0
    blk = synth.single_block(seed, n, r, info["gamma"], info["k"])
    dev = [pa.to_device(x, "cuda:0") for x in (blk.key, blk.a, blk.b, blk.c)]
    return blk, info, dev


def test_noalloc_matches_plan_entry_point(pa):
    import torch
    from paper_2105_13678_amd import binding
    cases = [(41, 1 << 20, (1 << 20) // 10), (42, 300_007, 29_000), (43, 1 << 20, (1 << 20) // 10),
             (44, (1 << 20) - 77, 100_003)]
    prev_N = None
    for seed, n, r in cases:
        blk, info, (key, a, b, c) = _inputs(pa, seed, n, r)
        say(f"[case] noalloc seed={seed} n={n} r={r} gamma={info['gamma']} k={info['k']} N={info['N']} "
            f"tables={'reused' if info['N'] == prev_N else 'built'}")
        prev_N = info["N"]
        out_na = torch.full((info["out_words"],), -1, dtype=torch.int64, device="cuda:0")
        st_na = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
        st = binding.hash_noalloc(n, r, key, a, b, c, out_na, st_na)
        assert st == pa.PA_OK, pa.status_string(st)
        torch.cuda.synchronize()
        got_status = pa.decode_status(int(st_na.cpu().numpy().view(np.uint32)[0]))
        got = pa.from_device(out_na)

        with pa.Plan(n, r) as plan:
            out_p = torch.full((info["out_words"],), -1, dtype=torch.int64, device="cuda:0")
            st_p = torch.full((1,), -1, dtype=torch.int32, device="cuda:0")
            plan.hash_async(key, a, b, c, out_p, st_p)
            torch.cuda.synchronize()
            want_status = pa.decode_status(int(st_p.cpu().numpy().view(np.uint32)[0]))
            want = pa.from_device(out_p)
        assert got_status == want_status == pa.PA_OK, (got_status, want_status)
        assert np.array_equal(got, want), f"noalloc differs from pa_hash_async (seed {seed})"
        st_o, out_o = oracle.hash(blk.key, n, r, info["gamma"], blk.a, blk.b, blk.c)
        assert st_o == 0 and np.array_equal(got, out_o), f"noalloc differs from the oracle (seed {seed})"


def test_noalloc_rejects_oversized_and_bad_arguments(pa):
    import torch
    from paper_2105_13678_amd import binding
    lib = binding.lib()
    n, r = 1 << 25, (1 << 25) // 10
    st, info = pa.plan_query(n, r)
    assert st == 0 and info["workspace_bytes"] + 256 > binding.NOALLOC_MAX_BYTES
    say(f"[case] noalloc limit n={n} r={r} workspace={info['workspace_bytes']}")
    dummy = torch.zeros(8, dtype=torch.int64, device="cuda:0")
    prm = binding.Params(n, r, 0, 0, 0, 0, 0)
    p = dummy.data_ptr()
    assert lib.pa_hash_noalloc(binding.ctypes.byref(prm), 0, p, p, p, p, p, p, None) == binding.PA_ERR_LIMIT
    prm = binding.Params(1 << 20, (1 << 20) // 10, 0, 0, 0, 0, 0)
    assert lib.pa_hash_noalloc(binding.ctypes.byref(prm), 0, p, p, p, p, p, None, None) == binding.PA_ERR_ARG
    assert lib.pa_hash_noalloc(binding.ctypes.byref(prm), 64, p, p, p, p, p, p, None) == binding.PA_ERR_ARG
    prm = binding.Params(100, 200, 0, 0, 0, 0, 0)
    assert lib.pa_hash_noalloc(binding.ctypes.byref(prm), 0, p, p, p, p, p, p, None) == binding.PA_ERR_ARG
