"""Write the stored expected values for the full-size parity cases.

Calls only the oracle (C oracle, cross-checked against the Python-int
definition with --check-defn) on the seeded synthetic inputs, and stores
digests of the outputs:

    python tests/golden/make_golden.py [--check-defn] [--jobs J] [case ...]

Cases (splitmix64 seed, n, r): the 2^20-bit single block (seed 1, r = n/10),
the 2.6e8-bit single block (seed 2, r = n/10), the paper-shaped CV block n = 10 * 25,964,951 with compression
ratio 0.0972 (Table 3; seed 6), one chunk of the largest Mersenne exponent
(gamma = 136,279,841, r = 2^27, seed 7), whose products need the longest
transform (2^24 points), and single chunks of gamma = 37,156,667 and
74,207,281 (seeds 8 and 9; 2^22- and 2^23-point transforms), the paper's
largest CV block, 8e8 bits with r = n/10 (Sec. 4; seed 5, gamma = 82,589,933,
k = 10), the top corner of the uneven-batch range (n = 2^28 - 1,
r = 0.3 n; seed 10), and the uneven-batch draws: 16 blocks with n
log-uniform in [2^22, 2^28] and r/n uniform in [0.05, 0.30] (splitmix64
seed 3, drawn by synth.uneven_blocks; one record per block,
"batched_seed3_16/<i>"), 4 blocks from the top octave [2^27, 2^28]
(seed 15) and the 64-block draw of the batched benchmark (seed 3).  Without
case names every case is recomputed; stored cases not named are kept.  With
--jobs J the cases (and the blocks of the batch) run in J processes.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import defn  # noqa: E402
from paper_2105_13678_amd import synth  # noqa: E402

CASES = {
    "single_block_2p20": dict(seed=1, n=1 << 20, r=(1 << 20) // 10),
    "single_block_2p6e8": dict(seed=2, n=260_000_000, r=26_000_000),
    "paper_cv_block": dict(seed=6, n=10 * 25964951, r=int(math.floor(0.0972 * 10 * 25964951))),
    "max_length_single_chunk": dict(seed=7, n=136279841 - 1, r=1 << 27),
    "len_2p22_single_chunk": dict(seed=8, n=37156667 - 1, r=37156667 - 2),
    "len_2p23_single_chunk": dict(seed=9, n=74207281 - 1, r=74207281 - 2),
    "cv_8e8_block": dict(seed=5, n=800_000_000, r=80_000_000),
    "corner_2p28_r03": dict(seed=10, n=(1 << 28) - 1, r=int(0.3 * ((1 << 28) - 1))),
}
# The uneven-batch draws (one record per block): 16 blocks over the whole
# range, and 4 from its top octave [2^27, 2^28].
BATCH = {
    "batched_seed3_16": dict(seed=3, count=16, n_lo_log2=22, n_hi_log2=28, f_lo=0.05, f_hi=0.30),
    "batched_top_seed15_4": dict(seed=15, count=4, n_lo_log2=27, n_hi_log2=28, f_lo=0.05, f_hi=0.30),
    "batched_seed3_64": dict(seed=3, count=64, n_lo_log2=22, n_hi_log2=28, f_lo=0.05, f_hi=0.30),
}


def digest(words: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(words, dtype=np.uint64).tobytes()).hexdigest()


def _shape(n, r):
    st, g, k = defn.plan_shape(n, r)
    assert st == 0
    return g, k


def batch_blocks(name):
    b = BATCH[name]
    return synth.uneven_blocks(b["seed"], b["count"], _shape, b["n_lo_log2"], b["n_hi_log2"], b["f_lo"], b["f_hi"])


def _record(task):
    """Oracle record of one task: (case name, None) or (batch name, block index)."""
    name, idx, check = task
    if idx is None:
        c = CASES[name]
        g, k = _shape(c["n"], c["r"])
        blk = synth.single_block(c["seed"], c["n"], c["r"], g, k)
        rec = dict(c, gamma=g, k=k)
        key = name
    else:
        blk = batch_blocks(name)[idx]
        rec = dict(BATCH[name], index=idx, n=blk.n, r=blk.r, gamma=blk.gamma, k=blk.k)
        key = f"{name}/{idx}"
    t0 = time.time()
    s, z, y, U = oracle.hash(blk.key, blk.n, blk.r, blk.gamma, blk.a, blk.b, blk.c, stages=True)
    dt = time.time() - t0
    rec.update(status=int(s), out_sha256=digest(z), y_sha256=digest(y), U_sha256=digest(U),
               out_head=[int(v) for v in z[:4]], out_tail=[int(v) for v in z[-4:]],
               oracle_seconds=round(dt, 1), checked_against_definition=False)
    if check:
        s2, z2, y2, U2 = defn.hash_words(blk.key, blk.n, blk.r, blk.gamma, blk.a, blk.b, blk.c)
        assert s2 == s and z2 == defn.words_to_int(z) and y2 == defn.words_to_int(y), key
        rec["checked_against_definition"] = True
    return key, rec


def main():
    check = "--check-defn" in sys.argv
    jobs = 1
    args = sys.argv[1:]
    if "--jobs" in args:
        i = args.index("--jobs")
        jobs = int(args[i + 1])
        del args[i:i + 2]
    names = [a for a in args if not a.startswith("--")] or list(CASES) + list(BATCH)
    tasks = []
    for name in names:
        if name in BATCH:
            tasks += [(name, i, check) for i in range(BATCH[name]["count"])]
        else:
            tasks.append((name, None, check))
    path = os.path.join(HERE, "full_size.json")

    def store(key, rec):
        # read, update and atomically replace: records other runs wrote meanwhile are kept
        out = json.load(open(path)) if os.path.exists(path) else {}
        out[key] = rec
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(out, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
        print(key, json.dumps(rec), flush=True)

    if jobs > 1:
        import multiprocessing as mp
        with mp.Pool(jobs) as pool:
            for key, rec in pool.imap_unordered(_record, tasks):
                store(key, rec)
    else:
        for task in tasks:
            store(*_record(task))


if __name__ == "__main__":
    main()
