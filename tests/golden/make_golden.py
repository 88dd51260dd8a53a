"""Write the stored expected values for the full-size parity cases.

Calls only the oracle (C oracle, cross-checked against the Python-int
definition with --check-defn) on the seeded synthetic inputs, and stores
digests of the outputs:

    python tests/golden/make_golden.py [--check-defn] [case ...]

Cases (splitmix64 seed, n, r): the 2^20-bit single block (seed 1, r = n/10),
the 2.6e8-bit single block (seed 2, r = n/10), the paper-shaped CV block n = 10 * 25,964,951 with compression
ratio 0.0972 (Table 3; seed 6), one chunk of the largest Mersenne exponent
(gamma = 136,279,841, r = 2^27, seed 7), whose products need the longest
transform (2^24 points), and single chunks of gamma = 37,156,667 and
74,207,281 (seeds 8 and 9; 2^22- and 2^23-point transforms).  Without case names every case is
recomputed; stored cases not named are kept.
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
}


def digest(words: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(words, dtype=np.uint64).tobytes()).hexdigest()


def main():
    check = "--check-defn" in sys.argv
    names = [a for a in sys.argv[1:] if not a.startswith("--")] or list(CASES)
    out = {}
    path = os.path.join(HERE, "full_size.json")
    if os.path.exists(path):
        out = json.load(open(path))
    for name in names:
        c = CASES[name]
        st, g, k = defn.plan_shape(c["n"], c["r"])
        blk = synth.single_block(c["seed"], c["n"], c["r"], g, k)
        t0 = time.time()
        s, z, y, U = oracle.hash(blk.key, c["n"], c["r"], g, blk.a, blk.b, blk.c, stages=True)
        dt = time.time() - t0
        rec = dict(c, gamma=g, k=k, status=int(s), out_sha256=digest(z), y_sha256=digest(y),
                   U_sha256=digest(U), out_head=[int(v) for v in z[:4]], out_tail=[int(v) for v in z[-4:]],
                   oracle_seconds=round(dt, 1), checked_against_definition=False)
        if check:
            s2, z2, y2, U2 = defn.hash_words(blk.key, c["n"], c["r"], g, blk.a, blk.b, blk.c)
            assert s2 == s and z2 == defn.words_to_int(z) and y2 == defn.words_to_int(y), name
            rec["checked_against_definition"] = True
        out[name] = rec
        print(name, json.dumps(rec), flush=True)
        json.dump(out, open(path, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
