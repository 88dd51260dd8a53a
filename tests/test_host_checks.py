"""Host-side checks under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

* The serving loop's resident-set accounting (pa_resident.hpp) driven by
  tests/host/resident_cache_check.cpp, built with g++ and both sanitizers.
* The batched path's multi-block launch tables and lookup (pa_multi.hpp)
  driven by tests/host/multi_launch_check.cpp.
* The host C++ of libpa (plan rule, batch, server, tuner, the launchers'
  host code) built with both sanitizers on the host side only and loaded
  into a child Python process: the plan rule over random shapes and every
  error path must give the same results as the regular library, with no
  sanitizer report.  No kernel runs (no GPU here).
"""
import glob
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2105_13678_amd", "csrc")
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def test_resident_cache_accounting(tmp_path):
    exe = str(tmp_path / "resident_cache_check")
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", *SAN, "-I" + CSRC, "-o", exe,
                           os.path.join(HERE, "host", "resident_cache_check.cpp")])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok"), out.stdout + out.stderr


def test_multi_launch_tables(tmp_path):
    """The batched path's multi-block launch tables and the lookup its kernels
    run (pa_multi.hpp), built with hipcc (host code under both sanitizers)."""
    sys.path.insert(0, ROOT)
    from paper_2105_13678_amd import build as b
    exe = str(tmp_path / "multi_launch_check")
    cmd = [b.hipcc(), "-x", "hip", f"--offload-arch={b.ARCH}", "-std=c++17", "-O1", "-g", "-I" + CSRC, "-o", exe,
           os.path.join(HERE, "host", "multi_launch_check.cpp")]
    for flag in SAN:
        cmd += ["-Xarch_host", flag]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok"), out.stdout + out.stderr


def _asan_runtime():
    cands = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return cands[-1] if cands else None


CHILD = r"""
import json, random, sys
sys.path.insert(0, sys.argv[1])
from paper_2105_13678_amd import binding
cases = json.loads(sys.stdin.read())
out = []
for n, r, g, B, f, c in cases:
    st, info = binding.plan_query(n, r, g, B, f, c)
    out.append([st, None if info is None else [info[k] for k in sorted(info) if k != "exact_log2"]])
lib = binding.lib()
names = [lib.pa_status_string(s).decode() for s in range(-11, 3)]
print(json.dumps({"plans": out, "names": names, "decode": [binding.decode_status(x) for x in range(8)]}))
"""


@pytest.mark.slow
def test_host_library_under_sanitizers(tmp_path):
    asan = _asan_runtime()
    if asan is None:
        pytest.skip("no clang AddressSanitizer runtime in this ROCm")
    sys.path.insert(0, ROOT)
    from paper_2105_13678_amd import build as b
    pkg = tmp_path / "paper_2105_13678_amd"
    pkg.mkdir()
    for f in ("__init__.py", "binding.py", "synth.py"):
        with open(os.path.join(ROOT, "paper_2105_13678_amd", f)) as src, open(pkg / f, "w") as dst:
            dst.write(src.read())
    (tmp_path / "include").mkdir()
    with open(os.path.join(ROOT, "include", "pa.h")) as src, open(tmp_path / "include" / "pa.h", "w") as dst:
        dst.write(src.read())
    objs, procs = [], []
    for s in b.SOURCES:  # compiled side by side
        obj = str(tmp_path / (s + ".o"))
        cmd = [b.hipcc(), "-x", "hip", "-c", os.path.join(CSRC, s), "-o", obj, "-g"]
        for flag in SAN:  # host code only: the device code is built as usual
            cmd += ["-Xarch_host", flag]
        procs.append(subprocess.Popen(cmd + b.flags(), stderr=subprocess.DEVNULL))
        objs.append(obj)
    assert all(p.wait() == 0 for p in procs)
    lib = str(pkg / "libpa.so")
    link = [b.hipcc(), "-shared", "-fPIC", f"--offload-arch={b.ARCH}", "-o", lib] + objs
    for flag in SAN[:2]:
        link += ["-Xarch_host", flag]
    subprocess.check_call(link)

    import random
    rng = random.Random(99)
    from oracle import defn
    cases = []
    for _ in range(3000):
        g = rng.choice(defn.MERSENNE_EXPONENTS)
        r = rng.randrange(1, max(2, g))
        n = rng.randrange(r + 1, r + 2 + rng.choice([10, 1000, 10 ** 6, 10 ** 9, 1 << 33]))
        cases.append([n, r, rng.choice([0, 0, g]), rng.choice([0, 0, 0, 8, 13, 29, 32, 33, 7]),
                      rng.choice([0, 0, 1, 2, 3]), rng.choice([0, 0, 0, 2, 5, 15])])
    cases += [[0, 0, 0, 0, 0, 0], [10, 20, 0, 0, 0, 0], [1 << 32, (1 << 32) // 10, 0, 0, 0, 0]]
    payload = json.dumps(cases)

    def run(root, preload):
        env = dict(os.environ)
        if preload:
            env["LD_PRELOAD"] = preload
            env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
            env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
        res = subprocess.run([sys.executable, "-c", CHILD, root], input=payload, capture_output=True, text=True,
                             env=env, timeout=600)
        assert res.returncode == 0, res.stderr[-4000:]
        assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr[-4000:]
        return json.loads(res.stdout.strip().splitlines()[-1])

    want = run(ROOT, None)
    got = run(str(tmp_path), asan)
    assert got == want
