"""Build libpa.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2105_13678_amd.build          # compile
    python -m paper_2105_13678_amd.build --asm    # also dump the gfx950 assembly

The library lands next to this file as ``libpa.so``; the Python binding loads
it from there.  Packed FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpa.so")
ARCH = "gfx950"

SOURCES = ["pa_api.cpp", "pa_batch.cpp", "pa_server.cpp", "pa_tune.cpp", "pa_kernels.hip", "pa_noalloc.hip",
           "pa_probe.hip"]
HEADERS = ["pa_internal.hpp", "ntt_device.hpp", "pa_multi.hpp", "pa_resident.hpp"]
DEVICE_SOURCES = ["pa_kernels.hip", "ntt_device.hpp", "pa_multi.hpp"]


def _code_only(text: str) -> str:
    """The source with comments removed and white space collapsed (the device
    sources hold no string literals), so that edits of comments alone keep
    the digest."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_digest() -> str:
    """sha256 over the code of libpa's device sources (comments and white
    space ignored): identifies the kernels a set of profiler counters was
    taken on."""
    import hashlib
    h = hashlib.sha256()
    for name in DEVICE_SOURCES:
        with open(os.path.join(CSRC, name), encoding="utf-8") as fh:
            h.update(name.encode() + b"\0" + _code_only(fh.read()).encode())
    return h.hexdigest()


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libpa)")


def flags() -> list[str]:
    return [
        "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I" + INCLUDE, "-I" + CSRC,
        "-Wall", "-Wno-unused-function",
    ]


def build(verbose: bool = False) -> str:
    """Compile every source and link libpa.so; always recompiles."""
    cc = hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [cc, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + flags()
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def dump_asm(out_dir: str) -> None:
    """Write the gfx950 device assembly of each .hip source to out_dir."""
    cc = hipcc()
    os.makedirs(out_dir, exist_ok=True)
    for src in SOURCES:
        if not src.endswith(".hip"):
            continue
        out = os.path.join(out_dir, os.path.splitext(src)[0] + ".s")
        subprocess.check_call([cc, "-x", "hip", "-S", "--cuda-device-only", os.path.join(CSRC, src),
                               "-o", out] + flags())


if __name__ == "__main__":
    print(build(verbose=True))
    if "--asm" in sys.argv:
        dump_asm(os.path.join(ROOT, "build", "asm"))  # build/ is not tracked
