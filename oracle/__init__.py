"""CPU oracle for the MMH-MH privacy-amplification hash.

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's CPU
baseline leg may import this package; the product path (the HIP library and its
Python binding) never does, and shares no code with it.

Two independent evaluations of the same definition (arXiv 2105.13678,
Algorithm 1 with MMH eq. (2) and MH eq. (4)):
  * ``defn``  -- Python arbitrary-precision ints, the definition written out;
  * ``hash``  -- plain C (schoolbook + Karatsuba products, fold mod 2^gamma-1),
                 fast enough for the full-size workloads.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import defn  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pa_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, RELOAD = 0, 2


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.oracle_plan.argtypes = [ctypes.c_uint64] * 3 + [u64p, u64p]
        lib.oracle_plan.restype = ctypes.c_int
        lib.oracle_hash.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.c_uint64] + [ctypes.c_void_p] * 6
        lib.oracle_hash.restype = ctypes.c_int
        lib.oracle_hash_threads.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                            ctypes.c_uint64] + [ctypes.c_void_p] * 6 + [ctypes.c_int]
        lib.oracle_hash_threads.restype = ctypes.c_int
        lib.oracle_mul.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                   ctypes.c_void_p]
        lib.oracle_mul.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def plan(n: int, r: int, gamma: int = 0):
    """(status, gamma, k) from the C oracle's own plan rule."""
    g = ctypes.c_uint64(0)
    k = ctypes.c_uint64(0)
    st = _load().oracle_plan(n, r, gamma, ctypes.byref(g), ctypes.byref(k))
    return st, g.value, k.value


def hash(key, n: int, r: int, gamma: int, a, b, c, stages: bool = False, threads: int = 1):
    """Evaluate the hash with the C oracle.

    key: ceil(n/64) uint64 words; a: k*W words; b, c: W words, W = ceil(gamma/64).
    Returns (status, out) or, with ``stages``, (status, out, y, U) where out is
    ceil(r/64) uint64 words and y, U are W-word arrays.  threads > 1 spreads
    the k products of the MMH sum over that many threads (same result)."""
    W = (gamma + 63) // 64
    key = np.ascontiguousarray(key, dtype=np.uint64)
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    c = np.ascontiguousarray(c, dtype=np.uint64)
    out = np.zeros((r + 63) // 64, dtype=np.uint64)
    y = np.zeros(W, dtype=np.uint64) if stages else None
    U = np.zeros(W, dtype=np.uint64) if stages else None
    if threads > 1:
        st = _load().oracle_hash_threads(_ptr(key), n, r, gamma, _ptr(a), _ptr(b), _ptr(c), _ptr(out),
                                         _ptr(y), _ptr(U), int(threads))
    else:
        st = _load().oracle_hash(_ptr(key), n, r, gamma, _ptr(a), _ptr(b), _ptr(c), _ptr(out),
                                 _ptr(y), _ptr(U))
    if stages:
        return st, out, y, U
    return st, out


def mul(a, b):
    """Exact product of two equal-length word arrays (2n words)."""
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    assert a.shape == b.shape
    out = np.zeros(2 * len(a), dtype=np.uint64)
    if _load().oracle_mul(_ptr(a), _ptr(b), len(a), _ptr(out)):
        raise MemoryError("oracle_mul")
    return out
