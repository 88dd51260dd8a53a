"""ctypes binding of libpa (include/pa.h).  Argument marshalling only: every
step of the hash runs in the HIP library; if the library is missing this
module raises instead of computing anything itself.

Device buffers are torch tensors (any 8-byte dtype, contiguous, on the plan's
device); torch supplies memory and the current HIP stream, nothing else.
"""
from __future__ import annotations

import ctypes
import functools
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpa.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pa.h")

PA_OK, PA_PENDING, PA_RELOAD = 0, 1, 2
PA_ERR_ARG, PA_ERR_NO_GAMMA, PA_ERR_GAMMA, PA_ERR_INEXACT = -1, -2, -3, -4
PA_ERR_SEED_B_EVEN, PA_ERR_SEED_RANGE, PA_ERR_NOMEM, PA_ERR_DEVICE = -5, -6, -7, -8
PA_ERR_BUSY, PA_ERR_LIMIT = -9, -10
PA_FLAG_POW2_LENGTHS = 1  # pa_params.flags: power-of-two transform lengths only
PA_FLAG_RADIX3_LENGTHS = 2  # pa_params.flags: lengths 3 * 2^m only
PA_FLAG_RADIX5_LENGTHS = 4  # pa_params.flags: lengths 5 * 2^m only (m <= 20)

# pa_phase, in order
PHASES = ["prologue", "mmh_col", "mmh_row", "mmh_colinv", "fold", "mh_col", "mh_row", "mh_colinv",
          "mh_carry", "finish"]
PROFILE_ALL = (1 << len(PHASES)) - 1


class PAError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})" if what else status_string(status))


class Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("r", ctypes.c_uint64), ("gamma", ctypes.c_uint64),
                ("B", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("col_lg", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("r", ctypes.c_uint64), ("gamma", ctypes.c_uint64),
                ("k", ctypes.c_uint64), ("B", ctypes.c_uint32), ("log2N", ctypes.c_uint32),
                ("L", ctypes.c_uint64), ("N", ctypes.c_uint64), ("key_words", ctypes.c_uint64),
                ("seed_words", ctypes.c_uint64), ("a_words", ctypes.c_uint64),
                ("out_words", ctypes.c_uint64), ("workspace_bytes", ctypes.c_uint64),
                ("exact_log2", ctypes.c_double), ("log2N1", ctypes.c_uint32),
                ("log2N2", ctypes.c_uint32), ("nprimes", ctypes.c_uint32), ("primes", ctypes.c_uint32 * 3),
                ("len_factor", ctypes.c_uint32), ("col_lg", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["primes"] = list(self.primes)
        return d


_lib = None
_VP = ctypes.c_void_p


class ServerCfg(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("max_inflight", ctypes.c_uint32), ("hbm_budget_bytes", ctypes.c_uint64),
                ("resident_budget_bytes", ctypes.c_uint64)]


class Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("r", ctypes.c_uint64), ("session", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("key", _VP), ("out", _VP)]


class Timing(ctypes.Structure):
    _fields_ = [("queued_ms", ctypes.c_double), ("device_ms", ctypes.c_double), ("total_ms", ctypes.c_double)]


class Block(ctypes.Structure):
    """pa_block: one block of a batched call (device pointers)."""
    _fields_ = [("n", ctypes.c_uint64), ("r", ctypes.c_uint64), ("key", _VP), ("a", _VP), ("b", _VP),
                ("c", _VP), ("out", _VP)]


def lib():
    """Load libpa.so (built in-tree); raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2105_13678_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        L.pa_plan_create.argtypes = [ctypes.POINTER(Params), ctypes.c_int, ctypes.POINTER(_VP)]
        L.pa_plan_create.restype = ctypes.c_int
        L.pa_plan_query.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(PlanInfo)]
        L.pa_plan_query.restype = ctypes.c_int
        L.pa_plan_get_info.argtypes = [_VP, ctypes.POINTER(PlanInfo)]
        L.pa_plan_get_info.restype = ctypes.c_int
        L.pa_plan_destroy.argtypes = [_VP]
        L.pa_plan_destroy.restype = None
        L.pa_hash.argtypes = [_VP] * 7
        L.pa_hash.restype = ctypes.c_int
        L.pa_hash_async.argtypes = [_VP] * 8
        L.pa_hash_async.restype = ctypes.c_int
        L.pa_hash_stages.argtypes = [_VP] * 9
        L.pa_hash_stages.restype = ctypes.c_int
        L.pa_hash_noalloc.argtypes = [ctypes.POINTER(Params), ctypes.c_int] + [_VP] * 7
        L.pa_hash_noalloc.restype = ctypes.c_int
        L.pa_plan_fill_scratch.argtypes = [_VP, ctypes.c_uint32, _VP]
        L.pa_plan_fill_scratch.restype = ctypes.c_int
        L.pa_plan_set_profiling.argtypes = [_VP, ctypes.c_uint32]
        L.pa_plan_set_profiling.restype = ctypes.c_int
        L.pa_plan_read_profile.argtypes = [_VP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint64)]
        L.pa_plan_read_profile.restype = ctypes.c_int
        L.pa_batch_plan_create.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(_VP)]
        L.pa_batch_plan_create.restype = ctypes.c_int
        L.pa_batch_plan_destroy.argtypes = [_VP]
        L.pa_batch_plan_destroy.restype = None
        L.pa_hash_batched.argtypes = [_VP, ctypes.POINTER(Block), ctypes.c_uint32, ctypes.POINTER(ctypes.c_int), _VP]
        L.pa_hash_batched.restype = ctypes.c_int
        L.pa_plan_tune.argtypes = [ctypes.POINTER(Params), ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(Params),
                                   ctypes.POINTER(ctypes.c_double)]
        L.pa_plan_tune.restype = ctypes.c_int
        L.pa_batch_plan_tune.argtypes = [_VP, ctypes.POINTER(Block), ctypes.c_uint32, ctypes.c_uint32,
                                         ctypes.POINTER(ctypes.c_uint32)]
        L.pa_batch_plan_tune.restype = ctypes.c_int
        L.pa_batch_plan_set_graphs.argtypes = [_VP, ctypes.c_int]
        L.pa_batch_plan_set_graphs.restype = ctypes.c_int
        L.pa_server_create.argtypes = [ctypes.POINTER(ServerCfg), ctypes.POINTER(_VP)]
        L.pa_server_create.restype = ctypes.c_int
        L.pa_server_destroy.argtypes = [_VP]
        L.pa_server_destroy.restype = None
        L.pa_server_set_seeds.argtypes = [_VP, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, _VP, _VP, _VP]
        L.pa_server_set_seeds.restype = ctypes.c_int
        L.pa_submit.argtypes = [_VP, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
        L.pa_submit.restype = ctypes.c_int
        L.pa_poll.argtypes = [_VP, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(Timing)]
        L.pa_poll.restype = ctypes.c_int
        L.pa_probe_valu.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.pa_probe_valu.restype = ctypes.c_int
        L.pa_probe_goldilocks.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double)]
        L.pa_probe_goldilocks.restype = ctypes.c_int
        L.pa_decode_status.argtypes = [ctypes.c_uint32]
        L.pa_decode_status.restype = ctypes.c_int
        L.pa_status_string.argtypes = [ctypes.c_int]
        L.pa_status_string.restype = ctypes.c_char_p
        _lib = L
    return _lib


def header_functions() -> list[str]:
    """Names of the functions include/pa.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(pa_[a-z_0-9]+)\s*\(", text, flags=re.M)


def status_string(status: int) -> str:
    try:
        return lib().pa_status_string(int(status)).decode()
    except RuntimeError:
        return f"status {status}"


def decode_status(flags: int) -> int:
    return lib().pa_decode_status(int(flags) & 0xFFFFFFFF)


def plan_query(n: int, r: int, gamma: int = 0, B: int = 0, flags: int = 0, col_lg: int = 0):
    """(status, info dict or None): the shape pa_plan_create would use."""
    prm = Params(n, r, gamma, B, flags, col_lg, 0)
    info = PlanInfo()
    st = lib().pa_plan_query(ctypes.byref(prm), ctypes.byref(info))
    return st, (info.as_dict() if st == PA_OK else None)


def probe_valu(device: int = 0):
    """pa_probe_valu: (butterflies per second, plain lane instructions per
    second) that register-only probe kernels reach on the device."""
    b, p = ctypes.c_double(), ctypes.c_double()
    st = lib().pa_probe_valu(int(device), ctypes.byref(b), ctypes.byref(p))
    if st != PA_OK:
        raise PAError(st, "pa_probe_valu")
    return b.value, p.value


def probe_goldilocks(device: int = 0):
    """pa_probe_goldilocks: (butterflies per second with a general twiddle
    product, with shift twiddles) modulo 2^64 - 2^32 + 1."""
    m, s = ctypes.c_double(), ctypes.c_double()
    st = lib().pa_probe_goldilocks(int(device), ctypes.byref(m), ctypes.byref(s))
    if st != PA_OK:
        raise PAError(st, "pa_probe_goldilocks")
    return m.value, s.value


def plan_tune(n: int, r: int, reps: int = 5, device: int = 0, gamma: int = 0, B: int = 0, flags: int = 0,
              col_lg: int = 0):
    """Time the candidate shapes of (n, r) on the device (pa_plan_tune);
    returns (params dict with B, flags and col_lg set, ms per hash)."""
    prm = Params(n, r, gamma, B, flags, col_lg, 0)
    best = Params()
    ms = ctypes.c_double()
    st = lib().pa_plan_tune(ctypes.byref(prm), int(device), int(reps), ctypes.byref(best), ctypes.byref(ms))
    if st != PA_OK:
        raise PAError(st, "pa_plan_tune")
    return {name: getattr(best, name) for name, _ in Params._fields_ if name != "reserved"}, ms.value


@functools.lru_cache(maxsize=4096)
def _buffer_words(n: int, r: int):
    """(key, a, seed, out) buffer words of shape (n, r) under the default plan
    rule, or None when it admits no plan (a pure function of (n, r))."""
    st, info = plan_query(n, r)
    if st != PA_OK:
        return None
    return info["key_words"], info["a_words"], info["seed_words"], info["out_words"]


def _dev_ptr(t, min_words: int, what: str, device) -> int:
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor")
    if t.device.type != "cuda" or (device is not None and t.device != device):
        raise ValueError(f"{what}: must live on {device}")
    if t.element_size() != 8 or not t.is_contiguous():
        raise ValueError(f"{what}: must be a contiguous 8-byte-element tensor")
    if t.numel() < min_words:
        raise ValueError(f"{what}: needs at least {min_words} words, got {t.numel()}")
    return t.data_ptr()


class Plan:
    """One (n, r) shape on one GPU; owns its device workspace."""

    def __init__(self, n: int, r: int, gamma: int = 0, B: int = 0, device: int = 0, flags: int = 0,
                 col_lg: int = 0):
        import torch
        self._h = _VP()
        self.device = torch.device("cuda", device)
        prm = Params(n, r, gamma, B, flags, col_lg, 0)
        st = lib().pa_plan_create(ctypes.byref(prm), int(device), ctypes.byref(self._h))
        if st != PA_OK:
            self._h = _VP()
            raise PAError(st, "pa_plan_create")
        info = PlanInfo()
        lib().pa_plan_get_info(self._h, ctypes.byref(info))
        self.info = info.as_dict()

    def __getattr__(self, name):
        info = self.__dict__.get("info")
        if info is not None and name in info:
            return info[name]
        raise AttributeError(name)

    def close(self):
        if self._h:
            lib().pa_plan_destroy(self._h)
            self._h = _VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _stream(self, stream):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return s.cuda_stream

    def _args(self, key, a, b, c, out):
        i = self.info
        return (_dev_ptr(key, i["key_words"], "key", self.device),
                _dev_ptr(a, i["a_words"], "a", self.device),
                _dev_ptr(b, i["seed_words"], "b", self.device),
                _dev_ptr(c, i["seed_words"], "c", self.device),
                _dev_ptr(out, i["out_words"], "out", self.device))

    def set_profiling(self, phases):
        """Time the given phases (names from PHASES, or "all"; empty = off)."""
        mask = PROFILE_ALL if phases == "all" else sum(1 << PHASES.index(p) for p in phases)
        st = lib().pa_plan_set_profiling(self._h, mask)
        if st != PA_OK:
            raise PAError(st, "pa_plan_set_profiling")

    def read_profile(self) -> dict:
        """{phase: mean ms per call} over the calls since the last read (phases
        not recorded are omitted); waits for the recorded events."""
        ms = (ctypes.c_double * len(PHASES))()
        n = (ctypes.c_uint64 * len(PHASES))()
        st = lib().pa_plan_read_profile(self._h, ms, n)
        if st != PA_OK:
            raise PAError(st, "pa_plan_read_profile")
        return {PHASES[i]: ms[i] / n[i] for i in range(len(PHASES)) if n[i]}

    def new_out(self):
        import torch
        return torch.zeros(self.info["out_words"], dtype=torch.int64, device=self.device)

    def hash(self, key, a, b, c, out=None, stream=None):
        """Blocking hash; returns (status, out)."""
        if out is None:
            out = self.new_out()
        args = self._args(key, a, b, c, out)
        st = lib().pa_hash(self._h, *args, self._stream(stream))
        return st, out

    def hash_async(self, key, a, b, c, out, d_status, stream=None):
        """Enqueue only; status flags land in the 1-word device tensor d_status."""
        import torch
        args = self._args(key, a, b, c, out)
        if d_status.device != self.device or d_status.numel() < 1:
            raise ValueError("d_status must be a device tensor")
        st = lib().pa_hash_async(self._h, *args, d_status.data_ptr(), self._stream(stream))
        if st != PA_OK:
            raise PAError(st, "pa_hash_async")
        return out

    def hash_stages(self, key, a, b, c, out=None, stream=None):
        """Blocking hash that also returns the stage values (status, out, y, U)."""
        import torch
        if out is None:
            out = self.new_out()
        W = self.info["seed_words"]
        y = torch.zeros(W, dtype=torch.int64, device=self.device)
        U = torch.zeros(W, dtype=torch.int64, device=self.device)
        args = self._args(key, a, b, c, out)
        st = lib().pa_hash_stages(self._h, *args, y.data_ptr(), U.data_ptr(), self._stream(stream))
        return st, out, y, U

    def fill_scratch(self, word: int, stream=None) -> int:
        """pa_plan_fill_scratch: fill the plan's scratch memory with a 32-bit
        pattern (enqueued on the stream; a debug aid for determinism tests)."""
        return lib().pa_plan_fill_scratch(self._h, int(word) & 0xFFFFFFFF, self._stream(stream))


NOALLOC_MAX_BYTES = 64 << 20  # PA_NOALLOC_MAX_BYTES


def hash_noalloc(n: int, r: int, key, a, b, c, out, d_status, device: int = 0, gamma: int = 0, B: int = 0,
                 flags: int = 0, col_lg: int = 0, stream=None) -> int:
    """pa_hash_noalloc: enqueue the hash of one block without a plan and
    without any allocation (the library's static device array holds every
    buffer); status flags land in the 1-word device tensor d_status.
    Returns the call's status (host-side errors only)."""
    import torch
    st, info = plan_query(n, r, gamma, B, flags, col_lg)
    if st != PA_OK:
        return st
    dev = torch.device("cuda", device)
    args = (_dev_ptr(key, info["key_words"], "key", dev), _dev_ptr(a, info["a_words"], "a", dev),
            _dev_ptr(b, info["seed_words"], "b", dev), _dev_ptr(c, info["seed_words"], "c", dev),
            _dev_ptr(out, info["out_words"], "out", dev))
    if d_status.device != dev or d_status.numel() < 1:
        raise ValueError("d_status must be a device tensor")
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    prm = Params(n, r, gamma, B, flags, col_lg, 0)
    return lib().pa_hash_noalloc(ctypes.byref(prm), int(device), *args, d_status.data_ptr(), s.cuda_stream)


class BatchPlan:
    """Batched hashing of blocks of uneven (n, r) on one GPU (pa_hash_batched)."""

    def __init__(self, max_blocks: int, max_total_bits: int, device: int = 0):
        import torch
        self._h = _VP()
        self.device = torch.device("cuda", device)
        self.max_blocks = max_blocks
        st = lib().pa_batch_plan_create(int(max_blocks), int(max_total_bits), int(device), ctypes.byref(self._h))
        if st != PA_OK:
            self._h = _VP()
            raise PAError(st, "pa_batch_plan_create")

    def close(self):
        if self._h:
            lib().pa_batch_plan_destroy(self._h)
            self._h = _VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @staticmethod
    def new_out(r: int, device):
        import torch
        return torch.zeros((r + 63) // 64, dtype=torch.int64, device=device)

    def hash(self, blocks, stream=None):
        """blocks: sequence of (n, r, key, a, b, c, out) with device tensors.
        Returns (call status, [per-block status]).  Buffer sizes are checked
        against each block's plan; a block whose (n, r) admits no plan is
        passed through and gets its plan error in the per-block status."""
        import torch
        arr = (Block * len(blocks))()
        for i, (n, r, key, a, b, c, out) in enumerate(blocks):
            w = _buffer_words(n, r)
            if w is not None:
                ptrs = (_dev_ptr(key, w[0], "key", self.device), _dev_ptr(a, w[1], "a", self.device),
                        _dev_ptr(b, w[2], "b", self.device), _dev_ptr(c, w[2], "c", self.device),
                        _dev_ptr(out, w[3], "out", self.device))
            else:
                ptrs = tuple(t.data_ptr() if t is not None else 0 for t in (key, a, b, c, out))
            arr[i] = Block(n, r, *ptrs)
        per = (ctypes.c_int * len(blocks))()
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        st = lib().pa_hash_batched(self._h, arr, len(blocks), per, s.cuda_stream)
        return st, list(per)

    def set_graphs(self, enable: bool = True):
        """Capture block lists into HIP graphs and replay them (pa_batch_plan_set_graphs)."""
        st = lib().pa_batch_plan_set_graphs(self._h, 1 if enable else 0)
        if st != PA_OK:
            raise PAError(st, "pa_batch_plan_set_graphs")

    def tune(self, blocks, reps: int = 5) -> int:
        """Autotune the (gamma, k) classes of blocks (sequence of (n, r, ...);
        only n and r are read) for later hash calls; returns the number of
        classes tuned now (pa_batch_plan_tune)."""
        arr = (Block * len(blocks))()
        for i, blk in enumerate(blocks):
            arr[i] = Block(blk[0], blk[1], 0, 0, 0, 0, 0)
        tuned = ctypes.c_uint32()
        st = lib().pa_batch_plan_tune(self._h, arr, len(blocks), int(reps), ctypes.byref(tuned))
        if st != PA_OK:
            raise PAError(st, "pa_batch_plan_tune")
        return tuned.value


def _host_ptr(x, min_words: int, what: str) -> int:
    """Address of a host buffer: a contiguous uint64/int64 numpy array or a
    CPU torch tensor (pinned for asynchronous copies)."""
    import numpy as np
    try:
        import torch
        if isinstance(x, torch.Tensor):
            if x.device.type != "cpu" or x.element_size() != 8 or not x.is_contiguous():
                raise ValueError(f"{what}: needs a contiguous 8-byte CPU tensor")
            if x.numel() < min_words:
                raise ValueError(f"{what}: needs at least {min_words} words")
            return x.data_ptr()
    except ImportError:
        pass
    if not isinstance(x, np.ndarray) or x.dtype.itemsize != 8 or not x.flags["C_CONTIGUOUS"]:
        raise ValueError(f"{what}: needs a contiguous 8-byte numpy array")
    if x.size < min_words:
        raise ValueError(f"{what}: needs at least {min_words} words")
    return x.ctypes.data


class Server:
    """Serving loop (pa_server_*): submit requests, poll tickets."""

    def __init__(self, max_inflight: int, hbm_budget_bytes: int, device: int = 0, resident_budget_bytes: int = 0):
        self._h = _VP()
        self._live = {}  # ticket -> buffers kept alive until the request is done
        cfg = ServerCfg(int(device), int(max_inflight), int(hbm_budget_bytes), int(resident_budget_bytes))
        st = lib().pa_server_create(ctypes.byref(cfg), ctypes.byref(self._h))
        if st != PA_OK:
            self._h = _VP()
            raise PAError(st, "pa_server_create")

    def close(self):
        if self._h:
            lib().pa_server_destroy(self._h)
            self._h = _VP()
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_seeds(self, session: int, gamma: int, kmax: int, a, b, c) -> int:
        W = (gamma + 63) // 64
        return lib().pa_server_set_seeds(self._h, session, gamma, kmax, _host_ptr(a, kmax * W, "a"),
                                         _host_ptr(b, W, "b"), _host_ptr(c, W, "c"))

    def submit(self, n: int, r: int, session: int, key, out):
        """(status, ticket); key and out are host buffers kept alive here
        until the ticket is polled done."""
        req = Request(n, r, session, 0, _host_ptr(key, (n + 63) // 64, "key"), _host_ptr(out, (r + 63) // 64, "out"))
        t = ctypes.c_uint64(0)
        st = lib().pa_submit(self._h, ctypes.byref(req), ctypes.byref(t))
        if st == PA_OK:
            self._live[t.value] = (key, out)
        return st, t.value

    def poll(self, ticket: int):
        """(poll status, request status, timing dict or None)."""
        res = ctypes.c_int(0)
        tm = Timing()
        st = lib().pa_poll(self._h, ticket, ctypes.byref(res), ctypes.byref(tm))
        if st == PA_OK:
            self._live.pop(ticket, None)
            return st, res.value, {"queued_ms": tm.queued_ms, "device_ms": tm.device_ms, "total_ms": tm.total_ms}
        return st, None, None

    def wait(self, ticket: int, timeout_s: float = 60.0, sleep_s: float = 0.0002):
        import time
        t_end = time.monotonic() + timeout_s
        while True:
            st, res, tm = self.poll(ticket)
            if st != PA_PENDING:
                return st, res, tm
            if time.monotonic() > t_end:
                raise TimeoutError(f"ticket {ticket} not done after {timeout_s} s")
            time.sleep(sleep_s)
