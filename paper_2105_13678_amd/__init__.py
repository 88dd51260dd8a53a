"""MMH-MH privacy-amplification hash (arXiv 2105.13678) on AMD MI355X.

The hash runs in libpa.so (hand-written HIP for gfx950, C interface in
include/pa.h); this package is its Python binding plus the seeded synthetic
input generators.  Importing the package loads nothing; the library is loaded
on first use and a missing library is an error, never a fallback.
"""
from .binding import (PA_FLAG_POW2_LENGTHS, PA_FLAG_RADIX3_LENGTHS, PA_FLAG_RADIX5_LENGTHS, PA_OK, PA_PENDING, PA_RELOAD,  # noqa: F401
                      BatchPlan, PAError, Plan, Server, decode_status, lib, plan_query, plan_tune, probe_goldilocks, probe_valu,
                      status_string)

__all__ = ["Plan", "BatchPlan", "Server", "PAError", "plan_query", "status_string", "decode_status", "lib", "PA_OK",
           "PA_RELOAD", "PA_FLAG_POW2_LENGTHS", "PA_FLAG_RADIX3_LENGTHS", "PA_FLAG_RADIX5_LENGTHS", "plan_tune",
           "probe_goldilocks", "probe_valu", "to_device", "from_device"]


def to_device(words, device="cuda"):
    """uint64 numpy array -> int64 torch tensor on the device (bit-identical)."""
    import numpy as np
    import torch
    arr = np.ascontiguousarray(words, dtype=np.uint64).view(np.int64)
    return torch.from_numpy(arr.copy()).to(device)


def from_device(t):
    """int64 torch tensor -> uint64 numpy array (bit-identical)."""
    import numpy as np
    return t.detach().cpu().numpy().view(np.uint64).copy()
