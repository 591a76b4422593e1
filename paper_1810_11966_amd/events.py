"""Python binding of event building from a time-ordered hit stream
(include/trig_events.h), argument marshalling only: torch device tensors in,
their pointers to the C ABI, the library's kernels do the work."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

from . import trig

TRIG_EVENTS_UNSORTED, TRIG_EVENTS_CAPACITY = 1, 4

_bound = False


def _lib():
    global _bound
    lib = trig.load()
    if not _bound:
        lib.trig_build_events_workspace_bytes.restype = ctypes.c_size_t
        lib.trig_build_events_workspace_bytes.argtypes = [ctypes.c_int64]
        lib.trig_build_events.restype = ctypes.c_int
        lib.trig_build_events.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_size_t, ctypes.c_void_p]
        _bound = True
    return lib


def workspace_bytes(n_hits: int) -> int:
    return int(_lib().trig_build_events_workspace_bytes(int(n_hits)))


@dataclass
class BuildResult:
    offsets: "object"    # int64[capacity] device tensor; the first n_events + 1 entries are valid
    n_events: "object"   # int64[1] device tensor
    status: "object"     # uint32[1] (as int32)
    workspace: "object"


def build_events(t, gap: int, capacity: Optional[int] = None, stream: Optional[int] = None,
                 workspace=None, out: Optional[BuildResult] = None) -> BuildResult:
    """t: int64 cuda tensor of hit times in stream order; gap: the largest
    time difference between neighbouring hits of one event; capacity: length
    of the offsets output (default n_hits + 1, always enough).  ``out``: a
    previous result whose tensors are written again (its status keeps its
    bits: they are OR-ed in)."""
    import torch

    if not isinstance(t, torch.Tensor) or t.dtype != torch.int64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("t must be a contiguous int64 tensor on a GPU")
    dev = t.device
    n = t.numel()
    if out is not None:
        offsets, n_events, status = out.offsets, out.n_events, out.status
        cap = offsets.numel()
    else:
        cap = int(capacity) if capacity is not None else n + 1
        offsets = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
        n_events = torch.zeros(1, dtype=torch.int64, device=dev)
        status = torch.zeros(1, dtype=torch.int32, device=dev)
    need = workspace_bytes(n)
    if workspace is None or workspace.numel() < need + 256:
        workspace = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    addr = workspace.data_ptr()
    aligned = (addr + 255) & ~255
    s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
    args = (t.data_ptr() if n else None, n, int(gap), offsets.data_ptr(), cap, n_events.data_ptr(),
            status.data_ptr(), aligned, workspace.numel() - (aligned - addr), s)
    rc = _lib().trig_build_events(*args)
    if rc:
        raise trig.TrigError(rc, "trig_build_events")
    res = BuildResult(offsets, n_events, status, workspace)
    res._args = args  # the marshalled arguments, for repeat()
    return res


def repeat(res: BuildResult) -> None:
    """Run the call that produced ``res`` again on the same tensors (its
    arguments marshalled once: for timing loops)."""
    rc = _lib().trig_build_events(*res._args)
    if rc:
        raise trig.TrigError(rc, "trig_build_events")
