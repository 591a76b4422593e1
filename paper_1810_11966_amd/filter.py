"""Python binding of the trigger-station filter (include/trig_filter.h),
argument marshalling only: torch device tensors in, their pointers to the
C ABI, the library's kernels do the work."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

from . import trig

TRIG_FILTER_MALFORMED, TRIG_FILTER_CAPACITY = 1, 4


class TrigRawEvents(ctypes.Structure):
    _fields_ = [("n_events", ctypes.c_int32), ("offsets", ctypes.c_void_p), ("n_hits", ctypes.c_int64),
                ("station", ctypes.c_void_p), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p)]


class TrigFilterParams(ctypes.Structure):
    _fields_ = [("layers", ctypes.c_uint8 * 3), ("reserved", ctypes.c_uint8), ("out_capacity", ctypes.c_int32),
                ("out_layer_offsets", ctypes.c_void_p), ("out_x", ctypes.c_void_p), ("out_y", ctypes.c_void_p),
                ("out_status", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t)]


_bound = False


def _lib():
    global _bound
    lib = trig.load()
    if not _bound:
        lib.trig_filter_workspace_bytes.restype = ctypes.c_size_t
        lib.trig_filter_workspace_bytes.argtypes = [ctypes.c_int32]
        lib.trig_filter_stations.restype = ctypes.c_int
        lib.trig_filter_stations.argtypes = [ctypes.POINTER(TrigRawEvents), ctypes.POINTER(TrigFilterParams),
                                             ctypes.c_void_p]
        _bound = True
    return lib


def workspace_bytes(n_events: int) -> int:
    return int(_lib().trig_filter_workspace_bytes(int(n_events)))


@dataclass
class FilterResult:
    layer_offsets: "object"   # int32[3E+1] device tensor
    x: "object"               # fp32[capacity]
    y: "object"
    status: "object"          # uint32[1] (as int32)
    workspace: "object"


def filter_stations(offsets, station, x, y, layers: Sequence[int], capacity: int,
                    stream: Optional[int] = None, workspace=None,
                    out: Optional[FilterResult] = None) -> FilterResult:
    """offsets int64[E+1], station uint8[H], x/y fp32[H] (cuda tensors);
    layers: the three trigger station numbers; capacity: length of the x/y
    outputs (at least the number of trigger hits).  ``out``: a previous
    result for the same batch whose tensors are written again (its status
    keeps its bits: they are OR-ed in)."""
    import torch

    dev = offsets.device
    n = offsets.numel() - 1
    ev = TrigRawEvents(n, offsets.data_ptr(), station.numel(), station.data_ptr() if station.numel() else None,
                       x.data_ptr() if x.numel() else None, y.data_ptr() if y.numel() else None)
    cap = int(capacity)
    if out is not None:
        out_off, out_x, out_y, status = out.layer_offsets, out.x, out.y, out.status
        if out_off.numel() != 3 * n + 1 or out_x.numel() < max(cap, 1):
            raise ValueError("out does not fit this batch")
        if workspace is None:
            workspace = out.workspace
    else:
        out_off = torch.empty(3 * n + 1, dtype=torch.int32, device=dev)
        out_x = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
        out_y = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
        status = torch.zeros(1, dtype=torch.int32, device=dev)
    need = workspace_bytes(n)
    if workspace is None:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    p = TrigFilterParams()
    for k in range(3):
        p.layers[k] = int(layers[k])
    p.reserved = 0
    p.out_capacity = cap
    p.out_layer_offsets = out_off.data_ptr()
    p.out_x = out_x.data_ptr()
    p.out_y = out_y.data_ptr()
    p.out_status = status.data_ptr()
    p.workspace = workspace.data_ptr()
    p.workspace_bytes = workspace.numel()
    s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
    rc = _lib().trig_filter_stations(ctypes.byref(ev), ctypes.byref(p), s)
    if rc:
        raise trig.TrigError(rc, "trig_filter_stations")
    res = FilterResult(out_off, out_x, out_y, status, workspace)
    res._call = (ev, p, s)  # the marshalled arguments, for repeat()
    return res


def repeat(res: FilterResult) -> None:
    """Run the call that produced ``res`` again on the same tensors (its
    arguments marshalled once: for timing loops)."""
    ev, p, s = res._call
    rc = _lib().trig_filter_stations(ctypes.byref(ev), ctypes.byref(p), s)
    if rc:
        raise trig.TrigError(rc, "trig_filter_stations")
