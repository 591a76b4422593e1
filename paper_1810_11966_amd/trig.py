"""Python binding of libtrig (include/trig.h): argument marshalling only.

Every step of the selection runs in the library's HIP kernels; PyTorch only
provides device memory and the stream.  The functions keep the C names:

    trig_params_init() -> TrigParams
    trig_workspace_bytes(n_events, params) -> int
    trig_select(events, hits, params, out_counts, out_accept, stream) -> int
    trig_autotune(events, hits, params, out_counts, out_accept, reps, stream)
        -> (int, TrigAutotuneResult)
    trig_autotune_reset()
    trig_strerror(code) -> str

plus ``select(offsets, x, y, ...)`` and ``autotune(offsets, x, y, ...)``,
which allocate the outputs (and the workspace) with torch on the inputs'
device and raise TrigError on failure.
The library must be built (python -m paper_1810_11966_amd.build); loading
fails loudly otherwise, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtrig.so")

TRIG_ABI_VERSION = 2
TRIG_NOALLOC_SCRATCH_BYTES = 4 << 20
TRIG_OK, TRIG_EINVAL, TRIG_EWORKSPACE, TRIG_EHIP, TRIG_EUNSUPPORTED = 0, -1, -2, -3, -4
TRIG_COUNT_MALFORMED, TRIG_COUNT_OVERFLOW = -1, -2
TRIG_STATUS_MALFORMED, TRIG_STATUS_OVERFLOW = 1, 2
TRIG_TEST_MSD, TRIG_TEST_SLOPE_WINDOW, TRIG_TEST_MSD_BASIS = 0, 1, 2
TRIG_EXEC_PLAIN, TRIG_EXEC_PERSISTENT, TRIG_EXEC_BINNED = 0, 1, 2
TRIG_EXEC_AUTOTUNE, TRIG_OUT_COMPACT, TRIG_EXEC_PRUNED = 4, 8, 16
TRIG_ACCEPT_TWO_PARTICLES, TRIG_DECISION_ONLY = 32, 64

TESTS = {"msd": TRIG_TEST_MSD, "window": TRIG_TEST_SLOPE_WINDOW, "msd_basis": TRIG_TEST_MSD_BASIS}
FORMS = {
    "plain": TRIG_EXEC_PLAIN,
    "pruned": TRIG_EXEC_PRUNED,
    "persistent": TRIG_EXEC_PERSISTENT,
    "persistent_pruned": TRIG_EXEC_PERSISTENT | TRIG_EXEC_PRUNED,
    "binned": TRIG_EXEC_BINNED,
    "persistent_binned": TRIG_EXEC_PERSISTENT | TRIG_EXEC_BINNED,
    "auto": TRIG_EXEC_AUTOTUNE,
}

# Every symbol include/trig.h declares.
EXPORTED = ("trig_params_init", "trig_params_check", "trig_workspace_bytes", "trig_select", "trig_select_noalloc",
            "trig_autotune", "trig_autotune_reset", "trig_autotune_save", "trig_autotune_load",
            "trig_autotune_lookup", "trig_set_kernel_events", "trig_strerror", "trig_last_error_detail", "trig_probe_valu",
            "trig_probe_copy", "trig_server_create", "trig_server_submit", "trig_server_poll",
            "trig_server_release", "trig_server_pause", "trig_server_stats_get", "trig_server_now", "trig_server_destroy",
            "trig_filter_workspace_bytes", "trig_filter_stations", "trig_build_events_workspace_bytes",
            "trig_build_events")


class TrigEventsCsr(ctypes.Structure):
    _fields_ = [("n_events", ctypes.c_int32), ("layer_offsets", ctypes.c_void_p)]


class TrigHits(ctypes.Structure):
    _fields_ = [("n_hits", ctypes.c_int32), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("z", ctypes.c_void_p)]


class TrigParams(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("test", ctypes.c_int32),
                ("z", ctypes.c_float * 3), ("msd_max", ctypes.c_float * 2),
                ("ndf", ctypes.c_int32), ("slope_window", ctypes.c_float * 2),
                ("min_triplets", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("out_accepted_ids", ctypes.c_void_p), ("out_n_accepted", ctypes.c_void_p),
                ("out_status", ctypes.c_void_p), ("tile_pairs", ctypes.c_int32),
                ("block_events", ctypes.c_int32), ("block_hits", ctypes.c_int32),
                ("block_waves", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]


class TrigAutotuneResult(ctypes.Structure):
    _fields_ = [("n_candidates", ctypes.c_int32), ("mult_class", ctypes.c_int32),
                ("block_hits", ctypes.c_int32), ("block_waves", ctypes.c_int32),
                ("block_events", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("binned", ctypes.c_int32), ("ms_best", ctypes.c_float), ("ms_rule", ctypes.c_float)]


class TrigError(RuntimeError):
    def __init__(self, code: int, detail: str):
        super().__init__(f"trig error {code}: {trig_strerror(code)} ({detail})")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libtrig.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1810_11966_amd.build`")
    lib = ctypes.CDLL(path)
    lib.trig_params_init.restype = ctypes.c_int
    lib.trig_params_init.argtypes = [ctypes.POINTER(TrigParams)]
    lib.trig_workspace_bytes.restype = ctypes.c_size_t
    lib.trig_workspace_bytes.argtypes = [ctypes.POINTER(TrigEventsCsr), ctypes.POINTER(TrigParams)]
    lib.trig_select.restype = ctypes.c_int
    lib.trig_select.argtypes = [ctypes.POINTER(TrigEventsCsr), ctypes.POINTER(TrigHits),
                                ctypes.POINTER(TrigParams), ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p]
    lib.trig_select_noalloc.restype = ctypes.c_int
    lib.trig_select_noalloc.argtypes = lib.trig_select.argtypes
    lib.trig_autotune.restype = ctypes.c_int
    lib.trig_autotune.argtypes = [ctypes.POINTER(TrigEventsCsr), ctypes.POINTER(TrigHits),
                                  ctypes.POINTER(TrigParams), ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_int32, ctypes.POINTER(TrigAutotuneResult), ctypes.c_void_p]
    lib.trig_autotune_reset.restype = None
    lib.trig_autotune_reset.argtypes = []
    lib.trig_autotune_save.restype = ctypes.c_int
    lib.trig_autotune_save.argtypes = [ctypes.c_char_p]
    lib.trig_autotune_load.restype = ctypes.c_int
    lib.trig_autotune_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32)]
    lib.trig_autotune_lookup.restype = ctypes.c_int
    lib.trig_autotune_lookup.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(TrigAutotuneResult)]
    lib.trig_set_kernel_events.restype = ctypes.c_int
    lib.trig_set_kernel_events.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.trig_strerror.restype = ctypes.c_char_p
    lib.trig_strerror.argtypes = [ctypes.c_int]
    lib.trig_last_error_detail.restype = ctypes.c_char_p
    lib.trig_last_error_detail.argtypes = []
    lib.trig_probe_valu.restype = ctypes.c_int
    lib.trig_probe_valu.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_void_p,
                                    ctypes.c_void_p]
    lib.trig_probe_copy.restype = ctypes.c_int
    lib.trig_probe_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.c_void_p]
    _lib = lib
    return lib


def trig_params_init() -> TrigParams:
    p = TrigParams()
    rc = load().trig_params_init(ctypes.byref(p))
    if rc:
        raise TrigError(rc, "trig_params_init")
    return p


def make_params(test: str = "msd", z=None, msd_max=None, ndf: Optional[int] = None,
                slope_window=None, min_triplets: Optional[int] = None, flags: int = 0,
                tile_pairs: int = 0, block_events: int = 0, block_hits: int = 0,
                block_waves: int = 0) -> TrigParams:
    """Defaults from trig_params_init(), overridden by the given values."""
    p = trig_params_init()
    p.test = TESTS[test] if isinstance(test, str) else int(test)
    if z is not None:
        for i in range(3):
            p.z[i] = float(z[i])
    if msd_max is not None:
        p.msd_max[0], p.msd_max[1] = (float(v) for v in msd_max)
    if ndf is not None:
        p.ndf = int(ndf)
    if slope_window is not None:
        p.slope_window[0], p.slope_window[1] = (float(v) for v in slope_window)
    if min_triplets is not None:
        p.min_triplets = int(min_triplets)
    p.flags = int(flags)
    p.tile_pairs = int(tile_pairs)
    p.block_events = int(block_events)
    p.block_hits = int(block_hits)
    p.block_waves = int(block_waves)
    return p


def trig_workspace_bytes(n_events: int, params: TrigParams) -> int:
    ev = TrigEventsCsr(int(n_events), None)
    return int(load().trig_workspace_bytes(ctypes.byref(ev), ctypes.byref(params)))


def trig_select(events: TrigEventsCsr, hits: TrigHits, params: TrigParams, out_counts: int,
                out_accept: int, stream: int) -> int:
    """Raw call: device addresses as ints, stream as a hipStream_t int (0 =
    null stream)."""
    return int(load().trig_select(ctypes.byref(events), ctypes.byref(hits), ctypes.byref(params),
                                  ctypes.c_void_p(out_counts or None), ctypes.c_void_p(out_accept or None),
                                  ctypes.c_void_p(stream or None)))


def trig_select_noalloc(events: TrigEventsCsr, hits: TrigHits, params: TrigParams, out_counts: int,
                        out_accept: int, stream: int) -> int:
    """Raw call of the allocation-free variant (params.workspace must be
    None, workspace_bytes 0): the library's static device scratch."""
    return int(load().trig_select_noalloc(ctypes.byref(events), ctypes.byref(hits), ctypes.byref(params),
                                          ctypes.c_void_p(out_counts or None), ctypes.c_void_p(out_accept or None),
                                          ctypes.c_void_p(stream or None)))


def trig_autotune(events: TrigEventsCsr, hits: TrigHits, params: TrigParams, out_counts: int,
                  out_accept: int, reps: int, stream: int):
    """Raw call (see trig_select); returns (code, TrigAutotuneResult)."""
    r = TrigAutotuneResult()
    rc = int(load().trig_autotune(ctypes.byref(events), ctypes.byref(hits), ctypes.byref(params),
                                  ctypes.c_void_p(out_counts or None), ctypes.c_void_p(out_accept or None),
                                  int(reps), ctypes.byref(r), ctypes.c_void_p(stream or None)))
    return rc, r


def trig_autotune_reset() -> None:
    load().trig_autotune_reset()


def autotune_save(path: str) -> None:
    """Write the recorded shapes to the cache file ``path``."""
    rc = load().trig_autotune_save(str(path).encode())
    if rc:
        raise TrigError(rc, trig_last_error_detail())


def autotune_load(path: str) -> int:
    """Record the shapes of the cache file ``path`` for this process's
    matching devices; returns the number recorded."""
    n = ctypes.c_int32(0)
    rc = load().trig_autotune_load(str(path).encode(), ctypes.byref(n))
    if rc:
        raise TrigError(rc, trig_last_error_detail())
    return int(n.value)


def autotune_lookup(test: str, mult_class: int):
    """The shape recorded for the current device, test and class, or None."""
    found = ctypes.c_int32(0)
    res = TrigAutotuneResult()
    rc = load().trig_autotune_lookup(TESTS[test], int(mult_class), ctypes.byref(found), ctypes.byref(res))
    if rc:
        raise TrigError(rc, trig_last_error_detail())
    if not found.value:
        return None
    return {"block_hits": res.block_hits, "block_waves": res.block_waves, "persistent": res.persistent,
            "binned": res.binned}


def trig_set_kernel_events(start: int, stop: int) -> int:
    """hipEvent_t handles (ints) recorded around the dominant kernel of the
    following trig_select calls of this thread; 0, 0 switches off."""
    return int(load().trig_set_kernel_events(ctypes.c_void_p(start or None), ctypes.c_void_p(stop or None)))


def trig_strerror(code: int) -> str:
    return load().trig_strerror(int(code)).decode()


def trig_last_error_detail() -> str:
    return load().trig_last_error_detail().decode()


@dataclass
class SelectResult:
    counts: "object"           # torch.int32 [E]
    accept: "object"           # torch.uint8 [E]
    ids: "object" = None       # torch.int32 [E] (first n_accepted valid) when compact
    n_accepted: "object" = None  # torch.int32 [1] when compact
    status: "object" = None    # torch.int32 [1] (uint32 bits) when requested
    workspace: "object" = None  # torch.uint8 workspace, kept alive with the result


def _check_tensor(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor on a GPU")


def _prepare(offsets, x, y, test, form, compact, want_status, stream, workspace, out, param_kw, hit_z=None):
    import torch
    _check_tensor(offsets, torch.int32, "offsets")
    _check_tensor(x, torch.float32, "x")
    _check_tensor(y, torch.float32, "y")
    if x.numel() != y.numel():
        raise ValueError("x and y differ in length")
    if hit_z is not None:
        _check_tensor(hit_z, torch.float32, "hit_z")
        if hit_z.numel() != x.numel():
            raise ValueError("hit_z and x differ in length")
    n_ev = (offsets.numel() - 1) // 3
    if offsets.numel() != 3 * n_ev + 1:
        raise ValueError("offsets must hold 3*n_events+1 entries")
    dev = offsets.device
    extra = int(param_kw.pop("extra_flags", 0))
    flags = FORMS[form] | (TRIG_OUT_COMPACT if compact else 0) | extra
    p = make_params(test=test, flags=flags, **param_kw)
    if out is None:
        counts = torch.empty(n_ev, dtype=torch.int32, device=dev)
        accept = torch.empty(n_ev, dtype=torch.uint8, device=dev)
    else:
        counts, accept = out
    res = SelectResult(counts, accept)
    if compact:
        res.ids = torch.empty(max(n_ev, 1), dtype=torch.int32, device=dev)
        res.n_accepted = torch.zeros(1, dtype=torch.int32, device=dev)
        p.out_accepted_ids = res.ids.data_ptr()
        p.out_n_accepted = res.n_accepted.data_ptr()
    if want_status:
        res.status = torch.zeros(1, dtype=torch.int32, device=dev)
        p.out_status = res.status.data_ptr()
    nbytes = trig_workspace_bytes(n_ev, p)
    if nbytes:
        if workspace is None or workspace.numel() < nbytes + 256:
            workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        addr = workspace.data_ptr()
        aligned = (addr + 255) & ~255
        p.workspace = aligned
        p.workspace_bytes = workspace.numel() - (aligned - addr)
    s = torch.cuda.current_stream(dev).cuda_stream if stream is None else int(stream)
    ev = TrigEventsCsr(n_ev, offsets.data_ptr())
    hits = TrigHits(x.numel(), x.data_ptr(), y.data_ptr(), hit_z.data_ptr() if hit_z is not None else None)
    res.workspace = workspace  # kept until the result is dropped (the call is asynchronous)
    return p, res, ev, hits, s


def select(offsets, x, y, *, hit_z=None, test: str = "msd", form: str = "plain", compact: bool = False,
           want_status: bool = False, stream=None, workspace=None, out=None, **param_kw) -> SelectResult:
    """Run trig_select on torch device tensors (int32 offsets [3E+1], float32
    x, y [H], optional float32 per-hit z positions ``hit_z`` [H]).  ``form``
    is a key of FORMS;
    extra keywords go to make_params (``extra_flags`` is OR-ed into the
    flags).  ``out`` may hold preallocated (counts, accept) tensors."""
    p, res, ev, hits, s = _prepare(offsets, x, y, test, form, compact, want_status, stream, workspace,
                                   out, param_kw, hit_z=hit_z)
    rc = trig_select(ev, hits, p, res.counts.data_ptr(), res.accept.data_ptr(), s)
    if rc:
        raise TrigError(rc, trig_last_error_detail())
    return res


def autotune(offsets, x, y, *, test: str = "msd", reps: int = 3, compact: bool = False,
             want_status: bool = False, stream=None, workspace=None, out=None, **param_kw):
    """Run trig_autotune on torch device tensors (form "auto"); returns
    (SelectResult, TrigAutotuneResult).  Synchronises the stream."""
    p, res, ev, hits, s = _prepare(offsets, x, y, test, "auto", compact, want_status, stream, workspace,
                                   out, param_kw)
    rc, info = trig_autotune(ev, hits, p, res.counts.data_ptr(), res.accept.data_ptr(), reps, s)
    if rc:
        raise TrigError(rc, trig_last_error_detail())
    return res, info
