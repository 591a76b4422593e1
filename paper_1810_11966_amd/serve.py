"""Python binding of the serving runtime (include/trig_serve.h), argument
marshalling only, plus a stream driver that submits timeslices at their
arrival times and collects per-slice latencies."""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import trig

TRIG_EBUSY, TRIG_ETIMEOUT = -5, -6


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("pinned_budget_bytes", ctypes.c_size_t),
                ("n_streams", ctypes.c_int32), ("max_pending", ctypes.c_int32),
                ("device", ctypes.c_int32), ("reserved", ctypes.c_int32), ("params", trig.TrigParams)]


class SliceResult(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int32), ("n_events", ctypes.c_int32),
                ("counts", ctypes.c_void_p), ("accept", ctypes.c_void_p), ("accepted_ids", ctypes.c_void_p),
                ("n_accepted", ctypes.c_int32), ("event_status", ctypes.c_uint32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected_busy", ctypes.c_uint64), ("events_completed", ctypes.c_uint64),
                ("pending", ctypes.c_int32), ("in_flight", ctypes.c_int32), ("max_in_flight", ctypes.c_int32),
                ("hbm_in_use", ctypes.c_size_t), ("hbm_peak", ctypes.c_size_t)]


_bound = False


def _lib():
    global _bound
    lib = trig.load()
    if not _bound:
        vp = ctypes.c_void_p
        lib.trig_params_check.restype = ctypes.c_int
        lib.trig_params_check.argtypes = [ctypes.POINTER(trig.TrigParams)]
        lib.trig_server_create.restype = ctypes.c_int
        lib.trig_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
        lib.trig_server_submit.restype = ctypes.c_int
        lib.trig_server_submit.argtypes = [vp, vp, vp, vp, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_uint64)]
        lib.trig_server_poll.restype = ctypes.c_int
        lib.trig_server_poll.argtypes = [vp, ctypes.POINTER(SliceResult), ctypes.c_int32]
        lib.trig_server_release.restype = ctypes.c_int
        lib.trig_server_release.argtypes = [vp, ctypes.c_uint64]
        lib.trig_server_pause.restype = ctypes.c_int
        lib.trig_server_pause.argtypes = [vp, ctypes.c_int32]
        lib.trig_server_stats_get.restype = ctypes.c_int
        lib.trig_server_stats_get.argtypes = [vp, ctypes.POINTER(ServerStats)]
        lib.trig_server_now.restype = ctypes.c_double
        lib.trig_server_now.argtypes = [vp]
        lib.trig_server_destroy.restype = ctypes.c_int
        lib.trig_server_destroy.argtypes = [vp]
        _bound = True
    return lib


@dataclass
class Finished:
    ticket: int
    status: int
    counts: np.ndarray
    accept: np.ndarray
    ids: np.ndarray
    event_status: int
    t_submit: float
    t_admit: float
    t_done: float


class Server:
    """A trig_server; results are copied out of the server's pinned memory."""

    def __init__(self, hbm_budget_bytes: int, pinned_budget_bytes: int, n_streams: int = 4,
                 max_pending: int = 64, device: int = 0, params: Optional[trig.TrigParams] = None):
        lib = _lib()
        cfg = ServerConfig()
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        cfg.pinned_budget_bytes = int(pinned_budget_bytes)
        cfg.n_streams = int(n_streams)
        cfg.max_pending = int(max_pending)
        cfg.device = int(device)
        cfg.params = params if params is not None else trig.make_params(flags=trig.TRIG_EXEC_PRUNED)
        h = ctypes.c_void_p()
        rc = lib.trig_server_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc:
            raise trig.TrigError(rc, trig.trig_last_error_detail())
        self._h = h

    def submit(self, offsets: np.ndarray, x: np.ndarray, y: np.ndarray) -> Optional[int]:
        """Ticket, or None when the server is busy (poll, then retry)."""
        off = np.ascontiguousarray(offsets, dtype=np.int32)
        xs = np.ascontiguousarray(x, dtype=np.float32)
        ys = np.ascontiguousarray(y, dtype=np.float32)
        t = ctypes.c_uint64()
        rc = _lib().trig_server_submit(self._h, off.ctypes.data, xs.ctypes.data if xs.size else None,
                                       ys.ctypes.data if ys.size else None, (len(off) - 1) // 3, len(xs),
                                       ctypes.byref(t))
        if rc == TRIG_EBUSY:
            return None
        if rc:
            raise trig.TrigError(rc, trig.trig_last_error_detail())
        return int(t.value)

    def poll(self, timeout_ms: int = 0) -> Optional[Finished]:
        r = SliceResult()
        rc = _lib().trig_server_poll(self._h, ctypes.byref(r), int(timeout_ms))
        if rc == TRIG_ETIMEOUT:
            return None
        if rc:
            raise trig.TrigError(rc, "trig_server_poll")
        n = r.n_events
        if r.status == 0 and n:
            counts = np.ctypeslib.as_array(ctypes.cast(r.counts, ctypes.POINTER(ctypes.c_int32)), (n,)).copy()
            accept = np.ctypeslib.as_array(ctypes.cast(r.accept, ctypes.POINTER(ctypes.c_uint8)), (n,)).copy()
            ids = (np.ctypeslib.as_array(ctypes.cast(r.accepted_ids, ctypes.POINTER(ctypes.c_int32)),
                                         (r.n_accepted,)).copy() if r.n_accepted else np.zeros(0, np.int32))
        else:
            counts = np.zeros(0, np.int32)
            accept = np.zeros(0, np.uint8)
            ids = np.zeros(0, np.int32)
        f = Finished(int(r.ticket), int(r.status), counts, accept, ids, int(r.event_status),
                     float(r.t_submit), float(r.t_admit), float(r.t_done))
        _lib().trig_server_release(self._h, r.ticket)
        return f

    def pause(self, paused: bool = True) -> None:
        """Stop (or resume) admitting queued slices."""
        rc = _lib().trig_server_pause(self._h, 1 if paused else 0)
        if rc:
            raise trig.TrigError(rc, "trig_server_pause")

    def stats(self) -> ServerStats:
        st = ServerStats()
        _lib().trig_server_stats_get(self._h, ctypes.byref(st))
        return st

    def now(self) -> float:
        return float(_lib().trig_server_now(self._h))

    def close(self):
        if getattr(self, "_h", None):
            _lib().trig_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def run_stream(server: Server, slices, arrivals_s, pace: bool = True, poll_ms: int = 1,
               deadline_s: float = 300.0, submit_threads: int = 1, trace: Optional[dict] = None):
    """Submits ``slices`` (EventSet-like objects with offsets, x, y) at
    ``arrivals_s`` (seconds from now; if pace is False, as fast as possible)
    and returns {ticket: Finished} plus the index -> ticket map and the wall
    time.  With ``submit_threads`` > 1, slices are submitted by that many
    threads (concurrent arrivals stage in parallel; each thread takes the next
    slice in arrival order).  Busy servers are retried after a short wait.
    Raises TimeoutError if the stream has not finished after ``deadline_s``.
    ``trace`` (a dict) receives per slice index: how late its submitter woke
    after the arrival time, the busy retries, and the seconds spent in the
    accepted submit call (the host copy into pinned staging)."""
    import threading

    done, tickets = {}, {}
    start = time.perf_counter()
    lock = threading.Lock()
    next_i = [0]
    errors = []

    def submitter():
        while True:
            with lock:
                i = next_i[0]
                next_i[0] += 1
            if i >= len(slices):
                return
            if pace:
                dt = arrivals_s[i] - (time.perf_counter() - start)
                if dt > 0:
                    time.sleep(dt)
            s = slices[i]
            woke = time.perf_counter() - start
            retries = 0
            while True:
                if time.perf_counter() - start > deadline_s:
                    errors.append(TimeoutError(f"slice {i} not accepted before the deadline"))
                    return
                t_call = time.perf_counter()
                try:
                    t = server.submit(s.offsets, s.x, s.y)
                except Exception as e:  # surfaced in the caller
                    errors.append(e)
                    return
                if t is not None:
                    with lock:
                        tickets[i] = t
                        if trace is not None:
                            trace[i] = {"wake_late_s": woke - (arrivals_s[i] if pace else 0.0),
                                        "busy_retries": retries, "submit_call_s": time.perf_counter() - t_call}
                    break
                retries += 1
                time.sleep(poll_ms / 1e3)

    threads = [threading.Thread(target=submitter, daemon=True) for _ in range(max(1, submit_threads))]
    for th in threads:
        th.start()
    while len(done) < len(slices):
        if errors:
            raise errors[0]
        if time.perf_counter() - start > deadline_s:
            raise TimeoutError(f"stream unfinished: {len(tickets)} submitted, {len(done)} done")
        f = server.poll(poll_ms)
        while f is not None:
            done[f.ticket] = f
            f = server.poll(0)
    for th in threads:
        th.join()
    return done, tickets, time.perf_counter() - start
