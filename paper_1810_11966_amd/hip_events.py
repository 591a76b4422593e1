"""Minimal ctypes access to HIP events (timing on an explicit stream)."""
from __future__ import annotations

import ctypes

_hip = None


def _lib():
    global _hip
    if _hip is None:
        for name in ("libamdhip64.so", "libamdhip64.so.7", "/opt/rocm/lib/libamdhip64.so"):
            try:
                _hip = ctypes.CDLL(name)
                break
            except OSError:
                continue
        if _hip is None:
            raise RuntimeError("libamdhip64.so not found")
        _hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        _hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        _hip.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        _hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        _hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
    return _hip


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what} failed with hipError {rc}")


class HipEvent:
    def __init__(self):
        h = ctypes.c_void_p()
        _check(_lib().hipEventCreate(ctypes.byref(h)), "hipEventCreate")
        self.handle = h.value

    def record(self, stream: int):
        _check(_lib().hipEventRecord(ctypes.c_void_p(self.handle), ctypes.c_void_p(stream or None)),
               "hipEventRecord")

    def synchronize(self):
        _check(_lib().hipEventSynchronize(ctypes.c_void_p(self.handle)), "hipEventSynchronize")

    def elapsed_ms(self, end: "HipEvent") -> float:
        ms = ctypes.c_float()
        _check(_lib().hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(self.handle),
                                          ctypes.c_void_p(end.handle)), "hipEventElapsedTime")
        return float(ms.value)

    def __del__(self):
        try:
            if self.handle and _hip is not None:
                _hip.hipEventDestroy(ctypes.c_void_p(self.handle))
        except Exception:
            pass
