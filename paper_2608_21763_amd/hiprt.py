"""Minimal ctypes access to HIP events (for timing on the library's own stream)."""
from __future__ import annotations

import ctypes
import ctypes.util
import os

_hip = None


def _loaded_hip_runtime():
    """Path of the HIP runtime already mapped into this process (PyTorch's), if any."""
    try:
        with open("/proc/self/maps") as fh:
            for line in fh:
                p = line.split()[-1]
                if "libamdhip64.so" in os.path.basename(p):
                    return p
    except OSError:
        pass
    return None


def _lib():
    global _hip
    if _hip is None:
        for cand in (_loaded_hip_runtime() or "", "/opt/rocm/lib/libamdhip64.so",
                     ctypes.util.find_library("amdhip64") or ""):
            if cand and os.path.exists(cand):
                _hip = ctypes.CDLL(cand)
                break
        if _hip is None:
            raise ImportError("libamdhip64.so not found")
        _hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        _hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        _hip.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        _hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        _hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    return _hip


class HipEvent:
    def __init__(self):
        self.h = ctypes.c_void_p()
        rc = _lib().hipEventCreate(ctypes.byref(self.h))
        if rc != 0:
            raise RuntimeError(f"hipEventCreate failed: {rc}")

    @property
    def handle(self) -> int:
        return self.h.value

    def record(self, stream: int = 0):
        _lib().hipEventRecord(self.h, ctypes.c_void_p(stream))

    def synchronize(self):
        _lib().hipEventSynchronize(self.h)

    def elapsed_ms(self, end: "HipEvent") -> float:
        ms = ctypes.c_float()
        rc = _lib().hipEventElapsedTime(ctypes.byref(ms), self.h, end.h)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed: {rc}")
        return ms.value

    def __del__(self):
        try:
            if self.h.value:
                _lib().hipEventDestroy(self.h)
        except Exception:
            pass
