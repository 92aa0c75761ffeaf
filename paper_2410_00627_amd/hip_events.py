"""Raw hipEvent_t handles through ctypes, for per-kernel timing with the profiled entry point."""
from __future__ import annotations

import ctypes
import ctypes.util
import os

_hip = None


def hip():
    global _hip
    if _hip is None:
        cands = [os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib", "libamdhip64.so"),
                 ctypes.util.find_library("amdhip64") or "libamdhip64.so"]
        err = None
        for c in cands:
            try:
                _hip = ctypes.CDLL(c)
                break
            except OSError as e:  # pragma: no cover
                err = e
        if _hip is None:
            raise OSError(f"libamdhip64 not found: {err}")
        _hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        _hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        _hip.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        _hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        _hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    return _hip


class EventArray:
    """n hipEvent_t handles; `.arr` is the ctypes array passed to the C ABI."""

    def __init__(self, n: int):
        self.n = n
        self.arr = (ctypes.c_void_p * n)()
        for i in range(n):
            h = ctypes.c_void_p()
            code = hip().hipEventCreate(ctypes.byref(h))
            if code != 0:
                raise RuntimeError(f"hipEventCreate failed: {code}")
            self.arr[i] = h
        self._keep = True

    def elapsed_ms(self, a: int, b: int) -> float:
        ms = ctypes.c_float(0)
        hip().hipEventSynchronize(self.arr[b])
        code = hip().hipEventElapsedTime(ctypes.byref(ms), self.arr[a], self.arr[b])
        if code != 0:
            raise RuntimeError(f"hipEventElapsedTime failed: {code}")
        return float(ms.value)

    def __len__(self):
        return self.n

    def close(self):
        for i in range(self.n):
            if self.arr[i]:
                hip().hipEventDestroy(self.arr[i])
                self.arr[i] = None
