"""Raw HIP events (hipEventCreate / hipEventElapsedTime via ctypes) for
timing work the library enqueues itself: torch.cuda.Event creates its
handle lazily on its own record(), so it cannot be recorded by the library."""

from __future__ import annotations

import ctypes
import ctypes.util

_hip = None


def _lib():
    global _hip
    if _hip is None:
        for name in ("libamdhip64.so", "libamdhip64.so.7", "libamdhip64.so.6"):
            try:
                _hip = ctypes.CDLL(name)
                break
            except OSError:
                continue
        if _hip is None:
            raise OSError("libamdhip64 not found")
        _hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        _hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                             ctypes.c_void_p]
        _hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        _hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        _hip.hipEventSynchronize.argtypes = [ctypes.c_void_p]
    return _hip


class HipEvent:
    def __init__(self):
        h = ctypes.c_void_p()
        rc = _lib().hipEventCreate(ctypes.byref(h))
        if rc != 0:
            raise RuntimeError(f"hipEventCreate failed ({rc})")
        self.cuda_event = h.value

    def record(self, stream_handle):
        rc = _lib().hipEventRecord(ctypes.c_void_p(self.cuda_event), stream_handle)
        if rc != 0:
            raise RuntimeError(f"hipEventRecord failed ({rc})")

    def synchronize(self):
        _lib().hipEventSynchronize(ctypes.c_void_p(self.cuda_event))

    def elapsed_ms(self, end: "HipEvent") -> float:
        ms = ctypes.c_float()
        rc = _lib().hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(self.cuda_event),
                                        ctypes.c_void_p(end.cuda_event))
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return float(ms.value)

    def __del__(self):
        try:
            if self.cuda_event and _hip is not None:
                _hip.hipEventDestroy(ctypes.c_void_p(self.cuda_event))
        except Exception:
            pass
