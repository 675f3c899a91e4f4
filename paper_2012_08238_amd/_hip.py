"""Minimal ctypes access to HIP timing events of the runtime torch already loaded
(plumbing for the benchmark: events that the library records on its stream)."""
from __future__ import annotations

import ctypes as C

_rt = None


def _runtime():
    global _rt
    if _rt is None:
        import torch  # noqa: F401  (ensures the HIP runtime is loaded and initialised)
        rt = C.CDLL("libamdhip64.so", mode=C.RTLD_GLOBAL)
        rt.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        rt.hipEventDestroy.argtypes = [C.c_void_p]
        rt.hipEventSynchronize.argtypes = [C.c_void_p]
        rt.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        _rt = rt
    return _rt


class HipEvent:
    """A timing-enabled hipEvent_t."""

    def __init__(self):
        h = C.c_void_p()
        rc = _runtime().hipEventCreate(C.byref(h))
        if rc != 0:
            raise RuntimeError(f"hipEventCreate failed: {rc}")
        self.handle = h.value

    def elapsed_ms(self, end: "HipEvent") -> float:
        t = C.c_float()
        rc = _runtime().hipEventSynchronize(end.handle)
        if rc == 0:
            rc = _runtime().hipEventElapsedTime(C.byref(t), self.handle, end.handle)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed: {rc}")
        return t.value

    def __del__(self):
        try:
            if self.handle:
                _runtime().hipEventDestroy(self.handle)
        except Exception:
            pass
