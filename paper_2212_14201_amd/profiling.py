"""Binding of the library's per-launch kernel timing (HIP events)."""
from __future__ import annotations

import ctypes

from .qvm import check, lib, _vp


class QvmKernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double),
                ("flops", ctypes.c_double)]


def _declare():
    L = lib()
    L.qvm_profile_begin.argtypes = [_vp]
    L.qvm_profile_begin.restype = ctypes.c_int
    L.qvm_profile_end.argtypes = [_vp, ctypes.POINTER(QvmKernelStat), ctypes.c_int32,
                                  ctypes.POINTER(ctypes.c_int32)]
    L.qvm_profile_end.restype = ctypes.c_int
    return L


def begin(sv):
    check(_declare().qvm_profile_begin(sv.handle))


def end(sv) -> dict:
    """Stop recording; returns {kernel class: {launches, total_ms, bytes, flops}}."""
    L = _declare()
    arr = (QvmKernelStat * 16)()
    cnt = ctypes.c_int32()
    check(L.qvm_profile_end(sv.handle, arr, 16, ctypes.byref(cnt)))
    out = {}
    for i in range(min(cnt.value, 16)):
        r = arr[i]
        out[r.name.decode()] = {"launches": int(r.launches), "total_ms": float(r.total_ms),
                                "bytes": float(r.bytes), "flops": float(r.flops)}
    return out
