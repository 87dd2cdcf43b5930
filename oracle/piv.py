"""Oracle of PIV frame pairs (sec. 1: the velocity is measured from the displacement of the
particles between two frames): the second frame's particles are the first frame's advanced by a
prescribed velocity field (``orc_displace_sources`` in oracle.c, FP64, classical RK4 on the
trilinear velocity).  Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _ptr, lib


def displace_sources(src, vel, origin, spacing, dt, substeps):
    """Second frame of a PIV pair (``orc_displace_sources``): float64 [n][4]."""
    src = np.ascontiguousarray(src, dtype=np.float32)
    vel = np.ascontiguousarray(vel, dtype=np.float32)
    nz, ny, nx = vel.shape[:3]
    out = np.zeros((src.shape[0], 4))
    o = np.ascontiguousarray(origin, dtype=np.float64)
    s = np.ascontiguousarray(spacing, dtype=np.float64)
    l = lib()
    l.orc_displace_sources.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int, C.c_int, C.c_int,
                                       C.c_void_p, C.c_void_p, C.c_double, C.c_int, C.c_void_p]
    l.orc_displace_sources(_ptr(src), src.shape[0], _ptr(vel), nx, ny, nz, _ptr(o), _ptr(s), float(dt),
                           int(substeps), _ptr(out))
    return out
