"""Algorithmic FLOP count of one step on a given state (host tool ``libbn2d_flops.so``).

Counts every +, -, *, /, sqrt and exp of the kernel's own formulation (bn2d_physics.h compiled on
the host with a counting scalar), walked once per fluid cell and once per edge: the work the method
needs, without the kernel's redundant halo recomputation."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "bn2d_flops.cpp")
LIB = os.path.join(HERE, "libbn2d_flops.so")


def build() -> str:
    tmp = LIB + ".tmp"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-w", "-o", tmp, SRC])
    os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        d = ctypes.c_double
        L.bn2d_count_flops.argtypes = [ctypes.c_int, ctypes.c_int, d, d, d, d, d, d, d, d, d, d,
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint8),
                                       ctypes.POINTER(d), ctypes.POINTER(d), d,
                                       ctypes.POINTER(ctypes.c_ulonglong)]
        L.bn2d_count_flops.restype = ctypes.c_int
        _lib = L
    return _lib


def count(s, q, y0, dt) -> dict:
    """FLOPs of one step of scenario ``s`` from state ``q`` ([4, ny, nx]) with free surface ``y0``."""
    L = _load()
    q = np.ascontiguousarray(q, dtype=np.float64)
    y0 = np.ascontiguousarray(y0, dtype=np.float64)
    bc = (ctypes.c_int32 * 4)(*[int(b) for b in s.bc])
    solid = None
    keep = None
    if getattr(s, "solid", None) is not None:
        keep = np.ascontiguousarray(s.solid, dtype=np.uint8)
        solid = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    out = (ctypes.c_ulonglong * 6)()
    dp = ctypes.POINTER(ctypes.c_double)
    L.bn2d_count_flops(int(s.nx), int(s.ny), s.x0, s.x1, s.y0, s.y1, s.g, s.k0, s.rho0, s.alpha_liq,
                       s.alpha_gas, s.cfl, bc, solid, q.ctypes.data_as(dp), y0.ctypes.data_as(dp), float(dt), out)
    names = ["reconstruction", "x_edges", "y_edges", "update", "detector_cfl", "fluid_cells"]
    res = {n: int(v) for n, v in zip(names, out)}
    res["total"] = sum(res[n] for n in names[:5])
    res["per_fluid_cell"] = res["total"] / max(res["fluid_cells"], 1)
    return res
