"""ctypes wrapper of the FP64 C projector (projector.c).  Test infrastructure only.

``forward(geom, x, angles)`` returns the rows of G x for the listed angles, packed as
[len(angles)][plane][radial]; ``backward(geom, y, angles)`` takes y packed the same way
and returns the image G^T y.  ``angles=None`` means all angles in order.  The operator of
the paper is A = diag(mult) G; the multiplicative factors are applied by the callers.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Iterable, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "projector.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
MAX_SEG = 128


class _Geom(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("vx", ctypes.c_double), ("vy", ctypes.c_double), ("vz", ctypes.c_double),
                ("n_rad", ctypes.c_int32), ("d_rad", ctypes.c_double),
                ("n_ang", ctypes.c_int32), ("n_seg", ctypes.c_int32),
                ("seg_planes", ctypes.c_int32 * MAX_SEG),
                ("seg_tan", ctypes.c_double * MAX_SEG),
                ("seg_pitch", ctypes.c_int32 * MAX_SEG)]


def build(force: bool = False) -> str:
    """Compile projector.c with gcc (-O2, OpenMP, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", tmp,
                               "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        gp = ctypes.POINTER(_Geom)
        lib.orc_forward.argtypes = [gp, ip, ctypes.c_int32, dp, dp]
        lib.orc_forward.restype = None
        lib.orc_backward.argtypes = [gp, ip, ctypes.c_int32, dp, dp]
        lib.orc_backward.restype = None
        lib.orc_ray.argtypes = [gp, dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        lib.orc_ray.restype = ctypes.c_double
        _lib = lib
    return _lib


def _geom(g) -> _Geom:
    s = _Geom()
    s.nx, s.ny, s.nz = g.nx, g.ny, g.nz
    s.vx, s.vy, s.vz = g.vx, g.vy, g.vz
    s.n_rad, s.d_rad, s.n_ang = g.n_rad, g.d_rad, g.n_ang
    s.n_seg = g.n_seg
    if g.n_seg > MAX_SEG:
        raise ValueError("too many segments")
    pitch = getattr(g, "seg_pitch", ()) or (1,) * g.n_seg
    for i, (n, t, pt) in enumerate(zip(g.seg_planes, g.seg_tan, pitch)):
        s.seg_planes[i] = n
        s.seg_tan[i] = t
        s.seg_pitch[i] = pt
    return s


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _angles(g, angles: Optional[Iterable[int]]):
    if angles is None:
        angles = range(g.n_ang)
    return np.ascontiguousarray(np.asarray(list(angles), dtype=np.int32))


def forward(g, x: np.ndarray, angles=None) -> np.ndarray:
    """Rows of G x for the listed angles, packed [len(angles)][plane][radial]."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(g.image_shape)
    ang = _angles(g, angles)
    out = np.zeros((len(ang), g.n_planes, g.n_rad), dtype=np.float64)
    gs = _geom(g)
    lib.orc_forward(ctypes.byref(gs), ang.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                    len(ang), _dptr(x), _dptr(out))
    return out


def backward(g, y: np.ndarray, angles=None) -> np.ndarray:
    """G^T y for y packed [len(angles)][plane][radial] over the listed angles."""
    lib = _load()
    ang = _angles(g, angles)
    y = np.ascontiguousarray(y, dtype=np.float64).reshape(len(ang), g.n_planes, g.n_rad)
    out = np.zeros(g.image_shape, dtype=np.float64)
    gs = _geom(g)
    lib.orc_backward(ctypes.byref(gs), ang.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                     len(ang), _dptr(y), _dptr(out))
    return out


def ray(g, x: np.ndarray, a: int, q: int, k: int) -> float:
    """Single ray sum (G x)[a, q, k]."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(g.image_shape)
    gs = _geom(g)
    return lib.orc_ray(ctypes.byref(gs), _dptr(x), a, q, k)
