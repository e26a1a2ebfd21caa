"""ctypes wrapper of the FP64 C projector (projector.c).  Test infrastructure only.

``forward(geom, x, angles)`` returns the rows of G x for the listed angles, packed as
[len(angles)][plane][radial]; ``backward(geom, y, angles)`` takes y packed the same way
and returns the image G^T y.  ``angles=None`` means all angles in order.  The operator of
the paper is A = diag(mult) G; the multiplicative factors are applied by the callers.

With span compression (the scanner model's data planes, see ``compression``) G = C G1:
G1 projects every ring pair (the C projector's planes) and C sums the ring pairs of each
data plane; G^T = G1^T C^T.
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
                ("seg_pitch", ctypes.c_int32 * MAX_SEG),
                ("det_radius", ctypes.c_double), ("nonarc", ctypes.c_int32),
                ("oblique_s", ctypes.c_int32)]


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
    s.det_radius = getattr(g, "det_radius", 0.0)
    s.nonarc = int(bool(getattr(g, "nonarc", False)))
    s.oblique_s = int(bool(getattr(g, "oblique_s", False)))
    return s


def _order(d: int) -> int:
    """Position of ring difference (or data segment) d in the order 0, +1, -1, +2, -2, ..."""
    return 0 if d == 0 else (2 * d - 1 if d > 0 else -2 * d)


def compression(g):
    """(map, data plane counts) of span compression, or None without it.

    Built from the ring pairs (r1, r2) of rings = (nz + 1) / 2 rings: the pair's ring-pair
    plane is plane min(r1, r2) of the segment of ring difference d = r2 - r1; its data
    segment is G = round(|d| / span) with the sign of d (|d| <= (span-1)/2: segment 0),
    and within that segment its plane is the ring sum r1 + r2 minus the segment's smallest
    ring sum, G span - (span-1)/2 (0 for segment 0).  map[q] is the data plane of ring-pair
    plane q."""
    span = getattr(g, "span", 0)
    if not span:
        return None
    rings = (g.nz + 1) // 2
    h = (span - 1) // 2
    dmax = max(((i + 1) // 2) for i in range(g.n_seg))
    seg_start = np.concatenate([[0], np.cumsum(g.seg_planes)[:-1]])
    pairs = []  # (ring-pair plane, data segment order, local data plane)
    for r1 in range(rings):
        for r2 in range(rings):
            d = r2 - r1
            if abs(d) > dmax:
                continue
            q = seg_start[_order(d)] + min(r1, r2)
            grp = (abs(d) + h) // span
            smin = 0 if grp == 0 else grp * span - h
            pairs.append((q, _order(grp if d >= 0 else -grp), r1 + r2 - smin))
    n_dseg = max(p[1] for p in pairs) + 1
    counts = np.zeros(n_dseg, dtype=np.int64)
    for _, ds, loc in pairs:
        counts[ds] = max(counts[ds], loc + 1)
    dstart = np.concatenate([[0], np.cumsum(counts)[:-1]])
    m = np.full(g.n_planes, -1, dtype=np.int64)
    for q, ds, loc in pairs:
        m[q] = dstart[ds] + loc
    if (m < 0).any():
        raise ValueError("ring-pair planes without a ring pair")
    return m, counts


def n_data_planes(g) -> int:
    c = compression(g)
    return g.n_planes if c is None else int(c[1].sum())


def compress(g, y1: np.ndarray) -> np.ndarray:
    """C y1: ring-pair rows [..][ring-pair plane][radial] -> data rows (sums)."""
    c = compression(g)
    if c is None:
        return y1
    m, counts = c
    out = np.zeros(y1.shape[:-2] + (int(counts.sum()), y1.shape[-1]), dtype=y1.dtype)
    np.add.at(out, (Ellipsis, m, slice(None)), y1)
    return out


def expand(g, y: np.ndarray) -> np.ndarray:
    """C^T y: data rows -> ring-pair rows (each ring pair takes its data plane's value)."""
    c = compression(g)
    return y if c is None else y[..., c[0], :]


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _angles(g, angles: Optional[Iterable[int]]):
    if angles is None:
        angles = range(g.n_ang)
    return np.ascontiguousarray(np.asarray(list(angles), dtype=np.int32))


def forward(g, x: np.ndarray, angles=None) -> np.ndarray:
    """Rows of G x for the listed angles, packed [len(angles)][data plane][radial]."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(g.image_shape)
    ang = _angles(g, angles)
    out = np.zeros((len(ang), g.n_planes, g.n_rad), dtype=np.float64)
    gs = _geom(g)
    lib.orc_forward(ctypes.byref(gs), ang.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                    len(ang), _dptr(x), _dptr(out))
    return compress(g, out)


def backward(g, y: np.ndarray, angles=None) -> np.ndarray:
    """G^T y for y packed [len(angles)][data plane][radial] over the listed angles."""
    lib = _load()
    ang = _angles(g, angles)
    y = np.asarray(y, dtype=np.float64).reshape(len(ang), n_data_planes(g), g.n_rad)
    y = np.ascontiguousarray(expand(g, y))
    out = np.zeros(g.image_shape, dtype=np.float64)
    gs = _geom(g)
    lib.orc_backward(ctypes.byref(gs), ang.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                     len(ang), _dptr(y), _dptr(out))
    return out


def ray(g, x: np.ndarray, a: int, q: int, k: int) -> float:
    """Single data bin (G x)[a, q, k]: the ray sum, or with span compression the sum of the
    ray sums of the data plane's ring pairs."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(g.image_shape)
    gs = _geom(g)
    c = compression(g)
    if c is None:
        return lib.orc_ray(ctypes.byref(gs), _dptr(x), a, q, k)
    return float(sum(lib.orc_ray(ctypes.byref(gs), _dptr(x), a, int(q1), k)
                     for q1 in np.nonzero(c[0] == q)[0]))
