"""Scanner and image geometry descriptions (parameters only, no arithmetic of the method).

A geometry is the set of numbers that both the CPU oracle and the HIP library need to
describe the same system: image grid, radial sampling, number of angles over [0, pi),
and the oblique segments (plane count and axial slope per segment).  The paper leaves
the geometry to its projector package (Section "Numerical Results"); the reading used
everywhere in this repository is a parallel-beam, ray-driven Joseph model:

* voxel centres ``(i - (n-1)/2) * v`` per axis, image stored ``[z][y][x]``;
* angle ``phi_a = a * pi / n_ang``, radial position ``s_k = (k - (n_rad-1)/2) * d_rad``;
* segment ``g`` holds ``N_g`` planes with axial centres ``(p - (N_g-1)/2) * pitch_g * vz``
  (``pitch_g`` = 1, or 2 for the ring pairs of span 1, whose ring pitch is two image
  planes) and a constant axial slope ``tau_g`` (dz per mm of in-plane path);
* sinogram stored ``[angle][plane][radial]``, planes ordered by segment 0, +1, -1, +2, -2 ...

Scanner model (optional, the closer model of a ring scanner with detector radius ``R``):

* ``nonarc``: radial bins are not arc-corrected; bin ``k`` sits at
  ``s_k = R sin((k - (n_rad-1)/2) d_rad / R)`` (equal steps of the angle on the ring);
* ``oblique_s``: a line of response between two rings at radial position ``s`` spans the
  chord ``2 sqrt(R^2 - s^2)``, so its axial slope is ``tau_g R / sqrt(R^2 - s^2)`` rather
  than the constant ``tau_g``;
* ``span`` (odd, >= 3; 0 = off): the data planes are sums of the projector's ring-pair
  planes (segments of single ring differences ``d = 0, +1, -1, ...`` at pitch 2): ring
  differences ``|d| <= (span-1)/2`` form data segment 0, ``d`` in ``+-[g span - (span-1)/2,
  g span + (span-1)/2]`` data segment ``+-g``, and within a data segment the ring pairs
  with the same ring sum form one plane (the axial compression of PET scanners);
* detector gaps are bins of zero efficiency, i.e. zeros of ``mult`` (see ``synth.gaps``).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Tuple


@dataclasses.dataclass(frozen=True)
class Geometry:
    nx: int
    ny: int
    nz: int
    vx: float
    vy: float
    vz: float
    n_rad: int
    d_rad: float
    n_ang: int
    seg_planes: Tuple[int, ...] = (1,)
    seg_tan: Tuple[float, ...] = (0.0,)
    seg_pitch: Tuple[int, ...] = ()  # empty: every segment has pitch 1
    det_radius: float = 0.0  # detector ring radius R (mm) of the scanner model
    nonarc: bool = False     # radial bins at R sin((k - c) d_rad / R)
    oblique_s: bool = False  # axial slope tau_g R / sqrt(R^2 - s^2)
    span: int = 0            # data planes: 0 the projector's; odd >= 3 ring-sum compression

    def __post_init__(self):
        if len(self.seg_planes) != len(self.seg_tan):
            raise ValueError("seg_planes and seg_tan differ in length")
        if self.seg_pitch and len(self.seg_pitch) != len(self.seg_planes):
            raise ValueError("seg_pitch and seg_planes differ in length")
        for n, pt in zip(self.seg_planes, self.pitches):
            span = 1 + pt * (n - 1)  # image planes from the first plane to the last
            if pt not in (1, 2) or n <= 0 or span > self.nz or (self.nz - span) % 2:
                raise ValueError(f"segment of {n} planes at pitch {pt} incompatible with "
                                 f"nz={self.nz}")
        if self.nonarc or self.oblique_s:
            if not self.det_radius > 0:
                raise ValueError("the scanner model needs det_radius > 0")
            half = 0.5 * (self.n_rad - 1) * self.d_rad
            if (self.nonarc and half / self.det_radius >= 0.5 * math.pi) or \
                    (not self.nonarc and half >= self.det_radius):
                raise ValueError("radial bins beyond the detector ring")
        if self.span:
            if self.span < 3 or self.span % 2 == 0:
                raise ValueError("span must be odd and >= 3")
            rings = self.seg_planes[0]
            if self.nz != 2 * rings - 1:
                raise ValueError("span compression needs nz = 2 rings - 1")
            for n, pt, d in zip(self.seg_planes, self.pitches, self.ring_diffs):
                if pt != 2 or n != rings - abs(d):
                    raise ValueError("span compression needs ring-pair segments 0, +1, -1, ...")

    @property
    def pitches(self) -> Tuple[int, ...]:
        return tuple(self.seg_pitch) if self.seg_pitch else (1,) * len(self.seg_planes)

    @property
    def n_seg(self) -> int:
        return len(self.seg_planes)

    @property
    def n_planes(self) -> int:
        return int(sum(self.seg_planes))

    @property
    def ring_diffs(self) -> Tuple[int, ...]:
        """Ring difference of each segment in the order 0, +1, -1, +2, -2, ..."""
        return tuple(((i + 1) // 2) * (1 if i % 2 else -1) if i else 0
                     for i in range(self.n_seg))

    @property
    def data_seg_planes(self) -> Tuple[int, ...]:
        """Plane counts of the data segments (the projector's segments when span is 0)."""
        if not self.span:
            return tuple(self.seg_planes)
        h = (self.span - 1) // 2
        dmax = max(abs(d) for d in self.ring_diffs)
        out = [self.nz]  # data segment 0: every ring sum 0 .. 2 (rings - 1)
        g = 1
        while g * self.span - h <= dmax:
            n = self.nz - 2 * (g * self.span - h)
            out += [n, n]
            g += 1
        return tuple(out)

    @property
    def n_data_planes(self) -> int:
        return int(sum(self.data_seg_planes))

    @property
    def image_shape(self) -> Tuple[int, int, int]:
        return (self.nz, self.ny, self.nx)

    @property
    def sino_shape(self) -> Tuple[int, int, int]:
        return (self.n_ang, self.n_data_planes, self.n_rad)

    @property
    def n_vox(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_bins(self) -> int:
        return self.n_ang * self.n_data_planes * self.n_rad

    def plane_segment(self, q: int) -> Tuple[int, int]:
        """Return (segment, local plane index) of sinogram plane q."""
        for g, n in enumerate(self.seg_planes):
            if q < n:
                return g, q
            q -= n
        raise IndexError(q)

    def subset_angles(self, n_subsets: int, i: int):
        """Equidistantly divided angles: subset i holds angles i, i+m, i+2m, ..."""
        return list(range(i, self.n_ang, n_subsets))


def slice64_2d() -> Geometry:
    """2-D single slice: 64x64 image at 4 mm, 90 angles x 95 radial bins at 4 mm."""
    return Geometry(nx=64, ny=64, nz=1, vx=4.0, vy=4.0, vz=4.0,
                    n_rad=95, d_rad=4.0, n_ang=90)


def span11_segments(nz: int, n_seg: int, vz: float, ring_radius: float = 328.0):
    """Span-11 style oblique segments: 0, +1, -1, ... with N_g = nz - 2(11|g| - 5).

    The axial slope of segment g is the mean ring difference 11|g| times the ring pitch
    (2 vz) over the detector diameter (2 R)."""
    planes, tans = [nz], [0.0]
    g = 1
    while len(planes) < n_seg:
        n = nz - 2 * (11 * g - 5)
        if n <= 0:
            raise ValueError("too many segments for nz")
        t = 11 * g * (2.0 * vz) / (2.0 * ring_radius)
        planes += [n, n]
        tans += [t, -t]
        g += 1
    return tuple(planes[:n_seg]), tuple(tans[:n_seg])


def mmr(nz: int = 127, n_seg: int = 11, n_rad: int = 344, n_ang: int = 252,
        nxy: int = 344, vxy: float = 2.08, vz: float = 2.08) -> Geometry:
    """mMR-shaped span-11 cylinder: 344x344x127 at 2.08 mm, 344 x 252 x 837."""
    planes, tans = span11_segments(nz, n_seg, vz)
    return Geometry(nx=nxy, ny=nxy, nz=nz, vx=vxy, vy=vxy, vz=vz,
                    n_rad=n_rad, d_rad=vxy, n_ang=n_ang,
                    seg_planes=planes, seg_tan=tans)


def warmstart_geometry() -> Geometry:
    """Half in-plane resolution mMR: 172x172x127 voxels at 4.16 x 4.16 x 2.08 mm, sinogram
    172 radial (4.16 mm) x 126 angles x 837 span-11 planes."""
    return mmr(nxy=172, vxy=4.16, n_rad=172, n_ang=126)


def small_3d(nxy: int = 24, nz: int = 9, n_rad: int = 26, n_ang: int = 12,
             v: float = 4.0, tan1: float = 0.25) -> Geometry:
    """Small oblique test geometry: segments 0 (nz planes) and +-1 (nz-4 planes)."""
    return Geometry(nx=nxy, ny=nxy, nz=nz, vx=v, vy=v, vz=v, n_rad=n_rad, d_rad=v,
                    n_ang=n_ang, seg_planes=(nz, nz - 4, nz - 4),
                    seg_tan=(0.0, tan1, -tan1))


def span1_segments(rings: int, max_ring_diff: int, vz: float, ring_radius: float = 328.0):
    """Span-1 (uncompressed) segments of a scanner with `rings` detector rings at a ring
    pitch of two image planes (nz = 2 rings - 1): one segment per ring difference d = 0,
    +1, -1, ..., +D, -D, holding the rings - |d| ring pairs (r, r + d), whose axial centres
    sit on every other image plane; axial slope d (2 vz) / (2 R)."""
    planes, tans, pitch = [], [], []
    for k in range(2 * max_ring_diff + 1):
        d = (k + 1) // 2 * (1 if k % 2 else -1) if k else 0
        planes.append(rings - abs(d))
        tans.append(d * (2.0 * vz) / (2.0 * ring_radius))
        pitch.append(2)
    return tuple(planes), tuple(tans), tuple(pitch)


def mmr_span1(rings: int = 64, max_ring_diff: int = 60, n_rad: int = 344, n_ang: int = 252,
              nxy: int = 344, vxy: float = 2.08, vz: float = 2.08) -> Geometry:
    """mMR-shaped span-1 data: 64 rings, ring differences up to 60 (121 segments, 4084
    planes), image 344 x 344 x 127 at 2.08 mm, sinogram 344 x 252 x 4084 (354,033,792
    bins)."""
    planes, tans, pitch = span1_segments(rings, max_ring_diff, vz)
    return Geometry(nx=nxy, ny=nxy, nz=2 * rings - 1, vx=vxy, vy=vxy, vz=vz,
                    n_rad=n_rad, d_rad=vxy, n_ang=n_ang, seg_planes=planes, seg_tan=tans,
                    seg_pitch=pitch)


def slab_span1(rings: int = 8, max_ring_diff: int = 7, nxy: int = 344, v: float = 2.08,
               n_ang: int = 252) -> Geometry:
    """Span-1 slab of the mMR: `rings` rings (nz = 2 rings - 1 image planes) with every ring
    difference up to max_ring_diff, 344 x 344 in-plane, 252 angles."""
    planes, tans, pitch = span1_segments(rings, max_ring_diff, v)
    return Geometry(nx=nxy, ny=nxy, nz=2 * rings - 1, vx=v, vy=v, vz=v, n_rad=nxy, d_rad=v,
                    n_ang=n_ang, seg_planes=planes, seg_tan=tans, seg_pitch=pitch)


def mmr_scanner(rings: int = 64, max_ring_diff: int = 60, span: int = 11, n_rad: int = 344,
                n_ang: int = 252, nxy: int = 344, vxy: float = 2.08, vz: float = 2.08,
                det_radius: float = 328.0) -> Geometry:
    """mMR-shaped closer scanner model: the span-11 data (344 x 252 x 837) as sums of the
    4084 ring-pair planes of 64 rings (ring differences up to 60), non-arc-corrected radial
    bins and s-dependent obliquity on a 328 mm detector ring; image 344 x 344 x 127."""
    planes, tans, pitch = span1_segments(rings, max_ring_diff, vz, det_radius)
    return Geometry(nx=nxy, ny=nxy, nz=2 * rings - 1, vx=vxy, vy=vxy, vz=vz,
                    n_rad=n_rad, d_rad=vxy, n_ang=n_ang, seg_planes=planes, seg_tan=tans,
                    seg_pitch=pitch, det_radius=det_radius, nonarc=True, oblique_s=True,
                    span=span)


def scanner_small(rings: int = 8, max_ring_diff: int = 7, span: int = 3, nxy: int = 24,
                  n_rad: int = 26, n_ang: int = 12, v: float = 4.0,
                  det_radius: float = 60.0) -> Geometry:
    """Small scanner-model geometry with strong effects: a 60 mm ring (radial bins up to
    50 mm from the axis, s-dependent slopes up to 2.4 times the central one), span 3."""
    planes, tans, pitch = span1_segments(rings, max_ring_diff, v, det_radius)
    return Geometry(nx=nxy, ny=nxy, nz=2 * rings - 1, vx=v, vy=v, vz=v, n_rad=n_rad,
                    d_rad=v, n_ang=n_ang, seg_planes=planes, seg_tan=tans, seg_pitch=pitch,
                    det_radius=det_radius, nonarc=True, oblique_s=True, span=span)


def slab(nz: int, nxy: int = 344, v: float = 2.08) -> Geometry:
    """mMR slab: segment 0 (nz planes) plus +-1 (nz-12 planes), 252 angles."""
    planes, tans = span11_segments(nz, 3, v)
    return Geometry(nx=nxy, ny=nxy, nz=nz, vx=v, vy=v, vz=v, n_rad=nxy, d_rad=v,
                    n_ang=int(round(252 * nxy / 344)), seg_planes=planes, seg_tan=tans)


def slice_2d(n: int, v: float = 2.08) -> Geometry:
    """2-D N x N slice at 2.08 mm with N radial bins and round(252 N / 344) angles."""
    return Geometry(nx=n, ny=n, nz=1, vx=v, vy=v, vz=v, n_rad=n, d_rad=v,
                    n_ang=int(round(252 * n / 344)))


def fov_diagonal(g: Geometry) -> float:
    return math.hypot(g.nx * g.vx, g.ny * g.vy)
