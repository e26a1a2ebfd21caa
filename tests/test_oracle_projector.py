"""Pins of the FP64 oracle projector against geometry that does not come from it:
analytic line integrals of ellipses/ellipsoids, exact chord lengths, the 90-degree
rotation covariance of the parallel-beam model, column sums at phi = 0, and the
adjoint identity between the ray-driven forward and the independent scatter adjoint."""
import ctypes
import math

import numpy as np
import pytest

import synth
from oracle import projector as proj
from synth import Geometry
from synth.phantom import Ellipsoid, line_integrals, voxelise


def _rand(shape, seed):
    return np.random.default_rng(seed).random(shape)


@pytest.mark.parametrize("geom", [synth.slice64_2d(), synth.small_3d(),
                                  synth.small_3d(nxy=17, nz=7, n_rad=21, n_ang=10),
                                  synth.slab_span1(rings=4, max_ring_diff=3, nxy=12, v=4.0,
                                                   n_ang=6)])
def test_adjoint_identity(geom):
    x = _rand(geom.image_shape, 1)
    y = _rand(geom.sino_shape, 2)
    lhs = np.vdot(proj.forward(geom, x), y)
    rhs = np.vdot(x, proj.backward(geom, y))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    ang = [0, 3, geom.n_ang - 1]
    lhs = np.vdot(proj.forward(geom, x, ang), y[ang])
    rhs = np.vdot(x, proj.backward(geom, y[ang], ang))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_ray_matches_forward():
    g = synth.small_3d()
    x = _rand(g.image_shape, 3)
    full = proj.forward(g, x)
    for (a, q, k) in [(0, 0, 5), (4, 10, 13), (7, 15, 0), (11, 18, 25)]:
        assert proj.ray(g, x, a, q, k) == full[a, q, k]


def test_phi0_column_sums():
    """At phi = 0 with radial bins on the column centres, ray k is column k times vy."""
    g = Geometry(nx=10, ny=7, nz=1, vx=2.0, vy=3.0, vz=2.0, n_rad=10, d_rad=2.0, n_ang=8)
    x = _rand(g.image_shape, 4)
    s = proj.forward(g, x, [0])[0, 0]
    np.testing.assert_allclose(s, 3.0 * x[0].sum(axis=0), rtol=1e-14)


def test_constant_image_chords():
    """Ones image: a ray that stays inside samples every row (or column) with weight 1,
    so its sum is the number of samples times the 3-D step length."""
    g = Geometry(nx=20, ny=20, nz=15, vx=1.0, vy=1.0, vz=1.0, n_rad=20, d_rad=1.0,
                 n_ang=8, seg_planes=(15, 11, 11), seg_tan=(0.0, 0.02, -0.02))
    one = np.ones(g.image_shape)
    s = proj.forward(g, one)
    # phi = 0, central radial bins, central plane of each segment
    for q, tau in [(7, 0.0), (15 + 5, 0.02), (26 + 5, -0.02)]:
        for k in (9, 10):
            assert s[0, q, k] == pytest.approx(20 * math.sqrt(1 + tau * tau), rel=1e-13)
    # phi = pi/2 samples columns
    assert s[4, 7, 9] == pytest.approx(20.0, rel=1e-13)
    # 45 degrees (tie goes to rows), central ray: each row step is sqrt(2)
    assert s[2, 7, 9] == pytest.approx(s[2, 7, 10])
    assert s[2, 7, 9] >= 19 * math.sqrt(2) - 1e-9


def test_rotation_covariance():
    """Projection at phi + pi/2 of the image rotated by +90 degrees equals the projection
    at phi of the original (also for oblique planes): pins the column branch against the
    row branch."""
    g = Geometry(nx=16, ny=16, nz=7, vx=2.0, vy=2.0, vz=2.0, n_rad=19, d_rad=2.0,
                 n_ang=16, seg_planes=(7, 5, 5), seg_tan=(0.0, 0.15, -0.15))
    x = _rand(g.image_shape, 5)
    # rotated image: x'(X, Y) = x(Y, -X)  ->  x'[z, j, i] = x[z, nx-1-i, j]
    xr = np.empty_like(x)
    n = g.nx
    for j in range(n):
        for i in range(n):
            xr[:, j, i] = x[:, n - 1 - i, j]
    half = g.n_ang // 2
    for a in range(half):
        if 4 * a == g.n_ang:
            continue  # 45 degrees: rows on both sides of the tie, not covariant
        p0 = proj.forward(g, x, [a])
        p1 = proj.forward(g, xr, [a + half])
        np.testing.assert_allclose(p1, p0, rtol=1e-11, atol=1e-11)


def _ellipse_case(nxy, v):
    g = Geometry(nx=nxy, ny=nxy, nz=1, vx=v, vy=v, vz=v, n_rad=int(round(140 / v)),
                 d_rad=v, n_ang=24)
    ells = [Ellipsoid(20.0, -12.0, 0.0, 30.0, 18.0, math.inf, 0.4, 1.0),
            Ellipsoid(-25.0, 20.0, 0.0, 12.0, 20.0, math.inf, 1.1, 2.0)]
    return g, ells


def test_against_analytic_ellipses_2d():
    """Joseph projection of a voxelised off-centre phantom approaches the exact line
    integrals as the voxels shrink (pins angle and radial sign conventions)."""
    errs = []
    for nxy, v in [(32, 4.0), (64, 2.0), (128, 1.0)]:
        g, ells = _ellipse_case(nxy, v)
        ref = line_integrals(g, ells)
        img = voxelise(g, ells, supersample=4)
        est = proj.forward(g, img)
        errs.append(np.linalg.norm(est - ref) / np.linalg.norm(ref))
    assert errs[-1] < 0.02
    assert errs[0] > errs[1] > errs[2]
    # a mirrored phantom must NOT match (the comparison is sensitive to sign errors)
    g, ells = _ellipse_case(128, 1.0)
    mirrored = [Ellipsoid(-e.cx, e.cy, e.cz, e.ax, e.ay, e.az, -e.theta, e.value) for e in ells]
    est = proj.forward(g, voxelise(g, mirrored, supersample=4))
    ref = line_integrals(g, ells)
    assert np.linalg.norm(est - ref) / np.linalg.norm(ref) > 0.3


def test_against_analytic_ellipsoids_oblique():
    """Same for oblique planes: an ellipsoid off-centre in z pins the sign and size of
    the axial slope and the 3-D step length."""
    errs = []
    for n, v in [(24, 4.0), (48, 2.0)]:
        tau = 0.3
        nz = n // 2 + 1
        g = Geometry(nx=n, ny=n, nz=nz, vx=v, vy=v, vz=v, n_rad=n + 4, d_rad=v, n_ang=12,
                     seg_planes=(nz, nz - 4, nz - 4), seg_tan=(0.0, tau, -tau))
        ells = [Ellipsoid(10.0, -6.0, 8.0, 18.0, 12.0, 10.0, 0.3, 1.0),
                Ellipsoid(-12.0, 10.0, -6.0, 8.0, 10.0, 9.0, 0.9, 2.0)]
        ref = line_integrals(g, ells)
        est = proj.forward(g, voxelise(g, ells, supersample=4))
        errs.append(np.linalg.norm(est - ref) / np.linalg.norm(ref))
        # flip the axial slope sign: must not match
        gf = Geometry(nx=n, ny=n, nz=nz, vx=v, vy=v, vz=v, n_rad=n + 4, d_rad=v, n_ang=12,
                      seg_planes=(nz, nz - 4, nz - 4), seg_tan=(0.0, -tau, tau))
        wrong = line_integrals(gf, ells)
        sl = slice(nz, None)
        assert np.linalg.norm(est[:, sl] - wrong[:, sl]) > 3 * np.linalg.norm(est[:, sl] - ref[:, sl])
        # total activity along the rays is conserved to within 2 %
        assert abs(est.sum() / ref.sum() - 1) < 0.02
    # first-order convergence (voxelised edges): the error halves with the voxel size
    assert errs[-1] < 0.09
    assert errs[1] < 0.6 * errs[0]


def test_subset_packing():
    g = synth.small_3d()
    x = _rand(g.image_shape, 6)
    full = proj.forward(g, x)
    ang = g.subset_angles(4, 1)
    np.testing.assert_array_equal(proj.forward(g, x, ang), full[ang])
    y = _rand(g.sino_shape, 7)
    parts = sum(proj.backward(g, y[g.subset_angles(4, i)], g.subset_angles(4, i))
                for i in range(4))
    np.testing.assert_allclose(parts, proj.backward(g, y), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("max_rd", [0, 4])
def test_span1_ring_pair_plane_centres(max_rd):
    """Span 1: the plane of ring pair (r1, r2), rings at every other image plane, is
    centred on image plane r1 + r2.  With the image f = z index (constant in-plane), the
    central ray at phi = 0 of a pair's plane averages f over a path symmetric about the
    plane centre, so its sum over the ny rows is ny L (r1 + r2) with L = vy sqrt(1 + tau^2)
    (the ring pairs come from the ring indices here, not from the geometry's tables)."""
    rings, ny = 5, 9
    R = 1000.0  # shallow slopes: every ray stays inside the z range
    planes, tans, pitch = synth.span1_segments(rings, max_rd, 2.0, ring_radius=R)
    g = Geometry(nx=ny, ny=ny, nz=2 * rings - 1, vx=2.0, vy=2.0, vz=2.0, n_rad=ny, d_rad=2.0,
                 n_ang=4, seg_planes=planes, seg_tan=tans, seg_pitch=pitch)
    img = np.broadcast_to(np.arange(g.nz, dtype=float)[:, None, None], g.image_shape).copy()
    q = 0
    for k in range(2 * max_rd + 1):
        d = (k + 1) // 2 * (1 if k % 2 else -1) if k else 0
        tau = d * 2.0 * 2.0 / (2.0 * R)
        assert tans[k] == pytest.approx(tau, rel=1e-15)
        for r1 in range(rings):
            r2 = r1 + d
            if not 0 <= r2 < rings:
                continue
            got = proj.ray(g, img, 0, q, ny // 2)
            assert got == pytest.approx(ny * 2.0 * math.sqrt(1 + tau * tau) * (r1 + r2),
                                        rel=1e-12, abs=1e-12)
            q += 1
    assert q == g.n_planes


def test_span1_against_analytic_ellipsoids():
    """Span-1 segments (ring pairs at a pitch of two planes, slopes up to 0.3) of an
    off-centre ellipsoid phantom: the Joseph projection of the voxelised phantom approaches
    the exact line integrals as the voxels shrink."""
    errs = []
    for n, v in [(24, 4.0), (48, 2.0)]:
        rings = n // 4 + 1
        planes, tans, pitch = synth.span1_segments(rings, 2, v, ring_radius=v * 10.0 / 3.0)
        g = Geometry(nx=n, ny=n, nz=2 * rings - 1, vx=v, vy=v, vz=v, n_rad=n + 4, d_rad=v,
                     n_ang=12, seg_planes=planes, seg_tan=tans, seg_pitch=pitch)
        ells = [Ellipsoid(10.0, -6.0, 8.0, 18.0, 12.0, 10.0, 0.3, 1.0),
                Ellipsoid(-12.0, 10.0, -6.0, 8.0, 10.0, 9.0, 0.9, 2.0)]
        ref = line_integrals(g, ells)
        est = proj.forward(g, voxelise(g, ells, supersample=4))
        errs.append(np.linalg.norm(est - ref) / np.linalg.norm(ref))
        assert abs(est.sum() / ref.sum() - 1) < 0.02
    assert errs[-1] < 0.09
    assert errs[1] < 0.6 * errs[0]


# ---------------------------------------------------------------- scanner model
def _scanner_2d(nonarc=True):
    """One image plane, 32 x 32 at 4 mm, 41 radial bins of 4 mm on a 60 mm ring."""
    return Geometry(nx=32, ny=32, nz=1, vx=4.0, vy=4.0, vz=4.0, n_rad=41, d_rad=4.0,
                    n_ang=8, det_radius=60.0, nonarc=nonarc)


@pytest.mark.parametrize("nonarc", [True, False])
def test_scanner_radial_profile_of_a_hot_column(nonarc):
    """phi = 0 rays run along y at x = s_k; one hot voxel column at x index i0 gives the
    radial profile v_y max(0, 1 - |s_k / v_x + (n_x - 1) / 2 - i0|) exactly, with s_k =
    R sin(t_k / R) for non-arc-corrected bins (t_k = (k - 20) 4 mm) and s_k = t_k else."""
    g = _scanner_2d(nonarc)
    x = np.zeros(g.image_shape)
    i0 = 28  # x = 50 mm from the axis: bins 2-3 apart between the two samplings
    x[0, 17, i0] = 1.0
    prof = proj.forward(g, x, [0])[0, 0]
    t = (np.arange(g.n_rad) - 20) * 4.0
    s = 60.0 * np.sin(t / 60.0) if nonarc else t
    want = 4.0 * np.maximum(0.0, 1.0 - np.abs(s / 4.0 + 15.5 - i0))
    np.testing.assert_allclose(prof, want, rtol=0, atol=1e-12)
    assert prof.max() > 0


def test_scanner_slope_depends_on_radial_position():
    """A uniform image: the phi = 0 ray of a ring-difference-1 plane crosses every row
    inside the image, so its sum is n_y v_y sqrt(1 + tau(s)^2) with tau(s) = tau_1 R /
    sqrt(R^2 - s^2), s = R sin(t / R); tau_1 = 1 (2 v_z) / (2 R)."""
    rings, R, v = 16, 60.0, 4.0
    planes, tans, pitch = synth.span1_segments(rings, 1, v, R)
    g = Geometry(nx=32, ny=32, nz=2 * rings - 1, vx=v, vy=v, vz=v, n_rad=41, d_rad=v,
                 n_ang=8, seg_planes=planes, seg_tan=tans, seg_pitch=pitch, det_radius=R,
                 nonarc=True, oblique_s=True)
    assert tans[1] == pytest.approx(2 * v / (2 * R))
    x = np.ones(g.image_shape)
    q = planes[0] + 7  # segment +1 (d = 1), its central ring pair (7, 8)
    for k in (20, 26, 31, 35):
        t = (k - 20) * v
        s = R * math.sin(t / R)
        if abs(s / v + 15.5) > 31 or s / v + 15.5 < 0:
            continue
        tau = tans[1] * R / math.sqrt(R * R - s * s)
        want = 32 * v * math.sqrt(1.0 + tau * tau)
        assert proj.ray(g, x, 0, q, k) == pytest.approx(want, rel=1e-12)
    # a constant slope would give the same sum for every bin
    assert proj.ray(g, x, 0, q, 35) > proj.ray(g, x, 0, q, 20) * 1.002


def test_scanner_compression_counts():
    """Span-11 data plane of ring sum S in segment 0 sums the ring pairs with |d| <= 5,
    d = S mod 2 and both rings among the 64: #{d : |d| <= min(5, S, 126 - S), d = S mod 2};
    in segment +1 (d = 6 .. 16) its first plane (S = 6) holds the pair (0, 6) only.  Every
    ring pair sits in one data plane: 4084 pairs in 837 planes."""
    g = synth.mmr_scanner()
    m, counts = proj.compression(g)
    assert tuple(counts) == (127, 115, 115, 93, 93, 71, 71, 49, 49, 27, 27)
    per = np.bincount(m, minlength=int(counts.sum()))
    assert per.sum() == 4084 == g.n_planes
    for S in range(127):
        lim = min(5, S, 126 - S)
        want = sum(1 for d in range(-lim, lim + 1) if (d - S) % 2 == 0)
        assert per[S] == want
    # segment +1 (d = 6 .. 16): its first planes S = 6, 7 hold (0, 6) and (0, 7); S = 8
    # holds (1, 7) and (0, 8); its last plane S = 120 holds (57, 63) only
    assert per[127] == 1 and per[128] == 1 and per[129] == 2
    assert per[127 + 115 - 1] == 1


def test_scanner_bins_are_sums_of_single_rays():
    """Data bin (a, q, k) of the scanner model equals the sum of the single ray sums of
    the ring pairs (r1, r2) found by direct search (|r2 - r1| in the data segment's range,
    r1 + r2 = the plane's ring sum), each ray evaluated on its own."""
    g = synth.scanner_small()
    x = _rand(g.image_shape, 11)
    full = proj.forward(g, x, [3])[0]
    lib = proj._load()
    gs = proj._geom(g)
    rings, span, h = 8, 3, 1
    seg_start = np.concatenate([[0], np.cumsum(g.seg_planes)[:-1]])
    order = lambda d: 0 if d == 0 else (2 * d - 1 if d > 0 else -2 * d)  # noqa: E731
    dstart = np.concatenate([[0], np.cumsum(g.data_seg_planes)[:-1]])
    for (dseg, sgn, lo, hi, smin) in [(0, 0, -1, 1, 0), (1, 1, 2, 4, 2), (2, -1, -4, -2, 2),
                                      (3, 1, 5, 7, 5), (4, -1, -7, -5, 5)]:
        for loc in range(g.data_seg_planes[dseg]):
            S = loc + smin
            for k in (3, 13, 22):
                want = 0.0
                for r1 in range(rings):
                    r2 = S - r1
                    if not 0 <= r2 < rings or not lo <= r2 - r1 <= hi:
                        continue
                    d = r2 - r1
                    q1 = int(seg_start[order(d)] + min(r1, r2))
                    want += lib.orc_ray(ctypes.byref(gs), proj._dptr(np.ascontiguousarray(x)),
                                        3, q1, k)
                assert full[dstart[dseg] + loc, k] == pytest.approx(want, rel=1e-13, abs=1e-13)


def test_scanner_adjoint_identity():
    g = synth.scanner_small()
    x = _rand(g.image_shape, 12)
    y = _rand(g.sino_shape, 13)
    lhs = np.vdot(proj.forward(g, x), y)
    rhs = np.vdot(x, proj.backward(g, y))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
