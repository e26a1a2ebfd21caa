"""Seeded synthetic PET inputs: ellipse / ellipsoid phantoms with analytic sinograms.

Nothing here is the reconstruction method.  The expected data are exact line integrals
through the continuous phantom (chord length of each ellipsoid times its value), so the
data do not come from either projector under test.  Every random number is drawn from a
``numpy.random.Generator(PCG64(seed))``.

Outputs (all float32, sinogram ``[angle][plane][radial]``, image ``[z][y][x]``):
``b`` Poisson counts, ``r`` background, ``mult`` = normalisation * attenuation factors,
``x_true`` voxelised activity, ``mu`` voxelised attenuation, ``side`` MR-like image.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

from .geometry import Geometry

MU_WATER = 0.0096  # 1/mm


@dataclasses.dataclass
class Ellipsoid:
    cx: float
    cy: float
    cz: float
    ax: float
    ay: float
    az: float  # math.inf for a 2-D ellipse (infinite cylinder along z)
    theta: float  # rotation about z
    value: float


def radial_positions(g: Geometry) -> np.ndarray:
    """Radial position (mm) of every bin: equal steps, or with the scanner model's
    non-arc-corrected sampling R sin((k - c) d_rad / R)."""
    t = (np.arange(g.n_rad) - 0.5 * (g.n_rad - 1)) * g.d_rad
    return g.det_radius * np.sin(t / g.det_radius) if g.nonarc else t


def lor_data_plane(g: Geometry) -> np.ndarray:
    """Data plane of every projector plane: the identity, or with span compression the
    plane of the ring pair's data segment and ring sum."""
    if not g.span:
        return np.arange(g.n_planes)
    h = (g.span - 1) // 2
    counts = g.data_seg_planes
    base = np.concatenate([[0], np.cumsum(counts)[:-1]])
    out = []
    for n, d in zip(g.seg_planes, g.ring_diffs):
        grp = (abs(d) + h) // g.span
        seg = 0 if grp == 0 else (2 * grp - 1 if d > 0 else 2 * grp)
        smin = 0 if grp == 0 else grp * g.span - h
        ring_sum = 2 * np.arange(n) + abs(d)
        out.append(base[seg] + ring_sum - smin)
    return np.concatenate(out)


def _ray_slopes(g: Geometry, r: np.ndarray) -> np.ndarray:
    """Axial slope of every projector plane (rows) at radial positions r (columns)."""
    tau = np.concatenate([np.full(n, t) for n, t in zip(g.seg_planes, g.seg_tan)])[:, None]
    if g.oblique_s:
        tau = tau * (g.det_radius / np.sqrt(g.det_radius ** 2 - r ** 2))[None, :]
    return np.broadcast_to(tau, (g.n_planes, g.n_rad))


def _ray_params(g: Geometry, a: int):
    """Per-ray start points and direction for angle a (all projector planes x radial
    bins)."""
    phi = math.pi * a / g.n_ang
    c, s = math.cos(phi), math.sin(phi)
    r = radial_positions(g)
    zp = []
    for n, pt in zip(g.seg_planes, g.pitches):
        zp.append((np.arange(n) - 0.5 * (n - 1)) * pt * g.vz)
    zp = np.concatenate(zp)[:, None]
    px = np.broadcast_to(r * c, (g.n_planes, g.n_rad))
    py = np.broadcast_to(r * s, (g.n_planes, g.n_rad))
    pz = np.broadcast_to(zp, (g.n_planes, g.n_rad))
    dx, dy = -s, c
    dz = _ray_slopes(g, r)
    return px, py, pz, dx, dy, dz


def chord_lengths(g: Geometry, a: int, e: Ellipsoid) -> np.ndarray:
    """3-D length of every ray of angle a inside ellipsoid e, shape [planes][radial]."""
    px, py, pz, dx, dy, dz = _ray_params(g, a)
    ct, st = math.cos(e.theta), math.sin(e.theta)
    # rotate into the ellipsoid frame
    ox, oy, oz = px - e.cx, py - e.cy, pz - e.cz
    ux = ct * ox + st * oy
    uy = -st * ox + ct * oy
    uz = oz
    wx = ct * dx + st * dy
    wy = -st * dx + ct * dy
    wz = dz
    iax, iay = 1.0 / e.ax ** 2, 1.0 / e.ay ** 2
    iaz = 0.0 if math.isinf(e.az) else 1.0 / e.az ** 2
    alpha = wx * wx * iax + wy * wy * iay + wz * wz * iaz
    beta = wx * ux * iax + wy * uy * iay + wz * uz * iaz
    gamma = ux * ux * iax + uy * uy * iay + uz * uz * iaz - 1.0
    disc = beta * beta - alpha * gamma
    dt = np.where(disc > 0, 2.0 * np.sqrt(np.maximum(disc, 0.0)) / alpha, 0.0)
    return dt * np.sqrt(1.0 + dz * dz)


def line_integrals(g: Geometry, ells: List[Ellipsoid], mean: bool = False) -> np.ndarray:
    """Line integrals of the phantom per data bin: with span compression the sum over the
    bin's lines of response (or, with mean, their average)."""
    out = np.zeros(g.sino_shape, dtype=np.float64)
    dp = lor_data_plane(g)
    cnt = np.bincount(dp, minlength=g.n_data_planes).astype(np.float64)[:, None]
    for a in range(g.n_ang):
        acc = np.zeros((g.n_planes, g.n_rad))
        for e in ells:
            acc += e.value * chord_lengths(g, a, e)
        np.add.at(out[a], dp, acc)
        if mean:
            out[a] /= cnt
    return out


def voxelise(g: Geometry, ells: List[Ellipsoid], supersample: int = 2) -> np.ndarray:
    """Mean of the phantom over each voxel, by point sampling on a sub-grid."""
    img = np.zeros(g.image_shape, dtype=np.float64)
    ss = supersample
    offs = (np.arange(ss) + 0.5) / ss - 0.5
    zs_sub = offs if g.nz > 1 else np.array([0.0])
    x0 = (np.arange(g.nx) - 0.5 * (g.nx - 1)) * g.vx
    y0 = (np.arange(g.ny) - 0.5 * (g.ny - 1)) * g.vy
    z0 = (np.arange(g.nz) - 0.5 * (g.nz - 1)) * g.vz
    n = 0
    for oz in zs_sub:
        Z = (z0 + oz * g.vz)[:, None, None]
        for oy in offs:
            Y = (y0 + oy * g.vy)[None, :, None]
            for ox in offs:
                X = (x0 + ox * g.vx)[None, None, :]
                for e in ells:
                    ct, st = math.cos(e.theta), math.sin(e.theta)
                    u = ct * (X - e.cx) + st * (Y - e.cy)
                    v = -st * (X - e.cx) + ct * (Y - e.cy)
                    w = 0.0 if math.isinf(e.az) else (Z - e.cz) / e.az
                    inside = (u / e.ax) ** 2 + (v / e.ay) ** 2 + w ** 2 <= 1.0
                    img += e.value * inside
                n += 1
    return img / n


def _non_overlapping(rng, body: Ellipsoid, count: int, rmin: float, rmax: float,
                     flat: bool, taken=None):
    """Random ellipsoids inside `body` whose bounding spheres do not overlap."""
    out = [] if taken is None else list(taken)
    made = []
    tries = 0
    while len(made) < count and tries < 20000:
        tries += 1
        ax, ay = rng.uniform(rmin, rmax, size=2)
        az = math.inf if flat else rng.uniform(rmin, rmax)
        if not flat:
            # keep the ellipsoid inside the body along z too: in thin slabs (body.az small)
            # a drawn az could exceed the body, and an inner ellipsoid with a negative
            # value would make the total activity negative outside the body
            az = min(az, 0.8 * body.az)
        R = max(ax, ay) if flat else max(ax, ay, az)
        # centre uniformly inside the body's shrunken ellipsoid
        u = rng.uniform(-1, 1, size=3)
        if flat:
            u[2] = 0.0
        if np.sum(u * u) > 1.0:
            continue
        shrink = 0.8
        cx = body.cx + u[0] * max(body.ax - R / shrink, 0) * shrink
        cy = body.cy + u[1] * max(body.ay - R / shrink, 0) * shrink
        cz = 0.0 if flat else body.cz + u[2] * max(body.az - R / shrink, 0) * shrink
        ok = True
        for o in out:
            Ro = max(o.ax, o.ay) if flat else max(o.ax, o.ay, o.az)
            d = math.sqrt((cx - o.cx) ** 2 + (cy - o.cy) ** 2 + (0 if flat else (cz - o.cz) ** 2))
            if d < R + Ro + 1.0:
                ok = False
                break
        if not ok:
            continue
        e = Ellipsoid(cx, cy, cz, ax, ay, az, rng.uniform(0, math.pi), 0.0)
        out.append(e)
        made.append(e)
    return made


def phantom_2d(rng, g: Geometry, n_ellipses: int = 8):
    """Body ellipse (activity 1, water attenuation) with n random inner ellipses whose
    total activity is U(0, 4).  Returns (activity ellipses, attenuation ellipses)."""
    fov = 0.5 * min(g.nx * g.vx, g.ny * g.vy)
    body = Ellipsoid(0.0, 0.0, 0.0, 0.85 * fov, 0.7 * fov, math.inf, 0.0, 1.0)
    inner = _non_overlapping(rng, body, n_ellipses, 0.06 * fov, 0.2 * fov, flat=True)
    for e in inner:
        e.value = rng.uniform(0.0, 4.0) - body.value
    act = [body] + inner
    att = [dataclasses.replace(body, value=MU_WATER)]
    return act, att


def phantom_brain(rng, g: Geometry, n_min: int = 8, n_max: int = 12, vary: bool = False):
    """Head ellipsoid (water), brain (activity 1), 8-12 inner ellipsoids with total
    activity U(0, 4), and two ventricles of activity 0.  With vary, the head is scaled by
    U(0.85, 1.1) per axis and rotated by U(-0.2, 0.2) rad, the brain sits at a random
    offset of up to 6 mm with its own scale U(0.9, 1.05) inside it, and the ventricles'
    length, width, spread and angle vary too (drawn before the inner ellipsoids)."""
    zext = 0.5 * g.nz * g.vz
    if vary:
        sh = rng.uniform(0.85, 1.1, 3)
        rot = float(rng.uniform(-0.2, 0.2))
        sb = rng.uniform(0.9, 1.05, 3) * sh
        off = rng.uniform(-6.0, 6.0, 2)
        vl, vw = float(rng.uniform(18.0, 30.0)), float(rng.uniform(5.0, 9.0))
        vs, va = float(rng.uniform(9.0, 15.0)), float(rng.uniform(0.05, 0.3))
    else:
        sh, rot, sb, off = np.ones(3), 0.0, np.ones(3), np.zeros(2)
        vl, vw, vs, va = 25.0, 7.0, 12.0, 0.15
    head = Ellipsoid(0.0, 0.0, 0.0, 80.0 * sh[0], 100.0 * sh[1],
                     min(95.0 * sh[2], 0.9 * zext), rot, 0.25)
    brain = Ellipsoid(off[0], 5.0 + off[1], 0.0, 68.0 * sb[0], 86.0 * sb[1],
                      min(80.0 * sb[2], 0.8 * zext), rot, 0.75)
    vz = min(22.0, 0.35 * brain.az)
    vent = [Ellipsoid(off[0] - vs, 5.0 + off[1], 0.0, vw, vl, vz, rot + va, -1.0),
            Ellipsoid(off[0] + vs, 5.0 + off[1], 0.0, vw, vl, vz, rot - va, -1.0)]
    count = int(rng.integers(n_min, n_max + 1))
    inner = _non_overlapping(rng, brain, count, 6.0, 16.0, flat=False, taken=vent)
    for e in inner:
        e.value = rng.uniform(0.0, 4.0) - 1.0
    act = [head, brain] + vent + inner
    att = [dataclasses.replace(head, value=MU_WATER)]
    labels = dict(head=head, brain=brain, vent=vent, inner=inner)
    return act, att, labels


def _gauss_blur_radial(sino: np.ndarray, sigma_bins: float) -> np.ndarray:
    from scipy.ndimage import gaussian_filter1d
    return gaussian_filter1d(sino, sigma_bins, axis=-1, mode="constant", truncate=4.0)


def make_data(g: Geometry, seed: int, counts: float, act, att,
              background: str = "const10"):
    """Analytic expected data and Poisson counts.

    background "const10": r constant = 10% of the mean trues.
    background "rs30": smooth randoms (constant) + scatter (trues blurred along the radial
    direction with sigma 50 mm), half each, summing to 30% of the trues.
    The activity is scaled so that the expected total count equals `counts`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    norm = rng.uniform(0.8, 1.2, size=g.sino_shape)
    # attenuation of a compressed bin: that of its mean line of response
    att_int = line_integrals(g, att, mean=True)
    mult = norm * np.exp(-att_int)
    geo = line_integrals(g, act)
    trues = mult * geo
    if background == "const10":
        rshape = np.full(g.sino_shape, 0.1 * trues.mean())
    elif background == "rs30":
        scatter = _gauss_blur_radial(trues, 50.0 / g.d_rad)
        scatter *= 0.15 * trues.sum() / max(scatter.sum(), 1e-30)
        randoms = np.full(g.sino_shape, 0.15 * trues.mean())
        rshape = scatter + randoms
    else:
        raise ValueError(background)
    scale = counts / (trues.sum() + rshape.sum())
    ybar = scale * (trues + rshape)
    if not np.all(np.isfinite(ybar)) or ybar.min() < 0:
        raise ValueError("negative or non-finite expected counts (activity < 0 somewhere)")
    b = rng.poisson(ybar).astype(np.float32)
    return dict(b=b, r=(scale * rshape).astype(np.float32),
                mult=mult.astype(np.float32), scale=scale)


def slice64_problem(seed: int = 18080100):
    """The small 2-D problem: 64x64 slice, 8 ellipses, activity 0-4, water attenuation, normalisation
    U(0.8, 1.2), constant background 10% of mean, 1e5 expected counts."""
    from .geometry import slice64_2d
    g = slice64_2d()
    rng = np.random.Generator(np.random.PCG64(seed))
    act, att = phantom_2d(rng, g)
    d = make_data(g, seed + 1, 1e5, act, att, "const10")
    d["x_true"] = (d["scale"] * voxelise(g, act)).astype(np.float32)
    d["mu"] = voxelise(g, att).astype(np.float32)
    d["geom"] = g
    return d


def side_image(rng, g: Geometry, labels, noise: float = 0.05) -> np.ndarray:
    """MR-like side image: WM 1.0 (brain), GM 0.6 (inner ellipsoids), CSF 0.2
    (ventricles), background 0, plus N(0, noise^2)."""
    brain = dataclasses.replace(labels["brain"], value=1.0)
    parts = [brain]
    parts += [dataclasses.replace(e, value=0.6 - 1.0) for e in labels["inner"]]
    parts += [dataclasses.replace(e, value=0.2 - 1.0) for e in labels["vent"]]
    img = voxelise(g, parts, supersample=1)
    img += rng.normal(0.0, noise, size=img.shape)
    return img.astype(np.float32)


def brain_problem(g: Geometry, seed: int, counts: float, with_side: bool = False,
                  gaps: bool = False):
    """Brain-like 3-D problem with randoms + scatter at 30% of trues; with gaps, the bins
    of gap detectors (synth.gaps) have zero efficiency, background and counts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    act, att, labels = phantom_brain(rng, g)
    d = make_data(g, seed + 1, counts, act, att, "rs30")
    if gaps:
        from .gaps import gap_mask
        mk = gap_mask(g)[:, None, :].astype(np.float32)
        for key in ("b", "r", "mult"):
            d[key] = d[key] * mk
    d["x_true"] = (d["scale"] * voxelise(g, act, supersample=1)).astype(np.float32)
    d["geom"] = g
    if with_side:
        d["side"] = side_image(np.random.Generator(np.random.PCG64(seed + 2)), g, labels)
    return d


# ---------------------------------------------------------------- torch (device) version
def _torch_chords(torch, g: Geometry, angles, e: Ellipsoid, device):
    """Chord lengths of all rays of the given angles through ellipsoid e, FP64 on device:
    shape [len(angles)][planes][radial]."""
    f64 = torch.float64
    a = torch.as_tensor(angles, dtype=f64, device=device)[:, None, None]
    phi = math.pi * a / g.n_ang
    c, s = torch.cos(phi), torch.sin(phi)
    r = torch.as_tensor(radial_positions(g), dtype=f64, device=device)[None, None, :]
    zp = torch.cat([(torch.arange(n, dtype=f64, device=device) - 0.5 * (n - 1)) * pt * g.vz
                    for n, pt in zip(g.seg_planes, g.pitches)])[None, :, None]
    tau = torch.as_tensor(np.array(_ray_slopes(g, radial_positions(g)), dtype=np.float64),
                          dtype=f64, device=device)[None, :, :]
    ct, st = math.cos(e.theta), math.sin(e.theta)
    ox, oy, oz = r * c - e.cx, r * s - e.cy, zp - e.cz
    ux, uy, uz = ct * ox + st * oy, -st * ox + ct * oy, oz
    dx, dy = -s, c
    wx, wy, wz = ct * dx + st * dy, -st * dx + ct * dy, tau
    iax, iay = 1.0 / e.ax ** 2, 1.0 / e.ay ** 2
    iaz = 0.0 if math.isinf(e.az) else 1.0 / e.az ** 2
    alpha = wx * wx * iax + wy * wy * iay + wz * wz * iaz
    beta = wx * ux * iax + wy * uy * iay + wz * uz * iaz
    gamma = ux * ux * iax + uy * uy * iay + uz * uz * iaz - 1.0
    disc = beta * beta - alpha * gamma
    dt = torch.where(disc > 0, 2.0 * torch.sqrt(torch.clamp(disc, min=0.0)) / alpha,
                     torch.zeros_like(disc))
    return dt * torch.sqrt(1.0 + tau * tau)


def line_integrals_torch(g: Geometry, ells, device, batch: int = 12, mean: bool = False):
    """line_integrals on a torch device (FP64)."""
    import torch
    out = torch.zeros(g.sino_shape, dtype=torch.float64, device=device)
    dp = torch.as_tensor(lor_data_plane(g), device=device)
    cnt = torch.bincount(dp, minlength=g.n_data_planes).to(torch.float64)[None, :, None]
    for a0 in range(0, g.n_ang, batch):
        ang = list(range(a0, min(a0 + batch, g.n_ang)))
        acc = torch.zeros((len(ang), g.n_planes, g.n_rad), dtype=torch.float64, device=device)
        for e in ells:
            acc += e.value * _torch_chords(torch, g, ang, e, device)
        if g.span:
            red = torch.zeros((len(ang), g.n_data_planes, g.n_rad), dtype=torch.float64,
                              device=device)
            red.index_add_(1, dp, acc)
            acc = red / cnt if mean else red
        out[a0:a0 + len(ang)] = acc
    return out


def brain_problem_torch(g: Geometry, seed: int, counts: float, device, with_side=False,
                        host_poisson=False, gaps=False, vary=False):
    """The brain-like 3-D problem generated on a torch device (float32 outputs): same
    phantom parameters as brain_problem, analytic data in FP64, randoms + scatter at 30%
    of trues, normalisation U(0.8, 1.2), Poisson counts (torch generator seeded, or with
    host_poisson a NumPy PCG64 generator seeded from `seed` on the host)."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    act, att, labels = phantom_brain(rng, g, vary=vary)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed + 1)
    norm = torch.rand(g.sino_shape, generator=gen, device=device, dtype=torch.float64) * 0.4 + 0.8
    mult = norm * torch.exp(-line_integrals_torch(g, att, device, mean=True))
    del norm
    trues = mult * line_integrals_torch(g, act, device)
    sigma = 50.0 / g.d_rad
    half = int(math.ceil(4 * sigma))
    kern = torch.exp(-0.5 * (torch.arange(-half, half + 1, device=device, dtype=torch.float64)
                             / sigma) ** 2)
    kern = kern / kern.sum()
    # zero-padded Gaussian blur along the radial axis as one banded matrix product:
    # scatter[.., i] = sum_j trues[.., j] kern[j - i + half]
    idx = torch.arange(g.n_rad, device=device)
    off = idx.view(-1, 1) - idx.view(1, -1) + half
    band = torch.where((off >= 0) & (off <= 2 * half), kern[off.clamp(0, 2 * half)],
                       torch.zeros((), dtype=torch.float64, device=device))
    scatter = (trues.view(-1, g.n_rad) @ band).view(g.sino_shape)
    scatter *= 0.15 * trues.sum() / scatter.sum().clamp(min=1e-30)
    rshape = scatter + 0.15 * trues.mean()
    del scatter
    scale = counts / (trues.sum() + rshape.sum())
    ybar = scale * (trues + rshape)
    # a Poisson sampler given a negative or NaN rate is undefined (on the device, torch's
    # sampler faulted the GPU on such rates): check before sampling
    if not bool(torch.isfinite(ybar).all()) or float(ybar.min()) < 0:
        raise ValueError("negative or non-finite expected counts (activity < 0 somewhere)")
    if host_poisson:
        hrng = np.random.Generator(np.random.PCG64(seed + 3))
        b = torch.from_numpy(hrng.poisson(ybar.cpu().numpy()).astype(np.float32)).to(device)
    else:
        b = torch.poisson(ybar, generator=gen).to(torch.float32)
    del ybar, trues
    d = dict(b=b, r=(scale * rshape).to(torch.float32), mult=mult.to(torch.float32),
             scale=float(scale), geom=g, ellipsoids=act)
    if gaps:
        from .gaps import gap_mask
        mk = torch.as_tensor(gap_mask(g), dtype=torch.float32, device=device)[:, None, :]
        for key in ("b", "r", "mult"):
            d[key] = d[key] * mk
    if with_side:
        d["side"] = torch.from_numpy(
            side_image(np.random.Generator(np.random.PCG64(seed + 2)), g, labels)).to(device)
    return d
