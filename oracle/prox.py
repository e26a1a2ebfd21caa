"""Proximal operators and conjugates of the PET model, FP64.  Test infrastructure only.

Prox convention: prox^S_f(v) = argmin_z 1/2 ||z - v||^2_{S} + f(z) with ||x||^2_S =
<S^{-1} x, x> (Section 2.2, definition of the proximal operator).  The printed
definition omits the factor 1/2, but the printed closed form of the KL-dual prox only
holds with it, so the 1/2 convention is the reading used throughout.
"""
from __future__ import annotations

import numpy as np


def phi(u, b, r):
    """Per-bin Poisson distance phi(u) = u + r - b log(u + r) - b + b log b for u + r >= 0
    (Section 2.1, local distance), with 0 log 0 = 0 and -log 0 = inf."""
    u = np.asarray(u, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    s = u + r
    with np.errstate(divide="ignore", invalid="ignore"):
        blogb = np.where(b > 0, b * np.log(np.where(b > 0, b, 1.0)), 0.0)
        blogs = np.where(b > 0, b * np.log(np.where(s > 0, s, 1.0)), 0.0)
        val = s - b - blogs + blogb
        val = np.where((b > 0) & (s <= 0), np.inf, val)
        val = np.where(s < 0, np.inf, val)
    return val


def phi_conj(y, b, r):
    """Convex conjugate phi*(y) = -y r - b log(1 - y) for y <= 1, else inf
    (Section 2.2, conjugate of the PET distance)."""
    y = np.asarray(y, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        one_m = 1.0 - y
        blog = np.where(b > 0, b * np.log(np.where(one_m > 0, one_m, 1.0)), 0.0)
        val = -y * r - blog
        val = np.where((b > 0) & (one_m <= 0), np.inf, val)
        val = np.where(y > 1, np.inf, val)
    return val


def prox_kl_dual(v, sigma, b, r):
    """prox^sigma_{phi*}(v) = 1/2 [w + 1 - sqrt((w - 1)^2 + 4 sigma b)], w = v + sigma r
    (Section 2.2, closed form of the prox of the conjugate PET distance).

    Evaluated in the algebraically identical cancellation-free form: with q = w - 1 and
    c = 4 sigma b, 1 + (q - sqrt(q^2 + c))/2 for q <= 0 and 1 - c / (2 (q + sqrt(q^2 + c)))
    for q > 0 (multiply and divide by the conjugate surd)."""
    v = np.asarray(v, dtype=np.float64)
    w = v + sigma * r
    q = w - 1.0
    c = 4.0 * sigma * b
    root = np.sqrt(q * q + c)
    with np.errstate(divide="ignore", invalid="ignore"):
        pos = 1.0 - c / (2.0 * (q + root))
    neg = 1.0 + 0.5 * (q - root)
    return np.where(q > 0, pos, neg)


def prox_kl_dual_literal(v, sigma, b, r):
    """The printed closed form, unrearranged (accurate only when w is moderate)."""
    w = np.asarray(v, dtype=np.float64) + sigma * r
    return 0.5 * (w + 1.0 - np.sqrt((w - 1.0) ** 2 + 4.0 * sigma * b))


def prox_nonneg(x):
    """prox of the non-negativity indicator: max(x, 0) (Section 2.2, example)."""
    return np.maximum(x, 0.0)


def project_l2_ball(v, alpha, axis=0):
    """Projection onto {p : ||p_v||_2 <= alpha at every voxel}: the prox of the conjugate
    of alpha ||.||_{2,1} (an indicator), used for the TV, dTV and TGV dual blocks.
    `axis` indexes the vector components; v = 0 maps to 0."""
    v = np.asarray(v, dtype=np.float64)
    nrm = np.sqrt(np.sum(v * v, axis=axis, keepdims=True))
    with np.errstate(divide="ignore", invalid="ignore"):
        scale = np.where(nrm > alpha, alpha / nrm, 1.0)
    return v * scale


def clip_linf_ball(v, alpha):
    """Projection onto {|p_c| <= alpha}: prox of the conjugate of alpha ||.||_{1,1} (aTV)."""
    return np.clip(v, -alpha, alpha)
