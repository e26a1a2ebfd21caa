"""Detector gaps of the scanner model (input generation only).

A ring of n_det = 2 n_ang detectors; view a and radial bin k (t = k - n_rad // 2) join
detectors i = (a + ceil(t / 2)) mod n_det and j = (a - floor(t / 2) + n_det / 2) mod n_det,
so i - j = t - n_det / 2 (opposite detectors at t = 0) and the mid-angle of the pair
follows the view.  Detectors are grouped in blocks of `block` positions whose last one is
a gap (no crystal, as between the detector blocks of the mMR: 8 crystals and one gap per
block of 9).  Every line of response with a gap at either end has zero efficiency: the
bin's multiplicative factor, its background and its counts are zero.
"""
from __future__ import annotations

import numpy as np


def gap_mask(g, block: int = 9) -> np.ndarray:
    """[n_ang][n_rad] array: 0.0 for bins with a gap detector at either end, else 1.0."""
    n_det = 2 * g.n_ang
    a = np.arange(g.n_ang)[:, None]
    t = np.arange(g.n_rad)[None, :] - g.n_rad // 2
    i = (a + (t + 1) // 2) % n_det        # ceil(t / 2)
    j = (a - np.floor_divide(t, 2) + n_det // 2) % n_det
    gap = (i % block == block - 1) | (j % block == block - 1)
    return np.where(gap, 0.0, 1.0)
