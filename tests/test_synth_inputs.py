"""The seeded input recipes produce valid PET data: non-negative activity everywhere
(so every expected count is >= 0 and the Poisson sampler gets valid rates), including the
thin 344 x 344 x 16 slab of the batched workload, whose inner ellipsoids once reached
outside the brain along z and made the activity negative there."""
import numpy as np
import pytest

import synth
from synth.phantom import phantom_brain, voxelise


@pytest.mark.parametrize("geom", [synth.slab(16), synth.slab(32), synth.slice_2d(128),
                                  synth.small_3d(nxy=40, nz=9, n_rad=44, n_ang=24, v=5.0,
                                                 tan1=0.3)])
def test_brain_phantom_activity_non_negative(geom):
    g = synth.Geometry(nx=64, ny=64, nz=geom.nz, vx=geom.vx * geom.nx / 64,
                       vy=geom.vy * geom.ny / 64, vz=geom.vz, n_rad=8, d_rad=1.0, n_ang=4,
                       seg_planes=(geom.nz,), seg_tan=(0.0,))
    for j in range(64 if geom.nz == 16 else 16):
        rng = np.random.Generator(np.random.PCG64(18080500 + j))
        act, _, labels = phantom_brain(rng, geom)
        for e in labels["inner"]:
            assert e.az <= labels["brain"].az
        # the voxelised activity on a grid finer than the ellipsoids
        assert voxelise(g, act, supersample=1).min() >= -1e-12


def test_batch_recipe_problem_38_is_valid():
    """Problem 38 of the batched workload (a 344 x 344 x 16 slab): finite, non-negative
    expected counts and Poisson data."""
    torch = pytest.importorskip("torch")
    from synth.phantom import brain_problem_torch
    rng = np.random.Generator(np.random.PCG64(18080500))
    for _ in range(39):  # the batch recipe's draws of problems 0 .. 38
        rng.integers(8, 65), rng.random()
        counts = float(10 ** rng.uniform(5, 7))
    d = brain_problem_torch(synth.slab(16), 18080500 + 38, counts, torch.device("cpu"),
                            host_poisson=True)
    assert float(d["b"].min()) >= 0 and bool(torch.isfinite(d["r"]).all())
