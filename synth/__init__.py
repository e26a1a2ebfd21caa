"""Seeded synthetic inputs shared by the CPU oracle tests and the HIP path.

Holds geometry parameters and phantom/data generation only: no projector, prox or
iteration of the reconstruction method lives here."""
from .geometry import (Geometry, slice64_2d, mmr, mmr_span1, mmr_scanner, scanner_small,
                       small_3d, slab, slab_span1, slice_2d, span1_segments, span11_segments,
                       warmstart_geometry)
from .gaps import gap_mask
from .phantom import (Ellipsoid, brain_problem, slice64_problem, line_integrals,
                      make_data, phantom_2d, phantom_brain, voxelise)

__all__ = ["Geometry", "slice64_2d", "mmr", "mmr_span1", "mmr_scanner", "scanner_small",
           "gap_mask", "small_3d", "slab", "slab_span1",
           "slice_2d", "warmstart_geometry", "span1_segments", "span11_segments", "Ellipsoid", "brain_problem", "slice64_problem",
           "line_integrals", "make_data", "phantom_2d", "phantom_brain", "voxelise"]
